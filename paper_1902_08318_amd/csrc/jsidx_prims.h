// Hardware primitives used by the indexing kernel (gfx950 / wave64).
//
// The kernel is written against this small set of functions only, so every
// instruction-level choice sits in one place: byte permutes (v_perm_b32),
// 4x8-bit dot products (v_dot4_u32_u8), funnel byte shifts (v_alignbyte_b32),
// wave ballots, lane shuffles, workgroup barriers and agent-scope atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define JSIDX_DEV __device__ __forceinline__
#define JSIDX_DEVFN __device__

namespace jsidx {
namespace prim {

JSIDX_DEV uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) { return __builtin_amdgcn_perm(hi, lo, sel); }
JSIDX_DEV uint32_t udot4(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_udot4(a, b, c, false); }
JSIDX_DEV uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s) { return __builtin_amdgcn_alignbyte(hi, lo, s); }

JSIDX_DEV uint32_t tid() { return threadIdx.x; }
JSIDX_DEV uint32_t block() { return blockIdx.x; }
JSIDX_DEV uint32_t grid() { return gridDim.x; }
JSIDX_DEV uint32_t lane() { return __lane_id(); }
JSIDX_DEV uint32_t wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

JSIDX_DEV uint64_t ballot(bool p) { return __ballot(p); }
JSIDX_DEV uint32_t shfl(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src); }
JSIDX_DEV uint32_t shfl_up(uint32_t v, int d) { return (uint32_t)__shfl_up((int)v, d); }
JSIDX_DEV uint32_t shfl_xor(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m); }
// Bit `lane` of a wave-uniform mask (v_cndmask on the mask as a lane mask).
JSIDX_DEV bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
// Set bits of m below this lane.
JSIDX_DEV uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
JSIDX_DEV uint32_t readlane(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
// Inclusive prefix sum over the wave: DPP row shifts 1, 2, 4, 8 inside rows of
// 16 lanes, then row broadcasts of lanes 15 and 31.
JSIDX_DEV uint32_t incl_scan(uint32_t v) {
  v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false);
  return v;
}
// Inclusive prefix maximum over the wave (same DPP pattern).
JSIDX_DEV uint32_t incl_max_scan(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x111, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x112, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x114, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x118, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false));
  return v;
}
// Value of the previous lane (DPP wave_shr:1); lane 0 gets `fill`.
JSIDX_DEV uint32_t shr1(uint32_t v, uint32_t fill) { return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xF, 0xF, false); }
// Value of the previous lane, lane 0 getting lane 63's (DPP wave_ror:1).
JSIDX_DEV uint32_t ror1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x13C, 0xF, 0xF, false); }
// (hi:lo >> s) truncated to 32 bits (v_alignbit_b32).
JSIDX_DEV uint32_t alignbit(uint32_t hi, uint32_t lo, uint32_t s) { return __builtin_amdgcn_alignbit(hi, lo, s); }

JSIDX_DEV void sync() { __syncthreads(); }
// LDS written by some lanes of a wave is visible to the wave's other lanes.
JSIDX_DEV void wave_sync() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __asm__ __volatile__("" ::: "memory");
}
JSIDX_DEV int sync_count(bool p) { return __syncthreads_count(p); }
JSIDX_DEV void sleep() { __builtin_amdgcn_s_sleep(1); }
// Look-back waits give up after this many sleeps (about half a second).
constexpr uint32_t kSpinLimit = 1u << 23;
// Waits until this wave's memory operations have completed (s_waitcnt 0),
// without the L2 write-back and invalidate of an agent-scope fence.  Enough
// to order device-scope atomic accesses (the descriptor protocol uses only
// those) before a later one.
JSIDX_DEV void wait_mem() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0);
  __asm__ __volatile__("" ::: "memory");
}

JSIDX_DEV uint64_t ld_agent(const uint64_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
JSIDX_DEV uint32_t ld_agent32(const uint32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
JSIDX_DEV void st_agent(uint64_t* p, uint64_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
JSIDX_DEV void st_agent32(uint32_t* p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
JSIDX_DEV uint32_t add_agent32(uint32_t* p, uint32_t v) { return atomicAdd(p, v); }
JSIDX_DEV void min_lds(int32_t* p, int32_t v) { atomicMin(p, v); }
// Workgroup-shared (LDS) counters read and updated by several waves.
JSIDX_DEV uint32_t add_lds32(uint32_t* p, uint32_t v) { return atomicAdd(p, v); }
JSIDX_DEV uint32_t ld_lds32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
JSIDX_DEV void st_lds32(uint32_t* p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

// One instance per workgroup (LDS).
template <class T>
JSIDX_DEV T& lds_object() {
  __shared__ T obj;
  return obj;
}

// Timing hooks for probe builds (no-ops in the library).
JSIDX_DEV void trace(int64_t, int) {}
JSIDX_DEV void trace_count(int64_t, int) {}
#ifdef JSIDX_PROBE
// Probe builds only: tile t's event k gets the 100 MHz real-time clock, and
// event 7 the wave's hardware id, in a buffer the probe host code sets.
extern __device__ uint64_t* g_probe;
JSIDX_DEV void dtrace(int64_t t, int k) {
  if (g_probe && __lane_id() == 0) {
    g_probe[t * 8 + k] = __builtin_amdgcn_s_memrealtime();
    if (k == 0) g_probe[t * 8 + 7] = (uint64_t)__builtin_amdgcn_s_getreg((4 << 0) | (0 << 6) | (31 << 11));
  }
}
// Probe builds only: adds v to tile t's counter word (slot 6).
JSIDX_DEV void dcount(int64_t t, uint64_t v) {
  if (g_probe && __lane_id() == 0) g_probe[t * 8 + 6] += v;
}
#else
JSIDX_DEV void dtrace(int64_t, int) {}
JSIDX_DEV void dcount(int64_t, uint64_t) {}
#endif

JSIDX_DEV uint4 load16(const uint8_t* p) { return *reinterpret_cast<const uint4*>(p); }
JSIDX_DEV uint32_t load4(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }
JSIDX_DEV uint64_t load8(const uint64_t* p) { return *p; }
JSIDX_DEV uint32_t load1(const uint8_t* p) { return *p; }
JSIDX_DEV uint32_t or_agent32(uint32_t* p, uint32_t v) { return atomicOr(p, v); }
JSIDX_DEV uint64_t or_agent64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
JSIDX_DEV void st_out(uint32_t* p, uint32_t v) { *p = v; }
// 16 bytes to a 4-byte aligned global address (one vector store: global
// accesses only need dword alignment).
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
JSIDX_DEV void st_out4(uint32_t* p, uint4 v) {
  const u32x4_a4 w = {v.x, v.y, v.z, v.w};
  *reinterpret_cast<u32x4_a4*>(p) = w;
}
// 16 bytes from / to a 16-byte aligned LDS address.
JSIDX_DEV uint4 ld_lds128(const uint32_t* p) { return *reinterpret_cast<const uint4*>(p); }
JSIDX_DEV void st_lds128(uint32_t* p, uint4 v) { *reinterpret_cast<uint4*>(p) = v; }
// Single LDS bytes and words.
JSIDX_DEV uint32_t lds_ld1(const uint8_t* p) { return *p; }
JSIDX_DEV void lds_st1(uint8_t* p, uint32_t v) { *p = (uint8_t)v; }
JSIDX_DEV void lds_st4(uint32_t* p, uint32_t v) { *p = v; }
JSIDX_DEV void st_byte(uint8_t* p, uint32_t v) { *p = (uint8_t)v; }
JSIDX_DEV void st_pair(uint2* p, uint32_t x, uint32_t y) { *p = make_uint2(x, y); }
JSIDX_DEV uint2 ld_pair(const uint2* p) { return *p; }

}  // namespace prim
}  // namespace jsidx
