// CPU emulation of the kernel primitives -- TEST INFRASTRUCTURE ONLY.
//
// Lets the indexing kernel body (paper_1902_08318_amd/csrc/jsidx_kernel.h)
// run unchanged on the host: every workgroup is 256 OS threads, every wave 64
// of them; ballots and shuffles exchange values through a per-wave slot array
// between two wave barriers; LDS is per-workgroup host memory.  The byte
// permute, dot product and byte-align instructions are emulated from their ISA
// definitions.  Every global load and store is bounds-checked against ranges
// the harness registers, so an access the GPU would make out of range aborts
// here instead.
#pragma once
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>

#define JSIDX_DEV inline
#define JSIDX_DEVFN inline
#define JSIDX_CONSTANT static const

struct uint4 {
  uint32_t x, y, z, w;
};
struct uint2 {
  uint32_t x, y;
};

namespace jsidx {
namespace prim {

struct Barrier {
  std::mutex m;
  std::condition_variable cv;
  int n;
  int count = 0;
  uint64_t gen = 0;
  explicit Barrier(int n_) : n(n_) {}
  void wait() {
    std::unique_lock<std::mutex> lk(m);
    uint64_t g = gen;
    if (++count == n) {
      count = 0;
      gen++;
      cv.notify_all();
    } else {
      cv.wait(lk, [&] { return gen != g; });
    }
  }
};

struct WaveCtx {
  Barrier bar{64};
  uint64_t slot[64];
};

struct GroupCtx {
  explicit GroupCtx(int threads) : bar(threads) {}
  Barrier bar;
  WaveCtx waves[16];
  std::atomic<int> count{0};
  int count_result = 0;
  alignas(64) unsigned char lds[1 << 18];
};

struct Range {
  const void* lo;
  const void* hi;
};

struct EmuEnv {
  Range reads[8];
  int nreads = 0;
  Range writes[8];
  int nwrites = 0;
  std::atomic<long> violations{0};
};

struct ThreadCtx {
  uint32_t tid, block, grid;
  GroupCtx* g;
  EmuEnv* env;
};

extern thread_local ThreadCtx tctx;

inline void check(const void* p, size_t n, bool write) {
  EmuEnv* e = tctx.env;
  const Range* r = write ? e->writes : e->reads;
  int nr = write ? e->nwrites : e->nreads;
  const char* c = (const char*)p;
  for (int i = 0; i < nr; i++)
    if (c >= (const char*)r[i].lo && c + n <= (const char*)r[i].hi) return;
  if (e->violations.fetch_add(1) < 5)
    fprintf(stderr, "cpu_emu: out-of-range %s of %zu bytes at %p (block %u tid %u)\n", write ? "store" : "load", n, p,
            tctx.block, tctx.tid);
}

inline uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  uint64_t data = ((uint64_t)hi << 32) | lo;
  uint32_t out = 0;
  for (int k = 0; k < 4; k++) {
    uint32_t s = (sel >> (8 * k)) & 0xFFu, b;
    if (s >= 13) b = 0xFF;
    else if (s == 12) b = 0;
    else if (s >= 8) {
      static const int src[4] = {1, 3, 5, 7};
      b = ((data >> (8 * src[s - 8] + 7)) & 1) ? 0xFF : 0;
    } else b = (uint32_t)(data >> (8 * s)) & 0xFFu;
    out |= b << (8 * k);
  }
  return out;
}
inline uint32_t udot4(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t s = c;
  for (int k = 0; k < 4; k++) s += ((a >> (8 * k)) & 0xFF) * ((b >> (8 * k)) & 0xFF);
  return s;
}
inline uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * (s & 3)));
}

inline uint32_t tid() { return tctx.tid; }
inline uint32_t block() { return tctx.block; }
inline uint32_t grid() { return tctx.grid; }
inline uint32_t lane() { return tctx.tid & 63u; }
inline uint32_t wave_id() { return tctx.tid >> 6; }

inline WaveCtx& wave() { return tctx.g->waves[tctx.tid >> 6]; }
inline uint64_t ballot(bool p) {
  WaveCtx& w = wave();
  w.slot[lane()] = p ? 1 : 0;
  w.bar.wait();
  uint64_t m = 0;
  for (int i = 0; i < 64; i++) m |= (w.slot[i] ? 1ull : 0ull) << i;
  w.bar.wait();
  return m;
}
inline uint32_t exchange(uint32_t v, int src) {
  WaveCtx& w = wave();
  w.slot[lane()] = v;
  w.bar.wait();
  uint32_t r = (uint32_t)w.slot[src & 63];
  w.bar.wait();
  return r;
}
inline uint32_t shfl(uint32_t v, int src) { return exchange(v, src); }
inline uint32_t shfl_up(uint32_t v, int d) {
  int src = (int)lane() - d;
  return exchange(v, src < 0 ? (int)lane() : src);
}
inline uint32_t shfl_xor(uint32_t v, int m) { return exchange(v, (int)(lane() ^ (uint32_t)m)); }
inline bool lane_bit(uint64_t m) { return (m >> lane()) & 1ull; }
inline uint32_t mbcnt(uint64_t m) {
  const uint32_t l = lane();
  return (uint32_t)__builtin_popcountll(l ? (m & (~0ull >> (64 - l))) : 0ull);
}
inline uint32_t readlane(uint32_t v, int l) { return exchange(v, l); }
inline uint32_t incl_max_scan(uint32_t v) {
  WaveCtx& w = wave();
  w.slot[lane()] = v;
  w.bar.wait();
  uint32_t s = 0;
  for (uint32_t i = 0; i <= lane(); i++) s = s > (uint32_t)w.slot[i] ? s : (uint32_t)w.slot[i];
  w.bar.wait();
  return s;
}
inline uint32_t shr1(uint32_t v, uint32_t fill) {
  uint32_t r = exchange(v, lane() == 0 ? 0 : (int)lane() - 1);
  return lane() == 0 ? fill : r;
}
inline uint32_t ror1(uint32_t v) { return exchange(v, lane() == 0 ? 63 : (int)lane() - 1); }
inline uint32_t alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (s & 31));
}
inline uint32_t incl_scan(uint32_t v) {
  WaveCtx& w = wave();
  w.slot[lane()] = v;
  w.bar.wait();
  uint32_t s = 0;
  for (uint32_t i = 0; i <= lane(); i++) s += (uint32_t)w.slot[i];
  w.bar.wait();
  return s;
}

inline void sync() { tctx.g->bar.wait(); }
inline void wave_sync() { wave().bar.wait(); }
inline int sync_count(bool p) {
  GroupCtx* g = tctx.g;
  if (p) g->count.fetch_add(1);
  g->bar.wait();
  if (tctx.tid == 0) g->count_result = g->count.exchange(0);
  g->bar.wait();
  int r = g->count_result;
  g->bar.wait();
  return r;
}
inline void sleep() { std::this_thread::sleep_for(std::chrono::microseconds(20)); }
constexpr uint32_t kSpinLimit = 1u << 20;  // ~20 s of emulated waiting
inline void wait_mem() { std::atomic_thread_fence(std::memory_order_seq_cst); }

inline uint64_t ld_agent(const uint64_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
inline uint32_t ld_agent32(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
inline void st_agent(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
inline void st_agent32(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
inline uint32_t add_agent32(uint32_t* p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline uint32_t or_agent32(uint32_t* p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
inline uint64_t or_agent64(uint64_t* p, uint64_t v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
inline void min_lds(int32_t* p, int32_t v) {
  int32_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
  }
}

inline uint32_t add_lds32(uint32_t* p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline uint32_t ld_lds32(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
inline void st_lds32(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }

template <class T>
inline T& lds_object() {
  static_assert(sizeof(T) <= sizeof(GroupCtx::lds), "LDS object too large");
  return *reinterpret_cast<T*>(tctx.g->lds);
}

inline void trace(int64_t, int) {}
inline void trace_count(int64_t, int) {}
inline void dtrace(int64_t, int) {}
inline void dcount(int64_t, uint64_t) {}

inline uint4 load16(const uint8_t* p) {
  check(p, 16, false);
  if ((uintptr_t)p & 15) {
    fprintf(stderr, "cpu_emu: misaligned 16-byte load at %p\n", (const void*)p);
    tctx.env->violations++;
  }
  uint4 v;
  memcpy(&v, p, 16);
  return v;
}
inline uint32_t load4(const uint8_t* p) {
  check(p, 4, false);
  uint32_t v;
  memcpy(&v, p, 4);
  return v;
}
inline uint32_t load1(const uint8_t* p) {
  check(p, 1, false);
  return *p;
}
inline uint64_t load8(const uint64_t* p) {
  check(p, 8, false);
  return *p;
}
inline void st_out(uint32_t* p, uint32_t v) {
  check(p, 4, true);
  *p = v;
}
inline void st_out4(uint32_t* p, uint4 v) {
  check(p, 16, true);
  if ((uintptr_t)p & 3) {
    fprintf(stderr, "cpu_emu: misaligned 16-byte store at %p\n", (void*)p);
    tctx.env->violations++;
  }
  memcpy(p, &v, 16);
}
// LDS accesses must stay inside the workgroup's LDS.
inline void lds_check(const void* p, size_t n, size_t align) {
  const unsigned char* b = tctx.g->lds;
  const unsigned char* q = static_cast<const unsigned char*>(p);
  if (q < b || q + n > b + sizeof(GroupCtx::lds) || ((uintptr_t)q & (align - 1))) {
    fprintf(stderr, "cpu_emu: LDS access of %zu bytes at %p outside the workgroup's LDS or misaligned\n", n, p);
    tctx.env->violations++;
  }
}
inline uint4 ld_lds128(const uint32_t* p) {
  lds_check(p, 16, 16);
  if ((uintptr_t)p & 15) {
    fprintf(stderr, "cpu_emu: misaligned 16-byte LDS read at %p\n", (const void*)p);
    tctx.env->violations++;
  }
  uint4 v;
  memcpy(&v, p, 16);
  return v;
}
inline void st_lds128(uint32_t* p, uint4 v) {
  lds_check(p, 16, 16);
  memcpy(p, &v, 16);
}
inline uint32_t lds_ld1(const uint8_t* p) {
  lds_check(p, 1, 1);
  return *p;
}
inline void lds_st1(uint8_t* p, uint32_t v) {
  lds_check(p, 1, 1);
  *p = (uint8_t)v;
}
inline void lds_st4(uint32_t* p, uint32_t v) {
  lds_check(p, 4, 4);
  *p = v;
}
inline void st_byte(uint8_t* p, uint32_t v) {
  check(p, 1, true);
  *p = (uint8_t)v;
}
inline uint2 ld_pair(const uint2* p) {
  check(p, 8, false);
  return *p;
}
inline void st_pair(uint2* p, uint32_t x, uint32_t y) {
  check(p, 8, true);
  p->x = x;
  p->y = y;
}

}  // namespace prim
}  // namespace jsidx
