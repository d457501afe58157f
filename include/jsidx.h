/*
 * jsidx.h -- C ABI of the MI355X (gfx950) stage-1 JSON structural indexer.
 *
 * Stage 1 of Langdale & Lemire, "Parsing Gigabytes of JSON per Second"
 * (arXiv 1902.08318), Sec. 3.1: given the bytes of a JSON document, find the
 * positions of every structural character (, : [ ] { }) outside strings,
 * every opening quote, and every pseudo-structural byte (a byte outside
 * strings that is neither white space nor structural nor a quote and follows
 * a structural, white-space or quote byte; Sec. 3.1.3), in increasing order,
 * as uint32 offsets (Sec. 3.1.4).  Quotes preceded by an odd-length run of
 * backslashes are escaped (Sec. 3.1.1, Fig. 3); the string ranges are the
 * inclusive prefix XOR of the unescaped quotes (Fig. 4); closing quotes are
 * not indexed (last step of Fig. 5).  The input is also validated as UTF-8
 * against the table of well-formed byte sequences of Sec. 3.1.5; the error
 * is accumulated over the document and reported once (Sec. 3.1.5, last
 * paragraph), it never changes the index.  The byte before a document counts
 * as white space, so a scalar root value is indexed.
 *
 * All entry points are asynchronous on the HIP stream they are given; data
 * pointers are DEVICE pointers owned by the caller.  The library never reads
 * or writes host memory on behalf of a call.
 *
 * Input contract.  Document bytes are read-only and never modified.  The
 * kernels load whole aligned 16-byte granules: a granule that holds at least
 * one byte of the input may be read in full, including bytes just before the
 * first or just after the last input byte (an aligned granule never crosses a
 * page, so this never faults); such bytes never influence any result.
 *
 * Output contract.  The index and the flags are a total function of the bytes:
 * both are produced for every document, valid JSON or not.  Flags are sound,
 * not complete: a set bit proves the document is not valid JSON; zero flags
 * do not prove it is (number, string and structure checks belong to stage 2).
 *
 * Beyond stage 1 the library offers, on one document's index: minification
 * (jsidx_minify), the tape's scope links with the structure check
 * (jsidx_scopes), and the stage-2 tape itself with parsed numbers, normalized
 * strings and checked literals (jsidx_tape).  The kernels after the index
 * read only bytes inside the document.  jsidx_set_variant selects variants
 * of the indexing kernel with one of the paper's stage-1 optimizations turned
 * off (its ablation, App. B).
 */
#ifndef JSIDX_H
#define JSIDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque stream handle: a hipStream_t (0 = the legacy default stream). */
typedef void *jsidx_stream_t;

/* ---- status codes (API errors; nothing is launched when one is returned) */
#define JSIDX_OK 0
#define JSIDX_E_INVAL (-1)       /* NULL pointer, len >= 2^32, ndocs == 0   */
#define JSIDX_E_NOWORKSPACE (-2) /* workspace could not be allocated          */
#define JSIDX_E_HIP (-3)         /* a HIP runtime call failed                 */
#define JSIDX_E_TOO_LARGE (-4)   /* input exceeds what the workspace can hold */

/* ---- per-document flag bits written to out_err ---------------------------
 * Document validity is NOT a status code: it is reported per document. */
#define JSIDX_ERR_UTF8 0x1u            /* not well-formed UTF-8 (Sec. 3.1.5
                                          table), including a multi-byte
                                          sequence cut off by the end        */
#define JSIDX_ERR_UNCLOSED_STRING 0x2u /* odd number of unescaped quotes:
                                          the document ends inside a string  */
#define JSIDX_ERR_TRAILING_ESCAPE 0x4u /* the document ends with an odd run
                                          of backslashes                      */
#define JSIDX_ERR_EMPTY 0x8u           /* the index is empty (empty or
                                          all-white-space document)           */
#define JSIDX_ERR_UNBALANCED 0x10u      /* jsidx_scopes: a bracket has no
                                          partner                             */
#define JSIDX_ERR_MISMATCHED 0x20u      /* jsidx_scopes: a '{' linked with a
                                          ']' or a '[' with a '}'             */
#define JSIDX_ERR_SYNTAX 0x40u          /* jsidx_scopes: the entries' tokens
                                          do not form one JSON value          */
#define JSIDX_ERR_OFFSETS 0x40000000u  /* not indexed: the batch's offsets
                                          decrease somewhere (out_n is 0)     */
#define JSIDX_ERR_CAPACITY 0x80000000u /* not indexed: the batch is larger
                                          than the stream's reserved
                                          workspace (out_n is 0)              */

/*
 * jsidx_build -- index one document (Sec. 3.1).
 *   buf      device pointer to `len` bytes (any alignment).
 *   len      byte count, 0 <= len < 2^32 (positions are uint32, Sec. 3.1.4).
 *   out_idx  device array of at least max(len, 1) uint32: receives the
 *            positions in increasing order; entries past *out_n unspecified.
 *   out_n    device uint32: number of positions written.
 *   out_err  device uint32: JSIDX_ERR_* flags of the document.
 *   stream   hipStream_t to run on.
 * Returns JSIDX_OK or a negative JSIDX_E_* code (then nothing was launched).
 * The first call on a stream may allocate the stream's workspace (see
 * jsidx_reserve); later calls of a size the workspace covers allocate nothing.
 * One launch: tiles of 16 KiB are taken in increasing order by the running
 * waves, and each tile's carries (string parity, entry count, a multi-byte
 * UTF-8 sequence cut at its start) come from the tiles before it by a
 * two-level look-back (Sec. 3.1: the blocks are independent given the
 * carries).
 */
int jsidx_build(const uint8_t *buf, uint64_t len, uint32_t *out_idx,
                uint32_t *out_n, uint32_t *out_err, jsidx_stream_t stream);

/*
 * jsidx_build_batch -- index many independent documents in one launch.
 *   bufs     device pointer to the concatenated document bytes.
 *   offsets  device array of ndocs+1 nondecreasing uint64: document d is
 *            bufs[offsets[d] .. offsets[d+1]); offsets[0] may be nonzero;
 *            each document must be shorter than 2^32 bytes.
 *   ndocs    number of documents, >= 1.
 *   out_idx  device array of at least max(offsets[ndocs], 1) uint32; document d
 *            writes its positions (relative to its own first byte) to
 *            out_idx[offsets[d] .. offsets[d] + out_n[d]).
 *   out_n, out_err  device arrays of ndocs uint32 (count and flags per doc).
 * Each document's results are identical to jsidx_build on that document.
 * Offsets are read on the device.  After jsidx_reserve on the stream, the
 * call never synchronises and never allocates, and a batch larger than the
 * reserved size is not indexed: every out_err[d] is set to JSIDX_ERR_CAPACITY
 * and out_n[d] to 0.  Without a reservation the call copies offsets[0] and
 * offsets[ndocs] to the host (synchronising the stream) and grows the stream's
 * workspace if needed.
 * Offsets are checked on the device before anything is indexed (a first,
 * small kernel reads all ndocs+1 of them): if offsets[d+1] < offsets[d] for
 * any d, no document is indexed, no byte of bufs is read and no entry of
 * out_idx is written, and every out_n[d] is set to 0 and every out_err[d] to
 * JSIDX_ERR_OFFSETS (the device-side form of rejecting the argument, since
 * the offsets are not on the host).
 */
int jsidx_build_batch(const uint8_t *bufs, const uint64_t *offsets,
                      uint32_t ndocs, uint32_t *out_idx, uint32_t *out_n,
                      uint32_t *out_err, jsidx_stream_t stream);

/*
 * jsidx_build_noalloc -- jsidx_build for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and stream behaviour as
 * jsidx_build, for documents of at most JSIDX_NOALLOC_MAX_LEN bytes (larger
 * ones return JSIDX_E_TOO_LARGE and launch nothing).  The call never
 * allocates or frees memory: its workspace is a fixed device array inside the
 * library (168.5 KiB on every device the library runs on, held until the
 * process ends), zeroed by a small kernel on `stream` the first time the
 * device is used.  Every call on one device shares that array, so calls that
 * overlap in time on one device (on different streams, or from several host
 * threads without ordering) race and give wrong results; calls ordered on one
 * stream are safe.  It shares its kernels with jsidx_build.
 */
#define JSIDX_NOALLOC_MAX_LEN 268435440ull /* 256 MiB - 16 */
int jsidx_build_noalloc(const uint8_t *buf, uint64_t len, uint32_t *out_idx,
                        uint32_t *out_n, uint32_t *out_err,
                        jsidx_stream_t stream);

/*
 * jsidx_minify -- minify one document: drop the white-space characters
 * (TAB LF CR SPACE) outside strings and keep every other byte in order, the
 * paper's minified form of a document (its table of dataset sizes; its
 * appendix on the effect of minification).  A byte is inside a string from an
 * unescaped opening quote through the byte before the closing quote, with the
 * escapes and string ranges of Sec. 3.1.1 (Figs. 3 and 4); a backslash outside
 * strings escapes the next byte, which is still dropped if it is white space.
 *   buf      device pointer to `len` bytes (any alignment), 0 <= len < 2^32.
 *   out      device array of at least max(len, 1) bytes: the kept bytes; bytes
 *            past *out_n unspecified.
 *   out_n    device uint32: number of bytes kept.
 *   out_err  device uint32: the same flags as jsidx_build for these bytes
 *            (JSIDX_ERR_EMPTY: nothing is kept, which happens exactly when
 *            the index is empty).
 * Same stream, workspace and error behaviour as jsidx_build.
 */
int jsidx_minify(const uint8_t *buf, uint64_t len, uint8_t *out,
                 uint32_t *out_n, uint32_t *out_err, jsidx_stream_t stream);

/*
 * jsidx_minify_batch -- minify many independent documents in one launch.
 * Document d's kept bytes go to out[offsets[d] .. offsets[d] + out_n[d]);
 * out has at least max(offsets[ndocs], 1) bytes.  Arguments, reservation and
 * capacity behaviour as jsidx_build_batch; each document's results are
 * identical to jsidx_minify on that document.
 */
int jsidx_minify_batch(const uint8_t *bufs, const uint64_t *offsets,
                       uint32_t ndocs, uint8_t *out, uint32_t *out_n,
                       uint32_t *out_err, jsidx_stream_t stream);

/*
 * jsidx_scopes -- the scope links of a document's structural index: the
 * paper's tape links the start of each object or array to its end and back
 * (Sec. 3, Fig. 2).  Entries are taken in order with a bracket stack: an
 * opening bracket ({ or [) is pushed; a closing one (} or ]) is linked with
 * the opener on top, which is popped (JSIDX_ERR_MISMATCHED if their kinds
 * differ), or, with nothing open, left unlinked (JSIDX_ERR_UNBALANCED); an
 * opener still open at the end is unlinked (JSIDX_ERR_UNBALANCED).
 * It also checks the structure the way the paper's stage 2 does while it
 * builds the tape (Sec. 3.2): taking each entry as a token (a bracket, ':',
 * ',', a string at '"', any other byte an atom), the sequence must be one
 * JSON value -- each token allowed after the one before it, with a ','
 * followed by a key in an object and by a value in an array, a key followed
 * by ':' -- else JSIDX_ERR_SYNTAX, which an empty index, JSIDX_ERR_UNBALANCED
 * and JSIDX_ERR_MISMATCHED always imply.  Token contents (numbers, literals,
 * string escapes) are not checked.
 *   buf        device pointer to the document's `len` bytes, len < 2^32.
 *   idx        device array of the document's n index entries, as jsidx_build
 *              writes them (positions below len; a position at or past len
 *              counts as a non-bracket entry and is never read).
 *   out_match  device array of n uint32: the entry number of each bracket's
 *              partner, 0xFFFFFFFF for unlinked brackets and other entries.
 *   out_err    device uint32: 0 or the three flags above.
 * The computation is parallel (depth by a scan of clamped depth changes,
 * then each opener's partner is the first later entry of at most its depth)
 * and gives exactly the stack's links; the structure check then looks at each
 * entry, a few entries around it and the link of a closer just before a
 * comma.  A per-stream workspace of about 9 bytes per entry is allocated on
 * first use and grown as needed (synchronising the stream); after
 * jsidx_scopes_reserve for at least n entries the call never allocates or
 * synchronises, so it can be captured in a HIP graph.  Asynchronous on
 * `stream`.
 */
int jsidx_scopes(const uint8_t *buf, uint64_t len, const uint32_t *idx,
                 uint32_t n, uint32_t *out_match, uint32_t *out_err,
                 jsidx_stream_t stream);

/*
 * jsidx_scopes_batch -- jsidx_scopes for many independent documents in one
 * call (the paper's stage 2 takes each document on its own, Sec. 3.2; here
 * the documents' entries are laid end to end, the depth starts again at each
 * document's first entry, and a document's levels are offset past every
 * level of the documents before it, so that no link or check crosses into
 * another document).
 *   bufs       device pointer to the concatenated document bytes.
 *   offsets    device array of ndocs+1 nondecreasing uint64, as for
 *              jsidx_build_batch (document d is bufs[offsets[d] ..
 *              offsets[d+1])).
 *   ndocs      number of documents, >= 1.
 *   idx        device array: document d's n[d] entries at idx + offsets[d],
 *              positions relative to its first byte, as jsidx_build_batch
 *              writes them.
 *   n          device array of ndocs uint32: each document's entry count
 *              (jsidx_build_batch's out_n).
 *   out_match  device array laid out like idx: document d's links at
 *              out_match + offsets[d], entry numbers relative to the
 *              document (0xFFFFFFFF: unlinked or not a bracket).
 *   out_err    device array of ndocs uint32: each document's flags, exactly
 *              those jsidx_scopes gives for it alone.
 * Results per document are identical to jsidx_scopes on that document.
 * After jsidx_scopes_reserve(max_entries, max_ndocs) on the stream with
 * max_ndocs >= ndocs, the call never allocates or synchronises (it can be
 * captured in a HIP graph), and a batch with more than max_entries entries
 * in total is not linked: every out_err[d] is set to JSIDX_ERR_CAPACITY and
 * out_match is left as it was.  Without a reservation the call copies
 * offsets[0] and offsets[ndocs] to the host (synchronising the stream) and
 * sizes the workspace for one entry per byte (about 17 bytes per byte).
 * Returns JSIDX_E_INVAL for NULL pointers or ndocs == 0.
 */
int jsidx_scopes_batch(const uint8_t *bufs, const uint64_t *offsets,
                       uint32_t ndocs, const uint32_t *idx, const uint32_t *n,
                       uint32_t *out_match, uint32_t *out_err,
                       jsidx_stream_t stream);

/*
 * jsidx_scopes_reserve -- sizes the stream's scope workspace for documents
 * of up to max_entries index entries (jsidx_scopes) and for batches of up to
 * max_entries entries in total in up to max_ndocs documents
 * (jsidx_scopes_batch; 0 counts as 1): about 17 bytes per entry and 4 per
 * document.  Synchronises the stream if it has to grow the workspace.
 * Returns JSIDX_E_TOO_LARGE for max_entries >= 2^31, JSIDX_E_NOWORKSPACE if
 * the allocation fails (the stream then has no scope workspace).
 */
int jsidx_scopes_reserve(uint64_t max_entries, uint32_t max_ndocs,
                         jsidx_stream_t stream);

/*
 * jsidx_tape -- the tape of the paper's stage 2 (Sec. 3, Fig. 2; Sec. 3.2)
 * from a document's index and its scope links: 64-bit words, the top 8 bits a
 * tag character.  Word 0 is 'r' with the index of the last word, which is 'r'
 * with 0.  Then in index order: '{' or '[' with one plus the index of its
 * closing word, '}' or ']' with the index of its opening word, '"' with the
 * offset of the string in the string buffer (a 32-bit little-endian length,
 * then the UTF-8 bytes; escapes decoded, \uXXXX and surrogate pairs as
 * UTF-8), 't' 'f' 'n' for the literals, and numbers as two words: 'l' and
 * the int64 value, or 'd' and the binary64 value (correctly rounded, ties to
 * even).  ':' and ',' take no word.
 *   buf, len   device pointer to the document (len < 2^32 - 2^16).
 *   idx, n     device array of the n index entries (jsidx_build's output for
 *              this document), n < 2^31.
 *   match      device array of n links from jsidx_scopes on the same index;
 *              the brackets' words take their partners from it (0 for an
 *              unlinked bracket).
 *   out_tape   device array of at least 2n + 2 uint64.
 *   out_tape_n device uint64: the number of words written.
 *   out_str    device buffer of at least len + 2n + 4 bytes.
 *   out_str_n  device uint64: the string buffer's size.
 *   out_err    device uint32: 0 or JSIDX_ERR_NUMBER (an atom that is not a
 *              number per the grammar -- minus, integer part without leading
 *              zeros, fraction, exponent -- or not ended by white space, a
 *              structural character or the end; an integer outside
 *              [-2^63, 2^63); a double that rounds to infinity),
 *              JSIDX_ERR_STRING (a byte below 0x20, an unknown escape, a bad
 *              \u, a lone surrogate, no closing quote), JSIDX_ERR_LITERAL (an
 *              atom starting with t, f or n that is not exactly true, false
 *              or null).  Every atom and string is checked, each on its own.
 * The tape is the paper's only when jsidx_scopes reported no flag and out_err
 * is 0.  A per-stream workspace of about 21 bytes per entry is allocated on
 * first use and grown as needed (synchronising the stream); after
 * jsidx_tape_reserve for at least n entries the call never allocates or
 * synchronises (it can be captured in a HIP graph).  Asynchronous on
 * `stream`; returns JSIDX_E_INVAL for NULL pointers or sizes out of range.
 */
#define JSIDX_ERR_NUMBER 0x100u
#define JSIDX_ERR_STRING 0x200u
#define JSIDX_ERR_LITERAL 0x400u
int jsidx_tape(const uint8_t *buf, uint64_t len, const uint32_t *idx,
               uint32_t n, const uint32_t *match, uint64_t *out_tape,
               uint64_t *out_tape_n, uint8_t *out_str, uint64_t *out_str_n,
               uint32_t *out_err, jsidx_stream_t stream);

/*
 * jsidx_tape_batch -- jsidx_tape for many independent documents in one call
 * (stage 2 takes each token on its own once the index is known, Sec. 3.2).
 * The documents' tapes are laid end to end in out_tape, and their string
 * buffers end to end in out_str; each document's tape is exactly what
 * jsidx_tape writes for it alone (word 0 its own 'r', links and string
 * offsets relative to its own tape and string buffer; an empty document's
 * tape is its two 'r' words).
 *   bufs, offsets, ndocs   as for jsidx_build_batch; the batch's bytes
 *              (offsets[ndocs] - offsets[0]) must be below 2^32 - 2^16.
 *   idx, n     jsidx_build_batch's index (document d's n[d] entries at
 *              idx + offsets[d]) and counts.
 *   match      jsidx_scopes_batch's links, in the same layout.
 *   out_tape   device array of tape_cap uint64 (2 * (entries + ndocs)
 *              always suffice).
 *   out_str    device buffer of str_cap bytes (the batch's bytes plus twice
 *              its entries, plus 4, always suffice).
 *   out_pos    device array of 4 * ndocs uint64: for document d, the index
 *              of its first word in out_tape, its word count, the offset of
 *              its string buffer in out_str and that buffer's size.
 *   out_err    device array of ndocs uint32: each document's flags, those
 *              jsidx_tape gives for it alone.
 * After jsidx_tape_reserve(max_entries, max_ndocs) on the stream with
 * max_ndocs >= ndocs, the call never allocates or synchronises (it can be
 * captured in a HIP graph).  A batch with more than max_entries + ndocs
 * entries and empty documents, whose bytes reach 2^32 - 2^16, or whose tape or
 * strings exceed tape_cap or str_cap, is not written: every out_err[d] is
 * set to JSIDX_ERR_CAPACITY.  Without a reservation the call copies
 * offsets[0] and offsets[ndocs] to the host (synchronising the stream) and
 * sizes the workspace for one entry per byte.  Returns JSIDX_E_INVAL for
 * NULL pointers or ndocs == 0.
 */
int jsidx_tape_batch(const uint8_t *bufs, const uint64_t *offsets,
                     uint32_t ndocs, const uint32_t *idx, const uint32_t *n,
                     const uint32_t *match, uint64_t *out_tape,
                     uint64_t tape_cap, uint8_t *out_str, uint64_t str_cap,
                     uint64_t *out_pos, uint32_t *out_err,
                     jsidx_stream_t stream);

/*
 * jsidx_tape_reserve -- sizes the stream's tape workspace for documents of up
 * to max_entries index entries (jsidx_tape) and for batches of up to
 * max_entries entries in up to max_ndocs documents (jsidx_tape_batch; 0
 * counts as 1): about 34 bytes per entry and 50 per document.  Synchronises
 * the stream if it has to grow the workspace.  Returns JSIDX_E_TOO_LARGE for
 * max_entries >= 2^31, JSIDX_E_NOWORKSPACE if the allocation fails (the
 * stream then has no tape workspace).
 */
int jsidx_tape_reserve(uint64_t max_entries, uint32_t max_ndocs,
                       jsidx_stream_t stream);

/*
 * jsidx_reserve -- size the workspace of `stream` for inputs of up to
 * max_total_len bytes in total (single document or batch) in up to
 * max_ndocs documents, and switch batch calls on that stream to the
 * no-synchronisation mode described above.  Call it before capturing a HIP
 * graph so that the captured calls allocate nothing (a later jsidx_build
 * larger than the reservation still grows it).  The workspace (tile
 * descriptors and counters, plus 2 bits per input byte of deferred masks:
 * about a quarter of the input size) is owned by the library, kept per stream
 * until jsidx_release.  Its size depends on the bytes only: per-document
 * state lives in the caller's out_n and out_err, and documents are found
 * from the offsets in place, so max_ndocs is accepted and not used (0 is
 * allowed).  Returns JSIDX_E_NOWORKSPACE if the allocation fails; the
 * stream then has no workspace and the next call allocates one.
 */
int jsidx_reserve(uint64_t max_total_len, uint32_t max_ndocs,
                  jsidx_stream_t stream);

/* Bytes of workspace needed for total_len input bytes in ndocs documents
 * (ndocs does not change the size; see jsidx_reserve). */
size_t jsidx_workspace_bytes(uint64_t total_len, uint32_t ndocs);

/* Free the workspace of `stream` (synchronises the stream first). */
int jsidx_release(jsidx_stream_t stream);

/*
 * jsidx_stream_diag -- synchronise `stream` and return in *out_flags the
 * sticky diagnostic word of its workspace (0 = healthy; bit 0: a tile's wait
 * for its predecessor's carry gave up after about half a second, so some
 * results of that launch may be wrong -- never expected, it guards against a
 * hang).  Clears the word.
 */
int jsidx_stream_diag(jsidx_stream_t stream, uint32_t *out_flags);

/*
 * jsidx_set_tile_rows -- tuning: the tile size by input size, for later
 * batched launches (jsidx_build_batch, jsidx_minify, jsidx_minify_batch) on
 * every device and stream of the process (the autotuner of the Python package
 * measures and sets it).  jsidx_build and jsidx_build_noalloc run a kernel
 * with a fixed tile size (8 rows) and ignore the table.  A batched launch cuts
 * its input into tiles of `rows` rows of 2 KiB; one wave indexes a tile row
 * after row, so small tiles shorten each wave's serial work and large tiles
 * make fewer tiles (less per-tile work, fewer carries to resolve).
 *   rows_by_log2  host array of n entries: entry b applies to launches whose
 *                 span (bytes from the 16-byte granule holding the first byte
 *                 to the last byte) has floor(log2(span)) == b; 0 keeps the
 *                 built-in choice (the largest tile that still gives every
 *                 wave of the device one), otherwise 2, 4, 8 or 16.
 *   n             0..64; n == 0 restores the built-in choice everywhere.
 * Returns JSIDX_E_INVAL (table unchanged) for other values.  Results never
 * depend on the tile size.
 */
int jsidx_set_tile_rows(const uint8_t *rows_by_log2, uint32_t n);

/*
 * jsidx_set_variant -- the indexing kernel used by later jsidx_build and
 * jsidx_build_batch launches on every device and stream of the process: the
 * default (0) or a variant with one of the paper's stage-1 optimizations
 * turned off, as in its ablation (App. B, Table of optimizations):
 *   JSIDX_VARIANT_NAIVE_CLASSIFY  classes by one comparison per class
 *                                 character and byte, ORed together, instead
 *                                 of nibble logic (Sec. 3.1.2);
 *   JSIDX_VARIANT_XOR_LOOP        the in-string mask by toggling at each
 *                                 quote, one step per quote, instead of the
 *                                 shift/XOR ladder (the GPU has no carry-less
 *                                 multiply; Sec. 3.1.1);
 *   JSIDX_VARIANT_DIRECT_FLATTEN  every lane stores its own positions with a
 *                                 trailing-zero loop instead of staging dense
 *                                 rows in LDS (Sec. 3.1.4, Fig. 6).
 * Results never depend on the variant.  Returns JSIDX_E_INVAL (unchanged)
 * for any other value.  Minify always uses the default kernel.
 */
#define JSIDX_VARIANT_NAIVE_CLASSIFY 1u
#define JSIDX_VARIANT_XOR_LOOP 2u
#define JSIDX_VARIANT_DIRECT_FLATTEN 4u
int jsidx_set_variant(uint32_t variant);

/* Rows per tile that a batched launch over `span` bytes would use on the
 * current device (written to *out_rows). */
int jsidx_tile_rows(uint64_t span, uint32_t *out_rows);

/* Human-readable text for a status code. */
const char *jsidx_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* JSIDX_H */
