/*
 * jsidx_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, byte-at-a-time CPU definition of stage 1 of the JSON parser
 * of Langdale & Lemire, "Parsing Gigabytes of JSON per Second" (Sec. 3.1):
 * the structural index (structural, opening-quote and pseudo-structural byte
 * positions) plus per-document validity flags.  Only tests/, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library; the product
 * path (the HIP library) never links or calls it, and the two share no code.
 *
 * Everything here is exact integer work.  One state variable is stepped per
 * input byte, in document order, with no blocking or reordering:
 *
 *   esc     -- this byte is escaped: the bytes just before it are a run of
 *              backslashes of odd length (Sec. 3.1.1, Fig. 3: only an odd run
 *              escapes what follows; an even run is a series of escaped
 *              backslashes).
 *   in_str  -- inclusive prefix XOR of the unescaped quotes seen so far
 *              (Sec. 3.1.1, Fig. 4: an opening quote is inside the string
 *              range, a closing quote is outside it).
 *   pred    -- the previous byte was structural, white space or an unescaped
 *              quote (Sec. 3.1.3, Fig. 5: the candidates for pseudo-structural
 *              characters are the successors of such bytes).  The byte before
 *              the document counts as white space, so that a scalar root value
 *              is indexed (reading of the paper, which never shows a document
 *              that does not start with a brace).
 *
 * Byte classes (Sec. 3.1.2, Table "vectorized classification"):
 *   structural  , : [ ] { }      (0x2C 0x3A 0x5B 0x5D 0x7B 0x7D)
 *   white space TAB LF CR SPACE  (0x09 0x0A 0x0D 0x20)
 *   quote 0x22, backslash 0x5C, everything else "other" (incl. bytes >= 0x80).
 *
 * A byte i is emitted into the index (Sec. 3.1.3, last row of Fig. 5) iff
 *   - it is an unescaped quote that opens a string, or
 *   - it is a structural byte outside strings, or
 *   - it is outside strings, is neither white space, structural nor an
 *     unescaped quote, and its predecessor set `pred` (pseudo-structural).
 * Closing quotes are removed (last step of Fig. 5).
 *
 * UTF-8 validation (Sec. 3.1.5, Table "unicode"): the document must be a
 * concatenation of the byte sequences that table lists; a multi-byte sequence
 * cut off by the end of the document is an error.  The check never changes
 * the index.
 *
 * Flags at end of document (bit values match include/jsidx.h by definition,
 * not by sharing a header):
 *   0x1 UTF8             not a concatenation of well-formed sequences
 *   0x2 UNCLOSED_STRING  in_str is set after the last byte
 *   0x4 TRAILING_ESCAPE  the document ends with an odd run of backslashes
 *   0x8 EMPTY            the index is empty
 */
#include <stddef.h>
#include <stdint.h>

#define OR_ERR_UTF8 0x1u
#define OR_ERR_UNCLOSED_STRING 0x2u
#define OR_ERR_TRAILING_ESCAPE 0x4u
#define OR_ERR_EMPTY 0x8u

/* ---- UTF-8: the rows of the paper's table of well-formed sequences ----
 * Each row gives the accepted range of the first byte and of each following
 * byte; a row with `len` bytes uses the first `len` ranges. */
struct utf8_row {
  int len;
  uint8_t lo[4];
  uint8_t hi[4];
};

static const struct utf8_row UTF8_ROWS[] = {
    {1, {0x00, 0, 0, 0}, {0x7F, 0, 0, 0}},
    {2, {0xC2, 0x80, 0, 0}, {0xDF, 0xBF, 0, 0}},
    {3, {0xE0, 0xA0, 0x80, 0}, {0xE0, 0xBF, 0xBF, 0}},
    {3, {0xE1, 0x80, 0x80, 0}, {0xEC, 0xBF, 0xBF, 0}},
    {3, {0xED, 0x80, 0x80, 0}, {0xED, 0x9F, 0xBF, 0}},
    {3, {0xEE, 0x80, 0x80, 0}, {0xEF, 0xBF, 0xBF, 0}},
    {4, {0xF0, 0x90, 0x80, 0x80}, {0xF0, 0xBF, 0xBF, 0xBF}},
    {4, {0xF1, 0x80, 0x80, 0x80}, {0xF3, 0xBF, 0xBF, 0xBF}},
    {4, {0xF4, 0x80, 0x80, 0x80}, {0xF4, 0x8F, 0xBF, 0xBF}},
};
#define N_UTF8_ROWS (sizeof(UTF8_ROWS) / sizeof(UTF8_ROWS[0]))

/* Length of the well-formed sequence starting at buf[i], or 0 if none of the
 * table's rows matches there (including a sequence cut off at `len`). */
static int utf8_match(const uint8_t *buf, uint64_t len, uint64_t i) {
  for (size_t r = 0; r < N_UTF8_ROWS; r++) {
    const struct utf8_row *row = &UTF8_ROWS[r];
    if (buf[i] < row->lo[0] || buf[i] > row->hi[0]) continue;
    if (i + (uint64_t)row->len > len) return 0; /* truncated at end */
    for (int k = 1; k < row->len; k++) {
      uint8_t b = buf[i + (uint64_t)k];
      if (b < row->lo[k] || b > row->hi[k]) return 0;
    }
    return row->len;
  }
  return 0;
}

/* 1 if buf[0..len) is a concatenation of the table's sequences. */
int oracle_utf8_valid(const uint8_t *buf, uint64_t len) {
  uint64_t i = 0;
  while (i < len) {
    int n = utf8_match(buf, len, i);
    if (n == 0) return 0;
    i += (uint64_t)n;
  }
  return 1;
}

static int is_structural(uint8_t b) {
  return b == 0x2C || b == 0x3A || b == 0x5B || b == 0x5D || b == 0x7B || b == 0x7D;
}

static int is_whitespace(uint8_t b) {
  return b == 0x09 || b == 0x0A || b == 0x0D || b == 0x20;
}

/* Index one document.  out_idx must have room for `len` entries (one per
 * byte at most).  Returns the number of entries written; *out_err receives the
 * flags.  Positions are relative to buf. */
uint32_t oracle_index(const uint8_t *buf, uint64_t len, uint32_t *out_idx,
                      uint32_t *out_err) {
  int esc = 0, in_str = 0, pred = 1;
  uint32_t n = 0;
  for (uint64_t i = 0; i < len; i++) {
    uint8_t b = buf[i];
    int c = is_structural(b);
    int w = is_whitespace(b);
    int q = (b == 0x22) && !esc;
    if (q) in_str ^= 1;
    int r = in_str;
    int emit = (q && r) || (!r && c) || (!r && !q && !w && !c && pred);
    if (emit) out_idx[n++] = (uint32_t)i;
    pred = c || w || q;
    esc = (b == 0x5C) && !esc;
  }
  uint32_t err = 0;
  if (!oracle_utf8_valid(buf, len)) err |= OR_ERR_UTF8;
  if (in_str) err |= OR_ERR_UNCLOSED_STRING;
  if (esc) err |= OR_ERR_TRAILING_ESCAPE;
  if (n == 0) err |= OR_ERR_EMPTY;
  *out_err = err;
  return n;
}

/* Index a batch: document d is bufs[offsets[d] .. offsets[d+1]), indexed on its
 * own with fresh state.  Its entries go to out_idx[offsets[d] ...] (so out_idx
 * holds offsets[ndocs] entries) and are
 * relative to the document start; out_n[d] and out_err[d] get its count and
 * flags.  Returns 0, or -1 if the offsets decrease. */
int oracle_index_batch(const uint8_t *bufs, const uint64_t *offsets,
                       uint32_t ndocs, uint32_t *out_idx, uint32_t *out_n,
                       uint32_t *out_err) {
  for (uint32_t d = 0; d < ndocs; d++) {
    if (offsets[d + 1] < offsets[d]) return -1;
  }
  for (uint32_t d = 0; d < ndocs; d++) {
    uint64_t a = offsets[d], e = offsets[d + 1];
    out_n[d] = oracle_index(bufs + a, e - a, out_idx + a, &out_err[d]);
  }
  return 0;
}

/* Minify one document: the paper's "minified" form of its dataset-size table
 * omits the white-space characters outside quotes.  Byte i is kept iff it is
 * not white space or it lies inside a string, with in_str and esc stepped
 * exactly as in oracle_index (the opening quote through the byte before the
 * closing quote are inside).  Kept bytes go to out in order (out has room for
 * len bytes); returns their number.  *out_err gets the flags of oracle_index
 * for the same bytes, with EMPTY meaning that nothing is kept. */
uint32_t oracle_minify(const uint8_t *buf, uint64_t len, uint8_t *out,
                       uint32_t *out_err) {
  int esc = 0, in_str = 0;
  uint32_t n = 0;
  for (uint64_t i = 0; i < len; i++) {
    uint8_t b = buf[i];
    int q = (b == 0x22) && !esc;
    if (q) in_str ^= 1;
    if (!is_whitespace(b) || in_str) out[n++] = b;
    esc = (b == 0x5C) && !esc;
  }
  uint32_t err = 0;
  if (!oracle_utf8_valid(buf, len)) err |= OR_ERR_UTF8;
  if (in_str) err |= OR_ERR_UNCLOSED_STRING;
  if (esc) err |= OR_ERR_TRAILING_ESCAPE;
  if (n == 0) err |= OR_ERR_EMPTY;
  *out_err = err;
  return n;
}

/* Minify a batch: document d's kept bytes go to out[offsets[d] ...], out_n[d]
 * and out_err[d] get its count and flags.  Returns 0, or -1 if the offsets
 * decrease. */
int oracle_minify_batch(const uint8_t *bufs, const uint64_t *offsets,
                        uint32_t ndocs, uint8_t *out, uint32_t *out_n,
                        uint32_t *out_err) {
  for (uint32_t d = 0; d < ndocs; d++) {
    if (offsets[d + 1] < offsets[d]) return -1;
  }
  for (uint32_t d = 0; d < ndocs; d++) {
    uint64_t a = offsets[d], e = offsets[d + 1];
    out_n[d] = oracle_minify(bufs + a, e - a, out + a, &out_err[d]);
  }
  return 0;
}

/* Scope matching over a document's structural index (the scope links of the
 * tape, Sec. 3 and Fig. 2: a scope start is linked to its end and back).  The
 * entries are taken in order with a stack: an opening bracket ( { or [ ) is
 * pushed; a closing bracket ( } or ] ) is linked with the entry on top of the
 * stack, which is popped, and sets MISMATCHED if their kinds differ; a closing
 * bracket with the stack empty is left unlinked and sets UNBALANCED, as does
 * any opening bracket still on the stack at the end.  match[i] receives the
 * entry number of i's partner, or 0xFFFFFFFF for unlinked brackets and for
 * entries that are not brackets.  stack must have room for n entries.
 * Returns the flags (0x10 UNBALANCED, 0x20 MISMATCHED). */
uint32_t oracle_scopes(const uint8_t *buf, const uint32_t *idx, uint32_t n,
                       uint32_t *match, uint32_t *stack) {
  uint32_t top = 0, err = 0;
  for (uint32_t i = 0; i < n; i++) {
    uint8_t b = buf[idx[i]];
    match[i] = 0xFFFFFFFFu;
    if (b == 0x7B || b == 0x5B) {
      stack[top++] = i;
    } else if (b == 0x7D || b == 0x5D) {
      if (top == 0) {
        err |= 0x10u;
      } else {
        uint32_t j = stack[--top];
        match[i] = j;
        match[j] = i;
        if ((buf[idx[j]] == 0x7B) != (b == 0x7D)) err |= 0x20u;
      }
    }
  }
  if (top) err |= 0x10u;
  return err;
}

/* Structure of a document's index entries against the JSON grammar (the
 * structural-sequence check that follows the index, Sec. 3.2): each entry is a
 * token -- { } [ ] : , an opening quote (a string) or anything else (the start
 * of a number or literal, an "atom") -- and the tokens must form exactly one
 * value: objects hold "string : value" members separated by commas, arrays
 * hold values separated by commas, nothing follows the root value, and the
 * document is not empty.  Token contents (digits, escapes) are not checked.
 * Returns 0x40 (SYNTAX) if the sequence is not valid, else 0.  stack needs
 * room for n entries. */
enum { OT_OBJ = 1, OT_ARR, OT_CLOSE_OBJ, OT_CLOSE_ARR, OT_COLON, OT_COMMA, OT_STR, OT_ATOM };
enum { ST_VALUE, ST_DONE, ST_KEY_OR_CLOSE, ST_COLON, ST_OBJ_VALUE, ST_OBJ_NEXT, ST_KEY,
       ST_VALUE_OR_CLOSE, ST_ARR_VALUE, ST_ARR_NEXT };

static int token_of(uint8_t b) {
  switch (b) {
    case 0x7B: return OT_OBJ;
    case 0x5B: return OT_ARR;
    case 0x7D: return OT_CLOSE_OBJ;
    case 0x5D: return OT_CLOSE_ARR;
    case 0x3A: return OT_COLON;
    case 0x2C: return OT_COMMA;
    case 0x22: return OT_STR;
    default: return OT_ATOM;
  }
}

uint32_t oracle_structure(const uint8_t *buf, const uint32_t *idx, uint32_t n,
                          uint32_t *stack) {
  /* stack holds, per open scope, the state to return to in the parent */
  uint32_t top = 0;
  int st = ST_VALUE;  /* the root expects one value */
  for (uint32_t i = 0; i < n; i++) {
    int t = token_of(buf[idx[i]]);
    int value_start = (t == OT_OBJ || t == OT_ARR || t == OT_STR || t == OT_ATOM);
    switch (st) {
      case ST_VALUE: case ST_OBJ_VALUE: case ST_ARR_VALUE: case ST_VALUE_OR_CLOSE:
        if (st == ST_VALUE_OR_CLOSE && t == OT_CLOSE_ARR) {
          if (top == 0) return 0x40u;
          st = (int)stack[--top];
          break;
        }
        if (!value_start) return 0x40u;
        {
          int after = st == ST_VALUE ? ST_DONE : (st == ST_OBJ_VALUE ? ST_OBJ_NEXT : ST_ARR_NEXT);
          if (t == OT_OBJ) { stack[top++] = (uint32_t)after; st = ST_KEY_OR_CLOSE; }
          else if (t == OT_ARR) { stack[top++] = (uint32_t)after; st = ST_VALUE_OR_CLOSE; }
          else st = after;
        }
        break;
      case ST_KEY_OR_CLOSE: case ST_KEY:
        if (st == ST_KEY_OR_CLOSE && t == OT_CLOSE_OBJ) {
          if (top == 0) return 0x40u;
          st = (int)stack[--top];
          break;
        }
        if (t != OT_STR) return 0x40u;
        st = ST_COLON;
        break;
      case ST_COLON:
        if (t != OT_COLON) return 0x40u;
        st = ST_OBJ_VALUE;
        break;
      case ST_OBJ_NEXT:
        if (t == OT_COMMA) { st = ST_KEY; break; }
        if (t != OT_CLOSE_OBJ || top == 0) return 0x40u;
        st = (int)stack[--top];
        break;
      case ST_ARR_NEXT:
        if (t == OT_COMMA) { st = ST_ARR_VALUE; break; }
        if (t != OT_CLOSE_ARR || top == 0) return 0x40u;
        st = (int)stack[--top];
        break;
      default: /* ST_DONE: nothing may follow the root value */
        return 0x40u;
    }
  }
  return st == ST_DONE ? 0u : 0x40u;
}
