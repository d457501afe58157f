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
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

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

/* ---- The tape (Sec. 3, Fig. 2; stage 2, Sec. 3.2) ----------------------------
 * oracle_tape walks the index entries in order and writes the tape: 64-bit
 * words tagged with a character in bits 56..63.
 *   - root: word 0 is 'r' with the index of the last word, the last word 'r'
 *     with 0;
 *   - '{' or '[': the tag with one plus the index of its closing word; '}' or
 *     ']': the tag with the index of its opening word;
 *   - a string: '"' with the offset of its entry in the string buffer, which
 *     holds a 32-bit little-endian length and then the UTF-8 bytes;
 *   - true, false, null: 't', 'f', 'n';
 *   - a number: 'l' and the int64 value, or 'd' and the binary64 value.
 * ':' and ',' write nothing.
 * Each atom and string is checked on its own (Sec. 3.2: the locations of all
 * tokens are known, so none depends on another), and the flags collect the
 * errors of all of them: NUMBER (0x100), STRING (0x200), LITERAL (0x400).
 * The tape is written only when the structure is valid (oracle_structure) and
 * no flag is set; otherwise *tape_n and *str_n are 0.
 *
 * Numbers (Sec. 3.2, number grammar of the JSON specification): an optional
 * minus, then 0 or a digit 1-9 followed by digits, then optionally '.' and
 * digits, then optionally e/E, an optional sign and digits.  Without fraction
 * and exponent the number is an integer and must lie in [-2^63, 2^63).  With
 * either it is a double: the correctly rounded (nearest, ties to even)
 * binary64 value of the decimal, taken from the C library's strtod on the
 * validated text; a value that rounds to infinity is an error (1e309).  The
 * atom must end at white space, a structural character or the end of the
 * document.
 * Strings (Sec. 3.2.2): the bytes up to the closing quote; a byte below 0x20
 * is an error; escapes \" \\ \/ \b \f \n \r \t and \uXXXX (four hex digits),
 * where a high surrogate D800-DBFF must be followed by \u and a low surrogate
 * DC00-DFFF (the pair is one code point) and a lone surrogate is an error; the
 * code point is written as UTF-8.  A string that does not close before the
 * end of the document is an error.
 * Literals: an atom starting with t, f or n must be exactly true, false or
 * null, ending as numbers end (else LITERAL); every other atom is read as a
 * number (so ".1" or "abc" is a NUMBER error).
 * stack needs room for n entries; tape for 2n + 2 words; strbuf for len + 2n
 * bytes. */
#define OR_ERR_NUMBER 0x100u
#define OR_ERR_STRING 0x200u
#define OR_ERR_LITERAL 0x400u

static int atom_end(const uint8_t *buf, uint64_t len, uint64_t p) {
  return p >= len || is_whitespace(buf[p]) || is_structural(buf[p]);
}

static int hexval(uint8_t c) {
  if (c >= '0' && c <= '9') return c - '0';
  if (c >= 'a' && c <= 'f') return c - 'a' + 10;
  if (c >= 'A' && c <= 'F') return c - 'A' + 10;
  return -1;
}

/* four hex digits at p; -1 if not */
static int32_t hex4(const uint8_t *buf, uint64_t len, uint64_t p) {
  int32_t v = 0;
  if (p + 4 > len) return -1;
  for (int k = 0; k < 4; k++) {
    int h = hexval(buf[p + k]);
    if (h < 0) return -1;
    v = v * 16 + h;
  }
  return v;
}

static uint32_t put_utf8(uint8_t *out, uint32_t cp) {
  if (cp < 0x80) { out[0] = (uint8_t)cp; return 1; }
  if (cp < 0x800) { out[0] = (uint8_t)(0xC0 | (cp >> 6)); out[1] = (uint8_t)(0x80 | (cp & 0x3F)); return 2; }
  if (cp < 0x10000) {
    out[0] = (uint8_t)(0xE0 | (cp >> 12)); out[1] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
    out[2] = (uint8_t)(0x80 | (cp & 0x3F));
    return 3;
  }
  out[0] = (uint8_t)(0xF0 | (cp >> 18)); out[1] = (uint8_t)(0x80 | ((cp >> 12) & 0x3F));
  out[2] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F)); out[3] = (uint8_t)(0x80 | (cp & 0x3F));
  return 4;
}

/* The string whose opening quote is at q: decoded bytes to out (room for the
 * raw length), their count to *n.  Returns 0 or OR_ERR_STRING. */
static uint32_t decode_string(const uint8_t *buf, uint64_t len, uint64_t q, uint8_t *out, uint32_t *n) {
  uint64_t p = q + 1;
  uint32_t k = 0;
  *n = 0;
  for (;;) {
    if (p >= len) return OR_ERR_STRING;  /* never closed */
    uint8_t c = buf[p];
    if (c == '"') break;
    if (c < 0x20) return OR_ERR_STRING;
    if (c != '\\') { out[k++] = c; p++; continue; }
    if (p + 1 >= len) return OR_ERR_STRING;
    uint8_t e = buf[p + 1];
    p += 2;
    switch (e) {
      case '"': out[k++] = '"'; break;
      case '\\': out[k++] = '\\'; break;
      case '/': out[k++] = '/'; break;
      case 'b': out[k++] = 0x08; break;
      case 'f': out[k++] = 0x0C; break;
      case 'n': out[k++] = 0x0A; break;
      case 'r': out[k++] = 0x0D; break;
      case 't': out[k++] = 0x09; break;
      case 'u': {
        int32_t u = hex4(buf, len, p);
        if (u < 0) return OR_ERR_STRING;
        p += 4;
        uint32_t cp = (uint32_t)u;
        if (cp >= 0xDC00 && cp <= 0xDFFF) return OR_ERR_STRING;  /* lone low surrogate */
        if (cp >= 0xD800 && cp <= 0xDBFF) {
          if (p + 2 > len || buf[p] != '\\' || buf[p + 1] != 'u') return OR_ERR_STRING;
          int32_t lo = hex4(buf, len, p + 2);
          if (lo < 0xDC00 || lo > 0xDFFF) return OR_ERR_STRING;
          p += 6;
          cp = 0x10000u + ((cp - 0xD800u) << 10) + ((uint32_t)lo - 0xDC00u);
        }
        k += put_utf8(out + k, cp);
        break;
      }
      default: return OR_ERR_STRING;
    }
  }
  *n = k;
  return 0;
}

/* The number at p.  Returns 0 (with *is_int and the value in *bits) or
 * OR_ERR_NUMBER. */
static uint32_t parse_number(const uint8_t *buf, uint64_t len, uint64_t p0, int *is_int, uint64_t *bits) {
  uint64_t p = p0;
  int neg = 0, frac = 0, expo = 0;
  if (p < len && buf[p] == '-') { neg = 1; p++; }
  if (p >= len || buf[p] < '0' || buf[p] > '9') return OR_ERR_NUMBER;
  uint64_t int_start = p;
  if (buf[p] == '0') p++;
  else while (p < len && buf[p] >= '0' && buf[p] <= '9') p++;
  uint64_t int_end = p;
  if (p < len && buf[p] == '.') {
    frac = 1;
    p++;
    uint64_t s = p;
    while (p < len && buf[p] >= '0' && buf[p] <= '9') p++;
    if (p == s) return OR_ERR_NUMBER;
  }
  if (p < len && (buf[p] == 'e' || buf[p] == 'E')) {
    expo = 1;
    p++;
    if (p < len && (buf[p] == '+' || buf[p] == '-')) p++;
    uint64_t s = p;
    while (p < len && buf[p] >= '0' && buf[p] <= '9') p++;
    if (p == s) return OR_ERR_NUMBER;
  }
  if (!atom_end(buf, len, p)) return OR_ERR_NUMBER;
  if (!frac && !expo) {
    /* integer: magnitude at most 2^63 - 1, or 2^63 when negative */
    const uint64_t lim = neg ? (1ull << 63) : (1ull << 63) - 1;
    uint64_t m = 0;
    for (uint64_t i = int_start; i < int_end; i++) {
      uint64_t d = (uint64_t)(buf[i] - '0');
      if (m > (lim - d) / 10) return OR_ERR_NUMBER;
      m = m * 10 + d;
    }
    *is_int = 1;
    *bits = neg ? (uint64_t)0 - m : m;
    return 0;
  }
  /* double: strtod on a NUL-terminated copy of the validated text */
  size_t L = (size_t)(p - p0);
  char small[64];
  char *txt = L < sizeof(small) ? small : (char *)malloc(L + 1);
  if (!txt) return OR_ERR_NUMBER;
  memcpy(txt, buf + p0, L);
  txt[L] = 0;
  double v = strtod(txt, NULL);
  if (txt != small) free(txt);
  if (isinf(v)) return OR_ERR_NUMBER;
  memcpy(bits, &v, 8);
  *is_int = 0;
  return 0;
}

static uint32_t check_literal(const uint8_t *buf, uint64_t len, uint64_t p, uint8_t *tag) {
  static const char *const words[3] = {"true", "false", "null"};
  for (int w = 0; w < 3; w++) {
    size_t L = strlen(words[w]);
    if (p + L <= len && memcmp(buf + p, words[w], L) == 0 && atom_end(buf, len, p + L)) {
      *tag = (uint8_t)words[w][0];
      return 0;
    }
  }
  return OR_ERR_LITERAL;
}

static uint64_t tagged(uint8_t tag, uint64_t payload) { return ((uint64_t)tag << 56) | payload; }

uint32_t oracle_tape(const uint8_t *buf, uint64_t len, const uint32_t *idx, uint32_t n, uint64_t *tape,
                     uint64_t *tape_n, uint8_t *strbuf, uint64_t *str_n, uint32_t *stack) {
  uint32_t flags = 0;
  uint64_t t = 1, s = 0;
  uint32_t top = 0;
  const int structure_ok = oracle_structure(buf, idx, n, stack) == 0;
  for (uint32_t i = 0; i < n; i++) {
    const uint64_t p = idx[i];
    const uint8_t b = buf[p];
    if (b == '{' || b == '[') {
      stack[top++] = (uint32_t)t;
      tape[t++] = tagged(b, 0);
    } else if (b == '}' || b == ']') {
      if (structure_ok) {
        const uint32_t o = stack[--top];
        tape[o] |= t + 1;
        tape[t++] = tagged(b, o);
      }
    } else if (b == ':' || b == ',') {
      /* no tape word */
    } else if (b == '"') {
      uint32_t k = 0;
      uint32_t e = decode_string(buf, len, p, strbuf + s + 4, &k);
      flags |= e;
      memcpy(strbuf + s, &k, 4);  /* little-endian host */
      tape[t++] = tagged('"', s);
      s += 4 + (uint64_t)k;
    } else if (b != 't' && b != 'f' && b != 'n') {  /* a number, or an invalid atom */
      int is_int = 0;
      uint64_t bits = 0;
      uint32_t e = parse_number(buf, len, p, &is_int, &bits);
      flags |= e;
      tape[t++] = tagged(is_int ? 'l' : 'd', 0);
      tape[t++] = bits;
    } else {
      uint8_t tag = 0;
      flags |= check_literal(buf, len, p, &tag);
      tape[t++] = tagged(tag, 0);
    }
  }
  if (!structure_ok || flags) {
    *tape_n = 0;
    *str_n = 0;
    return flags;
  }
  tape[0] = tagged('r', t);
  tape[t] = tagged('r', 0);
  *tape_n = t + 1;
  *str_n = s;
  return flags;
}
