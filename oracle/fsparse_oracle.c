/*
 * CPU oracle for Matlab-compatible sparse assembly -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The HIP product path never links, loads or calls
 * it, and it shares no code with that path.
 *
 * What it computes is the plain definition of S = sparse(i,j,s,m,n)
 * (Engblom & Lukarski, Section 2.1): S(i_k, j_k) collects s_k, repeated index
 * pairs are summed, and the result is the compressed-column triple
 *   jcS[0..n]   column pointers, jcS[0] = 0, jcS[n] = nnz     (Section 2.1)
 *   irS[0..nnz) zero-offset row indices, increasing within a column
 *   prS[0..nnz) values
 * plus the inverse rank ("irank", Section 2.2, eqs. (2.2)-(2.3)): for every
 * triplet k the position of its pair in (irS, prS), here called slot[k].
 *
 * Summation order: the serial post-processing of the paper (appendix
 * "Post-processing: finalize CCS format") adds the contributions into a
 * zero-initialised prS in increasing k.  So prS[t] is the left fold
 * ((+0.0 + s_k1) + s_k2) + ... over the triplets k1 < k2 < ... of pair t,
 * carried out in the value type (double or float), round to nearest even.
 *
 * Steps, written for checking by eye rather than for speed:
 *   1. validate: every index >= 1 (appendix pre-processing listing) and, as m
 *      and n are resolved here, <= m resp. <= n;
 *   2. order the triplet numbers k by (column, row, k) with qsort -- the
 *      sort-then-sweep description of the problem in Section 2.1;
 *   3. sweep that order: a new (column,row) pair opens a new slot t with
 *      irS[t] = row-1 and prS[t] = +0.0; every triplet then adds its value to
 *      prS[slot] and records slot[k] = t; per-column pair counts accumulate;
 *   4. jcS is the running sum of the per-column pair counts.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math) -shared -fPIC.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_INDEX 1
#define ORACLE_E_ARG 2
#define ORACLE_E_NOMEM 3

typedef struct {
  int32_t col;
  int32_t row;
  int64_t k;
} okey;

static int okey_cmp(const void *pa, const void *pb) {
  const okey *a = (const okey *)pa, *b = (const okey *)pb;
  if (a->col != b->col) return a->col < b->col ? -1 : 1;
  if (a->row != b->row) return a->row < b->row ? -1 : 1;
  if (a->k != b->k) return a->k < b->k ? -1 : 1;
  return 0;
}

/* Dimensions as the pre-processing defines them: the largest row and column
 * index (0 when there are no triplets); any index below 1 is an error. */
int oracle_dims(const int32_t *ii, const int32_t *jj, int64_t len,
                int64_t *m, int64_t *n) {
  int64_t M = 0, N = 0;
  if (len < 0) return ORACLE_E_ARG;
  for (int64_t k = 0; k < len; k++) {
    if (ii[k] < 1 || jj[k] < 1) return ORACLE_E_INDEX;
    if (ii[k] > M) M = ii[k];
    if (jj[k] > N) N = jj[k];
  }
  *m = M;
  *n = N;
  return ORACLE_OK;
}

/* Steps 1-2: validation and the (column,row,k) order. Caller frees *out. */
static int ordered_keys(const int32_t *ii, const int32_t *jj, int64_t len,
                        int64_t m, int64_t n, okey **out) {
  if (len < 0 || m < 0 || n < 0) return ORACLE_E_ARG;
  for (int64_t k = 0; k < len; k++) {
    if (ii[k] < 1 || ii[k] > m || jj[k] < 1 || jj[k] > n)
      return ORACLE_E_INDEX;
  }
  okey *key = (okey *)malloc((size_t)(len > 0 ? len : 1) * sizeof(okey));
  if (!key) return ORACLE_E_NOMEM;
  for (int64_t k = 0; k < len; k++) {
    key[k].col = jj[k];
    key[k].row = ii[k];
    key[k].k = k;
  }
  qsort(key, (size_t)len, sizeof(okey), okey_cmp);
  *out = key;
  return ORACLE_OK;
}

/* Steps 3-4 for one value type.  irS/prS need room for len entries (the
 * number of distinct pairs never exceeds len); slot may be NULL. */
#define DEFINE_ASSEMBLE(NAME, VT)                                              \
  int NAME(const int32_t *ii, const int32_t *jj, const VT *ss, int64_t len,   \
           int64_t m, int64_t n, int32_t *jcS, int32_t *irS, VT *prS,         \
           int32_t *slot, int64_t *nnz) {                                     \
    okey *key = NULL;                                                          \
    int st = ordered_keys(ii, jj, len, m, n, &key);                            \
    if (st != ORACLE_OK) return st;                                            \
    int64_t *count = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));       \
    if (!count) {                                                              \
      free(key);                                                               \
      return ORACLE_E_NOMEM;                                                   \
    }                                                                          \
    int64_t t = -1;                                                            \
    int32_t pcol = 0, prow = 0;                                                \
    for (int64_t p = 0; p < len; p++) {                                        \
      const okey q = key[p];                                                   \
      if (t < 0 || q.col != pcol || q.row != prow) {                           \
        t++;                                                                   \
        pcol = q.col;                                                          \
        prow = q.row;                                                          \
        irS[t] = q.row - 1;                                                    \
        prS[t] = (VT)0.0;                                                      \
        count[q.col - 1]++;                                                    \
      }                                                                        \
      prS[t] = prS[t] + ss[q.k];                                               \
      if (slot) slot[q.k] = (int32_t)t;                                        \
    }                                                                          \
    jcS[0] = 0;                                                                \
    for (int64_t c = 0; c < n; c++)                                            \
      jcS[c + 1] = (int32_t)(jcS[c] + count[c]);                               \
    *nnz = t + 1;                                                              \
    free(count);                                                               \
    free(key);                                                                 \
    return ORACLE_OK;                                                          \
  }

DEFINE_ASSEMBLE(oracle_assemble_f64, double)
DEFINE_ASSEMBLE(oracle_assemble_f32, float)

/* The paper's serial post-processing (appendix, "Post-processing: finalize
 * CCS format") with the inverse rank known: prS starts at +0.0 and every
 * triplet, in increasing k, adds its value to the entry its slot names.
 * Given the slot map of an assembly, this is the value pass on its own, so
 * it re-assembles new values on a known pattern.  Every slot must lie in
 * [0, nnz). */
#define DEFINE_POSTPROCESS(NAME, VT)                                           \
  int NAME(const int32_t *slot, const VT *ss, int64_t len, int64_t nnz,       \
           VT *prS) {                                                          \
    if (len < 0 || nnz < 0) return ORACLE_E_ARG;                               \
    for (int64_t k = 0; k < len; k++)                                          \
      if (slot[k] < 0 || slot[k] >= nnz) return ORACLE_E_ARG;                  \
    for (int64_t t = 0; t < nnz; t++) prS[t] = (VT)0.0;                        \
    for (int64_t k = 0; k < len; k++) prS[slot[k]] = prS[slot[k]] + ss[k];     \
    return ORACLE_OK;                                                          \
  }

DEFINE_POSTPROCESS(oracle_postprocess_f64, double)
DEFINE_POSTPROCESS(oracle_postprocess_f32, float)
