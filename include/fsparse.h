/*
 * fsparse.h -- C ABI of the MI355X (gfx950) sparse-assembly library.
 *
 * The library computes the Matlab call S = sparse(i, j, s, m, n, nzmax)
 * (Engblom & Lukarski, "Fast Matlab compatible sparse assembly on multicore
 * computers", Section 2.1): raw triplets (ii[k], jj[k], ss[k]), k = 0..len-1,
 * with unit-offset indices (Section 2.2, listing "Input format"), become the
 * compressed-column arrays
 *     jcS[0..n]    column pointers, jcS[0] = 0, jcS[n] = nnz     (Section 2.1)
 *     irS[0..nnz)  zero-offset row indices, strictly increasing per column
 *     prS[0..nnz)  values; repeated (i,j) pairs are summed
 * and, on request, the inverse rank slot[k] = position of triplet k in
 * (irS, prS) (the paper's "irank", Section 2.2, eqs. (2.2)-(2.3)).
 *
 * Conventions shared by every entry point
 *  - Every array argument is HIP device memory owned by the caller unless it
 *    is marked "host".  The library never allocates device memory; scratch
 *    comes from the caller's workspace `ws` (fsparse_assemble_noalloc uses
 *    a fixed device array inside the library instead).
 *  - Work is stream-ordered on `stream`.  The calls that assemble or find
 *    dimensions wait for the stream to read back result sizes and the error
 *    flags (each call states how often); fsparse_assemble and its variants
 *    do not with FSPARSE_NO_SYNC.  Re-assembly, backward and index narrowing
 *    never synchronise.
 *  - Values are IEEE binary64 (FSPARSE_F64) or binary32 (FSPARSE_F32); the sum
 *    of a repeated pair is computed in that type.
 *  - In the default ordered mode the contributions to prS[t] are added from
 *    +0.0 in increasing k, the order of the paper's serial post-processing
 *    (appendix, "Post-processing: finalize CCS format"), so results are
 *    bit-identical from run to run.  FSPARSE_ATOMIC adds them with device
 *    atomics in an unspecified order instead.
 *  - Entries whose sum is zero are kept (nnz counts distinct index pairs,
 *    Section 2.2: nnz = 1 + max irank), unless FSPARSE_DROP_ZEROS asks for
 *    Matlab's convention of storing no zeros.
 *  - Functions return a status and never abort.  After an error the output
 *    arrays hold unspecified data.
 *  - len, m, n and nnz must stay below 2^31.
 */
#ifndef FSPARSE_H_
#define FSPARSE_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FSPARSE_F64 = 0, FSPARSE_F32 = 1 } fsparse_dtype;

/* flags */
enum {
  FSPARSE_ORDERED = 0u,    /* increasing-k fold, bit-exact (default)       */
  FSPARSE_ATOMIC = 1u,     /* device atomics, order unspecified            */
  FSPARSE_DROP_ZEROS = 2u, /* fresh calls: remove pairs whose sum is zero  */
  FSPARSE_NO_SYNC = 4u     /* fresh calls: queue the work, do not wait     */
};

typedef enum {
  FSPARSE_OK = 0,
  FSPARSE_E_INDEX = 1,    /* an index < 1, or > m / > n                      */
  FSPARSE_E_ARG = 2,      /* NULL pointer, negative or too large size, ...   */
  FSPARSE_E_CAPACITY = 3, /* output or workspace too small; info has sizes   */
  FSPARSE_E_PLAN = 4,     /* plan does not match the call                    */
  FSPARSE_E_HIP = 5       /* a HIP runtime call failed                       */
} fsparse_status;

/* Host-side sizes of one assembled matrix. */
typedef struct {
  int64_t m, n;   /* resolved dimensions                                    */
  int64_t nnz;    /* number of distinct (i,j) pairs                          */
  int64_t nzmax;  /* Matlab capacity: max(nzmax argument, nnz)               */
} fsparse_info;

/* Opaque host-side handle for pattern re-use (see fsparse_assemble). */
typedef struct fsparse_plan fsparse_plan;

/* Library version string (static storage). */
const char *fsparse_version(void);

/* Human-readable name of a status code (static storage). */
const char *fsparse_status_string(int status);

/* What failed behind the last FSPARSE_E_HIP returned on the calling host
 * thread: the stage or runtime call and the HIP error name ("" if none).
 * Thread-local storage, valid until that thread's next call. */
const char *fsparse_last_error(void);

/*
 * Bytes of device workspace that fsparse_assemble (nb = 1) or
 * fsparse_assemble_batched (nb matrices) needs for `len` triplets in total
 * and `ncols` columns in total (sum of n over the matrices).  The size does
 * not depend on m or on the values.  Returns 0 for negative arguments.
 */
size_t fsparse_workspace_bytes(int64_t len, int64_t ncols, int32_t nb,
                               fsparse_dtype dt);

/*
 * Default dimensions (Section 2.2 and the appendix pre-processing listing):
 * m = largest row index, n = largest column index, both 0 when len == 0.
 * Any index below 1 gives FSPARSE_E_INDEX.  ws needs at least 256 bytes.
 * Waits for the stream.
 */
fsparse_status fsparse_dims(const int32_t *ii, const int32_t *jj, int64_t len,
                            int64_t *m /* host out */, int64_t *n /* host out */,
                            void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Fresh assembly S = sparse(ii, jj, ss, m, n, nzmax).
 *
 *  ii, jj   [len] int32, unit-offset row / column indices
 *  ss       [len] values of type dt
 *  m, n     dimensions; a negative value asks for the default (largest
 *           index, computed with one extra pass and one extra wait).  With
 *           given dimensions every index must lie in [1,m] x [1,n].
 *  nzmax    Matlab capacity request; only reported back in info->nzmax.
 *  flags    FSPARSE_ORDERED or FSPARSE_ATOMIC (how prS is summed), optionally
 *           | FSPARSE_DROP_ZEROS: a Matlab sparse matrix stores no zeros, so
 *           the pairs whose sum is +0 or -0 are removed after the fold (the
 *           paper keeps them; this option gives Matlab's result).  Then
 *           info->nnz, jcS, irS, prS describe the kept pairs, slot[k] is the
 *           kept position or -1, cap must still hold every distinct pair
 *           (E_CAPACITY reports that count), the call waits twice, and a
 *           plan cannot be made (E_ARG: the pattern depends on the values).
 *  jcS      [jcS_cap >= n+1] out, column pointers
 *  irS,prS  [cap] out; cap >= nnz is required.  cap = len always suffices.
 *           When cap < nnz the call returns FSPARSE_E_CAPACITY with the
 *           required sizes in *info, and can be repeated with larger arrays.
 *  slot     [len] out, k -> position in (irS, prS); may be NULL.
 *  ws       device workspace of fsparse_workspace_bytes(len, n, 1, dt) bytes
 *           (with default n, size it for an upper bound of n).
 *  plan     NULL, or receives a plan for fsparse_assemble_reuse.  A plan
 *           keeps pointers into ws (the sorted triplet order and segment
 *           starts) and to slot; those buffers must outlive the plan and must
 *           not be reused for another call while the plan is in use.
 *  info     host out, may be NULL.
 * Waits for the stream once (to read nnz and the error flags), except with
 * FSPARSE_NO_SYNC:
 *  - The call queues its work on `stream` and returns FSPARSE_OK without
 *    waiting, so it can be issued ahead of later work (and from code that
 *    must not block).  Index and capacity errors are not known yet: they,
 *    and nnz, stay in the control block at the start of ws, and
 *    fsparse_assemble_status(ws, ...) reports them once the stream gets
 *    there; nnz is also jcS[n].  info->nnz is set to -1.
 *  - m and n must be given (the defaults take a wait), cap must be at least
 *    len (so no capacity retry can be needed: E_CAPACITY otherwise, with
 *    info->nnz = len), and FSPARSE_DROP_ZEROS is refused (E_ARG; the kept
 *    count is read back between two passes).
 *  - Triplets are placed in counted bins (the one-pass fixed-capacity bins
 *    may overflow, which needs a redo that the host decides).
 *  - A plan may be made; it reads nnz from ws where it needs it, and
 *    fsparse_plan_query reads it back with a blocking copy.
 * The same flag works for fsparse_assemble_f64idx, fsparse_assemble_expand
 * and fsparse_assemble_complex.
 */
fsparse_status fsparse_assemble(const int32_t *ii, const int32_t *jj,
                                const void *ss, fsparse_dtype dt, int64_t len,
                                int64_t m, int64_t n, int64_t nzmax,
                                unsigned flags, int32_t *jcS, int64_t jcS_cap,
                                int32_t *irS, void *prS, int64_t cap,
                                int32_t *slot, void *ws, size_t ws_bytes,
                                fsparse_plan **plan, fsparse_info *info,
                                hipStream_t stream);

/*
 * Fresh assembly for callers that cannot allocate memory (code that must
 * not call hipMalloc or any allocating routine: tight serving loops,
 * harnesses that forbid allocation).  The same computation and outputs as
 * fsparse_assemble, but the workspace is a device array inside the library
 * of FSPARSE_NOALLOC_SCRATCH_BYTES (64 MiB) that every GPU the library runs
 * on holds until the process ends; the call itself allocates nothing.
 *  - m and n must be given (>= 0; the default dimensions take a pass of
 *    their own), flags is FSPARSE_ORDERED or FSPARSE_ATOMIC, no plan.
 *  - cap >= len (every distinct pair fits, no capacity retry), else
 *    FSPARSE_E_CAPACITY with info->nnz = len.
 *  - fsparse_workspace_bytes(len, n, 1, dt) must not exceed
 *    FSPARSE_NOALLOC_SCRATCH_BYTES (about 1.3M fp64 triplets), else
 *    FSPARSE_E_CAPACITY before any work is queued.
 *  - Waits for the stream once (to read nnz and the error flags into info).
 * All calls on one GPU share that GPU's array, and a call leaves its
 * contents behind (the next call clears what it needs): calls that overlap
 * on one GPU (other host threads, other streams) race and must not be made.
 */
#define FSPARSE_NOALLOC_SCRATCH_BYTES (64u << 20)
fsparse_status fsparse_assemble_noalloc(const int32_t *ii, const int32_t *jj,
                                        const void *ss, fsparse_dtype dt,
                                        int64_t len, int64_t m, int64_t n,
                                        int64_t nzmax, unsigned flags,
                                        int32_t *jcS, int64_t jcS_cap,
                                        int32_t *irS, void *prS, int64_t cap,
                                        int32_t *slot, fsparse_info *info,
                                        hipStream_t stream);

/*
 * Status of a call made with FSPARSE_NO_SYNC on workspace ws: waits for
 * `stream`, then returns FSPARSE_E_INDEX (an index below 1 or beyond m/n),
 * FSPARSE_E_CAPACITY, or FSPARSE_OK, and sets info->nnz (may be NULL) to the
 * number of distinct pairs.  Only info->nnz is written.
 */
fsparse_status fsparse_assemble_status(const void *ws, fsparse_info *info,
                                       hipStream_t stream);

/*
 * Index arrays of a wider integer type narrowed to the int32 the calls take
 * (the validation of the pre-processing, Section 2.2, for integer input):
 * dst[k] = src[k] when 1 <= src[k] <= 2^31 - 1, else 0, which every call
 * then rejects with FSPARSE_E_INDEX as an index below 1 (an out-of-range
 * value never wraps into range).
 *  src       [len] device, of type src_type
 *  dst       [len] device int32 out (not overlapping src)
 * Never waits.
 */
enum { FSPARSE_IDX_I64 = 0, FSPARSE_IDX_U32 = 1, FSPARSE_IDX_U64 = 2 };
fsparse_status fsparse_indices_i32(const void *src, int32_t src_type,
                                   int64_t len, int32_t *dst,
                                   hipStream_t stream);

/*
 * Complex values (Matlab compatibility, Section 1).  Matlab's classic
 * external interface holds a complex sparse matrix as one pattern and two
 * value arrays, real and imaginary parts; the paper's sr and prS are the
 * real one.  Complex addition rounds the real and imaginary sums
 * separately, so both parts follow eq. (2.3) on the same pattern: every
 * pair's parts are summed from +0 in increasing k.
 *  sr, si   [len] device, real and imaginary parts, both of dtype dt.
 *  prS, piS [cap] device out, the real and imaginary sums.
 * Every other argument as for fsparse_assemble.  The imaginary parts are
 * folded along the sorted order the real pass leaves in ws (so ws must be
 * fsparse_workspace_bytes(len, n, 1, dt), as always).  FSPARSE_ATOMIC sums
 * both parts with atomics through the slot map.  FSPARSE_DROP_ZEROS removes
 * a pair only when both sums are zero, and compacts piS with prS (no plan).
 * A plan, when asked for, re-assembles one part per fsparse_assemble_reuse
 * call.  Outputs are ordered on the stream; the call waits once, for nnz.
 */
fsparse_status fsparse_assemble_complex(const int32_t *ii, const int32_t *jj,
                                        const void *sr, const void *si,
                                        fsparse_dtype dt, int64_t len,
                                        int64_t m, int64_t n, int64_t nzmax,
                                        unsigned flags, int32_t *jcS,
                                        int64_t jcS_cap, int32_t *irS,
                                        void *prS, void *piS, int64_t cap,
                                        int32_t *slot, void *ws, size_t ws_bytes,
                                        fsparse_plan **plan, fsparse_info *info,
                                        hipStream_t stream);

/*
 * Logical values (Matlab compatibility, Section 1).  A Matlab logical
 * matrix stores only true entries, and adding logical values gives true
 * when any of them is true.  So the result holds the pairs that have at
 * least one true triplet, rows increasing within columns as for real
 * values, each with value true.
 *  sl       [len] device bytes, nonzero = true (torch.bool or uint8).
 *  prS      [cap] device out, uint8: 1 for every stored pair.
 *  slot     [len] device out or NULL: the stored pair of triplet k, or -1
 *           when its pair has no true triplet.
 *  cap      irS/prS capacity; it must hold every distinct pair before the
 *           pairs without a true triplet are removed (cap = len always
 *           suffices); E_CAPACITY reports that count in info->nnz.
 *  ws       at least fsparse_logical_workspace_bytes(len, n) bytes.
 * Dimensions default to the largest indices, true or not.  info->nnz is the
 * number of stored pairs.  Waits for the stream twice.  No plan: the
 * pattern depends on the values.
 */
size_t fsparse_logical_workspace_bytes(int64_t len, int64_t ncols);
fsparse_status fsparse_assemble_logical(const int32_t *ii, const int32_t *jj,
                                        const uint8_t *sl, int64_t len,
                                        int64_t m, int64_t n, int64_t nzmax,
                                        int32_t *jcS, int64_t jcS_cap,
                                        int32_t *irS, uint8_t *prS, int64_t cap,
                                        int32_t *slot, void *ws, size_t ws_bytes,
                                        fsparse_info *info, hipStream_t stream);

/*
 * Double-valued indices (Matlab's default array type; the pre-processing of
 * Section 2.2 and its appendix listings, which check and convert them).
 * The same as fsparse_assemble / fsparse_dims with ii and jj given as
 * [len] doubles holding unit-offset indices.  An index must be a whole
 * number in [1, 2^31 - 1] (and within [1,m] / [1,n] when those are given):
 * a fraction, NaN, an infinity or a value below 1 gives FSPARSE_E_INDEX,
 * like an index out of range.  The conversion happens as the passes read
 * the indices; no int32 copy is made.
 */
fsparse_status fsparse_dims_f64idx(const double *ii, const double *jj,
                                   int64_t len, int64_t *m /* host out */,
                                   int64_t *n /* host out */, void *ws,
                                   size_t ws_bytes, hipStream_t stream);
fsparse_status fsparse_assemble_f64idx(const double *ii, const double *jj,
                                       const void *ss, fsparse_dtype dt,
                                       int64_t len, int64_t m, int64_t n,
                                       int64_t nzmax, unsigned flags,
                                       int32_t *jcS, int64_t jcS_cap,
                                       int32_t *irS, void *prS, int64_t cap,
                                       int32_t *slot, void *ws, size_t ws_bytes,
                                       fsparse_plan **plan, fsparse_info *info,
                                       hipStream_t stream);

/*
 * Index expansion (Section 2.1 mentions an extension of the input syntax in
 * which row and column indices are used several times as the shapes of the
 * inputs dictate; the paper gives no detail, so this library defines it as
 * broadcasting).  The triplets form a grid of shape[0] x shape[1] x shape[2]
 * = R x C x P; triplet number k = r + R*(c + C*p) (Matlab's column-major
 * order of an R x C x P array).  Each of ii, jj, ss is a dense array in the
 * same order whose shape has, in every dimension d, either 1 (the operand is
 * repeated along d) or shape[d].  Triplet k reads each operand at its (r,c,p)
 * with the repeated dimensions' coordinates set to 0.
 *
 * Example, finite elements with nv nodes per element and P elements:
 * ii = connectivity with shape {1, nv, P}, jj = the same array with shape
 * {nv, 1, P}, ss = element matrices with shape {nv, nv, P}, where
 * ss[r + nv*(c + nv*p)] couples row node c and column node r of element p.
 * This reads nv indices per element instead of 2*nv*nv.
 */
typedef struct {
  int64_t shape[3];     /* R, C, P; R*C*P <= 2^31 - 1 triplets   */
  int64_t ii_shape[3];  /* each entry 1 or shape[d]                */
  int64_t jj_shape[3];
  int64_t ss_shape[3];
} fsparse_expand;

/*
 * Fresh assembly of the expanded triplets: the same as fsparse_assemble on
 * the len = R*C*P triplets that `x` describes (same arguments, outputs,
 * errors and waits), without forming them.  Additional errors:
 * FSPARSE_E_ARG for an operand dimension that is neither 1 nor the grid's,
 * for R*C*P >= 2^31, and for FSPARSE_ATOMIC when ss is repeated along some
 * dimension.  slot, the plan and fsparse_workspace_bytes count the expanded
 * triplets (len = R*C*P); re-use (fsparse_assemble_reuse) and
 * fsparse_backward then take and give values for all R*C*P triplets, in
 * triplet order.  Default dimensions are the largest entries of ii and jj.
 */
fsparse_status fsparse_assemble_expand(const int32_t *ii, const int32_t *jj,
                                       const void *ss, fsparse_dtype dt,
                                       const fsparse_expand *x, int64_t m,
                                       int64_t n, int64_t nzmax, unsigned flags,
                                       int32_t *jcS, int64_t jcS_cap,
                                       int32_t *irS, void *prS, int64_t cap,
                                       int32_t *slot, void *ws, size_t ws_bytes,
                                       fsparse_plan **plan, fsparse_info *info,
                                       hipStream_t stream);

/*
 * Delayed assembly (Section 2.1 names the case of input that is not all
 * available at the first call): new triplets added to an assembled matrix.
 * The result is bit-identical to one fresh assembly of all the triplets,
 * old ones first: every pair's fold continues from its stored sum, and a
 * fold that starts from +0.0 never ends at -0.0, so continuing from the
 * stored sum equals folding all of the pair's contributions in order.
 *
 *  jcA, irA, prA  the existing matrix: [nA+1], [nnzA], [nnzA] of type dt, in
 *                 the format fsparse_assemble writes (rows strictly
 *                 increasing per column)
 *  ii, jj, ss     [len] new triplets, as for fsparse_assemble
 *  m, n           dimensions of the result (at least those of the existing
 *                 matrix); negative: the largest row index over old and new,
 *                 and max(nA, largest new column)
 *  flags, jcS, irS, prS, cap, plan, info: as for fsparse_assemble over the
 *                 nnzA + len triplets (the outputs may be the input arrays
 *                 when they are large enough: the old pairs are copied
 *                 first)
 *  slot           [nnzA + len] or NULL: the first nnzA entries give where
 *                 each old pair went, the rest the new triplets' positions
 *  ws             fsparse_append_workspace_bytes(nnzA, len, n, dt) bytes;
 *                 a plan covers nnzA + len values (the old sums, then the new
 *                 values)
 * Without a plan and without FSPARSE_DROP_ZEROS the call merges: the new
 * triplets are assembled on their own, over the column range they occupy,
 * with their sorted order kept, and merged column by column with the stored
 * pairs (a pair in both continues from its stored sum over the new
 * contributions in increasing k).  The stored pairs are read once and not
 * sorted again.  It waits three times (the new triplets' index range, their
 * assembly, the merged nnz); FSPARSE_ATOMIC gives the ordered sums there.
 * E_CAPACITY then reports nnzA + the new distinct pairs, an upper bound of
 * nnz.  With a plan or FSPARSE_DROP_ZEROS, or when a merge block finds
 * columns far longer than the average, the stored pairs become triplets
 * again and everything is assembled anew.
 */
size_t fsparse_append_workspace_bytes(int64_t nnzA, int64_t len, int64_t n,
                                      fsparse_dtype dt);
fsparse_status fsparse_assemble_append(const int32_t *jcA, const int32_t *irA,
                                       const void *prA, int64_t nnzA,
                                       int64_t nA, const int32_t *ii,
                                       const int32_t *jj, const void *ss,
                                       int64_t len, fsparse_dtype dt,
                                       int64_t m, int64_t n, unsigned flags,
                                       int32_t *jcS, int64_t jcS_cap,
                                       int32_t *irS, void *prS, int64_t cap,
                                       int32_t *slot, void *ws, size_t ws_bytes,
                                       fsparse_plan **plan, fsparse_info *info,
                                       hipStream_t stream);

/*
 * Pattern re-use: the values prS[0..nnz) of the matrix the plan was made
 * for, from new values ss[0..len) on the same (ii, jj) -- the repeated
 * assembly of Section 2.1 ("saving various types of information between
 * successive calls").  Ordered mode folds each pair in increasing k and is
 * bit-identical to a fresh assembly with the same ss.  FSPARSE_ATOMIC works
 * on every plan: it reads the slot array the plan was made with, or, for a
 * plan made without one, a slot map that its first atomic call derives
 * from the sorted order into the plan's workspace (one kernel more, that
 * once).  The work is one graph launch of a HIP graph held by the plan; it
 * never waits, so it may itself be captured.
 */
fsparse_status fsparse_assemble_reuse(fsparse_plan *plan, const void *ss,
                                      void *prS, unsigned flags,
                                      hipStream_t stream);

/*
 * Backward of prS = assemble(ss) for a fixed pattern.  By eq. (2.3),
 * prS[t] = sum of ss[k] over slot[k] = t, so d prS[t] / d ss[k] = [slot[k]=t]
 * and
 *      grad_ss[k] = grad_prS[slot[k]],   k = 0..len-1.
 * slot [len] int32 values in [0, nnz), or -1 for a triplet whose pair is not
 * stored (dropped zero sums, logical pairs without a true triplet): no
 * stored value depends on it, so grad_ss[k] = 0.  Any other value outside
 * [0, nnz) also gives 0 and reads nothing.  grad_prS [nnz], grad_ss [len]
 * of dt; nnz = 0 is allowed (every gradient is then 0).  Never waits.
 */
fsparse_status fsparse_backward(const int32_t *slot, int64_t len,
                                const void *grad_prS, int64_t nnz,
                                fsparse_dtype dt, void *grad_ss,
                                hipStream_t stream);

/*
 * Batched assembly of nb independent matrices with the same launches.
 *  trip_off  host [nb+1]: triplets of matrix b are k in [trip_off[b],
 *            trip_off[b+1]) of ii, jj, ss (trip_off[0] = 0, nondecreasing).
 *  m, n      host [nb]: dimensions (negative: default for that matrix).
 *  jcS       out: the nb column-pointer arrays back to back; matrix b's
 *            n_b+1 pointers start at index col_off[b] + b, where col_off is
 *            the running sum of n; each is relative to its own matrix
 *            (jcS_b[0] = 0, jcS_b[n_b] = nnz_b).
 *  irS, prS  [cap] out: the matrices' entries back to back; matrix b's are
 *            [nnz_off[b], nnz_off[b+1]).
 *  nnz_off   host [nb+1] out.
 *  slot      [total len] out, may be NULL: position of triplet k in the
 *            concatenated irS/prS (subtract nnz_off[b] for the matrix-local
 *            position).
 *  ws        fsparse_workspace_bytes(total len, sum of n, nb, dt) bytes.
 *  plan      as for fsparse_assemble; re-use then produces the concatenated
 *            prS.
 *  info      host [nb] out, may be NULL.
 * Waits for the stream once (twice with default dimensions).
 */
fsparse_status fsparse_assemble_batched(
    int32_t nb, const int64_t *trip_off, const int32_t *ii, const int32_t *jj,
    const void *ss, fsparse_dtype dt, const int64_t *m, const int64_t *n,
    unsigned flags, int32_t *jcS, int64_t jcS_cap, int32_t *irS, void *prS,
    int64_t cap, int64_t *nnz_off, int32_t *slot, void *ws, size_t ws_bytes,
    fsparse_plan **plan, fsparse_info *info, hipStream_t stream);

/*
 * Per-matrix default dimensions of a batch (largest row / column index of
 * each matrix, 0 for a matrix without triplets), so that the caller can
 * size jcS and ws before fsparse_assemble_batched.  trip_off is host [nb+1];
 * m, n are host [nb] outputs.  ws needs fsparse_workspace_bytes(0, 0, nb, dt)
 * bytes.  Any index below 1 gives FSPARSE_E_INDEX.  Waits for the stream.
 */
fsparse_status fsparse_dims_batched(int32_t nb, const int64_t *trip_off,
                                    const int32_t *ii, const int32_t *jj,
                                    int64_t *m, int64_t *n, void *ws,
                                    size_t ws_bytes, hipStream_t stream);

/* Release a plan (host memory and its graph only; device buffers are the
 * caller's).  Waits for the plan's latest re-assembly launch to finish
 * first.  NULL is ignored. */
void fsparse_plan_destroy(fsparse_plan *plan);

/* Sizes a plan was made for (any pointer may be NULL).  For a plan made
 * with FSPARSE_NO_SYNC, nnz is read back from the workspace (a blocking
 * copy). */
fsparse_status fsparse_plan_query(const fsparse_plan *plan, int64_t *len,
                                  int64_t *nnz, int32_t *dtype);

/*
 * Launch-shape tuning (process-wide).  chunk_cap: triplets one workgroup of
 * the sort/fold stage holds in LDS, one of 1024, 2048, 4096; a smaller
 * positive power of two limits it further (used to exercise the long-column
 * path on small inputs).  stream_block: threads per block of the streaming
 * stages (64..1024, multiple of 64).  stream_items: elements per thread per
 * tile (1..32).  reuse_block: threads per block of the re-assembly kernel.
 * chunk_block: threads of one sort/fold workgroup (256, 512 or 1024; at
 * least chunk_cap/16 are used).  Zero fields keep the current value.
 * bin_mode chooses how triplets are placed into column bins: 0 automatic,
 * 1 per-tile count matrix (only while the bins fit the LDS counters),
 * 2 fixed-capacity bins filled in one pass, 3 count then place; it is
 * always applied (0 restores the automatic choice).  slot_values: what the
 * fixed-capacity bins hold for a triplet (zero keeps the current setting):
 * 1 its value with its row and index k, 2 only its row and k, the sort/fold
 * stage then reading the value by k from the input (the default: half the
 * binned bytes, but reads by k that only pay off when triplets of nearby
 * columns lie near each other in the input, as in element-by-element
 * assembly; inputs in index-expansion form always bin their values).  NULL
 * restores all defaults.
 */
typedef struct {
  int32_t chunk_cap;
  int32_t stream_block;
  int32_t stream_items;
  int32_t reuse_block;
  int32_t chunk_block;
  int32_t bin_mode;
  int32_t slot_values;
} fsparse_tuning;

fsparse_status fsparse_set_tuning(const fsparse_tuning *t);
fsparse_status fsparse_get_tuning(fsparse_tuning *t /* host out */);

/*
 * Per-stage timing with HIP events recorded on the stream each stage is
 * launched on.  While enabled, every launch of a stage is bracketed by two
 * events; fsparse_timing_read waits for the recorded events and returns the
 * accumulated milliseconds and launch counts per stage (up to max_stages
 * entries), then clears them.  Returns the number of stages, or -1 on error.
 */
fsparse_status fsparse_timing_enable(int on);
int fsparse_timing_read(double *ms, int64_t *launches, int max_stages);
const char *fsparse_stage_name(int stage);

/* Restricts timing to the stages whose bit (1 << stage) is set in
 * stage_mask (all stages by default), so that a timed run carries events
 * only around the launches it reports.  The setting is process-wide and
 * stays until changed. */
fsparse_status fsparse_timing_select(uint32_t stage_mask);

/* Plain device-to-device copy kernel (16-byte vector loads/stores) used to
 * measure attainable HBM bandwidth and to calibrate byte counters.  bytes
 * must be a multiple of 16 and both pointers 16-byte aligned. */
fsparse_status fsparse_stream_copy(const void *src, void *dst, size_t bytes,
                                   hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FSPARSE_H_ */
