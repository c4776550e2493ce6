// Device code of the gfx950 sparse-assembly pipeline.
//
// Fresh assembly of S = sparse(ii, jj, ss, m, n) (Section 2.1).  Columns are
// grouped into bins of w consecutive columns (any w; an in-bin column takes
// s bits, 2^s >= w), sized so an average bin fills 80% of the LDS of one bin
// workgroup.
//   count    per-tile LDS histograms of bins (dense mode: a tiles x bins
//            count matrix; claim mode: one device atomic per (tile, bin));
//            out-of-range columns are flagged here (pre-processing listing)
//   colscan  dense mode: column prefix sums of the count matrix, so every
//            tile knows its exclusive offset in every bin
//   binscan  single-pass decoupled look-back scan of the bin totals
//   scatter  every triplet goes to its bin as (row << s | in-bin column, k,
//            value), ranked inside the tile by an LDS atomic; slot mode
//            instead gives every bin a fixed place and claims space per
//            (tile, bin) in one pass, falling back to count-first when a bin
//            overflows
//   bin      one workgroup per bin: equal (column,row) pairs are grouped by
//            an LDS hash, the distinct rows of every column are ranked (rows
//            increase within a column, as Part 3 of Section 2.3 yields),
//            each pair's contributions are put in increasing k and folded
//            from +0.0 in that order (the serial post-processing order);
//            the bin's output offset comes from a chained look-back over the
//            bins, which also gives jcS (Part 4's running sum).  A bin
//            longer than the LDS is counted before this kernel and emitted
//            after it (k_slow_count, k_slow_emit).
// The sorted order of the contributions (perm) and the first sorted
// position of every output (seg) are kept for pattern re-use; slot[k] is
// the paper's inverse rank irank (Section 2.2, eqs. (2.2)-(2.3)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fsp {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

// error bits in Ctrl::err
constexpr uint32_t kErrCol = 1u;
constexpr uint32_t kErrRow = 2u;
constexpr uint32_t kErrCap = 4u;
constexpr uint32_t kErrSlot = 8u;  // a fixed-capacity bin overflowed: redo in two passes
constexpr uint32_t kErrRuns = 16u;  // a merge block's runs exceeded its LDS: merge otherwise

// Control block at the start of the workspace (zeroed before every call).
struct Ctrl {
  uint32_t err;
  uint32_t tick_scan;
  uint32_t tick_chunk;
  uint32_t nslow;  // bins longer than the LDS capacity, listed by the bin scan
  int64_t nnz;
  int64_t ltot;
  int32_t rmin, rmax, cmin, cmax;  // dims pass
  int32_t kept;                    // pairs left after dropping zero sums
  uint32_t pad1[19];
};
static_assert(sizeof(Ctrl) <= 256, "control block");

// One triplet in its column bucket.  (row, k) then the value; 16 bytes for
// fp64 (one dwordx4 access), 12 bytes for fp32.
template <typename VT>
struct Entry;
template <>
struct __attribute__((aligned(16))) Entry<double> {
  uint32_t row, k;
  double v;
};
template <>
struct Entry<float> {
  uint32_t row, k;
  float v;
};
// A binned triplet without its value (fixed-capacity bins, values read by k
// in the bin kernel).
struct __attribute__((aligned(8))) KeyEntry {
  uint32_t row, k;
};

// Several matrices assembled by the same launches: matrix b owns triplets
// [trip_off[b], trip_off[b+1]) and global columns [col_off[b], col_off[b+1]).
struct BatchDesc {
  const int64_t* trip_off;
  const int64_t* col_off;
  const int32_t* mdim;
  const int32_t* ndim;
  int32_t nb;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Look-back status words carry their flag and value in one 64-bit word and
// no other data is published through them, so relaxed device-scope atomics
// are enough (acquire/release would add cache invalidation and write-back
// around every access).
__device__ __forceinline__ uint64_t ld_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Cross-lane moves for wave scans, done by DPP on the VALU instead of LDS
// permutes.  CTRL: 0x110 + n = row_shr:n (n lanes up inside a row of 16),
// 0x142 = row_bcast:15 (lane 15 of each row into the next row), 0x143 =
// row_bcast:31 (lane 31 into rows 2 and 3).  ROWS masks the rows written;
// lanes without a source or outside ROWS read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp0(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp0(uint64_t v) {
  const uint32_t lo = dpp0<CTRL, ROWS>((uint32_t)v);
  const uint32_t hi = dpp0<CTRL, ROWS>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive sum over the 64 lanes (Hillis-Steele inside rows, then the row
// totals carried across rows).
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T x) {
  x += dpp0<0x111, 0xf>(x);
  x += dpp0<0x112, 0xf>(x);
  x += dpp0<0x114, 0xf>(x);
  x += dpp0<0x118, 0xf>(x);
  x += dpp0<0x142, 0xa>(x);
  x += dpp0<0x143, 0xc>(x);
  return x;
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  x = max(x, dpp0<0x111, 0xf>(x));
  x = max(x, dpp0<0x112, 0xf>(x));
  x = max(x, dpp0<0x114, 0xf>(x));
  x = max(x, dpp0<0x118, 0xf>(x));
  x = max(x, dpp0<0x142, 0xa>(x));
  x = max(x, dpp0<0x143, 0xc>(x));
  return x;
}

__device__ __forceinline__ uint32_t lane63(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint64_t lane63(uint64_t v) {
  return ((uint64_t)lane63((uint32_t)(v >> 32)) << 32) | lane63((uint32_t)v);
}

// Exclusive block-wide sum of one value per thread.  All threads call it.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* sWave,
                                                   uint32_t& total) {
  const int wid = threadIdx.x >> 6;
  uint32_t x = wave_incl_sum(v);
  if (lane_id() == 63) sWave[wid] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    uint32_t t = sWave[w];
    pre += (w < wid) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

template <int NT>
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t* sWave) {
  const int wid = threadIdx.x >> 6;
  uint32_t x = wave_incl_max(v);
  if (lane_id() == 63) sWave[wid] = x;
  __syncthreads();
  uint32_t pre = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    uint32_t t = sWave[w];
    if (w < wid) pre = pre > t ? pre : t;
  }
  // exclusive max within the wave: value of the previous lane
  uint32_t prev = __shfl_up(x, 1, 64);
  if (lane_id() == 0) prev = 0;
  __syncthreads();
  return pre > prev ? pre : prev;
}

// In-place exclusive prefix sum of arr[0..S) in LDS; returns the total.
// Up to 256 entries one wave scans four per lane; longer arrays are cut into
// one contiguous run per thread.  All threads call it; sWave holds NT/64 + 1
// words, and the caller must pass a barrier before calling it again.
template <int NT>
__device__ uint32_t lds_excl_scan(uint32_t* arr, int S, uint32_t* sWave) {
  constexpr int NW = NT / 64;
  const int wid = threadIdx.x >> 6;
  if (S <= 256) {
    if (wid == 0) {
      const int i0 = lane_id() * 4;
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = i0 + u < S ? arr[i0 + u] : 0u;
      const uint32_t sum = (v[0] + v[1]) + (v[2] + v[3]);
      const uint32_t inc = wave_incl_sum(sum);
      uint32_t run = inc - sum;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i0 + u < S) arr[i0 + u] = run;
        run += v[u];
      }
      if (lane_id() == 63) sWave[NW] = inc;
    }
    __syncthreads();
    return sWave[NW];
  }
  const int ipt = (S + NT - 1) / NT;
  const int lo = min(S, (int)threadIdx.x * ipt);
  const int hi = min(S, lo + ipt);
  uint32_t acc = 0;
  for (int i = lo; i < hi; ++i) acc += arr[i];
  const uint32_t x = wave_incl_sum(acc);
  if (lane_id() == 63) sWave[wid] = x;
  __syncthreads();
  uint32_t pre = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = sWave[w];
    pre += (w < wid) ? t : 0u;
    total += t;
  }
  uint32_t run = pre + x - acc;
  for (int i = lo; i < hi; ++i) {
    const uint32_t y = arr[i];
    arr[i] = run;
    run += y;
  }
  __syncthreads();
  return total;
}

// In-place inclusive running maximum of arr[0..S) in LDS.
template <int NT>
__device__ void lds_incl_max(uint32_t* arr, int S, uint32_t* sWave) {
  const int ipt = (S + NT - 1) / NT;
  const int lo = min(S, (int)threadIdx.x * ipt);
  const int hi = min(S, lo + ipt);
  uint32_t acc = 0;
  for (int i = lo; i < hi; ++i) acc = acc > arr[i] ? acc : arr[i];
  uint32_t run = block_excl_max<NT>(acc, sWave);
  for (int i = lo; i < hi; ++i) {
    uint32_t x = arr[i];
    run = run > x ? run : x;
    arr[i] = run;
  }
  __syncthreads();
}

// Chained look-back over tiles in ticket order (Merrill & Garland's single
// pass scan with decoupled look-back).  Called by the 64 lanes of one wave;
// returns the exclusive prefix of tile q and publishes its inclusive prefix.
__device__ int64_t lookback(uint64_t* status, int q, uint64_t agg) {
  const int lane = lane_id();
  if (q == 0) {
    if (lane == 0) st_status(&status[0], kFlagPrefix | agg);
    return 0;
  }
  if (lane == 0) st_status(&status[q], kFlagAgg | agg);
  int64_t excl = 0;
  int pred = q - 1;
  for (;;) {
    const int idx = pred - lane;
    const uint64_t s = (idx >= 0) ? ld_status(&status[idx]) : kFlagPrefix;
    const uint32_t flag = (uint32_t)(s >> 62);
    const uint64_t inval = __ballot(flag == 0);
    const uint64_t pref = __ballot(flag == 2);
    const int pl = pref ? (__ffsll((unsigned long long)pref) - 1) : 64;
    const uint64_t need = (pl >= 63) ? ~0ull : ((2ull << pl) - 1ull);
    if (inval & need) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint64_t v = (lane <= pl) ? (s & kValMask) : 0ull;
    v = wave_incl_sum(v);
    excl += (int64_t)lane63(v);
    if (pl < 64) break;
    pred -= 64;
  }
  if (lane == 0) st_status(&status[q], kFlagPrefix | (uint64_t)(excl + (int64_t)agg));
  return excl;
}

// The two halves of `lookback` for callers that have work to do between
// publishing their aggregate and needing their prefix.
__device__ __forceinline__ void lookback_publish(uint64_t* status, int q,
                                                 uint64_t agg) {
  if (lane_id() == 0)
    st_status(&status[q], (q == 0 ? kFlagPrefix : kFlagAgg) | agg);
}

// First read of the 64 words before tile q, issued ahead of lookback_wait so
// that its latency overlaps other work.  Any state it sees is usable: an
// aggregate stays that tile's aggregate, and a word not yet written is read
// again by lookback_wait.
// The first look-back window of bin q (q >= 1), loaded without a branch:
// lanes before bin 0 read status[0], and lookback_wait treats them as
// prefixes.  (No select here, so nothing waits for the load yet.)
__device__ __forceinline__ uint64_t lookback_probe(const uint64_t* status, int q) {
  return ld_status(&status[max(q - 1 - lane_id(), 0)]);
}

__device__ int64_t lookback_wait(uint64_t* status, int q, uint64_t agg,
                                 uint64_t probe) {
  const int lane = lane_id();
  if (q == 0) return 0;
  int64_t excl = 0;
  int pred = q - 1;
  bool first = true;
  for (;;) {
    const int idx = pred - lane;
    const uint64_t s = (idx < 0) ? kFlagPrefix : (first ? probe : ld_status(&status[idx]));
    first = false;
    const uint32_t flag = (uint32_t)(s >> 62);
    const uint64_t inval = __ballot(flag == 0);
    const uint64_t pref = __ballot(flag == 2);
    const int pl = pref ? (__ffsll((unsigned long long)pref) - 1) : 64;
    const uint64_t need = (pl >= 63) ? ~0ull : ((2ull << pl) - 1ull);
    if (inval & need) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint64_t v = (lane <= pl) ? (s & kValMask) : 0ull;
    v = wave_incl_sum(v);
    excl += (int64_t)lane63(v);
    if (pl < 64) break;
    pred -= 64;
  }
  if (lane == 0) st_status(&status[q], kFlagPrefix | (uint64_t)(excl + (int64_t)agg));
  return excl;
}

__device__ __forceinline__ int find_mat(const int64_t* off, int nb, int64_t e) {
  int lo = 0, hi = nb;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// zero fill, typed fill, copy
// ---------------------------------------------------------------------------
__global__ void k_zero(uint32_t* __restrict__ p, int64_t nwords) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst,
                         int64_t n16) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Where the streaming passes take a triplet's indices from: int32 arrays,
// the expansion map, or double arrays (Matlab's default array type).
enum IdxSrc { kIdxI32 = 0, kIdxExpand = 1, kIdxF64 = 2 };

// A unit-offset index held in a double (the pre-processing check of
// Section 2.2): a whole number in [1, 2^31 - 1] converts exactly; anything
// else (a fraction, NaN, an infinity, a value below 1 or beyond int32)
// becomes 0, which every pass rejects like any other index below 1.
__device__ __forceinline__ int32_t f64_index(double v) {
  return (v >= 1.0 && v <= 2147483647.0 && v == ceil(v)) ? (int32_t)v : 0;
}

// Index x of an index array of the given source (not the expansion map).
template <int SRC>
__device__ __forceinline__ int32_t ld_index(const int32_t* __restrict__ p, int64_t x) {
  if constexpr (SRC == kIdxF64)
    return f64_index(reinterpret_cast<const double*>(p)[x]);
  else
    return p[x];
}

// ---------------------------------------------------------------------------
// dims: largest / smallest index (the pre-processing pass, Section 2.2)
// ---------------------------------------------------------------------------
template <bool BATCHED, int SRC = kIdxI32>
__global__ void k_dims(const int32_t* __restrict__ ii,
                       const int32_t* __restrict__ jj, int64_t L,
                       BatchDesc bd, Ctrl* ctrl, int32_t* __restrict__ bmax) {
  int32_t rmax = 0, cmax = 0, rmin = INT32_MAX, cmin = INT32_MAX;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < L; e += stride) {
    const int32_t r = ld_index<SRC>(ii, e), c = ld_index<SRC>(jj, e);
    rmin = min(rmin, r);
    cmin = min(cmin, c);
    if (BATCHED) {
      // one atomic pair per wave when the whole wave is here and its
      // triplets share a matrix (matrices are long runs of triplets), else
      // one per triplet
      const int b = find_mat(bd.trip_off, bd.nb, e);
      const int b0 = __builtin_amdgcn_readfirstlane(b);
      if (__ballot(1) == ~0ull && __all(b == b0)) {
        int32_t wr = r, wc = c;
        for (int d = 32; d > 0; d >>= 1) {
          wr = max(wr, __shfl_xor(wr, d, 64));
          wc = max(wc, __shfl_xor(wc, d, 64));
        }
        if (lane_id() == 0) {
          atomicMax(&bmax[2 * b0], wr);
          atomicMax(&bmax[2 * b0 + 1], wc);
        }
      } else {
        atomicMax(&bmax[2 * b], r);
        atomicMax(&bmax[2 * b + 1], c);
      }
    } else {
      rmax = max(rmax, r);
      cmax = max(cmax, c);
    }
  }
  // wave reductions, then the block's through LDS, then one atomic per
  // block and field: every atomic goes to the same four words, which the
  // memory system serialises, so they are kept few
  for (int d = 32; d > 0; d >>= 1) {
    rmax = max(rmax, __shfl_xor(rmax, d, 64));
    cmax = max(cmax, __shfl_xor(cmax, d, 64));
    rmin = min(rmin, __shfl_xor(rmin, d, 64));
    cmin = min(cmin, __shfl_xor(cmin, d, 64));
  }
  __shared__ int32_t red[4][16];
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane_id() == 0) {
    red[0][w] = rmax;
    red[1][w] = cmax;
    red[2][w] = rmin;
    red[3][w] = cmin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < nw; ++v) {
      rmax = max(rmax, red[0][v]);
      cmax = max(cmax, red[1][v]);
      rmin = min(rmin, red[2][v]);
      cmin = min(cmin, red[3][v]);
    }
    atomicMax(&ctrl->rmax, rmax);
    atomicMax(&ctrl->cmax, cmax);
    atomicMin(&ctrl->rmin, rmin);
    atomicMin(&ctrl->cmin, cmin);
  }
}

// ---------------------------------------------------------------------------
// bucket: scatter (row, k, value) into the column buckets
// ---------------------------------------------------------------------------
template <typename VT>
__device__ __forceinline__ void store_entry(Entry<VT>* p, uint32_t row,
                                            uint32_t k, VT v);
template <>
__device__ __forceinline__ void store_entry<double>(Entry<double>* p,
                                                    uint32_t row, uint32_t k,
                                                    double v) {
  uint4 x;
  x.x = row;
  x.y = k;
  const uint64_t b = __double_as_longlong(v);
  x.z = (uint32_t)b;
  x.w = (uint32_t)(b >> 32);
  *reinterpret_cast<uint4*>(p) = x;
}
template <>
__device__ __forceinline__ void store_entry<float>(Entry<float>* p, uint32_t row,
                                                   uint32_t k, float v) {
  p->row = row;
  p->k = k;
  p->v = v;
}

template <typename VT>
__device__ __forceinline__ Entry<VT> load_entry(const Entry<VT>* p);
template <>
__device__ __forceinline__ Entry<double> load_entry<double>(const Entry<double>* p) {
  const uint4 x = *reinterpret_cast<const uint4*>(p);
  Entry<double> e;
  e.row = x.x;
  e.k = x.y;
  e.v = __longlong_as_double(((int64_t)x.w << 32) | (int64_t)x.z);
  return e;
}
template <>
__device__ __forceinline__ Entry<float> load_entry<float>(const Entry<float>* p) {
  return *p;
}

// ---------------------------------------------------------------------------
// Column bins.  Global column g (matrix b's column c is col_off[b] + c) lies
// in bin g / w; a bin is w consecutive columns (any w, not only powers of
// two, so that bins can be sized to the LDS), and the bin kernel handles one
// bin per workgroup.  Bin pointers come from per-tile LDS
// histograms: either a dense tiles x bins count matrix whose column prefix
// sums give every tile its exclusive offset in every bin (no device-wide
// atomics at all), or, with too many bins for that, one global claim per
// (tile, bin) that the tile touches.
// ---------------------------------------------------------------------------

// Bin geometry.  g / w is one multiply-high and a shift: for w = 2^s,
// mul = 1 and sh = s; otherwise, with l = ceil(log2 w), sh = 31 + l and
// mul = ceil(2^sh / w) < 2^32, and since mul * w - 2^sh < w <= 2^l the
// quotient is exact for every g < 2^31 (Granlund and Montgomery, division by
// invariant integers, 1994).  An in-bin column g - w * bin takes s = l bits.
struct BinGeo {
  uint32_t mul;
  int32_t sh;
  int32_t w;
  int32_t s;
};

__device__ __forceinline__ uint32_t bin_of(const BinGeo& G, int64_t g) {
  return (uint32_t)(((uint64_t)(uint32_t)g * G.mul) >> G.sh);
}

__device__ __forceinline__ uint32_t bin_col(const BinGeo& G, int64_t g, uint32_t q) {
  return (uint32_t)g - q * (uint32_t)G.w;
}

// Expanded input (the index-expansion extension of the input syntax,
// Section 2.1): the triplets form an R x C x P grid, triplet
// e = r + R * (c + C * p), and each of ii, jj, ss is a dense array over the
// same grid in which any dimension may be 1, read with stride 0 along it.
// The two quotients e / R and (e / R) / C use the bins' exact
// multiply-high division (e < 2^31).
struct Expand {
  BinGeo dR, dC;
  uint32_t R, C;
  uint32_t si[3], sj[3], sv[3];  // element strides of ii, jj, ss along r, c, p
};

struct ExpPos {
  uint32_t r, c, p;
};

__device__ __forceinline__ ExpPos exp_pos(const Expand& x, int64_t e) {
  ExpPos o;
  const uint32_t q = bin_of(x.dR, e);
  o.r = (uint32_t)e - q * x.R;
  o.p = bin_of(x.dC, q);
  o.c = q - o.p * x.C;
  return o;
}

__device__ __forceinline__ uint32_t exp_at(const uint32_t (&s)[3], const ExpPos& o) {
  return o.r * s[0] + o.c * s[1] + o.p * s[2];
}

// The matrix of the triplets a thread visits, in increasing order: its index,
// triplet end, column offset and dimensions, kept in registers.
struct MatCur {
  int b;
  int64_t end, coff;
  int32_t nd, md;
};

template <bool BATCHED>
__device__ __forceinline__ void mat_cur(const BatchDesc& bd, MatCur& c, int b) {
  if (!BATCHED) return;
  c.b = b;
  c.end = bd.trip_off[b + 1];
  c.coff = bd.col_off[b];
  c.nd = bd.ndim[b];
  c.md = bd.mdim[b];
}

// Global column of triplet e; the cursor walks forward over the matrices.
template <bool BATCHED>
__device__ __forceinline__ int64_t global_col(const BatchDesc& bd, MatCur& cur,
                                              int64_t e, int32_t c, int32_t n,
                                              int32_t m, int32_t& mb, bool& ok) {
  if (BATCHED) {
    while (cur.end <= e) mat_cur<true>(bd, cur, cur.b + 1);
    ok = (uint32_t)c < (uint32_t)cur.nd;
    mb = cur.md;
    return cur.coff + c;
  }
  ok = (uint32_t)c < (uint32_t)n;
  mb = m;
  return c;
}

template <bool BATCHED>
__device__ __forceinline__ int tile_first_mat(const BatchDesc& bd, int64_t t0,
                                              int64_t L, int* sB) {
  if (!BATCHED) return 0;
  if (threadIdx.x == 0) *sB = find_mat(bd.trip_off, bd.nb, min(t0, L - 1));
  __syncthreads();
  return *sB;
}

// Exclusive scan of in[0..n) (decoupled look-back) into out[0..n]; out[n]
// is the total.
// Bins above `cap` are appended to slowlist (count in *nslow).
template <int NT, int IPT>
__global__ void __launch_bounds__(NT)
k_scan_excl(const uint32_t* __restrict__ in, int32_t n, int32_t* __restrict__ out,
            uint64_t* status, uint32_t* ticket, uint32_t cap,
            uint32_t* __restrict__ nslow, int32_t* __restrict__ slowlist) {
  __shared__ uint32_t sWave[NT / 64];
  __shared__ int sTile;
  __shared__ int64_t sBase;
  if (threadIdx.x == 0) sTile = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int tile = sTile;
  const int64_t i0 = (int64_t)tile * NT * IPT + (int64_t)threadIdx.x * IPT;
  uint32_t v[IPT];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    v[j] = (i0 + j < n) ? in[i0 + j] : 0u;
    sum += v[j];
  }
  uint32_t total;
  const uint32_t pre = block_excl_sum<NT>(sum, sWave, total);
  if (threadIdx.x < 64) {
    const int64_t ex = lookback(status, tile, total);
    if (threadIdx.x == 0) sBase = ex;
  }
  __syncthreads();
  int64_t run = sBase + pre;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if (i0 + j <= n) out[i0 + j] = (int32_t)run;
    run += v[j];
    if (v[j] > cap) slowlist[atomicAdd(nslow, 1u)] = (int32_t)(i0 + j);
  }
}

// Tile of the dense passes handled by this block.  Workgroups are dealt to
// the 8 XCDs in turn (block i to XCD i mod 8); giving XCD x the consecutive
// tiles [x*per, (x+1)*per) means that the scatter writes of neighbouring
// tiles into a bin land in the same L2 and leave it as whole lines.  The
// grid has 8*per blocks; those past the last tile return at once.
__device__ __forceinline__ int64_t xcd_tile(int64_t L, int32_t TS) {
  const int64_t T = (L + TS - 1) / TS;
  const int64_t per = (T + 7) >> 3;
  const int64_t t = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  return t < T ? t : -1;
}

// Element x of p by a 32-bit byte offset (x * sizeof(T) < 2^32): with p in
// scalar registers the load needs one vector register for its address.
template <typename T>
__device__ __forceinline__ T ld_off32(const T* __restrict__ p, uint32_t x) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) +
                                     x * (uint32_t)sizeof(T));
}

// triplets whose loads one thread keeps in flight: dense count, dense
// scatter, claim scatter
constexpr int kDenseU = 8;
// spare bucket places past the last one: the claim scatter's unplaced
// triplets go to place trash + (lane % kSpare)
constexpr int kSpare = 64;
constexpr int kDenseSU = 8;
constexpr int kScatterU = 4;

// dense mode, pass 1: per-tile bin histogram -> row `tile` of cnt[T][B].
// As the first kernel of the call it also clears the control block and the
// look-back words (zero[0..zwords)), which no later kernel of the call uses
// before it is done; so it reports a bad column not in the control block
// but in its own word tilebad[tile], which the column scan reads.
template <bool BATCHED, int SRC>
__global__ void k_count_dense(const int32_t* __restrict__ jj, int64_t L,
                              int32_t n, BatchDesc bd, BinGeo G, int32_t B,
                              int32_t TS, uint32_t* __restrict__ cnt,
                              uint32_t* __restrict__ zero, int64_t zwords,
                              uint32_t* __restrict__ tilebad, Expand ex) {
  extern __shared__ uint32_t hist[];
  __shared__ int sB;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < zwords;
       i += (int64_t)gridDim.x * blockDim.x)
    zero[i] = 0u;
  const int64_t tile = xcd_tile(L, TS);
  if (tile < 0) return;
  const int64_t t0 = tile * TS;
  const int64_t t1 = min(L, t0 + TS);
  for (int i = threadIdx.x; i < B; i += blockDim.x) hist[i] = 0u;
  MatCur b;
  mat_cur<BATCHED>(bd, b, tile_first_mat<BATCHED>(bd, t0, L, &sB));
  __syncthreads();
  bool bad = false;
  int32_t mb;
  // kDenseU column loads in flight per thread, then their counts
  const int64_t nt = blockDim.x;
  for (int64_t eb = t0 + threadIdx.x; eb < t1; eb += kDenseU * nt) {
    int32_t cj[kDenseU];
#pragma unroll
    for (int u = 0; u < kDenseU; ++u) {
      const int64_t e = min(eb + u * nt, t1 - 1);  // no branch
      if constexpr (SRC == kIdxExpand)
        cj[u] = jj[exp_at(ex.sj, exp_pos(ex, e))];
      else
        cj[u] = ld_index<SRC>(jj, e);
    }
#pragma unroll
    for (int u = 0; u < kDenseU; ++u) {
      const int64_t e = eb + u * nt;
      if (e >= t1) break;
      bool ok;
      const int64_t g = global_col<BATCHED>(bd, b, e, cj[u] - 1, n, 0, mb, ok);
      if (!ok) { bad = true; continue; }
      atomicAdd(&hist[bin_of(G, g)], 1u);
    }
  }
  __syncthreads();
  uint32_t* row = cnt + tile * B;
  for (int i = threadIdx.x; i < B; i += blockDim.x) row[i] = hist[i];
  const int anybad = __syncthreads_or(bad ? 1 : 0);
  if (threadIdx.x == 0) tilebad[tile] = anybad ? 1u : 0u;
}

// dense mode, pass 2 and the bin pointers in one kernel: the column prefix
// sums of the count matrix give every tile its offset inside every bin, and
// the bin totals, chained over groups of 64 bins by a look-back, give the
// bin pointers (binstart[B] is the total).  A block takes 64 bins (one per
// lane, so every row access is coalesced) and splits the tiles into NT/64
// segments that are summed in parallel and then rewritten as running
// prefixes.  Groups are taken by ticket, so a group waits only for groups
// already started.  Bins above `cap` are appended to slowlist.  The first
// group also raises the bad-column flag from the count pass's tile words.
template <int NT>
__global__ void __launch_bounds__(NT)
k_colscan_bins(uint32_t* __restrict__ cnt, int32_t T, int32_t B,
               int32_t* __restrict__ binstart, uint64_t* status, uint32_t* ticket,
               uint32_t cap, uint32_t* __restrict__ nslow,
               int32_t* __restrict__ slowlist,
               const uint32_t* __restrict__ tilebad, Ctrl* ctrl) {
  constexpr int NSEG = NT / 64;
  __shared__ uint32_t part[NSEG][64];
  __shared__ int sG;
  if (threadIdx.x == 0) sG = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int grp = sG;
  if (grp == 0) {
    int bad = 0;
    for (int i = threadIdx.x; i < T; i += NT) bad |= tilebad[i] ? 1 : 0;
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&ctrl->err, kErrCol);
  }
  const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const int b = grp * 64 + lane;
  const int per = (T + NSEG - 1) / NSEG;
  const int t0 = min(T, seg * per), t1 = min(T, t0 + per);
  uint32_t sum = 0;
  if (b < B) {
    int t = t0;
    for (; t + 8 <= t1; t += 8) {
      uint32_t c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) c[u] = cnt[(int64_t)(t + u) * B + b];
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += c[u];
    }
    for (; t < t1; ++t) sum += cnt[(int64_t)t * B + b];
  }
  part[seg][lane] = sum;
  __syncthreads();
  uint32_t run = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NSEG; ++k) {
    const uint32_t v = part[k][lane];
    run += k < seg ? v : 0u;
    all += v;
  }
  if (seg == 0) {
    const uint32_t mine = b < B ? all : 0u;
    const uint32_t inc = wave_incl_sum(mine);
    const int64_t base = lookback(status, grp, (uint64_t)lane63(inc));
    if (b < B) {
      binstart[b] = (int32_t)(base + inc - mine);
      if (mine > cap) slowlist[atomicAdd(nslow, 1u)] = b;
    }
    if (b == B - 1) binstart[B] = (int32_t)(base + inc);
  }
  if (b >= B) return;
  int t = t0;
  for (; t + 8 <= t1; t += 8) {
    uint32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = cnt[(int64_t)(t + u) * B + b];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cnt[(int64_t)(t + u) * B + b] = run;
      run += c[u];
    }
  }
  for (; t < t1; ++t) {
    const uint32_t c = cnt[(int64_t)t * B + b];
    cnt[(int64_t)t * B + b] = run;
    run += c;
  }
}

// dense mode, pass 3: scatter (row, k, value) and the in-bin column into
// the bins; the position inside the bin is an LDS atomic rank
template <typename VT, bool BATCHED, bool PACKED, int SRC>
__global__ void k_scatter_dense(const int32_t* __restrict__ ii,
                                const int32_t* __restrict__ jj,
                                const VT* __restrict__ ss, int64_t L, int32_t m,
                                int32_t n, BatchDesc bd, BinGeo G, int32_t B,
                                int32_t TS, const uint32_t* __restrict__ offs,
                                const int32_t* __restrict__ binstart,
                                Entry<VT>* __restrict__ bucket,
                                uint32_t* __restrict__ bcol, uint32_t trash,
                                Ctrl* ctrl, Expand ex) {
  extern __shared__ uint32_t ctr[];
  __shared__ int sB;
  const int64_t tile = xcd_tile(L, TS);
  if (tile < 0) return;
  const int64_t t0 = tile * TS;
  const int64_t t1 = min(L, t0 + TS);
  const uint32_t* orow = offs + tile * B;
  for (int i = threadIdx.x; i < B; i += blockDim.x)
    ctr[i] = (uint32_t)binstart[i] + orow[i];
  MatCur b;
  mat_cur<BATCHED>(bd, b, tile_first_mat<BATCHED>(bd, t0, L, &sB));
  __syncthreads();
  bool badr = false;
  // the loads of kDenseSU triplets are issued together, then their LDS
  // ranks, then their stores (a triplet without a place, past the tile or
  // with a bad column, is stored to the spare place `trash`, so that the
  // stores need no branch)
  // (loads address the tile's arrays by 32-bit offsets from tile bases held
  // in scalar registers, which keeps eight triplets' loads within the
  // register budget)
  const int64_t nt = blockDim.x;
  const int32_t* __restrict__ jt = jj + t0;
  const int32_t* __restrict__ it = ii + t0;
  const VT* __restrict__ st = ss + t0;
  for (int64_t eb = t0 + threadIdx.x; eb < t1; eb += kDenseSU * nt) {
    int32_t cj[kDenseSU], ri[kDenseSU];
    VT sv[kDenseSU];
#pragma unroll
    for (int u = 0; u < kDenseSU; ++u) {
      const int64_t e = eb + u * nt;
      if (e < t1) {
        if constexpr (SRC == kIdxExpand) {
          const ExpPos o = exp_pos(ex, e);
          cj[u] = jj[exp_at(ex.sj, o)];
          ri[u] = ii[exp_at(ex.si, o)];
          sv[u] = ss[exp_at(ex.sv, o)];
        } else if constexpr (SRC == kIdxF64) {
          const uint32_t x = (uint32_t)(e - t0);
          cj[u] = f64_index(ld_off32(reinterpret_cast<const double*>(jj) + t0, x));
          ri[u] = f64_index(ld_off32(reinterpret_cast<const double*>(ii) + t0, x));
          sv[u] = ld_off32(st, x);
        } else {
          const uint32_t x = (uint32_t)(e - t0);
          cj[u] = ld_off32(jt, x);
          ri[u] = ld_off32(it, x);
          sv[u] = ld_off32(st, x);
        }
      }
    }
    uint32_t pos[kDenseSU], key[kDenseSU], bc[kDenseSU];
#pragma unroll
    for (int u = 0; u < kDenseSU; ++u) {
      const int64_t e = eb + u * nt;
      pos[u] = trash;
      if (e < t1) {
        bool ok;
        int32_t mb;
        const int64_t g = global_col<BATCHED>(bd, b, e, cj[u] - 1, n, m, mb, ok);
        if (ok) {  // a bad column is flagged by the count pass
          const int32_t r = ri[u] - 1;
          badr |= (uint32_t)r >= (uint32_t)mb;
          const uint32_t q = bin_of(G, g);
          bc[u] = bin_col(G, g, q);
          key[u] = PACKED ? (((uint32_t)r << G.s) | bc[u]) : (uint32_t)r;
          pos[u] = atomicAdd(&ctr[q], 1u);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kDenseSU; ++u) {
      store_entry<VT>(&bucket[pos[u]], key[u], (uint32_t)(eb + u * nt), sv[u]);
      if (!PACKED) bcol[pos[u]] = bc[u];
    }
  }
  if (badr) atomicOr(&ctrl->err, kErrRow);
}

// claim mode: tiles of NT*IPT triplets; bins of the tile live in registers
template <bool BATCHED, int SRC, int NT, int IPT>
__device__ __forceinline__ void tile_bins(const int32_t* __restrict__ jj,
                                          int64_t L, int32_t n, const BatchDesc& bd,
                                          const BinGeo& G, int64_t t0, int* sB,
                                          int32_t (&bn)[IPT], int32_t (&cj)[IPT],
                                          int32_t& lo, int32_t& hi, bool& bad,
                                          const Expand& ex) {
  MatCur b;
  mat_cur<BATCHED>(bd, b, tile_first_mat<BATCHED>(bd, t0, L, sB));
  lo = INT32_MAX;
  hi = -1;
  int32_t mb;
  // all column loads in flight at once (clamped index: no branch)
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t e = min(t0 + (int64_t)j * NT + threadIdx.x, L - 1);
    if constexpr (SRC == kIdxExpand)
      cj[j] = jj[exp_at(ex.sj, exp_pos(ex, e))];
    else
      cj[j] = ld_index<SRC>(jj, e);
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t e = t0 + (int64_t)j * NT + threadIdx.x;
    bn[j] = -1;
    if (e < L) {
      bool ok;
      const int64_t g = global_col<BATCHED>(bd, b, e, cj[j] - 1, n, 0, mb, ok);
      if (ok) {
        bn[j] = (int32_t)bin_of(G, g);
        lo = min(lo, bn[j]);
        hi = max(hi, bn[j]);
      } else {
        bad = true;
      }
    }
  }
}

template <int NT>
__device__ __forceinline__ void block_minmax(int32_t& lo, int32_t& hi,
                                             int32_t* sLo, int32_t* sHi) {
  for (int d = 32; d > 0; d >>= 1) {
    lo = min(lo, __shfl_xor(lo, d, 64));
    hi = max(hi, __shfl_xor(hi, d, 64));
  }
  if (threadIdx.x == 0) {
    *sLo = INT32_MAX;
    *sHi = -1;
  }
  __syncthreads();
  if (lane_id() == 0) {
    atomicMin(sLo, lo);
    atomicMax(sHi, hi);
  }
  __syncthreads();
  lo = *sLo;
  hi = *sHi;
}

template <bool BATCHED, int SRC, int NT, int IPT>
__global__ void __launch_bounds__(NT)
k_count_claim(const int32_t* __restrict__ jj, int64_t L, int32_t n,
              BatchDesc bd, BinGeo G, int32_t WMAX,
              uint32_t* __restrict__ bincnt, Ctrl* ctrl, Expand ex) {
  extern __shared__ uint32_t hist[];
  __shared__ int sB;
  __shared__ int32_t sLo, sHi;
  const int64_t t0 = (int64_t)blockIdx.x * NT * IPT;
  int32_t bn[IPT], cj[IPT], lo, hi;
  bool bad = false;
  tile_bins<BATCHED, SRC, NT, IPT>(jj, L, n, bd, G, t0, &sB, bn, cj, lo, hi, bad, ex);
  block_minmax<NT>(lo, hi, &sLo, &sHi);
  if (bad) atomicOr(&ctrl->err, kErrCol);
  if (hi < lo) return;
  const int width = hi - lo + 1;
  if (width <= WMAX) {
    for (int i = threadIdx.x; i < width; i += NT) hist[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      if (bn[j] >= 0) atomicAdd(&hist[bn[j] - lo], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < width; i += NT)
      if (hist[i]) atomicAdd(&bincnt[lo + i], hist[i]);
  } else {
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      if (bn[j] >= 0) atomicAdd(&bincnt[bn[j]], 1u);
  }
}

template <typename VT, bool BATCHED, bool PACKED, int SRC, int NT, int IPT, bool KEYS>
__global__ void __launch_bounds__(NT)
k_scatter_claim(const int32_t* __restrict__ ii, const int32_t* __restrict__ jj,
                const VT* __restrict__ ss, int64_t L, int32_t m, int32_t n,
                BatchDesc bd, BinGeo G, int32_t WMAX,
                const int32_t* __restrict__ binstart, int32_t slotcap,
                uint32_t* __restrict__ binfill, Entry<VT>* __restrict__ bucket,
                uint32_t* __restrict__ bcol, uint32_t trash, Ctrl* ctrl,
                Expand ex) {
  extern __shared__ uint32_t hist[];
  __shared__ int sB;
  __shared__ int32_t sLo, sHi;
  __shared__ bool sStop;
  const int64_t t0 = (int64_t)blockIdx.x * NT * IPT;
  int32_t bn[IPT], cj[IPT], lo, hi;
  bool bad = false;
  tile_bins<BATCHED, SRC, NT, IPT>(jj, L, n, bd, G, t0, &sB, bn, cj, lo, hi, bad, ex);
  // the rows too, so that their loads overlap the placement
  int32_t rpre[IPT];
  if constexpr (SRC != kIdxExpand) {
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      rpre[j] = ld_index<SRC>(ii, min(t0 + (int64_t)j * NT + threadIdx.x, L - 1));
  }
  // (block_minmax ends with a barrier after thread 0's reads below)
  if (slotcap > 0 && threadIdx.x == 0)
    sStop = (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
             kErrSlot) != 0;
  block_minmax<NT>(lo, hi, &sLo, &sHi);
  // a fixed-capacity bin is full: the call is redone with counts, so the
  // tiles that start later have nothing to place
  if (hi < lo || (slotcap > 0 && sStop)) return;
  const int width = hi - lo + 1;
  const bool narrow = width <= WMAX;
  uint32_t rk[IPT];
  if (narrow) {
    for (int i = threadIdx.x; i < width; i += NT) hist[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      rk[j] = bn[j] >= 0 ? atomicAdd(&hist[bn[j] - lo], 1u) : 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < width; i += NT) {
      const uint32_t h = hist[i];
      if (h) {
        const uint32_t c = atomicAdd(&binfill[lo + i], h);
        hist[i] = (slotcap > 0 ? (uint32_t)(lo + i) * (uint32_t)slotcap
                               : (uint32_t)binstart[lo + i]) + c;
      }
    }
    __syncthreads();
  }
  MatCur b;
  mat_cur<BATCHED>(bd, b, BATCHED ? sB : 0);
  bool badr = false, over = false;
  // kScatterU triplets at a time: their loads together, then their places,
  // then their stores (a triplet without a place goes to the spare place
  // `trash`, so that the stores need no branch)
#pragma unroll
  for (int j0 = 0; j0 < IPT; j0 += kScatterU) {
    int32_t ri[kScatterU];
    VT sv[kScatterU];
#pragma unroll
    for (int u = 0; u < kScatterU; ++u) {
      const int64_t e = min(t0 + (int64_t)(j0 + u) * NT + threadIdx.x, L - 1);
      if constexpr (SRC == kIdxExpand) {
        const ExpPos o = exp_pos(ex, e);
        ri[u] = ii[exp_at(ex.si, o)];
        sv[u] = ss[exp_at(ex.sv, o)];
      } else {
        ri[u] = rpre[j0 + u];
        if constexpr (!KEYS) sv[u] = ss[e];
      }
    }
    uint32_t pos[kScatterU], key[kScatterU], bc[kScatterU];
#pragma unroll
    for (int u = 0; u < kScatterU; ++u) {
      const int j = j0 + u;
      const int64_t e = t0 + (int64_t)j * NT + threadIdx.x;
      pos[u] = trash + (threadIdx.x & (kSpare - 1));
      if (bn[j] >= 0) {
        bool ok;
        int32_t mb;
        const int64_t g = global_col<BATCHED>(bd, b, e, cj[j] - 1, n, m, mb, ok);
        const int32_t r = ri[u] - 1;
        badr |= (uint32_t)r >= (uint32_t)mb;
        uint32_t p;
        if (narrow) {
          p = hist[bn[j] - lo] + rk[j];
        } else {
          const uint32_t c = atomicAdd(&binfill[bn[j]], 1u);
          p = (slotcap > 0 ? (uint32_t)bn[j] * (uint32_t)slotcap : (uint32_t)binstart[bn[j]]) + c;
        }
        if (slotcap > 0 && p - (uint32_t)bn[j] * (uint32_t)slotcap >= (uint32_t)slotcap) {
          over = true;  // this bin is full: the call is redone in two passes
        } else {
          bc[u] = bin_col(G, g, (uint32_t)bn[j]);
          key[u] = PACKED ? (((uint32_t)r << G.s) | bc[u]) : (uint32_t)r;
          pos[u] = p;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kScatterU; ++u) {
      const uint32_t k = (uint32_t)(t0 + (int64_t)(j0 + u) * NT + threadIdx.x);
      if constexpr (KEYS)
        reinterpret_cast<KeyEntry*>(bucket)[pos[u]] = KeyEntry{key[u], k};
      else
        store_entry<VT>(&bucket[pos[u]], key[u], k, sv[u]);
      if (!PACKED) bcol[pos[u]] = bc[u];
    }
  }
  if (badr) atomicOr(&ctrl->err, kErrRow);
  if (over) atomicOr(&ctrl->err, kErrSlot);
}

// ---------------------------------------------------------------------------
// chunk: sort/group/fold one window of the bucket array in LDS
// ---------------------------------------------------------------------------
template <typename VT>
struct ChunkArgs {
  const int32_t* colptr;     // [N+1] triplet column pointers
  const int32_t* chunk_col;  // [Q+1]
  Entry<VT>* bucket;         // [Ltot] (overwritten only on the long path)
  const VT* vals;            // values by triplet when the bins hold KeyEntry
  Entry<VT>* tmp;            // [Ltot] scratch of the long path
  int32_t N;                 // columns (all matrices)
  int32_t T;                 // window length (triplets)
  int32_t cap;               // LDS capacity in use (power of two <= CAP)
  int32_t Q;                 // number of windows
  uint64_t* status;          // [Q] look-back words
  Ctrl* ctrl;
  int32_t* jcS;              // [N+1] column pointers, global numbering
  int32_t* irS;              // [out_cap]
  VT* prS;                   // [out_cap]
  int64_t out_cap;
  int32_t* slot;             // [Ltot] or null
  int32_t* perm;             // [Ltot] or null: k of the p-th sorted triplet
  int32_t* seg;              // [nnz+1] or null: first sorted position of slot
  uint64_t* phase;           // per-bin phase timestamps (profiling builds only)
  Ctrl* hostctrl;            // host-visible copy of err and nnz, or null
  int32_t rshift;            // rows are stored as (row << rshift) | column
  int64_t pshift;            // compact triplet position = bucket position + pshift
  int32_t nbl;               // rank buckets per column: 2^nbl row ranges
  int32_t bsh;               // row >> bsh is the row's range
};

// Look-back words of the bin kernel carry two running sums at once: the
// distinct pairs (low 31 bits) and the binned triplets (next 31 bits).
constexpr uint64_t kLow31 = (1ull << 31) - 1;
__device__ __forceinline__ uint64_t pack_agg(uint64_t triplets, uint64_t pairs) {
  return (triplets << 31) | pairs;
}

// Rank cell of a row word inside its in-bin column.  Rows past m (flagged as
// an index error, but still binned) are clamped into the last range.
template <typename VT>
__device__ __forceinline__ uint32_t rank_cell(const ChunkArgs<VT>& a, uint32_t c,
                                              uint32_t rword) {
  const uint32_t b = (rword >> a.rshift) >> a.bsh;
  return (c << a.nbl) + min(b, (1u << a.nbl) - 1u);
}

// Phase timestamps of the bin kernel, compiled in only with
// -DFSP_PHASE_TIMING (16 slots per bin, 100 MHz wall clock).
#ifdef FSP_PHASE_TIMING
#define FSP_PHASE(a, q, i)                                          \
  if ((a).phase && threadIdx.x == 0)                               \
    (a).phase[(int64_t)(q) * 16 + (i)] = wall_clock64();
#else
#define FSP_PHASE(a, q, i)
#endif

__device__ __forceinline__ uint32_t pair_hash(uint32_t cs, uint32_t row) {
  uint32_t h = cs * 0x9E3779B1u ^ (row + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return h;
}

// LDS carve-up for capacity CAP (bytes):
//   [0, 8CAP)          hash table u32[2CAP] | dlist u32[CAP] + gout u32[CAP]
//                      | placed values VT[CAP] | long path keys u64[CAP]
//   [8CAP, 12CAP)      rows u32[CAP]  | placed k u32[CAP]
//   [12CAP, 16CAP)     column start (+1) per entry | group of placed entry
//                      ([8CAP,16CAP) = long path values VT[CAP])
//   [16CAP, 20CAP)     column end by column start
//   [20CAP, 24CAP)     group counts by representative | sorted index
//   [24CAP, 28CAP)     group row by output index
//   [28CAP, 32CAP+4)   distinct per column start -> exclusive scan
//   [32CAP+4, 36CAP+8) group sizes by output index -> exclusive scan
//   tail               wave totals, misc
template <int CAP>
struct Lds {
  static constexpr int kBytes = 36 * CAP + 8 + 64 * 4 + 8 * 8 + 16;
};

template <typename VT, int CAP, int NT>
struct ChunkCtx {
  unsigned char* smem;
  __device__ uint32_t* ht() const { return reinterpret_cast<uint32_t*>(smem); }
  __device__ uint32_t* dlist() const { return ht(); }
  __device__ uint32_t* gout() const { return ht() + CAP; }
  __device__ VT* mval() const { return reinterpret_cast<VT*>(smem); }
  __device__ uint64_t* lkey() const { return reinterpret_cast<uint64_t*>(smem); }
  __device__ VT* lval() const { return reinterpret_cast<VT*>(smem + 8 * CAP); }
  __device__ uint32_t* row() const { return reinterpret_cast<uint32_t*>(smem + 8 * CAP); }
  __device__ uint32_t* cs() const { return reinterpret_cast<uint32_t*>(smem + 12 * CAP); }
  __device__ uint32_t* cend() const { return reinterpret_cast<uint32_t*>(smem + 16 * CAP); }
  __device__ uint32_t* cnt() const { return reinterpret_cast<uint32_t*>(smem + 20 * CAP); }
  __device__ uint32_t* grow() const { return reinterpret_cast<uint32_t*>(smem + 24 * CAP); }
  __device__ uint32_t* cd() const { return reinterpret_cast<uint32_t*>(smem + 28 * CAP); }
  __device__ uint32_t* gs() const { return reinterpret_cast<uint32_t*>(smem + 32 * CAP + 4); }
  __device__ uint32_t* wave() const { return reinterpret_cast<uint32_t*>(smem + 36 * CAP + 8); }
  __device__ int64_t* misc() const {
    return reinterpret_cast<int64_t*>(smem + 36 * CAP + 8 + 64 * 4 + 8);
  }
};

// Columns [cb, ce) whose triplets are bucket[e0, e1), e1 - e0 <= cap.
// Groups, ranks and folds them.  The output offset of the batch is obtained
// by `base_of(D)` (look-back, or a given offset) once the distinct count D is
// known; with EMIT false only D is computed.  Returns D.
template <typename VT, int CAP, int NT, bool EMIT, typename BaseFn>
__device__ uint32_t batch(const ChunkArgs<VT>& a, const ChunkCtx<VT, CAP, NT>& x,
                          int cb, int ce, int e0, int e1, BaseFn base_of) {
  constexpr int EPT = CAP / NT;
  constexpr int H = 2 * CAP;
  const int tid = threadIdx.x;
  const int span = e1 - e0;
  uint32_t* ht = x.ht();
  uint32_t* row = x.row();
  uint32_t* cs = x.cs();
  uint32_t* cend = x.cend();
  uint32_t* cnt = x.cnt();
  uint32_t* cd = x.cd();

  // P1: clear, load, mark column starts
  for (int i = tid; i < H; i += NT) ht[i] = kEmpty;
  for (int i = tid; i < span; i += NT) {
    cs[i] = 0;
    cnt[i] = 0;
    cd[i] = 0;
  }
  if (tid == 0) cd[span] = 0;
  uint32_t kr[EPT];
  VT vr[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span) {
      const Entry<VT> en = load_entry<VT>(&a.bucket[e0 + i]);
      row[i] = en.row;
      kr[j] = en.k;
      vr[j] = en.v;
    }
  }
  __syncthreads();
  for (int c = cb + tid; c < ce; c += NT) {
    const int s = a.colptr[c] - e0, t = a.colptr[c + 1] - e0;
    if (t > s) {
      cs[s] = (uint32_t)s + 1u;
      cend[s] = (uint32_t)t;
    }
  }
  __syncthreads();
  lds_incl_max<NT>(cs, span, x.wave());

  // P2: group equal (column, row) pairs with a hash table of entry indices
  uint32_t repa[EPT], dpos[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span) {
      const uint32_t c0 = cs[i], r0 = row[i];
      uint32_t h = pair_hash(c0, r0) & (H - 1);
      uint32_t rep;
      for (;;) {
        const uint32_t old = atomicCAS(&ht[h], kEmpty, (uint32_t)i);
        if (old == kEmpty) { rep = (uint32_t)i; break; }
        if (cs[old] == c0 && row[old] == r0) { rep = old; break; }
        h = (h + 1) & (H - 1);
      }
      const uint32_t arr = atomicAdd(&cnt[rep], 1u);
      repa[j] = rep | (arr << 16);
      dpos[j] = (rep == (uint32_t)i) ? atomicAdd(&cd[c0 - 1], 1u) : kEmpty;
    }
  }
  __syncthreads();

  // P3: distinct pairs before each position; the batch's output offset
  const uint32_t D = lds_excl_scan<NT>(cd, span + 1, x.wave());
  if (EMIT) {
    if (tid < 64) {
      const int64_t b = base_of(D);
      if (tid == 0) x.misc()[1] = b;
    }
  } else {
    return D;
  }
  uint32_t* dlist = x.dlist();
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span && dpos[j] != kEmpty) dlist[cd[cs[i] - 1] + dpos[j]] = (uint32_t)i;
  }
  __syncthreads();

  // P4: rank the distinct rows of every column
  uint32_t* gout = x.gout();
  uint32_t* gs = x.gs();
  uint32_t* grow = x.grow();
  for (int d = tid; d < (int)D; d += NT) {
    const uint32_t i = dlist[d];
    const uint32_t c0 = cs[i] - 1;
    const uint32_t r0 = row[i];
    const uint32_t lo = cd[c0], hi = cd[cend[c0]];
    uint32_t rk = 0;
    for (uint32_t t = lo; t < hi; ++t) rk += row[dlist[t]] < r0 ? 1u : 0u;
    const uint32_t o = lo + rk;
    gout[i] = o;
    gs[o] = cnt[i];
    grow[o] = r0;
  }
  if (tid == 0) gs[D] = 0;
  __syncthreads();

  // P5: start of every group in the sorted order
  lds_excl_scan<NT>(gs, (int)D + 1, x.wave());

  // P6: place every triplet into its group (arrival order for now)
  uint32_t posr[EPT], orr[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span) {
      const uint32_t o = gout[repa[j] & 0xFFFFu];
      orr[j] = o;
      posr[j] = gs[o] + (repa[j] >> 16);
    }
  }
  __syncthreads();
  VT* mval = x.mval();
  uint32_t* mk = row;   // k of placed triplets
  uint32_t* mgrp = cs;  // group of placed triplets
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span) {
      mk[posr[j]] = kr[j];
      mval[posr[j]] = vr[j];
      mgrp[posr[j]] = orr[j];
    }
  }
  __syncthreads();

  // P7: order each group's triplets by k (rank by counting)
  // order each group by k: values go straight to their sorted place (the
  // column-end / count arrays are free by now), so do the k of the plan
  VT* sval = reinterpret_cast<VT*>(x.cend());
  for (int p = tid; p < span; p += NT) {
    const uint32_t o = mgrp[p];
    const uint32_t g0 = gs[o], g1 = gs[o + 1];
    const uint32_t kk = mk[p];
    uint32_t r4[4] = {0u, 0u, 0u, 0u};
    uint32_t t = g0;
    for (; t + 4 <= g1; t += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) r4[u] += mk[t + u] < kk ? 1u : 0u;
    }
    uint32_t rk = (r4[0] + r4[1]) + (r4[2] + r4[3]);
    for (; t < g1; ++t) rk += mk[t] < kk ? 1u : 0u;
    sval[g0 + rk] = mval[p];
    if (a.perm) a.perm[e0 + g0 + rk + a.pshift] = (int32_t)kk;
  }
  __syncthreads();

  // P8: emit
  const int64_t base = x.misc()[1];
  if (a.slot)
    for (int p = tid; p < span; p += NT) a.slot[mk[p]] = (int32_t)(base + mgrp[p]);
  bool over = false;
  for (int o = tid; o < (int)D; o += NT) {
    const uint32_t g0 = gs[o], g1 = gs[o + 1];
    // left fold from +0.0 in increasing k; loads four ahead
    VT acc = (VT)0;
    uint32_t t = g0;
    for (; t + 4 <= g1; t += 4) {
      const VT v0 = sval[t], v1 = sval[t + 1], v2 = sval[t + 2], v3 = sval[t + 3];
      acc = acc + v0;
      acc = acc + v1;
      acc = acc + v2;
      acc = acc + v3;
    }
    for (; t < g1; ++t) acc = acc + sval[t];
    const int64_t out = base + o;
    if (out < a.out_cap) {
      a.irS[out] = (int32_t)(grow[o] >> a.rshift);
      a.prS[out] = acc;
    } else {
      over = true;
    }
    if (a.seg) a.seg[out] = (int32_t)(e0 + g0 + a.pshift);
  }
  if (over) atomicOr(&a.ctrl->err, kErrCap);
  for (int c = cb + tid; c < ce; c += NT)
    a.jcS[c] = (int32_t)(base + cd[a.colptr[c] - e0]);
  __syncthreads();
  return D;
}

// ---- long path: one column with more triplets than the LDS holds --------
__device__ __forceinline__ uint64_t ekey(uint32_t row, uint32_t k) {
  return ((uint64_t)row << 32) | (uint64_t)k;
}

// Sorts bucket[a0, a0+len) by (row, k) with a bitonic sort of LDS tiles
// followed by merge passes between `bucket` and `tmp`; returns which array
// holds the result (0 = bucket, 1 = tmp).
template <typename VT, int CAP, int NT>
__device__ int long_sort(const ChunkArgs<VT>& a, const ChunkCtx<VT, CAP, NT>& x,
                         int a0, int len) {
  const int tid = threadIdx.x;
  const int TS = a.cap;
  uint64_t* key = x.lkey();
  VT* val = x.lval();
  for (int t0 = 0; t0 < len; t0 += TS) {
    const int tl = min(TS, len - t0);
    int P = 1;
    while (P < tl) P <<= 1;
    for (int i = tid; i < P; i += NT) {
      if (i < tl) {
        const Entry<VT> en = load_entry<VT>(&a.bucket[a0 + t0 + i]);
        key[i] = ekey(en.row, en.k);
        val[i] = en.v;
      } else {
        key[i] = ~0ull;
        val[i] = (VT)0;
      }
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < P / 2; i += NT) {
          const int lo = 2 * i - (i & (j - 1));
          const int hi = lo + j;
          const bool up = (lo & k) == 0;
          const uint64_t kl = key[lo], kh = key[hi];
          if ((kl > kh) == up) {
            key[lo] = kh;
            key[hi] = kl;
            const VT t = val[lo];
            val[lo] = val[hi];
            val[hi] = t;
          }
        }
        __syncthreads();
      }
    }
    for (int i = tid; i < tl; i += NT)
      store_entry<VT>(&a.tmp[a0 + t0 + i], (uint32_t)(key[i] >> 32),
                      (uint32_t)key[i], val[i]);
    __syncthreads();
  }
  __threadfence();
  __syncthreads();
  Entry<VT>* src = a.tmp;
  Entry<VT>* dst = a.bucket;
  int where = 1;
  for (int w = TS; w < len; w <<= 1) {
    for (int idx = tid; idx < len; idx += NT) {
      const int r = idx / w;
      const int ps = (r & ~1) * w;  // start of the pair of runs
      const int i = idx - r * w;
      const Entry<VT> en = load_entry<VT>(&src[a0 + idx]);
      const uint64_t kk = ekey(en.row, en.k);
      int os, ol;  // other run
      if ((r & 1) == 0) {
        os = (r + 1) * w;
        ol = max(0, min(w, len - os));
      } else {
        os = (r - 1) * w;
        ol = w;
      }
      int lo = 0, hi = ol;  // count of other-run keys below kk
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const Entry<VT> om = load_entry<VT>(&src[a0 + os + mid]);
        if (ekey(om.row, om.k) < kk) lo = mid + 1; else hi = mid;
      }
      store_entry<VT>(&dst[a0 + ps + i + lo], en.row, en.k, en.v);
    }
    __threadfence();
    __syncthreads();
    Entry<VT>* t = src;
    src = dst;
    dst = t;
    where ^= 1;
  }
  return where;
}

// Distinct rows of a sorted long column.
template <typename VT, int NT>
__device__ uint32_t long_count(const Entry<VT>* s, int a0, int len,
                               uint32_t* sWave) {
  uint32_t c = 0;
  for (int p = threadIdx.x; p < len; p += NT) {
    const uint32_t r = s[a0 + p].row;
    c += (p == 0 || s[a0 + p - 1].row != r) ? 1u : 0u;
  }
  uint32_t total;
  block_excl_sum<NT>(c, sWave, total);
  return total;
}

// Emits a sorted long column whose first output slot is `base`.
template <typename VT, int CAP, int NT>
__device__ void long_emit(const ChunkArgs<VT>& a, const ChunkCtx<VT, CAP, NT>& x,
                          const Entry<VT>* s, int a0, int len, int64_t base) {
  const int tid = threadIdx.x;
  bool over = false;
  int64_t run = 0;  // heads before the current tile
  for (int t0 = 0; t0 < len; t0 += NT) {
    const int p = t0 + tid;
    uint32_t head = 0;
    uint32_t r = 0;
    if (p < len) {
      r = s[a0 + p].row;
      head = (p == 0 || s[a0 + p - 1].row != r) ? 1u : 0u;
    }
    uint32_t total;
    const uint32_t pre = block_excl_sum<NT>(head, x.wave(), total);
    if (p < len) {
      const int64_t g = run + pre + head - 1;  // group of position p
      const int64_t out = base + g;
      const Entry<VT> en = s[a0 + p];
      if (a.perm) a.perm[a0 + p + a.pshift] = (int32_t)en.k;
      if (a.slot) a.slot[en.k] = (int32_t)out;
      if (head) {
        VT acc = (VT)0;
        int t = p;
        do {
          acc = acc + s[a0 + t].v;
          ++t;
        } while (t < len && s[a0 + t].row == r);
        if (out < a.out_cap) {
          a.irS[out] = (int32_t)(r >> a.rshift);
          a.prS[out] = acc;
        } else {
          over = true;
        }
        if (a.seg) a.seg[out] = (int32_t)(a0 + p + a.pshift);
      }
    }
    run += total;
  }
  if (over) atomicOr(&a.ctrl->err, kErrCap);
  __syncthreads();
}

// Columns [cb, cl) whose triplets do not fit the LDS at once: they are taken
// in batches of consecutive columns that fit, and columns longer than the
// capacity take the long path.  One sweep either counts the distinct pairs
// (emit false; long columns are sorted here) or emits them from output
// offset `off` on (a.pshift set).  Returns the offset after the last pair.
template <typename VT, int CAP, int NT>
__device__ int64_t chunk_sweep(ChunkArgs<VT>& a, const ChunkCtx<VT, CAP, NT>& x,
                               int cb, int cl, bool emit, int64_t off) {
  int64_t* misc = x.misc();
  int c = cb;
  while (c < cl) {
    __syncthreads();
    if (threadIdx.x == 0) {
      // largest ce in (c, cl] with colptr[ce] - colptr[c] <= cap
      const int64_t lim = (int64_t)a.colptr[c] + a.cap;
      int lo = c, hi = cl;  // colptr[lo] - colptr[c] <= cap
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.colptr[mid] <= lim) lo = mid; else hi = mid - 1;
      }
      misc[2] = (lo == c) ? c + 1 : lo;
      misc[3] = (lo == c) ? 1 : 0;
    }
    __syncthreads();
    const int ce = (int)misc[2];
    const bool is_long = misc[3] != 0;
    const int e0 = a.colptr[c], e1 = a.colptr[ce];
    uint32_t D;
    if (is_long) {
      int where;
      if (!emit) {
        where = long_sort<VT, CAP, NT>(a, x, e0, e1 - e0);
      } else {
        // same pass count as in the counting sweep
        where = 1;
        for (int w = a.cap; w < e1 - e0; w <<= 1) where ^= 1;
      }
      const Entry<VT>* s = where ? a.tmp : a.bucket;
      D = long_count<VT, NT>(s, e0, e1 - e0, x.wave());
      if (emit) {
        if (threadIdx.x == 0) a.jcS[c] = (int32_t)off;
        long_emit<VT, CAP, NT>(a, x, s, e0, e1 - e0, off);
      }
    } else if (!emit) {
      D = batch<VT, CAP, NT, false>(a, x, c, ce, e0, e1,
                                    [](uint32_t) -> int64_t { return 0; });
      __syncthreads();
    } else {
      const int64_t o = off;
      D = batch<VT, CAP, NT, true>(a, x, c, ce, e0, e1,
                                   [o](uint32_t) -> int64_t { return o; });
    }
    off += D;
    c = ce;
  }
  __syncthreads();
  return off;
}

// ---------------------------------------------------------------------------
// bin kernel: one workgroup per bin of w consecutive columns
// ---------------------------------------------------------------------------

// Where the bins are and how blocks take them.
struct BinSrc {
  const int32_t* binstart;  // [B+1] (counted modes)
  const uint32_t* binfill;  // [B] (fixed-capacity mode)
  const uint32_t* bcol;     // in-bin columns, or null for packed keys
  int32_t slotcap;          // > 0: bin q owns places [q*slotcap, (q+1)*slotcap)
  int32_t B;
  uint32_t* tick;
  const uint32_t* slowD;    // distinct pairs of each slow bin
  uint64_t* slowB;          // look-back prefix of each slow bin (written)
};

// A bin's range in the bucket and, when it fits the LDS, its entries in
// registers: the bin kernel loads the next bin while finishing the current.
template <typename VT, int EPT, bool KEYS>
struct BinRegs {
  int q, e0, e1;
  typename std::conditional<KEYS, KeyEntry, Entry<VT>>::type en[EPT];
};

// Issue the loads of bin q's range.  The same three words are read in every
// mode (binstart always has B+1 entries and binfill B), and nothing is
// computed from them yet, so the loads stay in flight until bin_range.
// One vector load with a different word per lane (lane 0 binstart[q],
// lane 1 binstart[q+1], lane 2 binfill[q]): a wave-uniform load would be
// moved to scalar registers, and waited for, at once.  A ticket past the
// last bin reads bin B-1's words; bin_range then makes its range empty.
template <class R>
__device__ __forceinline__ void bin_bounds(const BinSrc& src, R& r, uint32_t& w) {
  const int qc = min(r.q, src.B - 1);
  const int lane = lane_id();
  const uint32_t* p = lane == 2 ? &src.binfill[qc]
                                : reinterpret_cast<const uint32_t*>(&src.binstart[qc + (lane & 1)]);
  w = *p;
}

template <class R>
__device__ __forceinline__ void bin_range(const BinSrc& src, R& r, uint32_t w) {
  r.e0 = (int)__builtin_amdgcn_readlane(w, 0);
  r.e1 = (int)__builtin_amdgcn_readlane(w, 1);
  const uint32_t fill = __builtin_amdgcn_readlane(w, 2);
  if (src.slotcap > 0) {
    r.e0 = r.q * src.slotcap;
    r.e1 = r.e0 + (int)min(fill, (uint32_t)src.slotcap);
  }
  if (r.q >= src.B) r.e0 = r.e1 = 0;
}

// The same EPT loads on every path (indices clamped into the bin, an empty
// bin reading its first place, which is at most the bucket's spare place),
// so that later waits for other loads never have to cover these.  A slow
// bin's entries are not used (the slow path reads the bucket).
template <typename VT, int NT, int EPT, bool KEYS>
__device__ __forceinline__ void bin_load(const ChunkArgs<VT>& a, const BinSrc& src,
                                         BinRegs<VT, EPT, KEYS>& r) {
  const int last = max(r.e1 - r.e0 - 1, 0);
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = threadIdx.x + j * NT;
    if constexpr (KEYS)
      r.en[j] = reinterpret_cast<const KeyEntry*>(a.bucket)[r.e0 + min(i, last)];
    else
      r.en[j] = load_entry<VT>(&a.bucket[r.e0 + min(i, last)]);
  }
}

// LDS of the bin kernel (bytes, capacity CAP).  The small arrays that
// threads address by their own index come first, where LDS instructions
// reach them by immediate offsets (below 64 KB), then three regions of 8CAP
// bytes whose tenants change phase by phase (see bin_fast), and 32 bytes of
// padding for reads past the last region's end.
constexpr int al16(int x) { return (x + 15) & ~15; }
template <int CAP>
struct BinLds {
  static constexpr int kMisc = 0;                          // int64[8]
  static constexpr int kWave = 64;                         // u32[64]
  static constexpr int kCd = 320;                          // u32[CAP+1]
  static constexpr int kGs = al16(kCd + 4 * (CAP + 1));    // u32[CAP+1]
  static constexpr int kGrow = al16(kGs + 4 * (CAP + 1));  // u32[CAP]
  static constexpr int kR0 = al16(kGrow + 4 * CAP);
  static constexpr int kR1 = kR0 + 8 * CAP;
  static constexpr int kR2 = kR1 + 8 * CAP;
  static constexpr int kBytes = kR2 + 8 * CAP + 32;
};

// Fast path: the bin's triplets fit the LDS and are already in registers.
// Equal (column,row) pairs are grouped by hashing straight away and the
// triplets of a pair are counted at their pair's hash slot.  Each rank cell
// (a column's row range) counts its distinct pairs and, once the groups are
// complete, their triplets, in one packed word, so one scan of the cells
// gives the column offsets, a coarse rank and the first place of every
// cell's triplets.  Ranking the distinct rows of a cell then also gives
// their groups' first places (no scan of the group sizes).  Contributions of
// a pair are put in increasing k and folded from +0.0.  Meanwhile the next
// bin (ticket `tk`, taken by thread 0) has its range and entries fetched
// into `nx`.  Returns base + distinct count.
//
// LDS (BinLds; a region's later tenants take it once the earlier ones are
// dead):
//   R0 (8CAP)   hash keys u32[2CAP] -> distinct list u32[CAP]
//               -> placed values VT[CAP]
//   R1 (8CAP)   triplets per hash slot u32[2CAP] -> (output, first place)
//               per hash slot -> k-ordered values VT[CAP]
//   R2 (8CAP)   entry rows and columns u32[CAP] each (unshared columns)
//               -> (row, triplets) per distinct u32x2[CAP] -> placed k
//               u32[CAP] + group of placed u32[CAP]
//   grow        row of each output
//   cd          (distinct, triplets) per rank cell, then scanned
//   gs          first place of each output's group (+ the end)
template <typename VT, int CAP, int NT, bool KEYS>
__device__ int64_t bin_fast(const ChunkArgs<VT>& a, const BinSrc& src,
                            const ChunkCtx<VT, CAP, NT>& x,
                            const BinRegs<VT, CAP / NT, KEYS>& cur, int c0, int c1,
                            uint32_t tk, BinRegs<VT, CAP / NT, KEYS>& nx) {
  constexpr int EPT = CAP / NT;
  constexpr int H = 2 * CAP;
  const int tid = threadIdx.x;
  const int q = cur.q, e0 = cur.e0, e1 = cur.e1;
  const int span = e1 - e0;
  const int wc = c1 - c0;
  const uint32_t cmask = (1u << a.rshift) - 1u;  // packed keys only
  // packed words are unique keys of the (column, row) pairs (never kEmpty):
  // the hash table then holds the keys themselves, else entry indices
  const bool keyed = src.bcol == nullptr;
  FSP_PHASE(a, q, 1)
  using LY = BinLds<CAP>;
  unsigned char* sm = x.smem;
  int64_t* misc = reinterpret_cast<int64_t*>(sm + LY::kMisc);
  uint32_t* wave = reinterpret_cast<uint32_t*>(sm + LY::kWave);
  uint32_t* ht = reinterpret_cast<uint32_t*>(sm + LY::kR0);
  uint32_t* dlist = ht;
  VT* mval = reinterpret_cast<VT*>(sm + LY::kR0);
  uint32_t* hcnt = reinterpret_cast<uint32_t*>(sm + LY::kR1);
  VT* sval = reinterpret_cast<VT*>(sm + LY::kR1);
  uint32_t* row = reinterpret_cast<uint32_t*>(sm + LY::kR2);
  uint32_t* col = reinterpret_cast<uint32_t*>(sm + LY::kR2 + 4 * CAP);
  uint2* drc = reinterpret_cast<uint2*>(sm + LY::kR2);
  uint32_t* mk = reinterpret_cast<uint32_t*>(sm + LY::kR2);
  uint32_t* mgrp = reinterpret_cast<uint32_t*>(sm + LY::kR2 + 4 * CAP);
  uint32_t* grow = reinterpret_cast<uint32_t*>(sm + LY::kGrow);
  uint32_t* cd = reinterpret_cast<uint32_t*>(sm + LY::kCd);
  uint32_t* gs = reinterpret_cast<uint32_t*>(sm + LY::kGs);

  // rank cells: distinct pairs (low half) and triplets (high half) of each
  // (column, row range) cell
  const int ncell = wc << a.nbl;
  {
    uint4* h4 = reinterpret_cast<uint4*>(ht);
    uint4* c4 = reinterpret_cast<uint4*>(hcnt);
    const uint4 e = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int i = tid; i < H / 4; i += NT) {
      h4[i] = e;
      c4[i] = z;
    }
  }
  for (int i = tid; i <= ncell; i += NT) cd[i] = 0u;
  uint32_t rr[EPT], kr[EPT];
  VT vr[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    rr[j] = cur.en[j].row;
    kr[j] = cur.en[j].k;
    if constexpr (KEYS) {
      // read by k now, first used when the triplets are placed
      vr[j] = (VT)0;
      if (tid + j * NT < span) vr[j] = a.vals[kr[j]];
    } else {
      vr[j] = cur.en[j].v;
    }
  }
  if (!keyed) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = tid + j * NT;
      if (i < span) {
        row[i] = rr[j];
        col[i] = src.bcol[e0 + i];
      }
    }
  }
  __syncthreads();

  FSP_PHASE(a, q, 2)
  // group equal (column,row) pairs.  The first probes of all of a thread's
  // triplets are issued together, then collisions are resolved, then the
  // slot and cell counters are bumped, so the LDS atomics overlap.  The
  // triplet that claims an empty slot represents its pair.
  // hh: hash slot, then slot | arrival << 16; cell: rank cell, then
  // cell | place among its cell's distinct pairs << 16 (0xFFFF: not a
  // representative)
  uint32_t hh[EPT], cell[EPT], arr[EPT];
  if (keyed) {
    // the table holds keys; a probe ends at an empty slot or at its own key
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = tid + j * NT;
      if (i < span) {
        const uint32_t r = rr[j];
        cell[j] = rank_cell(a, r & cmask, r);
        hh[j] = pair_hash(r & cmask, r) & (H - 1);
        arr[j] = atomicCAS(&ht[hh[j]], kEmpty, r);
      }
    }
    FSP_PHASE(a, q, 10)
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = tid + j * NT;
      if (i < span) {
        // triangular probing: growing steps visit every slot of the
        // power-of-two table without building long runs
        const uint32_t r = rr[j];
        uint32_t old = arr[j], h = hh[j], step = 1;
        while (old != kEmpty && old != r) {
          h = (h + step++) & (H - 1);
          old = atomicCAS(&ht[h], kEmpty, r);
        }
        hh[j] = h;
        arr[j] = old;
      }
    }
  } else {
    // the table holds entry indices; a probe compares the stored pair
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = tid + j * NT;
      if (i < span) {
        const uint32_t c = col[i], r = rr[j];
        cell[j] = rank_cell(a, c, r);
        hh[j] = pair_hash(c, r) & (H - 1);
        arr[j] = atomicCAS(&ht[hh[j]], kEmpty, (uint32_t)i);
      }
    }
    FSP_PHASE(a, q, 10)
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = tid + j * NT;
      if (i < span) {
        uint32_t old = arr[j], h = hh[j], step = 1;
        if (old != kEmpty) {
          const uint32_t c = col[i], r = rr[j];
          while (old != kEmpty) {
            if (col[old] == c && row[old] == r) break;
            h = (h + step++) & (H - 1);
            old = atomicCAS(&ht[h], kEmpty, (uint32_t)i);
          }
        }
        hh[j] = h;
        arr[j] = old;
      }
    }
  }
  FSP_PHASE(a, q, 11)
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span) {
      const bool rep = arr[j] == kEmpty;
      const uint32_t av = atomicAdd(&hcnt[hh[j]], 1u);
      const uint32_t cw = rep ? atomicAdd(&cd[cell[j]], 0x10001u) : 0xFFFFu;
      hh[j] |= av << 16;
      cell[j] |= (cw & 0xFFFFu) << 16;
    }
  }
  FSP_PHASE(a, q, 12)
  if (tid == 0) misc[7] = tk;
  FSP_PHASE(a, q, 13)
  __syncthreads();
  // the groups are complete: representatives add the rest of their group's
  // triplets to their cell
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span && (cell[j] >> 16) != 0xFFFFu) {
      const uint32_t c = hcnt[hh[j] & 0xFFFFu];
      if (c > 1u) atomicAdd(&cd[cell[j] & 0xFFFFu], (c - 1u) << 16);
    }
  }
  __syncthreads();
  // next bin: its range now, its entries once the placement is done
  nx.q = (int)misc[7];
  uint32_t nfill = 0;
  bin_bounds(src, nx, nfill);

  FSP_PHASE(a, q, 3)
  // distinct pairs and triplets per cell -> offsets; publish the bin's count
  // now, read the prefix of the earlier bins only when emitting
  const uint32_t D = lds_excl_scan<NT>(cd, ncell + 1, wave) & 0xFFFFu;
  if (tid < 64) lookback_publish(a.status, q, pack_agg((uint64_t)span, D));
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span && (cell[j] >> 16) != 0xFFFFu) {
      const uint32_t cl = cell[j] & 0xFFFFu, h = hh[j] & 0xFFFFu;
      const uint32_t d = (cd[cl] & 0xFFFFu) + (cell[j] >> 16);
      dlist[d] = h | (cl << 16);
      drc[d] = make_uint2(rr[j], hcnt[h]);
    }
  }
  __syncthreads();

  FSP_PHASE(a, q, 4)
  // rank the distinct rows of every cell; the triplets of the smaller rows
  // give the group's first place.  Each hash slot then holds its pair's
  // output index (low half) and first place (high half).
  // (EPT distinct rows per thread at a time, so that their loads overlap)
  for (int d0 = tid; d0 < (int)D; d0 += EPT * NT) {
    uint32_t dw[EPT], lo[EPT], hi[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int d = d0 + u * NT;
      dw[u] = d < (int)D ? dlist[d] : kEmpty;
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      if (dw[u] != kEmpty) {
        const uint32_t cl = dw[u] >> 16;
        lo[u] = cd[cl];
        hi[u] = cd[cl + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      if (dw[u] == kEmpty) continue;
      // count smaller rows and their triplets, four reads in flight per
      // step; reads past the cell's end stay inside the LDS block and are
      // masked out
      const uint32_t r0 = drc[d0 + u * NT].x, t0 = lo[u] & 0xFFFFu, e = hi[u] & 0xFFFFu;
      uint32_t rk = 0, tri = 0;
      for (uint32_t t = t0; t < e; t += 4) {
        const uint2 v0 = drc[t], v1 = drc[t + 1], v2 = drc[t + 2], v3 = drc[t + 3];
        const bool b0 = v0.x < r0, b1 = t + 1 < e && v1.x < r0;
        const bool b2 = t + 2 < e && v2.x < r0, b3 = t + 3 < e && v3.x < r0;
        rk += (b0 ? 1u : 0u) + (b1 ? 1u : 0u) + (b2 ? 1u : 0u) + (b3 ? 1u : 0u);
        tri += (b0 ? v0.y : 0u) + (b1 ? v1.y : 0u) + (b2 ? v2.y : 0u) + (b3 ? v3.y : 0u);
      }
      const uint32_t o = t0 + rk;
      const uint32_t g = (lo[u] >> 16) + tri;
      hcnt[dw[u] & 0xFFFFu] = o | (g << 16);
      grow[o] = r0;
      gs[o] = g;
    }
  }
  if (tid == 0) gs[D] = (uint32_t)span;
  __syncthreads();
  FSP_PHASE(a, q, 5)
  // every pair occurs once (common for scattered inputs): group o is the
  // single place o, so there is nothing to order by k
  const bool uniq = D == (uint32_t)span;
  FSP_PHASE(a, q, 6)

  // values in sorted place: the placed values themselves when every pair
  // occurs once, else the k-ordered copy
  VT* ovals = uniq ? mval : sval;
  // sorted position of a triplet: its own (every pair once: its output
  // index), else the placed one's
  uint32_t spos[EPT];
  uint64_t probe = 0;
  // place triplets into their groups (by arrival), to be ordered by k
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int i = tid + j * NT;
    if (i < span) {
      const uint32_t w = hcnt[hh[j] & 0xFFFFu];
      const uint32_t o = w & 0xFFFFu;
      const uint32_t p = (w >> 16) + (hh[j] >> 16);
      spos[j] = p;
      mval[p] = vr[j];
      if (!uniq) {
        mk[p] = kr[j];
        mgrp[p] = o;
      }
    }
  }
  bin_range(src, nx, nfill);
  bin_load<VT, NT, EPT, KEYS>(a, src, nx);
  if (tid < 64) probe = lookback_probe(a.status, q);
  if (!uniq) {
    __syncthreads();
    FSP_PHASE(a, q, 15)
    // order each group by k: values go straight to their sorted place, so do
    // the k of the plan
#pragma unroll
    for (int jj = 0; jj < EPT; ++jj) {
      const int p = tid + jj * NT;
      if (p >= span) break;
      const uint32_t o = mgrp[p];
      const uint32_t g0 = gs[o], g1 = gs[o + 1];
      const uint32_t kk = mk[p];
      // eight reads in flight per step while eight remain, then four, then
      // one at a time
      uint32_t r8[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
      uint32_t t = g0;
      for (; t + 8 <= g1; t += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) r8[u] += mk[t + u] < kk ? 1u : 0u;
      }
      if (t + 4 <= g1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) r8[u] += mk[t + u] < kk ? 1u : 0u;
        t += 4;
      }
      uint32_t rk = ((r8[0] + r8[1]) + (r8[2] + r8[3])) + ((r8[4] + r8[5]) + (r8[6] + r8[7]));
      for (; t + 2 <= g1; t += 2) {
        const uint32_t v0 = mk[t], v1 = mk[t + 1];
        rk += (v0 < kk ? 1u : 0u) + (v1 < kk ? 1u : 0u);
      }
      if (t < g1) rk += mk[t] < kk ? 1u : 0u;
      sval[g0 + rk] = mval[p];
      spos[jj] = g0 + rk;
    }
  }
  FSP_PHASE(a, q, 7)
  if (tid < 64) {
    const int64_t b = lookback_wait(a.status, q, pack_agg((uint64_t)span, D), probe);
    if (tid == 0) {
      misc[1] = b & kLow31;
      misc[5] = (b >> 31) + span;  // compact triplets up to this bin's end
      misc[6] = (b >> 31) - e0;
    }
  }
  __syncthreads();
  FSP_PHASE(a, q, 9)

  // emit
  const int64_t base = misc[1];
  const int64_t pshift = misc[6];
  // perm and slot: from the thread's own triplets (uniq), else from the
  // placed ones
  if (a.perm) {
#pragma unroll
    for (int jj = 0; jj < EPT; ++jj) {
      const int p = tid + jj * NT;
      if (p < span) a.perm[e0 + spos[jj] + pshift] = (int32_t)(uniq ? kr[jj] : mk[p]);
    }
  }
  if (a.slot) {
    if (uniq) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int i = tid + j * NT;
        if (i < span) a.slot[kr[j]] = (int32_t)(base + spos[j]);
      }
    } else {
      for (int p = tid; p < span; p += NT) a.slot[mk[p]] = (int32_t)(base + mgrp[p]);
    }
  }
  // a thread's outputs (at most EPT: D <= span <= CAP) go through each step
  // together, so that their LDS reads overlap: bounds and rows, first terms,
  // remaining terms, stores
  bool over = false;
  uint32_t g0[EPT], g1[EPT], rw[EPT];
  VT acc[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int o = tid + u * NT;
    g0[u] = 0u;
    g1[u] = 0u;
    if (o < (int)D) {
      g0[u] = uniq ? (uint32_t)o : gs[o];
      g1[u] = uniq ? (uint32_t)o + 1u : gs[o + 1];
      rw[u] = grow[o];
    }
  }
  // left fold from +0.0 in increasing k
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    acc[u] = (VT)0;
    if (g0[u] < g1[u]) acc[u] = acc[u] + ovals[g0[u]];
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    uint32_t t = g0[u] + 1u;
    for (; t + 4 <= g1[u]; t += 4) {
      const VT v0 = ovals[t], v1 = ovals[t + 1], v2 = ovals[t + 2], v3 = ovals[t + 3];
      acc[u] = acc[u] + v0;
      acc[u] = acc[u] + v1;
      acc[u] = acc[u] + v2;
      acc[u] = acc[u] + v3;
    }
    for (; t < g1[u]; ++t) acc[u] = acc[u] + ovals[t];
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int o = tid + u * NT;
    if (o < (int)D) {
      const int64_t out = base + o;
      if (out < a.out_cap) {
        a.irS[out] = (int32_t)(rw[u] >> a.rshift);
        a.prS[out] = acc[u];
      } else {
        over = true;
      }
      if (a.seg) a.seg[out] = (int32_t)(e0 + g0[u] + pshift);
    }
  }
  if (over) atomicOr(&a.ctrl->err, kErrCap);
  for (int c = tid; c < wc; c += NT)
    a.jcS[c0 + c] = (int32_t)(base + (cd[c << a.nbl] & 0xFFFFu));
  FSP_PHASE(a, q, 8)
  return base + D;
}

// Bins with more triplets than the LDS holds ("slow" bins) are listed by the
// bin scan and handled outside the bin kernel: k_slow_count sorts each by
// column into the scratch array and counts its distinct pairs, the bin
// kernel only passes that count through the look-back (recording the
// prefix), and k_slow_emit emits the bin from the recorded prefix.  Between
// the two, the bin kernel touches no slow bin's data.

// Column-sorts slow bin [e0, e1) (columns [c0, c1)) into the scratch array
// by a counting sort in LDS, writes its column pointers, and points `a` at
// the sorted copy.
template <typename VT, int CAP, int NT>
__device__ void slow_sort(ChunkArgs<VT>& a, const uint32_t* __restrict__ bcol,
                          int32_t* __restrict__ colptr_g,
                          const ChunkCtx<VT, CAP, NT>& x, int c0, int c1, int e0,
                          int e1) {
  const int tid = threadIdx.x;
  const int span = e1 - e0;
  const int wc = c1 - c0;
  uint32_t* hist = x.cd();  // CAP+1 entries, wc <= CAP
  for (int i = tid; i <= wc; i += NT) hist[i] = 0u;
  __syncthreads();
  const uint32_t cmask = (1u << a.rshift) - 1u;
  auto colof = [&](int i) -> uint32_t {
    return bcol ? bcol[e0 + i] : (a.bucket[e0 + i].row & cmask);
  };
  for (int i = tid; i < span; i += NT) atomicAdd(&hist[colof(i)], 1u);
  __syncthreads();
  lds_excl_scan<NT>(hist, wc + 1, x.wave());
  for (int c = tid; c <= wc; c += NT) colptr_g[c0 + c] = e0 + (int32_t)hist[c];
  __syncthreads();
  for (int i = tid; i < span; i += NT) {
    const uint32_t p = atomicAdd(&hist[colof(i)], 1u);
    const Entry<VT> en = load_entry<VT>(&a.bucket[e0 + i]);
    store_entry<VT>(&a.tmp[e0 + p], en.row, en.k, en.v);
  }
  __threadfence();
  __syncthreads();
  a.colptr = colptr_g;
  Entry<VT>* t = a.bucket;
  a.bucket = a.tmp;
  a.tmp = t;
}

// Range of bin q in the bucket (counted modes; slow bins never occur with
// fixed-capacity bins).
__device__ __forceinline__ void slow_range(const int32_t* __restrict__ binstart, int q,
                                           int& e0, int& e1) {
  e0 = binstart[q];
  e1 = binstart[q + 1];
}

template <typename VT, int CAP, int NT>
__global__ void __launch_bounds__(NT)
k_slow_count(ChunkArgs<VT> a, const int32_t* __restrict__ binstart,
             const uint32_t* __restrict__ bcol, int32_t* __restrict__ colptr_g,
             int32_t w, const int32_t* __restrict__ slowlist,
             uint32_t* __restrict__ slowD) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[Lds<CAP>::kBytes];
  ChunkCtx<VT, CAP, NT> x{smem};
  const int nslow = (int)a.ctrl->nslow;
  for (int i = blockIdx.x; i < nslow; i += gridDim.x) {
    const int q = slowlist[i];
    int e0, e1;
    slow_range(binstart, q, e0, e1);
    const int c0 = (int)min((int64_t)a.N, (int64_t)q * w);
    const int c1 = (int)min((int64_t)a.N, ((int64_t)q + 1) * w);
    ChunkArgs<VT> b = a;
    slow_sort<VT, CAP, NT>(b, bcol, colptr_g, x, c0, c1, e0, e1);
    const int64_t D = chunk_sweep<VT, CAP, NT>(b, x, c0, c1, false, 0);
    if (threadIdx.x == 0) slowD[q] = (uint32_t)D;
  }
}

template <typename VT, int CAP, int NT>
__global__ void __launch_bounds__(NT)
k_slow_emit(ChunkArgs<VT> a, const int32_t* __restrict__ binstart,
            int32_t* __restrict__ colptr_g, int32_t w,
            const int32_t* __restrict__ slowlist,
            const uint64_t* __restrict__ slowB) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[Lds<CAP>::kBytes];
  ChunkCtx<VT, CAP, NT> x{smem};
  const int nslow = (int)a.ctrl->nslow;
  for (int i = blockIdx.x; i < nslow; i += gridDim.x) {
    const int q = slowlist[i];
    int e0, e1;
    slow_range(binstart, q, e0, e1);
    const int c0 = (int)min((int64_t)a.N, (int64_t)q * w);
    const int c1 = (int)min((int64_t)a.N, ((int64_t)q + 1) * w);
    ChunkArgs<VT> b = a;
    b.colptr = colptr_g;  // the copy sorted by k_slow_count
    Entry<VT>* t = b.bucket;
    b.bucket = b.tmp;
    b.tmp = t;
    const uint64_t pre = slowB[q];
    b.pshift = (int64_t)(pre >> 31) - e0;
    chunk_sweep<VT, CAP, NT>(b, x, c0, c1, true, (int64_t)(pre & kLow31));
  }
}

// Persistent: every block takes bins in ticket order until none is left,
// fetching the next bin while the current one is processed.  A block waits
// in the look-back only for bins with smaller tickets.  Every started bin
// publishes its count before it waits, and the smallest ticket not yet
// published is always either being processed or the next bin of a block
// whose current bin has only published bins before it, so every wait ends.
// A block holds at most one ticket beyond the bin it processes.
// Waves per SIMD that the LDS lets the bin kernel have (160 KB per CU),
// asked of the register allocator when it still leaves 128 registers a lane
// (else no request): at 2048 entries and 512 threads two workgroups then
// share a CU.
template <int CAP, int NT>
constexpr int bin_waves() {
  constexpr int blocks = (160 * 1024) / BinLds<CAP>::kBytes;
  constexpr int w = blocks * (NT / 64) / 4;
  return w >= 1 && w <= 4 ? w : 1;
}

template <typename VT, int CAP, int NT, bool KEYS>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(bin_waves<CAP, NT>())))
k_bin(ChunkArgs<VT> a, BinSrc src, int32_t w) {
  constexpr int EPT = CAP / NT;
  __shared__ __attribute__((aligned(16))) unsigned char smem[BinLds<CAP>::kBytes];
  ChunkCtx<VT, CAP, NT> x{smem};
  int64_t* misc = reinterpret_cast<int64_t*>(smem + BinLds<CAP>::kMisc);
  const int N = a.N;
  const int B = src.B;
  if (threadIdx.x == 0) misc[0] = (int64_t)atomicAdd(src.tick, 1u);
  __syncthreads();
  BinRegs<VT, EPT, KEYS> cur, nx;
  cur.q = (int)misc[0];
  if (cur.q < B) {
    uint32_t fill;
    bin_bounds(src, cur, fill);
    bin_range(src, cur, fill);
    bin_load<VT, NT, EPT, KEYS>(a, src, cur);
  }
  while (cur.q < B) {
    const int q = cur.q;
#ifdef FSP_PHASE_TIMING
    if (a.phase && threadIdx.x == 0) a.phase[(int64_t)q * 16] = wall_clock64();
#endif
    const int c0 = (int)min((int64_t)N, (int64_t)q * w);
    const int c1 = (int)min((int64_t)N, ((int64_t)q + 1) * w);
    // ticket of the next bin; only thread 0 holds (and later reads) it, so
    // the value needs no merge with the other lanes and no early wait
    uint32_t tk;
    if (threadIdx.x == 0) tk = atomicAdd(src.tick, 1u);
    int64_t end = 0;
    if (cur.e1 - cur.e0 <= a.cap) {
      end = bin_fast<VT, CAP, NT, KEYS>(a, src, x, cur, c0, c1, tk, nx);
    } else {
      // a slow bin: counted before this kernel, emitted after it; here its
      // count only passes through the look-back
      const int span = cur.e1 - cur.e0;
      if (threadIdx.x < 64) {
        const uint32_t D = src.slowD[q];
        const int64_t b = lookback(a.status, q, pack_agg((uint64_t)span, D));
        if (threadIdx.x == 0) {
          src.slowB[q] = (uint64_t)b;
          misc[1] = (b & kLow31) + D;
          misc[5] = (b >> 31) + span;  // compact triplets up to this bin's end
        }
      }
      __syncthreads();
      end = misc[1];
      if (threadIdx.x == 0) misc[7] = (int64_t)tk;
      __syncthreads();
      nx.q = (int)misc[7];
      if (nx.q < B) {
        uint32_t fill;
        bin_bounds(src, nx, fill);
        bin_range(src, nx, fill);
        bin_load<VT, NT, EPT, KEYS>(a, src, nx);
      }
    }
    if (q == B - 1 && threadIdx.x == 0) {
      a.jcS[N] = (int32_t)end;
      a.ctrl->nnz = end;
      if (a.seg) a.seg[end] = (int32_t)misc[5];
      if (a.hostctrl) {
        // nnz and the error bits of the earlier kernels go straight to
        // host-visible memory (visible to the host once the call's stream
        // is synchronized); a capacity overflow shows as nnz > capacity
        const uint32_t err =
            __hip_atomic_load(&a.ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.hostctrl->err, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&a.hostctrl->nnz, end, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    __syncthreads();  // the LDS is reused by the next bin
    cur = nx;
  }
}

// ---------------------------------------------------------------------------
// batched: per-matrix column pointers from the global ones
// ---------------------------------------------------------------------------
__global__ void k_batched_jcs(const int32_t* __restrict__ jcg,
                              const int64_t* __restrict__ col_off, int32_t nb,
                              int64_t total, int32_t* __restrict__ jcS,
                              int64_t* __restrict__ nnz_off, int64_t* host_off) {
  {
    // the matrices' offsets, on the device and in the caller's pinned host
    // memory (system-scope stores, read once the stream is synchronized)
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t b = i0; b <= nb; b += (int64_t)gridDim.x * blockDim.x) {
      const int64_t v = jcg[col_off[b]];
      nnz_off[b] = v;
      if (host_off)
        __hip_atomic_store(&host_off[b], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  // each block takes one contiguous range of positions and its threads step
  // through it together (coalesced); matrix b owns positions
  // [col_off[b] + b, col_off[b+1] + b + 1); a thread's positions increase by
  // the block size, so after one search its matrix only moves forward
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t p1 = min(total, (int64_t)(blockIdx.x + 1) * per);
  const int64_t stride = blockDim.x;
  int64_t idx = (int64_t)blockIdx.x * per + threadIdx.x;
  if (idx >= p1) return;
  int lo = 0, hi = nb;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (col_off[mid] + mid <= idx) lo = mid; else hi = mid;
  }
  int64_t first = col_off[lo], start = first + lo, next = col_off[lo + 1] + lo + 1;
  int32_t jb = jcg[first];
  while (idx < p1) {
    while (idx >= next) {
      ++lo;
      first = col_off[lo];
      start = next;
      next = col_off[lo + 1] + lo + 1;
      jb = jcg[first];
    }
    if (idx + 3 * stride < min(p1, next)) {
      // four positions of one matrix: their loads in flight together
      const int32_t* src = jcg + first + (idx - start);
      const int32_t v0 = src[0], v1 = src[stride], v2 = src[2 * stride], v3 = src[3 * stride];
      jcS[idx] = v0 - jb;
      jcS[idx + stride] = v1 - jb;
      jcS[idx + 2 * stride] = v2 - jb;
      jcS[idx + 3 * stride] = v3 - jb;
      idx += 4 * stride;
    } else {
      jcS[idx] = jcg[first + (idx - start)] - jb;
      idx += stride;
    }
  }
}

// ---------------------------------------------------------------------------
// re-assembly, atomic accumulation, backward
// ---------------------------------------------------------------------------
// Re-use tiles: tile t owns the outputs j whose first sorted position
// seg[j] lies in [t*TP, (t+1)*TP); rtile[t] is the first of them.  seg is
// strictly increasing (every output has a contribution).
__global__ void k_reuse_tiles(const int32_t* __restrict__ seg,
                              const int64_t* __restrict__ nnz_dev, int32_t TP,
                              int64_t T, int32_t* __restrict__ rtile) {
  const int64_t nnz = *nnz_dev;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; j <= nnz; j += stride) {
    const int64_t lo = j == 0 ? 0 : (int64_t)seg[j - 1] / TP + 1;
    const int64_t hi = min((int64_t)seg[j] / TP, T);
    for (int64_t t = lo; t <= hi; ++t) rtile[t] = (int32_t)j;
    if (j == nnz)
      for (int64_t t = hi + 1; t <= T; ++t) rtile[t] = (int32_t)nnz;
  }
}

// Ordered re-assembly: the block gathers the values of its tile's
// contributions in sorted order into LDS (one independent gather per
// thread and position, perm read coalesced), then every output folds its
// run from +0.0 in increasing k, reading LDS.  Runs longer than the LDS
// stage fold straight from global memory.
template <typename VT, int TP, int NT>
__global__ void __launch_bounds__(NT)
k_reuse(const int32_t* __restrict__ perm, const int32_t* __restrict__ seg,
        const int32_t* __restrict__ rtile, const VT* __restrict__ ss,
        VT* __restrict__ prS) {
  constexpr int LCAP = 2 * TP;
  __shared__ VT val[LCAP];
  const int t = blockIdx.x;
  const int J0 = rtile[t], J1 = rtile[t + 1];
  if (J0 >= J1) return;
  const int P0 = seg[J0], P1 = seg[J1];
  if (P1 - P0 <= LCAP) {
    // four positions per thread at a time: their index loads, then their
    // gathers, all in flight together (clamped indices: no branch)
    for (int p0 = P0 + threadIdx.x; p0 < P1; p0 += 4 * NT) {
      int32_t pk[4];
      VT v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pk[u] = perm[min(p0 + u * NT, P1 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = ss[pk[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (p0 + u * NT < P1) val[p0 + u * NT - P0] = v[u];
    }
    __syncthreads();
    for (int j = J0 + threadIdx.x; j < J1; j += NT) {
      const int a = seg[j] - P0, b = seg[j + 1] - P0;
      VT acc = (VT)0;
      int q = a;
      for (; q + 4 <= b; q += 4) {
        const VT v0 = val[q], v1 = val[q + 1], v2 = val[q + 2], v3 = val[q + 3];
        acc = acc + v0;
        acc = acc + v1;
        acc = acc + v2;
        acc = acc + v3;
      }
      for (; q < b; ++q) acc = acc + val[q];
      prS[j] = acc;
    }
  } else {
    for (int j = J0 + threadIdx.x; j < J1; j += NT) {
      const int a = seg[j], b = seg[j + 1];
      VT acc = (VT)0;
      for (int q = a; q < b; ++q) acc = acc + ss[perm[q]];
      prS[j] = acc;
    }
  }
}

// The slot map from a plan's sorted order: every position p of output j's
// run seg[j]..seg[j+1] holds a triplet number perm[p] whose slot is j.
// (nnz is read on the device: the plan may not have read it back.)
__global__ void k_slot_from_order(const int32_t* __restrict__ perm,
                                  const int32_t* __restrict__ seg,
                                  const int64_t* __restrict__ nnz_dev,
                                  int32_t* __restrict__ slot) {
  const int64_t nnz = *nnz_dev;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; j < nnz; j += stride)
    for (int32_t p = seg[j]; p < seg[j + 1]; ++p) slot[perm[p]] = (int32_t)j;
}

template <typename VT>
__global__ void k_fill(VT* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = (VT)0;
}

// The same with the count in device memory (a call that has not read nnz
// back to the host), at most nmax entries.
template <typename VT>
__global__ void k_fill_dev(VT* __restrict__ p, const int64_t* __restrict__ ndev,
                           int64_t nmax) {
  const int64_t n = min(*ndev, nmax);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = (VT)0;
}

template <typename VT>
__global__ void k_atomic(const int32_t* __restrict__ slot,
                         const VT* __restrict__ ss, int64_t L,
                         VT* __restrict__ prS) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; k < L; k += stride) unsafeAtomicAdd(&prS[slot[k]], ss[k]);
}

// grad_ss[k] = grad_prS[slot[k]]; a triplet of a pair that is not stored
// (slot -1 after dropping zeros or false logical pairs) moves no stored
// value, so its gradient is 0.  Slots outside [0, nnz) read nothing.
template <typename VT>
__global__ void k_backward(const int32_t* __restrict__ slot,
                           const VT* __restrict__ g, int64_t L, int64_t nnz,
                           VT* __restrict__ gs) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; k < L; k += stride) {
    const int32_t s = slot[k];
    gs[k] = (s >= 0 && s < nnz) ? g[s] : (VT)0;
  }
}

// Wide integer indices narrowed to int32 for the passes: a value that is not
// in [1, 2^31 - 1] becomes 0, which every pass rejects as an index below 1
// (instead of wrapping into range).
template <typename IT>
__global__ void k_narrow_index(const IT* __restrict__ src, int64_t L,
                               int32_t* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; k < L; k += stride) {
    const IT v = src[k];
    dst[k] = (v >= (IT)1 && v <= (IT)2147483647) ? (int32_t)v : 0;
  }
}

// ---------------------------------------------------------------------------
// delayed assembly: an assembled matrix (jcA, irA, prA) as its own triplets,
// one per stored pair in storage order, ahead of the new triplets.  Column
// of entry e: the last c with jcA[c] <= e.  A block takes NT*EPT
// consecutive entries and finds the columns c0, c1 of its first and last
// entry by binary search over jcA[0..n]; when jcA[c0..c1+1] fits its LDS
// window (empty columns can make it long) every entry searches the window,
// otherwise jcA[c0..c1+1] in global memory.  Reads and writes coalesced.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t ccs_col(const int32_t* __restrict__ p,
                                           int64_t lo, int64_t hi, int64_t e) {
  while (hi - lo > 1) {  // p[lo] <= e < p[hi]
    const int64_t mid = (lo + hi) >> 1;
    if (p[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

template <typename VT, int NT, int EPT>
__global__ void __launch_bounds__(NT)
k_ccs_triplets(const int32_t* __restrict__ jcA, const int32_t* __restrict__ irA,
               const VT* __restrict__ prA, int64_t n, int64_t nnzA,
               int32_t* __restrict__ ii, int32_t* __restrict__ jj,
               VT* __restrict__ ss) {
  constexpr int TE = NT * EPT;
  constexpr int WSZ = TE + 2;
  __shared__ int32_t win[WSZ];
  __shared__ int64_t sC[2];
  const int64_t E0 = (int64_t)blockIdx.x * TE;
  if (E0 >= nnzA) return;  // the whole block
  const int64_t E1 = min(E0 + TE, nnzA) - 1;
  if (threadIdx.x == 0) sC[0] = ccs_col(jcA, 0, n, E0);
  if (threadIdx.x == NT - 1) sC[1] = ccs_col(jcA, 0, n, E1);
  __syncthreads();
  const int64_t c0 = sC[0], c1 = sC[1];
  const int64_t cnt = c1 - c0 + 2;  // jcA[c0 .. c1+1]; c1 + 1 <= n
  const bool inwin = cnt <= WSZ;
  if (inwin) {
    for (int t = threadIdx.x; t < cnt; t += NT) win[t] = jcA[c0 + t];
    __syncthreads();
  }
  for (int k = threadIdx.x; k < TE; k += NT) {
    const int64_t e = E0 + k;
    if (e > E1) break;
    const int64_t c = inwin ? c0 + ccs_col(win, 0, cnt - 1, e)
                            : ccs_col(jcA, c0, c1 + 1, e);
    ii[e] = irA[e] + 1;
    jj[e] = (int32_t)c + 1;
    ss[e] = prA[e];
  }
}

// ---------------------------------------------------------------------------
// delayed assembly by merge.  The stored matrix A (rows strictly increasing
// per column) and the new triplets, assembled on their own into B with the
// sorted order of their triplets kept (permB: triplet of each sorted
// position; segB: first sorted position of each of B's pairs), are merged
// column by column, one thread per column.  A pair of A alone keeps its
// stored sum (folded once from +0.0, as a stored pair is the first
// contribution of its pair); a pair of B alone keeps B's sum; a pair in both
// continues from the stored sum over B's contributions in increasing k.
// That is the fold of one assembly of A's pairs (as triplets, first) and the
// new triplets.
// ---------------------------------------------------------------------------
constexpr int kMergeRows = 2048;  // rows (and values) of A and of B one merge block stages

// B is assembled on its own column range: its column j is column j + boff
// of the result, j in [0, nB).
struct MergeCols {
  int32_t nA;    // A's columns (A is empty past them)
  int32_t boff;  // result column of B's first column
  int32_t nB;    // B's columns
};

__device__ __forceinline__ void merge_ranges(const int32_t* __restrict__ jcA,
                                             const int32_t* __restrict__ jcB,
                                             const MergeCols& mc, int64_t c, int32_t& a0,
                                             int32_t& a1, int32_t& b0, int32_t& b1) {
  a0 = jcA[min(c, (int64_t)mc.nA)];
  a1 = jcA[min(c + 1, (int64_t)mc.nA)];
  const int64_t cb = min(max(c - mc.boff, (int64_t)0), (int64_t)mc.nB);
  const int64_t cb1 = min(max(c + 1 - mc.boff, (int64_t)0), (int64_t)mc.nB);
  b0 = jcB[cb];
  b1 = jcB[cb1];
}

// Rows in r[x, x + len) (increasing) below `row`.
__device__ __forceinline__ int32_t lower_rank(const int32_t* r, int32_t x, int32_t len,
                                              int32_t row) {
  int32_t lo = 0, hi = len;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (r[x + mid] < row) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// A run of rows and values [t0, t1) (at most kMergeRows) into LDS, eight
// loads per thread in flight before their stores.
template <typename VT, int NT>
__device__ __forceinline__ void merge_stage(const int32_t* __restrict__ ir,
                                            const VT* __restrict__ pr, int32_t t0,
                                            int32_t t1, int32_t* rs, VT* vs) {
  constexpr int U = 8;
  for (int32_t b = t0 + (int32_t)threadIdx.x; b < t1; b += NT * U) {
    int32_t r[U];
    VT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t t = min(b + u * NT, t1 - 1);
      r[u] = ir[t];
      v[u] = pr[t];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t t = b + u * NT;
      if (t < t1) {
        rs[t - t0] = r[u];
        vs[t - t0] = v[u];
      }
    }
  }
}

// One block merges NT / G consecutive columns, G lanes (a power of two, 8 to
// 64, within one wave) per column, blocks in ticket order.  The block's
// runs of A and of B (contiguous in both) are loaded into LDS with
// coalesced loads.  In a column, a row's merged position is the number of
// distinct rows below it over A and B: for A's i-th row with p rows of B
// below it, i + p - (common rows among A's first i); for B's j-th row with
// q rows of A below it, j + q - (common rows among A's first q).  Binary
// searches give p and q, a ballot scan over A's rows the common prefix.  A
// row present in both is written by A's lane, which continues the stored
// sum over B's contributions in increasing k.  The block sums its columns'
// counts and chains its total to the earlier blocks by a look-back.  A block
// whose runs exceed kMergeRows writes nothing and flags kErrRuns (the host
// merges otherwise); a stored row outside [0, m) flags an index error.
template <typename VT, int NT>
__global__ void __launch_bounds__(NT)
k_merge(const int32_t* __restrict__ jcA, const int32_t* __restrict__ irA,
        const VT* __restrict__ prA, MergeCols mc, const int32_t* __restrict__ jcB,
        const int32_t* __restrict__ irB, const VT* __restrict__ prB,
        const int32_t* __restrict__ segB, const int32_t* __restrict__ permB,
        const VT* __restrict__ ss, int32_t n, int32_t m, int32_t* __restrict__ jcS,
        int32_t* __restrict__ irS, VT* __restrict__ prS, int32_t* __restrict__ slotA,
        int32_t* __restrict__ mapB, uint64_t* status, Ctrl* ctrl, int32_t G) {
  __shared__ int32_t rA[kMergeRows];
  __shared__ int32_t rB[kMergeRows];
  __shared__ uint32_t cA[kMergeRows];  // common rows among A's rows before
  __shared__ VT vA[kMergeRows];
  __shared__ VT vB[kMergeRows];
  __shared__ uint32_t sWave[NT / 64];
  __shared__ int sTile;
  __shared__ int64_t sBase;
  if (threadIdx.x == 0) sTile = (int)atomicAdd(&ctrl->tick_scan, 1u);
  __syncthreads();
  const int tile = sTile;
  const int cpb = NT / G;
  const int64_t cb = (int64_t)tile * cpb;
  const int64_t ce = min(cb + cpb, (int64_t)n);
  // the block's runs
  int32_t A0, A1, B0, B1, t0, t1;
  merge_ranges(jcA, jcB, mc, cb, A0, t0, B0, t1);
  merge_ranges(jcA, jcB, mc, ce - 1, t0, A1, t1, B1);
  const bool fits = A1 - A0 <= kMergeRows && B1 - B0 <= kMergeRows;
  if (fits) {
    merge_stage<VT, NT>(irA, prA, A0, A1, rA, vA);
    merge_stage<VT, NT>(irB, prB, B0, B1, rB, vB);
  } else if (threadIdx.x == 0) {
    atomicOr(&ctrl->err, kErrRuns);
  }
  __syncthreads();
  const int g = (int)threadIdx.x & (G - 1);
  const int64_t c = cb + (int64_t)threadIdx.x / G;
  const bool mine = fits && c < ce;
  int32_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
  uint32_t common = 0;
  if (mine) {
    merge_ranges(jcA, jcB, mc, c, a0, a1, b0, b1);
    const int32_t la = a1 - a0, lb = b1 - b0, xa = a0 - A0, xb = b0 - B0;
    // rows increase within a column: the first and last bound them all
    if (g == 0 && la > 0 && (rA[xa] < 0 || rA[xa + la - 1] >= m))
      atomicOr(&ctrl->err, kErrRow);
    // the column's lanes take A's rows G at a time (the same trip count in
    // every lane of the column)
    const int lane = lane_id();
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (lane & ~(G - 1));
    const uint64_t below = (1ull << lane) - 1ull;
    for (int32_t i0 = 0; i0 < la; i0 += G) {
      const int32_t i = i0 + g;
      bool com = false;
      if (i < la) {
        const int32_t ra = rA[xa + i];
        const int32_t p = lower_rank(rB, xb, lb, ra);
        com = p < lb && rB[xb + p] == ra;
      }
      const uint64_t bal = __ballot(com) & gmask;
      if (i < la) cA[xa + i] = common + (uint32_t)__popcll(bal & below);
      common += (uint32_t)__popcll(bal);
    }
  }
  const uint32_t cnt = mine ? (uint32_t)((a1 - a0) + (b1 - b0)) - common : 0u;
  uint32_t total;
  const uint32_t pre = block_excl_sum<NT>(g == 0 ? cnt : 0u, sWave, total);
  if (threadIdx.x < 64) {
    const int64_t ex = lookback(status, tile, total);
    if (threadIdx.x == 0) sBase = ex;
  }
  __syncthreads();
  if (!mine) return;
  // the column's first lane holds its offset; the others' prefix includes it
  const int64_t col0 = sBase + (g == 0 ? pre : pre - cnt);
  if (g == 0) {
    jcS[c] = (int32_t)col0;
    if (c == n - 1) jcS[n] = (int32_t)(col0 + cnt);
  }
  const int32_t la = a1 - a0, lb = b1 - b0, xa = a0 - A0, xb = b0 - B0;
  for (int32_t i = g; i < la; i += G) {
    const int32_t ra = rA[xa + i];
    const int32_t p = lower_rank(rB, xb, lb, ra);
    const int32_t o = (int32_t)(col0 + i + p - (int32_t)cA[xa + i]);
    VT v = (VT)0 + vA[xa + i];
    if (p < lb && rB[xb + p] == ra) {
      for (int32_t t = segB[b0 + p], e = segB[b0 + p + 1]; t < e; ++t) v = v + ss[permB[t]];
      if (mapB) mapB[b0 + p] = o;
    }
    irS[o] = ra;
    prS[o] = v;
    if (slotA) slotA[a0 + i] = o;
  }
  for (int32_t j = g; j < lb; j += G) {
    const int32_t rb = rB[xb + j];
    const int32_t q = lower_rank(rA, xa, la, rb);
    if (q < la && rA[xa + q] == rb) continue;  // written with A's row
    const int32_t o =
        (int32_t)(col0 + j + q - (int32_t)(q < la ? cA[xa + q] : common));
    irS[o] = rb;
    prS[o] = vB[xb + j];
    if (mapB) mapB[b0 + j] = o;
  }
}

// Column indices moved down by `off` (B's own column range).
__global__ void k_shift_index(const int32_t* __restrict__ jj, int64_t len, int32_t off,
                              int32_t* __restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = jj[k] - off;
}

// slot of new triplet k: the merged position of its pair in B.
__global__ void k_slot_gather(const int32_t* __restrict__ slotB, int64_t len,
                              const int32_t* __restrict__ mapB, int32_t* __restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = mapB[slotB[k]];
}

// Rows the stored pairs need (largest 0-based row + 1), into *out (which
// starts at 0).
__global__ void k_rowmax(const int32_t* __restrict__ irA, int64_t nnzA, int32_t* out) {
  int32_t mx = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnzA;
       t += (int64_t)gridDim.x * blockDim.x)
    mx = max(mx, irA[t] + 1);
  if (mx > 0) atomicMax(out, mx);
}

// ---------------------------------------------------------------------------
// drop zeros: remove the pairs whose sum is zero (+0 or -0; with imaginary
// parts, zero in both), as a Matlab sparse matrix stores no zeros.  One
// pass in ticket order.  Tile q holds IPT rows of NT consecutive pairs
// (row j = pairs [q*NT*IPT + j*NT, +NT), one per thread, so loads and
// stores are coalesced); wave ballots count the kept pairs per row, the
// look-back gives the tile's output offset, and the kept pairs are written
// in place.  A tile writes only at or below its own end, where earlier
// tiles or its own threads have already loaded: a tile publishes its count
// only after all its loads have returned (the count depends on every
// loaded word), and gets its offset only once every earlier tile has
// published.  excl[j] = kept pairs before j; excl[nnz] = the total.
// ---------------------------------------------------------------------------
template <typename VT, int NT, int IPT>
__global__ void __launch_bounds__(NT)
k_drop_pass(int32_t* __restrict__ irS, VT* __restrict__ prS, VT* __restrict__ piS,
            int32_t n, int32_t* __restrict__ excl, uint64_t* status, uint32_t* ticket) {
  constexpr int NW = NT / 64;
  __shared__ uint32_t sCnt[IPT][NW];
  __shared__ int sTile;
  __shared__ int64_t sBase;
  if (threadIdx.x == 0) sTile = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int tile = sTile;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)tile * NT * IPT + threadIdx.x;
  const uint64_t lt = (1ull << lane) - 1ull;
  int32_t r[IPT];
  VT pr[IPT], pi[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t i = t0 + (int64_t)j * NT;
    r[j] = 0;
    pr[j] = (VT)0;
    pi[j] = (VT)0;
    if (i < n) {
      r[j] = irS[i];
      pr[j] = prS[i];
      if (piS) pi[j] = piS[i];
    }
  }
  uint32_t keep = 0u, rk[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    // r[j] >= 0 always holds; testing it makes the count wait for the load
    const bool k = t0 + (int64_t)j * NT < n && r[j] >= 0 &&
                   (pr[j] != (VT)0 || pi[j] != (VT)0);
    const uint64_t m = __ballot(k);
    rk[j] = (uint32_t)__popcll(m & lt);
    if (lane == 0) sCnt[j][wid] = (uint32_t)__popcll(m);
    keep |= (k ? 1u : 0u) << j;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    uint32_t total = 0u;
#pragma unroll
    for (int j = 0; j < IPT; ++j)
#pragma unroll
      for (int w = 0; w < NW; ++w) total += sCnt[j][w];
    const int64_t ex = lookback(status, tile, total);
    if (threadIdx.x == 0) sBase = ex;
  }
  __syncthreads();
  int64_t run = sBase;  // kept pairs before the current row
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    uint32_t before = 0u, row = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t c = sCnt[j][w];
      before += w < wid ? c : 0u;
      row += c;
    }
    const int64_t i = t0 + (int64_t)j * NT;
    const int64_t pos = run + before + rk[j];
    if (i <= n) excl[i] = (int32_t)pos;
    if ((keep >> j) & 1u) {
      irS[pos] = r[j];
      prS[pos] = pr[j];
      if (piS) piS[pos] = pi[j];
    }
    run += row;
  }
}

// jcS[c] = kept pairs before the column's old start; slot[k] = the new place
// of its pair, or -1 when the pair was removed
__global__ void k_drop_renumber(const int32_t* __restrict__ excl,
                                int32_t* __restrict__ jcS, int64_t n,
                                int32_t* __restrict__ slot, int64_t L) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t c = t; c <= n; c += stride) jcS[c] = excl[jcS[c]];
  if (slot)
    for (int64_t k = t; k < L; k += stride) {
      const int32_t s = slot[k];
      slot[k] = excl[s + 1] > excl[s] ? excl[s] : -1;
    }
}

// logical values: 0/1 indicators (fp32) for the fold, whose sums are nonzero
// exactly where a triplet is true (a fold of ones from +0 never returns to
// zero, and saturates at 2^24 rather than wrap); the stored pairs are true
__global__ void k_logical_ind(const uint8_t* __restrict__ sl, int64_t L,
                              float* __restrict__ v) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; k < L; k += stride) v[k] = sl[k] ? 1.0f : 0.0f;
}

__global__ void k_fill_true(uint8_t* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 1u;
}


}  // namespace fsp
