// Host side of the C ABI declared in include/fsparse.h: argument checks,
// workspace layout, launches, the single readback of a fresh assembly,
// re-use plans (HIP graphs) and per-stage event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fsparse.h"
#include "kernels.h"

using fsp::BatchDesc;
using fsp::ChunkArgs;
using fsp::Ctrl;
using fsp::Entry;

#ifdef FSP_PHASE_TIMING
// profiling builds only: device buffer for per-bin phase timestamps
static uint64_t* g_phase = nullptr;
extern "C" void fsparse_phase_buffer(void* p) { g_phase = (uint64_t*)p; }
#endif

namespace {

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
// Defaults: the shapes the autotuner picks on MI355X for the mesh and
// random benchmark inputs (2048-entry bins with 512 threads, two bin
// workgroups per CU).
struct Tuning {
  int cap = 2048;
  int sblock = 256;
  int sitems = 8;
  int rblock = 512;
  int cblock = 512;  // threads of one bin workgroup
  int bmode = 0;     // 0 automatic, else 1 + BinMode to force one
  int keys = 1;      // fixed-capacity bins hold (row, k) only; values read by k
};
std::mutex g_mu;
Tuning g_tune;

Tuning tuning() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tune;
}

int kernel_cap(int cap) { return cap <= 1024 ? 1024 : (cap <= 2048 ? 2048 : 4096); }

// ---------------------------------------------------------------------------
// stage timing
// ---------------------------------------------------------------------------
enum Stage {
  kDims, kInit, kHist, kScan, kBucket, kChunk, kBatchedJcs, kAtomic,
  kReuse, kBackward, kCopy, kFill, kColScan, kDrop, kAppend, kNumStages
};
const char* kStageNames[kNumStages] = {
    "dims", "init", "count", "binscan", "scatter", "bin", "batched_jcs",
    "atomic", "reuse", "backward", "copy", "fill", "colscan", "drop_zeros", "append"};

struct Rec {
  int stage;
  hipEvent_t a, b;
};
bool g_timing = false;
uint32_t g_stage_mask = 0xFFFFFFFFu;  // stages bracketed while timing
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;  // recycled timing events
double g_ms[kNumStages];
int64_t g_cnt[kNumStages];

template <typename F>
hipError_t launch_raw(int stage, hipStream_t s, F&& f);

// The last HIP failure behind an FSPARSE_E_HIP on this host thread.
thread_local char t_last_error[160] = "";

void note_error(const char* where, hipError_t e) {
  snprintf(t_last_error, sizeof(t_last_error), "%s: %s (%d)", where, hipGetErrorName(e),
           (int)e);
}

template <typename F>
hipError_t launch(int stage, hipStream_t s, F&& f) {
  const hipError_t e = launch_raw(stage, s, f);
  if (e != hipSuccess)
    note_error(stage >= 0 && stage < kNumStages ? kStageNames[stage] : "launch", e);
  return e;
}

// Set while fsparse_assemble_noalloc runs on this thread: its launches
// carry no timing events (creating one would allocate).
thread_local bool t_noalloc = false;

template <typename F>
hipError_t launch_raw(int stage, hipStream_t s, F&& f) {
  bool timing;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    timing = g_timing && !t_noalloc && stage >= 0 && stage < 32 &&
             ((g_stage_mask >> stage) & 1u);
  }
  if (!timing) {
    f();
    return hipGetLastError();
  }
  Rec r{stage, nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_pool.size() >= 2) {
      r.a = g_pool.back();
      g_pool.pop_back();
      r.b = g_pool.back();
      g_pool.pop_back();
    }
  }
  // timing only: no system-scope fence at the events, so that recording
  // them writes back and invalidates no caches between the timed launches
  if (!r.a && (hipEventCreateWithFlags(&r.a, hipEventDisableSystemFence) != hipSuccess ||
               hipEventCreateWithFlags(&r.b, hipEventDisableSystemFence) != hipSuccess))
    return hipErrorOutOfMemory;
  hipEventRecord(r.a, s);
  f();
  hipError_t e = hipGetLastError();
  hipEventRecord(r.b, s);
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back(r);
  return e;
}

// ---------------------------------------------------------------------------
// device properties
// ---------------------------------------------------------------------------
// Per-device values are looked up once (device ids below kMaxDev).
constexpr int kMaxDev = 64;

int cur_device() {
  int dev = 0;
  hipGetDevice(&dev);
  return (dev >= 0 && dev < kMaxDev) ? dev : 0;
}

int num_cus() {
  static std::atomic<int> cache[kMaxDev];
  const int dev = cur_device();
  int cus = cache[dev].load(std::memory_order_relaxed);
  if (cus > 0) return cus;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess ||
      cus <= 0)
    cus = 256;
  cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

// Blocks of `kernel` that fit the device at once (persistent launches).
// The larger of the runtime's occupancy figure and one computed from the
// kernel's own LDS and register use (64 KB of VGPRs per SIMD lane group: 512
// per lane, at most 8 waves per SIMD, 4 SIMDs per CU).  More blocks than
// fit is harmless for the ticket-driven kernels (late blocks find no work),
// fewer would leave CUs idle.
// The kernel is a template argument, so each instantiation (each bin
// capacity and block size) keeps its own cached figure; kernels of one
// function type must not share it.
template <auto kernel>
int64_t resident(int block) {
  // one cache per kernel (each is launched with one block size)
  static std::atomic<int> cache[kMaxDev];
  const int dev = cur_device();
  int per = cache[dev].load(std::memory_order_relaxed);
  if (per <= 0) {
    int api = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&api, kernel, block, 0) !=
        hipSuccess)
      api = 0;
    int own = 0;
    hipFuncAttributes fa{};
    int lds_cu = 0;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) == hipSuccess &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              dev) == hipSuccess &&
        lds_cu > 0) {
      const int by_lds = fa.sharedSizeBytes > 0 ? lds_cu / (int)fa.sharedSizeBytes : 32;
      const int regs = std::max(8, (fa.numRegs + 7) / 8 * 8);
      const int wpsimd = std::min(8, 512 / regs);
      const int wblk = (block + 63) / 64;
      const int by_waves = (4 * wpsimd) / std::max(1, wblk);
      own = std::min(by_lds, by_waves);
    }
    // a failed query above falls back to the other figure; its error must
    // not be taken for the failure of the next launch
    (void)hipGetLastError();
    per = std::max(1, std::max(api, own));
    cache[dev].store(per, std::memory_order_relaxed);
  }
  return (int64_t)per * num_cus();
}

int grid_for(int64_t n, int block, int per_cu = 8) {
  int64_t g = (n + block - 1) / block;
  const int64_t cap = (int64_t)num_cus() * per_cu;
  if (g > cap) g = cap;
  return (int)std::max<int64_t>(1, g);
}

// pinned readback buffer, one per host thread
struct Pinned {
  void* p = nullptr;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local Pinned t_pinned;
constexpr size_t kPinnedBytes = 1 << 16;
void* pinned() {
  if (!t_pinned.p) {
    if (hipHostMalloc(&t_pinned.p, kPinnedBytes, hipHostMallocDefault) != hipSuccess)
      t_pinned.p = nullptr;
  }
  return t_pinned.p;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
constexpr int kScanNT = 256;
constexpr int kScanIPT = 16;
constexpr int64_t kScanTile = (int64_t)kScanNT * kScanIPT;
constexpr int64_t kDenseBins = 16384;       // LDS counters of the dense mode
constexpr int kBinFill = 80;                // percent of the capacity per bin
constexpr int64_t kDenseMatrix = 8 << 20;   // tiles x bins counters
// claim tiles: 256 threads with 8 triplets each (2048 per tile).  Measured
// on the fixed-capacity scatter of batched_64 (ms): 256x8 0.52, 512x8 0.56,
// 256x16 0.64, 128x16 0.59, 1024x8 0.66, 512x16 0.73, 64x16 0.80.
constexpr int kClaimNT = 256;
constexpr int kClaimIPT = 8;
constexpr int kClaimWindow = 4096;          // LDS bins of one claim tile
constexpr int kReuseTP = 2048;              // sorted positions per re-use tile

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Column bins: w columns per bin (2^s >= w), sized so that an average bin
// fills kBinFill percent of the bin kernel's LDS capacity.
enum BinMode { kDense = 0, kSlot = 1, kClaim = 2 };

struct Geom {
  int s;
  int64_t w, B, TS, T;
  uint32_t mul;     // bin of g = (g * mul) >> sh  (exact for g < 2^31)
  int sh;
  bool dense;
  int mode;         // BinMode
  int64_t slotcap;  // fixed bin capacity of the slot mode
  int64_t nslot;    // bucket places of the slot mode
};

// Bin width for an average fill of `fill` percent of the capacity, and the
// multiply-shift that divides by it.
// x / w for x < 2^31 as a multiply-high and a shift (the device's bin_of)
void set_divisor(Geom& g, int64_t w) {
  g.w = w;
  g.s = 0;
  while ((int64_t(1) << g.s) < w) ++g.s;
  if ((int64_t(1) << g.s) == w) {
    g.mul = 1u;
    g.sh = g.s;
  } else {
    g.sh = 31 + g.s;
    g.mul = (uint32_t)(((uint64_t(1) << g.sh) + (uint64_t)w - 1) / (uint64_t)w);
  }
}

// Fill (percent) of fixed-capacity bins: the mean m of a bin whose count of
// randomly placed triplets (about Poisson, standard deviation sqrt(m)) stays
// kSlotSigmas deviations below the capacity, m + kSlotSigmas*sqrt(m) = cap.
constexpr double kSlotSigmas = 5.8;
double slot_fill(int cap) {
  const double r = 0.5 * (-kSlotSigmas + std::sqrt(kSlotSigmas * kSlotSigmas + 4.0 * cap));
  return 100.0 * r * r / cap;
}

void set_width(Geom& g, int64_t L, int64_t N, int cap, double fill) {
  int64_t w = 1;
  if (L > 0) {
    const double target =
        std::max(1.0, (double)cap * fill / 100.0) * (double)N / (double)L;
    w = (int64_t)std::min<double>(target, (double)cap);
    w = std::max<int64_t>(1, w);
  }
  set_divisor(g, w);
  g.B = std::max<int64_t>(1, (N + w - 1) / w);
}

// `refit`: the geometry after fixed-capacity places overflowed.  That points
// to columns of uneven density, so the counted placement then uses bins of
// half the average fill, which keeps more of the dense bins within the LDS.
Geom make_geom(int64_t L, int64_t N, int cap, int force_mode, int blk,
               bool refit = false) {
  Geom g{};
  // an average bin fills kBinFill percent of the LDS capacity: a bin's cost
  // is mostly latency, so fuller bins mean fewer of them; a bin that still
  // overflows takes the slow path
  set_width(g, L, N, cap, refit ? kBinFill / 2 : kBinFill);
  if (refit) force_mode = 1 + kClaim;
  // few bins: a tiles x bins count matrix gives the tile offsets (dense);
  // many bins: every bin gets a fixed place of `cap` triplets so one pass
  // (claims per tile and bin) places the triplets, and an overflowing bin
  // makes the call fall back to counting first (kClaim)
  const bool fits_dense = g.B <= kDenseBins;
  const bool fits_slot = g.B * (int64_t)cap < (int64_t(1) << 31);
  g.mode = fits_dense ? kDense : (fits_slot ? kSlot : kClaim);
  if (force_mode == 1 + kDense && fits_dense) g.mode = kDense;
  if (force_mode == 1 + kSlot && fits_slot) g.mode = kSlot;
  if (force_mode == 1 + kClaim) g.mode = kClaim;
  // fixed places: fuller bins still (slot_fill: a place overflows only far
  // out in the tail of a bin's size)
  if (g.mode == kSlot) set_width(g, L, N, cap, slot_fill(cap));
  g.dense = g.mode == kDense;
  if (g.dense) {
    // tiles x bins count matrix: at most kDenseMatrix words, and while at
    // least 512 tiles remain, at most L/4 words (its passes then move about
    // a byte per triplet)
    g.TS = 4096;
    for (;;) {
      const int64_t T = (L + g.TS - 1) / g.TS;
      const bool big = T * g.B > kDenseMatrix;
      const bool heavy = T * g.B > L / 4 && T / 2 >= 512;
      if (!(big || heavy) || g.TS >= (1 << 22)) break;
      g.TS *= 2;
    }
    // between R and 2R tiles (R: the blocks of the dense passes that fit on
    // the chip at once, about 16 waves per CU), R larger tiles leave no
    // part-empty second round
    const int64_t R = (int64_t)num_cus() * std::max(1, 1024 / std::max(64, blk));
    const int64_t T = (L + g.TS - 1) / g.TS;
    if (T > R && T < 2 * R) g.TS = (L + R - 1) / R;
  } else {
    g.TS = (int64_t)kClaimNT * kClaimIPT;  // the claim kernels' tile
  }
  g.T = std::max<int64_t>(1, (L + g.TS - 1) / g.TS);
  g.slotcap = cap;
  g.nslot = g.mode == kSlot ? g.B * (int64_t)cap : 0;
  return g;
}

struct Layout {
  Geom g;
  int64_t mmax;  // largest m over the matrices (batched)
  size_t ctrl, scan_st, bin_st, bincnt, binfill, bmax, zero_end;
  size_t binstart, cntmat, tilebad, bcol, colptr, bucket, tmp, perm, seg, islot, rtile;
  size_t slowlist, slowd, slowb, dropst;
  size_t b_trip, b_col, b_m, b_n, jcg, nnzoff;
  size_t total;
  int64_t nscan;
};

Layout make_layout(int64_t L, int64_t N, int nb, int esize, const Tuning& tu,
                   bool refit = false) {
  Layout o{};
  o.g = make_geom(L, N, tu.cap, tu.bmode, tu.sblock, refit);
  const int64_t B = o.g.B;
  // look-back words: scan tiles of the bin scan, or 64-bin groups of the
  // dense column scan
  o.nscan = std::max<int64_t>((B + 1 + kScanTile - 1) / kScanTile, (B + 63) / 64);
  size_t p = 0;
  o.ctrl = p;        p = al(p + sizeof(Ctrl));
  o.scan_st = p;     p = al(p + 8 * (size_t)o.nscan);
  o.bin_st = p;      p = al(p + 8 * (size_t)B);
  o.bincnt = p;      p = al(p + 4 * (size_t)B);
  o.binfill = p;     p = al(p + 4 * (size_t)B);
  o.bmax = p;        p = al(p + 8 * (size_t)nb);
  o.zero_end = p;
  o.binstart = p;    p = al(p + 4 * (size_t)(B + 1));
  o.cntmat = p;      p = al(p + (o.g.dense ? 4 * (size_t)o.g.T * B : 0));
  o.tilebad = p;     p = al(p + (o.g.dense ? 4 * (size_t)o.g.T : 0));
  const int64_t nb_places = std::max(L, o.g.nslot);
  // spare places past the end of the bucket (and of bcol) for the stores of
  // unplaced triplets: one for the dense scatter, kSpare (one per lane of a
  // wave) for the claim scatter, where a full fixed-capacity bin can send
  // many triplets there
  o.bcol = p;        p = al(p + 4 * (size_t)(nb_places + fsp::kSpare));
  o.colptr = p;      p = al(p + 4 * (size_t)(N + 1));
  o.bucket = p;      p = al(p + (size_t)esize * (nb_places + fsp::kSpare));
  o.tmp = p;         p = al(p + (size_t)esize * L);
  o.perm = p;        p = al(p + 4 * (size_t)L);
  o.seg = p;         p = al(p + 4 * (size_t)(L + 1));
  o.islot = p;       p = al(p + 4 * (size_t)L);
  o.rtile = p;       p = al(p + 4 * (size_t)(L / kReuseTP + 3));
  o.slowlist = p;    p = al(p + 4 * (size_t)B);
  o.slowd = p;       p = al(p + 4 * (size_t)B);
  o.slowb = p;       p = al(p + 8 * (size_t)B);
  // drop zeros: look-back words of the scan over the pairs, and its ticket
  o.dropst = p;      p = al(p + 64 + 8 * (size_t)((L + 1 + kScanTile - 1) / kScanTile));
  o.b_trip = p;      p = al(p + 8 * (size_t)(nb + 1));
  o.b_col = p;       p = al(p + 8 * (size_t)(nb + 1));
  o.b_m = p;         p = al(p + 4 * (size_t)nb);
  o.b_n = p;         p = al(p + 4 * (size_t)nb);
  o.nnzoff = p;      p = al(p + 8 * (size_t)(nb + 1));
  o.jcg = p;         p = al(p + (nb > 1 ? 4 * (size_t)(N + 1) : 0));
  o.total = p;
  return o;
}

int esize_of(fsparse_dtype dt) { return dt == FSPARSE_F64 ? 16 : 12; }

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

#define HIPCHK(x)                              \
  do {                                         \
    const hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) {                    \
      note_error(#x, e_);                      \
      return FSPARSE_E_HIP;                    \
    }                                          \
  } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct fsparse_plan {
  int64_t len = 0, nnz = 0;       // nnz < 0: not read back yet (see dnnz)
  const int64_t* dnnz = nullptr;  // nnz in device memory (the control block)
  fsparse_dtype dt = FSPARSE_F64;
  int device = 0;
  hipEvent_t done = nullptr;      // recorded after every graph launch
  const int32_t* perm = nullptr;
  const int32_t* seg = nullptr;
  const int32_t* slot = nullptr;
  int32_t* islot = nullptr;        // where a missing slot map is derived
  const int32_t* rtile = nullptr;  // first output of every re-use tile
  int64_t ntiles = 0;
  int rblock = 256;
  // ordered re-use graph: one kernel node
  hipGraph_t g_ord = nullptr;
  hipGraphExec_t x_ord = nullptr;
  hipGraphNode_t n_ord = nullptr;
  const void* ss_ord = nullptr;
  void* pr_ord = nullptr;
  // atomic re-use graph: fill node -> atomic node
  hipGraph_t g_at = nullptr;
  hipGraphExec_t x_at = nullptr;
  hipGraphNode_t n_fill = nullptr, n_at = nullptr;
  const void* ss_at = nullptr;
  void* pr_at = nullptr;
};

namespace {

template <typename VT>
void* reuse_fn(int nt) {
  if (nt <= 256) return reinterpret_cast<void*>(&fsp::k_reuse<VT, kReuseTP, 256>);
  if (nt <= 512) return reinterpret_cast<void*>(&fsp::k_reuse<VT, kReuseTP, 512>);
  return reinterpret_cast<void*>(&fsp::k_reuse<VT, kReuseTP, 1024>);
}
template <typename VT>
void* fill_fn() {
  return reinterpret_cast<void*>(&fsp::k_fill_dev<VT>);
}
template <typename VT>
void* atomic_fn() {
  return reinterpret_cast<void*>(&fsp::k_atomic<VT>);
}

// Records the plan's completion event after its latest launch, so that
// destroying the plan can wait for launches still queued.
fsparse_status plan_mark(fsparse_plan* pl, hipStream_t stream) {
  if (!pl->done && hipEventCreateWithFlags(&pl->done, hipEventDisableTiming) != hipSuccess) {
    pl->done = nullptr;
    return FSPARSE_E_HIP;
  }
  return hipEventRecord(pl->done, stream) == hipSuccess ? FSPARSE_OK : FSPARSE_E_HIP;
}

fsparse_status plan_reuse_ordered(fsparse_plan* pl, const void* ss, void* prS,
                                  hipStream_t stream) {
  const int blk = pl->rblock <= 256 ? 256 : (pl->rblock <= 512 ? 512 : 1024);
  const int32_t* perm = pl->perm;
  const int32_t* seg = pl->seg;
  const int32_t* rtile = pl->rtile;
  void* args[] = {(void*)&perm, (void*)&seg, (void*)&rtile, (void*)&ss, (void*)&prS};
  hipKernelNodeParams kp{};
  kp.func = pl->dt == FSPARSE_F64 ? reuse_fn<double>(blk) : reuse_fn<float>(blk);
  kp.gridDim = dim3((unsigned)pl->ntiles);
  kp.blockDim = dim3(blk);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  if (!pl->x_ord) {
    HIPCHK(hipGraphCreate(&pl->g_ord, 0));
    HIPCHK(hipGraphAddKernelNode(&pl->n_ord, pl->g_ord, nullptr, 0, &kp));
    HIPCHK(hipGraphInstantiate(&pl->x_ord, pl->g_ord, nullptr, nullptr, 0));
    pl->ss_ord = ss;
    pl->pr_ord = prS;
  } else if (pl->ss_ord != ss || pl->pr_ord != prS) {
    HIPCHK(hipGraphExecKernelNodeSetParams(pl->x_ord, pl->n_ord, &kp));
    pl->ss_ord = ss;
    pl->pr_ord = prS;
  }
  hipError_t e = launch(kReuse, stream, [&] { (void)hipGraphLaunch(pl->x_ord, stream); });
  if (e != hipSuccess) return FSPARSE_E_HIP;
  return plan_mark(pl, stream);
}

fsparse_status plan_reuse_atomic(fsparse_plan* pl, const void* ss, void* prS,
                                 hipStream_t stream) {
  const int blk = pl->rblock;
  const int gf = grid_for(pl->nnz >= 0 ? pl->nnz : pl->len, blk, 8);
  const int ga = grid_for(pl->len, blk, 16);
  const int32_t* slot = pl->slot;
  const int64_t* dnnz = pl->dnnz;
  int64_t len = pl->len;
  void* fargs[] = {(void*)&prS, (void*)&dnnz, (void*)&len};
  void* aargs[] = {(void*)&slot, (void*)&ss, (void*)&len, (void*)&prS};
  hipKernelNodeParams fp{}, ap{};
  fp.func = pl->dt == FSPARSE_F64 ? fill_fn<double>() : fill_fn<float>();
  fp.gridDim = dim3(gf);
  fp.blockDim = dim3(blk);
  fp.kernelParams = fargs;
  ap.func = pl->dt == FSPARSE_F64 ? atomic_fn<double>() : atomic_fn<float>();
  ap.gridDim = dim3(ga);
  ap.blockDim = dim3(blk);
  ap.kernelParams = aargs;
  if (!pl->x_at) {
    HIPCHK(hipGraphCreate(&pl->g_at, 0));
    HIPCHK(hipGraphAddKernelNode(&pl->n_fill, pl->g_at, nullptr, 0, &fp));
    HIPCHK(hipGraphAddKernelNode(&pl->n_at, pl->g_at, &pl->n_fill, 1, &ap));
    HIPCHK(hipGraphInstantiate(&pl->x_at, pl->g_at, nullptr, nullptr, 0));
    pl->ss_at = ss;
    pl->pr_at = prS;
  } else if (pl->ss_at != ss || pl->pr_at != prS) {
    HIPCHK(hipGraphExecKernelNodeSetParams(pl->x_at, pl->n_fill, &fp));
    HIPCHK(hipGraphExecKernelNodeSetParams(pl->x_at, pl->n_at, &ap));
    pl->ss_at = ss;
    pl->pr_at = prS;
  }
  hipError_t e = launch(kReuse, stream, [&] { (void)hipGraphLaunch(pl->x_at, stream); });
  if (e != hipSuccess) return FSPARSE_E_HIP;
  return plan_mark(pl, stream);
}

// Removes the zero sums from the nnz pairs in place (irS, prS, jcS, and
// slot when given; with piS, complex sums zero in both parts, and piS is
// compacted too); the kept count lands in h->kept once the stream is done.
template <typename VT>
hipError_t drop_zeros(void* ws, const Layout& lo, int64_t nnz, int64_t n, int64_t L,
                      int32_t* jcS, int32_t* irS, VT* prS, int32_t* slot,
                      Ctrl* h, hipStream_t stream, VT* piS = nullptr) {
  int32_t* excl = at<int32_t>(ws, lo.seg);             // nnz + 1 words
  uint32_t* ticket = at<uint32_t>(ws, lo.dropst);
  uint64_t* status = at<uint64_t>(ws, lo.dropst + 64);
  const int64_t tiles = (nnz + 1 + kScanTile - 1) / kScanTile;
  const int64_t zw = (64 + 8 * tiles) / 4;
  hipError_t e = launch(kDrop, stream, [&] {
    hipLaunchKernelGGL(fsp::k_zero, dim3(grid_for(zw, 256, 4)), dim3(256), 0, stream,
                       ticket, zw);
    hipLaunchKernelGGL((fsp::k_drop_pass<VT, kScanNT, kScanIPT>), dim3((unsigned)tiles),
                       dim3(kScanNT), 0, stream, irS, prS, piS, (int32_t)nnz, excl,
                       status, ticket);
    hipLaunchKernelGGL(fsp::k_drop_renumber,
                       dim3(grid_for(std::max<int64_t>(n + 1, slot ? L : 0), 256, 4)),
                       dim3(256), 0, stream, (const int32_t*)excl, jcS, n, slot, L);
  });
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(&h->kept, excl + nnz, sizeof(int32_t), hipMemcpyDeviceToHost,
                        stream);
}

// nnz < 0: the count is only in device memory (dnnz), at most L
template <typename VT>
hipError_t launch_atomic_values(const int32_t* slot, const void* ss, int64_t L,
                                void* prS, int64_t nnz, int blk,
                                hipStream_t stream,
                                const int64_t* dnnz = nullptr) {
  hipError_t e = launch(kFill, stream, [&] {
    if (nnz >= 0)
      hipLaunchKernelGGL(fsp::k_fill<VT>, dim3(grid_for(nnz, blk)), dim3(blk), 0,
                         stream, (VT*)prS, nnz);
    else
      hipLaunchKernelGGL(fsp::k_fill_dev<VT>, dim3(grid_for(L, blk)), dim3(blk), 0,
                         stream, (VT*)prS, dnnz, L);
  });
  if (e != hipSuccess) return e;
  return launch(kAtomic, stream, [&] {
    hipLaunchKernelGGL(fsp::k_atomic<VT>, dim3(grid_for(L, blk, 16)), dim3(blk),
                       0, stream, slot, (const VT*)ss, L, (VT*)prS);
  });
}

// The shared pipeline of fresh and batched assembly.
// SRC: where triplet e's indices come from (int32 arrays, the expansion map
// `ex`, or double arrays).
template <typename VT, bool BATCHED, int SRC = fsp::kIdxI32>
hipError_t run_pipeline(const int32_t* ii, const int32_t* jj, const VT* ss,
                        int64_t L, int32_t m, int32_t n, BatchDesc bd,
                        int64_t N, const Layout& lo, const Tuning& tu,
                        void* ws, int32_t* jcS_target, int32_t* irS, VT* prS,
                        int64_t cap, int32_t* slot, bool keep_plan,
                        int mode, hipStream_t stream, Ctrl* hostctrl = nullptr,
                        fsp::Expand ex = fsp::Expand{}) {
  const Geom& g = lo.g;
  Ctrl* ctrl = at<Ctrl>(ws, lo.ctrl);
  hipError_t e;
  const int64_t zwords = (int64_t)(lo.zero_end / 4);
  // the dense count pass clears the control block and look-back words
  // itself; the other modes need them cleared first
  if (mode != kDense) {
    e = launch(kInit, stream, [&] {
      hipLaunchKernelGGL(fsp::k_zero, dim3(grid_for(zwords, 256, 4)), dim3(256), 0,
                         stream, at<uint32_t>(ws, 0), zwords);
    });
    if (e != hipSuccess) return e;
  }
  uint32_t* bincnt = at<uint32_t>(ws, lo.bincnt);
  uint32_t* binfill = at<uint32_t>(ws, lo.binfill);
  int32_t* binstart = at<int32_t>(ws, lo.binstart);
  uint32_t* cntmat = at<uint32_t>(ws, lo.cntmat);
  uint32_t* bcol = at<uint32_t>(ws, lo.bcol);
  Entry<VT>* bucket = at<Entry<VT>>(ws, lo.bucket);
  const int s = g.s, B = (int)g.B, w = (int)g.w;
  const fsp::BinGeo G{g.mul, g.sh, w, s};
  const int blk = tu.sblock;
  // rows and in-bin columns share one word when (m << s) fits 32 bits with
  // the all-ones word to spare (the bin kernel's empty hash slot)
  int64_t mmax = m;
  if (BATCHED) mmax = lo.mmax;
  const int packed = (mmax < (int64_t(1) << (32 - s))) ? 1 : 0;
  const int32_t slotcap = mode == kSlot ? (int32_t)g.slotcap : 0;
  // fixed-capacity bins may hold (row, k) alone: the bin kernel then reads
  // the values by k (not with the expansion map, whose values are indexed
  // by grid point)
  const bool keys = mode == kSlot && tu.keys && SRC != fsp::kIdxExpand;
  // 1. bin counts (the slot mode has none)
  if (mode != kSlot) e = launch(kHist, stream, [&] {
    if (mode == kDense)
      hipLaunchKernelGGL((fsp::k_count_dense<BATCHED, SRC>), dim3((unsigned)(8 * ((g.T + 7) / 8))), dim3(blk),
                         (size_t)B * 4, stream, jj, L, n, bd, G, B, (int32_t)g.TS,
                         cntmat, at<uint32_t>(ws, 0), zwords,
                         at<uint32_t>(ws, lo.tilebad), ex);
    else
      hipLaunchKernelGGL((fsp::k_count_claim<BATCHED, SRC, kClaimNT, kClaimIPT>),
                         dim3((unsigned)g.T), dim3(kClaimNT),
                         (size_t)kClaimWindow * 4, stream, jj, L, n, bd, G,
                         kClaimWindow, bincnt, ctrl, ex);
  });
  if (e != hipSuccess) return e;
  // 2. bin pointers (dense mode: with the column scan of the count matrix)
  if (mode == kDense) {
    e = launch(kColScan, stream, [&] {
      hipLaunchKernelGGL(fsp::k_colscan_bins<1024>, dim3((unsigned)((B + 63) / 64)),
                         dim3(1024), 0, stream, cntmat, (int32_t)g.T, B, binstart,
                         at<uint64_t>(ws, lo.scan_st), &ctrl->tick_scan,
                         (uint32_t)tu.cap, &ctrl->nslow, at<int32_t>(ws, lo.slowlist),
                         at<uint32_t>(ws, lo.tilebad), ctrl);
    });
  } else if (mode != kSlot) {
    e = launch(kScan, stream, [&] {
      hipLaunchKernelGGL((fsp::k_scan_excl<kScanNT, kScanIPT>),
                         dim3((unsigned)((B + 1 + kScanTile - 1) / kScanTile)),
                         dim3(kScanNT), 0, stream, bincnt, B, binstart,
                         at<uint64_t>(ws, lo.scan_st), &ctrl->tick_scan,
                         (uint32_t)tu.cap, &ctrl->nslow, at<int32_t>(ws, lo.slowlist));
    });
  }
  if (e != hipSuccess) return e;
  // 3. scatter into the bins
  e = launch(kBucket, stream, [&] {
    if (mode == kDense) {
      if (packed)
        hipLaunchKernelGGL((fsp::k_scatter_dense<VT, BATCHED, true, SRC>), dim3((unsigned)(8 * ((g.T + 7) / 8))),
                           dim3(blk), (size_t)B * 4, stream, ii, jj, ss, L, m, n, bd,
                           G, B, (int32_t)g.TS, cntmat, binstart, bucket, bcol,
                           (uint32_t)std::max<int64_t>(L, g.nslot), ctrl, ex);
      else
        hipLaunchKernelGGL((fsp::k_scatter_dense<VT, BATCHED, false, SRC>), dim3((unsigned)(8 * ((g.T + 7) / 8))),
                           dim3(blk), (size_t)B * 4, stream, ii, jj, ss, L, m, n, bd,
                           G, B, (int32_t)g.TS, cntmat, binstart, bucket, bcol,
                           (uint32_t)std::max<int64_t>(L, g.nslot), ctrl, ex);
    } else {
      const uint32_t trash = (uint32_t)std::max<int64_t>(L, g.nslot);
#define FSP_CLAIM(P, K)                                                        \
  hipLaunchKernelGGL((fsp::k_scatter_claim<VT, BATCHED, P, SRC, kClaimNT, kClaimIPT, K>), \
                     dim3((unsigned)g.T), dim3(kClaimNT), (size_t)kClaimWindow * 4, \
                     stream, ii, jj, ss, L, m, n, bd, G, kClaimWindow, binstart,  \
                     slotcap, binfill, bucket, bcol, trash, ctrl, ex)
      if constexpr (SRC != fsp::kIdxExpand) {
        if (keys) {
          if (packed) FSP_CLAIM(true, true); else FSP_CLAIM(false, true);
          return;
        }
      }
      if (packed) FSP_CLAIM(true, false); else FSP_CLAIM(false, false);
#undef FSP_CLAIM
    }
  });
  if (e != hipSuccess) return e;
  // 4. one workgroup per bin: group, rank, order, fold, emit
  ChunkArgs<VT> a{};
  a.colptr = nullptr;
  a.chunk_col = nullptr;
  a.bucket = bucket;
  a.vals = keys ? ss : nullptr;
  a.tmp = at<Entry<VT>>(ws, lo.tmp);
  a.N = (int32_t)N;
  a.T = 0;
  a.cap = tu.cap;
  a.Q = B;
  a.status = at<uint64_t>(ws, lo.bin_st);
  a.ctrl = ctrl;
  a.jcS = jcS_target;
  a.irS = irS;
  a.prS = prS;
  a.out_cap = cap;
  a.slot = slot;
  a.perm = keep_plan ? at<int32_t>(ws, lo.perm) : nullptr;
  a.seg = keep_plan ? at<int32_t>(ws, lo.seg) : nullptr;
  a.hostctrl = hostctrl;
#ifdef FSP_PHASE_TIMING
  a.phase = g_phase;
#endif
  a.rshift = packed ? s : 0;
  {
    // rank cells: split a column's rows into 2^nbl ranges so that a range
    // holds about two distinct rows of an average column, with at most 256
    // cells per bin (one wave then scans them)
    const int64_t per_col = std::max<int64_t>(1, L / std::max<int64_t>(1, N));
    int nbl = 0;
    while ((int64_t(4) << nbl) <= per_col && ((int64_t)g.w << (nbl + 1)) <= 256) ++nbl;
    int rowbits = 0;
    while ((int64_t(1) << rowbits) < mmax) ++rowbits;
    a.nbl = nbl;
    a.bsh = std::max(0, rowbits - nbl);
  }
  const uint32_t* bcol_in = packed ? nullptr : bcol;
  int32_t* colptr_g = at<int32_t>(ws, lo.colptr);
  const int kc = kernel_cap(tu.cap);
  const int nt = std::max(kc / 8, std::min(tu.cblock, kc));  // <= 8 triplets per thread
  int32_t* slowlist = at<int32_t>(ws, lo.slowlist);
  uint32_t* slowd = at<uint32_t>(ws, lo.slowd);
  uint64_t* slowb = at<uint64_t>(ws, lo.slowb);
  fsp::BinSrc src{binstart, binfill, bcol_in, slotcap, (int32_t)B, &ctrl->tick_chunk,
                  slowd, slowb};
  const unsigned sgrid = (unsigned)num_cus();
  // bins longer than the LDS: counted before the bin kernel, emitted after
  // (fixed-capacity bins never are)
  const bool may_slow = mode != kSlot;
  e = launch(kChunk, stream, [&] {
#define FSP_BIN(C, T)                                                          \
  do {                                                                         \
    if (may_slow)                                                              \
      hipLaunchKernelGGL((fsp::k_slow_count<VT, C, T>), dim3(sgrid), dim3(T), 0, \
                         stream, a, binstart, bcol_in, colptr_g, w, slowlist, \
                         slowd);                                               \
    if (keys)                                                                  \
      hipLaunchKernelGGL((fsp::k_bin<VT, C, T, true>),                         \
                         dim3((unsigned)std::min<int64_t>(B, resident<fsp::k_bin<VT, C, T, true>>(T))), \
                         dim3(T), 0, stream, a, src, w);                       \
    else                                                                       \
      hipLaunchKernelGGL((fsp::k_bin<VT, C, T, false>),                        \
                         dim3((unsigned)std::min<int64_t>(B, resident<fsp::k_bin<VT, C, T, false>>(T))), \
                         dim3(T), 0, stream, a, src, w);                       \
    if (may_slow)                                                              \
      hipLaunchKernelGGL((fsp::k_slow_emit<VT, C, T>), dim3(sgrid), dim3(T), 0, \
                         stream, a, binstart, colptr_g, w, slowlist, slowb);   \
  } while (0)
    if (kc == 1024) {
      if (nt <= 256) FSP_BIN(1024, 256); else if (nt <= 512) FSP_BIN(1024, 512); else FSP_BIN(1024, 1024);
    } else if (kc == 2048) {
      if (nt <= 256) FSP_BIN(2048, 256); else if (nt <= 512) FSP_BIN(2048, 512); else FSP_BIN(2048, 1024);
    } else {
      if (nt <= 512) FSP_BIN(4096, 512); else FSP_BIN(4096, 1024);
    }
#undef FSP_BIN
  });
  return e;
}

// Tile table of the re-use kernel (first output of every tile); reads the
// distinct count from the control block, so it can be queued before the
// readback.
hipError_t launch_reuse_tiles(void* ws, const Layout& lo, int64_t L,
                              hipStream_t stream) {
  const int64_t T = (L + kReuseTP - 1) / kReuseTP;
  return launch(kReuse, stream, [&] {
    hipLaunchKernelGGL(fsp::k_reuse_tiles, dim3(grid_for(L + 1, 256, 8)), dim3(256), 0,
                       stream, at<int32_t>(ws, lo.seg), &at<Ctrl>(ws, lo.ctrl)->nnz,
                       kReuseTP, T, at<int32_t>(ws, lo.rtile));
  });
}

// The ordered fold of a second value array along the sorted order and runs
// (perm, seg, rtile) a fresh pass with a kept plan leaves in the workspace.
hipError_t launch_reuse_direct(void* ws, const Layout& lo, int64_t L, fsparse_dtype dt,
                               int rblock, const void* ss, void* prS,
                               hipStream_t stream) {
  const int blk = rblock <= 256 ? 256 : (rblock <= 512 ? 512 : 1024);
  const int64_t T = (L + kReuseTP - 1) / kReuseTP;
  const int32_t* perm = at<int32_t>(ws, lo.perm);
  const int32_t* seg = at<int32_t>(ws, lo.seg);
  const int32_t* rtile = at<int32_t>(ws, lo.rtile);
  void* args[] = {(void*)&perm, (void*)&seg, (void*)&rtile, (void*)&ss, (void*)&prS};
  const void* fn = dt == FSPARSE_F64 ? reuse_fn<double>(blk) : reuse_fn<float>(blk);
  return launch(kReuse, stream, [&] {
    (void)hipLaunchKernel(fn, dim3((unsigned)T), dim3(blk), args, 0, stream);
  });
}

fsparse_status check_dt(fsparse_dtype dt) {
  return (dt == FSPARSE_F64 || dt == FSPARSE_F32) ? FSPARSE_OK : FSPARSE_E_ARG;
}

// Flags of the fresh calls: FSPARSE_NO_SYNC needs given dimensions (the
// defaults take a wait) and excludes dropping zeros (the kept count is read
// back between two passes).
fsparse_status check_flags(unsigned flags, int64_t m, int64_t n) {
  if (flags & ~(unsigned)(FSPARSE_ATOMIC | FSPARSE_DROP_ZEROS | FSPARSE_NO_SYNC))
    return FSPARSE_E_ARG;
  if ((flags & FSPARSE_NO_SYNC) && (m < 0 || n < 0 || (flags & FSPARSE_DROP_ZEROS)))
    return FSPARSE_E_ARG;
  return FSPARSE_OK;
}

constexpr int64_t kMaxI32 = 0x7FFFFFFE;

// Per-matrix largest row / column index of a batch (defaults of the batched
// call).  ws needs the small-table layout of make_layout(0, 0, nb, ...).
fsparse_status batched_dims(int32_t nb, const int64_t* trip_off,
                            const int32_t* ii, const int32_t* jj, int64_t L,
                            fsparse_dtype dt, const Tuning& tu, void* ws,
                            size_t ws_bytes, int64_t* mm, int64_t* nn,
                            hipStream_t stream) {
  Layout pre = make_layout(0, 0, nb, esize_of(dt), tu);
  if (ws_bytes < pre.total) return FSPARSE_E_CAPACITY;
  Ctrl* hi = static_cast<Ctrl*>(pinned());
  if (!hi || sizeof(Ctrl) + 8 * (size_t)nb > kPinnedBytes) return FSPARSE_E_ARG;
  std::memset(hi, 0, sizeof(Ctrl));
  hi->rmin = INT32_MAX;
  hi->cmin = INT32_MAX;
  HIPCHK(hipMemcpyAsync(ws, hi, sizeof(Ctrl), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemsetAsync(at<char>(ws, pre.bmax), 0, 8 * (size_t)nb, stream));
  HIPCHK(hipMemcpyAsync(at<int64_t>(ws, pre.b_trip), trip_off,
                        8 * (size_t)(nb + 1), hipMemcpyHostToDevice, stream));
  BatchDesc bd{at<int64_t>(ws, pre.b_trip), nullptr, nullptr, nullptr, nb};
  hipError_t e = launch(kDims, stream, [&] {
    hipLaunchKernelGGL(fsp::k_dims<true>, dim3(grid_for(L, 256, 8)), dim3(256),
                       0, stream, ii, jj, L, bd, (Ctrl*)ws,
                       at<int32_t>(ws, pre.bmax));
  });
  if (e != hipSuccess) return FSPARSE_E_HIP;
  char* h = reinterpret_cast<char*>(hi);
  HIPCHK(hipMemcpyAsync(h + sizeof(Ctrl), at<char>(ws, pre.bmax), 8 * (size_t)nb,
                        hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(h, ws, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const Ctrl* hc = reinterpret_cast<const Ctrl*>(h);
  if (hc->rmin < 1 || hc->cmin < 1) return FSPARSE_E_INDEX;
  const int32_t* bm = reinterpret_cast<const int32_t*>(h + sizeof(Ctrl));
  for (int b = 0; b < nb; ++b) {
    if (mm[b] < 0) mm[b] = bm[2 * b];
    if (nn[b] < 0) nn[b] = bm[2 * b + 1];
  }
  return FSPARSE_OK;
}

// ---------------------------------------------------------------------------
// scratch of the no-allocation entry point
// ---------------------------------------------------------------------------
// A device array of FSPARSE_NOALLOC_SCRATCH_BYTES held by every GPU the
// library runs on, for the whole process.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address on each GPU is
// looked up once (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[FSPARSE_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch[kMaxDev];

// The device address of the current device's scratch array, or null.
void* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* fsparse_version(void) { return "fsparse-mi355x 0.1 (gfx950)"; }

const char* fsparse_last_error(void) { return t_last_error; }

const char* fsparse_status_string(int s) {
  switch (s) {
    case FSPARSE_OK: return "ok";
    case FSPARSE_E_INDEX: return "index out of range";
    case FSPARSE_E_ARG: return "invalid argument";
    case FSPARSE_E_CAPACITY: return "capacity too small";
    case FSPARSE_E_PLAN: return "plan does not match";
    case FSPARSE_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

// Workspace of a call with tuning tu, with room for the geometry of a refit
// after fixed-capacity places overflow.
static size_t workspace_bytes_for(int64_t len, int64_t ncols, int32_t nb, fsparse_dtype dt,
                           const Tuning& tu) {
  return std::max(make_layout(len, ncols, nb, esize_of(dt), tu).total,
                  make_layout(len, ncols, nb, esize_of(dt), tu, true).total);
}

// Tuning of the new triplets' own assembly in delayed assembly: bins of at
// most 2048 entries (512 threads a workgroup).  Appended triplets are a part
// of the input whose density can vary across their columns (the growing
// region of a mesh, say); the fixed-capacity fill at 2048 entries (88%)
// leaves them a wider relative margin than 4096-entry bins (91%), which on
// the last tenth of fem3d_100 overflowed and took the counted redo.
static Tuning append_tuning() {
  Tuning tu = tuning();
  if (tu.cap > 2048) {
    tu.cap = 2048;
    tu.cblock = 512;
  }
  return tu;
}

size_t fsparse_workspace_bytes(int64_t len, int64_t ncols, int32_t nb,
                               fsparse_dtype dt) {
  if (len < 0 || ncols < 0 || nb < 1 || check_dt(dt) != FSPARSE_OK) return 0;
  return workspace_bytes_for(len, ncols, nb, dt, tuning());
}

// Default dimensions; with f64, ii and jj point to doubles (an index that is
// not a whole number in [1, 2^31 - 1] reads as 0: E_INDEX).
static fsparse_status dims_impl(const int32_t* ii, const int32_t* jj, int64_t len,
                                int64_t* m, int64_t* n, void* ws, size_t ws_bytes,
                                hipStream_t stream, bool f64, int64_t* cmin = nullptr) {
  if (!m || !n || len < 0 || len > kMaxI32 || !ws || ws_bytes < 256)
    return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj)) return FSPARSE_E_ARG;
  if (len == 0) {
    *m = 0;
    *n = 0;
    if (cmin) *cmin = 1;
    return FSPARSE_OK;
  }
  Ctrl* h = static_cast<Ctrl*>(pinned());
  if (!h) return FSPARSE_E_HIP;
  std::memset(h, 0, sizeof(Ctrl));
  h->rmin = INT32_MAX;
  h->cmin = INT32_MAX;
  HIPCHK(hipMemcpyAsync(ws, h, sizeof(Ctrl), hipMemcpyHostToDevice, stream));
  BatchDesc bd{};
  hipError_t e = launch(kDims, stream, [&] {
    if (f64)
      hipLaunchKernelGGL((fsp::k_dims<false, fsp::kIdxF64>), dim3(grid_for(len, 1024, 2)),
                         dim3(1024), 0, stream, ii, jj, len, bd, (Ctrl*)ws,
                         (int32_t*)nullptr);
    else
      hipLaunchKernelGGL(fsp::k_dims<false>, dim3(grid_for(len, 1024, 2)), dim3(1024),
                         0, stream, ii, jj, len, bd, (Ctrl*)ws, (int32_t*)nullptr);
  });
  if (e != hipSuccess) return FSPARSE_E_HIP;
  HIPCHK(hipMemcpyAsync(h, ws, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (h->rmin < 1 || h->cmin < 1) return FSPARSE_E_INDEX;
  *m = h->rmax;
  *n = h->cmax;
  if (cmin) *cmin = h->cmin;
  return FSPARSE_OK;
}

fsparse_status fsparse_dims(const int32_t* ii, const int32_t* jj, int64_t len,
                            int64_t* m, int64_t* n, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  return dims_impl(ii, jj, len, m, n, ws, ws_bytes, stream, false);
}

fsparse_status fsparse_dims_f64idx(const double* ii, const double* jj, int64_t len,
                                   int64_t* m, int64_t* n, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
  return dims_impl(reinterpret_cast<const int32_t*>(ii),
                   reinterpret_cast<const int32_t*>(jj), len, m, n, ws, ws_bytes,
                   stream, true);
}

// Fresh assembly once the dimensions are known; `src` says where the
// indices come from (with kIdxExpand, ii, jj and ss are read through `ex`;
// with kIdxF64, ii and jj point to doubles).
static fsparse_status assemble_impl(const int32_t* ii, const int32_t* jj,
                             const void* ss, fsparse_dtype dt, int64_t len,
                             int64_t m, int64_t n, int64_t nzmax,
                             unsigned flags, int32_t* jcS, int64_t jcS_cap,
                             int32_t* irS, void* prS, int64_t cap,
                             int32_t* slot, void* ws, size_t ws_bytes,
                             fsparse_plan** plan, fsparse_info* info,
                             hipStream_t stream, int src,
                             const fsp::Expand* ex,
                             const void* si = nullptr, void* piS = nullptr,
                             bool keep_order = false, Layout* lo_out = nullptr,
                             const Tuning* tu_in = nullptr) {
  if (info) {
    info->m = m;
    info->n = n;
    info->nnz = 0;
    info->nzmax = std::max<int64_t>(nzmax, 0);
  }
  if (jcS_cap < n + 1) return FSPARSE_E_CAPACITY;
  // without a wait the host cannot redo the call, so fixed-capacity bins
  // (which may overflow and need a counted redo) give way to counting first,
  // and cap must hold every distinct pair there can be (len)
  const bool nosync = (flags & FSPARSE_NO_SYNC) != 0;
  if (nosync && cap < len) {
    if (info) info->nnz = len;
    return FSPARSE_E_CAPACITY;
  }
  Tuning tu = tu_in ? *tu_in : tuning();
  Layout lo = make_layout(len, n, 1, esize_of(dt), tu);
  if (nosync && lo.g.mode == kSlot) {
    tu.bmode = 1 + kClaim;
    lo = make_layout(len, n, 1, esize_of(dt), tu);
  }
  if (ws_bytes < lo.total) return FSPARSE_E_CAPACITY;
  if (lo_out) *lo_out = lo;
  Ctrl* ctrl = at<Ctrl>(ws, lo.ctrl);
  // complex values: the imaginary parts are folded along the sorted order
  // that the real parts' pass leaves in the workspace
  const bool keep = plan != nullptr || si != nullptr || keep_order;
  // the re-use tiles serve the re-use kernel (plans, imaginary parts) only
  const bool tiles = plan != nullptr || si != nullptr;
  // the atomic sums need a slot map (the caller's, else an internal one);
  // a plan's ordered re-use and the imaginary fold read only the sorted
  // order, and a plan derives its slot map on its first atomic re-use
  const bool use_islot = (plan != nullptr || si != nullptr) && (flags & FSPARSE_ATOMIC);
  int32_t* slot_used = slot ? slot : (use_islot ? at<int32_t>(ws, lo.islot) : nullptr);
  if (len == 0) {
    hipError_t e = launch(kInit, stream, [&] {
      hipLaunchKernelGGL(fsp::k_zero, dim3(grid_for(n + 1, 256, 4)), dim3(256), 0,
                         stream, (uint32_t*)jcS, (int64_t)(n + 1));
      // the control block (nnz = 0, no error) for fsparse_assemble_status
      hipLaunchKernelGGL(fsp::k_zero, dim3(1), dim3(64), 0, stream,
                         (uint32_t*)ctrl, (int64_t)(sizeof(Ctrl) / 4));
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
    if (!nosync) HIPCHK(hipStreamSynchronize(stream));
  } else if (nosync) {
    // queue everything; nnz and the error bits stay in the control block
    BatchDesc bd{};
    const fsp::Expand x = ex ? *ex : fsp::Expand{};
    hipError_t e;
#define FSP_RUN(VT, S)                                                          \
  run_pipeline<VT, false, S>(ii, jj, (const VT*)ss, len, (int32_t)m, (int32_t)n, bd, n, \
                             lo, tu, ws, jcS, irS, (VT*)prS, cap, slot_used, keep, \
                             lo.g.mode, stream, nullptr, x)
    if (dt == FSPARSE_F64)
      e = src == fsp::kIdxExpand ? FSP_RUN(double, fsp::kIdxExpand)
        : src == fsp::kIdxF64    ? FSP_RUN(double, fsp::kIdxF64)
                                 : FSP_RUN(double, fsp::kIdxI32);
    else
      e = src == fsp::kIdxExpand ? FSP_RUN(float, fsp::kIdxExpand)
        : src == fsp::kIdxF64    ? FSP_RUN(float, fsp::kIdxF64)
                                 : FSP_RUN(float, fsp::kIdxI32);
#undef FSP_RUN
    if (e != hipSuccess) return FSPARSE_E_HIP;
    if (tiles && launch_reuse_tiles(ws, lo, len, stream) != hipSuccess) return FSPARSE_E_HIP;
    const int64_t* dnnz = &ctrl->nnz;
    if (info) info->nnz = -1;
    if (flags & FSPARSE_ATOMIC) {
      if (!slot_used) return FSPARSE_E_ARG;
      hipError_t ea = dt == FSPARSE_F64
          ? launch_atomic_values<double>(slot_used, ss, len, prS, -1, tu.rblock, stream, dnnz)
          : launch_atomic_values<float>(slot_used, ss, len, prS, -1, tu.rblock, stream, dnnz);
      if (ea != hipSuccess) return FSPARSE_E_HIP;
    }
    if (si) {
      hipError_t ei;
      if (flags & FSPARSE_ATOMIC)
        ei = dt == FSPARSE_F64
            ? launch_atomic_values<double>(slot_used, si, len, piS, -1, tu.rblock, stream, dnnz)
            : launch_atomic_values<float>(slot_used, si, len, piS, -1, tu.rblock, stream, dnnz);
      else
        ei = launch_reuse_direct(ws, lo, len, dt, tu.rblock, si, piS, stream);
      if (ei != hipSuccess) return FSPARSE_E_HIP;
    }
    if (plan) {
      fsparse_plan* pl = new (std::nothrow) fsparse_plan();
      if (!pl) return FSPARSE_E_ARG;
      pl->len = len;
      pl->nnz = -1;
      pl->dnnz = dnnz;
      pl->dt = dt;
      hipGetDevice(&pl->device);
      pl->perm = at<int32_t>(ws, lo.perm);
      pl->seg = at<int32_t>(ws, lo.seg);
      pl->slot = slot_used;
      pl->islot = at<int32_t>(ws, lo.islot);
      pl->rtile = at<int32_t>(ws, lo.rtile);
      pl->ntiles = (len + kReuseTP - 1) / kReuseTP;
      pl->rblock = tu.rblock;
      *plan = pl;
    }
    return FSPARSE_OK;
  } else {
    BatchDesc bd{};
    Ctrl* h = static_cast<Ctrl*>(pinned());
    if (!h) return FSPARSE_E_HIP;
    int mode = lo.g.mode;
    for (;;) {
      const fsp::Expand x = ex ? *ex : fsp::Expand{};
      hipError_t e;
#define FSP_RUN(VT, S)                                                          \
  run_pipeline<VT, false, S>(ii, jj, (const VT*)ss, len, (int32_t)m, (int32_t)n, bd, n, \
                             lo, tu, ws, jcS, irS, (VT*)prS, cap, slot_used, keep, \
                             mode, stream, h, x)
      if (dt == FSPARSE_F64)
        e = src == fsp::kIdxExpand ? FSP_RUN(double, fsp::kIdxExpand)
          : src == fsp::kIdxF64    ? FSP_RUN(double, fsp::kIdxF64)
                                   : FSP_RUN(double, fsp::kIdxI32);
      else
        e = src == fsp::kIdxExpand ? FSP_RUN(float, fsp::kIdxExpand)
          : src == fsp::kIdxF64    ? FSP_RUN(float, fsp::kIdxF64)
                                   : FSP_RUN(float, fsp::kIdxI32);
#undef FSP_RUN
      if (e != hipSuccess) return FSPARSE_E_HIP;
      if (tiles && launch_reuse_tiles(ws, lo, len, stream) != hipSuccess) return FSPARSE_E_HIP;
      // the bin kernel's last block has written err and nnz into h
      HIPCHK(hipStreamSynchronize(stream));
      // a full fixed-capacity bin: count first, in narrower bins, and redo
      if ((h->err & fsp::kErrSlot) && mode == kSlot) {
        lo = make_layout(len, n, 1, esize_of(dt), tu, true);
        if (ws_bytes < lo.total) return FSPARSE_E_CAPACITY;
        slot_used = slot ? slot : (use_islot ? at<int32_t>(ws, lo.islot) : nullptr);
        mode = lo.g.mode;
        continue;
      }
      break;
    }
    if (lo_out) *lo_out = lo;
    const uint32_t err = h->err;
    const int64_t nnz = h->nnz;
    if (info) {
      info->nnz = nnz;
      info->nzmax = std::max<int64_t>(nzmax, nnz);
    }
    if (err & (fsp::kErrCol | fsp::kErrRow)) return FSPARSE_E_INDEX;
    if ((err & fsp::kErrCap) || nnz > cap) return FSPARSE_E_CAPACITY;
    if (flags & FSPARSE_ATOMIC) {
      if (!slot_used) {
        // the atomic sum needs the slot map: use the internal one
        return FSPARSE_E_ARG;
      }
      hipError_t ea = dt == FSPARSE_F64
          ? launch_atomic_values<double>(slot_used, ss, len, prS, nnz, tu.rblock, stream)
          : launch_atomic_values<float>(slot_used, ss, len, prS, nnz, tu.rblock, stream);
      if (ea != hipSuccess) return FSPARSE_E_HIP;
    }
    if (si) {
      hipError_t ei;
      if (flags & FSPARSE_ATOMIC)
        ei = dt == FSPARSE_F64
            ? launch_atomic_values<double>(slot_used, si, len, piS, nnz, tu.rblock, stream)
            : launch_atomic_values<float>(slot_used, si, len, piS, nnz, tu.rblock, stream);
      else
        ei = launch_reuse_direct(ws, lo, len, dt, tu.rblock, si, piS, stream);
      if (ei != hipSuccess) return FSPARSE_E_HIP;
    }
    if (flags & FSPARSE_DROP_ZEROS) {
      hipError_t ed = dt == FSPARSE_F64
          ? drop_zeros<double>(ws, lo, nnz, n, len, jcS, irS, (double*)prS, slot, h, stream,
                               (double*)piS)
          : drop_zeros<float>(ws, lo, nnz, n, len, jcS, irS, (float*)prS, slot, h, stream,
                              (float*)piS);
      if (ed != hipSuccess) return FSPARSE_E_HIP;
      HIPCHK(hipStreamSynchronize(stream));
      if (info) info->nnz = h->kept;
    }
    if (plan) {
      fsparse_plan* pl = new (std::nothrow) fsparse_plan();
      if (!pl) return FSPARSE_E_ARG;
      pl->len = len;
      pl->nnz = nnz;
      pl->dnnz = &at<Ctrl>(ws, lo.ctrl)->nnz;
      pl->dt = dt;
      hipGetDevice(&pl->device);
      pl->perm = at<int32_t>(ws, lo.perm);
      pl->seg = at<int32_t>(ws, lo.seg);
      pl->slot = slot_used;
      pl->islot = at<int32_t>(ws, lo.islot);
      pl->rtile = at<int32_t>(ws, lo.rtile);
      pl->ntiles = (len + kReuseTP - 1) / kReuseTP;
      pl->rblock = tu.rblock;
      *plan = pl;
    }
    return FSPARSE_OK;
  }
  if (plan) {
    fsparse_plan* pl = new (std::nothrow) fsparse_plan();
    if (!pl) return FSPARSE_E_ARG;
    pl->dt = dt;
    hipGetDevice(&pl->device);
    pl->rblock = tu.rblock;
    *plan = pl;
  }
  return FSPARSE_OK;
}

fsparse_status fsparse_assemble(const int32_t* ii, const int32_t* jj,
                                const void* ss, fsparse_dtype dt, int64_t len,
                                int64_t m, int64_t n, int64_t nzmax,
                                unsigned flags, int32_t* jcS, int64_t jcS_cap,
                                int32_t* irS, void* prS, int64_t cap,
                                int32_t* slot, void* ws, size_t ws_bytes,
                                fsparse_plan** plan, fsparse_info* info,
                                hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK) return FSPARSE_E_ARG;
  if (len < 0 || len > kMaxI32 || m > kMaxI32 || n > kMaxI32) return FSPARSE_E_ARG;
  if (check_flags(flags, m, n) != FSPARSE_OK) return FSPARSE_E_ARG;
  // the pattern of a call that drops zeros depends on the values: no plan
  if ((flags & FSPARSE_DROP_ZEROS) && plan) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !ss)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (plan) *plan = nullptr;
  if (m < 0 || n < 0) {
    int64_t dm = 0, dn = 0;
    fsparse_status st = fsparse_dims(ii, jj, len, &dm, &dn, ws, ws_bytes, stream);
    if (st != FSPARSE_OK) return st;
    if (m < 0) m = dm;
    if (n < 0) n = dn;
  }
  return assemble_impl(ii, jj, ss, dt, len, m, n, nzmax, flags, jcS, jcS_cap, irS,
                       prS, cap, slot, ws, ws_bytes, plan, info, stream,
                       fsp::kIdxI32, nullptr);
}

fsparse_status fsparse_assemble_noalloc(const int32_t* ii, const int32_t* jj,
                                        const void* ss, fsparse_dtype dt,
                                        int64_t len, int64_t m, int64_t n,
                                        int64_t nzmax, unsigned flags,
                                        int32_t* jcS, int64_t jcS_cap,
                                        int32_t* irS, void* prS, int64_t cap,
                                        int32_t* slot, fsparse_info* info,
                                        hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK) return FSPARSE_E_ARG;
  if (len < 0 || len > kMaxI32 || m < 0 || n < 0 || m > kMaxI32 || n > kMaxI32)
    return FSPARSE_E_ARG;
  if (flags & ~(unsigned)FSPARSE_ATOMIC) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !ss)) return FSPARSE_E_ARG;
  if (!jcS || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (info) {
    info->m = m;
    info->n = n;
    info->nnz = 0;
    info->nzmax = std::max<int64_t>(nzmax, 0);
  }
  // every distinct pair must fit without a capacity retry
  if (cap < len) {
    if (info) info->nnz = len;
    return FSPARSE_E_CAPACITY;
  }
  if (fsparse_workspace_bytes(len, n, 1, dt) > (size_t)FSPARSE_NOALLOC_SCRATCH_BYTES)
    return FSPARSE_E_CAPACITY;
  void* ws = scratch_ptr();
  if (!ws) return FSPARSE_E_HIP;
  struct NoAlloc {
    NoAlloc() { t_noalloc = true; }
    ~NoAlloc() { t_noalloc = false; }
  } guard;
  // the queued pipeline (counted bins: no host-decided redo), which clears
  // the control block and look-back words it uses, then one wait to read
  // them back
  fsparse_status st = assemble_impl(ii, jj, ss, dt, len, m, n, nzmax,
                                    flags | FSPARSE_NO_SYNC, jcS, jcS_cap, irS, prS,
                                    cap, slot, ws, FSPARSE_NOALLOC_SCRATCH_BYTES,
                                    nullptr, info, stream, fsp::kIdxI32, nullptr);
  if (st != FSPARSE_OK) return st;
  fsparse_info got{};
  st = fsparse_assemble_status(ws, &got, stream);
  if (info) {
    info->nnz = got.nnz;
    info->nzmax = std::max<int64_t>(nzmax, got.nnz);
  }
  return st;
}

fsparse_status fsparse_assemble_f64idx(const double* ii, const double* jj,
                                       const void* ss, fsparse_dtype dt,
                                       int64_t len, int64_t m, int64_t n,
                                       int64_t nzmax, unsigned flags,
                                       int32_t* jcS, int64_t jcS_cap,
                                       int32_t* irS, void* prS, int64_t cap,
                                       int32_t* slot, void* ws, size_t ws_bytes,
                                       fsparse_plan** plan, fsparse_info* info,
                                       hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK) return FSPARSE_E_ARG;
  if (len < 0 || len > kMaxI32 || m > kMaxI32 || n > kMaxI32) return FSPARSE_E_ARG;
  if (check_flags(flags, m, n) != FSPARSE_OK) return FSPARSE_E_ARG;
  // the pattern of a call that drops zeros depends on the values: no plan
  if ((flags & FSPARSE_DROP_ZEROS) && plan) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !ss)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (plan) *plan = nullptr;
  if (m < 0 || n < 0) {
    int64_t dm = 0, dn = 0;
    fsparse_status st = fsparse_dims_f64idx(ii, jj, len, &dm, &dn, ws, ws_bytes, stream);
    if (st != FSPARSE_OK) return st;
    if (m < 0) m = dm;
    if (n < 0) n = dn;
  }
  return assemble_impl(reinterpret_cast<const int32_t*>(ii),
                       reinterpret_cast<const int32_t*>(jj), ss, dt, len, m, n,
                       nzmax, flags, jcS, jcS_cap, irS, prS, cap, slot, ws,
                       ws_bytes, plan, info, stream, fsp::kIdxF64, nullptr);
}

fsparse_status fsparse_assemble_complex(const int32_t* ii, const int32_t* jj,
                                        const void* sr, const void* si,
                                        fsparse_dtype dt, int64_t len, int64_t m,
                                        int64_t n, int64_t nzmax, unsigned flags,
                                        int32_t* jcS, int64_t jcS_cap, int32_t* irS,
                                        void* prS, void* piS, int64_t cap,
                                        int32_t* slot, void* ws, size_t ws_bytes,
                                        fsparse_plan** plan, fsparse_info* info,
                                        hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK) return FSPARSE_E_ARG;
  if (len < 0 || len > kMaxI32 || m > kMaxI32 || n > kMaxI32) return FSPARSE_E_ARG;
  if (check_flags(flags, m, n) != FSPARSE_OK) return FSPARSE_E_ARG;
  if ((flags & FSPARSE_DROP_ZEROS) && plan) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !sr || !si)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS || !piS))) return FSPARSE_E_ARG;
  if (plan) *plan = nullptr;
  if (m < 0 || n < 0) {
    int64_t dm = 0, dn = 0;
    fsparse_status st = fsparse_dims(ii, jj, len, &dm, &dn, ws, ws_bytes, stream);
    if (st != FSPARSE_OK) return st;
    if (m < 0) m = dm;
    if (n < 0) n = dn;
  }
  return assemble_impl(ii, jj, sr, dt, len, m, n, nzmax, flags, jcS, jcS_cap, irS,
                       prS, cap, slot, ws, ws_bytes, plan, info, stream, fsp::kIdxI32,
                       nullptr, si, piS);
}

// Logical values: the fp32 pipeline on 0/1 indicators with the zero sums
// dropped; ws holds the pipeline's workspace, then the indicators, then the
// fp32 sums.
static size_t logical_head(int64_t len, int64_t ncols) {
  const size_t h = fsparse_workspace_bytes(len, ncols, 1, FSPARSE_F32);
  return (h + 255) & ~size_t(255);
}

size_t fsparse_logical_workspace_bytes(int64_t len, int64_t ncols) {
  if (len < 0 || ncols < 0) return 0;
  const size_t h = logical_head(len, ncols);
  if (h == 0) return 0;
  const size_t a = (4 * (size_t)std::max<int64_t>(len, 1) + 255) & ~size_t(255);
  return h + 2 * a;
}

fsparse_status fsparse_assemble_logical(const int32_t* ii, const int32_t* jj,
                                        const uint8_t* sl, int64_t len, int64_t m,
                                        int64_t n, int64_t nzmax, int32_t* jcS,
                                        int64_t jcS_cap, int32_t* irS, uint8_t* prS,
                                        int64_t cap, int32_t* slot, void* ws,
                                        size_t ws_bytes, fsparse_info* info,
                                        hipStream_t stream) {
  if (len < 0 || len > kMaxI32 || m > kMaxI32 || n > kMaxI32) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !sl)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (m < 0 || n < 0) {
    int64_t dm = 0, dn = 0;
    fsparse_status st = fsparse_dims(ii, jj, len, &dm, &dn, ws, ws_bytes, stream);
    if (st != FSPARSE_OK) return st;
    if (m < 0) m = dm;
    if (n < 0) n = dn;
  }
  fsparse_info li{};
  li.m = m;
  li.n = n;
  li.nzmax = std::max<int64_t>(nzmax, 0);
  if (info) *info = li;
  const size_t head = logical_head(len, n);
  if (ws_bytes < fsparse_logical_workspace_bytes(len, n)) return FSPARSE_E_CAPACITY;
  const int64_t L1 = std::max<int64_t>(len, 1);
  const size_t a = (4 * (size_t)L1 + 255) & ~size_t(255);
  float* v = at<float>(ws, head);
  float* pf = at<float>(ws, head + a);
  if (len > 0) {
    hipError_t e = launch(kFill, stream, [&] {
      hipLaunchKernelGGL(fsp::k_logical_ind, dim3(grid_for(len, 256, 8)), dim3(256), 0,
                         stream, sl, len, v);
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
  }
  // irS and the fp32 sums hold min(cap, len) pairs (nnz <= len)
  fsparse_status st = assemble_impl(ii, jj, v, FSPARSE_F32, len, m, n, nzmax,
                                    FSPARSE_DROP_ZEROS, jcS, jcS_cap, irS, pf,
                                    std::min(cap, L1), slot, ws, head, nullptr, &li,
                                    stream, fsp::kIdxI32, nullptr);
  if (info) *info = li;
  if (st != FSPARSE_OK) return st;
  if (li.nnz > 0) {
    hipError_t e = launch(kFill, stream, [&] {
      hipLaunchKernelGGL(fsp::k_fill_true, dim3(grid_for(li.nnz, 256, 8)), dim3(256), 0,
                         stream, prS, li.nnz);
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
  }
  return FSPARSE_OK;
}

// Exact division by d on [0, 2^31) in the bins' multiply-high form.
static fsp::BinGeo divisor(int64_t d) {
  Geom g{};
  set_divisor(g, d);
  return fsp::BinGeo{g.mul, g.sh, (int32_t)g.w, g.s};
}

fsparse_status fsparse_assemble_expand(const int32_t* ii, const int32_t* jj,
                                       const void* ss, fsparse_dtype dt,
                                       const fsparse_expand* x, int64_t m,
                                       int64_t n, int64_t nzmax, unsigned flags,
                                       int32_t* jcS, int64_t jcS_cap, int32_t* irS,
                                       void* prS, int64_t cap, int32_t* slot,
                                       void* ws, size_t ws_bytes,
                                       fsparse_plan** plan, fsparse_info* info,
                                       hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK || !x) return FSPARSE_E_ARG;
  if (m > kMaxI32 || n > kMaxI32) return FSPARSE_E_ARG;
  if (check_flags(flags, m, n) != FSPARSE_OK) return FSPARSE_E_ARG;
  // the pattern of a call that drops zeros depends on the values: no plan
  if ((flags & FSPARSE_DROP_ZEROS) && plan) return FSPARSE_E_ARG;
  int64_t len = 1;
  for (int d = 0; d < 3; ++d) {
    if (x->shape[d] < 0 || x->shape[d] > kMaxI32) return FSPARSE_E_ARG;
    len *= x->shape[d];
    if (len > kMaxI32) return FSPARSE_E_ARG;
  }
  // every operand dimension is 1 or the grid's; strides of a dense array
  const int64_t* shp[3] = {x->ii_shape, x->jj_shape, x->ss_shape};
  int64_t size[3];
  uint32_t stride[3][3];
  bool full_ss = true;
  for (int a = 0; a < 3; ++a) {
    int64_t st = 1;
    for (int d = 0; d < 3; ++d) {
      const int64_t k = shp[a][d];
      if (k != 1 && k != x->shape[d]) return FSPARSE_E_ARG;
      stride[a][d] = (k == 1) ? 0u : (uint32_t)st;
      st *= k;
      if (a == 2 && k != x->shape[d]) full_ss = false;
    }
    size[a] = st;
  }
  // the order-free sum reads ss by triplet number
  if ((flags & FSPARSE_ATOMIC) && !full_ss) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !ss)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (plan) *plan = nullptr;
  if (m < 0 || n < 0) {
    // with at least one triplet every operand element is used, so the
    // largest index of an operand is the largest over the triplets
    int64_t dm = 0, dn = 0, dummy = 0;
    if (len > 0) {
      fsparse_status st = fsparse_dims(ii, ii, size[0], &dm, &dummy, ws, ws_bytes, stream);
      if (st != FSPARSE_OK) return st;
      st = fsparse_dims(jj, jj, size[1], &dummy, &dn, ws, ws_bytes, stream);
      if (st != FSPARSE_OK) return st;
    }
    if (m < 0) m = dm;
    if (n < 0) n = dn;
  }
  fsp::Expand ex{};
  ex.dR = divisor(std::max<int64_t>(1, x->shape[0]));
  ex.dC = divisor(std::max<int64_t>(1, x->shape[1]));
  ex.R = (uint32_t)x->shape[0];
  ex.C = (uint32_t)x->shape[1];
  for (int d = 0; d < 3; ++d) {
    ex.si[d] = stride[0][d];
    ex.sj[d] = stride[1][d];
    ex.sv[d] = stride[2][d];
  }
  return assemble_impl(ii, jj, ss, dt, len, m, n, nzmax, flags, jcS, jcS_cap, irS,
                       prS, cap, slot, ws, ws_bytes, plan, info, stream,
                       fsp::kIdxExpand, &ex);
}

// Delayed assembly: the stored pairs of the existing matrix, then the new
// triplets, as one triplet list at the head of the workspace.
static size_t append_head(int64_t Lc, fsparse_dtype dt) {
  const size_t vb = dt == FSPARSE_F64 ? 8 : 4;
  return al(4 * (size_t)Lc) * 2 + al(vb * (size_t)Lc);
}

// Workspace of the merge path: its control block, B's CCS, slot map and
// merged positions, and the look-back words of the merge blocks; then the
// fresh assembly's workspace for the new triplets.
struct MergeLayout {
  size_t ctrl, jcB, irB, prB, slotB, mapB, jjB, st, head;
};

// (nB: B's columns; n: the result's)
static MergeLayout merge_layout(int64_t len, int64_t nB, int64_t n, fsparse_dtype dt) {
  const size_t vb = dt == FSPARSE_F64 ? 8 : 4;
  const int64_t nscan = n + 1;  // look-back words, one per merge block (at most one per column)
  MergeLayout o{};
  size_t p = 0;
  o.ctrl = p;   p = al(p + sizeof(Ctrl));
  o.jcB = p;    p = al(p + 4 * (size_t)(nB + 1));
  o.irB = p;    p = al(p + 4 * (size_t)std::max<int64_t>(len, 1));
  o.prB = p;    p = al(p + vb * (size_t)std::max<int64_t>(len, 1));
  o.slotB = p;  p = al(p + 4 * (size_t)len);
  o.mapB = p;   p = al(p + 4 * (size_t)len);
  o.jjB = p;    p = al(p + 4 * (size_t)len);
  o.st = p;     p = al(p + 8 * (size_t)nscan);
  o.head = p;
  return o;
}

size_t fsparse_append_workspace_bytes(int64_t nnzA, int64_t len, int64_t n,
                                      fsparse_dtype dt) {
  if (nnzA < 0 || len < 0 || n < 0 || check_dt(dt) != FSPARSE_OK) return 0;
  // the larger of the two paths: merge (plain calls) and re-assembly of all
  // the pairs as triplets (plans, dropped zeros)
  const size_t w = fsparse_workspace_bytes(nnzA + len, n, 1, dt);
  const size_t wm = workspace_bytes_for(len, n, 1, dt, append_tuning());
  if (!w || !wm) return 0;
  return std::max(append_head(nnzA + len, dt) + w, merge_layout(len, n, n, dt).head + wm);
}

// Delayed assembly by re-assembly of everything: the stored pairs become
// triplets (first, in storage order), followed by the new ones.
static fsparse_status append_resort(const int32_t* jcA, const int32_t* irA,
                                    const void* prA, int64_t nnzA, int64_t nA,
                                    const int32_t* ii, const int32_t* jj,
                                    const void* ss, int64_t len, fsparse_dtype dt,
                                    int64_t m, int64_t n, unsigned flags,
                                    int32_t* jcS, int64_t jcS_cap, int32_t* irS,
                                    void* prS, int64_t cap, int32_t* slot,
                                    void* ws, size_t ws_bytes,
                                    fsparse_plan** plan, fsparse_info* info,
                                    hipStream_t stream) {
  const int64_t Lc = nnzA + len;
  const size_t head = append_head(Lc, dt);
  if (ws_bytes < head + 256) return FSPARSE_E_CAPACITY;
  const size_t vb = dt == FSPARSE_F64 ? 8 : 4;
  int32_t* ic = static_cast<int32_t*>(ws);
  int32_t* jc = at<int32_t>(ws, al(4 * (size_t)Lc));
  void* sc = at<char>(ws, 2 * al(4 * (size_t)Lc));
  void* ws2 = at<char>(ws, head);
  const size_t ws2_bytes = ws_bytes - head;
  // the stored pairs first (their own order), then the new triplets: every
  // pair's fold continues from its stored sum, which equals folding all of
  // its contributions in order (a fold from +0.0 never ends at -0.0)
  if (nnzA > 0) {
    hipError_t e = launch(kAppend, stream, [&] {
      // one block per 2048 stored pairs (the kernel's NT * EPT)
      const dim3 grid((unsigned)((nnzA + 2047) / 2048));
      if (dt == FSPARSE_F64)
        hipLaunchKernelGGL((fsp::k_ccs_triplets<double, 256, 8>), grid, dim3(256), 0,
                           stream, jcA, irA, (const double*)prA, nA, nnzA, ic, jc,
                           (double*)sc);
      else
        hipLaunchKernelGGL((fsp::k_ccs_triplets<float, 256, 8>), grid, dim3(256), 0,
                           stream, jcA, irA, (const float*)prA, nA, nnzA, ic, jc,
                           (float*)sc);
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
  }
  if (len > 0) {
    HIPCHK(hipMemcpyAsync(ic + nnzA, ii, 4 * (size_t)len, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(jc + nnzA, jj, 4 * (size_t)len, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(static_cast<char*>(sc) + vb * nnzA, ss, vb * (size_t)len,
                          hipMemcpyDeviceToDevice, stream));
  }
  if (m < 0 || n < 0) {
    int64_t dm = 0, dn = 0;
    fsparse_status st = dims_impl(ic, jc, Lc, &dm, &dn, ws2, ws2_bytes, stream, false);
    if (st != FSPARSE_OK) return st;
    if (m < 0) m = dm;
    if (n < 0) n = std::max(dn, nA);
  }
  return assemble_impl(ic, jc, sc, dt, Lc, m, n, 0, flags, jcS, jcS_cap, irS, prS, cap,
                       slot, ws2, ws2_bytes, plan, info, stream, fsp::kIdxI32, nullptr);
}

// Delayed assembly by merge (no plan, no dropped zeros): the new triplets
// are assembled on their own with their sorted order kept, then merged with
// the stored columns.  Waits twice (the fresh call's wait, then nnz).
static fsparse_status append_merge(const int32_t* jcA, const int32_t* irA,
                                   const void* prA, int64_t nnzA, int64_t nA,
                                   const int32_t* ii, const int32_t* jj,
                                   const void* ss, int64_t len, fsparse_dtype dt,
                                   int64_t m, int64_t n, int32_t* jcS,
                                   int64_t jcS_cap, int32_t* irS, void* prS,
                                   int64_t cap, int32_t* slot, void* ws,
                                   size_t ws_bytes, fsparse_info* info,
                                   hipStream_t stream) {
  Ctrl* h = static_cast<Ctrl*>(pinned());
  if (!h) return FSPARSE_E_HIP;
  // the new triplets' index range (B is assembled on its own columns, so
  // that new triplets in a part of the matrix fill its bins as they would
  // fill those of a matrix of that part alone)
  if (ws_bytes < 256) return FSPARSE_E_CAPACITY;
  int64_t dm = 0, dn = 0, dc = 1;
  {
    fsparse_status st = dims_impl(ii, jj, len, &dm, &dn, ws, ws_bytes, stream, false, &dc);
    if (st != FSPARSE_OK) return st;
  }
  if (m < 0) {
    // and the stored matrix's rows
    Ctrl* c = static_cast<Ctrl*>(ws);
    hipError_t e = launch(kDims, stream, [&] {
      hipLaunchKernelGGL(fsp::k_zero, dim3(1), dim3(64), 0, stream, (uint32_t*)c,
                         (int64_t)(sizeof(Ctrl) / 4));
      if (nnzA > 0)
        hipLaunchKernelGGL(fsp::k_rowmax, dim3(grid_for(nnzA, 256, 8)), dim3(256), 0,
                           stream, irA, nnzA, &c->rmax);
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
    HIPCHK(hipMemcpyAsync(h, c, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    m = std::max<int64_t>(dm, h->rmax);
  }
  if (n < 0) n = std::max(dn, nA);
  if (info) {
    info->m = m;
    info->n = n;
    info->nnz = 0;
    info->nzmax = 0;
  }
  if (m > kMaxI32 || n > kMaxI32) return FSPARSE_E_ARG;
  if (nA > n || dn > n) return FSPARSE_E_INDEX;
  if (jcS_cap < n + 1) return FSPARSE_E_CAPACITY;
  // B's columns: [boff, boff + nB) of the result
  const int64_t boff = len > 0 ? dc - 1 : 0;
  const int64_t nB = len > 0 ? dn - boff : 0;
  const MergeLayout ml = merge_layout(len, nB, n, dt);
  if (ws_bytes < ml.head) return FSPARSE_E_CAPACITY;
  Ctrl* ctrl = at<Ctrl>(ws, ml.ctrl);
  int32_t* jcB = at<int32_t>(ws, ml.jcB);
  int32_t* irB = at<int32_t>(ws, ml.irB);
  void* prB = at<char>(ws, ml.prB);
  int32_t* slotB = slot ? at<int32_t>(ws, ml.slotB) : nullptr;
  int32_t* mapB = slot ? at<int32_t>(ws, ml.mapB) : nullptr;
  void* ws2 = at<char>(ws, ml.head);
  const int32_t* jjB = jj;
  if (boff > 0) {
    int32_t* sh = at<int32_t>(ws, ml.jjB);
    hipError_t e = launch(kAppend, stream, [&] {
      hipLaunchKernelGGL(fsp::k_shift_index, dim3(grid_for(len, 256, 16)), dim3(256), 0,
                         stream, jj, len, (int32_t)boff, sh);
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
    jjB = sh;
  }
  // B: the new triplets alone, ordered, with their sorted order kept
  Layout lo{};
  fsparse_info ib{};
  const Tuning tb = append_tuning();
  fsparse_status st = assemble_impl(ii, jjB, ss, dt, len, m, nB, 0, FSPARSE_ORDERED, jcB,
                                    nB + 1, irB, prB, std::max<int64_t>(len, 1), slotB,
                                    ws2, ws_bytes - ml.head, nullptr, &ib, stream,
                                    fsp::kIdxI32, nullptr, nullptr, nullptr, true, &lo,
                                    &tb);
  if (st != FSPARSE_OK) return st;
  const int32_t* permB = at<int32_t>(ws2, lo.perm);
  const int32_t* segB = at<int32_t>(ws2, lo.seg);
  // every stored pair and every new pair fits: the merge is written in one
  // pass (the count is then exact in jcS[n])
  const int64_t bound = nnzA + ib.nnz;
  if (bound > cap) {
    if (info) info->nnz = bound;
    return FSPARSE_E_CAPACITY;
  }
  // lanes per column: about the rows a column holds on either side (a
  // power of two, 8 to 64); a block of 1024 threads then stages about 1024
  // rows a side, half its LDS, which leaves room for uneven columns
  const int64_t per = std::max<int64_t>(nnzA / std::max<int64_t>(nA, 1),
                                        ib.nnz / std::max<int64_t>(nB, 1)) + 1;
  int G = 8;
  while (G < 64 && G < per) G *= 2;
  constexpr int NT = 1024;
  const int64_t tiles = (n + NT / G - 1) / (NT / G);
  const fsp::MergeCols mc{(int32_t)nA, (int32_t)boff, (int32_t)nB};
  hipError_t e = launch(kAppend, stream, [&] {
    hipLaunchKernelGGL(fsp::k_zero, dim3(1), dim3(64), 0, stream, (uint32_t*)ctrl,
                       (int64_t)(sizeof(Ctrl) / 4));
    hipLaunchKernelGGL(fsp::k_zero, dim3(grid_for(2 * tiles + 2, 256, 4)), dim3(256), 0,
                       stream, at<uint32_t>(ws, ml.st), (int64_t)(2 * tiles + 2));
    if (n == 0) {
      hipLaunchKernelGGL(fsp::k_zero, dim3(1), dim3(64), 0, stream, (uint32_t*)jcS,
                         (int64_t)1);
      return;
    }
#define FSP_MERGE(VT)                                                                \
  hipLaunchKernelGGL((fsp::k_merge<VT, NT>), dim3((unsigned)tiles), dim3(NT), 0, stream,  \
                     jcA, irA, (const VT*)prA, mc, jcB, irB, (const VT*)prB,              \
                     segB, permB, (const VT*)ss, (int32_t)n, (int32_t)m, jcS, irS,        \
                     (VT*)prS, slot, mapB, at<uint64_t>(ws, ml.st), ctrl, G)
    if (dt == FSPARSE_F64)
      FSP_MERGE(double);
    else
      FSP_MERGE(float);
#undef FSP_MERGE
    if (slot && len > 0)
      hipLaunchKernelGGL(fsp::k_slot_gather, dim3(grid_for(len, 256, 16)), dim3(256), 0,
                         stream, slotB, len, mapB, slot + nnzA);
  });
  if (e != hipSuccess) return FSPARSE_E_HIP;
  int32_t* hnnz = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(h) + 256);
  HIPCHK(hipMemcpyAsync(h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hnnz, jcS + n, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (info) {
    info->nnz = *hnnz;
    info->nzmax = *hnnz;
  }
  if (h->err & (fsp::kErrRow | fsp::kErrCol)) return FSPARSE_E_INDEX;
  // columns far longer than the average: merge by re-assembling everything
  if (h->err & fsp::kErrRuns)
    return append_resort(jcA, irA, prA, nnzA, nA, ii, jj, ss, len, dt, m, n,
                         FSPARSE_ORDERED, jcS, jcS_cap, irS, prS, cap, slot, ws, ws_bytes,
                         nullptr, info, stream);
  return FSPARSE_OK;
}

fsparse_status fsparse_assemble_append(const int32_t* jcA, const int32_t* irA,
                                       const void* prA, int64_t nnzA, int64_t nA,
                                       const int32_t* ii, const int32_t* jj,
                                       const void* ss, int64_t len, fsparse_dtype dt,
                                       int64_t m, int64_t n, unsigned flags,
                                       int32_t* jcS, int64_t jcS_cap, int32_t* irS,
                                       void* prS, int64_t cap, int32_t* slot,
                                       void* ws, size_t ws_bytes,
                                       fsparse_plan** plan, fsparse_info* info,
                                       hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK) return FSPARSE_E_ARG;
  if (nnzA < 0 || len < 0 || nA < 0 || nnzA + len > kMaxI32 || m > kMaxI32 ||
      n > kMaxI32 || nA > kMaxI32)
    return FSPARSE_E_ARG;
  if (flags & ~(unsigned)(FSPARSE_ATOMIC | FSPARSE_DROP_ZEROS)) return FSPARSE_E_ARG;
  if ((flags & FSPARSE_DROP_ZEROS) && plan) return FSPARSE_E_ARG;
  if (!jcA || (nnzA > 0 && (!irA || !prA))) return FSPARSE_E_ARG;
  if (len > 0 && (!ii || !jj || !ss)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (plan) *plan = nullptr;
  // plain calls merge; a plan (whose values are the stored sums and the new
  // values) or dropped zeros take the whole re-assembly below
  if (!plan && !(flags & FSPARSE_DROP_ZEROS))
    return append_merge(jcA, irA, prA, nnzA, nA, ii, jj, ss, len, dt, m, n, jcS, jcS_cap,
                        irS, prS, cap, slot, ws, ws_bytes, info, stream);
  return append_resort(jcA, irA, prA, nnzA, nA, ii, jj, ss, len, dt, m, n, flags, jcS,
                       jcS_cap, irS, prS, cap, slot, ws, ws_bytes, plan, info, stream);
}

fsparse_status fsparse_assemble_reuse(fsparse_plan* plan, const void* ss,
                                      void* prS, unsigned flags,
                                      hipStream_t stream) {
  if (!plan) return FSPARSE_E_PLAN;
  // (re-assembly never waits: FSPARSE_NO_SYNC changes nothing here)
  if (flags & ~(unsigned)(FSPARSE_ATOMIC | FSPARSE_NO_SYNC)) return FSPARSE_E_ARG;
  if (plan->nnz == 0) return FSPARSE_OK;
  if (!ss || !prS) return FSPARSE_E_ARG;
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != plan->device) return FSPARSE_E_PLAN;
  if (flags & FSPARSE_ATOMIC) {
    if (!plan->slot) {
      if (!plan->islot || !plan->perm || !plan->seg || !plan->dnnz) return FSPARSE_E_PLAN;
      const int32_t* perm = plan->perm;
      const int32_t* seg = plan->seg;
      int32_t* islot = plan->islot;
      const int64_t* dnnz = plan->dnnz;
      const int64_t nb = plan->nnz >= 0 ? plan->nnz : plan->len;
      hipError_t e = launch(kReuse, stream, [&] {
        hipLaunchKernelGGL(fsp::k_slot_from_order, dim3(grid_for(nb, 256, 8)), dim3(256),
                           0, stream, perm, seg, dnnz, islot);
      });
      if (e != hipSuccess) return FSPARSE_E_HIP;
      plan->slot = islot;
    }
    return plan_reuse_atomic(plan, ss, prS, stream);
  }
  return plan_reuse_ordered(plan, ss, prS, stream);
}

fsparse_status fsparse_backward(const int32_t* slot, int64_t len,
                                const void* grad_prS, int64_t nnz,
                                fsparse_dtype dt, void* grad_ss,
                                hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK || len < 0 || nnz < 0 || len > kMaxI32)
    return FSPARSE_E_ARG;
  if (len == 0) return FSPARSE_OK;
  if (!slot || !grad_ss || (nnz > 0 && !grad_prS)) return FSPARSE_E_ARG;
  const int blk = tuning().rblock;
  hipError_t e = launch(kBackward, stream, [&] {
    if (dt == FSPARSE_F64)
      hipLaunchKernelGGL(fsp::k_backward<double>, dim3(grid_for(len, blk, 16)),
                         dim3(blk), 0, stream, slot, (const double*)grad_prS, len,
                         nnz, (double*)grad_ss);
    else
      hipLaunchKernelGGL(fsp::k_backward<float>, dim3(grid_for(len, blk, 16)),
                         dim3(blk), 0, stream, slot, (const float*)grad_prS, len,
                         nnz, (float*)grad_ss);
  });
  return e == hipSuccess ? FSPARSE_OK : FSPARSE_E_HIP;
}

fsparse_status fsparse_assemble_batched(
    int32_t nb, const int64_t* trip_off, const int32_t* ii, const int32_t* jj,
    const void* ss, fsparse_dtype dt, const int64_t* m, const int64_t* n,
    unsigned flags, int32_t* jcS, int64_t jcS_cap, int32_t* irS, void* prS,
    int64_t cap, int64_t* nnz_off, int32_t* slot, void* ws, size_t ws_bytes,
    fsparse_plan** plan, fsparse_info* info, hipStream_t stream) {
  if (check_dt(dt) != FSPARSE_OK || nb < 1 || !trip_off || !m || !n || !nnz_off)
    return FSPARSE_E_ARG;
  if (flags & ~(unsigned)FSPARSE_ATOMIC) return FSPARSE_E_ARG;
  if (trip_off[0] != 0) return FSPARSE_E_ARG;
  for (int b = 0; b < nb; ++b)
    if (trip_off[b + 1] < trip_off[b]) return FSPARSE_E_ARG;
  const int64_t L = trip_off[nb];
  if (L > kMaxI32) return FSPARSE_E_ARG;
  if (L > 0 && (!ii || !jj || !ss)) return FSPARSE_E_ARG;
  if (!jcS || !ws || cap < 0 || (cap > 0 && (!irS || !prS))) return FSPARSE_E_ARG;
  if (plan) *plan = nullptr;
  std::vector<int64_t> mm(m, m + nb), nn(n, n + nb), col(nb + 1, 0);
  bool need_dims = false;
  for (int b = 0; b < nb; ++b) {
    if (mm[b] > kMaxI32 || nn[b] > kMaxI32) return FSPARSE_E_ARG;
    need_dims |= (mm[b] < 0 || nn[b] < 0);
  }
  const Tuning tu = tuning();
  // worst-case layout for the dims pass: tables must fit before N is known
  if (ws_bytes < 4096) return FSPARSE_E_CAPACITY;
  if (need_dims && L > 0) {
    fsparse_status st = batched_dims(nb, trip_off, ii, jj, L, dt, tu, ws,
                                     ws_bytes, mm.data(), nn.data(), stream);
    if (st != FSPARSE_OK) return st;
  }
  for (int b = 0; b < nb; ++b) {
    if (mm[b] < 0) mm[b] = 0;
    if (nn[b] < 0) nn[b] = 0;
    col[b + 1] = col[b] + nn[b];
  }
  const int64_t N = col[nb];
  if (N > kMaxI32) return FSPARSE_E_ARG;
  if (info)
    for (int b = 0; b < nb; ++b) {
      info[b].m = mm[b];
      info[b].n = nn[b];
      info[b].nnz = 0;
      info[b].nzmax = 0;
    }
  if (jcS_cap < N + nb) return FSPARSE_E_CAPACITY;
  Layout lo = make_layout(L, N, nb, esize_of(dt), tu);
  if (ws_bytes < lo.total) return FSPARSE_E_CAPACITY;
  lo.mmax = 0;
  for (int b = 0; b < nb; ++b) lo.mmax = std::max(lo.mmax, mm[b]);
  std::vector<int32_t> m32(nb), n32(nb);
  for (int b = 0; b < nb; ++b) {
    m32[b] = (int32_t)mm[b];
    n32[b] = (int32_t)nn[b];
  }
  // the four tables lie back to back in ws (b_trip, b_col, b_m, b_n): one
  // copy from pinned memory laid out the same way, else four copies
  auto put_tables = [&](const Layout& l) -> hipError_t {
    const size_t span = l.b_n + 4 * (size_t)nb - l.b_trip;
    char* hp = static_cast<char*>(pinned());
    if (hp && span <= kPinnedBytes) {
      std::memcpy(hp + (l.b_trip - l.b_trip), trip_off, 8 * (size_t)(nb + 1));
      std::memcpy(hp + (l.b_col - l.b_trip), col.data(), 8 * (size_t)(nb + 1));
      std::memcpy(hp + (l.b_m - l.b_trip), m32.data(), 4 * (size_t)nb);
      std::memcpy(hp + (l.b_n - l.b_trip), n32.data(), 4 * (size_t)nb);
      return hipMemcpyAsync(at<char>(ws, l.b_trip), hp, span, hipMemcpyHostToDevice,
                            stream);
    }
    hipError_t r = hipMemcpyAsync(at<int64_t>(ws, l.b_trip), trip_off,
                                  8 * (size_t)(nb + 1), hipMemcpyHostToDevice, stream);
    if (r == hipSuccess)
      r = hipMemcpyAsync(at<int64_t>(ws, l.b_col), col.data(), 8 * (size_t)(nb + 1),
                         hipMemcpyHostToDevice, stream);
    if (r == hipSuccess)
      r = hipMemcpyAsync(at<int32_t>(ws, l.b_m), m32.data(), 4 * (size_t)nb,
                         hipMemcpyHostToDevice, stream);
    if (r == hipSuccess)
      r = hipMemcpyAsync(at<int32_t>(ws, l.b_n), n32.data(), 4 * (size_t)nb,
                         hipMemcpyHostToDevice, stream);
    return r;
  };
  HIPCHK(put_tables(lo));
  BatchDesc bd{at<int64_t>(ws, lo.b_trip), at<int64_t>(ws, lo.b_col),
               at<int32_t>(ws, lo.b_m), at<int32_t>(ws, lo.b_n), nb};
  const bool keep = plan != nullptr;
  int32_t* slot_used = slot ? slot : (keep ? at<int32_t>(ws, lo.islot) : nullptr);
  int32_t* jcg = nb > 1 ? at<int32_t>(ws, lo.jcg) : jcS;
  int64_t* dnnz = at<int64_t>(ws, lo.nnzoff);
  Ctrl* ctrl = at<Ctrl>(ws, lo.ctrl);
  hipError_t e;
  if (L == 0) {
    e = launch(kInit, stream, [&] {
      hipLaunchKernelGGL(fsp::k_zero, dim3(grid_for(N + nb, 256, 4)), dim3(256), 0,
                         stream, (uint32_t*)jcS, (int64_t)(N + nb));
    });
    if (e != hipSuccess) return FSPARSE_E_HIP;
    HIPCHK(hipStreamSynchronize(stream));
    for (int b = 0; b <= nb; ++b) nnz_off[b] = 0;
    if (keep) {
      fsparse_plan* pl = new (std::nothrow) fsparse_plan();
      if (!pl) return FSPARSE_E_ARG;
      pl->dt = dt;
      hipGetDevice(&pl->device);
      *plan = pl;
    }
    return FSPARSE_OK;
  }
  char* h = static_cast<char*>(pinned());
  if (!h || sizeof(Ctrl) + 8 * (size_t)(nb + 1) > kPinnedBytes) return FSPARSE_E_ARG;
  int mode = lo.g.mode;
  for (;;) {
    // the bin kernel's last block writes nnz and the error bits of the
    // earlier kernels into the pinned control block, and the column-pointer
    // kernel writes the matrices' offsets beside it: no copy back
    if (dt == FSPARSE_F64)
      e = run_pipeline<double, true>(ii, jj, (const double*)ss, L, 0, 0, bd, N, lo,
                                     tu, ws, jcg, irS, (double*)prS, cap, slot_used,
                                     keep, mode, stream, reinterpret_cast<Ctrl*>(h));
    else
      e = run_pipeline<float, true>(ii, jj, (const float*)ss, L, 0, 0, bd, N, lo, tu,
                                    ws, jcg, irS, (float*)prS, cap, slot_used, keep,
                                    mode, stream, reinterpret_cast<Ctrl*>(h));
    if (e != hipSuccess) return FSPARSE_E_HIP;
    if (keep && launch_reuse_tiles(ws, lo, L, stream) != hipSuccess) return FSPARSE_E_HIP;
    if (nb > 1) {
      int64_t* hoff = reinterpret_cast<int64_t*>(h + sizeof(Ctrl));
      e = launch(kBatchedJcs, stream, [&] {
        hipLaunchKernelGGL(fsp::k_batched_jcs, dim3(grid_for((N + nb + 31) / 32, 256, 8)),
                           dim3(256), 0, stream, jcg, at<int64_t>(ws, lo.b_col), nb,
                           (int64_t)(N + nb), jcS, dnnz, hoff);
      });
      if (e != hipSuccess) return FSPARSE_E_HIP;
    }
    HIPCHK(hipStreamSynchronize(stream));
    if ((reinterpret_cast<const Ctrl*>(h)->err & fsp::kErrSlot) && mode == kSlot) {
      // a full fixed-capacity bin: count first, in narrower bins, and redo
      const int64_t mmax = lo.mmax;
      Layout l2 = make_layout(L, N, nb, esize_of(dt), tu, true);
      if (ws_bytes < l2.total) return FSPARSE_E_CAPACITY;
      // the batch tables sit at the same offsets only if the bin regions
      // kept their size: copy them again
      l2.mmax = mmax;
      lo = l2;
      HIPCHK(put_tables(lo));
      bd = BatchDesc{at<int64_t>(ws, lo.b_trip), at<int64_t>(ws, lo.b_col),
                     at<int32_t>(ws, lo.b_m), at<int32_t>(ws, lo.b_n), nb};
      slot_used = slot ? slot : (keep ? at<int32_t>(ws, lo.islot) : nullptr);
      jcg = nb > 1 ? at<int32_t>(ws, lo.jcg) : jcS;
      dnnz = at<int64_t>(ws, lo.nnzoff);
      ctrl = at<Ctrl>(ws, lo.ctrl);
      mode = lo.g.mode;
      continue;
    }
    break;
  }
  const Ctrl* hc = reinterpret_cast<const Ctrl*>(h);
  const int64_t nnz = hc->nnz;
  if (nb > 1) {
    std::memcpy(nnz_off, h + sizeof(Ctrl), 8 * (size_t)(nb + 1));
  } else {
    nnz_off[0] = 0;
    nnz_off[1] = nnz;
  }
  if (info)
    for (int b = 0; b < nb; ++b) {
      info[b].nnz = nnz_off[b + 1] - nnz_off[b];
      info[b].nzmax = info[b].nnz;
    }
  if (hc->err & (fsp::kErrCol | fsp::kErrRow)) return FSPARSE_E_INDEX;
  // (an overflow flagged after the last bin shows as nnz beyond the capacity)
  if ((hc->err & fsp::kErrCap) || nnz > cap) return FSPARSE_E_CAPACITY;
  if (flags & FSPARSE_ATOMIC) {
    if (!slot_used) return FSPARSE_E_ARG;
    hipError_t ea = dt == FSPARSE_F64
        ? launch_atomic_values<double>(slot_used, ss, L, prS, nnz, tu.rblock, stream)
        : launch_atomic_values<float>(slot_used, ss, L, prS, nnz, tu.rblock, stream);
    if (ea != hipSuccess) return FSPARSE_E_HIP;
  }
  if (keep) {
    fsparse_plan* pl = new (std::nothrow) fsparse_plan();
    if (!pl) return FSPARSE_E_ARG;
    pl->len = L;
    pl->nnz = nnz;
    pl->dnnz = &at<Ctrl>(ws, lo.ctrl)->nnz;
    pl->dt = dt;
    hipGetDevice(&pl->device);
    pl->perm = at<int32_t>(ws, lo.perm);
    pl->seg = at<int32_t>(ws, lo.seg);
    pl->slot = slot_used;
    pl->rtile = at<int32_t>(ws, lo.rtile);
    pl->ntiles = (L + kReuseTP - 1) / kReuseTP;
    pl->rblock = tu.rblock;
    *plan = pl;
  }
  return FSPARSE_OK;
}

fsparse_status fsparse_dims_batched(int32_t nb, const int64_t* trip_off,
                                    const int32_t* ii, const int32_t* jj,
                                    int64_t* m, int64_t* n, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  if (nb < 1 || !trip_off || !m || !n || !ws || trip_off[0] != 0)
    return FSPARSE_E_ARG;
  for (int b = 0; b < nb; ++b)
    if (trip_off[b + 1] < trip_off[b]) return FSPARSE_E_ARG;
  const int64_t L = trip_off[nb];
  if (L > kMaxI32 || (L > 0 && (!ii || !jj))) return FSPARSE_E_ARG;
  for (int b = 0; b < nb; ++b) {
    m[b] = -1;
    n[b] = -1;
  }
  if (L > 0) {
    // no values here: the fp32 layout, the smaller one, fits any workspace
    // sized for nb matrices
    fsparse_status st = batched_dims(nb, trip_off, ii, jj, L, FSPARSE_F32,
                                     tuning(), ws, ws_bytes, m, n, stream);
    if (st != FSPARSE_OK) return st;
  }
  for (int b = 0; b < nb; ++b) {
    if (m[b] < 0) m[b] = 0;
    if (n[b] < 0) n[b] = 0;
  }
  return FSPARSE_OK;
}

fsparse_status fsparse_assemble_status(const void* ws, fsparse_info* info,
                                       hipStream_t stream) {
  if (!ws) return FSPARSE_E_ARG;
  Ctrl c{};
  HIPCHK(hipMemcpyAsync(&c, ws, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (info) info->nnz = c.nnz;
  if (c.err & (fsp::kErrCol | fsp::kErrRow)) return FSPARSE_E_INDEX;
  if (c.err & fsp::kErrCap) return FSPARSE_E_CAPACITY;
  return FSPARSE_OK;
}

fsparse_status fsparse_indices_i32(const void* src, int32_t src_type, int64_t len,
                                   int32_t* dst, hipStream_t stream) {
  if (len < 0 || (len > 0 && (!src || !dst))) return FSPARSE_E_ARG;
  if (src_type != FSPARSE_IDX_I64 && src_type != FSPARSE_IDX_U32 &&
      src_type != FSPARSE_IDX_U64)
    return FSPARSE_E_ARG;
  if (len == 0) return FSPARSE_OK;
  hipError_t e = launch(kInit, stream, [&] {
    const dim3 g(grid_for(len, 256, 16)), b(256);
    if (src_type == FSPARSE_IDX_I64)
      hipLaunchKernelGGL(fsp::k_narrow_index<int64_t>, g, b, 0, stream,
                         (const int64_t*)src, len, dst);
    else if (src_type == FSPARSE_IDX_U32)
      hipLaunchKernelGGL(fsp::k_narrow_index<uint32_t>, g, b, 0, stream,
                         (const uint32_t*)src, len, dst);
    else
      hipLaunchKernelGGL(fsp::k_narrow_index<uint64_t>, g, b, 0, stream,
                         (const uint64_t*)src, len, dst);
  });
  return e == hipSuccess ? FSPARSE_OK : FSPARSE_E_HIP;
}

void fsparse_plan_destroy(fsparse_plan* plan) {
  if (!plan) return;
  // graph launches may still be queued: wait for the latest one first
  if (plan->done) {
    (void)hipEventSynchronize(plan->done);
    (void)hipEventDestroy(plan->done);
  }
  if (plan->x_ord) (void)hipGraphExecDestroy(plan->x_ord);
  if (plan->g_ord) (void)hipGraphDestroy(plan->g_ord);
  if (plan->x_at) (void)hipGraphExecDestroy(plan->x_at);
  if (plan->g_at) (void)hipGraphDestroy(plan->g_at);
  delete plan;
}

fsparse_status fsparse_plan_query(const fsparse_plan* plan, int64_t* len,
                                  int64_t* nnz, int32_t* dtype) {
  if (!plan) return FSPARSE_E_PLAN;
  if (len) *len = plan->len;
  if (nnz) {
    *nnz = plan->nnz;
    if (plan->nnz < 0 && plan->dnnz) {
      // a plan made without a wait: read the count now (a blocking copy)
      int64_t v = 0;
      if (hipMemcpy(&v, plan->dnnz, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
        return FSPARSE_E_HIP;
      *nnz = v;
    }
  }
  if (dtype) *dtype = (int32_t)plan->dt;
  return FSPARSE_OK;
}

fsparse_status fsparse_set_tuning(const fsparse_tuning* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!t) {
    g_tune = Tuning{};
    return FSPARSE_OK;
  }
  Tuning n = g_tune;
  if (t->chunk_cap) {
    const int c = t->chunk_cap;
    if (c < 2 || c > 4096 || (c & (c - 1))) return FSPARSE_E_ARG;
    n.cap = c;
  }
  if (t->stream_block) {
    const int b = t->stream_block;
    if (b < 64 || b > 1024 || (b % 64)) return FSPARSE_E_ARG;
    n.sblock = b;
  }
  if (t->stream_items) {
    if (t->stream_items < 1 || t->stream_items > 32) return FSPARSE_E_ARG;
    n.sitems = t->stream_items;
  }
  if (t->reuse_block) {
    const int b = t->reuse_block;
    if (b < 64 || b > 1024 || (b % 64)) return FSPARSE_E_ARG;
    n.rblock = b;
  }
  if (t->chunk_block) {
    const int b = t->chunk_block;
    if (b != 256 && b != 512 && b != 1024) return FSPARSE_E_ARG;
    n.cblock = b;
  }
  if (t->bin_mode < 0 || t->bin_mode > 3) return FSPARSE_E_ARG;
  n.bmode = t->bin_mode;
  if (t->slot_values < 0 || t->slot_values > 2) return FSPARSE_E_ARG;
  if (t->slot_values) n.keys = t->slot_values == 2 ? 1 : 0;
  g_tune = n;
  return FSPARSE_OK;
}

fsparse_status fsparse_get_tuning(fsparse_tuning* t) {
  if (!t) return FSPARSE_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  t->chunk_cap = g_tune.cap;
  t->stream_block = g_tune.sblock;
  t->stream_items = g_tune.sitems;
  t->reuse_block = g_tune.rblock;
  t->chunk_block = g_tune.cblock;
  t->bin_mode = g_tune.bmode;
  t->slot_values = g_tune.keys ? 2 : 1;
  return FSPARSE_OK;
}

fsparse_status fsparse_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_timing = on != 0;
  return FSPARSE_OK;
}

fsparse_status fsparse_timing_select(uint32_t stage_mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_stage_mask = stage_mask;
  return FSPARSE_OK;
}

int fsparse_timing_read(double* ms, int64_t* launches, int max_stages) {
  std::vector<Rec> recs;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    recs.swap(g_recs);
  }
  for (const Rec& r : recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess &&
        hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_mu);
      g_ms[r.stage] += t;
      g_cnt[r.stage] += 1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (int s = 0; s < kNumStages && s < max_stages; ++s) {
    if (ms) ms[s] = g_ms[s];
    if (launches) launches[s] = g_cnt[s];
    g_ms[s] = 0;
    g_cnt[s] = 0;
  }
  return kNumStages;
}

const char* fsparse_stage_name(int stage) {
  return (stage >= 0 && stage < kNumStages) ? kStageNames[stage] : "";
}

fsparse_status fsparse_stream_copy(const void* src, void* dst, size_t bytes,
                                   hipStream_t stream) {
  if (!src || !dst || (bytes % 16) || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
    return FSPARSE_E_ARG;
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return FSPARSE_OK;
  hipError_t e = launch(kCopy, stream, [&] {
    hipLaunchKernelGGL(fsp::k_copy16, dim3(grid_for(n16, 256, 16)), dim3(256), 0,
                       stream, (const uint4*)src, (uint4*)dst, n16);
  });
  return e == hipSuccess ? FSPARSE_OK : FSPARSE_E_HIP;
}

}  // extern "C"
