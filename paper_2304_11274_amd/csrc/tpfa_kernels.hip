// HIP kernels of the ensemble (persistent and grouped schedules), the
// hydrostatic reference column and the FP32 offsets, and the dispatch of
// single-grid launches to the per-precision translation units. The tile
// body they all share, and its design, is in tpfa_tile.h.
#include <algorithm>
#include <limits>
#include <mutex>
#include <type_traits>

#include "tpfa_tile.h"

namespace tpfa {

// ----------------------------------------------------------------------------
// Ensemble kernels. The work list (one item per tile and z chunk of a model,
// neighbouring tiles next to each other) is cut into kXcds contiguous bands,
// one per XCD: workgroup ids go to the XCDs in turn, so workgroup b runs on
// XCD b % kXcds, and a band's tiles share halo cells and the output lines at
// their common edges in that XCD's L2.
// Persistent schedule: 256-thread workgroups take items from their own band's
// device counter, then from the other bands once it is drained. A one-
// workgroup kernel launched before it (a kernel node, not a memset node, in
// the batch's graph) zeroes the counters.
// ----------------------------------------------------------------------------
constexpr int kPersistThreads = 256;
constexpr int kMixedTiles = 3;  // TILE value of the kernel that switches shape per model

// Band x of a list of n items: [start, start + len).
__device__ __forceinline__ void band_range(uint32_t n, uint32_t x, uint32_t &start,
                                           uint32_t &len) {
  const uint32_t q = n / kXcds, rem = n % kXcds;
  start = x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
  len = q + (x < rem ? 1u : 0u);
}

// Workgroups of a launch of `grid` workgroups that run on XCD x.
__device__ __forceinline__ uint32_t band_workgroups(uint32_t grid, uint32_t x) {
  return (grid + kXcds - 1 - x) / kXcds;
}

// Next item of a persistent workgroup (thread 0 only): from band `band`
// while it lasts, then from the following bands in turn; `left` counts the
// bands not yet found drained. Returns n once every band is drained. The
// first band_workgroups items of each band are the static first items of its
// workgroups, so a band's counter hands out the items after those.
__device__ __forceinline__ uint32_t claim_item(unsigned int *counter, uint32_t n,
                                               uint32_t &band, int &left) {
  while (left > 0) {
    uint32_t start, len;
    band_range(n, band, start, len);
    const uint32_t i =
        atomicAdd(&counter[band * kCounterStride], 1u) + band_workgroups(gridDim.x, band);
    if (i < len) return start + i;
    band = (band + 1) % kXcds;
    --left;
  }
  return n;
}

template <class S, int MODE, int TILE>
constexpr int persist_lds_bytes() {
  constexpr int a0 = tile_lds_bytes<S, MODE, 64, 4>();
  constexpr int a1 = tile_lds_bytes<S, MODE, 32, 8>();
  constexpr int a2 = tile_lds_bytes<S, MODE, 16, 16>();
  constexpr int af = tile_lds_bytes<S, MODE, 0, 0>();
  constexpr int m01 = a0 > a1 ? a0 : a1, m012 = m01 > a2 ? m01 : a2;
  return TILE == 0 ? a0
                   : TILE == 1 ? a1
                               : TILE == 2 ? a2
                                           : TILE == kFitTile ? af : (m012 > af ? m012 : af);
}

// One work item of an ensemble. TILE = 0, 1, 2, kFitTile: every model uses that
// 256-thread tile (one code path, fewer registers); TILE = kMixedTiles: the
// tile is read per model.
template <class S, int MODE, int TILE>
__device__ __forceinline__ void march_item(const Args &m, const WorkItem &w, char *smem, int tid) {
  if constexpr (TILE == 0) {
    march_tile<S, MODE, 64, 4>(m, w.bx, w.by, w.kb, smem, tid);
  } else if constexpr (TILE == 1) {
    march_tile<S, MODE, 32, 8>(m, w.bx, w.by, w.kb, smem, tid);
  } else if constexpr (TILE == 2) {
    march_tile<S, MODE, 16, 16>(m, w.bx, w.by, w.kb, smem, tid);
  } else if constexpr (TILE == kFitTile) {
    march_tile<S, MODE, 0, 0>(m, w.bx, w.by, w.kb, smem, tid);
  } else {
    switch (m.tile) {
      case 0: march_tile<S, MODE, 64, 4>(m, w.bx, w.by, w.kb, smem, tid); break;
      case 1: march_tile<S, MODE, 32, 8>(m, w.bx, w.by, w.kb, smem, tid); break;
      case kFitTile: march_tile<S, MODE, 0, 0>(m, w.bx, w.by, w.kb, smem, tid); break;
      default: march_tile<S, MODE, 16, 16>(m, w.bx, w.by, w.kb, smem, tid); break;
    }
  }
}

// One item; MODE carries the store kind (MODE_PLAIN: ordinary stores). The
// FP32 ensemble writes with ordinary stores unless every member's output rows
// are written in whole lines (padded rows with their padding writable): its
// models mostly have rows off 128-byte lines, where ordinary stores measured
// much faster (the partial lines of neighbouring tiles meet in L2), and a
// per-model choice (both tile bodies in one kernel) cost more registers than
// it saved. With whole-line rows non-temporal stores gained 2%.
template <class S, int MODE, int TILE>
__device__ __forceinline__ void run_item(const Args &m, const WorkItem &w, char *smem, int tid) {
  march_item<S, MODE, TILE>(m, w, smem, tid);
}

// Zeroes the band counters of a persistent launch (stream-ordered before it).
__global__ void reset_counters_kernel(unsigned int *counter) {
  if (threadIdx.x < kXcds) atomicExch(&counter[threadIdx.x * kCounterStride], 0u);
}

// The persistent kernel; TILE as for march_item. Workgroup b starts with
// item b / kXcds of its XCD's band (no claim), the item the grouped schedule
// would give it; after each item, thread 0 claims the next one. Items then
// start in claim order, as the hardware dispatcher starts the grouped
// schedule's workgroups, so neighbouring items run at the same time and share
// their halo and edge lines in L2. (Claiming the next item when the current
// one starts runs it one item's time after the items claimed beside it: on
// the 64-model ensemble 41% more DRAM reads and 5% more time than the grouped
// schedule.) The claim state (band, bands left) and the claimed index live
// in LDS, so no register is held across the tile body (those would cost the
// tile registers, hence occupancy). A workgroup ends without a memory fence:
// the counters are zeroed by the next launch's reset kernel. (Ending with an
// agent-scope fence, which writes back and invalidates the XCD's L2, cost
// 8-11% on that ensemble.)
template <class S, int MODE, int TILE>
__global__ void __launch_bounds__(kPersistThreads)
    persistent_kernel(const Args *__restrict__ models, const WorkItem *__restrict__ items,
                      int64_t n_items, unsigned int *counter) {
  __shared__ __attribute__((aligned(16))) char smem[persist_lds_bytes<S, MODE, TILE>()];
  __shared__ unsigned int s_next[2];  // claimed items, alternating per iteration
  __shared__ unsigned int s_band;
  __shared__ int s_left;
  const uint32_t n = (uint32_t)n_items;
  if (threadIdx.x == 0) {
    uint32_t band = blockIdx.x % kXcds;  // the band of this workgroup's XCD
    int left = kXcds;
    uint32_t start, len;
    band_range(n, band, start, len);
    const uint32_t l = blockIdx.x / kXcds;
    s_next[0] = l < len ? start + l : claim_item(counter, n, band, left);
    s_band = band;
    s_left = left;
  }
  __syncthreads();
  // the item index is uniform: keep it (and everything read through it) in
  // scalar registers
  unsigned int it = __builtin_amdgcn_readfirstlane(s_next[0]);
  for (int q = 1;; q ^= 1) {
    if (it >= n) break;
    const WorkItem w = items[it];
    const Args m = models[__builtin_amdgcn_readfirstlane(w.model)];
    // the thread index passes an empty asm per item: otherwise the compiler
    // hoists the tile's index arithmetic out of the item loop and keeps it
    // live across it (six more VGPRs in FP32, one wave per SIMD fewer)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    run_item<S, MODE, TILE>(m, w, smem, tid);
    // the slot s_next[q] was last read before the previous barrier
    if (threadIdx.x == 0) {
      uint32_t band = s_band;
      int left = s_left;
      s_next[q] = claim_item(counter, n, band, left);
      s_band = band;
      s_left = left;
    }
    __syncthreads();  // the tile's LDS is reused by the next item; s_next[q] is visible
    it = __builtin_amdgcn_readfirstlane(s_next[q]);
  }
}

// ----------------------------------------------------------------------------
// Small helpers: hydrostatic reference column and FP32 offsets.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double rho_ref(double p, double rho0, double cf, double p0) {
  return rho0 * exp(cf * (p - p0));
}

// pref[k+1] solves x - pref[k] = (rho(pref[k]) + rho(x))/2 * gk * dz; Newton per
// level until the iterate stops changing (sequential in k: one lane).
__global__ void hydrostatic_kernel(int nz, double G, double rho0, double cf, double p0,
                                   double p_top, double *pref) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double pk = p_top;
  pref[0] = pk;
  for (int k = 0; k + 1 < nz; ++k) {
    const double rk = rho_ref(pk, rho0, cf, p0);
    double x = pk + rk * G;
    for (int it = 0; it < 100; ++it) {
      const double rx = rho_ref(x, rho0, cf, p0);
      const double res = x - pk - 0.5 * (rk + rx) * G;
      const double der = 1.0 - 0.5 * cf * rx * G;
      const double xn = x - res / der;
      if (xn == x) break;
      x = xn;
    }
    pref[k + 1] = x;
    pk = x;
  }
}

// One thread per cell c = i + nx * row (row = j + ny * k), stored at
// i + ldx * row; padding cells are not touched.
__global__ void offset_kernel(int64_t nx, int64_t ldx, int64_t ny, int64_t n,
                              const double *__restrict__ p, const double *__restrict__ pref,
                              float *__restrict__ dp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    const int64_t row = c / nx, idx = c - row * nx + row * ldx;
    dp[idx] = (float)(p[idx] - pref[row / ny]);
  }
}

// ----------------------------------------------------------------------------
// Allocation-free ensemble run. The model table (Args of each model) and the
// first work item of each model live in `scratch`, a file-scope device array
// of fixed size: each GPU the library runs on holds its own copy until the
// process ends, and every call on that GPU shares it (calls that overlap on
// one GPU race). Upload launches write the table from their kernel arguments
// (so nothing is allocated, copied from host memory or set by a memset node);
// the grouped ensemble schedule then runs one workgroup per work item, which
// it decodes itself: the model by binary search over the first items, tile
// and z chunk in the natural order of a batch's work list (z chunk, tile row,
// tile), so the results are those of the batch.
// ----------------------------------------------------------------------------
constexpr size_t kScratchTable = (size_t)kStaticModels * sizeof(Args);
constexpr size_t kScratchBytes = kScratchTable + (size_t)(kStaticModels + 1) * sizeof(int64_t);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static_assert(sizeof(UploadBlock) <= 4096, "the arguments of one upload launch");
static_assert(sizeof(Args) % 8 == 0, "the table is copied in 8-byte words");

__global__ void __launch_bounds__(256) upload_kernel(const UploadBlock blk, unsigned char *scr) {
  const uint64_t *src = reinterpret_cast<const uint64_t *>(&blk.a[0]);
  uint64_t *dst = reinterpret_cast<uint64_t *>(scr) + (size_t)blk.first * (sizeof(Args) / 8);
  const int words = blk.count * (int)(sizeof(Args) / 8);
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  int64_t *item0 = reinterpret_cast<int64_t *>(scr + kScratchTable);
  if (threadIdx.x < (unsigned)blk.count) item0[blk.first + threadIdx.x] = blk.item0[threadIdx.x];
}

template <class S, int MODE, int TILE>
__global__ void __launch_bounds__(kPersistThreads)
    static_grouped_kernel(const unsigned char *__restrict__ scr, int n_models) {
  __shared__ __attribute__((aligned(16))) char smem[persist_lds_bytes<S, MODE, TILE>()];
  const Args *models = reinterpret_cast<const Args *>(scr);
  const int64_t *item0 = reinterpret_cast<const int64_t *>(scr + kScratchTable);
  // workgroup b is item l = b / kXcds of band b % kXcds, as in grouped_kernel
  uint32_t start, len;
  band_range(gridDim.x, blockIdx.x % kXcds, start, len);
  const int64_t t = (int64_t)start + blockIdx.x / kXcds;
  // the model: the last one whose first item is at most t
  int lo = 0, hi = n_models - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (item0[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const Args m = models[lo];
  const uint32_t l = (uint32_t)(t - item0[lo]);
  const uint32_t ntx = (uint32_t)m.ntx, nty = (uint32_t)m.nty;
  const uint32_t r1 = l / ntx, bz = r1 / nty;
  WorkItem w;
  w.model = lo;
  w.bx = (int)(l - r1 * ntx);
  w.by = (int)(r1 - bz * nty);
  w.kb = (int)bz * m.kz_chunk;
  run_item<S, MODE, TILE>(m, w, smem, threadIdx.x);
}

// This GPU's address of `scratch`, resolved once per device with that device
// current (each GPU holds its own copy; the array's name is not a device
// address in host code).
constexpr int kMaxDevices = 64;
static void *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

hipError_t static_scratch(void **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return hipSuccess;
}

hipError_t launch_upload(const UploadBlock &blk, void *scr, hipStream_t st) {
  upload_kernel<<<1, 256, 0, st>>>(blk, static_cast<unsigned char *>(scr));
  return hipGetLastError();
}

template <class S, int MODE>
static const void *static_fn(int tiles) {
  switch (tiles) {
    case 0: return reinterpret_cast<const void *>(&static_grouped_kernel<S, MODE, 0>);
    case 1: return reinterpret_cast<const void *>(&static_grouped_kernel<S, MODE, 1>);
    case 2: return reinterpret_cast<const void *>(&static_grouped_kernel<S, MODE, 2>);
    case kFitTile: return reinterpret_cast<const void *>(&static_grouped_kernel<S, MODE, kFitTile>);
    default: return reinterpret_cast<const void *>(&static_grouped_kernel<S, MODE, kMixedTiles>);
  }
}

static const void *static_ptr(tpfa_precision_t prec, int mode, int tiles) {
  const bool res = mode_kind(mode) == MODE_RESIDUAL;
  if (prec == TPFA_FP64)
    return res ? static_fn<double, MODE_RESIDUAL>(tiles) : static_fn<double, MODE_JACOBIAN>(tiles);
  if (has_plain_stores(mode))
    return res ? static_fn<float, MODE_RESIDUAL | MODE_PLAIN>(tiles)
               : static_fn<float, MODE_JACOBIAN | MODE_PLAIN>(tiles);
  return res ? static_fn<float, MODE_RESIDUAL>(tiles) : static_fn<float, MODE_JACOBIAN>(tiles);
}

hipError_t launch_static_grouped(tpfa_precision_t prec, int mode, int tiles, void *scr,
                                 int n_models, int64_t n_items, hipStream_t st) {
  const void *fn = static_ptr(prec, mode, tiles);
  const unsigned char *p = static_cast<const unsigned char *>(scr);
  void *args[] = {(void *)&p, (void *)&n_models};
  return hipLaunchKernel(fn, dim3((unsigned)n_items), dim3(kPersistThreads), args, 0, st);
}

// ----------------------------------------------------------------------------
// Bandwidth probe: the memory traffic of the Jacobian kernels without their
// arithmetic and without their halo, in the access pattern that measured
// fastest for it on MI355X among tile marches (64 x 8 and 128 x 8 column
// blocks, one or two cells per lane) and grid-stride loops (one or two cells
// per lane, 8k or 32k workgroups). Each 512-thread workgroup owns a block of
// columns and marches it through a chunk of 32 planes; per plane each lane
// reads p, k and the seal bytes of its cells and writes eight outputs,
// out[q][c] = p[c] + (q + seal[c]) k[c] (so that no load is dead), with
// non-temporal stores. The eight outputs go to eight planes (128 x 8 blocks,
// two consecutive x cells per lane: 16-byte FP64 accesses; rows of odd pitch
// take one cell per access), or to the runs of the sliced r + J layout
// (`slices` > 0: slice i / 64 of row j holds eight runs of 64 cells; 64 x 8
// blocks, one cell per lane, which measured 4% faster there than two).
// ----------------------------------------------------------------------------
constexpr int kProbeTx = 128, kProbeTy = 8, kProbeChunk = 32;

template <class S>
using vec2_t = S __attribute__((ext_vector_type(2)));

// CELLS x cells per lane: 64 CELLS x 8 column blocks of 512 lanes
template <class S, int CELLS, bool PAIR>
__global__ void __launch_bounds__(kProbeTx / 2 * kProbeTy)
    stream_probe_kernel(int nx, int ny, int nz, int ldx, int ntx, int nty, int slices,
                        const S *__restrict__ p, const S *__restrict__ k,
                        const uint8_t *__restrict__ seal, S *__restrict__ out) {
  const uint32_t b = blockIdx.x, r1 = b / (uint32_t)ntx, r2 = r1 / (uint32_t)nty;
  const int lanes = kProbeTx / 2;
  const int i = (int)(b - r1 * ntx) * lanes * CELLS + CELLS * (int)(threadIdx.x % lanes);
  const int j = (int)(r1 - r2 * nty) * kProbeTy + (int)(threadIdx.x / lanes);
  if (i >= nx || j >= ny) return;
  const bool two = CELLS == 2 && i + 1 < nx;
  const int kb = (int)r2 * kProbeChunk, ke = min(kb + kProbeChunk, nz);
  const size_t plane = (size_t)ldx * ny;
  // output: plane stride, run stride and the cell's offset in its plane
  const size_t oplane = slices ? (size_t)ny * slices * 512 : plane;
  const size_t nc = slices ? 64 : plane * nz;
  size_t c = (size_t)j * ldx + i + (size_t)kb * plane;
  size_t o = (slices ? ((size_t)j * slices + (i >> 6)) * 512 + (i & 63) : (size_t)j * ldx + i) +
             (size_t)kb * oplane;
#pragma unroll 2
  for (int kk = kb; kk < ke; ++kk, c += plane, o += oplane) {
    if (PAIR && two) {
      const vec2_t<S> pc = *(const vec2_t<S> *)(p + c), kc = *(const vec2_t<S> *)(k + c);
      const uint32_t sc = *(const uint16_t *)(seal + c);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        vec2_t<S> v;
        v.x = pc.x + S(q + (int)(sc & 255u)) * kc.x;
        v.y = pc.y + S(q + (int)(sc >> 8)) * kc.y;
        __builtin_nontemporal_store(v, (gptr<vec2_t<S>>)(out + q * nc + o));
      }
    } else {
#pragma unroll
      for (int e = 0; e < CELLS; ++e) {
        if (e == 1 && !two) break;
        const S pc = p[c + e], kc = k[c + e];
        const int sc = seal[c + e];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          __builtin_nontemporal_store(pc + S(q + sc) * kc, (gptr<S>)(out + q * nc + o + e));
      }
    }
  }
}

hipError_t launch_stream_probe(tpfa_precision_t prec, const tpfa_grid_t &g, const void *p,
                               const void *k, const uint8_t *seal, void *out, bool sliced,
                               hipStream_t st) {
  // planes: two cells per lane; sliced: one (each lane's eight stores then
  // fall in eight whole 64-cell runs of one slice)
  const int slices = sliced ? (int)((g.nx + 63) / 64) : 0;
  const int64_t tx = sliced ? kProbeTx / 2 : kProbeTx;
  const int ntx = (int)((g.nx + tx - 1) / tx);
  const int nty = (int)((g.ny + kProbeTy - 1) / kProbeTy);
  const int64_t nzc = (g.nz + kProbeChunk - 1) / kProbeChunk;
  const int64_t blocks = (int64_t)ntx * nty * nzc;
  if (blocks > (int64_t)std::numeric_limits<uint32_t>::max()) return hipErrorInvalidValue;
  const int ldx = (int)(g.ldx ? g.ldx : g.nx);
  const size_t elem = prec == TPFA_FP64 ? 8 : 4;
  // paired accesses need every pair of cells (even offset) aligned to 2 elements
  bool pair = ldx % 2 == 0 && reinterpret_cast<uintptr_t>(seal) % 2 == 0;
  for (const void *q : {p, k, (const void *)out})
    if (reinterpret_cast<uintptr_t>(q) % (2 * elem) != 0) pair = false;
  const dim3 grid((unsigned)blocks), block(kProbeTx / 2 * kProbeTy);
  const int nx = (int)g.nx, ny = (int)g.ny, nz = (int)g.nz;
  auto run = [&](const auto *pp, const auto *kk, auto *oo) {
    using S = std::remove_cv_t<std::remove_pointer_t<decltype(oo)>>;
    if (sliced)
      stream_probe_kernel<S, 1, false>
          <<<grid, block, 0, st>>>(nx, ny, nz, ldx, ntx, nty, slices, pp, kk, seal, oo);
    else if (pair)
      stream_probe_kernel<S, 2, true>
          <<<grid, block, 0, st>>>(nx, ny, nz, ldx, ntx, nty, slices, pp, kk, seal, oo);
    else
      stream_probe_kernel<S, 2, false>
          <<<grid, block, 0, st>>>(nx, ny, nz, ldx, ntx, nty, slices, pp, kk, seal, oo);
  };
  if (prec == TPFA_FP64)
    run(static_cast<const double *>(p), static_cast<const double *>(k), static_cast<double *>(out));
  else
    run(static_cast<const float *>(p), static_cast<const float *>(k), static_cast<float *>(out));
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Host launchers
// ----------------------------------------------------------------------------
hipError_t launch_march(tpfa_precision_t prec, Mode mode, int tile, const Args &a,
                        hipStream_t st) {
  if (a.nblocks <= 0) return hipSuccess;
  const int kind = mode_kind(mode);
  const int form = mode & (MODE_TRANS | MODE_K3 | MODE_WITH_R);
  if (prec == TPFA_FP64) return launch_march_f64(kind, form, tile, a, st);
  return a.plain ? launch_march_f32_plain(kind, form, tile, a, st)
                 : launch_march_f32(kind, form, tile, a, st);
}

// Residency of the single-grid kernels, from the runtime's occupancy query on
// the first use of each kernel (cached: the library runs on one device type).
bool march_residency(tpfa_precision_t prec, int mode, int tile, int &per_cu, int &cus) {
  static std::mutex mu;
  static int cache[2][4][8][kNumTiles];  // 0 unknown, -1 no answer, else workgroups per CU
  static int cu_count = 0;
  const int kind = mode_kind(mode);
  const int form = has_trans(mode) ? 1 : has_k3(mode) ? 2 : has_with_r(mode) ? 3 : 0;
  if (tile < 0 || tile >= kNumTiles) return false;
  std::lock_guard<std::mutex> lock(mu);
  int &slot = cache[prec == TPFA_FP64 ? 0 : 1][form][kind][tile];
  if (slot == 0) {
    const int fl = mode & (MODE_TRANS | MODE_K3 | MODE_WITH_R);
    const void *fn = prec == TPFA_FP64 ? march_kernel_f64(kind, fl, tile)
                                       : march_kernel_f32(kind, fl, tile);
    int dev = 0, n = 0, c = 0;
    if (fn && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kTiles[tile].threads, 0) ==
            hipSuccess &&
        n > 0 && c > 0) {
      // The runtime's answer counts LDS at byte granularity: for a tile of
      // 26.9 KB of LDS it said 6 workgroups per CU where 5 ran (a launch of 6
      // per CU took two rounds). Cap it by the CU's LDS in 2 KB granules.
      hipFuncAttributes at{};
      int lds_cu = 0;
      if (hipFuncGetAttributes(&at, fn) == hipSuccess && at.sharedSizeBytes > 0 &&
          hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                dev) == hipSuccess &&
          lds_cu > 0) {
        const size_t g = 2048, per = (at.sharedSizeBytes + g - 1) / g * g;
        n = std::max(1, std::min(n, (int)((size_t)lds_cu / per)));
      } else {
        (void)hipGetLastError();
      }
      slot = n;
      cu_count = c;
    } else {
      (void)hipGetLastError();
      slot = -1;
    }
  }
  if (slot < 0) return false;
  per_cu = slot;
  cus = cu_count;
  return true;
}

// One workgroup per work item, dispatched by the hardware: the alternative
// schedule of an ensemble launch (no counter, no item loop), with the same
// bands: the workgroups of band x are the ids b with b % kXcds = x.
template <class S, int MODE, int TILE>
__global__ void __launch_bounds__(kPersistThreads)
    grouped_kernel(const Args *__restrict__ models, const WorkItem *__restrict__ items) {
  __shared__ __attribute__((aligned(16))) char smem[persist_lds_bytes<S, MODE, TILE>()];
  // workgroup b is item l = b / kXcds of band b % kXcds (l < that band's length)
  uint32_t start, len;
  band_range(gridDim.x, blockIdx.x % kXcds, start, len);
  const WorkItem w = items[start + blockIdx.x / kXcds];
  const Args m = models[__builtin_amdgcn_readfirstlane(w.model)];
  run_item<S, MODE, TILE>(m, w, smem, threadIdx.x);
}

template <class S, int MODE>
static const void *grouped_fn(int tiles) {
  switch (tiles) {
    case 0: return reinterpret_cast<const void *>(&grouped_kernel<S, MODE, 0>);
    case 1: return reinterpret_cast<const void *>(&grouped_kernel<S, MODE, 1>);
    case 2: return reinterpret_cast<const void *>(&grouped_kernel<S, MODE, 2>);
    case kFitTile: return reinterpret_cast<const void *>(&grouped_kernel<S, MODE, kFitTile>);
    default: return reinterpret_cast<const void *>(&grouped_kernel<S, MODE, kMixedTiles>);
  }
}

static const void *grouped_ptr(tpfa_precision_t prec, int mode, int tiles) {
  const bool res = mode_kind(mode) == MODE_RESIDUAL;
  if (prec == TPFA_FP64)
    return res ? grouped_fn<double, MODE_RESIDUAL>(tiles) : grouped_fn<double, MODE_JACOBIAN>(tiles);
  if (has_plain_stores(mode))
    return res ? grouped_fn<float, MODE_RESIDUAL | MODE_PLAIN>(tiles)
               : grouped_fn<float, MODE_JACOBIAN | MODE_PLAIN>(tiles);
  return res ? grouped_fn<float, MODE_RESIDUAL>(tiles) : grouped_fn<float, MODE_JACOBIAN>(tiles);
}

hipError_t launch_grouped(tpfa_precision_t prec, int mode, int tiles, const Args *d_models,
                          const WorkItem *d_items, int64_t n_items, hipStream_t st) {
  const void *fn = grouped_ptr(prec, mode, tiles);
  void *args[] = {(void *)&d_models, (void *)&d_items};
  return hipLaunchKernel(fn, dim3((unsigned)n_items), dim3(kPersistThreads), args, 0, st);
}

template <class S, int MODE>
static const void *persist_fn(int tiles) {
  switch (tiles) {
    case 0: return reinterpret_cast<const void *>(&persistent_kernel<S, MODE, 0>);
    case 1: return reinterpret_cast<const void *>(&persistent_kernel<S, MODE, 1>);
    case 2: return reinterpret_cast<const void *>(&persistent_kernel<S, MODE, 2>);
    case kFitTile: return reinterpret_cast<const void *>(&persistent_kernel<S, MODE, kFitTile>);
    default: return reinterpret_cast<const void *>(&persistent_kernel<S, MODE, kMixedTiles>);
  }
}

static const void *persist_ptr(tpfa_precision_t prec, int mode, int tiles) {
  const bool res = mode_kind(mode) == MODE_RESIDUAL;
  if (prec == TPFA_FP64)
    return res ? persist_fn<double, MODE_RESIDUAL>(tiles) : persist_fn<double, MODE_JACOBIAN>(tiles);
  if (has_plain_stores(mode))
    return res ? persist_fn<float, MODE_RESIDUAL | MODE_PLAIN>(tiles)
               : persist_fn<float, MODE_JACOBIAN | MODE_PLAIN>(tiles);
  return res ? persist_fn<float, MODE_RESIDUAL>(tiles) : persist_fn<float, MODE_JACOBIAN>(tiles);
}

int persistent_workgroups(tpfa_precision_t prec, int mode, int tiles) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_ptr(prec, mode, tiles),
                                                   kPersistThreads, 0) != hipSuccess)
    return -1;
  if (per_cu < 1) per_cu = 1;
  return cus * per_cu;
}

hipError_t launch_persistent(tpfa_precision_t prec, int mode, int tiles, const Args *d_models,
                             const WorkItem *d_items, int64_t n_items, unsigned int *d_counter,
                             int n_workgroups, hipStream_t st) {
  reset_counters_kernel<<<1, 64, 0, st>>>(d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  void *args[] = {(void *)&d_models, (void *)&d_items, (void *)&n_items, (void *)&d_counter};
  return hipLaunchKernel(persist_ptr(prec, mode, tiles), dim3((unsigned)n_workgroups),
                         dim3(kPersistThreads), args, 0, st);
}

hipError_t launch_hydrostatic(const tpfa_grid_t &g, const tpfa_fluid_t &f, double p_top,
                              double *pref, hipStream_t st) {
  hydrostatic_kernel<<<1, 64, 0, st>>>((int)g.nz, g.gk * g.dz, f.rho0, f.cf, f.p0, p_top, pref);
  return hipGetLastError();
}

hipError_t launch_offset(const tpfa_grid_t &g, const double *p, const double *pref, float *dp,
                         hipStream_t st) {
  const int64_t n = g.nx * g.ny * g.nz;
  const int64_t blocks = (n + 255) / 256;
  const unsigned int grid = (unsigned int)(blocks < 65536 ? blocks : 65536);
  offset_kernel<<<grid, 256, 0, st>>>(g.nx, g.ldx ? g.ldx : g.nx, g.ny, n, p, pref, dp);
  return hipGetLastError();
}

}  // namespace tpfa

