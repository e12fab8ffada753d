// C-ABI layer of libtpfa.so: argument validation, launch-shape selection and
// the batched-ensemble object. Every argument error is detected here, on the
// host, before anything is enqueued; HIP errors are reported with their text.
// No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <exception>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/tpfa.h"
#include "tpfa_internal.h"

// the public op values are the kernel modes of the entry points
static_assert(int(TPFA_OP_RESIDUAL) == int(tpfa::MODE_RESIDUAL) &&
                  int(TPFA_OP_JACOBIAN) == int(tpfa::MODE_JACOBIAN) &&
                  int(TPFA_OP_VJP) == int(tpfa::MODE_VJP) &&
                  int(TPFA_OP_RESIDUAL10) == int(tpfa::MODE_RES10) &&
                  int(TPFA_OP_RESIDUAL_BE) == int(tpfa::MODE_RESIDUAL_BE) &&
                  int(TPFA_OP_JACOBIAN_BE) == int(tpfa::MODE_JACOBIAN_BE) &&
                  int(TPFA_OP_JVP) == int(tpfa::MODE_JVP) &&
                  int(TPFA_OP_JVP_BE) == int(tpfa::MODE_JVP_BE),
              "tpfa_op_t and the kernel modes disagree");

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int ok() {
  g_last_error.clear();
  return TPFA_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

// Row pitch of the arrays in cells: grid.ldx, or nx when it is 0.
int64_t pitch(const tpfa_grid_t &g) { return g.ldx ? g.ldx : g.nx; }

int check_grid(const tpfa_grid_t *g) {
  if (!g) return fail(TPFA_ERR_NULL, "grid is NULL");
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0)
    return fail(TPFA_ERR_SHAPE, "grid dimensions must be positive");
  const int64_t lim = std::numeric_limits<int32_t>::max();
  if (g->nx > lim || g->ny > lim || g->nz > lim)
    return fail(TPFA_ERR_SHAPE, "each grid dimension must fit in 32 bits");
  if (g->ldx != 0 && (g->ldx < g->nx || g->ldx > lim))
    return fail(TPFA_ERR_SHAPE, "the row pitch ldx must be 0 or at least nx (and fit in 32 bits)");
  const int64_t ld = pitch(*g);
  if (ld > std::numeric_limits<int64_t>::max() / g->ny ||
      ld * g->ny > std::numeric_limits<int64_t>::max() / 8 / 7 / g->nz)
    return fail(TPFA_ERR_SHAPE, "ldx*ny*nz overflows");
  if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) || !is_finite(g->dx) || !is_finite(g->dy) ||
      !is_finite(g->dz))
    return fail(TPFA_ERR_PARAM, "cell sizes must be positive and finite");
  if (!is_finite(g->gk)) return fail(TPFA_ERR_PARAM, "gk must be finite");
  return TPFA_OK;
}

int check_fluid(const tpfa_fluid_t *f) {
  if (!f) return fail(TPFA_ERR_NULL, "fluid is NULL");
  if (!(f->mu > 0) || !is_finite(f->mu)) return fail(TPFA_ERR_PARAM, "mu must be positive");
  if (!is_finite(f->rho0) || !is_finite(f->cf) || !is_finite(f->p0))
    return fail(TPFA_ERR_PARAM, "rho0, cf and p0 must be finite");
  return TPFA_OK;
}

int check_common(const tpfa_grid_t *g, const tpfa_fluid_t *f, const tpfa_rock_t *rk,
                 const tpfa_state_t *st, tpfa_precision_t prec, const tpfa_launch_t *launch) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_fluid(f))) return rc;
  if (!rk) return fail(TPFA_ERR_NULL, "rock is NULL");
  if (!st) return fail(TPFA_ERR_NULL, "state is NULL");
  if (prec != TPFA_FP64 && prec != TPFA_FP32)
    return fail(TPFA_ERR_PARAM, "unknown precision");
  // the kernels address a cell within its x-y plane with a 32-bit byte offset
  const int64_t elem = prec == TPFA_FP64 ? 8 : 4;
  if (pitch(*g) * g->ny > (int64_t)(std::numeric_limits<uint32_t>::max() / elem))
    return fail(TPFA_ERR_SHAPE, "an x-y plane of one array must hold fewer than 2^32 bytes");
  if (rk->tx || rk->ty || rk->tz) {
    if (!rk->tx || !rk->ty || !rk->tz)
      return fail(TPFA_ERR_NULL, "rock.tx, rock.ty and rock.tz are all required");
    if (rk->kx || rk->ky || rk->kz || rk->seal)
      return fail(TPFA_ERR_PARAM, "give either kx (and seal) or tx/ty/tz, not both");
  } else {
    if (!rk->kx) return fail(TPFA_ERR_NULL, "rock.kx is NULL");
    if ((rk->ky != nullptr) != (rk->kz != nullptr))
      return fail(TPFA_ERR_NULL, "rock.ky and rock.kz go together (both arrays or both NULL)");
    // with ky and kz arrays the ratios are not used
    if (!rk->ky &&
        (!(rk->ry >= 0) || !(rk->rz >= 0) || !is_finite(rk->ry) || !is_finite(rk->rz)))
      return fail(TPFA_ERR_PARAM, "ry and rz must be finite and >= 0");
  }
  if (!st->p) return fail(TPFA_ERR_NULL, "state.p is NULL");
  if (prec == TPFA_FP32 && !st->pref)
    return fail(TPFA_ERR_UNSUPPORTED, "the FP32 precision form needs state.pref");
  if (launch) {
    if (launch->tile < -1 || launch->tile >= tpfa::kNumTiles)
      return fail(TPFA_ERR_TILE, "unknown tile id");
    if (launch->kz_chunk < 0) return fail(TPFA_ERR_TILE, "kz_chunk must be >= 0");
    if ((launch->y_begin != 0 || launch->y_end != 0) &&
        !(launch->y_begin >= 0 && launch->y_begin < launch->y_end && launch->y_end <= g->ny))
      return fail(TPFA_ERR_PARAM, "row range must satisfy 0 <= y_begin < y_end <= ny");
  }
  return TPFA_OK;
}

// Launch-shape defaults from tile x z-chunk sweeps on MI355X (512x512x256 and
// 750x994x246): the Jacobian and the FP32 residual run best with 64x8 tiles,
// the vector-Jacobian / Jacobian-vector products (more registers) and the FP64
// residual (shared faces, more LDS) with 64x4, the 10-flux stencil with 128x4
// on grids at least 128 cells wide; narrow grids take narrower tiles. The
// FP64 Jacobian of the per-direction form (`form` = MODE_K3) needs more than
// 128 VGPRs, which leaves one 512-thread workgroup per CU: 64x4 measured 20%
// faster there. Sliced outputs are written in whole slices whatever nx is:
// 64x8 there (500x500x256 FP64: 1.01 ms against 1.10 ms with 128x4).
int default_tile(const tpfa_grid_t &g, tpfa::Mode mode, tpfa_precision_t prec, int form,
                 bool sliced) {
  if (g.nx <= 16) return 2;
  if (g.nx <= 32) return 1;
  const int b = tpfa::base_mode(mode);
  if (mode == tpfa::MODE_RES10) return g.nx >= 128 ? 4 : 0;
  if (b == tpfa::MODE_VJP || b == tpfa::MODE_JVP) return 0;
  if (b == tpfa::MODE_RESIDUAL && prec == TPFA_FP64) return 0;
  if (b == tpfa::MODE_JACOBIAN && prec == TPFA_FP64 && form == tpfa::MODE_K3) return 0;
  if (b == tpfa::MODE_JACOBIAN && prec == TPFA_FP64 && !sliced && (pitch(g) * 8) % 128 != 0) {
    // rows off 128-byte lines: 128-wide tiles halve the partial lines at tile
    // edges (10-15% faster on 500- and 750-wide grids) where they waste no
    // more lanes than 64-wide ones
    const int64_t w64 = (g.nx + 63) / 64 * 64, w128 = (g.nx + 127) / 128 * 128;
    if (w128 <= w64) return 4;
  }
  return 3;
}

// z planes per workgroup: 32 for the residual-only modes (64 for the FP32
// residual of the ratio form: on 512x512x256 32 / 64 / 128 planes took
// 0.253 / 0.248 / 0.247 ms, the FP64 residual ran 3-5% slower with 64 or 128)
// and the FP64
// Jacobians (0.7% faster than 16 there; 128 with sliced outputs: on
// 512x512x256 64 was 0.4% faster than 32 and 128 0.35% faster than 64, 256 no
// faster) and for the FP32 Jacobian of the ratio form (1% faster; 64 with
// sliced outputs, 1% faster than 32, while 16, 24 and 48 were slower), 16 for
// the other products (the FP32 backward-Euler and per-direction Jacobians ran
// 0.6-1.3% slower with 32).
int default_kz(tpfa::Mode mode, tpfa_precision_t prec, int form, bool sliced) {
  const int b = tpfa::base_mode(mode);
  if (mode == tpfa::MODE_RESIDUAL && form == 0 && prec == TPFA_FP32) return 64;
  if (b == tpfa::MODE_RESIDUAL || mode == tpfa::MODE_RES10) return 32;
  if (b == tpfa::MODE_JACOBIAN && prec == TPFA_FP64) return sliced ? 128 : 32;
  if (mode == tpfa::MODE_JACOBIAN && form == 0) return sliced ? 64 : 32;
  return 16;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(TPFA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace tpfa {

void fit_tile(int64_t nx, int64_t rows, int &tx, int &ty) {
  const int64_t nxt = (nx + kDynMaxTx - 1) / kDynMaxTx;
  tx = (int)std::max<int64_t>(kDynMinTx, (nx + nxt - 1) / nxt);
  int t = 256 / tx;
  if (2 * (tx + t) + 4 > 256) t = (256 - 4) / 2 - tx;
  const int64_t nyt = (rows + t - 1) / t;
  ty = (int)std::max<int64_t>(1, (rows + nyt - 1) / nyt);
}

void make_args(Args &a, const tpfa_grid_t &g, const tpfa_fluid_t &f, const tpfa_rock_t &rk,
               const tpfa_state_t &st, int tile, int kz_chunk, int flags, int64_t y0,
               int64_t y1) {
  std::memset(&a, 0, sizeof(a));
  TileShape ts{0, 0, 256};
  if (tile == kFitTile) {
    fit_tile(g.nx, y1 - y0, ts.tx, ts.ty);
    a.dtx = ts.tx;
    a.dty = ts.ty;
  } else {
    ts = kTiles[tile];
  }
  a.nx = (int32_t)g.nx;
  a.ny = (int32_t)g.ny;
  a.nz = (int32_t)g.nz;
  a.y0 = (int32_t)y0;
  a.y1 = (int32_t)y1;
  a.kz_chunk = (int32_t)std::min<int64_t>(kz_chunk, g.nz);
  // sliced outputs: the tiles reach the end of each row's last 64-cell slice,
  // so that every slice is written whole
  const int64_t xw = (flags & TPFA_LAUNCH_SLICED) ? (g.nx + 63) / 64 * 64 : g.nx;
  a.ntx = (int32_t)((xw + ts.tx - 1) / ts.tx);
  a.nty = (int32_t)((y1 - y0 + ts.ty - 1) / ts.ty);
  a.nzc = (int32_t)((g.nz + a.kz_chunk - 1) / a.kz_chunk);
  a.remap = (flags & TPFA_LAUNCH_XCD_REMAP) ? 1 : (flags & TPFA_LAUNCH_Y_FAST) ? 2 : 0;
  a.padw = (flags & TPFA_LAUNCH_PAD_WRITES) && pitch(g) > g.nx ? 1 : 0;
  a.tile = tile;
  a.ldx = (int32_t)pitch(g);
  a.plane = pitch(g) * g.ny;
  a.oplane = a.plane;
  a.orun = a.plane * g.nz;
  a.nblocks = (int64_t)a.ntx * a.nty * a.nzc;
  // face area over centre distance, per direction
  a.ax = g.dy * g.dz / g.dx;
  a.ay = g.dx * g.dz / g.dy;
  a.az = g.dx * g.dy / g.dz;
  a.ry = rk.ry;
  a.rz = rk.rz;
  a.gk = g.gk;
  a.dz = g.dz;
  a.rho0 = f.rho0;
  a.cf = f.cf;
  a.p0 = f.p0;
  a.mu = f.mu;
  // per-direction arrays carry their own scale: no ratios then
  const bool k3 = rk.ky != nullptr;
  a.a2x = 2.0 * a.ax;
  a.a2y = 2.0 * a.ay * (k3 ? 1.0 : rk.ry);
  a.a2z = 2.0 * a.az * (k3 ? 1.0 : rk.rz);
  a.inv_mu = 1.0 / f.mu;
  a.G = g.gk * g.dz;
  a.hc = 0.5 * f.cf * a.G;
  a.a2xf = (float)a.a2x;
  a.a2yf = (float)a.a2y;
  a.a2zf = (float)a.a2z;
  a.rho0f = (float)f.rho0;
  a.cff = (float)f.cf;
  a.inv_muf = (float)a.inv_mu;
  a.hcf = (float)a.hc;
  a.hgf = (float)(0.5 * a.G);
  a.p = st.p;
  a.pref = st.pref;
  a.kx = rk.kx;
  a.ky = rk.ky;
  a.kz = rk.kz;
  a.seal = rk.seal;
  a.tx = rk.tx;
  a.ty = rk.ty;
  a.tz = rk.tz;
}

}  // namespace tpfa

namespace {

// The XCD band order is part of the library's default launch where it measured
// faster on MI355X: on launches of at most kSmallCells computed cells in every
// mode of the permeability forms (256x256x128: the FP64 Jacobian 9%, the FP64
// residual 14%, the FP32 VJP and J v 8% faster), and on larger ones for the
// FP32 Jacobian and residual and the FP32 10-flux stencil with permeability
// input (the FP64 Jacobians ran 2-7% slower with it on 384x384x192 and
// 512x512x256). A caller that picks the tile also picks the flags.
constexpr int64_t kSmallCells = int64_t(1) << 24;

int default_flags(tpfa::Mode mode, tpfa_precision_t prec, int form, int64_t cells) {
  if (form == tpfa::MODE_TRANS) return 0;
  if (cells <= kSmallCells) return TPFA_LAUNCH_XCD_REMAP;
  if (prec != TPFA_FP32) return 0;
  const int b = tpfa::base_mode(mode);
  return b == tpfa::MODE_JACOBIAN || b == tpfa::MODE_RESIDUAL || mode == tpfa::MODE_RES10
             ? TPFA_LAUNCH_XCD_REMAP
             : 0;
}

// Small grids: a launch of the default z chunk that fills the GPU fewer than
// four times over is re-chunked so that its last round of workgroups is as
// full as possible. With C workgroups resident at once (the kernel's
// occupancy from the runtime, or 8 waves per SIMD where no device answers)
// and T tiles per chunk layer, the column is cut into L near-equal chunks of
// kz = ceil(nz / L) planes, L chosen to maximise (T L / C) / ceil(T L / C)
// (the used share of the launch's rounds) times kz / (kz + 2) (each chunk
// also loads the plane below it and fills its pipeline); chunks range from
// twice the default down to 4 planes. Measured: the FP32 residual + VJP on
// 256x256x128 (2048 workgroups of 64x4 with 16-plane chunks against 1280
// resident at 5 waves per SIMD) ran 0.075 ms, with 26-plane chunks (5 chunks,
// one full round) 0.065 ms; the FP32 residual there 0.054 -> 0.039 ms. Every
// chunk size computes the same values.
int fill_kz(const tpfa_grid_t &g, int64_t rows, int tile, int kz, tpfa_precision_t prec,
            int mode) {
  const tpfa::TileShape ts = tpfa::kTiles[tile];
  const int64_t tiles = ((g.nx + ts.tx - 1) / ts.tx) * ((rows + ts.ty - 1) / ts.ty);
  int per_cu = 0, cus = 0;
  if (!tpfa::march_residency(prec, mode, tile, per_cu, cus)) {
    cus = 256;
    per_cu = std::max(1, 4 * 8 / (ts.threads / 64));  // 8 waves per SIMD, 4 SIMDs per CU
  }
  const int64_t cap = (int64_t)cus * per_cu;
  const int64_t nz = g.nz;
  if (tiles * ((nz + kz - 1) / kz) >= 4 * cap) return kz;
  int best_kz = kz;
  double best = -1.0;
  const int64_t l_lo = std::max<int64_t>(1, (nz + 2 * kz - 1) / (2 * kz));
  const int64_t l_hi = std::max<int64_t>(l_lo, (nz + 3) / 4);
  for (int64_t L = l_lo; L <= l_hi; ++L) {
    const int64_t k = (nz + L - 1) / L;
    const int64_t chunks = (nz + k - 1) / k;
    const double rounds = (double)(tiles * chunks) / (double)cap;
    const double score = rounds / std::ceil(rounds) * (double)k / (double)(k + 2);
    if (score > best + 1e-9) {
      best = score;
      best_kz = (int)k;
    }
  }
  return best_kz;
}

// `form`: 0 (permeability with ratios), MODE_TRANS or MODE_K3. `fill`: adapt
// the default z chunk to small grids (single-grid launches; an ensemble fills
// the chip with its models). [y0, y1): the rows computed.
int resolve_launch(const tpfa_grid_t &g, tpfa::Mode mode, tpfa_precision_t prec, int form,
                   const tpfa_launch_t *launch, int &tile, int &kz, int &flags, int64_t &y0,
                   int64_t &y1, bool fill = true) {
  const bool dflt = !launch || launch->tile < 0;
  tile = dflt ? default_tile(g, mode, prec, form,
                             launch && (launch->flags & TPFA_LAUNCH_SLICED))
              : launch->tile;
  const bool rows = launch && launch->y_end > 0;
  y0 = rows ? launch->y_begin : 0;
  y1 = rows ? launch->y_end : g.ny;
  const bool sliced = launch && (launch->flags & TPFA_LAUNCH_SLICED);
  if (launch && launch->kz_chunk > 0)
    kz = launch->kz_chunk;
  else
    kz = fill ? fill_kz(g, y1 - y0, tile, default_kz(mode, prec, form, sliced), prec, mode | form)
              : default_kz(mode, prec, form, sliced);
  // the FP32 kernels hold per-plane constants of their chunk in LDS
  if (prec == TPFA_FP32) kz = std::min(kz, tpfa::kMaxChunk32);
  flags = launch ? launch->flags : 0;
  if (dflt) {
    const int64_t cells = g.nx * (y1 - y0) * g.nz;
    flags |= default_flags(mode, prec, form, cells);
    // the FP64 Jacobian with sliced outputs on large grids: the y-fast order
    // where a tile's x neighbours land on its XCD (tile rows a multiple of 8;
    // 512x512x256 with 64-plane chunks: 1.006 -> 1.001 ms)
    const int64_t nty = (y1 - y0 + tpfa::kTiles[tile].ty - 1) / tpfa::kTiles[tile].ty;
    if (sliced && prec == TPFA_FP64 && tpfa::base_mode(mode) == tpfa::MODE_JACOBIAN &&
        form == 0 && !(flags & TPFA_LAUNCH_XCD_REMAP) && nty % 8 == 0)
      flags |= TPFA_LAUNCH_Y_FAST;
  }
  return TPFA_OK;
}

// The rock form's mode flag: MODE_TRANS, MODE_K3 or 0.
int rock_form(const tpfa_rock_t &rk) {
  return rk.tx ? tpfa::MODE_TRANS : rk.ky ? tpfa::MODE_K3 : 0;
}

// TPFA_LAUNCH_SLICED: r and J in one array of 64-cell slices, for the
// Jacobian calls; r must be NULL (the residual is each slice's first run).
int set_sliced(tpfa::Args &a, int flags, int base_mode, tpfa_precision_t prec) {
  if (!(flags & TPFA_LAUNCH_SLICED)) return TPFA_OK;
  if (base_mode != tpfa::MODE_JACOBIAN)
    return fail(TPFA_ERR_UNSUPPORTED, "TPFA_LAUNCH_SLICED is for the Jacobian calls only");
  if (a.r)
    return fail(TPFA_ERR_PARAM,
                "with TPFA_LAUNCH_SLICED the residual is part of J: pass r = NULL");
  const int64_t es = prec == TPFA_FP64 ? 8 : 4;
  const int64_t slices = ((int64_t)a.nx + 63) / 64;
  if ((int64_t)a.ny * slices * 512 * es >= (int64_t(1) << 32))
    return fail(TPFA_ERR_SHAPE, "one z plane of the sliced r + J array holds 2^32 bytes or more");
  a.slices = (int32_t)slices;
  a.oplane = (int64_t)a.ny * slices * 512;
  a.orun = 64;
  a.r = a.J;
  a.J = static_cast<char *>(a.J) + 64 * es;
  return TPFA_OK;
}

// Output store kind: the FP32 kernels write with ordinary stores unless every
// output row starts on a 128-byte line (row pitch and output base pointers;
// sliced outputs: tiles of whole 64-cell slices); the FP64 kernels always
// write non-temporal (measured faster either way).
void set_store_kind(tpfa::Args &a, tpfa_precision_t prec) {
  bool lines = a.slices ? tpfa::kTiles[a.tile].tx % 64 == 0 : ((int64_t)a.ldx * 4) % 128 == 0;
  for (const void *q : {a.r, a.J, a.gp, a.gm, a.jv})
    if (q && reinterpret_cast<uintptr_t>(q) % 128 != 0) lines = false;
  a.plain = prec == TPFA_FP32 && !lines ? 1 : 0;
}

int run(tpfa::Mode mode, const tpfa_grid_t *g, const tpfa_fluid_t *f, const tpfa_rock_t *rk,
        const tpfa_state_t *st, tpfa_precision_t prec, const tpfa_launch_t *launch,
        tpfa::Args &a, void *stream) {
  int tile, kz, flags;
  int64_t y0, y1;
  const int form = rock_form(*rk);
  resolve_launch(*g, mode, prec, form, launch, tile, kz, flags, y0, y1);
  // a.r, a.J, a.w, a.gp, a.gm were set by the caller; keep them
  tpfa::Args b;
  tpfa::make_args(b, *g, *f, *rk, *st, tile, kz, flags, y0, y1);
  b.r = a.r;
  b.J = a.J;
  b.w = a.w;
  b.gp = a.gp;
  b.gm = a.gm;
  b.tne = a.tne;
  b.tse = a.tse;
  b.jv = a.jv;
  b.phi = a.phi;
  b.pprev = a.pprev;
  b.vdt = a.vdt;
  b.cr = a.cr;
  b.vdtf = a.vdtf;
  b.crf = a.crf;
  const int rc = set_sliced(b, flags, tpfa::base_mode(mode), prec);
  if (rc) return rc;
  set_store_kind(b, prec);
  if (b.nblocks > (int64_t)std::numeric_limits<uint32_t>::max())
    return fail(TPFA_ERR_SHAPE, "too many workgroups; use a larger kz_chunk");
  // the transmissibility and per-direction forms run the same modes with a flag
  const tpfa::Mode m = static_cast<tpfa::Mode>(mode | form);
  const hipError_t e = tpfa::launch_march(prec, m, tile, b, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

}  // namespace

extern "C" {

int tpfa_residual(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, const tpfa_rock_t *rock,
                  const tpfa_state_t *state, tpfa_precision_t prec, void *r,
                  const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!r) return fail(TPFA_ERR_NULL, "r is NULL");
    tpfa::Args a{};
    a.r = r;
    return run(tpfa::MODE_RESIDUAL, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_jacobian(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, const tpfa_rock_t *rock,
                  const tpfa_state_t *state, tpfa_precision_t prec, void *r, void *J,
                  const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!J) return fail(TPFA_ERR_NULL, "J is NULL");
    tpfa::Args a{};
    a.r = r;
    a.J = J;
    return run(tpfa::MODE_JACOBIAN, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_residual_vjp(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                      const tpfa_rock_t *rock, const tpfa_state_t *state,
                      tpfa_precision_t prec, const void *w, void *grad_p, void *grad_logk,
                      const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!w) return fail(TPFA_ERR_NULL, "w is NULL");
    if (!grad_p && !grad_logk) return fail(TPFA_ERR_NULL, "grad_p and grad_logk are both NULL");
    if (rock->tx)
      return fail(TPFA_ERR_UNSUPPORTED,
                  "the transmissibility form has its own product: tpfa_residual_vjp_trans");
    tpfa::Args a{};
    a.w = w;
    a.gp = grad_p;
    a.gm = grad_logk;
    return run(tpfa::MODE_VJP, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_residual_and_vjp(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                          const tpfa_rock_t *rock, const tpfa_state_t *state,
                          tpfa_precision_t prec, const void *w, void *r, void *grad_p,
                          void *grad_logk, const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!w) return fail(TPFA_ERR_NULL, "w is NULL");
    if (!r) return fail(TPFA_ERR_NULL, "r is NULL (without it, call tpfa_residual_vjp)");
    if (!grad_p && !grad_logk) return fail(TPFA_ERR_NULL, "grad_p and grad_logk are both NULL");
    if (rock->tx || rock->ky)
      return fail(TPFA_ERR_UNSUPPORTED,
                  "the residual with the VJP needs the permeability form with ry, rz ratios");
    tpfa::Args a{};
    a.w = w;
    a.r = r;
    a.gp = grad_p;
    a.gm = grad_logk;
    return run(static_cast<tpfa::Mode>(tpfa::MODE_VJP | tpfa::MODE_WITH_R), grid, fluid, rock,
               state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

// Accumulation fields of the backward-Euler modes from the descriptor.
int set_accumulation(const tpfa_grid_t *g, const tpfa_accum_t *acc, tpfa::Args &a) {
  if (!acc) return fail(TPFA_ERR_NULL, "accum is NULL");
  if (!acc->phi || !acc->p_prev) return fail(TPFA_ERR_NULL, "accum->phi and accum->p_prev are required");
  if (!(acc->dt > 0.0) || !std::isfinite(acc->dt))
    return fail(TPFA_ERR_PARAM, "accum->dt must be positive and finite");
  if (!std::isfinite(acc->cr)) return fail(TPFA_ERR_PARAM, "accum->cr must be finite");
  a.phi = acc->phi;
  a.pprev = acc->p_prev;
  a.vdt = (g->dx * g->dy * g->dz) / acc->dt;
  a.cr = acc->cr;
  a.vdtf = (float)a.vdt;
  a.crf = (float)acc->cr;
  return TPFA_OK;
}

int tpfa_residual_be(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                     const tpfa_rock_t *rock, const tpfa_state_t *state,
                     const tpfa_accum_t *accum, tpfa_precision_t prec, void *r,
                     const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!r) return fail(TPFA_ERR_NULL, "r is NULL");
    tpfa::Args a{};
    if ((rc = set_accumulation(grid, accum, a))) return rc;
    a.r = r;
    return run(tpfa::MODE_RESIDUAL_BE, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_jacobian_be(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                     const tpfa_rock_t *rock, const tpfa_state_t *state,
                     const tpfa_accum_t *accum, tpfa_precision_t prec, void *r, void *J,
                     const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!J) return fail(TPFA_ERR_NULL, "J is NULL");
    tpfa::Args a{};
    if ((rc = set_accumulation(grid, accum, a))) return rc;
    a.r = r;
    a.J = J;
    return run(tpfa::MODE_JACOBIAN_BE, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_jvp(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, const tpfa_rock_t *rock,
             const tpfa_state_t *state, const tpfa_accum_t *accum, tpfa_precision_t prec,
             const void *v, void *jv, void *r, const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!v) return fail(TPFA_ERR_NULL, "v is NULL");
    if (!jv) return fail(TPFA_ERR_NULL, "jv is NULL");
    tpfa::Args a{};
    if (accum && (rc = set_accumulation(grid, accum, a))) return rc;
    a.w = v;
    a.jv = jv;
    a.r = r;
    return run(accum ? tpfa::MODE_JVP_BE : tpfa::MODE_JVP, grid, fluid, rock, state, prec,
               launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_residual_vjp_trans(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                            const tpfa_rock_t *rock, const tpfa_state_t *state,
                            tpfa_precision_t prec, const void *w, void *grad_p, void *grad_logt,
                            const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!rock->tx)
      return fail(TPFA_ERR_UNSUPPORTED, "tpfa_residual_vjp_trans needs the transmissibility form");
    if (!w) return fail(TPFA_ERR_NULL, "w is NULL");
    if (!grad_p && !grad_logt) return fail(TPFA_ERR_NULL, "grad_p and grad_logt are both NULL");
    tpfa::Args a{};
    a.w = w;
    a.gp = grad_p;
    a.gm = grad_logt;
    return run(tpfa::MODE_VJP, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_residual10(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, const tpfa_rock_t *rock,
                    const tpfa_state_t *state, tpfa_precision_t prec, const void *tne,
                    const void *tse, void *r, const tpfa_launch_t *launch, void *stream) {
  try {
    int rc = check_common(grid, fluid, rock, state, prec, launch);
    if (rc) return rc;
    if (!tne || !tse) return fail(TPFA_ERR_NULL, "tne and tse are required");
    if (!r) return fail(TPFA_ERR_NULL, "r is NULL");
    tpfa::Args a{};
    a.r = r;
    a.tne = tne;
    a.tse = tse;
    return run(tpfa::MODE_RES10, grid, fluid, rock, state, prec, launch, a, stream);
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_hydrostatic(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, double p_top,
                     double *pref, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if ((rc = check_fluid(fluid))) return rc;
  if (!pref) return fail(TPFA_ERR_NULL, "pref is NULL");
  if (!is_finite(p_top)) return fail(TPFA_ERR_PARAM, "p_top must be finite");
  const hipError_t e =
      tpfa::launch_hydrostatic(*grid, *fluid, p_top, pref, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hydrostatic launch");
  return ok();
}

int tpfa_offset_pressure(const tpfa_grid_t *grid, const double *p, const double *pref,
                         float *dp, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!p || !pref || !dp) return fail(TPFA_ERR_NULL, "p, pref and dp are required");
  const hipError_t e =
      tpfa::launch_offset(*grid, p, pref, dp, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "offset launch");
  return ok();
}

static int stream_probe(const tpfa_grid_t *grid, tpfa_precision_t prec, const void *p,
                        const void *k, const uint8_t *seal, void *out, bool sliced,
                        void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (prec != TPFA_FP64 && prec != TPFA_FP32) return fail(TPFA_ERR_PARAM, "unknown precision");
  if (!p || !k || !seal || !out) return fail(TPFA_ERR_NULL, "p, k, seal and out are required");
  const int64_t es = prec == TPFA_FP64 ? 8 : 4;
  if (sliced && grid->ny * ((grid->nx + 63) / 64) * 512 * es >= (int64_t(1) << 32))
    return fail(TPFA_ERR_SHAPE, "one z plane of the sliced array holds 2^32 bytes or more");
  const hipError_t e = tpfa::launch_stream_probe(prec, *grid, p, k, seal, out, sliced,
                                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "probe launch");
  return ok();
}

int tpfa_stream_probe(const tpfa_grid_t *grid, tpfa_precision_t prec, const void *p,
                      const void *k, const uint8_t *seal, void *out, void *stream) {
  return stream_probe(grid, prec, p, k, seal, out, false, stream);
}

int tpfa_stream_probe_sliced(const tpfa_grid_t *grid, tpfa_precision_t prec, const void *p,
                             const void *k, const uint8_t *seal, void *out, void *stream) {
  return stream_probe(grid, prec, p, k, seal, out, true, stream);
}

// ---------------------------------------------------------------------------
// Batched ensemble
// ---------------------------------------------------------------------------

struct tpfa_batch {
  tpfa_precision_t prec;
  tpfa::Mode mode;
  tpfa::Args *d_models = nullptr;
  tpfa::WorkItem *d_items = nullptr;
  unsigned int *d_counter = nullptr;
  int64_t n_items = 0;
  int n_wg = 0;
  int tiles = 3;  // the tile shared by every model, or 3 for a mix
  int store = 0;  // tpfa::MODE_PLAIN: ordinary stores (see ensemble_store)
  int schedule = TPFA_SCHEDULE_PERSISTENT;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after every run: destroy waits for the last one
  bool ran = false;
};

static void batch_free(tpfa_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_models) (void)hipFree(b->d_models);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->done) (void)hipEventDestroy(b->done);
  delete b;
}

// Store kind of an ensemble launch: in FP32 ordinary stores (MODE_PLAIN)
// unless every member's output rows are written in whole lines (a row pitch
// of a multiple of 32 cells, and no padding, or TPFA_LAUNCH_PAD_WRITES with
// tiles whose lanes reach the pitch: not the fitted tile, which covers the
// cells only), where non-temporal ones measured 5% faster; FP64 always
// non-temporal.
static bool whole_line_rows(const tpfa::Args &a) {
  if (a.slices) return a.tile != tpfa::kFitTile && tpfa::kTiles[a.tile].tx % 64 == 0;
  if (a.ldx % 32 != 0) return false;
  if (a.ldx == a.nx) return true;
  return a.padw && a.tile != tpfa::kFitTile &&
         (int64_t)a.ntx * tpfa::kTiles[a.tile].tx >= (int64_t)a.ldx;
}
static int ensemble_store(tpfa_precision_t prec, bool all_whole_lines) {
  return prec == TPFA_FP32 && !all_whole_lines ? tpfa::MODE_PLAIN : 0;
}

static hipError_t batch_launch(tpfa_batch *b, hipStream_t st) {
  const int km = b->mode | b->store;
  if (b->schedule == TPFA_SCHEDULE_GROUPED)
    return tpfa::launch_grouped(b->prec, km, b->tiles, b->d_models, b->d_items, b->n_items, st);
  return tpfa::launch_persistent(b->prec, km, b->tiles, b->d_models, b->d_items, b->n_items,
                                 b->d_counter, b->n_wg, st);
}

// Captures the batch's one launch into a graph on a private stream.
static hipError_t batch_capture(tpfa_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = batch_launch(b, cs);
    e = hipStreamEndCapture(cs, &b->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  return e;
}

// Kernel arguments of ensemble member m (every check of an ensemble member;
// no allocation unless an error message is built).
static int batch_model(const tpfa_model_t &md, int m, tpfa_precision_t prec,
                       tpfa_batch_mode_t mode, tpfa::Args &a) {
  // the fitted tile exists for ensemble members only: the launch checks see a
  // default tile, its z chunk is the default one unless given
  tpfa_launch_t ln = md.launch;
  const bool fit = ln.tile == tpfa::kFitTile;
  if (fit) ln.tile = -1;
  int rc = check_common(&md.grid, &md.fluid, &md.rock, &md.state, prec, &ln);
  if (rc) return fail(rc, "model " + std::to_string(m) + ": " + g_last_error);
  if (md.rock.tx || md.rock.ky)
    return fail(TPFA_ERR_UNSUPPORTED, "model " + std::to_string(m) +
                                          ": the batch needs the permeability form with "
                                          "ry, rz ratios");
  if (mode == TPFA_BATCH_JACOBIAN && !md.J)
    return fail(TPFA_ERR_NULL, "model " + std::to_string(m) + ": J is NULL");
  if (mode == TPFA_BATCH_RESIDUAL && !md.r)
    return fail(TPFA_ERR_NULL, "model " + std::to_string(m) + ": r is NULL");
  int tile, kz, flags;
  int64_t y0, y1;
  resolve_launch(md.grid, mode == TPFA_BATCH_JACOBIAN ? tpfa::MODE_JACOBIAN
                                                      : tpfa::MODE_RESIDUAL,
                 prec, 0, &ln, tile, kz, flags, y0, y1, false);
  // the ensemble kernels hold the tile bodies 0, 1, 2 (64x4, 32x8, 16x16) and
  // the fitted tile; a default tile outside them (64x8 or 128x4) becomes 64x4
  if (fit) tile = tpfa::kFitTile;
  else if (ln.tile < 0 && tile > 2) tile = 0;
  if (tile > 2 && tile != tpfa::kFitTile)
    return fail(TPFA_ERR_TILE, "model " + std::to_string(m) +
                                   ": batched tiles must be tile 0, 1 or 2 (64x4, 32x8, "
                                   "16x16) or TPFA_TILE_FIT");
  tpfa::make_args(a, md.grid, md.fluid, md.rock, md.state, tile, kz, flags, y0, y1);
  a.r = md.r;
  a.J = mode == TPFA_BATCH_JACOBIAN ? md.J : nullptr;
  rc = set_sliced(a, flags,
                  mode == TPFA_BATCH_JACOBIAN ? tpfa::MODE_JACOBIAN : tpfa::MODE_RESIDUAL, prec);
  if (rc) return fail(rc, "model " + std::to_string(m) + ": " + g_last_error);
  return TPFA_OK;
}

int tpfa_batch_create(const tpfa_model_t *models, int n_models, tpfa_precision_t prec,
                      tpfa_batch_mode_t mode, tpfa_batch_t **out, void *stream) {
  try {
    if (!out) return fail(TPFA_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (!models) return fail(TPFA_ERR_NULL, "models is NULL");
    if (n_models <= 0) return fail(TPFA_ERR_SHAPE, "n_models must be positive");
    if (mode != TPFA_BATCH_RESIDUAL && mode != TPFA_BATCH_JACOBIAN)
      return fail(TPFA_ERR_PARAM, "unknown batch mode");
    std::vector<tpfa::Args> args(n_models);
    std::vector<tpfa::WorkItem> wl;
    for (int m = 0; m < n_models; ++m) {
      int rc = batch_model(models[m], m, prec, mode, args[m]);
      if (rc) return rc;
      // natural order: a tile's x neighbours follow it, so they run together
      // and share their halo cells and the output lines at their common edge
      // in L2
      const tpfa::Args &a = args[m];
      for (int bz = 0; bz < a.nzc; ++bz)
        for (int by = 0; by < a.nty; ++by)
          for (int bx = 0; bx < a.ntx; ++bx) wl.push_back({m, bx, by, bz * a.kz_chunk});
      if (wl.size() > (size_t)std::numeric_limits<uint32_t>::max() / 2)
        return fail(TPFA_ERR_SHAPE, "too many work items");
    }

    tpfa_batch *b = new tpfa_batch;
    b->prec = prec;
    b->mode = mode == TPFA_BATCH_JACOBIAN ? tpfa::MODE_JACOBIAN : tpfa::MODE_RESIDUAL;
    b->n_items = (int64_t)wl.size();
    b->tiles = args[0].tile;
    bool whole = true;
    for (const tpfa::Args &a : args) {
      if (a.tile != b->tiles) b->tiles = 3;
      whole = whole && whole_line_rows(a);
    }
    b->store = ensemble_store(prec, whole);
    const int wg = tpfa::persistent_workgroups(prec, b->mode | b->store, b->tiles);
    if (wg <= 0) {
      batch_free(b);
      return fail(TPFA_ERR_HIP, "could not query the device occupancy");
    }
    b->n_wg = (int)std::min<int64_t>(wg, b->n_items);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess) {
      b->done = nullptr;
      batch_free(b);
      return hip_fail(e, "batch event");
    }
    if ((e = hipMalloc(&b->d_models, sizeof(tpfa::Args) * args.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_items, sizeof(tpfa::WorkItem) * wl.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_counter, tpfa::kCounterWords * sizeof(unsigned int))) != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "batch allocation");
    }
    if ((e = hipMemcpyAsync(b->d_models, args.data(), sizeof(tpfa::Args) * args.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(b->d_items, wl.data(), sizeof(tpfa::WorkItem) * wl.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemsetAsync(b->d_counter, 0, tpfa::kCounterWords * sizeof(unsigned int), st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "batch upload");
    }
    if ((e = batch_capture(b)) != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "graph capture");
    }
    *out = b;
    return ok();
  } catch (const std::bad_alloc &) {
    return fail(TPFA_ERR_HIP, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

// Marks the end of a run on `st`, for tpfa_batch_destroy.
static int batch_mark(tpfa_batch *b, hipStream_t st) {
  const hipError_t e = hipEventRecord(b->done, st);
  if (e != hipSuccess) return hip_fail(e, "event record");
  b->ran = true;
  return ok();
}

int tpfa_batch_run(tpfa_batch_t *batch, void *stream) {
  if (!batch || !batch->exec) return fail(TPFA_ERR_NULL, "batch is NULL or empty");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = hipGraphLaunch(batch->exec, st);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return batch_mark(batch, st);
}

int tpfa_batch_run_eager(tpfa_batch_t *batch, void *stream) {
  if (!batch || !batch->d_items) return fail(TPFA_ERR_NULL, "batch is NULL or empty");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = batch_launch(batch, st);
  if (e != hipSuccess) return hip_fail(e, "ensemble launch");
  return batch_mark(batch, st);
}

int tpfa_batch_set_schedule(tpfa_batch_t *batch, int schedule) {
  if (!batch || !batch->d_items) return fail(TPFA_ERR_NULL, "batch is NULL or empty");
  if (schedule != TPFA_SCHEDULE_PERSISTENT && schedule != TPFA_SCHEDULE_GROUPED)
    return fail(TPFA_ERR_PARAM, "unknown schedule");
  if (batch->n_items > (int64_t)std::numeric_limits<uint32_t>::max() &&
      schedule == TPFA_SCHEDULE_GROUPED)
    return fail(TPFA_ERR_SHAPE, "too many work items for one workgroup each");
  batch->schedule = schedule;
  const hipError_t e = batch_capture(batch);
  if (e != hipSuccess) return hip_fail(e, "graph capture");
  return ok();
}

int tpfa_batch_info(const tpfa_batch_t *batch, int64_t *n_items, int *n_workgroups) {
  if (!batch) return fail(TPFA_ERR_NULL, "batch is NULL");
  if (n_items) *n_items = batch->n_items;
  if (n_workgroups) *n_workgroups = batch->n_wg;
  return ok();
}

void tpfa_batch_destroy(tpfa_batch_t *batch) {
  if (!batch) return;
  // runs of one batch are ordered (never concurrent), so the last one's end
  // is the end of all of them
  if (batch->ran) (void)hipEventSynchronize(batch->done);
  batch_free(batch);
}

int tpfa_ensemble_run_noalloc(const tpfa_model_t *models, int n_models, tpfa_precision_t prec,
                              tpfa_batch_mode_t mode, void *stream) {
  try {
    if (!models) return fail(TPFA_ERR_NULL, "models is NULL");
    if (n_models <= 0) return fail(TPFA_ERR_SHAPE, "n_models must be positive");
    if (n_models > tpfa::kStaticModels)
      return fail(TPFA_ERR_SHAPE, "an allocation-free run takes at most " +
                                      std::to_string(tpfa::kStaticModels) + " models");
    if (mode != TPFA_BATCH_RESIDUAL && mode != TPFA_BATCH_JACOBIAN)
      return fail(TPFA_ERR_PARAM, "unknown batch mode");
    // every member is checked before anything is enqueued
    tpfa::Args a;
    int64_t items = 0;
    int tiles = -1;
    bool whole = true;
    for (int m = 0; m < n_models; ++m) {
      const int rc = batch_model(models[m], m, prec, mode, a);
      if (rc) return rc;
      items += a.nblocks;
      tiles = (tiles < 0 || tiles == a.tile) ? a.tile : 3;
      whole = whole && whole_line_rows(a);
    }
    if (items > (int64_t)std::numeric_limits<uint32_t>::max())
      return fail(TPFA_ERR_SHAPE, "too many work items for one workgroup each");
    void *scr = nullptr;
    hipError_t e = tpfa::static_scratch(&scr);
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    tpfa::UploadBlock blk{};
    int64_t item = 0;
    for (int m0 = 0; m0 < n_models; m0 += tpfa::kUploadModels) {
      blk.first = m0;
      blk.count = std::min(tpfa::kUploadModels, n_models - m0);
      for (int q = 0; q < blk.count; ++q) {
        (void)batch_model(models[m0 + q], m0 + q, prec, mode, blk.a[q]);
        blk.item0[q] = item;
        item += blk.a[q].nblocks;
      }
      if ((e = tpfa::launch_upload(blk, scr, st)) != hipSuccess)
        return hip_fail(e, "model table upload");
    }
    const int km = (mode == TPFA_BATCH_JACOBIAN ? tpfa::MODE_JACOBIAN : tpfa::MODE_RESIDUAL) |
                   ensemble_store(prec, whole);
    if ((e = tpfa::launch_static_grouped(prec, km, tiles, scr, n_models, items, st)) !=
        hipSuccess)
      return hip_fail(e, "ensemble launch");
    return ok();
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_resolve_launch(const tpfa_grid_t *grid, int op, tpfa_precision_t prec,
                        const tpfa_rock_t *rock, const tpfa_launch_t *launch,
                        tpfa_launch_t *resolved) {
  try {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!rock || !resolved) return fail(TPFA_ERR_NULL, "rock and resolved are required");
    if (op < TPFA_OP_RESIDUAL || op > TPFA_OP_JVP_BE) return fail(TPFA_ERR_PARAM, "unknown op");
    if (prec != TPFA_FP64 && prec != TPFA_FP32)
      return fail(TPFA_ERR_PARAM, "unknown precision");
    if (launch) {
      if (launch->tile < -1 || launch->tile >= tpfa::kNumTiles)
        return fail(TPFA_ERR_TILE, "unknown tile id");
      if (launch->kz_chunk < 0) return fail(TPFA_ERR_TILE, "kz_chunk must be >= 0");
      if ((launch->y_begin != 0 || launch->y_end != 0) &&
          !(launch->y_begin >= 0 && launch->y_begin < launch->y_end &&
            launch->y_end <= grid->ny))
        return fail(TPFA_ERR_PARAM, "row range must satisfy 0 <= y_begin < y_end <= ny");
    }
    const tpfa::Mode mode = static_cast<tpfa::Mode>(op);
    int tile, kz, flags;
    int64_t y0, y1;
    resolve_launch(*grid, mode, prec, rock_form(*rock), launch, tile, kz, flags, y0, y1);
    resolved->tile = tile;
    resolved->kz_chunk = (int)std::min<int64_t>(kz, grid->nz);
    resolved->flags = flags;
    resolved->y_begin = y0;
    resolved->y_end = y1;
    return ok();
  } catch (const std::exception &e) {
    return fail(TPFA_ERR_HIP, e.what());
  } catch (...) {
    return fail(TPFA_ERR_HIP, "unknown exception");
  }
}

int tpfa_fit_tile_shape(int64_t nx, int64_t rows, int *tx, int *ty) {
  if (nx <= 0 || rows <= 0) return fail(TPFA_ERR_SHAPE, "nx and rows must be positive");
  if (!tx || !ty) return fail(TPFA_ERR_NULL, "tx and ty are required");
  tpfa::fit_tile(nx, rows, *tx, *ty);
  return ok();
}

int tpfa_num_tiles(void) { return tpfa::kNumTiles; }

int tpfa_tile_shape(int id, int *tx, int *ty, int *threads) {
  if (id < 0 || id >= tpfa::kNumTiles) return fail(TPFA_ERR_TILE, "unknown tile id");
  if (tx) *tx = tpfa::kTiles[id].tx;
  if (ty) *ty = tpfa::kTiles[id].ty;
  if (threads) *threads = tpfa::kTiles[id].threads;
  return ok();
}

const char *tpfa_strerror(int code) {
  switch (code) {
    case TPFA_OK: return "success";
    case TPFA_ERR_NULL: return "a required pointer is NULL";
    case TPFA_ERR_SHAPE: return "invalid grid shape";
    case TPFA_ERR_PARAM: return "invalid parameter";
    case TPFA_ERR_UNSUPPORTED: return "unsupported combination of arguments";
    case TPFA_ERR_HIP: return "HIP runtime error";
    case TPFA_ERR_TILE: return "unknown tile or z-chunk";
    default: return "unknown error code";
  }
}

const char *tpfa_last_error(void) { return g_last_error.c_str(); }

int tpfa_version(void) { return TPFA_VERSION; }

}  // extern "C"
