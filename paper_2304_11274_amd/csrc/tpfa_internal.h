// Internal interface between the C-ABI layer (tpfa_api.cpp) and the HIP
// kernels (tpfa_tile.h, tpfa_kernels.hip, tpfa_march_*.hip). Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpfa.h"

namespace tpfa {

// Kernel modes. The *_BE modes add the accumulation term of the backward-Euler
// residual; the JVP modes form J v without storing J.
enum Mode : int {
  MODE_RESIDUAL = 0,
  MODE_JACOBIAN = 1,
  MODE_VJP = 2,
  MODE_RES10 = 3,
  MODE_RESIDUAL_BE = 4,
  MODE_JACOBIAN_BE = 5,
  MODE_JVP = 6,
  MODE_JVP_BE = 7
};
// Flag added to a mode: the face transmissibilities are inputs (tx, ty, tz)
// instead of the harmonic average of kx.
constexpr int MODE_TRANS = 8;
// Flag added to an FP32 mode: the outputs are written with ordinary stores
// instead of non-temporal ones (grids whose rows do not start on 128-byte
// lines).
constexpr int MODE_PLAIN = 16;
// Flag added to a mode: per-direction permeability arrays (kx, ky, kz), each
// face taking the harmonic average of its own direction's k (no ratios).
constexpr int MODE_K3 = 32;
// Flag added to MODE_VJP (permeability form with ratios): the kernel also
// writes the residual, the value and gradient of w.r in one pass.
constexpr int MODE_WITH_R = 64;
constexpr int mode_kind(int m) { return m & 7; }
constexpr bool has_with_r(int m) { return (m & MODE_WITH_R) != 0; }
constexpr bool has_trans(int m) { return (m & MODE_TRANS) != 0; }
constexpr bool has_plain_stores(int m) { return (m & MODE_PLAIN) != 0; }
constexpr bool has_k3(int m) { return (m & MODE_K3) != 0; }
constexpr int base_mode(int m) {
  return mode_kind(m) == MODE_RESIDUAL_BE   ? MODE_RESIDUAL
         : mode_kind(m) == MODE_JACOBIAN_BE ? MODE_JACOBIAN
         : mode_kind(m) == MODE_JVP_BE      ? MODE_JVP
                                            : mode_kind(m);
}
constexpr bool has_accumulation(int m) {
  return mode_kind(m) == MODE_RESIDUAL_BE || mode_kind(m) == MODE_JACOBIAN_BE ||
         mode_kind(m) == MODE_JVP_BE;
}

// Tile table. A workgroup owns a TX x TY column block of one model and marches
// it through a chunk of z planes; each thread stages ceil(2 (TX + TY) / threads)
// cells of the halo ring. Wide tiles write long contiguous runs per plane.
struct TileShape {
  int tx, ty, threads;
};
// FP32 kernels keep two per-plane constants of their z chunk in LDS (the
// plane's reference density and the hydrostatic part of its z-face potential
// difference), so their chunk is at most this many planes.
constexpr int kMaxChunk32 = 128;
constexpr int kNumTiles = 10;
// Ensemble members may also take the fitted tile (id kFitTile): a tile of
// dtx x dty cells fitted to the member's rows, 256 threads (see fit_tile).
constexpr int kFitTile = 10;
constexpr int kDynMinTx = 8, kDynMaxTx = 64;
constexpr TileShape kTiles[kNumTiles] = {
    {64, 4, 256},  {32, 8, 256},  {16, 16, 256}, {64, 8, 512},  {128, 4, 512},
    {32, 16, 512}, {128, 2, 256}, {256, 1, 256}, {256, 2, 512}, {512, 1, 512}};

// Everything a kernel needs about one grid; passed by value (kernel argument)
// for single launches and stored in a device table for the batched kernel.
struct Args {
  int32_t nx, ny, nz;
  int32_t kz_chunk;   // z planes per workgroup
  int32_t ntx, nty, nzc;  // tiles along x, y and z chunks
  int32_t remap;      // workgroup order: 0 natural, 1 XCD bands of tile rows, 2 y fastest
  int32_t tile;       // index into kTiles
  int32_t plain;      // 1: ordinary output stores (FP32 rows off 128-byte lines)
  int32_t y0, y1;     // rows computed and written: [y0, y1) (others are read only)
  int32_t ldx;        // row pitch of every array, in cells (>= nx)
  int32_t dtx, dty;   // shape of the fitted tile (tile == kFitTile)
  int32_t padw;       // 1: tile lanes in the row padding (nx <= i < ldx) store zeros
  int32_t slices;     // 0: outputs in planes of the arrays' row pitch; n > 0: r and J in
                      // one sliced array of n slices of 64 cells per row
  int64_t plane;      // ldx * ny
  int64_t oplane;     // elements per z plane of an output array (plane; sliced: ny * slices * 512)
  int64_t orun;       // elements between the Jacobian's seven planes (ncell; sliced: 64)
  int64_t nblocks;    // ntx * nty * nzc
  // transmissibility geometric factors a_d and directional ratios (y, z)
  double ax, ay, az, ry, rz;
  double gk, dz;      // gravity along +k, cell size along k
  double rho0, cf, p0, mu;
  // derived constants of the FP64 path
  double a2x, a2y, a2z;  // 2 a_d r_d
  double inv_mu;         // 1 / mu
  double G;              // gk * dz: gravity potential drop across a z face per unit density
  double hc;             // 0.5 * cf * G
  // FP32 precision form
  float a2xf, a2yf, a2zf;
  float rho0f, cff, inv_muf, hcf;
  float hgf;             // 0.5 * G, for the density deviations of a z face
  // accumulation term of the backward-Euler residual: V / dt and the rock
  // compressibility (FP64 and FP32 copies)
  double vdt, cr;
  float vdtf, crf;
  const void *p;
  const double *pref;
  const void *kx;
  const void *ky;     // per-direction form: y and z permeabilities (else NULL)
  const void *kz;
  const uint8_t *seal;
  const void *w;      // cotangent (VJP) or direction v (JVP)
  const void *phi;    // reference porosity per cell (backward-Euler modes)
  const void *pprev;  // pressure of the previous time level, in the form of p
  const void *tx;    // transmissibility input: faces towards +x, +y, +z
  const void *ty;
  const void *tz;
  const void *tne;   // 10-flux stencil: diagonal transmissibilities
  const void *tse;
  void *r;
  void *J;
  void *gp;
  void *gm;           // grad ln kx; grad ln T [3][ncell] in the transmissibility form,
                      // grad ln kx, ln ky, ln kz [3][ncell] in the per-direction form
  void *jv;           // J v (JVP modes)
};

// The fitted tile of a member of nx x ny cells per plane (rows [y0, y1)): tx
// the row length of the fewest tiles of at most 64 cells covering a row, in
// near-equal parts (at least 8); ty the most rows 256 threads hold (and that
// one halo cell per thread covers the ring), then balanced over the rows.
void fit_tile(int64_t nx, int64_t rows, int &tx, int &ty);

// Fills the derived fields of `a` from the ABI structs (host only).
void make_args(Args &a, const tpfa_grid_t &g, const tpfa_fluid_t &f, const tpfa_rock_t &rk,
               const tpfa_state_t &st, int tile, int kz_chunk, int flags, int64_t y0,
               int64_t y1);

// Launchers (host). Return hipSuccess or the launch error.
hipError_t launch_march(tpfa_precision_t prec, Mode mode, int tile, const Args &a,
                        hipStream_t stream);
// Workgroups of a single-grid kernel (mode kind | form flags, tile; FP32 with
// non-temporal stores) resident per CU, and the CU count of the current
// device; false where no device answers.
bool march_residency(tpfa_precision_t prec, int mode, int tile, int &per_cu, int &cus);
hipError_t launch_hydrostatic(const tpfa_grid_t &g, const tpfa_fluid_t &f, double p_top,
                              double *pref, hipStream_t stream);
hipError_t launch_offset(const tpfa_grid_t &g, const double *p, const double *pref, float *dp,
                         hipStream_t stream);
hipError_t launch_stream_probe(tpfa_precision_t prec, const tpfa_grid_t &g, const void *p,
                               const void *k, const uint8_t *seal, void *out, bool sliced,
                               hipStream_t stream);

// Batched ensemble kernels (persistent and grouped schedules). The work list
// is cut into one band per XCD; the persistent schedule keeps one claim
// counter per band, each on its own 128-byte line (kCounterStride words
// apart) so that the bands' atomics do not contend for one line.
constexpr int kXcds = 8;
constexpr int kBatchCounters = kXcds;
constexpr int kCounterStride = 32;
constexpr int kCounterWords = kBatchCounters * kCounterStride;
struct WorkItem {
  int32_t model;
  int32_t bx, by, kb;
};
// `tiles`: 0, 1, 2 or kFitTile when every model uses that 256-thread tile, 3 for a mix.
// `mode`: MODE_RESIDUAL or MODE_JACOBIAN, in FP32 with MODE_PLAIN for ordinary stores
// (the batch's choice: ordinary unless every member's output rows are whole lines).
hipError_t launch_persistent(tpfa_precision_t prec, int mode, int tiles, const Args *d_models,
                             const WorkItem *d_items, int64_t n_items, unsigned int *d_counter,
                             int n_workgroups, hipStream_t stream);
int persistent_workgroups(tpfa_precision_t prec, int mode, int tiles);
hipError_t launch_grouped(tpfa_precision_t prec, int mode, int tiles, const Args *d_models,
                          const WorkItem *d_items, int64_t n_items, hipStream_t stream);

// Allocation-free ensemble run: the model table and each model's first work
// item live in a fixed-size device array of the library (one per GPU), written
// by upload launches whose kernel arguments carry up to kUploadModels models.
constexpr int kStaticModels = 256;
constexpr int kUploadModels = 8;
struct UploadBlock {
  int32_t first, count;            // table rows [first, first + count)
  int64_t item0[kUploadModels];    // first work item of each of these models
  Args a[kUploadModels];
};
// The device address of this GPU's array (resolved once per device).
hipError_t static_scratch(void **ptr);
hipError_t launch_upload(const UploadBlock &blk, void *scratch, hipStream_t stream);
hipError_t launch_static_grouped(tpfa_precision_t prec, int mode, int tiles, void *scratch,
                                 int n_models, int64_t n_items, hipStream_t stream);

}  // namespace tpfa
