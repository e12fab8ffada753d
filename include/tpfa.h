/*
 * tpfa.h -- C ABI of libtpfa.so: the TPFA flux residual, its 7-point Jacobian
 * and its vector-Jacobian product on a 3-D Cartesian grid, on one AMD MI355X
 * (gfx950) GPU.
 *
 * What is computed (paper "Massively Distributed Finite-Volume Flux
 * Computation", Sec. 3):
 *   rho_K      = rho0 * exp(cf * (p_K - p0))                        Eq. (5)
 *   lambda_K   = rho_K / mu                                         mobility, constant mu
 *   Ups_KL     = a_d * 2 k_K k_L / (k_K + k_L)                       two-point harmonic transmissibility
 *                (a_x = dy dz/dx, a_y = dx dz/dy, a_z = dx dy/dz; directional k;
 *                 0 on a sealed face or when k_K + k_L = 0)
 *   dPhi_KL    = (p_K - p_L) + (rho_K + rho_L)/2 * gk * (zeta_L - zeta_K)
 *                                                                    Eq. (3b), outflow orientation
 *   F_KL       = Ups_KL * lambda_up * dPhi_KL, lambda_up = lambda_K if
 *                dPhi_KL > 0, lambda_L if < 0, the lower index on a tie  Eqs. (3a), (4)
 *   r_K        = sum over the (up to six) face neighbours L of F_KL     Algorithm 1
 * zeta is the cell-centre coordinate along +k and gk the gravity component
 * along +k (k pointing down: gk = +9.81). Domain boundaries are no-flow. The
 * accumulation term of the backward-Euler residual, Eq. (2), is not included.
 *
 * Conventions for every entry point:
 *  - Arrays are structure-of-arrays with x fastest:
 *    idx = i + ldx * (j + ny * k), where ldx = grid.ldx (the row pitch) or nx
 *    when grid.ldx is 0 (contiguous arrays). Every per-cell array of one call
 *    (inputs and outputs, each plane of J and of the gradients) uses the same
 *    pitch; an array of P planes holds plane q at offset q * ldx * ny * nz.
 *    Cells with nx <= i < ldx are padding: never read as cells, and never
 *    written unless the launch sets TPFA_LAUNCH_PAD_WRITES. With
 *    TPFA_LAUNCH_SLICED the Jacobian calls write r and J into one array of
 *    64-cell row slices instead (layout at that flag).
 *  - Array pointers are DEVICE pointers (hipMalloc'ed or torch CUDA tensors)
 *    owned by the caller, unless stated otherwise. Structs are read on the host
 *    during the call and may be freed when it returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *    enqueue work and return without synchronising; they allocate nothing.
 *  - Precision: TPFA_FP64 -> every array (p, kx, r, J, w, grads) is double.
 *    TPFA_FP32 -> the "precision form": p holds FP32 offsets dp from an FP64
 *    reference profile pref[nz] (p_K = pref[k] + dp_K in FP64), kx and outputs
 *    are float; the z-face potential differences and the residual and J v sums
 *    are carried in FP64 and rounded once on store; the Jacobian diagonal and
 *    the six terms of each gradient are summed in float (no cancellation
 *    there beyond a few ulp of the sum of the terms' magnitudes).
 *  - Return value: TPFA_OK (0) or a negative TPFA_ERR_* code; the detail is in
 *    tpfa_last_error() (thread-local). No C++ exception crosses the ABI.
 *    Argument errors are detected on the host before anything is enqueued.
 *    Data values are never inspected: NaNs propagate, kx >= 0 is the caller's
 *    contract.
 */
#ifndef TPFA_H
#define TPFA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Library version: major * 10000 + minor * 100 + patch (tpfa_version() returns
   the built library's). The major number changes with the layout of the ABI
   structs: version 2 added tpfa_grid_t.ldx (row-pitched arrays); 2.1 added
   TPFA_LAUNCH_SLICED and tpfa_stream_probe_sliced. */
#define TPFA_VERSION 20100

#define TPFA_OK 0
#define TPFA_ERR_NULL (-1)        /* a required pointer is NULL */
#define TPFA_ERR_SHAPE (-2)       /* a dimension <= 0, 0 < ldx < nx, ldx*ny*nz overflows, or one x-y plane of an array holds 2^32 bytes or more */
#define TPFA_ERR_PARAM (-3)       /* mu <= 0, cell size <= 0, negative ratio, non-finite constant */
#define TPFA_ERR_UNSUPPORTED (-4) /* unsupported combination (see each call) */
#define TPFA_ERR_HIP (-5)         /* HIP runtime error, detail in tpfa_last_error() */
#define TPFA_ERR_TILE (-6)        /* unknown tile id or z-chunk out of range */

typedef enum { TPFA_FP64 = 0, TPFA_FP32 = 1 } tpfa_precision_t;

/* Grid: cell counts, cell sizes (m), gravity component along +k (m/s^2),
   and the row pitch of the arrays in cells (0 = nx; otherwise ldx >= nx, else
   TPFA_ERR_SHAPE). Rows that start on 128-byte lines (ldx * element size a
   multiple of 128 and 128-byte aligned base pointers) let each tile write
   whole lines (with TPFA_LAUNCH_PAD_WRITES, each row's last line too); on
   MI355X, contiguous rows that straddle lines at tile edges took the FP32
   residual + Jacobian on 500 x 500 x 256 1.45 times as long as rows padded to
   512 cells, and the FP64 one 1.18 times. */
typedef struct {
  int64_t nx, ny, nz;
  double dx, dy, dz;
  double gk;
  int64_t ldx;
} tpfa_grid_t;

/* Fluid, Eq. (5) and constant viscosity (SI): rho0 (kg/m^3), cf (1/Pa),
   p0 (Pa), mu (Pa s). */
typedef struct {
  double rho0, cf, p0, mu;
} tpfa_fluid_t;

/* Rock, in one of three forms.
   Permeability form: kx (m^2, dtype of the precision) is required. With ky
   and kz NULL the y and z permeabilities are ry*kx and rz*kx (ry, rz >= 0);
   with ky and kz both given (per-direction form: arrays of the same layout
   and dtype) each face along axis a takes k_a of its two cells and ry, rz
   are ignored. Each face gets the two-point harmonic transmissibility
   (Sec. 3). Only one of ky, kz: TPFA_ERR_NULL. seal may be NULL; bit a
   (0, 1, 2 = x, y, z) of seal[idx] closes the face between the cell and its
   +a neighbour (bits on domain-boundary faces are ignored).
   Transmissibility form: tx, ty, tz (m^3, dtype of the precision) give the
   transmissibility of the face between cell idx and its +x, +y, +z neighbour
   directly (the face-centred data the paper stores with each cell, Sec. 5,
   here once per face); entries on the last layer along a direction are
   ignored and T = 0 closes a face. Then kx, ky, kz and seal must be NULL and
   ry, rz are ignored. Supported by every entry point except
   tpfa_residual_vjp (use tpfa_residual_vjp_trans) and the batch
   (TPFA_ERR_UNSUPPORTED); the batch also rejects the per-direction form. */
typedef struct {
  const void *kx, *ky, *kz;
  double ry, rz;
  const uint8_t *seal;
  const void *tx, *ty, *tz;
} tpfa_rock_t;

/* State: TPFA_FP64 -> p is absolute pressure (double, Pa), pref ignored.
   TPFA_FP32 -> p is the float offset dp and pref (double[nz], device, finite)
   is required; the pressure of a cell in plane k is pref[k] + dp. The kernels
   split each density into its plane's reference density
   rho0 exp(cf (pref[k] - p0)), evaluated in FP64, and a float deviation, so
   the potential difference of a z face carries no float rounding of rho g dz
   whatever pref is (Sec. 3, Eqs. 3b and 5); a hydrostatic pref
   (tpfa_hydrostatic) keeps the offsets, and their rounding, small. */
typedef struct {
  const void *p;
  const double *pref;
} tpfa_state_t;

/* Optional launch shape (pass NULL for the defaults): tile = id from
   tpfa_tile_shape(), or -1 for the library's default launch; kz_chunk = z
   planes marched by one workgroup (0 = default, which a single-grid call
   shortens on small grids until the launch fills the GPU; in TPFA_FP32 at most
   128, larger values run as 128, since those kernels keep two constants per
   plane of their chunk on chip); flags bit 0 selects the
   XCD-aware workgroup order (the tiles of each z chunk are split into 8
   contiguous bands of tile rows, one per XCD). With tile = -1 (or NULL) the
   library also sets that bit where it measured faster; with an explicit tile
   the flags are taken as given. Results never depend on the launch shape.
   Row range (y slab): with y_end > 0, only the cells of rows
   y_begin <= j < y_end (0 <= y_begin < y_end <= ny) are computed and their
   outputs written; the grid's other rows are read as neighbours (a halo) and
   their outputs are left untouched. This is one GPU's launch in a y-slab
   decomposition, on its slab plus one halo row per side. y_begin = y_end = 0:
   every row. */
typedef struct {
  int tile;
  int kz_chunk;
  int flags;
  int64_t y_begin, y_end;
} tpfa_launch_t;

#define TPFA_LAUNCH_XCD_REMAP 1
/* flags bit 1 (ignored with bit 0): tiles in y-fast order, so that the
   workgroups of a tile's x neighbours are ny/TY ids apart (the hardware hands
   consecutive ids to the 8 XCDs in turn: with ny/TY a multiple of 8 they run
   on one XCD and share the x-halo lines in its L2). */
#define TPFA_LAUNCH_Y_FAST 2
/* flags bit 2: the row padding of the OUTPUT arrays (cells nx <= i < ldx of
   r, J, the gradients, J v) may be overwritten: the tile lanes that fall in
   the padding store zeros there, so that with ldx * element size a multiple
   of 128 and 128-byte aligned outputs each row's stores cover whole 128-byte
   lines. On MI355X a write that covers part of a line costs a read-modify-
   write in memory: on an ensemble of rows of 32 to 256 cells this flag with
   rows padded to 128 bytes took the FP32 Jacobian from 1.21 to 1.02 ms.
   Values of real cells do not change; inputs' padding is still never read.
   Kept from the caller's flags also with tile = -1. */
#define TPFA_LAUNCH_PAD_WRITES 4
/* flags bit 3, tpfa_jacobian and tpfa_jacobian_be only (TPFA_ERR_UNSUPPORTED
   elsewhere): r and J are written into ONE array, J, of 64-cell row slices,
   and r must be NULL (TPFA_ERR_PARAM otherwise). With S = ceil(nx / 64)
   slices per row, slice s of row j of plane k holds 8 runs of 64 values:
   run 0 the residual, runs 1..7 the Jacobian planes 0..6 of tpfa_jacobian,
   value (q, i, j, k) at element (((k ny + j) S + i / 64) 8 + q) 64 + i % 64;
   the array holds nz ny S 512 elements. This is the sliced ELLPACK order
   (slices of C = 64 rows, 7 diagonals) that a matrix-vector product reads in
   whole lines. The lanes of a row's last slice beyond nx store zeros, so
   every slice of a computed row is written whole; rows outside the launch's
   row range are left untouched. ldx applies to the inputs only; one z plane
   of the array must hold fewer than 2^32 bytes (TPFA_ERR_SHAPE). On MI355X
   the one output stream wrote faster than eight planes: a streaming kernel
   with the FP64 Jacobian's traffic (17 B read, 64 B written per cell) ran
   at 4.92 TB/s with eight output planes and 5.49 TB/s with the slices.
   The batch takes it per member (member r NULL). */
#define TPFA_LAUNCH_SLICED 8

/* Residual r[ncell] (paper Algorithm 1 with the Eq. (3)-(5) flux). */
int tpfa_residual(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                  const tpfa_rock_t *rock, const tpfa_state_t *state,
                  tpfa_precision_t prec, void *r, const tpfa_launch_t *launch,
                  void *stream);

/* Residual (r may be NULL) and Jacobian J[7][ncell]: plane 0 = dr_K/dp_K,
   planes 1..6 = dr_K/dp_L for the -x, +x, -y, +y, -z, +z neighbour L (0 where
   that neighbour does not exist). The paper names the flux derivatives with
   respect to the state as a key step of the simulator (Sec. 2) but computes
   only the residual; the derivative here is the exact derivative of the
   residual above on the side of each upwind switch that the choice took. */
int tpfa_jacobian(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                  const tpfa_rock_t *rock, const tpfa_state_t *state,
                  tpfa_precision_t prec, void *r, void *J,
                  const tpfa_launch_t *launch, void *stream);

/* Vector-Jacobian product of the residual with the cotangent w[ncell]:
   grad_p = J^T w (with respect to p, i.e. to dp in the precision form) and
   grad_logk[j] = sum_K w_K d r_K / d ln(kx_j), ky = ry kx and kz = rz kx
   following kx. In the per-direction form (ky, kz arrays) grad_logk holds
   three planes [3][ncell]: d(w.r)/d ln kx, ln ky, ln kz of each cell. The
   upwind choice is recomputed, not stored. Either output may be NULL (not
   both). The transmissibility form has tpfa_residual_vjp_trans. */
int tpfa_residual_vjp(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                      const tpfa_rock_t *rock, const tpfa_state_t *state,
                      tpfa_precision_t prec, const void *w, void *grad_p,
                      void *grad_logk, const tpfa_launch_t *launch, void *stream);

/* The residual r[ncell] (Algorithm 1, Eqs. 3-5) and the vector-Jacobian
   product of tpfa_residual_vjp in one pass over the grid: the value and the
   gradient of w.r, as an adjoint method needs them for a linear functional of
   the residual. r (required) is bitwise the r of tpfa_residual; grad_p and
   grad_logk (either may be NULL, not both) are bitwise those of
   tpfa_residual_vjp. One kernel reads p, k, seal and w once, and each
   face's flux serves both results (the two calls read the inputs twice and
   form each face's flux in both kernels). Permeability form with ry, rz
   ratios only (TPFA_ERR_UNSUPPORTED otherwise). */
int tpfa_residual_and_vjp(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                          const tpfa_rock_t *rock, const tpfa_state_t *state,
                          tpfa_precision_t prec, const void *w, void *r, void *grad_p,
                          void *grad_logk, const tpfa_launch_t *launch, void *stream);

/* Accumulation term of the full backward-Euler residual, Eq. (2):
     V_K (phi(p_K) rho(p_K) - phi(pn_K) rho(pn_K)) / dt,  V_K = dx dy dz,
   with rho from Eq. (5) and the porosity linear in pressure (Sec. 3 states
   that porosity depends linearly on p): phi(p) = phi_ref (1 + cr (p - p0)),
   p0 the fluid's reference pressure.
   phi    : phi_ref[ncell], device, dtype of the precision.
   p_prev : pressure of the previous time level [ncell], device, in the form
            of state->p (absolute FP64, or the FP32 offset from the same pref).
   dt     : time step (s), > 0 and finite; cr: rock compressibility (1/Pa). */
typedef struct {
  const void *phi;
  const void *p_prev;
  double dt;
  double cr;
} tpfa_accum_t;

/* Full backward-Euler residual of Eq. (2): the accumulation term above plus
   the flux sum of tpfa_residual. accum is required (TPFA_ERR_NULL), dt <= 0 or
   non-finite dt / cr give TPFA_ERR_PARAM. */
int tpfa_residual_be(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                     const tpfa_rock_t *rock, const tpfa_state_t *state,
                     const tpfa_accum_t *accum, tpfa_precision_t prec, void *r,
                     const tpfa_launch_t *launch, void *stream);

/* Its residual (r may be NULL) and 7-point Jacobian (layout of tpfa_jacobian);
   the accumulation derivative V/dt (phi_ref cr rho + phi cf rho) is on the
   diagonal. */
int tpfa_jacobian_be(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                     const tpfa_rock_t *rock, const tpfa_state_t *state,
                     const tpfa_accum_t *accum, tpfa_precision_t prec, void *r, void *J,
                     const tpfa_launch_t *launch, void *stream);

/* Matrix-free Jacobian-vector product jv = J v[ncell] (the operator a
   Newton-Krylov solver of Eq. (2) applies; the paper names such an operator as
   its next step, Sec. 8), without forming or storing J: the flux Jacobian of
   tpfa_jacobian, plus the accumulation diagonal when accum is not NULL. The
   residual is written too when r is not NULL (the flux residual, or the
   backward-Euler residual with accum). v and jv are device arrays of the
   precision's dtype; in the FP32 form v is a direction in dp. */
int tpfa_jvp(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, const tpfa_rock_t *rock,
             const tpfa_state_t *state, const tpfa_accum_t *accum, tpfa_precision_t prec,
             const void *v, void *jv, void *r, const tpfa_launch_t *launch, void *stream);

/* Vector-Jacobian product in the transmissibility form (rock->tx, ty, tz
   given; TPFA_ERR_UNSUPPORTED otherwise): grad_p = J^T w as in
   tpfa_residual_vjp, and grad_logt[3][ncell] with grad_logt[a][idx] =
   d(w.r)/d ln T of the face between idx and its +a neighbour (a = x, y, z;
   0 where that face does not exist), i.e. (w_idx - w_nb) F of that face,
   since F is linear in T. Either output may be NULL (not both). */
int tpfa_residual_vjp_trans(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                            const tpfa_rock_t *rock, const tpfa_state_t *state,
                            tpfa_precision_t prec, const void *w, void *grad_p,
                            void *grad_logt, const tpfa_launch_t *launch, void *stream);

/* Residual of the 10-flux stencil: the six faces above plus the four in-plane
   diagonal faces that the paper's kernel also evaluates (Sec. 3, Algorithm 1
   applied with four extra neighbours), whose transmissibilities the caller
   supplies: tne[idx] for the face (i,j)-(i+1,j+1) and tse[idx] for the face
   (i,j)-(i+1,j-1) (dtype of the precision; entries without that neighbour are
   ignored). Diagonal faces have no elevation difference and no seal bit (a zero
   transmissibility closes one). Residual only. */
int tpfa_residual10(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid,
                    const tpfa_rock_t *rock, const tpfa_state_t *state,
                    tpfa_precision_t prec, const void *tne, const void *tse, void *r,
                    const tpfa_launch_t *launch, void *stream);

/* Discrete hydrostatic reference column (double pref[nz], device): pref[0] =
   p_top and pref[k+1] - pref[k] = (rho(pref[k]) + rho(pref[k+1]))/2 * gk * dz,
   i.e. the profile whose vertical potential differences (Eq. 3b) vanish. The
   offset reference of the precision form. One small kernel on `stream`. */
int tpfa_hydrostatic(const tpfa_grid_t *grid, const tpfa_fluid_t *fluid, double p_top,
                     double *pref, void *stream);

/* Precision-form state from an FP64 pressure: dp[idx] = (float)(p[idx] - pref[k])
   for every cell (padding is not touched). */
int tpfa_offset_pressure(const tpfa_grid_t *grid, const double *p, const double *pref,
                         float *dp, void *stream);

/* ---- Bandwidth probe ---- */

/* The memory traffic of the Jacobian entry points without their arithmetic
   and without their halo, to measure the bandwidth the device reaches on that
   access pattern (the streaming measurement beside the roofline, as in the
   paper's Roofline analysis, Sec. 7): for every cell idx of `grid` (row pitch
   grid->ldx), out[q * ldx*ny*nz + idx] = p[idx] + (q + seal[idx]) * k[idx],
   q = 0..7, with p, k and out of the precision's type (double or float; 8 + 8
   + 1 bytes read and 64 written per cell in FP64, 4 + 4 + 1 and 32 in FP32).
   It marches 128 x 8 column blocks through 32-plane chunks with two x cells
   per lane (16-byte accesses in FP64 where the pitch is even and the pointers
   aligned), coalesced, with non-temporal stores: of the patterns measured on
   MI355X for this traffic, the fastest. Device pointers owned by the caller;
   padding cells are neither read nor written. Errors: the grid checks of the other calls,
   TPFA_ERR_PARAM (precision), TPFA_ERR_NULL, TPFA_ERR_HIP. */
int tpfa_stream_probe(const tpfa_grid_t *grid, tpfa_precision_t prec, const void *p,
                      const void *k, const uint8_t *seal, void *out, void *stream);

/* The same probe with the eight outputs in the layout of TPFA_LAUNCH_SLICED:
   output q of cell (i, j, k) at element (((k ny + j) S + i / 64) 8 + q) 64 +
   i % 64 of out (S = ceil(nx / 64), nz ny S 512 elements; lanes beyond nx are
   not written). TPFA_ERR_SHAPE where one z plane of out holds 2^32 bytes or
   more; the other errors as tpfa_stream_probe. It marches 64 x 8 column
   blocks with one cell per lane, each lane's eight stores falling in the eight
   runs of one slice: on this layout that pattern measured faster than two
   cells per lane. */
int tpfa_stream_probe_sliced(const tpfa_grid_t *grid, tpfa_precision_t prec, const void *p,
                             const void *k, const uint8_t *seal, void *out, void *stream);

/* ---- Batched ensemble: many independent grids in one persistent launch ---- */

/* One member of an ensemble. All pointers are device pointers that must stay
   valid while the batch is used; r may be NULL; J is required for
   TPFA_BATCH_JACOBIAN and ignored for TPFA_BATCH_RESIDUAL. launch.tile is -1
   (default: the single-grid default tile, or 64x4 where that default is a
   512-thread tile), one of the tiles the ensemble kernels hold: 0, 1, 2
   (64x4, 32x8, 16x16), or TPFA_TILE_FIT; any other tile gives TPFA_ERR_TILE.
   TPFA_TILE_FIT fits a tile of tx x ty cells (256 threads) to the member: tx
   the row length of the fewest tiles of at most 64 cells covering a row, in
   near-equal parts (at least 8), ty the most rows that 256 threads hold,
   balanced over the rows; members whose rows are not a multiple of 64 cells
   then leave fewer lanes idle than with a fixed tile. */
#define TPFA_TILE_FIT 10
typedef struct {
  tpfa_grid_t grid;
  tpfa_fluid_t fluid;
  tpfa_rock_t rock;
  tpfa_state_t state;
  void *r;
  void *J;
  tpfa_launch_t launch;
} tpfa_model_t;

typedef enum { TPFA_BATCH_RESIDUAL = 0, TPFA_BATCH_JACOBIAN = 1 } tpfa_batch_mode_t;

typedef struct tpfa_batch tpfa_batch_t; /* opaque */

/* Builds the work list (one item per tile and z-chunk of every model, models
   in the given order, each in z-chunk, tile-row, tile order) and the model
   table on the device (the batch owns these two device buffers and a block
   of work counters), and captures the launch into a HIP graph: a one-
   workgroup kernel that zeroes the work counters, then the persistent
   kernel.
   `stream` orders the uploads. */
int tpfa_batch_create(const tpfa_model_t *models, int n_models, tpfa_precision_t prec,
                      tpfa_batch_mode_t mode, tpfa_batch_t **out, void *stream);

/* Replays the captured graph on `stream`: all models, one persistent launch.
   Runs of one batch share its work counters (zeroed at the start of each
   run), so they must not overlap: never run one
   batch on two streams at once without ordering the runs (e.g. with an
   event). Different batches are independent. */
int tpfa_batch_run(tpfa_batch_t *batch, void *stream);

/* The same persistent kernel launched directly, without the graph. */
int tpfa_batch_run_eager(tpfa_batch_t *batch, void *stream);

/* How the one launch of a batch covers its work list, cut into 8
   contiguous bands, one per XCD (so that neighbouring tiles share an L2):
   TPFA_SCHEDULE_PERSISTENT (default): one workgroup per CU slot, taking work
   items from its XCD's band (a device counter per band), then from the other
   bands once that one is drained, until the list is drained;
   TPFA_SCHEDULE_GROUPED: one workgroup per work item, dispatched by the
   hardware. Re-captures the batch's graph; results are identical. */
#define TPFA_SCHEDULE_PERSISTENT 0
#define TPFA_SCHEDULE_GROUPED 1
int tpfa_batch_set_schedule(tpfa_batch_t *batch, int schedule);

/* Number of work items and of persistent workgroups of a batch. */
int tpfa_batch_info(const tpfa_batch_t *batch, int64_t *n_items, int *n_workgroups);

/* Frees the batch's device buffers and graph after waiting for the batch's
   last run (an event recorded by every run; other work on the device is not
   waited for). NULL is accepted. */
void tpfa_batch_destroy(tpfa_batch_t *batch);

/* ---- Ensemble run that allocates nothing ---- */

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   ensemble of tpfa_batch_create + tpfa_batch_run in one call that allocates
   nothing. The model table and each model's first work item are written into
   a fixed-size device array of the library (at most 256 models, 256 * 448 +
   257 * 8 bytes, about 114 KB; each GPU the library runs on holds its own
   copy until the process ends) by small upload launches on `stream`, then
   one grouped launch (one workgroup per work item, as
   TPFA_SCHEDULE_GROUPED) runs every model: the kernels and the results are
   those of a batch of the same models. Models are checked as by
   tpfa_batch_create, all before anything is enqueued. Every call on a GPU
   shares that GPU's array and leaves the last call's table in it: calls that
   overlap on one GPU (on two streams, or from two threads without ordering)
   race. Errors: those of tpfa_batch_create, and TPFA_ERR_SHAPE for more than
   256 models. */
int tpfa_ensemble_run_noalloc(const tpfa_model_t *models, int n_models, tpfa_precision_t prec,
                              tpfa_batch_mode_t mode, void *stream);

/* ---- Introspection ---- */

/* Operations of the single-grid entry points, for tpfa_resolve_launch. */
typedef enum {
  TPFA_OP_RESIDUAL = 0,    /* tpfa_residual */
  TPFA_OP_JACOBIAN = 1,    /* tpfa_jacobian */
  TPFA_OP_VJP = 2,         /* tpfa_residual_vjp, tpfa_residual_vjp_trans */
  TPFA_OP_RESIDUAL10 = 3,  /* tpfa_residual10 */
  TPFA_OP_RESIDUAL_BE = 4, /* tpfa_residual_be */
  TPFA_OP_JACOBIAN_BE = 5, /* tpfa_jacobian_be */
  TPFA_OP_JVP = 6,         /* tpfa_jvp without accum */
  TPFA_OP_JVP_BE = 7       /* tpfa_jvp with accum */
} tpfa_op_t;

/* The launch that a call of operation `op` with this grid, precision, rock
   form and launch argument would make, written to *resolved: tile id,
   z planes per workgroup (as run: at most nz), flags (the XCD band order
   included where the defaults set it) and row range [y_begin, y_end).
   Of `rock` only which arrays are given is read (it decides the form);
   nothing is dereferenced on the device and nothing is enqueued. Errors:
   TPFA_ERR_NULL (grid, rock or resolved NULL), the grid and launch checks of
   the calls, TPFA_ERR_PARAM for an unknown op or precision. */
int tpfa_resolve_launch(const tpfa_grid_t *grid, int op, tpfa_precision_t prec,
                        const tpfa_rock_t *rock, const tpfa_launch_t *launch,
                        tpfa_launch_t *resolved);

/* Number of compiled tile shapes; shape of tile `id`: TX x TY cells per
   workgroup plane and the workgroup size in threads. */
int tpfa_num_tiles(void);
int tpfa_tile_shape(int id, int *tx, int *ty, int *threads);
/* Shape of the fitted tile (TPFA_TILE_FIT, ensemble members only) for rows of
   nx cells and `rows` rows: tx x ty cells on 256 threads (tx ty <= 256).
   Errors: TPFA_ERR_SHAPE (nx or rows <= 0), TPFA_ERR_NULL. */
int tpfa_fit_tile_shape(int64_t nx, int64_t rows, int *tx, int *ty);

const char *tpfa_strerror(int code);
const char *tpfa_last_error(void);
int tpfa_version(void); /* TPFA_VERSION of the library's build */

#ifdef __cplusplus
}
#endif

#endif /* TPFA_H */
