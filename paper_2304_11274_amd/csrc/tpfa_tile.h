// The tile body of the HIP kernels for the TPFA flux residual, its Jacobian,
// vector-Jacobian and Jacobian-vector products on gfx950 (MI355X).
//
// Equations (paper Sec. 3): density Eq. (5), flux and potential difference
// Eq. (3a)/(3b) (outflow orientation dPhi_KL = Phi_K - Phi_L), single-point
// upwinding Eq. (4) with ties given to the lower linear index, residual
// assembly of Algorithm 1 (sum of the fluxes of a cell's face neighbours);
// optionally the accumulation term of the backward-Euler residual Eq. (2),
// the four in-plane diagonal faces the paper also computes, and face
// transmissibilities given as inputs instead of computed from k.
//
// Design. The path is a radius-1 stencil whose HBM traffic is fixed by its
// inputs (p, k, seal) and outputs (r and seven Jacobian planes), so nothing
// here is a dense contraction and nothing uses MFMA. A workgroup owns a
// TX x TY block of (i, j) columns and marches it through a chunk of z planes:
//  * every thread owns one column; the cell above and below stay in registers,
//    the -z face of plane k is the +z face it computed at plane k-1, and the
//    plane k+2 values are prefetched while plane k is computed;
//  * the x-y neighbours come from LDS: each plane (p, k, mobility, seal bits)
//    is staged with a one-cell halo ring, double buffered, one barrier per
//    plane; halo threads compute the density of their halo cell, interior
//    threads the density of their own cell, so each exp is evaluated once per
//    cell per workgroup;
//  * loads and stores are x-fastest and coalesced (a 64-lane wave covers
//    64 consecutive x cells when TX = 64; rows are ldx >= nx cells apart);
//    outputs are written once, with non-temporal stores, or ordinary ones in
//    the FP32 kernels where rows are off 128-byte lines;
//  * optionally, the tiles of each z chunk are split into one band of tile
//    rows per XCD, so that halo lines are shared within one L2.
// One tile body, specialised per mode at compile time, serves every entry
// point, the persistent ensemble kernel and the grouped one. The cell-gather
// form writes only owned cells: no atomics, deterministic, and every launch
// shape gives bit-identical results.
//
// Precision. FP64: every quantity in double; the flux of each face is formed
// as (Ups * lambda) * dPhi with Ups = (2 a k_Lo) * (k_Up * (1 / (k_Lo + k_Up)))
// and a reciprocal accurate to about one ulp, so every result agrees with the
// definition's evaluation order to about 1e-16 relative. FP32 precision form:
// a cell's density is split into the reference density of its plane,
// rho_k = rho0 exp(cf (pref[k] - p0)) (FP64, once per plane and workgroup),
// and a float deviation d = rho_k (exp(cf dp) - 1) from a series that has no
// cancellation. The z-face potential difference is then
//   [(pref[k] - pref[k+1]) + (rho_k + rho_k+1) G / 2]  (FP64 per-plane constant)
//   + (dp_Lo - dp_Up) + (d_Lo + d_Up) G / 2,
// whose large terms cancel inside the FP64 constant, so its error is
// relative to the deviations, not to rho G dz; it decides the upwind cell in
// FP64. x-y faces subtract offsets of one plane in float (whose sign is exact,
// so the upwind choice is the FP64 one); transmissibility, density, mobility,
// the flux/derivative products, the Jacobian diagonal and the six terms of
// each gradient are FP32; the residual and J v are accumulated in FP64 and
// rounded once on store.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tpfa_internal.h"

namespace tpfa {

// ----------------------------------------------------------------------------
// Per-precision cell quantities
// ----------------------------------------------------------------------------

// One cell as loaded from HBM.
template <class S>
struct Cell {
  S p;         // stored pressure value (absolute for FP64, offset from pref for FP32)
  S k;         // kx
  S w;         // cotangent w (VJP) or direction v (JVP) of the product modes
  S tn, ts;    // diagonal transmissibilities (10-flux stencil only)
  S phi, pn;   // reference porosity and previous-level pressure (backward-Euler modes)
  S tx, ty, tz;  // transmissibilities of the +x, +y, +z faces (transmissibility input)
  S ky, kz;    // y and z permeabilities (per-direction form; k holds kx)
  uint32_t s;  // seal bits
};

// Density-derived quantities of a cell, evaluated once per cell.
template <class S>
struct Props {
  S rho;  // density, Eq. (5)
  S lam;  // mobility rho / mu
  S dv;   // FP32 form: rho minus the plane's reference density (0 in FP64)
};

// exp(x) - 1 in float without the cancellation of exp(x) - 1 near 0: for
// |x| < 1/8 its Taylor series through x^6 / 720 (truncation below 1e-9
// relative), otherwise the hardware exponential (relative error then a few
// 1e-7, as for the density itself). The second case needs |dp| above 1e8 Pa
// at the workloads' compressibility, so the exponential is evaluated only
// when a lane of the wave needs it (a wave-uniform branch).
__device__ __forceinline__ float expm1_series(float x) {
  float c = fmaf(x, 1.0f / 720.0f, 1.0f / 120.0f);
  c = fmaf(x, c, 1.0f / 24.0f);
  c = fmaf(x, c, 1.0f / 6.0f);
  c = fmaf(x, c, 0.5f);
  c = fmaf(x, c, 1.0f);
  float m = x * c;
  const bool big = !(fabsf(x) < 0.125f);
  if (__builtin_amdgcn_ballot_w64(big) != 0) {
    asm volatile("");  // keeps the exponential inside the branch (not speculated)
    const float e = __expf(x) - 1.0f;
    m = big ? e : m;
  }
  return m;
}

// Eq. (5). FP64: rho0 exp(cf (p - p0)). FP32 form: rho = rho_k (1 + m) with the
// plane's reference density rho_k (rounded to float; FP64 where z faces need
// it) and m = exp(cf dp) - 1, so the deviation d = rho_k m carries no rounding
// of rho itself.
__device__ __forceinline__ Props<double> props(double p, double, const Args &a) {
  Props<double> q;
  q.rho = a.rho0 * exp(a.cf * (p - a.p0));
  q.lam = q.rho * a.inv_mu;
  q.dv = 0.0;
  return q;
}
__device__ __forceinline__ Props<float> props(float dp, float rk, const Args &a) {
  Props<float> q;
  const float m = expm1_series(a.cff * dp);
  q.dv = rk * m;
  q.rho = fmaf(rk, m, rk);
  q.lam = q.rho * a.inv_muf;
  return q;
}

// 1/x to about one ulp: hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// One face between a lower-index cell (Lo) and an upper-index cell (Up):
// F = F_{Lo,Up} (outflow of Lo), its pressure derivatives, and for the
// vector-Jacobian product the permeability weights k_Lo/(k_Lo+k_Up),
// k_Up/(k_Lo+k_Up) that give d Ups / d ln k.
template <class C>
struct Face {
  C F, dLo, dUp, qLo, qUp;
  C w;  // z faces: w or v of the lower cell (product modes only)
};

// Transmissibility 2 a r k_Lo k_Up / (k_Lo + k_Up) (A2 = 2 a r), closed when
// the face is sealed or k_Lo + k_Up = 0.
template <bool VJP>
__device__ __forceinline__ double trans64(double A2, double kLo, double kUp, bool open,
                                          Face<double> &f) {
  // k_Lo + k_Up = 0 (both cells impermeable or outside the domain) gives T = 0:
  // the sum is raised to the smallest normal number, which leaves every sum of
  // normal permeabilities unchanged and turns 0 * (1/0) into 0 * finite
  const double ks = fmax(kLo + kUp, 2.2250738585072014e-308);
  const double inv = rcp64(ks);
  if (VJP) {
    f.qLo = kLo * inv;
    f.qUp = kUp * inv;
  }
  const double T = (A2 * kLo) * (kUp * inv);
  return open ? T : 0.0;
}
template <bool VJP>
__device__ __forceinline__ float trans32(float A2, float kLo, float kUp, bool open,
                                         Face<float> &f) {
  const float ks = fmaxf(kLo + kUp, 1.17549435e-38f);
  const float inv = __builtin_amdgcn_rcpf(ks);
  const float qUp = kUp * inv;
  if (VJP) {
    f.qLo = kLo * inv;
    f.qUp = qUp;
  }
  const float T = (A2 * kLo) * qUp;
  return open ? T : 0.0f;
}

// Upwinded flux and derivatives from T, the potential difference and the
// pressure derivatives gLo = dPhi/dp_Lo, gUp = dPhi/dp_Up (1 and -1 on x/y
// faces). The upwind mobility is lambda_Lo when dPhi >= 0 (a tie goes to the
// lower index), and its pressure derivative is cf * lambda.
template <class C, bool DERIV, bool GRAV>
__device__ __forceinline__ void upwind(Face<C> &f, C T, C dphi, bool up, C lamLo, C lamUp,
                                       C cf, C gLo, C gUp) {
  const C lam = up ? lamLo : lamUp;
  const C TL = T * lam;
  f.F = TL * dphi;
  if (DERIV) {
    const C t = (cf * lam) * dphi;
    const C tLo = up ? t : C(0);
    const C tUp = t - tLo;
    if (GRAV) {
      f.dLo = fma(TL, gLo, T * tLo);
      f.dUp = fma(TL, gUp, T * tUp);
    } else {
      f.dLo = fma(T, tLo, TL);
      f.dUp = fma(T, tUp, -TL);
    }
  }
}

// x or y face (no elevation difference).
template <bool DERIV, bool VJP>
__device__ __forceinline__ Face<double> face_h(const Args &a, double A2, double kLo, double kUp,
                                               bool open, double pLo, double pUp, double lamLo,
                                               double lamUp) {
  Face<double> f;
  const double T = trans64<VJP>(A2, kLo, kUp, open, f);
  const double dphi = pLo - pUp;
  upwind<double, DERIV, false>(f, T, dphi, dphi >= 0.0, lamLo, lamUp, a.cf, 1.0, -1.0);
  return f;
}
// FP32 form: both cells lie in the same plane, so dPhi = dp_Lo - dp_Up and
// the sign of the rounded float difference is exact: the upwind choice is the
// one FP64 makes.
template <bool DERIV, bool VJP>
__device__ __forceinline__ Face<float> face_h(const Args &a, float A2, float kLo, float kUp,
                                              bool open, float pLo, float pUp, float lamLo,
                                              float lamUp) {
  Face<float> f;
  const float T = trans32<VJP>(A2, kLo, kUp, open, f);
  const float dphi = pLo - pUp;
  upwind<float, DERIV, false>(f, T, dphi, dphi >= 0.0f, lamLo, lamUp, a.cff, 1.0f, -1.0f);
  return f;
}

// x or y face with a given transmissibility (transmissibility input).
template <bool DERIV, class S>
__device__ __forceinline__ Face<S> face_ht(const Args &a, S T, S pLo, S pUp, S lamLo, S lamUp) {
  Face<S> f;
  const S dphi = pLo - pUp;
  const S cf = sizeof(S) == 8 ? S(a.cf) : S(a.cff);
  upwind<S, DERIV, false>(f, T, dphi, dphi >= S(0), lamLo, lamUp, cf, S(1), S(-1));
  return f;
}

// z face between planes k (Lo) and k+1 (Up): dPhi = (p_Lo - p_Up) + rho_avg G.
// FP32 form: `hk` = (pref[k] - pref[k+1]) + (rho_k + rho_k+1) G / 2 in FP64
// (zero up to rounding for a hydrostatic pref), plus the offsets' difference
// and the density deviations' share of rho_avg G, all summed in FP64.
__device__ __forceinline__ double zpot(double pLo, double pUp, double, const Props<double> &Lo,
                                       const Props<double> &Up, const Args &a) {
  const double ra = 0.5 * (Lo.rho + Up.rho);
  return fma(ra, a.G, pLo - pUp);
}
__device__ __forceinline__ double zpot(float pLo, float pUp, double hk, const Props<float> &Lo,
                                       const Props<float> &Up, const Args &a) {
  const float dg = (Lo.dv + Up.dv) * a.hgf;
  return (hk + ((double)pLo - (double)pUp)) + (double)dg;
}

template <bool DERIV, bool VJP, class S>
__device__ __forceinline__ Face<S> face_z(const Args &a, S kLo, S kUp, bool open, S pLo, S pUp,
                                          double hk, Props<S> Lo, Props<S> Up,
                                          bool tin = false, S Tin = S(0)) {
  Face<S> f;
  S T;
  if (tin)
    T = open ? Tin : S(0);
  else if constexpr (sizeof(S) == 8)
    T = trans64<VJP>(a.a2z, kLo, kUp, open, f);
  else
    T = trans32<VJP>(a.a2zf, kLo, kUp, open, f);
  const double dphi = zpot(pLo, pUp, hk, Lo, Up, a);
  const S hc = sizeof(S) == 8 ? S(a.hc) : S(a.hcf);
  const S cf = sizeof(S) == 8 ? S(a.cf) : S(a.cff);
  upwind<S, DERIV, true>(f, T, (S)dphi, dphi >= 0.0, Lo.lam, Up.lam, cf, fma(hc, Lo.rho, S(1)),
                         fma(hc, Up.rho, S(-1)));
  return f;
}

// FP32 vector-Jacobian product (permeability-ratio form), one in-plane face
// seen from the own cell C towards its neighbour N. With q_N = k_N / (k_C + k_N)
// the transmissibility is T = A2 k_C q_N, and with D = dp_C - dp_N and the
// upwind mobility lam_u,
//   F_CN = T lam_u D,   dF_CN/dp_C = T lam_u (1 + cf D) if C is upwind, else T lam_u,
//   dF_CN/d ln k_C = F_CN q_N.
// Both gradient terms carry the cotangent difference dw = w_C - w_N and the
// factor A2 k_C, which is applied once per cell and axis: gp and gm receive
// the terms divided by it. C_LO: C is the face's lower cell (its +x / +y face),
// so a tie D = 0 makes C upwind; otherwise N is upwind at a tie.
// WITH_F: also the face's flux F_Lo,Up (outflow of its lower cell) with the
// operands and operation order of the two-sided form (face_h), so that a
// residual summed from it is bitwise the residual kernels'.
template <bool C_LO, bool WITH_F = false>
__device__ __forceinline__ void vjp_face_own(float kC, float kN, bool open, float pC, float pN,
                                             float lamC, float lamN, float dw, float cf,
                                             float &gp, float &gm, float A2 = 0.0f,
                                             float *F = nullptr) {
  const float D = pC - pN;
  const float ks = fmaxf(kC + kN, 1.17549435e-38f);
  const float inv = __builtin_amdgcn_rcpf(ks);
  const float qN = kN * inv;
  const bool upC = C_LO ? D >= 0.0f : D > 0.0f;
  const float lu = upC ? lamC : lamN;
  const float X0 = (qN * lu) * dw;
  const float X = open ? X0 : 0.0f;
  gp = fmaf(X, upC ? fmaf(cf, D, 1.0f) : 1.0f, gp);
  gm = fmaf(X * D, qN, gm);
  if constexpr (WITH_F) {
    // T = (A2 k_Lo) (k_Up / (k_Lo + k_Up)), dPhi = p_Lo - p_Up
    const float T = C_LO ? (A2 * kC) * qN : (A2 * kN) * (kC * inv);
    *F = ((open ? T : 0.0f) * lu) * (C_LO ? D : pN - pC);
  }
}

// Global-address-space views of the argument pointers: the ensemble kernel
// reads them from its model table, where the compiler cannot infer the address
// space and would otherwise emit flat (generic) memory instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T *;

// Output store: non-temporal, or ordinary with the MODE_PLAIN flag. Where the
// rows of a grid do not start on 128-byte lines, the line at a tile's x edge
// is shared with the neighbouring tile; ordinary stores let the two parts meet
// in L2 before the line is written back, which measured much faster on MI355X
// for the FP32 kernels (a 64-cell FP32 row touches three lines, two of them
// partial) and slower for FP64 (five lines, two partial).
template <int MODE, class T>
__device__ __forceinline__ void st_out(T *p, T v) {
  if constexpr (has_plain_stores(MODE))
    *(gptr<T>)p = v;
  else
    __builtin_nontemporal_store(v, (gptr<T>)p);
}

// LDS of one workgroup (gfx950: 160 KiB per CU, all of it addressable by one
// workgroup).
constexpr int kMaxLds = 160 * 1024;

// Residual-only modes evaluate every in-plane face once, in its lower cell,
// and hand the flux to the upper cell through LDS: two buffers of the plane of
// p, k, mobility and of the +x, +y (and +x+y, +x-y) face fluxes. An FP64 face
// costs a double reciprocal with two Newton steps, so sharing saves more than
// the extra LDS traffic costs. In FP32 it pays for the six-face residual
// (512x512x256: 0.301 -> 0.287 ms; the kernel is VALU-bound) but not for the
// 10-flux stencil, whose two extra shared diagonal fluxes cost more LDS
// traffic than their arithmetic (750x994x246: 1.07 -> 1.18 ms): that one
// keeps the two-sided form in FP32.
template <class S, int MODE, int TX, int TY>
constexpr int share_lds_bytes() {
  return 2 * (TX + 2) * (TY + 2) * (int)sizeof(S) * (mode_kind(MODE) == MODE_RES10 ? 7 : 5);
}
template <class S, int MODE, int TX, int TY>
constexpr bool tile_shares() {
  return TX > 0 &&
         (base_mode(MODE) == MODE_RESIDUAL || mode_kind(MODE) == MODE_RES10) &&
         (sizeof(S) == 8 || mode_kind(MODE) != MODE_RES10) &&
         !has_k3(MODE) && share_lds_bytes<S, MODE, TX, TY>() <= kMaxLds;
}

// The fitted tile of the ensemble kernels (TX = TY = 0 in the templates): its
// shape comes from the model's arguments (dtx x dty, 8 <= dtx <= 64,
// dtx dty <= 256, 2 (dtx + dty) + 4 <= 256 so that one halo cell per thread
// covers the ring) and runs on 256 threads. Its LDS planes hold the largest
// such (dtx + 2)(dty + 2), plus one spare slot that idle threads stage into.
constexpr int dyn_max_hw() {
  int m = 0;
  for (int tx = kDynMinTx; tx <= kDynMaxTx; ++tx) {
    int ty = 256 / tx;
    if (2 * (tx + ty) + 4 > 256) ty = (256 - 4) / 2 - tx;
    const int hw = (tx + 2) * (ty + 2);
    m = hw > m ? hw : m;
  }
  return m + 1;
}
constexpr int kDynHW = dyn_max_hw();

// FP32 form: per-plane constants of the chunk (planes kb-1 .. kb+chunk), at
// the start of the tile's LDS: the hydrostatic part of each z face's potential
// difference (FP64) and each plane's reference density (float).
constexpr int kPlaneSlots = kMaxChunk32 + 2;
template <class S>
constexpr int plane_lds_bytes() {
  return sizeof(S) == 4 ? (kPlaneSlots * 12 + 15) / 16 * 16 : 0;
}

// Bytes of LDS one tile needs: two buffers of the (TX+2) x (TY+2) plane of
// p, k (or t_x), mobility, seal, plus w / v for the product modes, t_ne and
// t_se for the 10-flux stencil, t_y for the transmissibility form and k_y for
// the per-direction form, and the shared Jacobian faces; or the shared-face
// layout of the residual modes; after the FP32 form's per-plane constants.
// The FP32 Jacobian of the ratio form (and its backward-Euler variant) on
// 512-thread tiles also evaluates each in-plane face once, in its lower cell:
// F, dF/dp_Lo and dF/dp_Up go to LDS (one buffer of three values per
// direction) and the upper cell reads them after a second barrier in the
// plane. The face keeps the operands and operation order of the two-sided
// form, so the outputs are bitwise the same, with fewer VALU instructions
// (512x512x256, sliced outputs: 0.546 -> 0.535 ms). Only where the tile's LDS
// still lets four workgroups share a CU (64x8, 128x4, 32x16): the 256-thread
// tiles keep the two-sided form because the ensemble kernels size their LDS
// for the largest of them and six more plane arrays would cost those kernels
// a wave per SIMD, and the 256x2 and 512x1 tiles because theirs would.
template <class S, int MODE, int TX, int TY>
constexpr bool jacobian_shares() {
  constexpr int HW = (TX + 2) * (TY + 2);
  return sizeof(S) == 4 && TX * TY == 512 && base_mode(MODE) == MODE_JACOBIAN &&
         !has_trans(MODE) && !has_k3(MODE) &&
         4 * (plane_lds_bytes<S>() + 2 * HW * (3 * (int)sizeof(S) + 1) + 6 * HW * (int)sizeof(S)) <=
             kMaxLds;
}

template <class S, int MODE, int TX, int TY>
constexpr int tile_lds_bytes() {
  constexpr int HW = TX > 0 ? (TX + 2) * (TY + 2) : kDynHW;
  constexpr int B = base_mode(MODE);
  constexpr int arrays = 3 + (B == MODE_VJP || B == MODE_JVP ? 1 : 0) +
                         (mode_kind(MODE) == MODE_RES10 ? 2 : 0) +
                         (has_trans(MODE) || has_k3(MODE) ? 1 : 0);
  return plane_lds_bytes<S>() + (tile_shares<S, MODE, TX, TY>()
                                     ? share_lds_bytes<S, MODE, TX, TY>()
                                     : 2 * HW * ((int)sizeof(S) * arrays + 1)) +
         (jacobian_shares<S, MODE, TX, TY>() ? 6 * HW * (int)sizeof(S) : 0);
}

// Lower-cell faces a halo cell evaluates for the tile in the shared-face form.
constexpr uint32_t kPX = 1, kPY = 2, kNE = 4, kSE = 8;

// Fields a staged cell needs beyond p: a halo cell serves only the faces it
// shares with the tile, so each side of the ring loads only what those faces
// read (the own cell loads everything).
constexpr uint32_t kNeedK = 1, kNeedSeal = 2, kNeedTx = 4, kNeedTy = 8, kNeedTn = 16,
                   kNeedTs = 32, kNeedW = 64, kNeedKy = 128, kNeedAll = 255;

// Fluxes of a plane whose residual is completed at the next plane: its own
// lower-cell faces (+x, +y, +x+y, +x-y) and its two z faces.
template <class S>
struct Pending {
  S fpx, fpy, fzm, fzp, fne, fse;
  double acc;  // accumulation term (backward-Euler residual)
};

// Accumulation term of the backward-Euler residual of one cell and its
// pressure derivative: V/dt (phi(p) rho(p) - phi(pn) rho(pn)) with
// phi(p) = phi_ref (1 + c_r (p - p0)), and V/dt (phi_ref c_r rho + phi c_f rho).
// FP32 form: p - p0 = x_k + dp with the plane offset x_k, the previous level's
// density from the plane's reference density rho_k as for the current one; the
// two masses are FP32 products and their difference is taken in FP64.
__device__ __forceinline__ void accumulation(const Args &a, const Cell<double> &c,
                                             const Props<double> &d, double, double,
                                             double &term, double &diag) {
  const double phi1 = c.phi * (1.0 + a.cr * (c.p - a.p0));
  const double phi0 = c.phi * (1.0 + a.cr * (c.pn - a.p0));
  const double rho0 = a.rho0 * exp(a.cf * (c.pn - a.p0));
  const double m1 = phi1 * d.rho, m0 = phi0 * rho0;
  term = a.vdt * (m1 - m0);
  diag = a.vdt * ((c.phi * a.cr) * d.rho + phi1 * (a.cf * d.rho));
}
__device__ __forceinline__ void accumulation(const Args &a, const Cell<float> &c,
                                             const Props<float> &d, float xk, float rk,
                                             double &term, float &diag) {
  const float phi1 = c.phi * (1.0f + a.crf * (xk + c.p));
  const float phi0 = c.phi * (1.0f + a.crf * (xk + c.pn));
  const float rho0 = props(c.pn, rk, a).rho;
  const float m1 = phi1 * d.rho, m0 = phi0 * rho0;
  term = a.vdt * ((double)m1 - (double)m0);
  diag = a.vdtf * ((c.phi * a.crf) * d.rho + phi1 * (a.cff * d.rho));
}

// ----------------------------------------------------------------------------
// The tile body: columns [bx*TX, bx*TX+TX) x [by*TY, by*TY+TY), planes
// [kb, min(kb + kz_chunk, nz)).
// ----------------------------------------------------------------------------

// A per-thread byte offset passed through an empty asm that depends on the
// plane index: the compiler can no longer hoist a 64-bit copy of it out of the
// plane loop, so it keeps one 32-bit register and addresses with the
// scalar-base + 32-bit-offset form. In the FP32 kernels this saves 8 to 19
// registers (the VJP 81 -> 67, two more waves per SIMD); in FP64 it measured
// slightly slower and is not used. With it, the plane's base address is also
// pinned to scalar registers, or the compiler adds plane offset and thread
// offset in 64-bit vector registers once for several arrays (six VALU
// instructions per plane in the FP32 residual).
__device__ __forceinline__ uint32_t per_plane(uint32_t boff, int k) {
  asm("" : "+v"(boff) : "s"(k));
  return boff;
}

// Uniform (scalar) base of plane k of an array plus a per-thread 32-bit byte
// offset (made opaque per plane with FRESH).
template <bool FRESH = false, class T>
__device__ __forceinline__ T at(const T *base, size_t plane_elems, int k, uint32_t boff) {
  if constexpr (FRESH) boff = per_plane(boff, k);
  const char *pb = reinterpret_cast<const char *>(base + (size_t)k * plane_elems);
  if constexpr (FRESH) asm("" : "+s"(pb));
  return *(gptr<const T>)(pb + boff);
}
template <class T>
__device__ __forceinline__ T *at_w(T *base, size_t elems, uint32_t boff) {
  char *pb = reinterpret_cast<char *>(base + elems);
  return reinterpret_cast<T *>(pb + boff);
}

// The FP32 vector-Jacobian product of the permeability-ratio form takes its
// in-plane faces in the own cell's orientation (vjp_face_own); every other
// mode forms the faces' Face values.
template <class S, int MODE>
constexpr bool vjp_own() {
  return sizeof(S) == 4 && base_mode(MODE) == MODE_VJP && !has_trans(MODE) && !has_k3(MODE);
}

// Accumulates and stores one cell's outputs from its six faces (neighbour
// order -x, +x, -y, +y, -z, +z; odd faces have the cell as their lower cell).
// In the backward-Euler modes the accumulation term comes first, as in Eq. (2).
// vo: with vjp_own, the in-plane gradient sums of vjp_face_own (pressure x, y,
// then ln k x, y), which replace faces 0-3.
template <class S, int MODE>
__device__ __forceinline__ void emit(const Args &a, int k, size_t plane, int nz, uint32_t cb,
                                     const Cell<S> &c0, const Props<S> &d0, S xk, S rk,
                                     const Face<S> (&f)[6], const S (&wn)[6],
                                     const S (&fd)[4], const S (&vo)[4]) {
  if constexpr (sizeof(S) == 4) cb = per_plane(cb, k);
  constexpr int BASE = base_mode(MODE);
  constexpr bool ACC = has_accumulation(MODE);
  const size_t ko = (size_t)k * plane;
  if constexpr (BASE == MODE_VJP) {
    // grad_p[C] = sum (w_C - w_N) dF_CN/dp_C, grad_logk[C] = sum (w_C - w_N) F_CN k_N/(k_C+k_N)
    // per-direction form: the faces of axis d feed the ln k_d gradient only.
    // FP64: terms and sums in FP64. FP32 form: float terms and float sums of
    // the six terms (error below about 6 ulp of the sum of their magnitudes);
    // with vjp_own the in-plane terms arrive summed per axis and are scaled by
    // the axis' A2 k_C here
    constexpr bool OWN = vjp_own<S, MODE>();
    S gp = S(0), gm = S(0), gq[3] = {S(0), S(0), S(0)};
    if constexpr (OWN) {
      const float sx = a.a2xf * c0.k, sy = a.a2yf * c0.k;
      gp = fmaf(sx, vo[0], sy * vo[1]);
      gm = fmaf(sx, vo[2], sy * vo[3]);
    }
#pragma unroll
    for (int n = OWN ? 4 : 0; n < 6; ++n) {
      if constexpr (sizeof(S) == 4) {
        const float d = (n & 1) ? c0.w - wn[n] : wn[n] - c0.w;
        const float tp = d * ((n & 1) ? f[n].dLo : f[n].dUp);
        const float tm = d * (f[n].F * ((n & 1) ? f[n].qUp : f[n].qLo));
        gp = gp + tp;
        if constexpr (has_k3(MODE))
          gq[n >> 1] = gq[n >> 1] + tm;
        else if constexpr (!has_trans(MODE))
          gm = gm + tm;
      } else {
        const double d = (double)c0.w - (double)wn[n];
        if (n & 1) {  // own cell is Lo
          gp = fma(d, (double)f[n].dLo, gp);
          if constexpr (has_k3(MODE))
            gq[n >> 1] = fma(d, (double)(f[n].F * f[n].qUp), gq[n >> 1]);
          else if constexpr (!has_trans(MODE))
            gm = fma(d, (double)(f[n].F * f[n].qUp), gm);
        } else {      // own cell is Up
          gp = fma(-d, (double)f[n].dUp, gp);
          if constexpr (has_k3(MODE))
            gq[n >> 1] = fma(-d, (double)(f[n].F * f[n].qLo), gq[n >> 1]);
          else if constexpr (!has_trans(MODE))
            gm = fma(-d, (double)(f[n].F * f[n].qLo), gm);
        }
      }
    }
    if (a.gp) st_out<MODE>(at_w(static_cast<S *>(a.gp), ko, cb), (S)gp);
    if constexpr (has_with_r(MODE)) {
      // the residual in the residual kernels' order and precision (the faces'
      // F are theirs, bit for bit)
      double r = 0.0;
#pragma unroll
      for (int n = 0; n < 6; ++n) r = (n & 1) ? r + (double)f[n].F : r - (double)f[n].F;
      st_out<MODE>(at_w(static_cast<S *>(a.r), ko, cb), (S)r);
    }
    if constexpr (has_k3(MODE)) {
      // d(w.r)/d ln kx, ln ky, ln kz of the own cell, three planes [x, y, z]
      if (a.gm) {
        const size_t nc = (size_t)nz * plane;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          st_out<MODE>(at_w(static_cast<S *>(a.gm), (size_t)d * nc + ko, cb), (S)gq[d]);
      }
    } else if constexpr (has_trans(MODE)) {
      // given T: d(w.r)/d ln T of the +x, +y, +z face (own cell is its lower
      // cell) is (w_C - w_N) F, stored as three planes [x, y, z]
      if (a.gm) {
        const size_t nc = (size_t)nz * plane;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int n = 2 * d + 1;
          const double g = ((double)c0.w - (double)wn[n]) * (double)f[n].F;
          st_out<MODE>(at_w(static_cast<S *>(a.gm), (size_t)d * nc + ko, cb), (S)g);
        }
      }
    } else if (a.gm) {
      st_out<MODE>(at_w(static_cast<S *>(a.gm), ko, cb), (S)gm);
    }
  } else {
    double acc = 0.0;
    S dacc = S(0);
    if constexpr (ACC) accumulation(a, c0, d0, xk, rk, acc, dacc);
    // r and J: planes of the arrays, or the runs of a sliced array (oplane,
    // orun); the other outputs always take planes
    const size_t oko = (size_t)k * (size_t)a.oplane;
    // residual in the neighbour order, accumulated in FP64
    if (BASE != MODE_JVP || a.r) {
      double r = acc;
#pragma unroll
      for (int n = 0; n < 6; ++n) r = (n & 1) ? r + (double)f[n].F : r - (double)f[n].F;
      if constexpr (mode_kind(MODE) == MODE_RES10) {
        // diagonals -x-y, +x+y, +x-y, -x+y: the cell is the upper index of the
        // first and third, the lower of the second and fourth
#pragma unroll
        for (int n = 0; n < 4; ++n) r = (n & 1) ? r + (double)fd[n] : r - (double)fd[n];
      }
      if (a.r) st_out<MODE>(at_w(static_cast<S *>(a.r), oko, cb), (S)r);
    }
    if constexpr (BASE == MODE_JACOBIAN) {
      S *J = static_cast<S *>(a.J);
      const size_t nc = (size_t)a.orun;
      S dg = dacc;
#pragma unroll
      for (int n = 0; n < 6; ++n) dg = (n & 1) ? dg + f[n].dLo : dg - f[n].dUp;
      st_out<MODE>(at_w(J, oko, cb), dg);
#pragma unroll
      for (int n = 0; n < 6; ++n)
        st_out<MODE>(at_w(J, (size_t)(n + 1) * nc + oko, cb), (n & 1) ? f[n].dUp : -f[n].dLo);
    }
    if constexpr (BASE == MODE_JVP) {
      // (J v)_C = dacc v_C + sum over faces of dF_CN/dp_C v_C + dF_CN/dp_N v_N,
      // each face's pair summed in S and the row accumulated in FP64
      double jv = ACC ? (double)(dacc * c0.w) : 0.0;
#pragma unroll
      for (int n = 0; n < 6; ++n) {
        const S dC = (n & 1) ? f[n].dLo : -f[n].dUp;
        const S dN = (n & 1) ? f[n].dUp : -f[n].dLo;
        jv = jv + (double)(dC * c0.w + dN * wn[n]);
      }
      st_out<MODE>(at_w(static_cast<S *>(a.jv), ko, cb), (S)jv);
    }
  }
}

// exp(x) in FP64 for the FP32 form's per-plane constants, with no constant
// other than 1: x is halved j times until |x| / 2^j <= 1/16, exp of that by
// its Taylor series through the 10th power in nested form
// 1 + y (1 + y/2 (1 + y/3 (...))) (truncation below 1e-18 relative), then
// squared j times (relative error about 2^j ulp; j = 0 for |x| < 1/32). The
// loops are kept rolled: inlined into the ensemble kernels' item loop, the
// constants of a library exponential were hoisted out of that loop and held
// in registers across the whole tile body.
__device__ __forceinline__ double exp_halving(double x) {
  const int j = max(0, __builtin_amdgcn_frexp_exp(x) + 4);
  const double y = __builtin_amdgcn_ldexp(x, -j);
  double t = 1.0;
#pragma unroll 1
  for (int i = 10; i >= 1; --i) t = fma(y * t, rcp64((double)i), 1.0);
#pragma unroll 1
  for (int i = 0; i < j; ++i) t = t * t;
  return t;
}

// FP32 form: the reference density rho_k = rho0 exp(cf (pref[k] - p0)) of planes
// kb-1 .. ke (slot k - kb + 1; rounded to float) and the FP64 constant of the
// z face (k, k+1), (pref[k] - pref[k+1]) + (rho_k + rho_k+1) G / 2. Threads
// tid, tid + nt, ... take one plane each.
__device__ __forceinline__ void fill_plane_constants(const Args &a, int kb, int ke, int nz,
                                                     int tid, int nt, float *s_rk,
                                                     double *s_hk) {
  const int np = ke - kb + 2;
  for (int q = tid; q < np; q += nt) {
    const int k = kb - 1 + q;
    float rkf = 0.0f;
    double h = 0.0;
    if (k >= 0 && k < nz) {
      const double pk = *((gptr<const double>)a.pref + k);
      const double r0 = a.rho0 * exp_halving(a.cf * (pk - a.p0));
      rkf = (float)r0;
      if (k + 1 < nz) {
        const double pk1 = *((gptr<const double>)a.pref + k + 1);
        const double r1 = a.rho0 * exp_halving(a.cf * (pk1 - a.p0));
        h = (pk - pk1) + (0.5 * (r0 + r1)) * a.G;
      }
    }
    s_rk[q] = rkf;
    s_hk[q] = h;
  }
}

template <class S, int MODE, int TX, int TY>
struct Tile {
  // TX = TY = 0: the fitted tile, its shape read from the arguments at run time
  static constexpr bool DYN = TX == 0;
  static constexpr int W = TX + 2, H = TY + 2, HW = DYN ? kDynHW : W * H;
  static constexpr int BASE = base_mode(MODE);
  static constexpr bool ACC = has_accumulation(MODE);
  static constexpr bool VJP = BASE == MODE_VJP;
  static constexpr bool JVP = BASE == MODE_JVP;
  static constexpr bool NEEDW = VJP || JVP;  // neighbours' w (VJP) or v (JVP) staged in LDS
  static constexpr bool DERIV = BASE == MODE_JACOBIAN || VJP || JVP;
  static constexpr bool FP32 = sizeof(S) == 4;

  static constexpr bool R10 = mode_kind(MODE) == MODE_RES10;
  static constexpr bool TIN = has_trans(MODE);  // transmissibilities are inputs
  static constexpr bool K3 = has_k3(MODE);      // per-direction permeability arrays
  static constexpr bool YF = TIN || K3;         // a y-face field is staged (t_y or k_y)
  static constexpr bool SHARE = tile_shares<S, MODE, TX, TY>();
  static constexpr bool JSHARE = jacobian_shares<S, MODE, TX, TY>();
  static constexpr int NT = DYN ? 256 : TX * TY;  // threads
  static constexpr int NH = 2 * (TX + TY) + (R10 ? 4 : 0);  // halo ring (corners: 10-flux only)
  static constexpr int HC = DYN ? 1 : (NH + NT - 1) / NT;  // halo cells staged per thread
  // Halo cells are loaded one plane ahead; the FP32 Jacobian (short planes,
  // few registers) loads them two planes ahead, which measured faster on
  // MI355X there and slower everywhere else.
  static constexpr bool HALO2 = FP32 && BASE == MODE_JACOBIAN;
  // Per-side halo loads (each side of the ring loads only the fields its faces
  // read) save memory traffic but cost predicated branches: on MI355X they pay
  // off for the FP64 Jacobian only.
  static constexpr bool PICK = !FP32 && BASE == MODE_JACOBIAN;

  const Args &a;
  S *s_p, *s_k, *s_l, *s_w, *s_tn, *s_ts;
  S *s_fx, *s_fy, *s_fne, *s_fse;  // shared-face fluxes (residual-only modes)
  S *s_yf;  // y-face field, two-sided layout only: t_y (transmissibility input; t_x is
            // staged in s_k) or k_y (per-direction form; k_x is staged in s_k)
  uint8_t *s_s;
  S *s_jx, *s_jy;  // shared Jacobian faces: F, dLo, dUp of each slot's +x / +y face
  double *s_hk;  // FP32 form: hydrostatic part of the z-face potential, planes kb-1 .. ke
  float *s_rk;   // FP32 form: reference density of planes kb-1 .. ke
  size_t plane;
  int nz, kb, ke;
  bool inside;         // the thread's cell lies in the grid (staged as a real cell)
  bool own;            // ... and in the launch's row range, or a pad lane: its outputs are written
  bool tnv, tsv;       // 10-flux: the own cell's +x+y / +x-y diagonal face exists
  bool txv, tyv;       // transmissibility input: the own cell's +x / +y face exists
  int ol;
  uint32_t cb, cs;     // byte offset of the own cell within a plane (S elements / seal bytes)
  uint32_t sb;         // byte offset of the own cell's outputs (a padding cell's, for pad lanes)
  bool hv[HC];         // halo cell q lies in the domain
  uint32_t hr[HC];     // shared faces: lower-cell faces halo cell q evaluates (kPX | kPY | kNE | kSE)
  uint32_t hn[HC];     // fields halo cell q loads (kNeed*)
  int hl[HC];          // its LDS slot, -1 if the thread stages no q-th halo cell
  uint32_t hb[HC], hs[HC];
  S A2x, A2y;
  int dtx, dty, dw, dhw;  // fitted tile: shape, LDS row width and plane stride

  // the tile's shape: compile-time constants, or the fitted tile's
  __device__ __forceinline__ int tx_() const { if constexpr (DYN) return dtx; else return TX; }
  __device__ __forceinline__ int ty_() const { if constexpr (DYN) return dty; else return TY; }
  __device__ __forceinline__ int w_() const { if constexpr (DYN) return dw; else return W; }
  __device__ __forceinline__ int hw_() const { if constexpr (DYN) return dhw; else return HW; }

  __device__ __forceinline__ Tile(const Args &a_, int bx, int by, int kb_, char *smem, int tid_)
      : a(a_) {
    if constexpr (DYN) {
      dtx = a.dtx;
      dty = a.dty;
      dw = dtx + 2;
      dhw = dw * (dty + 2) + 1;  // + the spare slot of idle threads
    }
    s_hk = reinterpret_cast<double *>(smem);
    s_rk = reinterpret_cast<float *>(s_hk + kPlaneSlots);
    smem += plane_lds_bytes<S>();
    // arrays of two plane buffers each, HW apart (the largest fitted plane for
    // the fitted tile, whose planes take hw_() slots)
    s_p = reinterpret_cast<S *>(smem);
    s_k = s_p + 2 * HW;
    s_l = s_k + 2 * HW;
    s_w = s_l + 2 * HW;
    s_tn = s_w + (NEEDW ? 2 * HW : 0);
    s_ts = s_tn + (R10 ? 2 * HW : 0);
    s_yf = s_ts + (R10 ? 2 * HW : 0);
    s_jx = s_yf + (YF ? 2 * HW : 0);
    s_jy = s_jx + 3 * HW;
    s_s = reinterpret_cast<uint8_t *>(s_jx + (JSHARE ? 6 * HW : 0));
    s_fx = s_l + 2 * HW;
    s_fy = s_fx + 2 * HW;
    s_fne = s_fy + 2 * HW;
    s_fse = s_fne + (R10 ? 2 * HW : 0);
    const int nx = a.nx, ny = a.ny;
    const uint32_t ldx = (uint32_t)a.ldx;  // row pitch of the arrays (>= nx)
    nz = a.nz;
    kb = kb_;
    ke = min(kb + a.kz_chunk, nz);
    plane = (size_t)a.plane;
    const int tid = tid_;
    const int TXv = tx_(), TYv = ty_(), Wv = w_();
    const int tx = tid % TXv, ty = tid / TXv;
    // threads beyond the fitted tile's cells own no cell (they stage halo
    // cells only, and their own value into a spare slot)
    const bool active = !DYN || ty < TYv;
    // tile rows start at the launch's first row y0; rows of the grid outside
    // [y0, y1) are read as neighbours (a halo) but not written
    const int jb = a.y0 + by * TYv;
    const int i = bx * TXv + tx, j = jb + ty;
    inside = active && i < nx && j < ny;
    own = inside && j < a.y1;
    // lanes in the row padding store zeros there where the caller allows it
    // (whole-line output rows), and so do the lanes of a row's last 64-cell
    // slice beyond nx with sliced outputs; their loads stay those of an absent
    // cell
    const int padx = a.slices ? a.slices * 64 : a.padw ? (int)ldx : nx;
    const bool pad_lane = active && i >= nx && i < padx && j < ny && j < a.y1;
    tnv = inside && i + 1 < nx && j + 1 < ny;
    txv = inside && i + 1 < nx;
    tyv = inside && j + 1 < ny;
    tsv = inside && i + 1 < nx && j >= 1;
    const uint32_t col = inside ? (uint32_t)j * ldx + (uint32_t)i : 0u;
    ol = active ? (ty + 1) * Wv + tx + 1 : hw_() - 1;
    cb = col * (uint32_t)sizeof(S);
    cs = col;
    // sliced outputs: slice i / 64 of row j, 8 runs of 64 cells
    sb = a.slices ? (((uint32_t)j * (uint32_t)a.slices + (uint32_t)(i >> 6)) * 512u +
                     (uint32_t)(i & 63)) * (uint32_t)sizeof(S)
         : pad_lane ? ((uint32_t)j * ldx + (uint32_t)i) * (uint32_t)sizeof(S)
                    : cb;
    own = own || pad_lane;
    // halo ring: bottom row, top row, left column, right column
#pragma unroll
    for (int q = 0; q < HC; ++q) {
      const int h = tid + q * NT;
      int hi = -1, hj = -1, l = -1;
      uint32_t role = 0;  // faces into the tile whose lower cell is this halo cell
      uint32_t need = 0;  // fields those faces (and the tile's faces towards it) read
      const int NHv = 2 * (TXv + TYv) + (R10 ? 4 : 0);
      if (h < TXv) {  // bottom row: +y (and +x+y) faces
        hi = bx * TXv + h;
        hj = jb - 1;
        l = h + 1;
        role = kPY | (R10 ? kNE : 0u);
        need = (K3 ? kNeedKy : kNeedK) | kNeedSeal | kNeedTy | kNeedTn | kNeedW;
      } else if (h < 2 * TXv) {  // top row: +x-y faces
        hi = bx * TXv + h - TXv;
        hj = jb + TYv;
        l = (TYv + 1) * Wv + h - TXv + 1;
        role = R10 ? kSE : 0u;
        need = (K3 ? kNeedKy : kNeedK) | kNeedTs | kNeedW;
      } else if (h < 2 * TXv + TYv) {  // left column: +x (and both diagonal) faces
        hi = bx * TXv - 1;
        hj = jb + h - 2 * TXv;
        l = (h - 2 * TXv + 1) * Wv;
        role = kPX | (R10 ? kNE | kSE : 0u);
        need = kNeedK | kNeedSeal | kNeedTx | kNeedTn | kNeedTs | kNeedW;
      } else if (h < 2 * TXv + 2 * TYv) {  // right column: none (the tile's lower cells)
        hi = bx * TXv + TXv;
        hj = jb + h - 2 * TXv - TYv;
        l = (h - 2 * TXv - TYv + 1) * Wv + TXv + 1;
        need = kNeedK | kNeedW;
      } else if (h < NHv) {  // corners (10-flux stencil)
        const int c = h - 2 * TXv - 2 * TYv;
        const int cx = c & 1, cy = c >> 1;
        hi = cx ? bx * TXv + TXv : bx * TXv - 1;
        hj = cy ? jb + TYv : jb - 1;
        l = (cy ? TYv + 1 : 0) * Wv + (cx ? TXv + 1 : 0);
        role = c == 0 ? kNE : c == 2 ? kSE : 0u;
        need = c == 0 ? kNeedTn : c == 2 ? kNeedTs : 0u;
      }
      hr[q] = SHARE || JSHARE ? role : 0u;
      hn[q] = need;
      hl[q] = l;
      hv[q] = l >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
      const uint32_t hcol = hv[q] ? (uint32_t)hj * ldx + (uint32_t)hi : 0u;
      hb[q] = hcol * (uint32_t)sizeof(S);
      hs[q] = hcol;
    }
    A2x = FP32 ? S(a.a2xf) : S(a.a2x);
    A2y = FP32 ? S(a.a2yf) : S(a.a2y);
  }

  // FP32 form: the per-plane constants of planes kb-1 .. ke (at most
  // kPlaneSlots: the host limits FP32 chunks to kMaxChunk32 planes), one plane
  // per thread, followed by a barrier.
  __device__ __forceinline__ void plane_constants(int tid) const {
    if constexpr (FP32) {
      fill_plane_constants(a, kb, ke, nz, tid, NT, s_rk, s_hk);
      __syncthreads();
    }
  }

  // A cell outside the domain reads the plane's first cell (any finite value)
  // and gets k = 0, which closes every face that touches it (T = 0).
  // Fields outside `need` keep their previous (finite) values; nothing reads them.
  __device__ __forceinline__ void load_at(Cell<S> &c, int k, bool ok, uint32_t b, uint32_t bs,
                                          uint32_t need = kNeedAll) const {
    c.p = at<FP32>(static_cast<const S *>(a.p), plane, k, b);
    if (TIN) {
      c.k = S(0);
      if (need & kNeedTx) c.tx = at<FP32>(static_cast<const S *>(a.tx), plane, k, b);
      if (need & kNeedTy) c.ty = at<FP32>(static_cast<const S *>(a.ty), plane, k, b);
    } else {
      if (need & kNeedK) {
        const S kx = at<FP32>(static_cast<const S *>(a.kx), plane, k, b);
        c.k = ok ? kx : S(0);
      }
      if (K3 && (need & kNeedKy)) {
        const S ky = at<FP32>(static_cast<const S *>(a.ky), plane, k, b);
        c.ky = ok ? ky : S(0);
      }
    }
    if (need & kNeedSeal) c.s = a.seal ? (uint32_t)at<FP32>(a.seal, plane, k, bs) : 0u;
    if (NEEDW && (need & kNeedW)) c.w = at<FP32>(static_cast<const S *>(a.w), plane, k, b);
    if (R10) {
      if (need & kNeedTn) c.tn = at<FP32>(static_cast<const S *>(a.tne), plane, k, b);
      if (need & kNeedTs) c.ts = at<FP32>(static_cast<const S *>(a.tse), plane, k, b);
    }
  }
  // A diagonal face exists when both its cells lie in the domain; otherwise its
  // transmissibility is staged as 0 (whatever the caller's array holds there).
  // A halo cell's tne / tse serve only faces towards tile cells, so the halo
  // cell's own presence decides; the own cell checks its (i+1, j+-1) partner.
  __device__ __forceinline__ void load(Cell<S> &c, int k) const {
    load_at(c, k, inside, cb, cs);
    if (TIN) {
      // a face with a cell outside the domain does not exist
      c.tx = txv ? c.tx : S(0);
      c.ty = tyv ? c.ty : S(0);
      const S tz = at<FP32>(static_cast<const S *>(a.tz), plane, k, cb);
      c.tz = inside ? tz : S(0);
    }
    // a lane without a cell (a padding lane) has closed z faces
    if (K3) {
      const S kz = at<FP32>(static_cast<const S *>(a.kz), plane, k, cb);
      c.kz = inside ? kz : S(0);
    }
    if (ACC) {
      // a lane without a cell (a padding lane) gets porosity 0: no accumulation
      const S phi = at<FP32>(static_cast<const S *>(a.phi), plane, k, cb);
      c.phi = inside ? phi : S(0);
      c.pn = at<FP32>(static_cast<const S *>(a.pprev), plane, k, cb);
    }
    if (R10) {
      c.tn = tnv ? c.tn : S(0);
      c.ts = tsv ? c.ts : S(0);
    }
  }
  __device__ __forceinline__ void load_halo(Cell<S> (&h)[HC], int k) const {
#pragma unroll
    for (int q = 0; q < HC; ++q)
      if (hl[q] >= 0) {
        load_at(h[q], k, hv[q], hb[q], hs[q], PICK ? hn[q] : kNeedAll);
        if (TIN) {
          h[q].tx = hv[q] ? h[q].tx : S(0);
          h[q].ty = hv[q] ? h[q].ty : S(0);
        }
        if (R10) {
          h[q].tn = hv[q] ? h[q].tn : S(0);
          h[q].ts = hv[q] ? h[q].ts : S(0);
        }
      }
  }

  // FP32 form: pref[k]; x_k = pref[k] - p0 for the porosity law of the
  // accumulation term; the plane's reference density rho_k and the FP64
  // constant of the z face (k, k+1) from the chunk's per-plane constants
  __device__ __forceinline__ double pr(int k) const { return *((gptr<const double>)a.pref + k); }
  __device__ __forceinline__ S xoff(int k) const { return FP32 ? (S)(pr(k) - a.p0) : S(0); }
  __device__ __forceinline__ S rk(int k) const { return FP32 ? (S)s_rk[k - kb + 1] : S(0); }
  __device__ __forceinline__ double hk(int k) const { return FP32 ? s_hk[k - kb + 1] : 0.0; }

  // The -z face of the chunk's first plane: face (kb-1, kb), own cell is Up.
  __device__ __forceinline__ Face<S> first_zface(const Cell<S> &cur, const Props<S> &dcur) const {
    Face<S> f{};
    if (kb > 0) {
      Cell<S> pr;
      load(pr, kb - 1);
      const Props<S> dp = props(pr.p, rk(kb - 1), a);
      f = face_z<DERIV, VJP>(a, K3 ? pr.kz : pr.k, K3 ? cur.kz : cur.k, (pr.s & 4u) == 0u,
                             pr.p, cur.p, hk(kb - 1), dp, dcur, TIN, pr.tz);
      f.w = pr.w;
    }
    return f;
  }

  // Shared Jacobian faces: F, dLo, dUp of the face of slot l in the three
  // arrays of its direction. One buffer: a plane's faces are written after its
  // staging barrier and read before the next plane's.
  __device__ __forceinline__ void put_face(S *s_j, int l, const Face<S> &x) const {
    s_j[l] = x.F;
    s_j[HW + l] = x.dLo;
    s_j[2 * HW + l] = x.dUp;
  }
  __device__ __forceinline__ Face<S> get_face(const S *s_j, int l) const {
    Face<S> x{};
    x.F = s_j[l];
    x.dLo = s_j[HW + l];
    x.dUp = s_j[2 * HW + l];
    return x;
  }

  // One plane k. c0/d0: own cell at k; c1: own cell at k+1 (loaded), d1 is
  // computed here; c2 receives the prefetch of k+2. h0: halo cell at k, h1
  // receives the halo cell at k+1. zm: face (k-1, k); zp receives face (k, k+1).
  __device__ __forceinline__ void step(int k, const Cell<S> &c0, const Props<S> &d0,
                                       const Cell<S> &c1, Props<S> &d1, Cell<S> &c2,
                                       const Cell<S> (&h0)[HC], Cell<S> (&h1)[HC],
                                       Cell<S> (&h2)[HC], const Face<S> &zm, Face<S> &zp) const {
    const int b = ((k - kb) & 1) * hw_();
    const bool has_pz = k + 1 < nz;
    const S rkk = rk(k);
    if (k + 2 < nz && k + 2 <= ke) load(c2, k + 2);
    if (HALO2) {
      if (k + 2 < ke) load_halo(h2, k + 2);
    } else if (k + 1 < ke) {
      load_halo(h1, k + 1);
    }

    // stage plane k: own cell and halo cell (absent cells stage zeros, which
    // make every face towards them closed: T = 0)
    s_p[b + ol] = c0.p;
    s_k[b + ol] = TIN ? c0.tx : c0.k;
    if (YF && !SHARE) s_yf[b + ol] = TIN ? c0.ty : c0.ky;
    s_l[b + ol] = d0.lam;
    s_s[b + ol] = (uint8_t)c0.s;
    if (NEEDW) s_w[b + ol] = c0.w;
    if (R10) {
      s_tn[b + ol] = c0.tn;
      s_ts[b + ol] = c0.ts;
    }
    S hlam[HC];
#pragma unroll
    for (int q = 0; q < HC; ++q) {
      if (hl[q] < 0) continue;
      const Props<S> dh = props(h0[q].p, rkk, a);
      hlam[q] = dh.lam;
      const int l = b + hl[q];
      s_p[l] = h0[q].p;
      s_k[l] = TIN ? h0[q].tx : h0[q].k;
      if (YF && !SHARE) s_yf[l] = TIN ? h0[q].ty : h0[q].ky;
      s_l[l] = dh.lam;
      s_s[l] = (uint8_t)h0[q].s;
      if (NEEDW) s_w[l] = h0[q].w;
      if (R10) {
        s_tn[l] = h0[q].tn;
        s_ts[l] = h0[q].ts;
      }
    }
    __syncthreads();

    // on the last plane c1 holds a stale (finite) cell and the +z face is closed
    d1 = props(c1.p, rk(has_pz ? k + 1 : k), a);

    // the six faces, in the neighbour order -x, +x, -y, +y, -z, +z; a face
    // whose neighbour does not exist has T = 0 and contributes exact zeros
    Face<S> f[6];
    S wn[6];
    S vo[4] = {};
    const int Wv = w_();
    const int sl[4] = {ol - 1, ol + 1, ol - Wv, ol + Wv};
    if constexpr (vjp_own<S, MODE>()) {
      const float cf = a.cff;
      constexpr bool WR = has_with_r(MODE);
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int axis = n >> 1;
        const int q = b + sl[n];
        const float dw = c0.w - s_w[q];
        const uint32_t bit = 1u << axis;
        const float A2 = axis == 0 ? A2x : A2y;
        // the face's seal bit is its lower cell's
        const bool open = (((n & 1) ? c0.s : (uint32_t)s_s[q]) & bit) == 0u;
        if (n & 1)
          vjp_face_own<true, WR>(c0.k, s_k[q], open, c0.p, s_p[q], d0.lam, s_l[q], dw, cf,
                                 vo[axis], vo[2 + axis], A2, &f[n].F);
        else
          vjp_face_own<false, WR>(c0.k, s_k[q], open, c0.p, s_p[q], d0.lam, s_l[q], dw, cf,
                                  vo[axis], vo[2 + axis], A2, &f[n].F);
      }
    } else if constexpr (JSHARE) {
      // the +x and +y faces, whose lower cell is the own cell, for the own
      // cell and for its +x / +y neighbour (the -x / -y faces are read back
      // after the barrier below)
#pragma unroll
      for (int n = 1; n < 4; n += 2) {
        const int axis = n >> 1;
        const int q = b + sl[n];
        f[n] = face_h<true, false>(a, axis == 0 ? A2x : A2y, c0.k, s_k[q],
                                   (c0.s & (1u << axis)) == 0u, c0.p, s_p[q], d0.lam, s_l[q]);
      }
      put_face(s_jx, ol, f[1]);
      put_face(s_jy, ol, f[3]);
      // faces entering the tile from the -x / -y side of the halo ring
#pragma unroll
      for (int q = 0; q < HC; ++q) {
        const uint32_t role = hr[q];
        if (role == 0u) continue;
        const int l = b + hl[q];
        const Cell<S> &h = h0[q];
        if (role & kPX)
          put_face(s_jx, hl[q], face_h<true, false>(a, A2x, h.k, s_k[l + 1], (h.s & 1u) == 0u,
                                                    h.p, s_p[l + 1], hlam[q], s_l[l + 1]));
        if (role & kPY)
          put_face(s_jy, hl[q], face_h<true, false>(a, A2y, h.k, s_k[l + Wv], (h.s & 2u) == 0u,
                                                    h.p, s_p[l + Wv], hlam[q], s_l[l + Wv]));
      }
    } else {
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int axis = n >> 1;
        const int q = b + sl[n];
        const S pn = s_p[q];
        // k of the neighbour along this face's direction (k_y from its own
        // array in the per-direction form)
        const S kn = (K3 && axis == 1) ? s_yf[q] : s_k[q];
        const S kc = (K3 && axis == 1) ? c0.ky : c0.k;
        const S ln = s_l[q];
        const uint32_t sn = s_s[q];
        if (NEEDW) wn[n] = s_w[q];
        const uint32_t bit = 1u << axis;
        const S A2 = axis == 0 ? A2x : A2y;
        if constexpr (TIN) {
          // the face's transmissibility is stored on its lower cell
          const S T = (n & 1) ? (axis == 0 ? c0.tx : c0.ty) : (axis == 0 ? kn : s_yf[q]);
          f[n] = (n & 1) ? face_ht<DERIV>(a, T, c0.p, pn, d0.lam, ln)
                         : face_ht<DERIV>(a, T, pn, c0.p, ln, d0.lam);
        } else if (n & 1) {
          f[n] = face_h<DERIV, VJP>(a, A2, kc, kn, (c0.s & bit) == 0u, c0.p, pn, d0.lam, ln);
        } else {
          f[n] = face_h<DERIV, VJP>(a, A2, kn, kc, (sn & bit) == 0u, pn, c0.p, ln, d0.lam);
        }
      }
    }
    f[4] = zm;
    wn[4] = zm.w;
    zp = face_z<DERIV, VJP>(a, K3 ? c0.kz : c0.k, K3 ? c1.kz : c1.k,
                            has_pz && (c0.s & 4u) == 0u, c0.p, c1.p, has_pz ? hk(k) : 0.0,
                            d0, d1, TIN, c0.tz);
    zp.w = c0.w;
    f[5] = zp;
    wn[5] = c1.w;
    if constexpr (JSHARE) {
      __syncthreads();
      f[0] = get_face(s_jx, ol - 1);
      f[2] = get_face(s_jy, ol - Wv);
    }

    // the four in-plane diagonal faces of the 10-flux stencil: transmissibility
    // given (tne on the face's left end for (i,j)-(i+1,j+1), tse for
    // (i,j)-(i+1,j-1)), staged as 0 where the face does not exist
    S fd[4] = {};
    if constexpr (R10) {
      const int dsl[4] = {ol - Wv - 1, ol + Wv + 1, ol - Wv + 1, ol + Wv - 1};
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int q = b + dsl[n];
        const S pn = s_p[q], ln = s_l[q];
        // face transmissibility: stored on the face's left (i) end. A staged
        // halo cell's value is checked only against its own presence, which
        // covers every face towards a cell of the grid; a lane without a cell
        // (a padding lane) takes none.
        const S T = n == 0   ? (inside ? s_tn[q] : S(0))
                    : n == 1 ? c0.tn
                    : n == 2 ? c0.ts
                             : (inside ? s_ts[q] : S(0));
        // the lower-index cell is the neighbour for n = 0, 2 and the own cell for 1, 3
        const S pLo = (n & 1) ? c0.p : pn, pUp = (n & 1) ? pn : c0.p;
        const S lLo = (n & 1) ? d0.lam : ln, lUp = (n & 1) ? ln : d0.lam;
        const S dphi = pLo - pUp;
        fd[n] = (T * (dphi >= S(0) ? lLo : lUp)) * dphi;
      }
    }
    if (!own) return;
    emit<S, MODE>(a, k, plane, nz, sb, c0, d0, ACC ? xoff(k) : S(0), rkk, f, wn, fd, vo);
  }

  // ---- shared-face form (residual-only modes) ----------------------------
  // The face towards a neighbour N of higher index in the plane (+x, +y, and
  // for the 10-flux stencil +x+y, +x-y) is evaluated once, by the cell on its
  // -x / -y side, which is the face's lower cell (+x, +y, +x+y) or upper cell
  // (+x-y). Its flux goes to LDS; the other cell reads it after the next
  // barrier. Each face gets exactly the operands and operation order of the
  // two-sided form, and the residual is summed in the same order, so both
  // forms give bit-identical results.

  // F of the face from cell X (at LDS slot x, values passed in) to the slot
  // y of its +x, +y, +x+y or +x-y neighbour.
  __device__ __forceinline__ S fwd_face(uint32_t dir, int y, S pX, S kX, S lX, uint32_t sX,
                                        S tX) const {
    const S pn = s_p[y], ln = s_l[y];
    if (dir == kPX || dir == kPY) {
      if constexpr (TIN) return face_ht<false>(a, tX, pX, pn, lX, ln).F;
      const S A2 = dir == kPX ? A2x : A2y;
      const uint32_t bit = dir == kPX ? 1u : 2u;
      return face_h<false, false>(a, A2, kX, s_k[y], (sX & bit) == 0u, pX, pn, lX, ln).F;
    }
    // diagonal: X is the lower cell of the +x+y face and the upper cell of the +x-y face
    const bool lo = dir == kNE;
    const S pLo = lo ? pX : pn, pUp = lo ? pn : pX;
    const S lLo = lo ? lX : ln, lUp = lo ? ln : lX;
    const S dphi = pLo - pUp;
    return (tX * (dphi >= S(0) ? lLo : lUp)) * dphi;
  }

  // Residual of plane k of the own cell from its pending fluxes and the
  // neighbours' shared fluxes in LDS buffer bq (same order as emit()).
  __device__ __forceinline__ void finish(int k, int bq, const Pending<S> &pd) const {
    if (!own) return;
    double r = ACC ? pd.acc : 0.0;
    r = r - (double)s_fx[bq + ol - 1];
    r = r + (double)pd.fpx;
    r = r - (double)s_fy[bq + ol - W];
    r = r + (double)pd.fpy;
    r = r - (double)pd.fzm;
    r = r + (double)pd.fzp;
    if constexpr (R10) {
      // (a lane without a cell takes no diagonal flux of a halo cell, as above)
      r = r - (inside ? (double)s_fne[bq + ol - W - 1] : 0.0);
      r = r + (double)pd.fne;
      r = r - (double)pd.fse;
      r = r + (inside ? (double)s_fse[bq + ol + W - 1] : 0.0);
    }
    if (a.r) st_out<MODE>(at_w(static_cast<S *>(a.r), (size_t)k * plane, sb), (S)r);
  }

  // One plane k in the shared-face form: stage, complete plane k-1, evaluate
  // the z face (k, k+1) and the lower-cell in-plane faces of plane k.
  __device__ __forceinline__ void step_share(int k, const Cell<S> &c0, const Props<S> &d0,
                                             const Cell<S> &c1, Props<S> &d1, Cell<S> &c2,
                                             const Cell<S> (&h0)[HC], Cell<S> (&h1)[HC],
                                             Cell<S> (&h2)[HC], const Face<S> &zm, Face<S> &zp,
                                             Pending<S> &pd) const {
    static_assert(!DYN, "the fitted tile uses the two-sided form");
    const int b = ((k - kb) & 1) * HW;
    const bool has_pz = k + 1 < nz;
    const S rkk = rk(k);
    if (k + 2 < nz && k + 2 <= ke) load(c2, k + 2);
    if (HALO2) {
      if (k + 2 < ke) load_halo(h2, k + 2);
    } else if (k + 1 < ke) {
      load_halo(h1, k + 1);
    }

    s_p[b + ol] = c0.p;
    s_k[b + ol] = TIN ? c0.tx : c0.k;
    s_l[b + ol] = d0.lam;
    S hlam[HC];
#pragma unroll
    for (int q = 0; q < HC; ++q) {
      if (hl[q] < 0) continue;
      hlam[q] = props(h0[q].p, rkk, a).lam;
      const int l = b + hl[q];
      s_p[l] = h0[q].p;
      s_k[l] = TIN ? h0[q].tx : h0[q].k;
      s_l[l] = hlam[q];
    }
    __syncthreads();

    // plane k-1: its upper-cell fluxes were written before this barrier
    if (k > kb) finish(k - 1, HW - b, pd);

    d1 = props(c1.p, rk(has_pz ? k + 1 : k), a);
    zp = face_z<false, false>(a, c0.k, c1.k, has_pz && (c0.s & 4u) == 0u, c0.p, c1.p,
                              has_pz ? hk(k) : 0.0, d0, d1, TIN, c0.tz);

    const int o = b + ol;
    pd.fpx = fwd_face(kPX, o + 1, c0.p, c0.k, d0.lam, c0.s, c0.tx);
    pd.fpy = fwd_face(kPY, o + W, c0.p, c0.k, d0.lam, c0.s, c0.ty);
    s_fx[o] = pd.fpx;
    s_fy[o] = pd.fpy;
    if constexpr (R10) {
      pd.fne = fwd_face(kNE, o + W + 1, c0.p, c0.k, d0.lam, c0.s, c0.tn);
      pd.fse = fwd_face(kSE, o - W + 1, c0.p, c0.k, d0.lam, c0.s, c0.ts);
      s_fne[o] = pd.fne;
      s_fse[o] = pd.fse;
    }
    pd.fzm = zm.F;
    pd.fzp = zp.F;
    if constexpr (ACC) {
      S dacc;
      accumulation(a, c0, d0, xoff(k), rkk, pd.acc, dacc);
    }
    // faces entering the tile from the -x / -y side of the halo ring
#pragma unroll
    for (int q = 0; q < HC; ++q) {
      const uint32_t role = hr[q];
      if (role == 0u) continue;
      const int l = b + hl[q];
      const Cell<S> &h = h0[q];
      if (role & kPX) s_fx[l] = fwd_face(kPX, l + 1, h.p, h.k, hlam[q], h.s, h.tx);
      if (role & kPY) s_fy[l] = fwd_face(kPY, l + W, h.p, h.k, hlam[q], h.s, h.ty);
      if (R10 && (role & kNE)) s_fne[l] = fwd_face(kNE, l + W + 1, h.p, h.k, hlam[q], h.s, h.tn);
      if (R10 && (role & kSE)) s_fse[l] = fwd_face(kSE, l - W + 1, h.p, h.k, hlam[q], h.s, h.ts);
    }
  }
};


// One tile: columns of block (bx, by), planes from kb. `tid`: the thread's
// index in the workgroup (threadIdx.x, passed in so that a caller looping over
// tiles can keep it from being hoisted).
template <class S, int MODE, int TX, int TY>
__device__ __forceinline__ void march_tile(const Args &a, int bx, int by, int kb, char *smem,
                                           int tid = threadIdx.x) {
  const Tile<S, MODE, TX, TY> t(a, bx, by, kb, smem, tid);
  t.plane_constants(tid);
  // own column at planes k, k+1, k+2, halo cell at k, k+1 (and k+2 with HALO2),
  // z faces (k-1,k), (k,k+1)
  using T = Tile<S, MODE, TX, TY>;
  Cell<S> c0{}, c1{}, c2{}, h0[T::HC]{}, h1[T::HC]{}, h2[T::HC]{};
  Props<S> d0{}, d1{};
  Face<S> z0{}, z1{};
  t.load(c0, kb);
  t.load_halo(h0, kb);
  if (T::HALO2 && kb + 1 < t.ke) t.load_halo(h1, kb + 1);
  if (kb + 1 < t.nz) t.load(c1, kb + 1);
  d0 = props(c0.p, t.rk(kb), a);
  z0 = t.first_zface(c0, d0);
  if constexpr (T::SHARE && sizeof(S) == 4) {
    // FP32 residual modes: two planes per iteration with the register roles
    // swapped in the second, so that the halo cells, densities and z faces
    // need no copies between planes and the own column's three planes rotate
    // once per two planes (45 -> 55 VGPRs, still 8 waves per SIMD; the FP64
    // kernels would lose a wave per SIMD)
    Pending<S> pd{};
    int k = kb;
    for (; k + 1 < t.ke; k += 2) {
      t.step_share(k, c0, d0, c1, d1, c2, h0, h1, h2, z0, z1, pd);
      t.step_share(k + 1, c1, d1, c2, d0, c0, h1, h0, h2, z1, z0, pd);
      const Cell<S> c = c0;
      c0 = c2;
      c1 = c;
    }
    if (k < t.ke) t.step_share(k, c0, d0, c1, d1, c2, h0, h1, h2, z0, z1, pd);
    // the last plane's upper-cell fluxes
    __syncthreads();
    t.finish(t.ke - 1, ((t.ke - 1 - kb) & 1) * T::HW, pd);
  } else if constexpr (T::SHARE) {
    Pending<S> pd{};
    for (int k = kb; k < t.ke; ++k) {
      t.step_share(k, c0, d0, c1, d1, c2, h0, h1, h2, z0, z1, pd);
      c0 = c1;
      d0 = d1;
      c1 = c2;
#pragma unroll
      for (int q = 0; q < T::HC; ++q) {
        h0[q] = h1[q];
        if (T::HALO2) h1[q] = h2[q];
      }
      z0 = z1;
    }
    // the last plane's upper-cell fluxes
    __syncthreads();
    t.finish(t.ke - 1, ((t.ke - 1 - kb) & 1) * T::HW, pd);
  } else {
    for (int k = kb; k < t.ke; ++k) {
      t.step(k, c0, d0, c1, d1, c2, h0, h1, h2, z0, z1);
      c0 = c1;
      d0 = d1;
      c1 = c2;
#pragma unroll
      for (int q = 0; q < T::HC; ++q) {
        h0[q] = h1[q];
        if (T::HALO2) h1[q] = h2[q];
      }
      z0 = z1;
    }
  }
}

// XCD-aware order: the hardware hands consecutive workgroup ids to the 8 XCDs
// in turn. With the remap flag, the tiles of each z chunk (dispatched
// together, as in the plain order) are split into 8 contiguous bands of
// tile rows and each band goes to one XCD, so a tile's x and y neighbours
// mostly run on the same XCD and its halo lines are shared in that L2.
// Block ids and tile counts fit in 32 bits (the host refuses launches of 2^32
// or more workgroups), so the decoding runs in unsigned 32-bit arithmetic: two
// or three divisions by a runtime value and shifts for the 8 bands, instead of
// the emulated 64-bit divisions that made most of the workgroup prologue.
__device__ __forceinline__ void decode_tile(const Args &a, uint32_t b, int &bx, int &by, int &kb) {
  const uint32_t ntx = (uint32_t)a.ntx, nty = (uint32_t)a.nty;
  if (a.remap == 2) {
    // y-fast order: consecutive ids walk a tile column, so a tile's x
    // neighbours are nty ids away: on the same XCD when nty is a multiple of
    // 8, and dispatched close enough to be resident together
    const uint32_t r1 = b / nty, r2 = r1 / ntx;
    by = (int)(b - r1 * nty);
    bx = (int)(r1 - r2 * ntx);
    kb = (int)r2 * a.kz_chunk;
    return;
  }
  uint32_t t = b;
  if (a.remap) {
    const uint32_t C = ntx * nty;  // tiles per z chunk
    const uint32_t kc = b / C, u = b - kc * C;
    const uint32_t q = C >> 3, rem = C & 7u;
    const uint32_t x = u & 7u, l = u >> 3;  // band x (one XCD), position l in it
    t = kc * C + (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + l;
  }
  const uint32_t r1 = t / ntx, r2 = r1 / nty;
  bx = (int)(t - r1 * ntx);
  by = (int)(r1 - r2 * nty);
  kb = (int)r2 * a.kz_chunk;
}

template <class S, int MODE, int TX, int TY>
__global__ void __launch_bounds__(TX *TY)
    march_kernel(const Args a) {
  int bx, by, kb;
  decode_tile(a, blockIdx.x, bx, by, kb);
  __shared__ __attribute__((aligned(16))) char smem[tile_lds_bytes<S, MODE, TX, TY>()];
  march_tile<S, MODE, TX, TY>(a, bx, by, kb, smem);
}

// ----------------------------------------------------------------------------
// Host launch of one mode over the tile shapes (instantiated by the
// per-precision translation units).
// ----------------------------------------------------------------------------
template <class S, int MODE>
static hipError_t launch_t(int tile, const Args &a, hipStream_t st) {
  const dim3 grid((unsigned)a.nblocks);
  switch (tile) {
    case 0: march_kernel<S, MODE, 64, 4><<<grid, 256, 0, st>>>(a); break;
    case 1: march_kernel<S, MODE, 32, 8><<<grid, 256, 0, st>>>(a); break;
    case 2: march_kernel<S, MODE, 16, 16><<<grid, 256, 0, st>>>(a); break;
    case 3: march_kernel<S, MODE, 64, 8><<<grid, 512, 0, st>>>(a); break;
    case 4: march_kernel<S, MODE, 128, 4><<<grid, 512, 0, st>>>(a); break;
    case 5: march_kernel<S, MODE, 32, 16><<<grid, 512, 0, st>>>(a); break;
    case 6: march_kernel<S, MODE, 128, 2><<<grid, 256, 0, st>>>(a); break;
    case 7: march_kernel<S, MODE, 256, 1><<<grid, 256, 0, st>>>(a); break;
    case 8: march_kernel<S, MODE, 256, 2><<<grid, 512, 0, st>>>(a); break;
    case 9: march_kernel<S, MODE, 512, 1><<<grid, 512, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The kernel of one mode and tile shape (for occupancy queries).
template <class S, int MODE>
static const void *kernel_t(int tile) {
  switch (tile) {
    case 0: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 64, 4>);
    case 1: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 32, 8>);
    case 2: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 16, 16>);
    case 3: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 64, 8>);
    case 4: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 128, 4>);
    case 5: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 32, 16>);
    case 6: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 128, 2>);
    case 7: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 256, 1>);
    case 8: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 256, 2>);
    case 9: return reinterpret_cast<const void *>(&march_kernel<S, MODE, 512, 1>);
    default: return nullptr;
  }
}
template <class S, int F>
static const void *kernel_kind(int kind, int tile) {
  switch (kind) {
    case MODE_RESIDUAL: return kernel_t<S, MODE_RESIDUAL | F>(tile);
    case MODE_JACOBIAN: return kernel_t<S, MODE_JACOBIAN | F>(tile);
    case MODE_VJP: return kernel_t<S, MODE_VJP | F>(tile);
    case MODE_RES10: return kernel_t<S, MODE_RES10 | F>(tile);
    case MODE_RESIDUAL_BE: return kernel_t<S, MODE_RESIDUAL_BE | F>(tile);
    case MODE_JACOBIAN_BE: return kernel_t<S, MODE_JACOBIAN_BE | F>(tile);
    case MODE_JVP: return kernel_t<S, MODE_JVP | F>(tile);
    case MODE_JVP_BE: return kernel_t<S, MODE_JVP_BE | F>(tile);
    default: return nullptr;
  }
}

// Every mode kind with the flags F (MODE_TRANS or MODE_K3, MODE_PLAIN) of one
// instance set.
template <class S, int F>
static hipError_t launch_kind(int kind, int tile, const Args &a, hipStream_t st) {
  switch (kind) {
    case MODE_RESIDUAL: return launch_t<S, MODE_RESIDUAL | F>(tile, a, st);
    case MODE_JACOBIAN: return launch_t<S, MODE_JACOBIAN | F>(tile, a, st);
    case MODE_VJP: return launch_t<S, MODE_VJP | F>(tile, a, st);
    case MODE_RES10: return launch_t<S, MODE_RES10 | F>(tile, a, st);
    case MODE_RESIDUAL_BE: return launch_t<S, MODE_RESIDUAL_BE | F>(tile, a, st);
    case MODE_JACOBIAN_BE: return launch_t<S, MODE_JACOBIAN_BE | F>(tile, a, st);
    case MODE_JVP: return launch_t<S, MODE_JVP | F>(tile, a, st);
    case MODE_JVP_BE: return launch_t<S, MODE_JVP_BE | F>(tile, a, st);
    default: return hipErrorInvalidValue;
  }
}

// Single-grid launchers, one translation unit each (tpfa_march_f64.hip,
// tpfa_march_f32.hip, tpfa_march_f32_plain.hip) so that they compile in
// parallel. `kind` is a mode kind, `form` 0, MODE_TRANS or MODE_K3.
hipError_t launch_march_f64(int kind, int form, int tile, const Args &a, hipStream_t st);
hipError_t launch_march_f32(int kind, int form, int tile, const Args &a, hipStream_t st);
hipError_t launch_march_f32_plain(int kind, int form, int tile, const Args &a, hipStream_t st);
// The kernels those launch (non-temporal store kind for FP32).
const void *march_kernel_f64(int kind, int form, int tile);
const void *march_kernel_f32(int kind, int form, int tile);

}  // namespace tpfa
