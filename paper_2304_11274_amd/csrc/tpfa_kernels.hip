// HIP kernels for the TPFA flux residual, Jacobian and vector-Jacobian
// product on gfx950 (MI355X).
//
// Equations (paper Sec. 3): density Eq. (5), flux and potential difference
// Eq. (3a)/(3b) (outflow orientation dPhi_KL = Phi_K - Phi_L), single-point
// upwinding Eq. (4) with ties given to the lower linear index, residual
// assembly of Algorithm 1 (sum of the fluxes of a cell's face neighbours).
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
//    64 consecutive x cells when TX = 64); outputs are written once with
//    non-temporal stores;
//  * workgroups are numbered so that each of the 8 XCDs processes one
//    contiguous range of tiles, keeping halo re-reads in that XCD's L2.
// The cell-gather form writes only owned cells: no atomics, deterministic,
// and the same tile body serves the single-grid kernels and the persistent
// ensemble kernel, so both produce bit-identical results.
//
// Precision. FP64: every quantity in double, operation order of the
// definition (the flux of each face is formed as Ups * lambda * dPhi with
// Ups = a * ((2 k_K k_L) / (k_K + k_L))). FP32 precision form: p_K =
// pref[k] + dp_K is formed in FP64, so the potential difference and its
// upwind decision are FP64; transmissibility, density (single-precision exp),
// mobility and the flux/derivative products are FP32; the residual, the
// Jacobian diagonal and the gradients are accumulated in FP64 and rounded
// once on store.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tpfa_internal.h"

namespace tpfa {

// ----------------------------------------------------------------------------
// Per-precision cell quantities
// ----------------------------------------------------------------------------

template <class S>
struct Cell {
  S p;         // stored pressure value (absolute for FP64, offset for FP32)
  S k;         // kx
  S w;         // cotangent (vector-Jacobian product only)
  uint32_t s;  // seal bits
};

template <class S>
struct Props;

template <>
struct Props<double> {
  using C = double;
  double pa;   // absolute pressure
  double rho;  // density, Eq. (5)
  double lam;  // mobility rho / mu
  static __device__ __forceinline__ double absp(double v, double) { return v; }
  __device__ __forceinline__ void set(double v, double, const Args &a) {
    pa = v;
    rho = a.rho0 * exp(a.cf * (pa - a.p0));
    lam = rho / a.mu;
  }
};

template <>
struct Props<float> {
  using C = float;
  double pa;
  float rho;
  float lam;
  static __device__ __forceinline__ double absp(float v, double pref_k) {
    return pref_k + (double)v;
  }
  __device__ __forceinline__ void set(float v, double pref_k, const Args &a) {
    pa = pref_k + (double)v;
    rho = a.rho0f * __expf((float)(pa - a.p0) * a.cff);
    lam = rho * a.inv_muf;
  }
};

// One face between a lower-index cell (Lo) and an upper-index cell (Up).
template <class C>
struct Face {
  C F;    // F_{Lo,Up}: outflow of Lo
  C dLo;  // dF / dp_Lo
  C dUp;  // dF / dp_Up
  C qLo;  // k_Lo / (k_Lo + k_Up)   (vector-Jacobian product only)
  C qUp;  // k_Up / (k_Lo + k_Up)
};

// FP64 face. `A` is the geometric factor a_d, kLo/kUp the directional
// permeabilities, G = gk * dz on z faces and 0 (GRAV = false) otherwise.
template <bool GRAV, bool DERIV, bool VJP>
__device__ __forceinline__ Face<double> face64(const Args &a, double A, double kLo, double kUp,
                                                bool open, double pLo, double pUp,
                                                double rhoLo, double rhoUp, double lamLo,
                                                double lamUp) {
  Face<double> f;
  const double ks = kLo + kUp;
  double T;
  if (VJP) {
    const double inv = 1.0 / ks;
    f.qLo = kLo * inv;
    f.qUp = kUp * inv;
    T = A * ((2.0 * (kLo * kUp)) * inv);
  } else {
    T = A * ((2.0 * (kLo * kUp)) / ks);
  }
  T = (open && ks != 0.0) ? T : 0.0;
  double dphi = pLo - pUp;
  if (GRAV) dphi = dphi + ((0.5 * (rhoLo + rhoUp)) * a.gk) * a.dz;
  const bool up = dphi >= 0.0;  // a tie goes to the lower index
  const double lam = up ? lamLo : lamUp;
  f.F = (T * lam) * dphi;
  if (DERIV) {
    const double t = (a.cf * lam) * dphi;  // d(lambda_up)/dp_up * dPhi
    double gLo = 1.0, gUp = -1.0;          // dPhi/dp_Lo, dPhi/dp_Up
    if (GRAV) {
      gLo = 1.0 + ((0.5 * (a.cf * rhoLo)) * a.gk) * a.dz;
      gUp = -1.0 + ((0.5 * (a.cf * rhoUp)) * a.gk) * a.dz;
    }
    f.dLo = T * ((up ? t : 0.0) + lam * gLo);
    f.dUp = T * ((up ? 0.0 : t) + lam * gUp);
  }
  return f;
}

// FP32 face of the precision form: potential difference in FP64.
// A2 = 2 a_d r_d, kLo/kUp are kx (the ratio r_d cancels in k/(k+k)).
template <bool GRAV, bool DERIV, bool VJP>
__device__ __forceinline__ Face<float> face32(const Args &a, float A2, float kLo, float kUp,
                                               bool open, double pLo, double pUp, float rhoLo,
                                               float rhoUp, float lamLo, float lamUp) {
  Face<float> f;
  const float ks = kLo + kUp;
  const float inv = __builtin_amdgcn_rcpf(ks);
  const float qUp = kUp * inv;
  if (VJP) {
    f.qLo = kLo * inv;
    f.qUp = qUp;
  }
  float T = (A2 * kLo) * qUp;
  T = (open && ks > 0.0f) ? T : 0.0f;
  double dphi = pLo - pUp;
  if (GRAV) dphi = dphi + (double)(0.5f * (rhoLo + rhoUp)) * (a.gk * a.dz);
  const bool up = dphi >= 0.0;
  const float dphif = (float)dphi;
  const float lam = up ? lamLo : lamUp;
  f.F = (T * lam) * dphif;
  if (DERIV) {
    const float t = (a.cff * lam) * dphif;
    float gLo = 1.0f, gUp = -1.0f;
    if (GRAV) {
      gLo = 1.0f + (0.5f * a.cff * rhoLo) * a.gdzf;
      gUp = -1.0f + (0.5f * a.cff * rhoUp) * a.gdzf;
    }
    f.dLo = T * ((up ? t : 0.0f) + lam * gLo);
    f.dUp = T * ((up ? 0.0f : t) + lam * gUp);
  }
  return f;
}

template <class S, bool GRAV, bool DERIV, bool VJP>
__device__ __forceinline__ Face<typename Props<S>::C> face(const Args &a, int axis, S kxLo,
                                                          S kxUp, bool open, double pLo,
                                                          double pUp,
                                                          typename Props<S>::C rhoLo,
                                                          typename Props<S>::C rhoUp,
                                                          typename Props<S>::C lamLo,
                                                          typename Props<S>::C lamUp) {
  if constexpr (sizeof(S) == 8) {
    // directional permeability exactly as r_d * kx, geometric factor a_d
    const double A = axis == 0 ? a.ax : (axis == 1 ? a.ay : a.az);
    const double r = axis == 0 ? 1.0 : (axis == 1 ? a.ry : a.rz);
    const double kLo = axis == 0 ? (double)kxLo : r * (double)kxLo;
    const double kUp = axis == 0 ? (double)kxUp : r * (double)kxUp;
    return face64<GRAV, DERIV, VJP>(a, A, kLo, kUp, open, pLo, pUp, rhoLo, rhoUp, lamLo, lamUp);
  } else {
    const float A2 = axis == 0 ? a.ax2f : (axis == 1 ? a.ay2f : a.az2f);
    return face32<GRAV, DERIV, VJP>(a, A2, kxLo, kxUp, open, pLo, pUp, rhoLo, rhoUp, lamLo,
                                    lamUp);
  }
}

template <class S, int MODE>
__device__ __forceinline__ void load_cell(Cell<S> &c, const Args &a, int64_t idx, bool ok) {
  if (ok) {
    c.p = static_cast<const S *>(a.p)[idx];
    c.k = static_cast<const S *>(a.kx)[idx];
    c.s = a.seal ? (uint32_t)a.seal[idx] : 0u;
    if (MODE == MODE_VJP) c.w = static_cast<const S *>(a.w)[idx];
  } else {
    c.p = S(0);
    c.k = S(0);
    c.s = 0u;
    c.w = S(0);
  }
}

template <class T>
__device__ __forceinline__ void st_nt(T *base, int64_t idx, T v) {
  __builtin_nontemporal_store(v, base + idx);
}

// Bytes of LDS one tile needs.
template <class S, int MODE, int TX, int TY>
constexpr int tile_lds_bytes() {
  constexpr int HW = (TX + 2) * (TY + 2);
  return 2 * HW * ((int)sizeof(S) * (MODE == MODE_VJP ? 3 : 2) +
                   (int)sizeof(typename Props<S>::C) + 1);
}

// ----------------------------------------------------------------------------
// The tile body: columns [bx*TX, bx*TX+TX) x [by*TY, by*TY+TY), planes
// [kb, min(kb + kz_chunk, nz)).
// ----------------------------------------------------------------------------
template <class S, int MODE, int TX, int TY>
__device__ __forceinline__ void march_tile(const Args &a, int bx, int by, int kb, char *smem) {
  using P = Props<S>;
  using C = typename P::C;
  constexpr int W = TX + 2, H = TY + 2, HW = W * H;
  constexpr bool VJP = MODE == MODE_VJP;
  constexpr bool DERIV = MODE != MODE_RESIDUAL;
  constexpr bool FP32 = sizeof(S) == 4;

  S *s_p = reinterpret_cast<S *>(smem);
  S *s_k = s_p + 2 * HW;
  C *s_l = reinterpret_cast<C *>(s_k + 2 * HW);
  S *s_w = reinterpret_cast<S *>(s_l + 2 * HW);
  uint8_t *s_s = reinterpret_cast<uint8_t *>(s_w + (VJP ? 2 * HW : 0));

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane = a.plane;
  const int ke = min(kb + a.kz_chunk, nz);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int i = bx * TX + tx, j = by * TY + ty;
  const bool own = i < nx && j < ny;
  const int64_t col = own ? (int64_t)j * nx + i : 0;
  const int ol = (ty + 1) * W + tx + 1;

  // the halo cell this thread stages (threads beyond the ring stage none)
  int hl = -1, hi = -1, hj = -1;
  if (tid < TX) {
    hi = bx * TX + tid;
    hj = by * TY - 1;
    hl = tid + 1;
  } else if (tid < 2 * TX) {
    hi = bx * TX + tid - TX;
    hj = by * TY + TY;
    hl = (TY + 1) * W + tid - TX + 1;
  } else if (tid < 2 * TX + TY) {
    hi = bx * TX - 1;
    hj = by * TY + tid - 2 * TX;
    hl = (tid - 2 * TX + 1) * W;
  } else if (tid < 2 * TX + 2 * TY) {
    hi = bx * TX + TX;
    hj = by * TY + tid - 2 * TX - TY;
    hl = (tid - 2 * TX - TY + 1) * W + TX + 1;
  }
  const bool hv = hl >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
  const int64_t hcol = hv ? (int64_t)hj * nx + hi : 0;

  const bool has_mx = i > 0, has_px = i + 1 < nx;
  const bool has_my = j > 0, has_py = j + 1 < ny;

  const double *pref = a.pref;
  auto pref_at = [&](int k) -> double { return FP32 ? pref[k] : 0.0; };

  Cell<S> cur{}, nx1{}, pf{}, hcur{}, hnx{};
  P dcur{}, dnx1{};
  load_cell<S, MODE>(cur, a, kb * plane + col, own);
  load_cell<S, MODE>(hcur, a, kb * plane + hcol, hv);
  if (kb + 1 < nz) load_cell<S, MODE>(nx1, a, (kb + 1) * plane + col, own);
  dcur.set(cur.p, pref_at(kb), a);

  // -z face of the first plane of the chunk: face (kb-1, kb), own cell is Up
  Face<C> fmz{};
  S wmz = S(0);
  if (kb > 0) {
    Cell<S> pr;
    load_cell<S, MODE>(pr, a, (kb - 1) * plane + col, own);
    P dp;
    dp.set(pr.p, pref_at(kb - 1), a);
    fmz = face<S, true, DERIV, VJP>(a, 2, pr.k, cur.k, (pr.s & 4u) == 0u, dp.pa, dcur.pa,
                                    dp.rho, dcur.rho, dp.lam, dcur.lam);
    wmz = pr.w;
  }

  for (int k = kb; k < ke; ++k) {
    const int b = ((k - kb) & 1) * HW;
    const bool has_pz = k + 1 < nz;
    const double pref_k = pref_at(k);
    // prefetch: own column two planes ahead, halo one plane ahead
    if (k + 2 < nz && k + 2 <= ke) load_cell<S, MODE>(pf, a, (int64_t)(k + 2) * plane + col, own);
    if (k + 1 < ke) load_cell<S, MODE>(hnx, a, (int64_t)(k + 1) * plane + hcol, hv);

    // stage plane k: own cell and halo cell
    s_p[b + ol] = cur.p;
    s_k[b + ol] = cur.k;
    s_l[b + ol] = dcur.lam;
    s_s[b + ol] = (uint8_t)cur.s;
    if (VJP) s_w[b + ol] = cur.w;
    if (hl >= 0) {
      P dh;
      dh.set(hcur.p, pref_k, a);
      s_p[b + hl] = hcur.p;
      s_k[b + hl] = hcur.k;
      s_l[b + hl] = hv ? dh.lam : C(0);
      s_s[b + hl] = (uint8_t)hcur.s;
      if (VJP) s_w[b + hl] = hcur.w;
    }
    __syncthreads();

    if (has_pz) dnx1.set(nx1.p, pref_at(k + 1), a);

    // the six faces, in the neighbour order -x, +x, -y, +y, -z, +z
    Face<C> f[6] = {};
    S wn[6] = {};
    {
      const int sl[4] = {ol - 1, ol + 1, ol - W, ol + W};
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int axis = n >> 1;
        const bool lower_is_own = n & 1;
        const int q = b + sl[n];
        const S pn = s_p[q];
        const S kn = s_k[q];
        const C ln = s_l[q];
        const uint32_t sn = s_s[q];
        if (VJP) wn[n] = s_w[q];
        const double pna = P::absp(pn, pref_k);
        const uint32_t bit = 1u << axis;
        if (lower_is_own) {
          f[n] = face<S, false, DERIV, VJP>(a, axis, cur.k, kn, (cur.s & bit) == 0u, dcur.pa, pna,
                                            C(0), C(0), dcur.lam, ln);
        } else {
          f[n] = face<S, false, DERIV, VJP>(a, axis, kn, cur.k, (sn & bit) == 0u, pna, dcur.pa,
                                            C(0), C(0), ln, dcur.lam);
        }
      }
    }
    f[4] = fmz;
    wn[4] = wmz;
    if (has_pz) {
      f[5] = face<S, true, DERIV, VJP>(a, 2, cur.k, nx1.k, (cur.s & 4u) == 0u, dcur.pa, dnx1.pa,
                                       dcur.rho, dnx1.rho, dcur.lam, dnx1.lam);
      wn[5] = nx1.w;
    }
    const bool ex[6] = {has_mx, has_px, has_my, has_py, k > 0, has_pz};

    if (own) {
      const int64_t idx = (int64_t)k * plane + col;
      if constexpr (MODE == MODE_VJP) {
        double gp = 0.0, gm = 0.0;
#pragma unroll
        for (int n = 0; n < 6; ++n) {
          if (!ex[n]) continue;
          const double d = (double)cur.w - (double)wn[n];
          if (n & 1) {  // own cell is Lo
            gp += d * (double)f[n].dLo;
            gm += d * ((double)f[n].F * (double)f[n].qUp);
          } else {      // own cell is Up
            gp -= d * (double)f[n].dUp;
            gm -= d * ((double)f[n].F * (double)f[n].qLo);
          }
        }
        if (a.gp) st_nt(static_cast<S *>(a.gp), idx, (S)gp);
        if (a.gm) st_nt(static_cast<S *>(a.gm), idx, (S)gm);
      } else {
        double r = 0.0;
        double dg = 0.0;
        C off[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
          if (n & 1) {
            r += ex[n] ? (double)f[n].F : 0.0;
            if (DERIV) {
              dg += ex[n] ? (double)f[n].dLo : 0.0;
              off[n] = ex[n] ? f[n].dUp : C(0);
            }
          } else {
            r -= ex[n] ? (double)f[n].F : 0.0;
            if (DERIV) {
              dg -= ex[n] ? (double)f[n].dUp : 0.0;
              off[n] = ex[n] ? -f[n].dLo : C(0);
            }
          }
        }
        if (a.r) st_nt(static_cast<S *>(a.r), idx, (S)r);
        if constexpr (DERIV) {
          S *J = static_cast<S *>(a.J);
          const int64_t nc = (int64_t)nz * plane;
          st_nt(J, idx, (S)dg);
#pragma unroll
          for (int n = 0; n < 6; ++n) st_nt(J, (int64_t)(n + 1) * nc + idx, (S)off[n]);
        }
      }
    }

    // advance the column: the +z face becomes the next plane's -z face
    fmz = f[5];
    wmz = cur.w;
    cur = nx1;
    dcur = dnx1;
    nx1 = pf;
    hcur = hnx;
  }
}

// XCD-aware order: the hardware hands consecutive workgroup ids to the 8 XCDs
// in turn; renumber so that XCD x processes one contiguous range of tiles
// (x fastest, then y, then z chunk), which keeps a tile's halo neighbours in
// the same L2.
__device__ __forceinline__ void decode_tile(const Args &a, int64_t b, int &bx, int &by, int &kb) {
  int64_t t = b;
  if (a.remap) {
    const int64_t n = a.nblocks, q = n / 8, rem = n % 8;
    const int64_t x = b % 8, l = b / 8;
    t = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + l;
  }
  bx = (int)(t % a.ntx);
  t /= a.ntx;
  by = (int)(t % a.nty);
  t /= a.nty;
  kb = (int)t * a.kz_chunk;
}

template <class S, int MODE, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) march_kernel(const Args a) {
  __shared__ __attribute__((aligned(16))) char smem[tile_lds_bytes<S, MODE, TX, TY>()];
  int bx, by, kb;
  decode_tile(a, blockIdx.x, bx, by, kb);
  march_tile<S, MODE, TX, TY>(a, bx, by, kb, smem);
}

// ----------------------------------------------------------------------------
// Persistent ensemble kernel: 256-thread workgroups take work items (one tile
// and z chunk of one model) from a device counter until the list is drained.
// The last workgroup to finish resets the counters, so the next launch (or
// graph replay) on the stream starts from zero without a memset node.
// ----------------------------------------------------------------------------
constexpr int kPersistThreads = 256;

template <class S, int MODE>
constexpr int persist_lds_bytes() {
  constexpr int a0 = tile_lds_bytes<S, MODE, 64, 4>();
  constexpr int a1 = tile_lds_bytes<S, MODE, 32, 8>();
  constexpr int a2 = tile_lds_bytes<S, MODE, 16, 16>();
  return a0 > a1 ? (a0 > a2 ? a0 : a2) : (a1 > a2 ? a1 : a2);
}

template <class S, int MODE>
__global__ void __launch_bounds__(kPersistThreads)
    persistent_kernel(const Args *__restrict__ models, const WorkItem *__restrict__ items,
                      int64_t n_items, unsigned int *counter) {
  __shared__ __attribute__((aligned(16))) char smem[persist_lds_bytes<S, MODE>()];
  __shared__ unsigned int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&counter[0], 1u);
    __syncthreads();
    const unsigned int it = s_item;
    __syncthreads();  // s_item is rewritten next iteration
    if ((int64_t)it >= n_items) break;
    const WorkItem w = items[it];
    const Args m = models[w.model];
    switch (m.tile) {
      case 0: march_tile<S, MODE, 64, 4>(m, w.bx, w.by, w.kb, smem); break;
      case 1: march_tile<S, MODE, 32, 8>(m, w.bx, w.by, w.kb, smem); break;
      default: march_tile<S, MODE, 16, 16>(m, w.bx, w.by, w.kb, smem); break;
    }
    __syncthreads();  // LDS is reused by the next item
  }
  // workgroup done: the last one out resets both counters for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned int done = atomicAdd(&counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
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

__global__ void offset_kernel(int64_t plane, int64_t n, const double *__restrict__ p,
                              const double *__restrict__ pref, float *__restrict__ dp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride)
    dp[idx] = (float)(p[idx] - pref[idx / plane]);
}

// ----------------------------------------------------------------------------
// Host launchers
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
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_march(tpfa_precision_t prec, Mode mode, int tile, const Args &a,
                        hipStream_t st) {
  if (a.nblocks <= 0) return hipSuccess;
  if (prec == TPFA_FP64) {
    switch (mode) {
      case MODE_RESIDUAL: return launch_t<double, MODE_RESIDUAL>(tile, a, st);
      case MODE_JACOBIAN: return launch_t<double, MODE_JACOBIAN>(tile, a, st);
      default: return launch_t<double, MODE_VJP>(tile, a, st);
    }
  }
  switch (mode) {
    case MODE_RESIDUAL: return launch_t<float, MODE_RESIDUAL>(tile, a, st);
    case MODE_JACOBIAN: return launch_t<float, MODE_JACOBIAN>(tile, a, st);
    default: return launch_t<float, MODE_VJP>(tile, a, st);
  }
}

template <class S, int MODE>
static const void *persist_fn() {
  return reinterpret_cast<const void *>(&persistent_kernel<S, MODE>);
}

static const void *persist_ptr(tpfa_precision_t prec, Mode mode) {
  if (prec == TPFA_FP64)
    return mode == MODE_RESIDUAL ? persist_fn<double, MODE_RESIDUAL>()
                                 : persist_fn<double, MODE_JACOBIAN>();
  return mode == MODE_RESIDUAL ? persist_fn<float, MODE_RESIDUAL>()
                               : persist_fn<float, MODE_JACOBIAN>();
}

int persistent_workgroups(tpfa_precision_t prec, Mode mode) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_ptr(prec, mode),
                                                   kPersistThreads, 0) != hipSuccess)
    return -1;
  if (per_cu < 1) per_cu = 1;
  return cus * per_cu;
}

hipError_t launch_persistent(tpfa_precision_t prec, Mode mode, const Args *d_models,
                             const WorkItem *d_items, int64_t n_items, unsigned int *d_counter,
                             int n_workgroups, hipStream_t st) {
  const dim3 grid((unsigned)n_workgroups);
  if (prec == TPFA_FP64) {
    if (mode == MODE_RESIDUAL)
      persistent_kernel<double, MODE_RESIDUAL>
          <<<grid, kPersistThreads, 0, st>>>(d_models, d_items, n_items, d_counter);
    else
      persistent_kernel<double, MODE_JACOBIAN>
          <<<grid, kPersistThreads, 0, st>>>(d_models, d_items, n_items, d_counter);
  } else {
    if (mode == MODE_RESIDUAL)
      persistent_kernel<float, MODE_RESIDUAL>
          <<<grid, kPersistThreads, 0, st>>>(d_models, d_items, n_items, d_counter);
    else
      persistent_kernel<float, MODE_JACOBIAN>
          <<<grid, kPersistThreads, 0, st>>>(d_models, d_items, n_items, d_counter);
  }
  return hipGetLastError();
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
  offset_kernel<<<grid, 256, 0, st>>>(g.nx * g.ny, n, p, pref, dp);
  return hipGetLastError();
}

}  // namespace tpfa
