// TPFA flux oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously correct CPU reference for the flux part of the
// finite-volume residual of compressible single-phase Darcy flow, used to
// check the GPU library. Only the test suite, the smoke entry point and the
// CPU-baseline leg of the benchmark load it; it shares no source, header or
// helper with the GPU library.
//
// What it computes (paper, Sec. 3 "Finite Volume for Geologic Carbon Storage
// Simulation"):
//   rho_K      = rho_ref * exp(c_f * (p_K - p_ref))                   Eq. (5)
//   F_KL       = Ups_KL * lambda_upw * dPhi_KL                        Eq. (3a)
//   dPhi_KL    = (p_K - p_L) + rho_avg * g * (zeta_L - zeta_K)        Eq. (3b), read as Phi_K - Phi_L
//   rho_avg    = (rho_K + rho_L) / 2                                  "the average" of the two densities
//   lambda_upw = rho_K / mu if dPhi_KL > 0, else rho_L / mu           Eq. (4), tie -> lower index
//   r_K        = sum over the neighbours L of K of F_KL                Algorithm 1 / Eq. (2) flux sum
// evaluated exactly as Algorithm 1 orders it: an outer loop over cells K, an
// inner loop over the neighbours L of K, both densities evaluated for every
// (K, L) pair, and the flux added to r_K.
//
// Readings where the paper is silent or inconsistent (each one is listed in
// the design notes of the repository):
//  * Orientation of dPhi: Eq. (3b) as printed is Phi_L - Phi_K, which makes
//    Eq. (4) pick the downstream cell; F_KL is taken as the outflow of K, i.e.
//    dPhi_KL = Phi_K - Phi_L, so the upwind cell is the higher-potential one.
//  * zeta is the cell-centre coordinate along +k and g (grid.gk) the gravity
//    component along +k: with k pointing down, gk = +9.81 and hydrostatic
//    pressure grows with k.
//  * Ups_KL (no formula in the paper) is the two-point harmonic
//    transmissibility a_d * 2 k_K k_L / (k_K + k_L) with a_x = dy dz / dx,
//    a_y = dx dz / dy, a_z = dx dy / dz and the directional permeability;
//    a sealed face, or k_K + k_L = 0, has Ups = 0.
//  * Ties dPhi_KL = 0: the lower linear index is upwind, so that both sides of
//    a face make the same choice (the flux is 0 either way).
//  * Domain boundary: no-flow; boundary cells simply have fewer neighbours.
//  * The accumulation term of Eq. (2) is excluded from the flux residual, as
//    in the paper. The full backward-Euler residual (oracle_eval_be) adds it:
//      r_K = V_K (phi(p_K) rho(p_K) - phi(pn_K) rho(pn_K)) / dt + sum_L F_KL
//    with V_K = dx dy dz, pn the pressure of the previous time level, and the
//    porosity linear in pressure (the paper says porosity depends linearly on
//    p): phi(p) = phi_ref (1 + c_r (p - p_ref)), phi_ref given per cell, c_r
//    the rock compressibility, p_ref the fluid's reference pressure.
//
// Jacobian: the 7-point derivative of r with respect to p, stored as seven
// planes [diag, -x, +x, -y, +y, -z, +z]; plane 1+n holds dr_K/dp_L for the
// neighbour n of K (0 where that neighbour does not exist).
//
// Vector-Jacobian product with cotangent w: grad_p = J^T w and
// grad_logk[j] = sum_K w_K d r_K / d ln(kx_j), where ky = ry kx and kz = rz kx
// follow kx (ratios, not separate arrays). With per-direction arrays kx, ky,
// kz instead, grad_k3[a][j] = sum_K w_K d r_K / d ln(k_a,j) for a = x, y, z.
//
// Parity pins (tests/test_oracle_*.py): closed-form two-cell fluxes, the
// continuous hydrostatic column, the c_f = 0 graph Laplacian built by SciPy,
// complex-step derivatives for J and for the log-permeability gradient, a
// long-double evaluation, conservation, equilibria and scaling invariants.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>

extern "C" {

typedef struct {
  int64_t nx, ny, nz;
  double dx, dy, dz;
  double gk;  // gravity component along +k (m/s^2)
} oracle_grid;

typedef struct {
  double rho_ref, cf, p_ref, mu;
} oracle_fluid;

}  // extern "C"

namespace {

using cplx = std::complex<double>;

inline double real_part(double v) { return v; }
inline double real_part(long double v) { return (double)v; }
inline double real_part(const cplx& v) { return v.real(); }

template <class S>
struct Problem {
  const oracle_grid* g;
  const oracle_fluid* f;
  const S* p;                  // pressure per cell (Pa)
  const S* kx;                 // permeability along x (m^2)
  const S* ky;                 // NULL -> ry * kx
  const S* kz;                 // NULL -> rz * kx
  double ry, rz;
  const uint8_t* seal;         // NULL or bit a set: face towards +a neighbour closed
  const int8_t* force;         // NULL or [3][N]: +1 / -1 forces the lower / upper cell upwind
  const int8_t* force_diag = nullptr;  // NULL or [2][N]: the same for the in-plane diagonal
                                       //   faces (i,j)-(i+1,j+1) and (i,j)-(i+1,j-1), indexed
                                       //   by the face's left (i) end
  const S* tne = nullptr;      // NULL or the transmissibility of the face (i,j)-(i+1,j+1) of each cell
  const S* tse = nullptr;      // NULL or the transmissibility of the face (i,j)-(i+1,j-1) of each cell
  const S* tx = nullptr;       // NULL, or the transmissibilities of the faces towards +x, +y, +z
  const S* ty = nullptr;       //   given per cell (replace the harmonic average of k, the ratios
  const S* tz = nullptr;       //   and the seal bits)
  const S* phi = nullptr;      // NULL or phi_ref per cell: adds the accumulation term of Eq. (2)
  const S* p_prev = nullptr;   // pressure of the previous time level (with phi)
  double dt = 0.0, cr = 0.0;   // time step (s) and rock compressibility (1/Pa) (with phi)
  int64_t ncell() const { return g->nx * g->ny * g->nz; }
};

// Eq. (5)
template <class S>
S density(const S& p, const oracle_fluid& f) {
  using std::exp;
  return S(f.rho_ref) * exp(S(f.cf) * (p - S(f.p_ref)));
}

template <class S>
S perm(const Problem<S>& pb, int axis, int64_t c) {
  if (axis == 0) return pb.kx[c];
  if (axis == 1) return pb.ky ? pb.ky[c] : S(pb.ry) * pb.kx[c];
  return pb.kz ? pb.kz[c] : S(pb.rz) * pb.kx[c];
}

// face area over centre-to-centre distance for a face normal to `axis`
double geom_factor(const oracle_grid& g, int axis) {
  if (axis == 0) return g.dy * g.dz / g.dx;
  if (axis == 1) return g.dx * g.dz / g.dy;
  return g.dx * g.dy / g.dz;
}

// Neighbour n of a cell, n = 0..5 -> (-x, +x, -y, +y, -z, +z); with the four
// in-plane diagonal neighbours of the 10-flux stencil, n = 6..9 -> (-x-y),
// (+x+y), (+x-y), (-x+y).
struct Nb {
  bool exists;
  int64_t L;
  int axis;  // 0, 1, 2; 3 for a diagonal
  int side;  // -1 or +1 (cardinal); for a diagonal, +1 when the cell is the face's (i, j) end
};

Nb neighbour(const oracle_grid& g, int64_t i, int64_t j, int64_t k, int n) {
  static const int dx[4] = {-1, 1, 1, -1}, dy[4] = {-1, 1, -1, 1};
  Nb nb;
  int64_t ii = i, jj = j, kk = k;
  if (n < 6) {
    nb.axis = n / 2;
    nb.side = (n % 2) ? 1 : -1;
    if (nb.axis == 0) ii += nb.side;
    if (nb.axis == 1) jj += nb.side;
    if (nb.axis == 2) kk += nb.side;
  } else {
    nb.axis = 3;
    ii += dx[n - 6];
    jj += dy[n - 6];
    nb.side = dx[n - 6] > 0 ? 1 : -1;  // the cell is the face's left (i) end
  }
  nb.exists = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
  nb.L = nb.exists ? ii + g.nx * (jj + g.ny * kk) : -1;
  return nb;
}

template <class S>
struct FluxKL {
  S F;        // F_KL, outflow of K towards L
  S dF_dpK;   // dF_KL / dp_K
  S dF_dpL;   // dF_KL / dp_L
  S T;        // transmissibility
  S kK, kL;   // directional permeabilities of K and L
  S dPhi;     // potential difference Phi_K - Phi_L
};

// One flux of the inner loop of Algorithm 1, seen from cell K.
template <class S>
FluxKL<S> flux(const Problem<S>& pb, int64_t K, int64_t L, int axis, int side) {
  const oracle_grid& g = *pb.g;
  const oracle_fluid& f = *pb.f;
  FluxKL<S> out;
  const int64_t lo = K < L ? K : L;  // lower-index cell of the face

  if (axis == 3) {
    // in-plane diagonal face: transmissibility given, stored on its left (i) end
    out.kK = out.kL = S(0);
    const int64_t left = side > 0 ? K : L;
    const int64_t right = side > 0 ? L : K;
    // the right end lies 1 + nx (face towards +y) or 1 - nx (towards -y) further in index
    out.T = (right - left == 1 + g.nx) ? pb.tne[left] : pb.tse[left];
  } else if (pb.tx) {
    // transmissibility given per face, stored on the face's lower cell
    out.kK = out.kL = S(0);
    const S* t = axis == 0 ? pb.tx : axis == 1 ? pb.ty : pb.tz;
    out.T = t[lo];
  } else {
    // transmissibility (harmonic two-point form, closed if sealed)
    out.kK = perm(pb, axis, K);
    out.kL = perm(pb, axis, L);
    const bool sealed = pb.seal && ((pb.seal[lo] >> axis) & 1u);
    const S ksum = out.kK + out.kL;
    if (sealed || real_part(ksum) == 0.0)
      out.T = S(0);
    else
      out.T = S(geom_factor(g, axis)) * ((S(2) * (out.kK * out.kL)) / ksum);
  }

  // densities in K and L (Eq. 5), their average and pressure derivatives
  const S pK = pb.p[K], pL = pb.p[L];
  const S rhoK = density(pK, f), rhoL = density(pL, f);
  const S rho_avg = S(0.5) * (rhoK + rhoL);
  const S drhoK = S(f.cf) * rhoK, drhoL = S(f.cf) * rhoL;

  // elevation difference zeta_L - zeta_K along +k
  const double dzeta = axis == 2 ? side * g.dz : 0.0;
  const int force_axis = axis < 3 ? axis : 0;

  // potential difference (Eq. 3b, outflow orientation)
  out.dPhi = (pK - pL) + (rho_avg * S(g.gk)) * S(dzeta);
  const S dPhi_dpK = S(1) + (S(0.5) * drhoK * S(g.gk)) * S(dzeta);
  const S dPhi_dpL = S(-1) + (S(0.5) * drhoL * S(g.gk)) * S(dzeta);

  // single-point upwinding (Eq. 4); a tie goes to the lower index
  bool upK;
  int8_t forced = (pb.force && axis < 3) ? pb.force[(int64_t)force_axis * pb.ncell() + lo] : 0;
  if (axis == 3 && pb.force_diag) {
    const int64_t left = side > 0 ? K : L;
    const int64_t right = side > 0 ? L : K;
    const int d = (right - left == 1 + g.nx) ? 0 : 1;
    forced = pb.force_diag[(int64_t)d * pb.ncell() + left];
  }
  if (forced != 0) {
    upK = (forced > 0) == (K == lo);
  } else {
    const double d = real_part(out.dPhi);
    upK = d > 0.0 || (d == 0.0 && K < L);
  }
  const S lamK = rhoK / S(f.mu), lamL = rhoL / S(f.mu);
  const S dlamK = drhoK / S(f.mu), dlamL = drhoL / S(f.mu);
  const S lam = upK ? lamK : lamL;

  // flux (Eq. 3a) and its derivatives
  out.F = (out.T * lam) * out.dPhi;
  out.dF_dpK = out.T * ((upK ? dlamK * out.dPhi : S(0)) + lam * dPhi_dpK);
  out.dF_dpL = out.T * ((upK ? S(0) : dlamL * out.dPhi) + lam * dPhi_dpL);
  return out;
}

// phi(p) rho(p): fluid mass per unit bulk volume, the accumulated quantity of Eq. (2)
template <class S>
S mass_density(const Problem<S>& pb, int64_t c, const S& p) {
  const S phi = pb.phi[c] * (S(1) + S(pb.cr) * (p - S(pb.f->p_ref)));
  return phi * density(p, *pb.f);
}
// d/dp of phi(p) rho(p) = phi_ref c_r rho + phi(p) c_f rho
template <class S>
S mass_density_dp(const Problem<S>& pb, int64_t c, const S& p) {
  const S rho = density(p, *pb.f);
  const S phi = pb.phi[c] * (S(1) + S(pb.cr) * (p - S(pb.f->p_ref)));
  return (pb.phi[c] * S(pb.cr)) * rho + phi * (S(pb.f->cf) * rho);
}

struct Outputs {
  void* r = nullptr;       // [N]
  void* J = nullptr;       // [7][N]
  const void* v = nullptr; // [N] direction of the Jacobian-vector product
  void* jv = nullptr;      // [N] J v
  const double* w = nullptr;
  void* grad_p = nullptr;  // [N]
  void* grad_m = nullptr;  // [N] gradient with respect to ln kx
  void* grad_t = nullptr;  // [3][N] gradient with respect to ln T of the +x, +y, +z face of
                           //   each cell (transmissibility form: dF/d ln T = F)
  double* grad_t_scale = nullptr;  // [3][N] sum of |terms| of grad_t
  void* grad_k3 = nullptr; // [3][N] gradient with respect to ln kx, ln ky, ln kz (per-direction
                           //   permeability arrays: each face depends on its own direction's k)
  double* grad_k3_scale = nullptr;  // [3][N] sum of |terms| of grad_k3
  double* scale = nullptr; // [2][N]: sum |F_KL|, sum |dF_KL/dp_K|
  double* dphi = nullptr;  // [3][N]: dPhi of the face (c, c + e_a) seen from c; NaN if absent
};

template <class S>
void assemble(const Problem<S>& pb, const Outputs& o) {
  const oracle_grid& g = *pb.g;
  const int64_t N = pb.ncell();
  S* r = static_cast<S*>(o.r);
  S* J = static_cast<S*>(o.J);
  S* gp = static_cast<S*>(o.grad_p);
  S* gm = static_cast<S*>(o.grad_m);
  S* gt = static_cast<S*>(o.grad_t);
  S* gk = static_cast<S*>(o.grad_k3);

  // r := 0 (Algorithm 1), and the other accumulators
  S* jv = static_cast<S*>(o.jv);
  const S* v = static_cast<const S*>(o.v);
  for (int64_t c = 0; c < N; ++c) {
    if (r) r[c] = S(0);
    if (jv) jv[c] = S(0);
    if (J)
      for (int e = 0; e < 7; ++e) J[e * N + c] = S(0);
    if (gp) gp[c] = S(0);
    if (gm) gm[c] = S(0);
    if (gt)
      for (int a = 0; a < 3; ++a) gt[a * N + c] = S(0);
    if (o.grad_t_scale)
      for (int a = 0; a < 3; ++a) o.grad_t_scale[a * N + c] = 0.0;
    if (gk)
      for (int a = 0; a < 3; ++a) gk[a * N + c] = S(0);
    if (o.grad_k3_scale)
      for (int a = 0; a < 3; ++a) o.grad_k3_scale[a * N + c] = 0.0;
    if (o.scale) o.scale[c] = o.scale[N + c] = 0.0;
    if (o.dphi)
      for (int a = 0; a < 3; ++a) o.dphi[a * N + c] = NAN;
  }

  // for each cell K, for each neighbour L of K (Algorithm 1)
  for (int64_t k = 0; k < g.nz; ++k)
    for (int64_t j = 0; j < g.ny; ++j)
      for (int64_t i = 0; i < g.nx; ++i) {
        const int64_t K = i + g.nx * (j + g.ny * k);
        const int nn = pb.tne ? 10 : 6;
        if (pb.phi) {
          // accumulation term of Eq. (2): V_K (phi rho - phi_n rho_n) / dt
          const double vdt = (g.dx * g.dy * g.dz) / pb.dt;
          const S m1 = mass_density(pb, K, pb.p[K]);
          const S m0 = mass_density(pb, K, pb.p_prev[K]);
          const S dm = mass_density_dp(pb, K, pb.p[K]);
          if (r) r[K] += S(vdt) * (m1 - m0);
          if (J) J[K] += S(vdt) * dm;
          if (jv) jv[K] += (S(vdt) * dm) * v[K];
          if (o.scale) {
            o.scale[K] += vdt * (std::abs(real_part(m1)) + std::abs(real_part(m0)));
            o.scale[N + K] += vdt * std::abs(real_part(dm));
          }
        }
        for (int n = 0; n < nn; ++n) {
          const Nb nb = neighbour(g, i, j, k, n);
          if (!nb.exists) continue;
          const FluxKL<S> fl = flux(pb, K, nb.L, nb.axis, nb.side);
          if (r) r[K] += fl.F;
          if (J && n < 6) {
            J[K] += fl.dF_dpK;
            J[(1 + n) * N + K] = fl.dF_dpL;
          }
          if (jv) jv[K] += fl.dF_dpK * v[K] + fl.dF_dpL * v[nb.L];
          if (o.w) {
            const S wK = S(o.w[K]);
            if (gp) {
              gp[K] += wK * fl.dF_dpK;
              gp[nb.L] += wK * fl.dF_dpL;
            }
            // dUps/d ln k_K = Ups * k_L / (k_K + k_L); the ratios ry, rz cancel
            if (gm && real_part(fl.T) != 0.0) {
              const S ksum = fl.kK + fl.kL;
              gm[K] += wK * (fl.F * fl.kL / ksum);
              gm[nb.L] += wK * (fl.F * fl.kK / ksum);
            }
            // per-direction k: the face along axis a depends on k_a of its two
            // cells only, d F / d ln k_a,K = F k_a,L / (k_a,K + k_a,L)
            if (gk && nb.axis < 3 && real_part(fl.T) != 0.0) {
              const S ksum = fl.kK + fl.kL;
              const S tK = wK * (fl.F * fl.kL / ksum), tL = wK * (fl.F * fl.kK / ksum);
              gk[nb.axis * N + K] += tK;
              gk[nb.axis * N + nb.L] += tL;
              if (o.grad_k3_scale) {
                o.grad_k3_scale[nb.axis * N + K] += std::abs(real_part(tK));
                o.grad_k3_scale[nb.axis * N + nb.L] += std::abs(real_part(tL));
              }
            }
            // given T: d r_K / d ln T_KL = F_KL; T is stored on the face's lower cell
            if (gt && nb.axis < 3) {
              const int64_t lo = K < nb.L ? K : nb.L;
              gt[nb.axis * N + lo] += wK * fl.F;
              if (o.grad_t_scale)
                o.grad_t_scale[nb.axis * N + lo] += std::abs(real_part(wK * fl.F));
            }
          }
          if (o.scale) {
            o.scale[K] += std::abs(real_part(fl.F));
            o.scale[N + K] += std::abs(real_part(fl.dF_dpK));
          }
          if (o.dphi && n < 6 && nb.side > 0) o.dphi[nb.axis * N + K] = real_part(fl.dPhi);
        }
      }
}

// Rows of r and J for a list of cells, same inner loop as assemble().
void rows(const Problem<double>& pb, const int64_t* cells, int64_t n, double* r,
          double* J, double* scale, double* dphi) {
  const oracle_grid& g = *pb.g;
  for (int64_t q = 0; q < n; ++q) {
    const int64_t K = cells[q];
    const int64_t i = K % g.nx, j = (K / g.nx) % g.ny, k = K / (g.nx * g.ny);
    double rK = 0.0, s0 = 0.0, s1 = 0.0;
    double row[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < 6; ++e) {
      const Nb nb = neighbour(g, i, j, k, e);
      if (dphi) dphi[e * n + q] = NAN;
      if (!nb.exists) continue;
      const FluxKL<double> fl = flux(pb, K, nb.L, nb.axis, nb.side);
      rK += fl.F;
      row[0] += fl.dF_dpK;
      row[1 + e] = fl.dF_dpL;
      s0 += std::abs(fl.F);
      s1 += std::abs(fl.dF_dpK);
      if (dphi) dphi[e * n + q] = fl.dPhi;
    }
    if (r) r[q] = rK;
    if (J)
      for (int e = 0; e < 7; ++e) J[e * n + q] = row[e];
    if (scale) {
      scale[q] = s0;
      scale[n + q] = s1;
    }
  }
}

bool valid(const oracle_grid* g, const oracle_fluid* f, const void* p, const void* kx) {
  return g && f && p && kx && g->nx > 0 && g->ny > 0 && g->nz > 0 && g->dx > 0 &&
         g->dy > 0 && g->dz > 0 && f->mu > 0;
}

}  // namespace

extern "C" {

// r, J, grad_p, grad_logk, scale and dphi are each optional (NULL = not wanted);
// grad_p / grad_logk need w. ky/kz NULL means ry*kx / rz*kx. Returns 0, or -1 on
// invalid arguments.
int oracle_eval(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                const double* ky, const double* kz, double ry, double rz,
                const uint8_t* seal, const double* p, const int8_t* force,
                const double* w, double* r, double* J, double* grad_p,
                double* grad_logk, double* scale, double* dphi) {
  if (!valid(g, f, p, kx)) return -1;
  if ((grad_p || grad_logk) && !w) return -1;
  if (grad_logk && (ky || kz)) return -1;
  Problem<double> pb{g, f, p, kx, ky, kz, ry, rz, seal, force};
  Outputs o;
  o.r = r;
  o.J = J;
  o.w = w;
  o.grad_p = grad_p;
  o.grad_m = grad_logk;
  o.scale = scale;
  o.dphi = dphi;
  assemble(pb, o);
  return 0;
}

// r and the 7 Jacobian entries of the listed cells only (J as [7][n]); dphi
// (optional, [6][n]) receives the potential difference of each of the cell's
// six faces seen from the cell (NaN where the neighbour does not exist).
int oracle_rows(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                const double* ky, const double* kz, double ry, double rz,
                const uint8_t* seal, const double* p, const int8_t* force,
                const int64_t* cells, int64_t n, double* r, double* J, double* scale,
                double* dphi) {
  if (!valid(g, f, p, kx) || (n > 0 && !cells)) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  for (int64_t q = 0; q < n; ++q)
    if (cells[q] < 0 || cells[q] >= N) return -1;
  Problem<double> pb{g, f, p, kx, ky, kz, ry, rz, seal, force};
  rows(pb, cells, n, r, J, scale, dphi);
  return 0;
}

// Every input form at once: permeability (kx, ry, rz, seal) or given face
// transmissibilities (tx, ty, tz: then kx and seal are NULL); optional
// diagonal faces (tne, tse: the 10-flux stencil); optional accumulation term
// (phi non-NULL: phi, p_prev, dt, cr); outputs r, J, jv (needs v) and scale
// each optional.
int oracle_eval_general(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                        double ry, double rz, const uint8_t* seal, const double* tx,
                        const double* ty, const double* tz, const double* tne,
                        const double* tse, const double* p, const double* phi,
                        const double* p_prev, double dt, double cr, const double* v, double* r,
                        double* J, double* jv, double* scale) {
  const bool tin = tx || ty || tz;
  if (!g || !f || !p || (!kx && !tin)) return -1;
  if (tin && (!tx || !ty || !tz || kx || seal)) return -1;
  if (!(g->nx > 0 && g->ny > 0 && g->nz > 0 && g->dx > 0 && g->dy > 0 && g->dz > 0 &&
        f->mu > 0))
    return -1;
  if ((tne != nullptr) != (tse != nullptr)) return -1;
  if (phi && (!p_prev || !(dt > 0.0))) return -1;
  if (jv && !v) return -1;
  Problem<double> pb{g, f, p, kx, nullptr, nullptr, ry, rz, seal, nullptr};
  pb.tx = tx;
  pb.ty = ty;
  pb.tz = tz;
  pb.tne = tne;
  pb.tse = tse;
  pb.phi = phi;
  pb.p_prev = p_prev;
  pb.dt = dt;
  pb.cr = cr;
  Outputs o;
  o.r = r;
  o.J = J;
  o.v = v;
  o.jv = jv;
  o.scale = scale;
  assemble(pb, o);
  return 0;
}

// Vector-Jacobian product with cotangent w in either rock form: grad_p = J^T w,
// and in the transmissibility form grad_t[a][c] = d(w.r)/d ln T of the face
// between c and its +a neighbour, with grad_t_scale the sum of |terms|.
int oracle_vjp_general(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                       double ry, double rz, const uint8_t* seal, const double* tx,
                       const double* ty, const double* tz, const double* p, const double* w,
                       double* grad_p, double* grad_t, double* grad_t_scale) {
  const bool tin = tx || ty || tz;
  if (!g || !f || !p || !w || (!kx && !tin)) return -1;
  if (tin && (!tx || !ty || !tz || kx || seal)) return -1;
  if (grad_t && !tin) return -1;
  Problem<double> pb{g, f, p, kx, nullptr, nullptr, ry, rz, seal, nullptr};
  pb.tx = tx;
  pb.ty = ty;
  pb.tz = tz;
  Outputs o;
  o.w = w;
  o.grad_p = grad_p;
  o.grad_t = grad_t;
  o.grad_t_scale = grad_t_scale;
  assemble(pb, o);
  return 0;
}

// Complex-step directional derivative of the transmissibility-form residual
// with respect to ln T along d = (dx, dy, dz) (one direction per face array):
// r_im = Im r(T exp(i h d)).
int oracle_trans_cs(const oracle_grid* g, const oracle_fluid* f, const double* tx,
                    const double* ty, const double* tz, const double* p, const double* d,
                    double h, double* r_im) {
  if (!g || !f || !tx || !ty || !tz || !p || !d || !r_im) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  cplx* pc = new cplx[N];
  cplx* t[3] = {new cplx[N], new cplx[N], new cplx[N]};
  const double* src[3] = {tx, ty, tz};
  cplx* rc = new cplx[N];
  for (int64_t q = 0; q < N; ++q) {
    pc[q] = cplx(p[q], 0.0);
    for (int a = 0; a < 3; ++a) t[a][q] = src[a][q] * std::exp(cplx(0.0, h * d[a * N + q]));
  }
  Problem<cplx> pb{g, f, pc, nullptr, nullptr, nullptr, 1.0, 1.0, nullptr, nullptr};
  pb.tx = t[0];
  pb.ty = t[1];
  pb.tz = t[2];
  Outputs o;
  o.r = rc;
  assemble(pb, o);
  for (int64_t q = 0; q < N; ++q) r_im[q] = rc[q].imag();
  delete[] pc;
  for (cplx* a : t) delete[] a;
  delete[] rc;
  return 0;
}

// Complex-step J vp of the same general residual (transmissibilities and
// porosity are real inputs).
int oracle_eval_general_cs(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                           double ry, double rz, const uint8_t* seal, const double* tx,
                           const double* ty, const double* tz, const double* tne,
                           const double* tse, const double* p, const double* phi,
                           const double* p_prev, double dt, double cr, const double* vp,
                           double h, double* r_im) {
  const bool tin = tx || ty || tz;
  if (!g || !f || !p || !vp || !r_im || (!kx && !tin)) return -1;
  if (tin && (!tx || !ty || !tz || kx || seal)) return -1;
  if (phi && (!p_prev || !(dt > 0.0))) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  auto widen = [N](const double* a) -> cplx* {
    if (!a) return nullptr;
    cplx* c = new cplx[N];
    for (int64_t q = 0; q < N; ++q) c[q] = cplx(a[q], 0.0);
    return c;
  };
  cplx* pc = new cplx[N];
  for (int64_t q = 0; q < N; ++q) pc[q] = cplx(p[q], h * vp[q]);
  cplx *kc = widen(kx), *xc = widen(tx), *yc = widen(ty), *zc = widen(tz), *nc = widen(tne),
       *sc = widen(tse), *fc = widen(phi), *qc = widen(p_prev);
  cplx* rc = new cplx[N];
  Problem<cplx> pb{g, f, pc, kc, nullptr, nullptr, ry, rz, seal, nullptr};
  pb.tx = xc;
  pb.ty = yc;
  pb.tz = zc;
  pb.tne = nc;
  pb.tse = sc;
  pb.phi = fc;
  pb.p_prev = qc;
  pb.dt = dt;
  pb.cr = cr;
  Outputs o;
  o.r = rc;
  assemble(pb, o);
  for (int64_t q = 0; q < N; ++q) r_im[q] = rc[q].imag();
  for (cplx* a : {pc, kc, xc, yc, zc, nc, sc, fc, qc, rc}) delete[] a;
  return 0;
}

// Full backward-Euler residual of Eq. (2): accumulation term plus the flux
// sum, with phi_ref, p_prev, dt, cr as in the header. r, J, jv (= J v, needs
// v) and scale ([2][N]: sum of |terms| of r and of the diagonal) are optional.
int oracle_eval_be(const oracle_grid* g, const oracle_fluid* f, const double* kx, double ry,
                   double rz, const uint8_t* seal, const double* p, const double* phi,
                   const double* p_prev, double dt, double cr, const double* v, double* r,
                   double* J, double* jv, double* scale) {
  if (!valid(g, f, p, kx) || !phi || !p_prev || !(dt > 0.0)) return -1;
  if (jv && !v) return -1;
  Problem<double> pb{g, f, p, kx, nullptr, nullptr, ry, rz, seal, nullptr};
  pb.phi = phi;
  pb.p_prev = p_prev;
  pb.dt = dt;
  pb.cr = cr;
  Outputs o;
  o.r = r;
  o.J = J;
  o.v = v;
  o.jv = jv;
  o.scale = scale;
  assemble(pb, o);
  return 0;
}

// Complex-step directional derivative of the full backward-Euler residual
// along vp: r_im = Im r(p + i h vp), so r_im / h = J vp to rounding.
int oracle_eval_be_cs(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                      double ry, double rz, const uint8_t* seal, const double* p,
                      const double* phi, const double* p_prev, double dt, double cr,
                      const double* vp, double h, double* r_im) {
  if (!valid(g, f, p, kx) || !phi || !p_prev || !vp || !r_im || !(dt > 0.0)) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  cplx* pc = new cplx[N];
  cplx* kc = new cplx[N];
  cplx* fc = new cplx[N];
  cplx* qc = new cplx[N];
  cplx* rc = new cplx[N];
  for (int64_t c = 0; c < N; ++c) {
    pc[c] = cplx(p[c], h * vp[c]);
    kc[c] = cplx(kx[c], 0.0);
    fc[c] = cplx(phi[c], 0.0);
    qc[c] = cplx(p_prev[c], 0.0);
  }
  Problem<cplx> pb{g, f, pc, kc, nullptr, nullptr, ry, rz, seal, nullptr};
  pb.phi = fc;
  pb.p_prev = qc;
  pb.dt = dt;
  pb.cr = cr;
  Outputs o;
  o.r = rc;
  assemble(pb, o);
  for (int64_t c = 0; c < N; ++c) r_im[c] = rc[c].imag();
  delete[] pc;
  delete[] kc;
  delete[] fc;
  delete[] qc;
  delete[] rc;
  return 0;
}

// Residual of the 10-flux stencil: the six TPFA faces plus the four in-plane
// diagonal faces, whose transmissibilities are given per cell (tne: face with
// (i+1, j+1), tse: face with (i+1, j-1); entries without that neighbour are
// ignored). Optionally the flux scale sum |F| per cell. `force` (NULL or
// [5][N]) overrides the upwind choice of a face (+1 lower, -1 upper cell,
// 0 the rule): planes 0-2 the x, y, z faces by their lower cell, planes 3-4
// the diagonal faces (i,j)-(i+1,j+1) and (i,j)-(i+1,j-1) by their left end.
int oracle_residual10(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                      double ry, double rz, const uint8_t* seal, const double* tne,
                      const double* tse, const double* p, const int8_t* force, double* r,
                      double* scale) {
  if (!valid(g, f, p, kx) || !tne || !tse || !r) return -1;
  Problem<double> pb{g, f, p, kx, nullptr, nullptr, ry, rz, seal, force};
  if (force) pb.force_diag = force + 3 * pb.ncell();
  pb.tne = tne;
  pb.tse = tse;
  Outputs o;
  o.r = r;
  o.scale = scale;
  assemble(pb, o);
  return 0;
}

// Complex-step residual of the 10-flux stencil along a pressure direction vp.
int oracle_residual10_cs(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                         double ry, double rz, const uint8_t* seal, const double* tne,
                         const double* tse, const double* p, const double* vp, double h,
                         double* r_im) {
  if (!valid(g, f, p, kx) || !tne || !tse || !vp || !r_im) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  cplx* pc = new cplx[N];
  cplx* kc = new cplx[N];
  cplx* tn = new cplx[N];
  cplx* ts = new cplx[N];
  cplx* rc = new cplx[N];
  for (int64_t c = 0; c < N; ++c) {
    pc[c] = cplx(p[c], h * vp[c]);
    kc[c] = cplx(kx[c], 0.0);
    tn[c] = cplx(tne[c], 0.0);
    ts[c] = cplx(tse[c], 0.0);
  }
  Problem<cplx> pb{g, f, pc, kc, nullptr, nullptr, ry, rz, seal, nullptr};
  pb.tne = tn;
  pb.tse = ts;
  Outputs o;
  o.r = rc;
  assemble(pb, o);
  for (int64_t c = 0; c < N; ++c) r_im[c] = rc[c].imag();
  delete[] pc;
  delete[] kc;
  delete[] tn;
  delete[] ts;
  delete[] rc;
  return 0;
}

// The same residual and Jacobian evaluated in long double (inputs widened).
int oracle_eval_ld(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                   double ry, double rz, const uint8_t* seal, const double* p,
                   long double* r, long double* J) {
  if (!valid(g, f, p, kx)) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  long double* pl = (long double*)std::malloc(sizeof(long double) * N);
  long double* kl = (long double*)std::malloc(sizeof(long double) * N);
  if (!pl || !kl) {
    std::free(pl);
    std::free(kl);
    return -1;
  }
  for (int64_t c = 0; c < N; ++c) {
    pl[c] = p[c];
    kl[c] = kx[c];
  }
  Problem<long double> pb{g, f, pl, kl, nullptr, nullptr, ry, rz, seal, nullptr};
  Outputs o;
  o.r = r;
  o.J = J;
  assemble(pb, o);
  std::free(pl);
  std::free(kl);
  return 0;
}

// Complex-step evaluation: p -> p + i h vp and ln kx -> ln kx + i h vm (either
// direction may be NULL). Writes Re r and Im r; Im r / h is the directional
// derivative of r along (vp, vm) to machine precision away from upwind switches.
int oracle_eval_cs(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                   double ry, double rz, const uint8_t* seal, const double* p,
                   const double* vp, const double* vm, double h, double* r_re,
                   double* r_im) {
  if (!valid(g, f, p, kx) || !r_re || !r_im) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  cplx* pc = new cplx[N];
  cplx* kc = new cplx[N];
  cplx* rc = new cplx[N];
  for (int64_t c = 0; c < N; ++c) {
    pc[c] = cplx(p[c], vp ? h * vp[c] : 0.0);
    // exp(ln kx + i h vm) = kx * exp(i h vm)
    kc[c] = vm ? kx[c] * std::exp(cplx(0.0, h * vm[c])) : cplx(kx[c], 0.0);
  }
  Problem<cplx> pb{g, f, pc, kc, nullptr, nullptr, ry, rz, seal, nullptr};
  Outputs o;
  o.r = rc;
  assemble(pb, o);
  for (int64_t c = 0; c < N; ++c) {
    r_re[c] = rc[c].real();
    r_im[c] = rc[c].imag();
  }
  delete[] pc;
  delete[] kc;
  delete[] rc;
  return 0;
}

// Per-direction permeability form: kx, ky, kz given per cell (each face along
// axis a takes the harmonic average of k_a of its two cells; no ratios), with
// seal bits, optional diagonal faces (tne, tse), optional accumulation term
// (phi non-NULL: phi, p_prev, dt, cr). Outputs r, J, jv (needs v), scale
// ([2][N]), and with w: grad_p = J^T w, grad_k3[a][c] = d(w.r)/d ln k_a[c] and
// grad_k3_scale (sum of |terms|); each optional.
int oracle_eval_k3(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                   const double* ky, const double* kz, const uint8_t* seal, const double* tne,
                   const double* tse, const double* p, const double* phi, const double* p_prev,
                   double dt, double cr, const double* v, const double* w, double* r,
                   double* J, double* jv, double* scale, double* grad_p, double* grad_k3,
                   double* grad_k3_scale) {
  if (!valid(g, f, p, kx) || !ky || !kz) return -1;
  if ((tne != nullptr) != (tse != nullptr)) return -1;
  if (phi && (!p_prev || !(dt > 0.0))) return -1;
  if (jv && !v) return -1;
  if ((grad_p || grad_k3 || grad_k3_scale) && !w) return -1;
  Problem<double> pb{g, f, p, kx, ky, kz, 1.0, 1.0, seal, nullptr};
  pb.tne = tne;
  pb.tse = tse;
  pb.phi = phi;
  pb.p_prev = p_prev;
  pb.dt = dt;
  pb.cr = cr;
  Outputs o;
  o.r = r;
  o.J = J;
  o.v = v;
  o.jv = jv;
  o.scale = scale;
  o.w = w;
  o.grad_p = grad_p;
  o.grad_k3 = grad_k3;
  o.grad_k3_scale = grad_k3_scale;
  assemble(pb, o);
  return 0;
}

// Complex-step evaluation of the same form: p -> p + i h vp and
// ln k_a -> ln k_a + i h dk[a] (a = x, y, z; vp and dk may each be NULL).
// Im r / h is the directional derivative of r along (vp, dk).
int oracle_eval_k3_cs(const oracle_grid* g, const oracle_fluid* f, const double* kx,
                      const double* ky, const double* kz, const uint8_t* seal,
                      const double* tne, const double* tse, const double* p, const double* phi,
                      const double* p_prev, double dt, double cr, const double* vp,
                      const double* dk, double h, double* r_im) {
  if (!valid(g, f, p, kx) || !ky || !kz || !r_im) return -1;
  if ((tne != nullptr) != (tse != nullptr)) return -1;
  if (phi && (!p_prev || !(dt > 0.0))) return -1;
  const int64_t N = g->nx * g->ny * g->nz;
  auto widen = [N](const double* a) -> cplx* {
    if (!a) return nullptr;
    cplx* c = new cplx[N];
    for (int64_t q = 0; q < N; ++q) c[q] = cplx(a[q], 0.0);
    return c;
  };
  cplx* pc = new cplx[N];
  cplx* kc[3] = {new cplx[N], new cplx[N], new cplx[N]};
  const double* ks[3] = {kx, ky, kz};
  for (int64_t q = 0; q < N; ++q) {
    pc[q] = cplx(p[q], vp ? h * vp[q] : 0.0);
    // exp(ln k + i h d) = k exp(i h d)
    for (int a = 0; a < 3; ++a)
      kc[a][q] = dk ? ks[a][q] * std::exp(cplx(0.0, h * dk[a * N + q])) : cplx(ks[a][q], 0.0);
  }
  cplx *nc = widen(tne), *sc = widen(tse), *fc = widen(phi), *qc = widen(p_prev);
  cplx* rc = new cplx[N];
  Problem<cplx> pb{g, f, pc, kc[0], kc[1], kc[2], 1.0, 1.0, seal, nullptr};
  pb.tne = nc;
  pb.tse = sc;
  pb.phi = fc;
  pb.p_prev = qc;
  pb.dt = dt;
  pb.cr = cr;
  Outputs o;
  o.r = rc;
  assemble(pb, o);
  for (int64_t q = 0; q < N; ++q) r_im[q] = rc[q].imag();
  for (cplx* a : {pc, kc[0], kc[1], kc[2], nc, sc, fc, qc, rc}) delete[] a;
  return 0;
}

// Discrete hydrostatic column: pref[0] = p_top and, for every k,
// pref[k+1] - pref[k] = (rho(pref[k]) + rho(pref[k+1])) / 2 * gk * dz, so that the
// potential difference of the vertical face between two reference cells is zero.
// Solved level by level with Newton's method until the iterate stops changing.
int oracle_hydrostatic(const oracle_grid* g, const oracle_fluid* f, double p_top,
                       double* pref) {
  if (!g || !f || !pref || g->nz <= 0) return -1;
  const double G = g->gk * g->dz;
  pref[0] = p_top;
  for (int64_t k = 0; k + 1 < g->nz; ++k) {
    const double pk = pref[k];
    const double rk = density(pk, *f);
    double x = pk + rk * G;
    for (int it = 0; it < 100; ++it) {
      const double rx = density(x, *f);
      const double res = x - pk - 0.5 * (rk + rx) * G;
      const double der = 1.0 - 0.5 * f->cf * rx * G;
      const double xn = x - res / der;
      if (xn == x) break;
      x = xn;
    }
    pref[k + 1] = x;
  }
  return 0;
}

}  // extern "C"
