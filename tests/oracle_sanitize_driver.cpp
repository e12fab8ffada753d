// Host-only driver that runs every exported function of the CPU oracle on
// small odd grids; built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_oracle_sanitized.py to check the oracle's memory accesses and
// arithmetic for undefined behaviour. Test infrastructure only.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
typedef struct {
  int64_t nx, ny, nz;
  double dx, dy, dz;
  double gk;
} oracle_grid;
typedef struct {
  double rho_ref, cf, p_ref, mu;
} oracle_fluid;
int oracle_eval(const oracle_grid*, const oracle_fluid*, const double*, const double*,
                const double*, double, double, const uint8_t*, const double*, const int8_t*,
                const double*, double*, double*, double*, double*, double*, double*);
int oracle_rows(const oracle_grid*, const oracle_fluid*, const double*, const double*,
                const double*, double, double, const uint8_t*, const double*, const int8_t*,
                const int64_t*, int64_t, double*, double*, double*, double*);
int oracle_eval_ld(const oracle_grid*, const oracle_fluid*, const double*, double, double,
                   const uint8_t*, const double*, long double*, long double*);
int oracle_eval_cs(const oracle_grid*, const oracle_fluid*, const double*, double, double,
                   const uint8_t*, const double*, const double*, const double*, double, double*,
                   double*);
int oracle_hydrostatic(const oracle_grid*, const oracle_fluid*, double, double*);
int oracle_residual10(const oracle_grid*, const oracle_fluid*, const double*, double, double,
                      const uint8_t*, const double*, const double*, const double*,
                      const int8_t*, double*, double*);
int oracle_eval_be(const oracle_grid*, const oracle_fluid*, const double*, double, double,
                   const uint8_t*, const double*, const double*, const double*, double, double,
                   const double*, double*, double*, double*, double*);
int oracle_eval_general(const oracle_grid*, const oracle_fluid*, const double*, double, double,
                        const uint8_t*, const double*, const double*, const double*,
                        const double*, const double*, const double*, const double*,
                        const double*, double, double, const double*, double*, double*,
                        double*, double*);
int oracle_vjp_general(const oracle_grid*, const oracle_fluid*, const double*, double, double,
                       const uint8_t*, const double*, const double*, const double*,
                       const double*, const double*, double*, double*, double*);
int oracle_trans_cs(const oracle_grid*, const oracle_fluid*, const double*, const double*,
                    const double*, const double*, const double*, double, double*);
int oracle_eval_k3(const oracle_grid*, const oracle_fluid*, const double*, const double*,
                   const double*, const uint8_t*, const double*, const double*, const double*,
                   const double*, const double*, double, double, const double*, const double*,
                   double*, double*, double*, double*, double*, double*, double*);
int oracle_eval_k3_cs(const oracle_grid*, const oracle_fluid*, const double*, const double*,
                      const double*, const uint8_t*, const double*, const double*,
                      const double*, const double*, const double*, double, double,
                      const double*, const double*, double, double*);
}

static double unif(uint64_t& s, double a, double b) {
  s = s * 6364136223846793005ULL + 1442695040888963407ULL;
  return a + (b - a) * ((s >> 11) * (1.0 / 9007199254740992.0));
}

int main() {
  const int64_t shapes[][3] = {{1, 1, 1}, {3, 5, 7}, {7, 1, 2}, {1, 6, 3}, {4, 4, 4}};
  oracle_fluid fl{1000.0, 1e-9, 1e7, 1e-3};
  int fails = 0;
  uint64_t s = 12345;
  for (const auto& sh : shapes) {
    oracle_grid g{sh[0], sh[1], sh[2], 10.0, 10.0, 2.0, 9.81};
    const int64_t N = sh[0] * sh[1] * sh[2];
    std::vector<double> k(N), p(N), w(N), v(N), phi(N), pn(N), t(5 * N), d(3 * N);
    std::vector<uint8_t> seal(N);
    for (int64_t c = 0; c < N; ++c) {
      k[c] = 1e-13 * unif(s, 0.1, 10.0);
      p[c] = 1e7 + unif(s, -1e5, 1e5);
      w[c] = unif(s, -1, 1);
      v[c] = unif(s, -1, 1);
      phi[c] = unif(s, 0.1, 0.3);
      pn[c] = p[c] + unif(s, -1e4, 1e4);
      seal[c] = (uint8_t)(unif(s, 0, 8));
    }
    for (auto& x : t) x = 1e-13 * unif(s, 0.0, 5.0);
    for (auto& x : d) x = unif(s, -1, 1);
    std::vector<double> r(N), J(7 * N), gp(N), gm(N), sc(2 * N), dphi(3 * N), ri(N), jv(N),
        gt(3 * N), gs(3 * N), pref(sh[2]);
    std::vector<long double> rl(N), Jl(7 * N);
    std::vector<int64_t> cells = {0, N - 1, N / 2};
    fails += oracle_eval(&g, &fl, k.data(), nullptr, nullptr, 1.0, 0.1, seal.data(), p.data(),
                         nullptr, w.data(), r.data(), J.data(), gp.data(), gm.data(), sc.data(),
                         dphi.data()) != 0;
    // rows outputs are [.][n] for the n sampled cells
    std::vector<double> rr(3), rJ(7 * 3), rs(2 * 3), rd(6 * 3);
    fails += oracle_rows(&g, &fl, k.data(), nullptr, nullptr, 1.0, 0.1, seal.data(), p.data(),
                         nullptr, cells.data(), 3, rr.data(), rJ.data(), rs.data(),
                         rd.data()) != 0;
    fails += oracle_eval_ld(&g, &fl, k.data(), 1.0, 0.1, seal.data(), p.data(), rl.data(),
                            Jl.data()) != 0;
    fails += oracle_eval_cs(&g, &fl, k.data(), 1.0, 0.1, seal.data(), p.data(), v.data(),
                            nullptr, 1e-20, r.data(), ri.data()) != 0;
    fails += oracle_hydrostatic(&g, &fl, 1e7, pref.data()) != 0;
    fails += oracle_residual10(&g, &fl, k.data(), 1.0, 0.1, seal.data(), t.data(),
                               t.data() + N, p.data(), nullptr, r.data(), sc.data()) != 0;
    {
      std::vector<int8_t> f5(5 * N);
      for (int64_t c = 0; c < 5 * N; ++c) f5[c] = (int8_t)(c % 3 - 1);
      fails += oracle_residual10(&g, &fl, k.data(), 1.0, 0.1, seal.data(), t.data(),
                                 t.data() + N, p.data(), f5.data(), r.data(), sc.data()) != 0;
    }
    fails += oracle_eval_be(&g, &fl, k.data(), 1.0, 0.1, seal.data(), p.data(), phi.data(),
                            pn.data(), 3600.0, 5e-10, v.data(), r.data(), J.data(), jv.data(),
                            sc.data()) != 0;
    fails += oracle_eval_general(&g, &fl, nullptr, 1.0, 1.0, nullptr, t.data(), t.data() + N,
                                 t.data() + 2 * N, t.data() + 3 * N, t.data() + 4 * N, p.data(),
                                 phi.data(), pn.data(), 3600.0, 5e-10, v.data(), r.data(),
                                 J.data(), jv.data(), sc.data()) != 0;
    fails += oracle_vjp_general(&g, &fl, nullptr, 1.0, 1.0, nullptr, t.data(), t.data() + N,
                                t.data() + 2 * N, p.data(), w.data(), gp.data(), gt.data(),
                                gs.data()) != 0;
    fails += oracle_trans_cs(&g, &fl, t.data(), t.data() + N, t.data() + 2 * N, p.data(),
                             d.data(), 1e-20, ri.data()) != 0;
    std::vector<double> gk(3 * N), gks(3 * N);
    fails += oracle_eval_k3(&g, &fl, k.data(), t.data(), t.data() + N, seal.data(),
                            t.data() + 2 * N, t.data() + 3 * N, p.data(), phi.data(), pn.data(),
                            3600.0, 5e-10, v.data(), w.data(), r.data(), J.data(), jv.data(),
                            sc.data(), gp.data(), gk.data(), gks.data()) != 0;
    fails += oracle_eval_k3_cs(&g, &fl, k.data(), t.data(), t.data() + N, seal.data(),
                               t.data() + 2 * N, t.data() + 3 * N, p.data(), phi.data(),
                               pn.data(), 3600.0, 5e-10, v.data(), d.data(), 1e-20,
                               ri.data()) != 0;
  }
  std::printf("oracle sanitizer driver: %d failed calls\n", fails);
  return fails == 0 ? 0 : 1;
}
