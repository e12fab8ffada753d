"""Pins of the oracle's full backward-Euler residual, Eq. (2) (accumulation
term V (phi rho - phi_n rho_n) / dt plus the flux sum of Algorithm 1, porosity
linear in p) and of its Jacobian-vector product:

* one-cell closed form in 50-digit decimal arithmetic (value and derivative);
* complex-step directional derivative of the full residual against jv;
* reductions: phi = 0 or p = p_prev give the flux residual bit for bit;
* jv against SciPy's sparse product of the oracle's J with v;
* conservation: the residuals sum to the total accumulation.
"""
from decimal import Decimal as D, getcontext

import numpy as np
import pytest

import geomodel
from helpers import apply_J, sparse_J

getcontext().prec = 50
FL = geomodel.Fluid()
DT, CR = 3600.0, 5e-10


def rho_dec(p):
    return D(FL.rho0) * (D(FL.cf) * (D(p) - D(FL.p0))).exp()


def phi_dec(phi_ref, p):
    return D(phi_ref) * (1 + D(CR) * (D(p) - D(FL.p0)))


def test_single_cell_closed_form(orc):
    g = geomodel.Grid(1, 1, 1)
    p, pn, phi = 1.03e7, 1.01e7, 0.2
    out = orc.evaluate_be(g, FL, np.full((1, 1, 1), 1e-13), np.full((1, 1, 1), p),
                          np.full((1, 1, 1), phi), np.full((1, 1, 1), pn), DT, CR,
                          v=np.ones((1, 1, 1)), want=("r", "J", "jv", "scale"))
    vdt = D(g.dx) * D(g.dy) * D(g.dz) / D(DT)
    r = vdt * (phi_dec(phi, p) * rho_dec(p) - phi_dec(phi, pn) * rho_dec(pn))
    dr = vdt * (D(phi) * D(CR) * rho_dec(p) + phi_dec(phi, p) * D(FL.cf) * rho_dec(p))
    scale = float(vdt * (phi_dec(phi, p) * rho_dec(p) + phi_dec(phi, pn) * rho_dec(pn)))
    assert abs(out["r"].item() - float(r)) <= 4e-16 * scale
    assert abs(out["J"][0].item() - float(dr)) <= 4e-16 * abs(float(dr))
    assert np.all(out["J"][1:] == 0.0)
    assert out["jv"].item() == out["J"][0].item()
    assert out["scale"][0].item() == pytest.approx(scale, rel=1e-15)


def be_case(shape, seed):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed, nx, ny, nz, seal_prob=0.05, sigma=1.2)
    rng = np.random.default_rng(seed + 1000)
    phi = rng.uniform(0.1, 0.3, geo.grid.shape)
    return geo, phi, rng


@pytest.mark.parametrize("shape", [(3, 4, 5), (7, 1, 3), (1, 5, 6), (6, 6, 2), (2, 3, 9)])
def test_jvp_matches_complex_step(orc, shape):
    geo, phi, rng = be_case(shape, 31 + sum(shape))
    p = orc.pressure(geo)
    p_prev = p - rng.uniform(-5e4, 5e4, p.shape)
    v = rng.standard_normal(p.shape)
    out = orc.evaluate_be(geo.grid, geo.fluid, geo.kx, p, phi, p_prev, DT, CR, ry=geo.ry,
                          rz=geo.rz, seal=geo.seal, v=v, want=("jv", "J"))
    cs = orc.evaluate_be_cs(geo.grid, geo.fluid, geo.kx, p, phi, p_prev, DT, CR, v, ry=geo.ry,
                            rz=geo.rz, seal=geo.seal)
    scale = apply_J(np.abs(out["J"]), np.abs(v))
    assert np.all(np.abs(out["jv"] - cs) <= 1e-13 * scale + 1e-300)


def test_jv_is_sparse_J_times_v(orc):
    geo, phi, rng = be_case((9, 7, 5), 77)
    p = orc.pressure(geo)
    p_prev = orc.pressure(geo) + rng.uniform(-1e4, 1e4, p.shape)
    v = rng.standard_normal(p.shape)
    out = orc.evaluate_be(geo.grid, geo.fluid, geo.kx, p, phi, p_prev, DT, CR, ry=geo.ry,
                          rz=geo.rz, seal=geo.seal, v=v, want=("J", "jv"))
    ref = sparse_J(out["J"]) @ v.ravel()
    scale = apply_J(np.abs(out["J"]), np.abs(v)).ravel()
    assert np.all(np.abs(out["jv"].ravel() - ref) <= 1e-14 * scale)


@pytest.mark.parametrize("case", ["phi0", "same_p"])
def test_reduces_to_flux_residual(orc, case):
    geo, phi, rng = be_case((8, 5, 6), 5)
    p = orc.pressure(geo)
    if case == "phi0":
        phi = np.zeros_like(phi)
        p_prev = p + rng.uniform(-1e5, 1e5, p.shape)
    else:
        p_prev = p.copy()
    be = orc.evaluate_be(geo.grid, geo.fluid, geo.kx, p, phi, p_prev, DT, CR, ry=geo.ry,
                         rz=geo.rz, seal=geo.seal, want=("r", "J"))
    fx = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert np.array_equal(be["r"], fx["r"])
    if case == "phi0":
        assert np.array_equal(be["J"], fx["J"])
    else:  # the accumulation derivative remains on the diagonal
        assert np.array_equal(be["J"][1:], fx["J"][1:])
        assert np.all(be["J"][0] > fx["J"][0] - 1e-30)


def test_conservation_total_accumulation(orc):
    geo, phi, rng = be_case((10, 6, 7), 12)
    p = orc.pressure(geo)
    p_prev = p + rng.uniform(-1e5, 1e5, p.shape)
    out = orc.evaluate_be(geo.grid, geo.fluid, geo.kx, p, phi, p_prev, DT, CR, ry=geo.ry,
                          rz=geo.rz, seal=geo.seal, want=("r", "scale"))
    vdt = geo.grid.dx * geo.grid.dy * geo.grid.dz / DT
    rho = lambda q: FL.rho0 * np.exp(FL.cf * (q - FL.p0))  # noqa: E731
    ph = lambda q: phi * (1 + CR * (q - FL.p0))  # noqa: E731
    total = vdt * np.sum(ph(p) * rho(p) - ph(p_prev) * rho(p_prev))
    assert abs(out["r"].sum() - total) <= 64 * out["r"].size * 1.2e-16 * out["scale"][0].sum()
