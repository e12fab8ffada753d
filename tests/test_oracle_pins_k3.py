"""Pins of the oracle's per-direction permeability form (kx, ky, kz given per
cell; each face takes the two-point harmonic average of its own direction's
permeability, Sec. 3): two-cell closed forms in 50-digit decimal arithmetic,
independence of the other directions' arrays, the x <-> y transposition
symmetry, the reduction to the ratio form, conservation, and complex-step
derivatives with respect to p and to ln kx, ln ky, ln kz one direction at a
time (so that a gradient filed under the wrong axis fails)."""
from decimal import Decimal as D, getcontext

import numpy as np
import pytest

import geomodel
from helpers import apply_J

getcontext().prec = 50
FL = geomodel.Fluid()


def rho_dec(p):
    return D(FL.rho0) * (D(FL.cf) * (D(p) - D(FL.p0))).exp()


def harm(a, b):
    return D(2) * (D(a) * D(b)) / (D(a) + D(b))


def test_two_cell_y_closed_form(orc):
    """Two cells along y: only ky enters; kx and kz may be anything."""
    g = geomodel.Grid(1, 2, 1)
    p = np.array([1.02e7, 1.0e7]).reshape(1, 2, 1)
    ky = np.array([2e-13, 7e-13]).reshape(1, 2, 1)
    T = D(g.dx) * D(g.dz) / D(g.dy) * harm(2e-13, 7e-13)
    F = T * rho_dec(1.02e7) / D(FL.mu) * (D(1.02e7) - D(1.0e7))  # cell 0 upwind
    dFL = T * (-rho_dec(1.02e7) / D(FL.mu))  # d F / d p_1: only the potential moves
    for kx, kz in ((np.full((1, 2, 1), 1e-13), np.full((1, 2, 1), 3e-14)),
                   (np.array([5e-10, 1e-20]).reshape(1, 2, 1), np.zeros((1, 2, 1)))):
        out = orc.evaluate_k3(g, FL, p, kx, ky, kz, want=("r", "J"))
        r = out["r"].ravel()
        assert abs(r[0] - float(F)) <= 2e-16 * abs(float(F)) and r[1] == -r[0]
        assert abs(out["J"][4].ravel()[0] - float(dFL)) <= 2e-16 * abs(float(dFL))


def test_two_cell_z_closed_form_with_gravity(orc):
    g = geomodel.Grid(1, 1, 2, gk=9.81)
    p = np.array([1.0e7, 1.0e7 + 4e4]).reshape(2, 1, 1)
    kz = np.array([9e-14, 4e-14]).reshape(2, 1, 1)
    kx = ky = np.full((2, 1, 1), 1e-12)
    r = orc.evaluate_k3(g, FL, p, kx, ky, kz)["r"].ravel()
    r0, r1 = rho_dec(1.0e7), rho_dec(1.0e7 + 4e4)
    dphi = (D(1.0e7) - D(1.0e7 + 4e4)) + (r0 + r1) / 2 * D(9.81) * D(g.dz)
    lam = (r0 if dphi >= 0 else r1) / D(FL.mu)
    F = D(g.dx) * D(g.dy) / D(g.dz) * harm(9e-14, 4e-14) * lam * dphi
    assert abs(r[0] - float(F)) <= 4e-16 * abs(float(F)) and r[1] == -r[0]


def _model(seed=3, shape=(6, 5, 4), seal_prob=0.1):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed, nx, ny, nz, sigma=1.2, seal_prob=seal_prob)
    kx, ky, kz = geomodel.k3_fields(geo.kx, seed + 100)
    return geo, kx, ky, kz


def test_ratio_arrays_reduce_to_ratio_form(orc):
    """ky = ry kx and kz = rz kx as arrays give the ratio form's r and J
    exactly, and the three gradient planes sum to its d(w.r)/d ln kx."""
    geo = geomodel.random_small(5, 7, 6, 5, sigma=1.5, seal_prob=0.1, ry=0.7, rz=0.1)
    p = orc.pressure(geo)
    w = np.random.default_rng(2).standard_normal(geo.grid.shape)
    ky, kz = geo.ry * geo.kx, geo.rz * geo.kx
    a = orc.evaluate_k3(geo.grid, geo.fluid, p, geo.kx, ky, kz, seal=geo.seal, w=w,
                        want=("r", "J", "grad_p", "grad_k3", "grad_k3_scale"))
    b = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal, w=w,
                     want=("r", "J", "grad_p", "grad_logk"))
    assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["J"], b["J"])
    assert np.array_equal(a["grad_p"], b["grad_p"])
    s = a["grad_k3_scale"].sum(axis=0)
    assert np.all(np.abs(a["grad_k3"].sum(axis=0) - b["grad_logk"]) <= 1e-15 * s + 1e-300)


def _swap_xy(a):
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


def test_transposition_symmetry(orc):
    """Swapping the roles of x and y (cell sizes, kx <-> ky, seal bits 0 <-> 1)
    transposes r; the Jacobian's -x/+x and -y/+y planes trade places."""
    geo, kx, ky, kz = _model(seed=4, shape=(5, 7, 3))
    p = orc.pressure(geo)
    g = geomodel.Grid(5, 7, 3, dx=10.0, dy=6.0, dz=geo.grid.dz, gk=geo.grid.gk)
    a = orc.evaluate_k3(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, want=("r", "J", "scale"))
    g2 = geomodel.Grid(g.ny, g.nx, g.nz, dx=g.dy, dy=g.dx, dz=g.dz, gk=g.gk)
    s = geo.seal
    s2 = (s & 4) | ((s & 1) << 1) | ((s & 2) >> 1)
    b = orc.evaluate_k3(g2, geo.fluid, _swap_xy(p), _swap_xy(ky), _swap_xy(kx), _swap_xy(kz),
                        seal=_swap_xy(s2), want=("r", "J"))
    tol = 4e-16 * _swap_xy(a["scale"][0])
    assert np.all(np.abs(b["r"] - _swap_xy(a["r"])) <= tol)
    for e2, e in ((0, 0), (1, 3), (2, 4), (3, 1), (4, 2), (5, 5), (6, 6)):
        assert np.allclose(b["J"][e2], _swap_xy(a["J"][e]), rtol=1e-15, atol=0), e


def test_conservation(orc):
    geo, kx, ky, kz = _model(seed=6, shape=(8, 7, 6))
    p = orc.pressure(geo)
    out = orc.evaluate_k3(geo.grid, geo.fluid, p, kx, ky, kz, seal=geo.seal,
                          want=("r", "scale"))
    assert abs(out["r"].sum()) <= 16 * out["r"].size * 1.2e-16 * out["scale"][0].sum()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_log_k_gradient_complex_step_per_axis(orc, axis):
    """d(w.r)/d ln k_a along a random direction of one axis at a time equals
    the complex-step derivative of w.r; the other planes do not enter."""
    geo, kx, ky, kz = _model(seed=7 + axis)
    p = orc.pressure(geo)
    rng = np.random.default_rng(30 + axis)
    w = rng.standard_normal(geo.grid.shape)
    dk = np.zeros((3,) + geo.grid.shape)
    dk[axis] = rng.standard_normal(geo.grid.shape)
    out = orc.evaluate_k3(geo.grid, geo.fluid, p, kx, ky, kz, seal=geo.seal, w=w,
                          want=("grad_k3", "grad_k3_scale"))
    want = float(np.sum(w * orc.evaluate_k3_cs(geo.grid, geo.fluid, p, kx, ky, kz,
                                               seal=geo.seal, dk=dk)))
    got = float(np.sum(out["grad_k3"] * dk))
    scale = float(np.sum(out["grad_k3_scale"] * np.abs(dk)))
    assert abs(got - want) <= 1e-13 * scale, (got, want, scale)


def test_jacobian_and_jvp_complex_step(orc):
    """J (seven planes) and J v of the full form (diagonal faces and
    accumulation term included) against the complex-step derivative in p."""
    geo, kx, ky, kz = _model(seed=11, shape=(7, 6, 5))
    g = geo.grid
    p = orc.pressure(geo)
    be = geomodel.be_fields(g, 12)
    acc = dict(phi=be["phi"], p_prev=p - be["dp_step"], dt=be["dt"], cr=be["cr"])
    diag = geomodel.diagonal_t(g, 13)
    v = be["v"]
    out = orc.evaluate_k3(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, diag=diag, accum=acc,
                          v=v, want=("J", "jv", "scale"))
    cs = orc.evaluate_k3_cs(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, diag=diag, accum=acc,
                            vp=v)
    bound = 1e-12 * (out["scale"][1] * np.abs(v) + np.abs(out["jv"])).max()
    assert np.abs(out["jv"] - cs).max() <= bound
    # the seven planes carry the cardinal part; without diagonal faces J v is
    # exactly J applied to v up to rounding
    out6 = orc.evaluate_k3(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, accum=acc, v=v,
                           want=("J", "jv", "scale"))
    cs6 = orc.evaluate_k3_cs(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, accum=acc, vp=v)
    assert np.abs(apply_J(out6["J"], v) - cs6).max() <= bound


def test_zero_diagonals_reduce_to_six_faces(orc):
    geo, kx, ky, kz = _model(seed=14, shape=(5, 6, 4))
    p = orc.pressure(geo)
    z = np.zeros(geo.grid.shape)
    a = orc.evaluate_k3(geo.grid, geo.fluid, p, kx, ky, kz, seal=geo.seal, diag=(z, z))["r"]
    b = orc.evaluate_k3(geo.grid, geo.fluid, p, kx, ky, kz, seal=geo.seal)["r"]
    assert np.array_equal(a, b)
