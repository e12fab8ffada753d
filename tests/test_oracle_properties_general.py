"""Property tests (hypothesis) of the oracle's general evaluation on tiny
random grids: the transmissibility form with diagonal faces and the
accumulation term.

* conservation: without accumulation the residuals sum to zero; with it,
  to the total accumulation (V/dt sum (phi rho - phi_n rho_n));
* T -> 2T doubles every flux residual bit for bit (power-of-two scaling);
* complex-step J v of the whole residual equals the oracle's jv;
* the permeability form equals the transmissibility form fed the same
  harmonic transmissibilities (to rounding);
* J v is linear in v.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import geomodel
from helpers import apply_J

shapes = dict(nx=st.integers(1, 5), ny=st.integers(1, 5), nz=st.integers(1, 4))


def draw_case(seed, nx, ny, nz, closed):
    g = geomodel.Grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    geo = geomodel.random_small(seed, nx, ny, nz, sigma=1.0)
    trans = []
    for a in (2.0, 2.0, 5.0):
        t = a * 1e-13 * np.exp(rng.standard_normal(g.shape))
        t[rng.random(g.shape) < closed] = 0.0
        trans.append(t)
    diag = tuple(1e-13 * np.exp(rng.standard_normal(g.shape)) for _ in range(2))
    return g, geo, tuple(trans), diag, rng


@settings(max_examples=30, deadline=None)
@given(seed=st.integers(0, 10_000), closed=st.floats(0.0, 0.6), use_diag=st.booleans(),
       **shapes)
def test_general_conservation_and_scaling(orc, seed, closed, use_diag, nx, ny, nz):
    g, geo, tr, diag, rng = draw_case(seed, nx, ny, nz, closed)
    p = orc.pressure(geo)
    kw = dict(trans=tr, diag=diag if use_diag else None)
    out = orc.evaluate_general(g, geo.fluid, p, want=("r", "scale"), **kw)
    N = g.ncell
    assert abs(out["r"].sum()) <= 8 * N * 1.2e-16 * out["scale"][0].sum() + 1e-300
    tr2 = tuple(2.0 * t for t in tr)
    d2 = tuple(2.0 * t for t in diag) if use_diag else None
    r2 = orc.evaluate_general(g, geo.fluid, p, trans=tr2, diag=d2)["r"]
    assert np.array_equal(r2, 2.0 * out["r"])


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10_000), cr=st.floats(0.0, 1e-8), dt=st.floats(1.0, 1e6), **shapes)
def test_general_with_accumulation(orc, seed, cr, dt, nx, ny, nz):
    g, geo, tr, diag, rng = draw_case(seed, nx, ny, nz, 0.1)
    p = orc.pressure(geo)
    acc = dict(phi=rng.uniform(0.05, 0.35, g.shape), p_prev=p - rng.uniform(-1e5, 1e5, g.shape),
               dt=dt, cr=cr)
    v = rng.standard_normal(g.shape)
    kw = dict(trans=tr, diag=diag, accum=acc)
    out = orc.evaluate_general(g, geo.fluid, p, v=v, want=("r", "J", "jv", "scale"), **kw)
    # total: the fluxes cancel, the accumulation remains
    rho = lambda q: geo.fluid.rho0 * np.exp(geo.fluid.cf * (q - geo.fluid.p0))  # noqa: E731
    phi = lambda q: acc["phi"] * (1 + cr * (q - geo.fluid.p0))  # noqa: E731
    total = g.dx * g.dy * g.dz / dt * np.sum(phi(p) * rho(p) - phi(acc["p_prev"]) *
                                             rho(acc["p_prev"]))
    assert abs(out["r"].sum() - total) <= 64 * g.ncell * 1.2e-16 * out["scale"][0].sum()
    # complex step of the whole residual
    cs = orc.evaluate_general_cs(g, geo.fluid, p, v, **kw)
    bound = 1e-13 * (apply_J(np.abs(out["J"]), np.abs(v)) + np.abs(cs)) + 1e-300
    assert np.all(np.abs(out["jv"] - cs) <= bound)
    # linear in v
    jv2 = orc.evaluate_general(g, geo.fluid, p, v=2.0 * v, want=("jv",), **kw)["jv"]
    assert np.array_equal(jv2, 2.0 * out["jv"])


@settings(max_examples=30, deadline=None)
@given(seed=st.integers(0, 10_000), seal_prob=st.floats(0.0, 0.5), **shapes)
def test_permeability_form_equals_given_harmonic_t(orc, seed, seal_prob, nx, ny, nz):
    geo = geomodel.random_small(seed, nx, ny, nz, sigma=2.0, seal_prob=seal_prob)
    g = geo.grid
    p = orc.pressure(geo)
    k = geo.kx
    tr = []
    for axis, (a, r) in enumerate(((g.dy * g.dz / g.dx, 1.0), (g.dx * g.dz / g.dy, geo.ry),
                                   (g.dx * g.dy / g.dz, geo.rz))):
        kk = r * k
        nb = np.roll(kk, -1, axis=2 - axis)   # the +axis neighbour (wraps on the last layer)
        t = a * (2 * kk * nb) / (kk + nb)
        t[((geo.seal >> axis) & 1).astype(bool)] = 0.0
        tr.append(t)
    a = orc.evaluate(g, geo.fluid, k, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                     want=("r", "scale"))
    b = orc.evaluate_general(g, geo.fluid, p, trans=tuple(tr))["r"]
    assert np.all(np.abs(a["r"] - b) <= 1e-14 * a["scale"][0] + 1e-300)
