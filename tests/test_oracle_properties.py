"""Property tests of the oracle on tiny random grids (hypothesis): complex-step
derivative agreement, conservation, antisymmetry of two-cell fluxes."""
import numpy as np
from hypothesis import given, settings, strategies as st

import geomodel
from helpers import apply_J, apply_JT


@settings(max_examples=40, deadline=None)
@given(nx=st.integers(1, 5), ny=st.integers(1, 5), nz=st.integers(1, 5),
       seed=st.integers(0, 10_000), sigma=st.floats(0.0, 4.0),
       seal_prob=st.floats(0.0, 0.5), gk=st.sampled_from([9.81, 0.0, -9.81]))
def test_random_tiny_grids(orc, nx, ny, nz, seed, sigma, seal_prob, gk):
    geo = geomodel.random_small(seed, nx, ny, nz, sigma=sigma, seal_prob=seal_prob, gk=gk)
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "J", "scale"))
    N = geo.grid.ncell
    # conservation: the fluxes of every face cancel in the sum
    assert abs(out["r"].sum()) <= 4 * N * 1.2e-16 * out["scale"][0].sum() + 1e-300
    # column sums of J vanish
    cs = apply_JT(out["J"], np.ones(geo.grid.shape))
    assert np.all(np.abs(cs) <= 8 * 1.2e-16 * np.abs(out["J"]).sum(axis=0).max() * 7 + 1e-300)
    # complex step
    v = np.random.default_rng(seed).standard_normal(geo.grid.shape)
    _, jv = orc.evaluate_cs(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                            seal=geo.seal, vp=v)
    Jv = apply_J(out["J"], v)
    bound = 1e-14 * (np.abs(out["J"]).sum(axis=0) * np.abs(v).max()) + 1e-300
    assert np.all(np.abs(jv - Jv) <= bound)


@settings(max_examples=60, deadline=None)
@given(axis=st.integers(0, 2), pK=st.floats(5e6, 2e7), pL=st.floats(5e6, 2e7),
       kK=st.floats(1e-18, 1e-10), kL=st.floats(1e-18, 1e-10), gk=st.floats(-20, 20))
def test_two_cell_antisymmetry_bitwise(orc, axis, pK, pL, kK, kL, gk):
    shape = [1, 1, 1]
    shape[2 - axis] = 2
    g = geomodel.Grid(*(shape[::-1]), gk=gk)
    kx = np.array([kK, kL]).reshape(shape)
    p = np.array([pK, pL]).reshape(shape)
    out = orc.evaluate(g, geomodel.Fluid(), kx, p, ry=0.5, rz=0.1)
    r = out["r"].ravel()
    assert r[1] == -r[0]
    # the face derivatives seen from the two sides agree
    J = out["J"].reshape(7, 2)
    plus, minus = 2 + 2 * axis, 1 + 2 * axis
    assert J[minus, 1] == -J[0, 0] and J[0, 1] == -J[plus, 0]
