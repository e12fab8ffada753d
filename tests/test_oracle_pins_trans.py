"""Pins of the oracle's transmissibility-input form (face transmissibilities
given per cell, the face-centred data the paper stores, Sec. 5): two-cell
closed forms in 50-digit decimal arithmetic, the c_f = 0 graph Laplacian built
by SciPy from an explicit edge list with the given weights (six faces and the
two diagonal fields), and complex-step J v of the general residual (given T,
diagonal faces and accumulation term together)."""
from decimal import Decimal as D, getcontext

import numpy as np
import pytest
import scipy.sparse as sp

import geomodel
from helpers import apply_J

getcontext().prec = 50
FL = geomodel.Fluid()


def rho_dec(p):
    return D(FL.rho0) * (D(FL.cf) * (D(p) - D(FL.p0))).exp()


def test_two_cell_x_closed_form(orc):
    g = geomodel.Grid(2, 1, 1)
    p = np.array([1.0e7, 1.01e7]).reshape(1, 1, 2)
    tx = np.array([3.5e-13, 9.9]).reshape(1, 1, 2)  # the second entry has no +x face
    z = np.zeros((1, 1, 2))
    out = orc.evaluate_general(g, FL, p, trans=(tx, z, z), want=("r", "J"))
    # cell 1 has the higher pressure: it is upwind, F_01 < 0
    F = D(3.5e-13) * rho_dec(1.01e7) / D(FL.mu) * (D(1.0e7) - D(1.01e7))
    dF1 = D(3.5e-13) * (D(FL.cf) * rho_dec(1.01e7) / D(FL.mu) * (D(1.0e7) - D(1.01e7))
                        - rho_dec(1.01e7) / D(FL.mu))
    r = out["r"].ravel()
    assert abs(r[0] - float(F)) <= 2e-16 * abs(float(F)) and r[1] == -r[0]
    assert abs(out["J"][2].ravel()[0] - float(dF1)) <= 4e-16 * abs(float(dF1))


def test_two_cell_z_closed_form(orc):
    g = geomodel.Grid(1, 1, 2, gk=9.81)
    p = np.array([1.0e7, 1.0e7 + 5e4]).reshape(2, 1, 1)
    tz = np.array([7e-13, 0.0]).reshape(2, 1, 1)
    z = np.zeros((2, 1, 1))
    r = orc.evaluate_general(g, FL, p, trans=(z, z, tz))["r"].ravel()
    r0, r1 = rho_dec(1.0e7), rho_dec(1.0e7 + 5e4)
    dphi = (D(1.0e7) - D(1.0e7 + 5e4)) + (r0 + r1) / 2 * D(9.81) * D(2.0)
    lam = (r0 if dphi > 0 else r1) / D(FL.mu)
    F = D(7e-13) * lam * dphi
    assert abs(r[0] - float(F)) <= 4e-16 * abs(float(F)) and r[1] == -r[0]


@pytest.mark.parametrize("with_diag", [False, True])
def test_incompressible_graph_laplacian(orc, with_diag):
    nx, ny, nz = 6, 5, 4
    g = geomodel.Grid(nx, ny, nz, gk=0.0)
    fl = geomodel.Fluid(cf=0.0)
    rng = np.random.default_rng(17)
    tx, ty, tz, tne, tse = (rng.uniform(1e-13, 6e-13, g.shape) for _ in range(5))
    p = 1e7 + rng.uniform(-1e5, 1e5, g.shape)
    diag = (tne, tse) if with_diag else None
    r = orc.evaluate_general(g, fl, p, trans=(tx, ty, tz), diag=diag)["r"]
    idx = lambda i, j, k: i + nx * (j + ny * k)  # noqa: E731
    rows, cols, w = [], [], []

    def edge(a, b, t):
        rows.extend([a, b]); cols.extend([b, a]); w.extend([t, t])

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                a = idx(i, j, k)
                if i + 1 < nx:
                    edge(a, idx(i + 1, j, k), tx[k, j, i])
                if j + 1 < ny:
                    edge(a, idx(i, j + 1, k), ty[k, j, i])
                if k + 1 < nz:
                    edge(a, idx(i, j, k + 1), tz[k, j, i])
                if with_diag and i + 1 < nx and j + 1 < ny:
                    edge(a, idx(i + 1, j + 1, k), tne[k, j, i])
                if with_diag and i + 1 < nx and j >= 1:
                    edge(a, idx(i + 1, j - 1, k), tse[k, j, i])
    N = nx * ny * nz
    A = sp.csr_matrix((w, (rows, cols)), shape=(N, N))
    L = (fl.rho0 / fl.mu) * (sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A)
    want = L @ p.ravel()
    scale = (fl.rho0 / fl.mu) * (abs(A) @ np.abs(p.ravel() - p.mean()))
    assert np.all(np.abs(r.ravel() - want) <= 1e-9 * scale + 1e-12 * np.abs(want).max())


@pytest.mark.parametrize("shape", [(4, 3, 5), (7, 1, 3), (1, 6, 4), (5, 5, 2)])
def test_general_jvp_complex_step(orc, shape):
    g = geomodel.Grid(*shape)
    rng = np.random.default_rng(sum(shape))
    tx, ty, tz, tne, tse = (rng.uniform(0, 6e-13, g.shape) for _ in range(5))
    geo = geomodel.random_small(3, g.nx, g.ny, g.nz)
    p = orc.pressure(geo)
    acc = dict(phi=rng.uniform(0.1, 0.3, g.shape), p_prev=p - rng.uniform(-5e4, 5e4, g.shape),
               dt=3600.0, cr=5e-10)
    v = rng.standard_normal(g.shape)
    kw = dict(trans=(tx, ty, tz), diag=(tne, tse), accum=acc)
    out = orc.evaluate_general(g, geo.fluid, p, v=v, want=("J", "jv"), **kw)
    cs = orc.evaluate_general_cs(g, geo.fluid, p, v, **kw)
    # the diagonal faces are not in the 7-point J, so bound by |jv terms| via cs itself
    scale = apply_J(np.abs(out["J"]), np.abs(v)) + np.abs(cs)
    assert np.all(np.abs(out["jv"] - cs) <= 1e-13 * scale)


def test_general_matches_specialised_entries(orc):
    geo = geomodel.random_small(4, 9, 7, 5, seal_prob=0.05)
    p = orc.pressure(geo)
    a = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    b = orc.evaluate_general(geo.grid, geo.fluid, p, kx=geo.kx, ry=geo.ry, rz=geo.rz,
                             seal=geo.seal, want=("r", "J"))
    assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["J"], b["J"])


# ---------------------------------------------------------------------------
# Vector-Jacobian product of the transmissibility form: grad_p = J^T w and the
# gradient with respect to ln T of every face.
# ---------------------------------------------------------------------------

def test_vjp_trans_two_cell_closed_form(orc):
    g = geomodel.Grid(2, 1, 1)
    p = np.array([1.0e7, 1.01e7]).reshape(1, 1, 2)
    tx = np.array([3.5e-13, 0.0]).reshape(1, 1, 2)
    z = np.zeros((1, 1, 2))
    w = np.array([0.7, -1.3]).reshape(1, 1, 2)
    _, gt, _ = orc.vjp_general(g, FL, p, w, trans=(tx, z, z))
    F = D(3.5e-13) * rho_dec(1.01e7) / D(FL.mu) * (D(1.0e7) - D(1.01e7))
    want = (D(0.7) - D(-1.3)) * F
    assert abs(gt[0].ravel()[0] - float(want)) <= 4e-16 * abs(float(want))
    assert np.all(gt[0].ravel()[1:] == 0) and np.all(gt[1:] == 0)


@pytest.mark.parametrize("shape", [(4, 3, 5), (6, 1, 3), (1, 5, 4)])
def test_vjp_trans_dot_product_complex_step(orc, shape):
    g = geomodel.Grid(*shape)
    rng = np.random.default_rng(3 + sum(shape))
    tr = tuple(rng.uniform(0, 6e-13, g.shape) for _ in range(3))
    geo = geomodel.random_small(5, *shape)
    p = orc.pressure(geo)
    w = rng.standard_normal(g.shape)
    d = rng.standard_normal((3,) + g.shape)
    _, gt, gs = orc.vjp_general(g, geo.fluid, p, w, trans=tr)
    jd = orc.trans_cs(g, geo.fluid, p, tr, d)    # (dr / d ln T) d by complex step
    lhs, rhs = float(np.sum(gt * d)), float(np.sum(w * jd))
    assert abs(lhs - rhs) <= 1e-13 * float(np.sum(gs * np.abs(d)))


def test_vjp_trans_grad_p_is_sparse_JT_w(orc):
    g = geomodel.Grid(7, 5, 4)
    rng = np.random.default_rng(21)
    tr = tuple(rng.uniform(0, 6e-13, g.shape) for _ in range(3))
    geo = geomodel.random_small(6, 7, 5, 4)
    p = orc.pressure(geo)
    w = rng.standard_normal(g.shape)
    gp, _, _ = orc.vjp_general(g, geo.fluid, p, w, trans=tr)
    J = orc.evaluate_general(g, geo.fluid, p, trans=tr, want=("J",))["J"]
    from helpers import apply_JT, sparse_J
    ref = sparse_J(J).T @ w.ravel()
    scale = apply_JT(np.abs(J), np.abs(w)).ravel()
    assert np.all(np.abs(gp.ravel() - ref) <= 1e-14 * scale)
