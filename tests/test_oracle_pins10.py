"""Pins of the oracle's 10-flux stencil (the six TPFA faces plus the four
in-plane diagonal faces the paper also computes, Sec. 3, with caller-supplied
diagonal transmissibilities): closed forms, reduction to the 6-face residual,
the c_f = 0 graph Laplacian built by SciPy from an explicit edge list, and
conservation."""
from decimal import Decimal as D, getcontext

import numpy as np
import scipy.sparse as sp

import geomodel

getcontext().prec = 50
FL = geomodel.Fluid()


def rho_dec(p):
    return D(FL.rho0) * (D(FL.cf) * (D(p) - D(FL.p0))).exp()


def test_diagonal_pair_closed_form(orc):
    """2 x 2 x 1 grid, cardinal faces closed (k = 0): only the two diagonals
    carry flux. Cells: 0 = (0,0), 1 = (1,0), 2 = (0,1), 3 = (1,1)."""
    g = geomodel.Grid(2, 2, 1)
    kx = np.zeros((1, 2, 2))
    p = np.array([1.01e7, 1.02e7, 0.99e7, 1.0e7]).reshape(1, 2, 2)
    tne = np.zeros((1, 2, 2))
    tse = np.zeros((1, 2, 2))
    tne[0, 0, 0] = 3e-13   # face (0,0)-(1,1)
    tse[0, 1, 0] = 5e-13   # face (0,1)-(1,0)
    r, _ = orc.residual10(g, FL, kx, p, tne, tse)
    r = r.ravel()
    # face A: cells 0 (lower index) and 3; p0 > p3 so cell 0 is upwind
    Fa = D(3e-13) * rho_dec(1.01e7) / D(FL.mu) * (D(1.01e7) - D(1.0e7))
    # face B: cells 1 (lower index) and 2; p1 > p2 so cell 1 is upwind
    Fb = D(5e-13) * rho_dec(1.02e7) / D(FL.mu) * (D(1.02e7) - D(0.99e7))
    for got, want in ((r[0], Fa), (r[3], -Fa), (r[1], Fb), (r[2], -Fb)):
        assert abs(got - float(want)) <= 2e-16 * abs(float(want))
    assert r[0] == -r[3] and r[1] == -r[2]


def test_zero_diagonals_reduce_to_six_faces(orc):
    geo = geomodel.random_small(5, 7, 6, 5, seal_prob=0.1, sigma=1.5)
    p = orc.pressure(geo)
    z = np.zeros(geo.grid.shape)
    r10, _ = orc.residual10(geo.grid, geo.fluid, geo.kx, p, z, z, ry=geo.ry, rz=geo.rz,
                            seal=geo.seal)
    r6 = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                      want=("r",))["r"]
    assert np.array_equal(r10, r6)


def test_incompressible_is_graph_laplacian(orc):
    """c_f = 0 and no gravity: r = L p with L the weighted graph Laplacian of
    the cardinal edges (uniform k) and the diagonal edges (given T)."""
    nx, ny, nz = 5, 4, 3
    g = geomodel.Grid(nx, ny, nz, gk=0.0)
    fl = geomodel.Fluid(cf=0.0)
    k0 = 1e-13
    rng = np.random.default_rng(4)
    kx = np.full(g.shape, k0)
    tne = rng.uniform(1e-13, 5e-13, g.shape)
    tse = rng.uniform(1e-13, 5e-13, g.shape)
    p = 1e7 + rng.uniform(-1e5, 1e5, g.shape)
    r, _ = orc.residual10(g, fl, kx, p, tne, tse, ry=1.0, rz=1.0)
    lam = fl.rho0 / fl.mu
    idx = lambda i, j, k: i + nx * (j + ny * k)  # noqa: E731
    rows, cols, w = [], [], []

    def edge(a, b, t):
        rows.extend([a, b]); cols.extend([b, a]); w.extend([t, t])

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                a = idx(i, j, k)
                if i + 1 < nx:
                    edge(a, idx(i + 1, j, k), g.dy * g.dz / g.dx * k0)
                if j + 1 < ny:
                    edge(a, idx(i, j + 1, k), g.dx * g.dz / g.dy * k0)
                if k + 1 < nz:
                    edge(a, idx(i, j, k + 1), g.dx * g.dy / g.dz * k0)
                if i + 1 < nx and j + 1 < ny:
                    edge(a, idx(i + 1, j + 1, k), tne[k, j, i])
                if i + 1 < nx and j >= 1:
                    edge(a, idx(i + 1, j - 1, k), tse[k, j, i])
    N = nx * ny * nz
    A = sp.csr_matrix((w, (rows, cols)), shape=(N, N))
    L = lam * (sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A)
    want = L @ p.ravel()
    scale = lam * (abs(A) @ np.abs(p.ravel() - p.mean())) + 1e-30
    assert np.all(np.abs(r.ravel() - want) <= 1e-9 * scale + 1e-12 * np.abs(want).max())


def test_conservation_10(orc):
    geo = geomodel.random_small(9, 9, 8, 6, seal_prob=0.05, sigma=1.0)
    p = orc.pressure(geo)
    rng = np.random.default_rng(9)
    tne = rng.uniform(0, 4e-13, geo.grid.shape)
    tse = rng.uniform(0, 4e-13, geo.grid.shape)
    r, s = orc.residual10(geo.grid, geo.fluid, geo.kx, p, tne, tse, ry=geo.ry, rz=geo.rz,
                          seal=geo.seal)
    assert abs(r.sum()) <= 16 * r.size * 1.2e-16 * s.sum()
