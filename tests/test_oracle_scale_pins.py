"""Pins of the denominators of the per-cell relative error (R16 metric) that
every parity test divides by, independent of the oracle's code: closed forms in
50-digit decimal arithmetic for

* the flux scale s_K = sum_L |F_KL| and the diagonal scale sum_L |dF_KL/dp_K|
  of the 6-face residual (Sec. 3, Eqs. 3a-5; Algorithm 1's neighbour sum), on
  a three-cell line whose middle cell has an inflow and an outflow face (so
  r_K cancels and s_K does not), and with one face sealed;
* the same scales from the sampled-row evaluator;
* the 10-flux residual's scale with diagonal faces;
* the backward-Euler diagonal scale (accumulation derivative plus faces);
* the test-side scales of the vector-Jacobian product (helpers.vjp_scales);

plus the oracle's upwind override of the in-plane diagonal faces and the
10-flux checker's re-evaluation of flipped ties. A doubled, dropped or
wrong-signed term in any scale fails one of these.
"""
from decimal import Decimal as D, getcontext

import numpy as np
import pytest

import geomodel
from helpers import compare_res10, vjp_scales

getcontext().prec = 50
FL = geomodel.Fluid()


def rho_dec(p):
    return D(FL.rho0) * (D(FL.cf) * (D(p) - D(FL.p0))).exp()


def lam_dec(p):
    return rho_dec(p) / D(FL.mu)


def close(got, want, rel=4e-16):
    want = float(want)
    return abs(got - want) <= rel * abs(want)


def harm(a, k1, k2):
    """a 2 k1 k2 / (k1 + k2) in decimal."""
    return D(a) * D(2) * D(k1) * D(k2) / (D(k1) + D(k2))


# three cells along x: 0 -- 1 -- 2; p falls from 0 to 2 through cell 1, so the
# middle cell receives from cell 0 and sends to cell 2
P3 = [1.0e7 + 1e5, 1.0e7, 1.0e7 - 4e4]
K3 = [1e-13, 2e-13, 4e-13]


def line_faces():
    """Decimal F and derivatives of the faces (0,1) and (1,2), each seen from its
    lower cell: F, dF/dp_lower, dF/dp_upper."""
    out = []
    for lo, up in ((0, 1), (1, 2)):
        T = harm(2, K3[lo], K3[up])        # a_x = dy dz / dx = 2 m
        dphi = D(P3[lo]) - D(P3[up])
        assert dphi > 0                       # the lower cell is upwind on both faces
        lam, dlam = lam_dec(P3[lo]), D(FL.cf) * lam_dec(P3[lo])
        F = T * lam * dphi
        out.append((F, T * (dlam * dphi + lam), -T * lam))
    return out


def test_flux_and_diagonal_scales_three_cell_line(orc):
    g = geomodel.Grid(3, 1, 1)
    kx = np.array(K3).reshape(1, 1, 3)
    p = np.array(P3).reshape(1, 1, 3)
    out = orc.evaluate(g, FL, kx, p, want=("r", "J", "scale"))
    (Fa, dLa, dUa), (Fb, dLb, dUb) = line_faces()
    s0 = out["scale"][0].ravel()
    s1 = out["scale"][1].ravel()
    r = out["r"].ravel()
    # cell 0: face a as its lower cell; cell 1: upper cell of a, lower of b; cell 2: upper of b
    assert close(s0[0], abs(Fa)) and close(s0[1], abs(Fa) + abs(Fb)) and close(s0[2], abs(Fb))
    assert close(s1[0], abs(dLa))
    assert close(s1[1], abs(dUa) + abs(dLb))     # dF_10/dp_1 = -dF_01/dp_1 = -dUa
    assert close(s1[2], abs(dUb))
    # the middle residual cancels, its scale does not
    assert close(r[1], Fb - Fa, rel=1e-14) and abs(r[1]) < 0.5 * s0[1]
    # the sampled-row evaluator gives the same scales
    _, _, s = orc.rows(g, FL, kx, p, np.arange(3))
    assert np.array_equal(s[0], s0) and np.array_equal(s[1], s1)


def test_sealed_face_adds_nothing_to_the_scales(orc):
    g = geomodel.Grid(3, 1, 1)
    kx = np.array(K3).reshape(1, 1, 3)
    p = np.array(P3).reshape(1, 1, 3)
    seal = np.array([0, 1, 0], np.uint8).reshape(1, 1, 3)   # +x face of cell 1 closed
    out = orc.evaluate(g, FL, kx, p, seal=seal, want=("scale",))
    (Fa, dLa, dUa), _ = line_faces()
    s0, s1 = out["scale"][0].ravel(), out["scale"][1].ravel()
    assert close(s0[0], abs(Fa)) and close(s0[1], abs(Fa)) and s0[2] == 0.0
    assert close(s1[1], abs(dUa)) and s1[2] == 0.0


def test_ten_flux_scale_counts_the_diagonal_faces(orc):
    """2 x 2 x 1 grid with one open x face (row j = 0) and one diagonal face
    (0,0)-(1,1): the scale of each cell is the sum of |F| of its open faces."""
    g = geomodel.Grid(2, 2, 1)
    kx = np.array([2e-13, 3e-13, 0.0, 0.0]).reshape(1, 2, 2)  # cells (0,1), (1,1) impermeable
    p = np.array([1.01e7, 1.0e7, 0.98e7, 0.995e7]).reshape(1, 2, 2)
    tne = np.zeros((1, 2, 2))
    tse = np.zeros((1, 2, 2))
    tne[0, 0, 0] = 7e-13
    _, scale = orc.residual10(g, FL, kx, p, tne, tse)
    s = scale.ravel()
    Fx = harm(2, 2e-13, 3e-13) * lam_dec(1.01e7) * (D(1.01e7) - D(1.0e7))
    Fd = D(7e-13) * lam_dec(1.01e7) * (D(1.01e7) - D(0.995e7))
    assert close(s[0], abs(Fx) + abs(Fd)) and close(s[1], abs(Fx))
    assert s[2] == 0.0 and close(s[3], abs(Fd))


def test_backward_euler_diagonal_scale(orc):
    """Two cells along x with the accumulation term: the diagonal scale of each
    cell is V/dt |d(phi rho)/dp| plus |dF/dp_K| of its face."""
    dt, cr = 3600.0, 5e-10
    g = geomodel.Grid(2, 1, 1)
    kx = np.full((1, 1, 2), 1e-13)
    p = np.array([1.0e7 + 1e5, 1.0e7]).reshape(1, 1, 2)
    pn = np.array([1.0e7, 1.0e7 + 2e4]).reshape(1, 1, 2)
    phi = np.array([0.2, 0.25]).reshape(1, 1, 2)
    out = orc.evaluate_be(g, FL, kx, p, phi, pn, dt, cr, want=("scale",))
    vdt = D(g.dx) * D(g.dy) * D(g.dz) / D(dt)

    def dm(c):
        pc = D(p.ravel()[c])
        ph = D(phi.ravel()[c]) * (1 + D(cr) * (pc - D(FL.p0)))
        return D(phi.ravel()[c]) * D(cr) * rho_dec(pc) + ph * D(FL.cf) * rho_dec(pc)

    T = harm(2, 1e-13, 1e-13)
    lam = lam_dec(p.ravel()[0])
    dphi = D(p.ravel()[0]) - D(p.ravel()[1])
    dFK = T * (D(FL.cf) * lam * dphi + lam)   # face seen from cell 0 (upwind)
    dFL = T * lam                            # dF_10/dp_1 = -dF_01/dp_1 = T lam
    s1 = out["scale"][1].ravel()
    assert close(s1[0], vdt * abs(dm(0)) + abs(dFK), rel=1e-15)
    assert close(s1[1], vdt * abs(dm(1)) + abs(dFL), rel=1e-15)


def test_vjp_scales_three_cell_line(orc):
    """grad_p scale: sum_r |J_rc| |w_r| (the absolute terms of (J^T w)_c);
    ln k scale: twice the largest |w| of the cell and its neighbours times
    s_c, which bounds the sum of the absolute terms
    |(w_K - w_L) F k_L / (k_K + k_L)| over the cell's faces."""
    g = geomodel.Grid(3, 1, 1)
    kx = np.array(K3).reshape(1, 1, 3)
    p = np.array(P3).reshape(1, 1, 3)
    w = np.array([0.7, -1.3, 0.4]).reshape(1, 1, 3)
    out = orc.evaluate(g, FL, kx, p, want=("J", "scale"))
    sp_, sm = vjp_scales(out["J"], out["scale"], w)
    (Fa, dLa, dUa), (Fb, dLb, dUb) = line_faces()
    # dense J in decimal: row K, column L = dr_K / dp_L
    Jd = [[dLa, dUa, D(0)], [-dLa, -dUa + dLb, dUb], [D(0), -dLb, -dUb]]
    wd = [D(x) for x in w.ravel()]
    for c in range(3):
        want = sum(abs(Jd[rr][c]) * abs(wd[rr]) for rr in range(3))
        assert close(sp_.ravel()[c], want, rel=1e-15)
    aw = [abs(x) for x in wd]
    s0 = [abs(Fa), abs(Fa) + abs(Fb), abs(Fb)]
    wmax = [max(aw[0], aw[1]), max(aw), max(aw[1], aw[2])]
    # exact sums of the absolute terms of the ln k gradient
    qa0, qa1 = D(K3[1]) / (D(K3[0]) + D(K3[1])), D(K3[0]) / (D(K3[0]) + D(K3[1]))
    qb1, qb2 = D(K3[2]) / (D(K3[1]) + D(K3[2])), D(K3[1]) / (D(K3[1]) + D(K3[2]))
    da, db = wd[0] - wd[1], wd[1] - wd[2]
    terms = [abs(da * Fa * qa0), abs(da * Fa * qa1) + abs(db * Fb * qb1), abs(db * Fb * qb2)]
    for c in range(3):
        assert close(sm.ravel()[c], 2 * wmax[c] * s0[c], rel=1e-15)
        assert terms[c] <= 2 * wmax[c] * s0[c]


def test_forced_diagonal_upwind(orc):
    """The override of an in-plane diagonal face picks the forced cell's mobility
    (indexed by the face's (i, j) end; +1 lower-index cell, -1 upper)."""
    g = geomodel.Grid(2, 2, 1)
    kx = np.zeros((1, 2, 2))
    p = np.array([1.01e7, 1.02e7, 0.99e7, 1.0e7]).reshape(1, 2, 2)
    tne = np.zeros((1, 2, 2))
    tse = np.zeros((1, 2, 2))
    tne[0, 0, 0] = 3e-13   # face (0,0)-(1,1): cells 0 (lower) and 3
    tse[0, 1, 0] = 5e-13   # face (0,1)-(1,0): cells 1 (lower) and 2, stored at (0,1)
    force = np.zeros((5, 1, 2, 2), np.int8)
    force[3, 0, 0, 0] = -1   # upper cell 3 upwind although p0 > p3
    force[4, 0, 1, 0] = -1   # upper cell 2 upwind although p1 > p2
    r, _ = orc.residual10(g, FL, kx, p, tne, tse, force=force)
    r = r.ravel()
    Fa = D(3e-13) * lam_dec(1.0e7) * (D(1.01e7) - D(1.0e7))
    Fb = D(5e-13) * lam_dec(0.99e7) * (D(1.02e7) - D(0.99e7))
    assert close(r[0], Fa) and close(r[1], Fb) and r[3] == -r[0] and r[2] == -r[1]
    # forcing the rule's own choice changes nothing
    force[3, 0, 0, 0] = 1
    force[4, 0, 1, 0] = 1
    r1, _ = orc.residual10(g, FL, kx, p, tne, tse, force=force)
    r0, _ = orc.residual10(g, FL, kx, p, tne, tse)
    assert np.array_equal(r1, r0)


def test_ten_flux_checker_reevaluates_flipped_ties(orc):
    """3 x 3 x 1 grid whose pressures differ by at least 9.5 kPa across every
    face except one diagonal face (500 Pa). With a tie band of 1 kPa, a
    residual with that face's other upwind choice passes the 10-flux checker
    through the re-evaluation (the flip changes it by far more than the
    tolerance), and the same residual with an error at a cell away from the
    tie fails it."""
    g = geomodel.Grid(3, 3, 1)
    kx = np.full(g.shape, 1e-13)
    p = 1e7 + 1e4 * np.random.default_rng(2).permutation(9).astype(np.float64).reshape(g.shape)
    p[0, 1, 1] = p[0, 0, 0] + 500.0        # face (0,0)-(1,1) within the tie band
    tne = np.full(g.shape, 2e-13)
    tse = np.full(g.shape, 2e-13)
    force = np.zeros((5,) + g.shape, np.int8)
    force[3, 0, 0, 0] = 1    # the rule takes the upper cell (dPhi_lo = -500 Pa); force the lower
    r_alt, _ = orc.residual10(g, FL, kx, p, tne, tse, force=force)
    r_ref, scale = orc.residual10(g, FL, kx, p, tne, tse)
    d = np.abs(r_alt - r_ref) / scale
    assert d[0, 0, 0] > 1e-10 and d[0, 1, 1] > 1e-10
    assert np.count_nonzero(d) == 2
    rep = compare_res10(orc, g, FL, kx, p, tne, tse, r_alt, tol=1e-12, tau=1e3, ry=1.0,
                        rz=1.0, seal=None)
    assert rep["n_tie_cells"] == 2 and rep["max_err"] <= 1e-12
    bad = r_alt.copy()
    bad[0, 2, 2] += 1e-9 * scale[0, 2, 2]
    with pytest.raises(AssertionError):
        compare_res10(orc, g, FL, kx, p, tne, tse, bad, tol=1e-12, tau=1e3, ry=1.0, rz=1.0,
                      seal=None)
