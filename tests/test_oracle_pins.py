"""Pins of the FP64 oracle against what the mathematics fixes, independent of
the oracle's own code: closed forms evaluated in 50-digit decimal arithmetic,
the continuous hydrostatic column, SciPy's Kronecker-sum Laplacian for c_f = 0,
complex-step derivatives, a long-double evaluation, and invariants
(antisymmetry, conservation, equilibria, scaling, mirror symmetry).

Equations: paper Sec. 3, Eq. (3a)/(3b) flux and potential, Eq. (4) upwind,
Eq. (5) density; Algorithm 1 for the residual assembly.
"""
from decimal import Decimal as D, getcontext

import numpy as np
import pytest
import scipy.sparse as sp

import geomodel
from helpers import apply_J, apply_JT, shift, sparse_J

getcontext().prec = 50

FL = geomodel.Fluid()


def dexp(x):
    return D(x).exp()


def close(got, want, rel=4e-16, abs_=0.0):
    want = float(want)
    return abs(got - want) <= max(rel * abs(want), abs_)


def rho_dec(p):
    """Eq. (5) in decimal arithmetic."""
    return D(FL.rho0) * dexp(D(FL.cf) * (D(p) - D(FL.p0)))


# ---------------------------------------------------------------------------
# Two-cell closed forms
# ---------------------------------------------------------------------------

def test_x_pair_upwind_K(orc):
    """Equal permeabilities: the harmonic mean is k itself, a_x = dy dz / dx = 2 m,
    dPhi = +1e5 Pa > 0 so K is upwind and F = 2 k (rho_K / mu) 1e5."""
    g = geomodel.Grid(2, 1, 1)
    kx = np.full((1, 1, 2), 1e-13)
    p = np.array([FL.p0 + 1e5, FL.p0]).reshape(1, 1, 2)
    out = orc.evaluate(g, FL, kx, p)
    T = D(2) * D(1e-13)
    lamK = rho_dec(FL.p0 + 1e5) / D(FL.mu)
    F = T * lamK * D(100000)
    dK = T * lamK * (D(1) + D(FL.cf) * D(100000))
    dL = -T * lamK
    r, J = out["r"].ravel(), out["J"].reshape(7, 2)
    assert close(r[0], F) and close(r[1], -F)
    assert r[1] == -r[0]                       # antisymmetry, bitwise
    assert close(J[0, 0], dK) and close(J[2, 0], dL)     # diag, +x of K
    assert close(J[0, 1], -dL) and close(J[1, 1], -dK)   # diag, -x of L
    assert np.all(J[[1, 3, 4, 5, 6], 0] == 0) and np.all(J[[2, 3, 4, 5, 6], 1] == 0)
    # the printed magnitudes of this case (F ~ 2e-2 kg/s)
    assert close(r[0], D("0.020002000100003333"), rel=1e-15)


def test_x_pair_upwind_L_unequal_k(orc):
    """k = (1e-13, 4e-13): harmonic mean 1.6e-13; dPhi = -5e4 < 0 so L is
    upwind and only rho_L enters."""
    g = geomodel.Grid(2, 1, 1)
    kx = np.array([1e-13, 4e-13]).reshape(1, 1, 2)
    p = np.array([FL.p0 - 3e4, FL.p0 + 2e4]).reshape(1, 1, 2)
    out = orc.evaluate(g, FL, kx, p)
    T = D(2) * D(2) * D(1e-13) * D(4e-13) / (D(1e-13) + D(4e-13))
    lamL = rho_dec(FL.p0 + 2e4) / D(FL.mu)
    dphi = D(-50000)
    F = T * lamL * dphi
    dK = T * lamL
    dL = T * lamL * (D(FL.cf) * dphi - D(1))
    r, J = out["r"].ravel(), out["J"].reshape(7, 2)
    assert close(r[0], F, rel=1e-15) and r[1] == -r[0]
    assert close(J[0, 0], dK, rel=1e-15) and close(J[2, 0], dL, rel=1e-15)
    assert close(J[0, 1], -dL, rel=1e-15) and close(J[1, 1], -dK, rel=1e-15)


@pytest.mark.parametrize("gk", [9.81, -9.81])
def test_z_pair_gravity_drives_flow_down(orc, gk):
    """Equal pressures, one cell above the other: the heavier column pushes
    fluid down. With k pointing down (gk > 0) cell 0 is on top and F_01 > 0;
    with k pointing up (gk < 0) cell 1 is on top and F_01 < 0. Magnitude
    a_z k (rho0 / mu) rho0 |g| dz with a_z = dx dy / dz = 50 m."""
    g = geomodel.Grid(1, 1, 2, gk=gk)
    kx = np.full((2, 1, 1), 1e-13)
    p = np.full((2, 1, 1), FL.p0)
    out = orc.evaluate(g, FL, kx, p, rz=1.0)
    T = D(50) * D(1e-13)
    lam = D(FL.rho0) / D(FL.mu)
    F = T * lam * D(FL.rho0) * D(abs(gk)) * D(2)
    r = out["r"].ravel()
    assert close(abs(r[0]), F, rel=1e-15)
    assert (r[0] > 0) == (gk > 0)
    assert r[1] == -r[0]
    # derivatives: dPhi_01 = (p0 - p1) + rho_avg gk dz, drho/dp = cf rho
    J = out["J"].reshape(7, 2)
    c = D(FL.cf)
    G = D(gk) * D(2)
    dphi = D(FL.rho0) * G
    if gk > 0:   # upwind is cell 0
        dK = T * (c * lam * dphi + lam * (D(1) + D("0.5") * c * D(FL.rho0) * G))
        dL = T * lam * (D(-1) + D("0.5") * c * D(FL.rho0) * G)
    else:        # upwind is cell 1
        dK = T * lam * (D(1) + D("0.5") * c * D(FL.rho0) * G)
        dL = T * (c * lam * dphi + lam * (D(-1) + D("0.5") * c * D(FL.rho0) * G))
    assert close(J[0, 0], dK, rel=1e-15) and close(J[6, 0], dL, rel=1e-15)
    assert close(J[0, 1], -dL, rel=1e-15) and close(J[5, 1], -dK, rel=1e-15)


def test_sealed_face_carries_nothing(orc):
    g = geomodel.Grid(1, 2, 1)
    kx = np.full((1, 2, 1), 1e-13)
    p = np.array([FL.p0 + 1e5, FL.p0]).reshape(1, 2, 1)
    seal = np.array([2, 0], np.uint8).reshape(1, 2, 1)   # bit 1: +y face of cell 0
    out = orc.evaluate(g, FL, kx, p, seal=seal)
    assert np.all(out["r"] == 0) and np.all(out["J"] == 0)
    # a seal bit on a domain-boundary face has nothing to close
    seal2 = np.array([2, 7], np.uint8).reshape(1, 2, 1)
    out2 = orc.evaluate(g, FL, kx, p, seal=seal2)
    assert np.all(out2["r"] == 0)
    seal3 = np.array([5, 7], np.uint8).reshape(1, 2, 1)  # only x/z bits on cell 0
    out3 = orc.evaluate(g, FL, kx, p, seal=seal3)
    assert out3["r"].ravel()[0] > 0


def test_zero_permeability_face(orc):
    g = geomodel.Grid(2, 1, 1)
    kx = np.zeros((1, 1, 2))
    p = np.array([FL.p0 + 1e5, FL.p0]).reshape(1, 1, 2)
    out = orc.evaluate(g, FL, kx, p)
    assert np.all(out["r"] == 0) and np.all(out["J"] == 0)
    assert not np.any(np.isnan(out["J"]))


def test_tie_goes_to_lower_index(orc):
    """dPhi = 0 exactly: flux 0, and the derivative uses the lower cell's mobility
    from both sides of the face."""
    g = geomodel.Grid(2, 1, 1)
    kx = np.full((1, 1, 2), 1e-13)
    p = np.full((1, 1, 2), FL.p0 + 1e5)
    out = orc.evaluate(g, FL, kx, p)
    J = out["J"].reshape(7, 2)
    assert np.all(out["r"] == 0)
    # upwind = cell 0: dF/dp_0 = T lam_0, dF/dp_1 = -T lam_0 (lam_0 = lam_1 here)
    assert J[0, 0] == -J[2, 0] and J[0, 1] == -J[1, 1] and J[0, 0] == J[0, 1]


def test_forced_upwind(orc):
    g = geomodel.Grid(2, 1, 1)
    kx = np.full((1, 1, 2), 1e-13)
    p = np.array([FL.p0 + 1e5, FL.p0]).reshape(1, 1, 2)
    force = np.zeros((3, 1, 1, 2), np.int8)
    force[0, 0, 0, 0] = -1   # upper cell upwind although dPhi > 0
    out = orc.evaluate(g, FL, kx, p, force=force)
    lamL = rho_dec(FL.p0) / D(FL.mu)
    F = D(2e-13) * lamL * D(100000)
    assert close(out["r"].ravel()[0], F, rel=1e-15)


# ---------------------------------------------------------------------------
# Hydrostatic column
# ---------------------------------------------------------------------------

def test_hydrostatic_matches_continuous_column(orc):
    """dp/dzeta = rho(p) g integrates to p(zeta) = p0 - ln(1 - cf rho0 g zeta)/cf.
    The discrete profile (trapezoid rule in the face potential) differs by
    O(dz^2), far below 1e-2 Pa over 256 layers; a wrong density average or
    sign would be off by tens of Pa or more."""
    g = geomodel.Grid(1, 1, 256)
    pref = orc.hydrostatic(g, FL)
    c, rho0, gk = D(FL.cf), D(FL.rho0), D(g.gk)
    for k in (0, 1, 15, 100, 255):
        zeta = D(k) * D(g.dz)
        cont = D(FL.p0) - (D(1) - c * rho0 * gk * zeta).ln() / c
        assert abs(pref[k] - float(cont)) < 1e-2, k
    assert np.all(np.diff(pref) > 0)


def test_hydrostatic_first_layer_decimal(orc):
    """pref[1] solves x - p0 = (rho(p0) + rho(x))/2 g dz; Newton in 50 digits."""
    g = geomodel.Grid(1, 1, 2)
    pref = orc.hydrostatic(g, FL)
    G = D(g.gk) * D(g.dz)
    x = D(FL.p0) + D(FL.rho0) * G
    for _ in range(30):
        f = x - D(FL.p0) - (rho_dec(FL.p0) + rho_dec(x)) / 2 * G
        fp = D(1) - D(FL.cf) * rho_dec(x) / 2 * G
        x = x - f / fp
    assert close(pref[1], x, rel=2e-16)


def test_hydrostatic_equilibrium_gives_zero_flux(orc):
    """Discrete hydrostatic pressure with no noise: horizontal faces have equal
    pressures and vertical faces zero potential difference, so r vanishes to
    rounding relative to the face pressure jumps."""
    g = geomodel.Grid(5, 4, 40)
    pref = orc.hydrostatic(g, FL)
    p = np.broadcast_to(pref[:, None, None], g.shape).copy()
    kx = np.exp(np.random.default_rng(0).normal(np.log(1e-13), 1.0, g.shape))
    out = orc.evaluate(g, FL, kx, p, rz=0.1, want=("r", "J", "dphi"))
    r = out["r"]
    # magnitude of a single vertical face flux if the potential were off by dp
    Tz = 50 * 0.1 * kx.max() * 2
    lam = 1.1 * FL.rho0 / FL.mu
    jump = np.abs(np.diff(pref)).max()
    assert np.abs(r).max() <= 1e-12 * Tz * lam * jump
    assert np.nanmax(np.abs(out["dphi"][2])) <= 4 * np.spacing(pref.max())
    assert np.all(np.nan_to_num(out["dphi"][:2]) == 0.0)


def test_uniform_pressure_no_gravity_is_exact_zero(orc):
    g = geomodel.Grid(6, 5, 4, gk=0.0)
    geo = geomodel.random_small(3, 6, 5, 4, gk=0.0)
    p = np.full(g.shape, 1.23e7)
    out = orc.evaluate(g, FL, geo.kx, p, ry=0.7, rz=0.1, seal=geo.seal)
    assert np.all(out["r"] == 0.0)
    # J 1 = 0: each face contributes +T lam and -T lam to its row
    s = out["J"].sum(axis=0)
    assert np.abs(s).max() <= 1e-15 * np.abs(out["J"][0]).max()


# ---------------------------------------------------------------------------
# Textbook special case: cf = 0 makes r linear, r = L p + b, L the 7-point
# graph Laplacian (Kronecker sum of 1-D path Laplacians, Neumann ends).
# ---------------------------------------------------------------------------

def _path_diff(n):
    """(n-1) x n forward difference matrix."""
    if n == 1:
        return sp.csr_matrix((0, 1))
    return sp.diags([np.ones(n - 1), -np.ones(n - 1)], [0, 1], shape=(n - 1, n)).tocsr()


def test_incompressible_is_scaled_laplacian(orc):
    nx, ny, nz = 5, 4, 3
    g = geomodel.Grid(nx, ny, nz)
    fl = geomodel.Fluid(cf=0.0)
    k0, ry, rz = 2e-13, 0.5, 0.1
    kx = np.full(g.shape, k0)
    rng = np.random.default_rng(7)
    p = 1e7 + rng.uniform(-1e5, 1e5, g.shape)
    out = orc.evaluate(g, fl, kx, p, ry=ry, rz=rz)
    lam = fl.rho0 / fl.mu
    Dx, Dy, Dz = _path_diff(nx), _path_diff(ny), _path_diff(nz)
    Ix, Iy, Iz = (sp.identity(n) for n in (nx, ny, nz))
    # x fastest: index = i + nx (j + ny k) -> kron(z, kron(y, x))
    Lx = sp.kron(Iz, sp.kron(Iy, Dx.T @ Dx))
    Ly = sp.kron(Iz, sp.kron(Dy.T @ Dy, Ix))
    Lz = sp.kron(Dz.T @ Dz, sp.kron(Iy, Ix))
    ax, ay, az = g.dy * g.dz / g.dx, g.dx * g.dz / g.dy, g.dx * g.dy / g.dz
    L = lam * (ax * k0 * Lx + ay * ry * k0 * Ly + az * rz * k0 * Lz)
    # gravity: each vertical face adds +T lam rho0 g dz to its upper-index... lower cell
    Gz = sp.kron(Dz.T, sp.kron(Iy, Ix)) @ np.ones((nz - 1) * ny * nx)
    b = lam * az * rz * k0 * fl.rho0 * g.gk * g.dz * Gz
    Jsp = sparse_J(out["J"]).toarray()
    assert np.allclose(Jsp, L.toarray(), rtol=1e-14, atol=0)
    r_lin = L @ p.ravel() + b
    scale = np.abs(L).toarray() @ np.abs(p.ravel() - p.mean()) + np.abs(b) + 1.0
    assert np.all(np.abs(out["r"].ravel() - r_lin) <= 1e-12 * scale * 1e5)
    assert np.allclose(out["r"].ravel(), r_lin, rtol=1e-9, atol=1e-9 * np.abs(r_lin).max())


# ---------------------------------------------------------------------------
# Derivatives: complex step (Squire & Trapp) differentiates the branch taken,
# so it matches the analytic J to machine precision with no kink exclusion.
# ---------------------------------------------------------------------------

def _setup(seed, shape, gk=9.81, seal_prob=0.1):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed, nx, ny, nz, seal_prob=seal_prob, gk=gk, sigma=1.5)
    return geo


@pytest.mark.parametrize("seed,shape", [(1, (4, 3, 5)), (2, (1, 1, 7)), (3, (6, 1, 1)),
                                        (4, (3, 5, 2)), (5, (7, 6, 3))])
def test_jacobian_matches_complex_step(orc, seed, shape):
    geo = _setup(seed, shape)
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        v = rng.standard_normal(geo.grid.shape)
        re, jv = orc.evaluate_cs(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                                 seal=geo.seal, vp=v)
        Jv = apply_J(out["J"], v)
        scale = np.abs(out["J"]).sum(axis=0) * np.abs(v).max()
        assert np.all(np.abs(jv - Jv) <= 1e-14 * scale + 1e-300)
        assert np.array_equal(re, out["r"])
    # single columns
    N = geo.grid.ncell
    for c in rng.choice(N, size=min(N, 4), replace=False):
        e = np.zeros(N)
        e[c] = 1.0
        e = e.reshape(geo.grid.shape)
        _, col = orc.evaluate_cs(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                                 seal=geo.seal, vp=e)
        dense = sparse_J(out["J"]).toarray()[:, c]
        assert np.allclose(col.ravel(), dense, rtol=1e-13, atol=1e-13 * np.abs(dense).max())


def test_jacobian_matches_central_differences(orc):
    geo = _setup(11, (5, 4, 6))
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "J", "dphi"))
    h = 1.0
    rng = np.random.default_rng(12)
    v = rng.standard_normal(geo.grid.shape)
    rp = orc.evaluate(geo.grid, geo.fluid, geo.kx, p + h * v, ry=geo.ry, rz=geo.rz,
                      seal=geo.seal, want=("r",))["r"]
    rm = orc.evaluate(geo.grid, geo.fluid, geo.kx, p - h * v, ry=geo.ry, rz=geo.rz,
                      seal=geo.seal, want=("r",))["r"]
    fd = (rp - rm) / (2 * h)
    Jv = apply_J(out["J"], v)
    # no face is within 10 h of an upwind switch for this seed
    assert np.nanmin(np.abs(out["dphi"])) > 10 * h * 4
    assert np.allclose(fd, Jv, rtol=1e-7, atol=1e-7 * np.abs(Jv).max())


def test_long_double_bounds_rounding(orc):
    geo = _setup(21, (6, 5, 7))
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "J", "scale"))
    rl, Jl = orc.evaluate_ld(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                             seal=geo.seal)
    s = out["scale"]
    dr = np.abs(out["r"].astype(np.longdouble) - rl).astype(np.float64)
    assert np.all(dr <= 1e-15 * s[0])
    dd = np.abs(out["J"][0].astype(np.longdouble) - Jl[0]).astype(np.float64)
    assert np.all(dd <= 1e-15 * s[1])
    for n in range(1, 7):
        do = np.abs(out["J"][n].astype(np.longdouble) - Jl[n]).astype(np.float64)
        assert np.all(do <= 1e-15 * np.abs(out["J"][n]))  # ~8 roundings per entry


# ---------------------------------------------------------------------------
# Vector-Jacobian product
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,shape", [(31, (5, 4, 6)), (32, (1, 3, 9)), (33, (8, 2, 3))])
def test_vjp_pressure_is_transpose_product(orc, seed, shape):
    geo = _setup(seed, shape)
    p = orc.pressure(geo)
    w = np.random.default_rng(seed).standard_normal(geo.grid.shape)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       w=w, want=("r", "J", "grad_p", "grad_logk"))
    JT = sparse_J(out["J"]).T @ w.ravel()
    assert np.allclose(out["grad_p"].ravel(), JT, rtol=1e-12, atol=1e-14 * np.abs(JT).max())
    assert np.allclose(apply_JT(out["J"], w), out["grad_p"], rtol=1e-12,
                       atol=1e-14 * np.abs(JT).max())
    # dot-product test <w, J v> = <J^T w, v>
    v = np.random.default_rng(seed + 100).standard_normal(geo.grid.shape)
    lhs = np.dot(w.ravel(), apply_J(out["J"], v).ravel())
    rhs = np.dot(out["grad_p"].ravel(), v.ravel())
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(w).ravel() @ np.abs(apply_J(np.abs(out["J"]), np.abs(v))).ravel())


@pytest.mark.parametrize("seed,shape", [(41, (5, 4, 6)), (42, (3, 3, 3)), (43, (9, 1, 2))])
def test_vjp_logk_matches_complex_step(orc, seed, shape):
    geo = _setup(seed, shape)
    p = orc.pressure(geo)
    w = np.random.default_rng(seed).standard_normal(geo.grid.shape)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       w=w, want=("r", "grad_logk"))
    rng = np.random.default_rng(seed + 1)
    for _ in range(3):
        vm = rng.standard_normal(geo.grid.shape)
        _, dr = orc.evaluate_cs(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                                seal=geo.seal, vm=vm)
        lhs = np.dot(w.ravel(), dr.ravel())
        rhs = np.dot(out["grad_logk"].ravel(), vm.ravel())
        assert abs(lhs - rhs) <= 1e-12 * np.abs(w).ravel() @ np.abs(dr).ravel() + 1e-30
    # per-cell derivative for a few cells
    N = geo.grid.ncell
    for c in rng.choice(N, size=min(N, 5), replace=False):
        e = np.zeros(N)
        e[c] = 1.0
        _, dr = orc.evaluate_cs(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                                seal=geo.seal, vm=e.reshape(geo.grid.shape))
        want = np.dot(w.ravel(), dr.ravel())
        got = out["grad_logk"].ravel()[c]
        assert abs(got - want) <= 1e-12 * (np.abs(w).ravel() @ np.abs(dr).ravel()) + 1e-30


def test_vjp_constant_cotangent_vanishes(orc):
    """Sum_K r_K = 0 for every state, so w = 1 gives zero gradients."""
    geo = _setup(51, (6, 5, 4))
    p = orc.pressure(geo)
    w = np.ones(geo.grid.shape)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       w=w, want=("J", "grad_p", "grad_logk", "scale"))
    assert np.abs(out["grad_p"]).max() <= 1e-14 * np.abs(out["J"]).max() * 7
    assert np.abs(out["grad_logk"]).max() <= 1e-14 * out["scale"][0].max() * 7


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

def test_conservation_and_column_sums(orc):
    geo = geomodel.tiny16()
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "J", "scale"))
    N = geo.grid.ncell
    assert abs(out["r"].sum()) <= N * 1e-16 * out["scale"][0].sum()
    colsum = apply_JT(out["J"], np.ones(geo.grid.shape))
    assert np.all(np.abs(colsum) <= 1e-15 * 7 * np.abs(out["J"]).max(axis=0) * 4)


def test_scaling_is_bitwise(orc):
    geo = _setup(61, (5, 6, 4))
    p = orc.pressure(geo)
    a = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    b = orc.evaluate(geo.grid, geo.fluid, 2 * geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    fl2 = geomodel.Fluid(mu=geo.fluid.mu / 2)
    c = orc.evaluate(geo.grid, fl2, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert np.array_equal(b["r"], 2 * a["r"]) and np.array_equal(b["J"], 2 * a["J"])
    assert np.array_equal(c["r"], 2 * a["r"]) and np.array_equal(c["J"], 2 * a["J"])


def test_x_mirror(orc):
    geo = _setup(71, (7, 4, 5))
    p = orc.pressure(geo)
    a = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                     want=("r", "J", "scale"))
    # mirror in x: the +x face bit of cell i moves to cell nx-2-i
    seal = geo.seal[:, :, ::-1].copy()
    sx = (seal & 1)
    seal = (seal & 6) | np.concatenate([sx[:, :, 1:], np.zeros_like(sx[:, :, :1])], axis=2)
    b = orc.evaluate(geo.grid, geo.fluid, geo.kx[:, :, ::-1], p[:, :, ::-1], ry=geo.ry,
                     rz=geo.rz, seal=seal)
    rm = b["r"][:, :, ::-1]
    assert np.all(np.abs(rm - a["r"]) <= 1e-15 * a["scale"][0])
    Jm = b["J"][:, :, :, ::-1]
    Jm = Jm[[0, 2, 1, 3, 4, 5, 6]]
    assert np.all(np.abs(Jm[0] - a["J"][0]) <= 1e-15 * a["scale"][1])
    assert np.array_equal(Jm[1:], a["J"][1:])


def test_degenerate_grids(orc):
    g = geomodel.Grid(1, 1, 1)
    out = orc.evaluate(g, FL, np.full((1, 1, 1), 1e-13), np.full((1, 1, 1), 1e7))
    assert out["r"].ravel()[0] == 0 and np.all(out["J"] == 0)
    with pytest.raises(ValueError):
        orc.evaluate(geomodel.Grid(0, 1, 1), FL, np.zeros(0), np.zeros(0))


def test_rows_match_full_evaluation(orc):
    geo = _setup(81, (9, 7, 5))
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "J", "scale"))
    cells = np.array([0, 5, 62, 100, geo.grid.ncell - 1])
    r, J, s = orc.rows(geo.grid, geo.fluid, geo.kx, p, cells, ry=geo.ry, rz=geo.rz,
                       seal=geo.seal)
    assert np.array_equal(r, out["r"].ravel()[cells])
    assert np.array_equal(J, out["J"].reshape(7, -1)[:, cells])
    assert np.array_equal(s, out["scale"].reshape(2, -1)[:, cells])


def test_golden_regression(orc):
    """Fixture written by tests/golden/make_golden.py (oracle only)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "tiny16_oracle.json")
    doc = json.load(open(path))
    geo = geomodel.tiny16()
    p = orc.pressure(geo)
    r, J, s = orc.rows(geo.grid, geo.fluid, geo.kx, p, np.array(doc["cells"]), ry=geo.ry,
                       rz=geo.rz, seal=geo.seal)
    assert [float.hex(float(v)) for v in r] == doc["r"]
    assert [[float.hex(float(v)) for v in row] for row in J] == doc["J"]
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    assert [float.hex(float(v)) for v in pref] == doc["pref"]


def test_fd_gradients_32cube(orc):
    """Central differences of L = w . r on the 32^3 adjoint recipe: step 1e-4
    relative in ln k (smooth), 10 Pa in p (cells next to a face within 40 Pa
    of an upwind switch are skipped)."""
    geo = geomodel.fd32()
    p = orc.pressure(geo)
    w = geo.extra["w"][0]
    kw = dict(ry=geo.ry, rz=geo.rz, seal=geo.seal)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, w=w, want=("r", "grad_p", "grad_logk",
                                                                  "dphi"), **kw)
    from helpers import cells_touching, tie_faces
    kink = cells_touching(tie_faces(out["dphi"], 40.0)).ravel()
    rng = np.random.default_rng(3)
    N = geo.grid.ncell
    m = geo.logk.ravel()

    def L_of(kx=None, pp=None):
        r = orc.evaluate(geo.grid, geo.fluid, geo.kx if kx is None else kx,
                         p if pp is None else pp, want=("r",), **kw)["r"]
        return float(np.dot(w.ravel(), r.ravel()))

    for c in rng.choice(N, 48, replace=False):
        h = 1e-4 * abs(m[c])
        kp, km = geo.kx.copy().ravel(), geo.kx.copy().ravel()
        kp[c] = np.exp(m[c] + h)
        km[c] = np.exp(m[c] - h)
        fd = (L_of(kx=kp.reshape(geo.grid.shape)) - L_of(kx=km.reshape(geo.grid.shape))) / (2 * h)
        g = out["grad_logk"].ravel()[c]
        assert abs(fd - g) <= 1e-5 * max(abs(g), 1e-3 * np.abs(out["grad_logk"]).max()), (c, fd, g)
    checked = 0
    for c in rng.choice(N, 96, replace=False):
        if kink[c]:
            continue
        h = 10.0
        pp, pm = p.copy().ravel(), p.copy().ravel()
        pp[c] += h
        pm[c] -= h
        fd = (L_of(pp=pp.reshape(geo.grid.shape)) - L_of(pp=pm.reshape(geo.grid.shape))) / (2 * h)
        g = out["grad_p"].ravel()[c]
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 * np.abs(out["grad_p"]).max()), (c, fd, g)
        checked += 1
    assert checked >= 48
