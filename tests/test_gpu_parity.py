"""GPU parity: the HIP path through the C ABI against the FP64 oracle,
element by element, on small and odd shapes that span several tiles and a
ragged tail, for every compiled tile shape; plus determinism and invariants.

Tolerances: FP64 path 1e-12 and FP32 precision form 1e-5, in the per-cell
relative metric of tests/helpers.py (residual against the cell's flux scale,
diagonal against the sum of its face derivatives, off-diagonals against
themselves, exact zero where the oracle's scale is zero). Faces whose
potential difference lies within tau of zero may take either upwind choice.
"""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_full, compare_vjp, shift

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
TAU32 = 1e-4  # Pa: upwind tie band of the FP32 form (its |dPhi| error is below 1e-6 Pa)


def tau64(p):
    return 1e-9 * float(np.abs(p).max())


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


SHAPES = [(1, 1, 7), (7, 1, 1), (1, 7, 1), (3, 5, 7), (65, 3, 2), (70, 9, 37), (17, 33, 5),
          (1, 1, 1), (2, 2, 2), (130, 6, 70), (64, 4, 32), (33, 17, 40), (129, 13, 3)]


def small(shape, seed=7, gk=9.81, seal_prob=0.05):
    nx, ny, nz = shape
    return geomodel.random_small(seed + nx * 7 + ny * 13 + nz, nx, ny, nz, sigma=1.5,
                                 seal_prob=seal_prob, gk=gk)


def fp64_run(gpu, geo, p, **kw):
    r, J = gpu.jacobian(geo.grid, geo.fluid, dev(geo.kx), dev(p), seal=dev(geo.seal),
                        ry=geo.ry, rz=geo.rz, **kw)
    return host(r), host(J)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_fp64_jacobian_all_tiles(gpu, orc, shape):
    geo = small(shape)
    p = orc.pressure(geo)
    print(f"fp64 jacobian {shape}", flush=True)
    ref_r = ref_J = None
    for tile in range(len(gpu.tile_shapes())):
        r, J = fp64_run(gpu, geo, p, tile=tile)
        if ref_r is None:
            rep = compare_full(orc, geo.grid, geo.fluid, geo.kx, p, r, J, tol=TOL64,
                               tau=tau64(p), ry=geo.ry, rz=geo.rz, seal=geo.seal)
            assert rep["max_err"] <= TOL64, rep
            ref_r, ref_J = r, J
        else:  # every tile computes each cell the same way: bitwise equal
            assert np.array_equal(r, ref_r) and np.array_equal(J, ref_J), tile
    # residual-only kernel equals the residual of the Jacobian kernel
    r2 = host(gpu.residual(geo.grid, geo.fluid, dev(geo.kx), dev(p), seal=dev(geo.seal),
                           ry=geo.ry, rz=geo.rz))
    assert np.array_equal(r2, ref_r)


@pytest.mark.parametrize("kz", [1, 2, 3, 5, 36, 37, 64])
def test_fp64_kz_chunks_bitwise(gpu, orc, kz):
    geo = small((70, 9, 37))
    p = orc.pressure(geo)
    r0, J0 = fp64_run(gpu, geo, p)
    r, J = fp64_run(gpu, geo, p, kz_chunk=kz, tile=1)
    assert np.array_equal(r, r0) and np.array_equal(J, J0)
    r, J = fp64_run(gpu, geo, p, kz_chunk=kz, xcd_remap=True)
    assert np.array_equal(r, r0) and np.array_equal(J, J0)
    r, J = fp64_run(gpu, geo, p, kz_chunk=kz, xcd_remap="yfast")
    assert np.array_equal(r, r0) and np.array_equal(J, J0)


def test_fp64_tiny16_workload(gpu, orc):
    geo = geomodel.tiny16()
    p = orc.pressure(geo)
    r, J = fp64_run(gpu, geo, p)
    rep = compare_full(orc, geo.grid, geo.fluid, geo.kx, p, r, J, tol=TOL64, tau=tau64(p),
                       ry=geo.ry, rz=geo.rz, seal=geo.seal)
    ref = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    same = float(np.mean(r == ref["r"]))
    print(f"tiny16 fp64: max rel err {rep['max_err']:.3e}, bitwise-equal residuals {same:.3f}")
    assert rep["max_err"] <= TOL64


def fp32_inputs(orc, geo):
    pref = orc.hydrostatic(geo.grid, geo.fluid, geo.p_top)
    dp = geo.dp32()
    k32 = geo.kx32()
    return pref, dp, k32, orc.widen_fp32(dp, pref), k32.astype(np.float64)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_fp32_precision_form(gpu, orc, shape):
    geo = small(shape)
    pref, dp, k32, p_w, k_w = fp32_inputs(orc, geo)
    print(f"fp32 jacobian {shape}", flush=True)
    ref = None
    for tile in (0, 1, 2, 3):
        r, J = gpu.jacobian(geo.grid, geo.fluid, dev(k32), dev(dp), seal=dev(geo.seal),
                            pref=dev(pref), ry=geo.ry, rz=geo.rz, tile=tile)
        r, J = host(r), host(J)
        assert r.dtype == np.float32 and J.dtype == np.float32
        if ref is None:
            rep = compare_full(orc, geo.grid, geo.fluid, k_w, p_w, r, J, tol=TOL32, tau=TAU32,
                               ry=geo.ry, rz=geo.rz, seal=geo.seal)
            assert rep["max_err"] <= TOL32, rep
            ref = (r, J)
        else:
            assert np.array_equal(r, ref[0]) and np.array_equal(J, ref[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_output_store_kinds_bitwise(gpu, orc, prec):
    """64-cell rows start on 128-byte lines: with 128-byte-aligned outputs the
    FP32 kernels store non-temporal, with outputs one element off a line they
    use ordinary stores (FP64 stores non-temporal in both). Either way the
    same values land in every cell, for the Jacobian and the VJP."""
    geo = small((64, 6, 9))
    shape = geo.grid.shape
    n = int(np.prod(shape))
    if prec == "fp64":
        p, kx, pref, dt = orc.pressure(geo), geo.kx, None, torch.float64
    else:
        pref, dp, kx, _, _ = fp32_inputs(orc, geo)
        p, dt, pref = dp, torch.float32, dev(pref)
    args = (geo.grid, geo.fluid, dev(kx), dev(p))
    kw = dict(seal=dev(geo.seal), pref=pref, ry=geo.ry, rz=geo.rz)
    print(f"store kinds {prec}", flush=True)

    def off(planes):  # a contiguous view one element past a fresh allocation
        return torch.empty(planes * n + 1, dtype=dt, device="cuda")[1:].view(
            ((planes,) if planes > 1 else ()) + shape)

    r0, J0 = gpu.jacobian(*args, **kw)
    r1, J1 = gpu.jacobian(*args, r_out=off(1), J_out=off(7), **kw)
    assert r1.data_ptr() % 128 != 0
    assert torch.equal(r0, r1) and torch.equal(J0, J1)
    w = dev(np.random.default_rng(3).standard_normal(shape).astype(
        np.float64 if prec == "fp64" else np.float32))
    g0 = gpu.residual_vjp(*args, w, **kw)
    g1 = gpu.residual_vjp(*args, w, gp_out=off(1), gm_out=off(1), **kw)
    assert torch.equal(g0[0], g1[0]) and torch.equal(g0[1], g1[1])


def test_hydrostatic_and_offsets(gpu, orc):
    for gk, top, nz in ((9.81, 1e7, 256), (-9.81, 2e7, 40), (0.0, 1e7, 5)):
        g = geomodel.Grid(3, 2, nz, gk=gk)
        want = orc.hydrostatic(g, geomodel.Fluid(), top)
        got = host(gpu.hydrostatic(g, geomodel.Fluid(), top))
        assert np.allclose(got, want, rtol=4e-16, atol=0), np.abs(got - want).max()
    geo = small((9, 4, 6))
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    p = orc.pressure(geo)
    dp = host(gpu.offset_pressure(geo.grid, dev(p), dev(pref)))
    assert np.array_equal(dp, (p - pref[:, None, None]).astype(np.float32))


def test_uniform_pressure_no_gravity_exact_zero(gpu):
    geo = small((37, 11, 9), gk=0.0)
    p = np.full(geo.grid.shape, 1.3e7)
    r, J = fp64_run(gpu, geo, p)
    assert np.all(r == 0.0)
    rowsum = J[0] + sum(J[1 + n] for n in range(6))
    assert np.abs(rowsum).max() <= 1e-15 * 7 * np.abs(J).max()


def test_hydrostatic_equilibrium_on_gpu(gpu, orc):
    geo = small((33, 9, 50), seal_prob=0.0)
    pref = host(gpu.hydrostatic(geo.grid, geo.fluid))
    p = np.broadcast_to(pref[:, None, None], geo.grid.shape).copy()
    r, _ = fp64_run(gpu, geo, p)
    Tz = 50 * geo.rz * geo.kx.max() * 2
    lam = 1.1 * geo.fluid.rho0 / geo.fluid.mu
    assert np.abs(r).max() <= 1e-12 * Tz * lam * np.abs(np.diff(pref)).max()


def test_determinism_and_column_sums(gpu, orc):
    geo = small((130, 6, 70))
    p = orc.pressure(geo)
    a = fp64_run(gpu, geo, p)
    b = fp64_run(gpu, geo, p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    J = a[1]
    col = J[0].copy()
    for n in range(6):
        col += shift(J[1 + n], n ^ 1)
    assert np.all(np.abs(col) <= 1e-14 * np.abs(J).sum(axis=0) + 1e-300)


def test_two_cell_antisymmetry(gpu):
    for axis in range(3):
        shape = [1, 1, 1]
        shape[axis] = 2
        g = geomodel.Grid(*shape)
        kx = np.array([1e-13, 3e-13]).reshape(g.shape)
        p = np.array([1.01e7, 1.0e7]).reshape(g.shape)
        for prec in ("fp64", "fp32"):
            if prec == "fp64":
                r, _ = gpu.jacobian(g, geomodel.Fluid(), dev(kx), dev(p), rz=0.1)
            else:
                pref = np.array([1.0e7, 1.0e7 + 19620.0])[: g.nz]
                dp = (p - pref[:, None, None]).astype(np.float32)
                r, _ = gpu.jacobian(g, geomodel.Fluid(), dev(kx.astype(np.float32)), dev(dp),
                                    pref=dev(pref), rz=0.1)
            r = host(r).ravel()
            assert r[0] == -r[1] and r[0] != 0


# ---------------------------------------------------------------------------
# Vector-Jacobian product and autograd
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(3, 5, 7), (70, 9, 37), (1, 1, 9), (33, 17, 12), (2, 2, 2)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vjp_matches_oracle(gpu, orc, shape, prec):
    geo = small(shape)
    w = np.random.default_rng(sum(shape)).standard_normal(geo.grid.shape)
    print(f"vjp {prec} {shape}", flush=True)
    if prec == "fp64":
        p = orc.pressure(geo)
        gp, gm = gpu.residual_vjp(geo.grid, geo.fluid, dev(geo.kx), dev(p), dev(w),
                                  seal=dev(geo.seal), ry=geo.ry, rz=geo.rz)
        kx, tol, tau, wv = geo.kx, TOL64, tau64(p), w
    else:
        pref, dp, k32, p, kx = fp32_inputs(orc, geo)
        w32 = w.astype(np.float32)
        gp, gm = gpu.residual_vjp(geo.grid, geo.fluid, dev(k32), dev(dp), dev(w32),
                                  seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz)
        tol, tau, wv = TOL32, TAU32, w32.astype(np.float64)
    rep = compare_vjp(orc, geo.grid, geo.fluid, kx, p, wv, host(gp), host(gm), tol=tol,
                      tau=tau, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert rep["max_err"] <= tol, rep
    # single outputs
    gp2, gm2 = gpu.residual_vjp(geo.grid, geo.fluid, dev(kx if prec == "fp64" else k32),
                                dev(p if prec == "fp64" else dp),
                                dev(w if prec == "fp64" else w32), seal=dev(geo.seal),
                                pref=None if prec == "fp64" else dev(pref), ry=geo.ry,
                                rz=geo.rz, want_p=False)
    assert gp2 is None and np.array_equal(host(gm2), host(gm))


def test_autograd_gradcheck_fp64(gpu, orc):
    geo = small((3, 3, 4))
    p = orc.pressure(geo)
    scale = 1e5  # pressure in units of 1e5 Pa so that one step size suits both inputs
    ps = torch.tensor(p / scale, dtype=torch.float64, device="cuda", requires_grad=True)
    m = torch.tensor(geo.logk, dtype=torch.float64, device="cuda", requires_grad=True)
    seal = dev(geo.seal)

    def f(ps_, m_):
        return gpu.TPFAResidual.apply(ps_ * scale, m_, geo.grid, geo.fluid, seal, None,
                                      geo.ry, geo.rz)

    assert torch.autograd.gradcheck(f, (ps, m), eps=1e-6, atol=1e-9, rtol=1e-6)


def test_autograd_fp32_matches_oracle_vjp(gpu, orc):
    geo = geomodel.fd32()
    pref, dp, k32, p_w, _ = fp32_inputs(orc, geo)
    logk32 = np.log(k32.astype(np.float64)).astype(np.float32)
    w = geo.extra["w"][0].astype(np.float32)
    dpt = dev(dp).requires_grad_(True)
    mt = dev(logk32).requires_grad_(True)
    r = gpu.TPFAResidual.apply(dpt, mt, geo.grid, geo.fluid, dev(geo.seal), dev(pref), geo.ry,
                               geo.rz)
    (r * dev(w)).sum().backward()
    kx_w = np.exp(logk32.astype(np.float64))
    k_used = host(torch.exp(dev(logk32))).astype(np.float64)
    rep = compare_vjp(orc, geo.grid, geo.fluid, k_used, p_w, w.astype(np.float64),
                      host(dpt.grad), host(mt.grad), tol=TOL32, tau=TAU32, ry=geo.ry, rz=geo.rz,
                      seal=geo.seal)
    assert rep["max_err"] <= TOL32, rep
    assert np.allclose(k_used, kx_w, rtol=1e-6)


# ---------------------------------------------------------------------------
# Batched ensemble
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shapes", [[(2, 2, 2)], [(3, 1, 2), (1, 1, 1), (5, 4, 3)],
                                    [(70, 9, 37)] * 9],
                         ids=["one-item", "three-items", "nine-models"])
def test_ensemble_few_items(gpu, orc, shapes):
    """Fewer work items than XCD bands (so bands without items, and fewer
    persistent workgroups than bands), one item per model, and a batch whose
    bands all hold several items: both schedules, repeated graph replays (the
    claim counters are reset by the last workgroup of each launch), bitwise
    equal to single launches."""
    members, singles = [], []
    for m, shape in enumerate(shapes):
        geo = small(shape, seed=40 + m)
        p = orc.pressure(geo)
        d = dict(grid=geo.grid, fluid=geo.fluid, kx=dev(geo.kx), p=dev(p), seal=dev(geo.seal),
                 ry=geo.ry, rz=geo.rz, tile=0, kz_chunk=64)
        members.append(d)
        singles.append(gpu.jacobian(d["grid"], d["fluid"], d["kx"], d["p"], seal=d["seal"],
                                    ry=d["ry"], rz=d["rz"], tile=0, kz_chunk=64))
    print(f"ensemble of {len(shapes)} models", flush=True)
    ens = gpu.Ensemble(members)
    n_items, n_wg = ens.info()
    assert 1 <= n_wg <= max(n_items, 1)
    for schedule in ("persistent", "grouped", "persistent"):
        ens.set_schedule(schedule)
        for replay in range(4):
            for q in range(len(members)):
                ens.r[q].fill_(float("nan"))
                ens.J[q].fill_(float("nan"))
            ens.run(graph=(replay != 2))
            torch.cuda.synchronize()
            for q, (r, J) in enumerate(singles):
                assert torch.equal(ens.r[q], r) and torch.equal(ens.J[q], J), (schedule, replay, q)
    ens.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ensemble_matches_single_launches_and_oracle(gpu, orc, prec):
    models = geomodel.ensemble(n_models=12, scale=0.2)
    members, inputs = [], []
    for m, geo in enumerate(models):
        tile = m % 3  # every 256-thread tile shape in one persistent launch
        if prec == "fp32":
            pref, dp, k32, p_w, k_w = fp32_inputs(orc, geo)
            d = dict(grid=geo.grid, fluid=geo.fluid, kx=dev(k32), p=dev(dp), seal=dev(geo.seal),
                     pref=dev(pref), ry=geo.ry, rz=geo.rz, tile=tile, kz_chunk=8 + 3 * m)
            inputs.append((k_w, p_w))
        else:
            p = orc.pressure(geo)
            d = dict(grid=geo.grid, fluid=geo.fluid, kx=dev(geo.kx), p=dev(p),
                     seal=dev(geo.seal), ry=geo.ry, rz=geo.rz, tile=tile, kz_chunk=8 + 3 * m)
            inputs.append((geo.kx, p))
        members.append(d)
    ens = gpu.Ensemble(members)
    n_items, n_wg = ens.info()
    assert n_items > 0 and n_wg > 0
    singles = []
    for d in members:
        r, J = gpu.jacobian(d["grid"], d["fluid"], d["kx"], d["p"], seal=d["seal"],
                            pref=d.get("pref"), ry=d["ry"], rz=d["rz"], tile=d["tile"],
                            kz_chunk=d["kz_chunk"])
        singles.append((r, J))
    for replay in range(5):
        for q in range(len(members)):
            ens.r[q].fill_(float("nan"))
            ens.J[q].fill_(float("nan"))
        if replay == 3:
            ens.set_schedule("grouped")
        ens.run(graph=(replay != 1))
        torch.cuda.synchronize()
        for q, (r, J) in enumerate(singles):
            assert torch.equal(ens.r[q], r) and torch.equal(ens.J[q], J), (replay, q)
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
    tol = TOL32 if prec == "fp32" else TOL64
    for q, geo in enumerate(models):
        k_w, p_w = inputs[q]
        tau = TAU32 if prec == "fp32" else tau64(p_w)
        rep = compare_full(orc, geo.grid, geo.fluid, k_w, p_w, host(ens.r[q]), host(ens.J[q]),
                           tol=tol, tau=tau, ry=geo.ry, rz=geo.rz, seal=geo.seal)
        assert rep["max_err"] <= tol, (q, rep)
    ens.close()


# ---------------------------------------------------------------------------
# Residual-only kernels evaluate every in-plane face once and pass its flux
# through LDS; they must reproduce the Jacobian kernels' residual (which
# evaluates each face from both sides) bit for bit, for every tile shape and
# z-chunk and in the ensemble kernels.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(70, 9, 37), (129, 13, 3), (17, 33, 5), (1, 6, 4), (5, 1, 9)],
                         ids=lambda s: "x".join(map(str, s)) if isinstance(s, tuple) else s)
def test_shared_face_residual_bitwise(gpu, orc, shape, prec):
    geo = small(shape, seed=23)
    if prec == "fp64":
        k, p, pref = dev(geo.kx), dev(orc.pressure(geo)), None
    else:
        pref_h, dp, k32, _, _ = fp32_inputs(orc, geo)
        k, p, pref = dev(k32), dev(dp), dev(pref_h)
    kw = dict(seal=dev(geo.seal), pref=pref, ry=geo.ry, rz=geo.rz)
    print(f"shared-face residual {prec} {shape}", flush=True)
    r_ref, _ = gpu.jacobian(geo.grid, geo.fluid, k, p, **kw)
    r_ref = host(r_ref)
    for tile in range(len(gpu.tile_shapes())):
        for kz in (0, 1, 2, 5):
            r = host(gpu.residual(geo.grid, geo.fluid, k, p, tile=tile, kz_chunk=kz, **kw))
            assert np.array_equal(r, r_ref), (tile, kz)


# ---------------------------------------------------------------------------
# The FP32 Jacobian on the 64x8, 128x4 and 32x16 tiles evaluates each in-plane
# face once, in its lower cell, and hands F and both derivatives to the upper
# cell through LDS; the other tiles evaluate each face from both sides. Both
# give the same r and J bit for bit, in the ratio form and the backward-Euler
# Jacobian, for every tile shape and z-chunk.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(70, 9, 37), (129, 13, 3), (17, 33, 5), (1, 6, 4), (5, 1, 9)],
                         ids=lambda s: "x".join(map(str, s)))
def test_shared_face_fp32_jacobian_bitwise(gpu, orc, shape):
    geo = small(shape, seed=29)
    pref_h, dp, k32, _, _ = fp32_inputs(orc, geo)
    rng = np.random.default_rng(sum(shape))
    phi = rng.uniform(0.1, 0.3, geo.grid.shape).astype(np.float32)
    dpn = (dp - rng.uniform(0.0, 1e4, geo.grid.shape)).astype(np.float32)
    acc = dict(phi=dev(phi), p_prev=dev(dpn), dt=86400.0, cr=1e-9)
    k, p = dev(k32), dev(dp)
    kw = dict(seal=dev(geo.seal), pref=dev(pref_h), ry=geo.ry, rz=geo.rz)
    print(f"shared-face fp32 jacobian {shape}", flush=True)
    ref = None
    for tile in range(len(gpu.tile_shapes())):
        for kz in (0, 1, 5):
            out = [host(x) for x in gpu.jacobian(geo.grid, geo.fluid, k, p, tile=tile,
                                                 kz_chunk=kz, **kw)]
            out += [host(x) for x in gpu.jacobian_be(geo.grid, geo.fluid, k, p, acc, tile=tile,
                                                     kz_chunk=kz, **kw)]
            if ref is None:
                ref = out
            else:
                assert all(np.array_equal(x, y) for x, y in zip(out, ref)), (tile, kz)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ensemble_residual_mode_matches_single_launches(gpu, orc, prec):
    models = geomodel.ensemble(n_models=9, scale=0.15, base_seed=4100)
    members = []
    for m, geo in enumerate(models):
        if prec == "fp32":
            pref, dp, k32, _, _ = fp32_inputs(orc, geo)
            d = dict(grid=geo.grid, fluid=geo.fluid, kx=dev(k32), p=dev(dp), seal=dev(geo.seal),
                     pref=dev(pref), ry=geo.ry, rz=geo.rz, tile=m % 3, kz_chunk=4 + 5 * m)
        else:
            d = dict(grid=geo.grid, fluid=geo.fluid, kx=dev(geo.kx), p=dev(orc.pressure(geo)),
                     seal=dev(geo.seal), ry=geo.ry, rz=geo.rz, tile=m % 3, kz_chunk=4 + 5 * m)
        members.append(d)
    ens = gpu.Ensemble(members, mode="residual")
    singles = [gpu.jacobian(d["grid"], d["fluid"], d["kx"], d["p"], seal=d["seal"],
                            pref=d.get("pref"), ry=d["ry"], rz=d["rz"])[0] for d in members]
    for replay in range(4):
        for q in range(len(members)):
            ens.r[q].fill_(float("nan"))
        if replay == 2:
            ens.set_schedule("grouped")
        ens.run(graph=(replay != 1))
        torch.cuda.synchronize()
        for q, r in enumerate(singles):
            assert torch.equal(ens.r[q], r), (replay, q)
    ens.close()
