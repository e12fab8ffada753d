"""GPU parity of the per-direction permeability form (kx, ky, kz arrays, each
face taking the harmonic average of its own direction's permeability) against
the oracle, through every entry point that accepts it: residual, Jacobian,
10-flux residual, backward-Euler residual and Jacobian, Jacobian-vector
product, and the vector-Jacobian product with its three ln k gradient planes;
the autograd Function of the form. FP64 (1e-12, tiles bitwise equal) and the
FP32 precision form (1e-5 on widened inputs), in the per-cell relative metric
of tests/helpers.py. ky and kz are the geomodel's kx times independent
log-normal factors (kz around 0.1 kx), seal bits on 5% of faces."""
import numpy as np
import pytest
import torch

import geomodel
from helpers import apply_J, apply_JT, compare_full, rel_err, shift

pytestmark = pytest.mark.gpu

SHAPES = [(3, 5, 7), (70, 9, 37), (17, 33, 5), (129, 13, 3), (1, 6, 4), (64, 4, 9)]
TAU32 = 1e-4  # Pa: upwind tie band of the FP32 form (its |dPhi| error is below 1e-6 Pa)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def k3_case(shape, seed):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed, nx, ny, nz, sigma=1.2, seal_prob=0.05)
    k3 = geomodel.k3_fields(geo.kx, seed + 7)
    diag = geomodel.diagonal_t(geo.grid, seed + 8)
    be = geomodel.be_fields(geo.grid, seed + 9)
    return geo, k3, diag, be


def check(got, ref, scale, tol, what):
    e = rel_err(np.asarray(got, np.float64), ref, scale)
    assert e.max() <= tol, (what, float(e.max()))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_k3_fp64_every_entry_point(gpu, orc, shape):
    geo, (kx, ky, kz), diag, be = k3_case(shape, 20 + sum(shape))
    g = geo.grid
    p = orc.pressure(geo)
    acc_h = dict(phi=be["phi"], p_prev=p - be["dp_step"], dt=be["dt"], cr=be["cr"])
    acc = dict(phi=dev(acc_h["phi"]), p_prev=dev(acc_h["p_prev"]), dt=be["dt"], cr=be["cr"])
    kxd, pd, vd, sd = dev(kx), dev(p), dev(be["v"]), dev(geo.seal)
    print(f"per-direction permeability fp64 {shape}", flush=True)
    ref10 = orc.evaluate_k3(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, diag=diag,
                            want=("r", "scale"))
    refbe = orc.evaluate_k3(g, geo.fluid, p, kx, ky, kz, seal=geo.seal, accum=acc_h,
                            v=be["v"], want=("r", "J", "jv", "scale"))
    first = None
    for tile in range(len(gpu.tile_shapes())):
        kw = dict(seal=sd, ky=dev(ky), kz=dev(kz), tile=tile)
        out = (host(gpu.residual(g, geo.fluid, kxd, pd, **kw)),
               *map(host, gpu.jacobian(g, geo.fluid, kxd, pd, **kw)),
               host(gpu.residual10(g, geo.fluid, kxd, pd, dev(diag[0]), dev(diag[1]), **kw)),
               host(gpu.residual_be(g, geo.fluid, kxd, pd, acc, **kw)),
               *map(host, gpu.jacobian_be(g, geo.fluid, kxd, pd, acc, **kw)),
               host(gpu.jvp(g, geo.fluid, kxd, pd, vd, accum=acc, **kw)[0]))
        r, rj, J, r10, rbe, rbej, Jbe, jv = out
        assert np.array_equal(r, rj) and np.array_equal(rbe, rbej)
        if first is None:
            rep = compare_full(orc, g, geo.fluid, kx, p, r, J, tol=1e-12,
                               tau=1e-9 * float(np.abs(p).max()), ry=1.0, rz=1.0,
                               seal=geo.seal, ky=ky, kz=kz)
            assert rep["max_err"] <= 1e-12, rep
            check(r10, ref10["r"], ref10["scale"][0], 1e-12, "r10")
            check(rbe, refbe["r"], refbe["scale"][0], 1e-12, "r be")
            check(Jbe[0], refbe["J"][0], refbe["scale"][1], 1e-12, "J be diag")
            for n in range(1, 7):
                check(Jbe[n], refbe["J"][n], np.abs(refbe["J"][n]), 1e-12, f"J be plane {n}")
            scale = apply_J(np.abs(refbe["J"]), np.abs(be["v"]))
            assert np.all(np.abs(jv - refbe["jv"]) <= 1e-12 * scale + 1e-300)
            first = out
        else:
            for a, b in zip(out, first):
                assert np.array_equal(a, b), tile


@pytest.mark.parametrize("shape", SHAPES[:4], ids=lambda s: "x".join(map(str, s)))
def test_k3_fp32(gpu, orc, shape):
    geo, k3, diag, be = k3_case(shape, 40 + sum(shape))
    g = geo.grid
    pref = orc.hydrostatic(g, geo.fluid)
    dp = geo.dp32(0)
    k32 = tuple(k.astype(np.float32) for k in k3)
    d32 = tuple(t.astype(np.float32) for t in diag)
    print(f"per-direction permeability fp32 {shape}", flush=True)
    p_w = orc.widen_fp32(dp, pref)
    kw3 = tuple(k.astype(np.float64) for k in k32)
    ref10 = orc.evaluate_k3(g, geo.fluid, p_w, *kw3, seal=geo.seal,
                            diag=tuple(t.astype(np.float64) for t in d32), want=("r", "scale"))
    first = None
    for tile in (None, 0, 3):
        kw = dict(seal=dev(geo.seal), pref=dev(pref), ky=dev(k32[1]), kz=dev(k32[2]), tile=tile)
        r = host(gpu.residual(g, geo.fluid, dev(k32[0]), dev(dp), **kw))
        rj, J = map(host, gpu.jacobian(g, geo.fluid, dev(k32[0]), dev(dp), **kw))
        r10 = host(gpu.residual10(g, geo.fluid, dev(k32[0]), dev(dp), dev(d32[0]), dev(d32[1]),
                                  **kw))
        assert r.dtype == np.float32 and np.array_equal(r, rj)
        if first is None:
            rep = compare_full(orc, g, geo.fluid, kw3[0], p_w, r, J, tol=1e-5, tau=TAU32,
                               ry=1.0, rz=1.0, seal=geo.seal, ky=kw3[1], kz=kw3[2])
            assert rep["max_err"] <= 1e-5, rep
            check(r10, ref10["r"], ref10["scale"][0], 1e-5, "r10")
            first = (r, J, r10)
        else:
            assert all(np.array_equal(a, b) for a, b in zip((r, J, r10), first)), tile


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(3, 5, 7), (70, 9, 37), (129, 13, 3), (64, 4, 9)],
                         ids=lambda s: "x".join(map(str, s)))
def test_k3_vjp(gpu, orc, shape, prec):
    """grad_p = J^T w and the three planes d(w.r)/d ln kx, ln ky, ln kz."""
    geo, k3, _, be = k3_case(shape, 60 + sum(shape))
    g = geo.grid
    w = be["v"]
    if prec == "fp64":
        p = orc.pressure(geo)
        kd = tuple(dev(k) for k in k3)
        pd, wd, p_w, kw3, w_w, tol, extra = dev(p), dev(w), p, k3, w, 1e-12, {}
    else:
        pref = orc.hydrostatic(g, geo.fluid)
        dp = geo.dp32(0)
        k32 = tuple(k.astype(np.float32) for k in k3)
        w32 = w.astype(np.float32)
        kd = tuple(dev(k) for k in k32)
        pd, wd = dev(dp), dev(w32)
        p_w, kw3, w_w, tol = (orc.widen_fp32(dp, pref), tuple(k.astype(np.float64) for k in k32),
                              w32.astype(np.float64), 1e-5)
        extra = dict(pref=dev(pref))
    print(f"per-direction vjp {prec} {shape}", flush=True)
    ref = orc.evaluate_k3(g, geo.fluid, p_w, *kw3, seal=geo.seal, w=w_w,
                          want=("J", "scale", "grad_p", "grad_k3"))
    gp_scale = apply_JT(np.abs(ref["J"]), np.abs(w_w))
    # per-cell magnitude of a log-permeability gradient: twice the largest
    # |w| of the cell and its neighbours times the cell's flux scale
    aw = np.abs(w_w)
    wmax = aw.copy()
    for n in range(6):
        wmax = np.maximum(wmax, shift(aw, n))
    gk_scale = 2.0 * wmax * ref["scale"][0]
    first = None
    for tile in ((0, 3, 4) if prec == "fp64" else (None, 1)):
        gp, gk = gpu.residual_vjp(g, geo.fluid, kd[0], pd, wd, seal=dev(geo.seal), ky=kd[1],
                                  kz=kd[2], tile=tile, **extra)
        gp, gk = host(gp), host(gk)
        assert gk.shape == (3,) + g.shape
        if first is None:
            check(gp, ref["grad_p"], gp_scale, tol, "grad_p")
            for a in range(3):
                check(gk[a], ref["grad_k3"][a], gk_scale, tol, f"grad ln k axis {a}")
            first = (gp, gk)
        else:
            assert np.array_equal(gp, first[0]) and np.array_equal(gk, first[1]), tile


def test_k3_ratio_arrays_close_to_ratio_form(gpu, orc):
    """ky = ry kx and kz = rz kx given as arrays: the same residual and
    Jacobian as the ratio form up to the rounding of the factored products."""
    geo = geomodel.random_small(3, 33, 17, 9, sigma=1.5, seal_prob=0.05, ry=0.5, rz=0.1)
    p = orc.pressure(geo)
    kx = dev(geo.kx)
    a = gpu.jacobian(geo.grid, geo.fluid, kx, dev(p), seal=dev(geo.seal), ry=geo.ry, rz=geo.rz)
    b = gpu.jacobian(geo.grid, geo.fluid, kx, dev(p), seal=dev(geo.seal),
                     ky=dev(geo.ry * geo.kx), kz=dev(geo.rz * geo.kx))
    ref = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "J", "scale"))
    check(host(a[0]), host(b[0]), ref["scale"][0], 1e-14, "r")
    check(host(a[1])[0], host(b[1])[0], ref["scale"][1], 1e-14, "J diag")


def test_aniso_function_gradcheck_fp64(gpu, orc):
    geo = geomodel.random_small(6, 3, 4, 3, seal_prob=0.1)
    p = orc.pressure(geo)
    logk3 = np.log(np.stack(geomodel.k3_fields(geo.kx, 9)))
    scale = 1e5
    seal = dev(geo.seal)

    def f(ps_, lk_):
        return gpu.TPFAAnisoResidual.apply(ps_ * scale, lk_, geo.grid, geo.fluid, seal)

    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda",  # noqa: E731
                               requires_grad=True)
    assert torch.autograd.gradcheck(f, (t(p / scale), t(logk3)), eps=1e-6, atol=1e-9,
                                    rtol=1e-6)


def test_aniso_function_matches_oracle(gpu, orc):
    geo = geomodel.random_small(8, 33, 17, 9, seal_prob=0.05)
    p = orc.pressure(geo)
    k3 = geomodel.k3_fields(geo.kx, 10)
    w = np.random.default_rng(11).standard_normal(p.shape)
    pt = torch.tensor(p, dtype=torch.float64, device="cuda", requires_grad=True)
    lk = torch.tensor(np.log(np.stack(k3)), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    r = gpu.TPFAAnisoResidual.apply(pt, lk, geo.grid, geo.fluid, dev(geo.seal))
    r.backward(dev(w))
    # the Function forms k = exp(ln k) on the GPU; the oracle takes those values
    kk = torch.exp(lk.detach()).cpu().numpy()
    ref = orc.evaluate_k3(geo.grid, geo.fluid, p, kk[0], kk[1], kk[2], seal=geo.seal, w=w,
                          want=("r", "J", "scale", "grad_p", "grad_k3", "grad_k3_scale"))
    check(r.detach().cpu().numpy(), ref["r"], ref["scale"][0], 1e-12, "r")
    check(pt.grad.cpu().numpy(), ref["grad_p"], apply_JT(np.abs(ref["J"]), np.abs(w)), 1e-12,
          "grad_p")
    gk = lk.grad.cpu().numpy()
    for a in range(3):
        check(gk[a], ref["grad_k3"][a], ref["grad_k3_scale"][a], 1e-12, f"grad ln k {a}")
