"""GPU parity of the transmissibility-input form (rock given as face
transmissibilities tx, ty, tz instead of kx, ratios and seal bits) against the
oracle's general evaluation, through every entry point that accepts it:
residual, Jacobian, 10-flux residual, backward-Euler residual and Jacobian,
Jacobian-vector product. FP64 (1e-12, every tile bitwise equal) and the FP32
precision form (1e-5 on widened inputs). The transmissibilities are drawn per
face, log-normal around the values the permeability form gives, with 5% of
faces closed (T = 0)."""
import numpy as np
import pytest
import torch

import geomodel
from helpers import apply_J, crop_mask, rel_err

pytestmark = pytest.mark.gpu

SHAPES = [(3, 5, 7), (70, 9, 37), (17, 33, 5), (129, 13, 3), (1, 6, 4)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def trans_case(shape, seed):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed, nx, ny, nz, sigma=1.0, seal_prob=0.0)
    rng = np.random.default_rng(seed + 99)
    g = geo.grid
    ts = []
    for a in (g.dy * g.dz / g.dx, g.dx * g.dz / g.dy, 0.1 * g.dx * g.dy / g.dz):
        t = a * 1e-13 * np.exp(rng.standard_normal(g.shape))
        t[rng.random(g.shape) < 0.05] = 0.0
        ts.append(t)
    diag = tuple(1e-13 * np.exp(rng.standard_normal(g.shape)) for _ in range(2))
    be = geomodel.be_fields(g, seed + 5)
    return geo, tuple(ts), diag, be


def check(got, ref, scale, tol, what):
    e = rel_err(np.asarray(got, np.float64), ref, scale)
    assert e.max() <= tol, (what, float(e.max()))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_trans_fp64(gpu, orc, shape):
    geo, tr, diag, be = trans_case(shape, 50 + sum(shape))
    g = geo.grid
    p = orc.pressure(geo)
    acc_h = dict(phi=be["phi"], p_prev=p - be["dp_step"], dt=be["dt"], cr=be["cr"])
    acc = dict(phi=dev(acc_h["phi"]), p_prev=dev(acc_h["p_prev"]), dt=be["dt"], cr=be["cr"])
    trd, pd, vd = tuple(dev(t) for t in tr), dev(p), dev(be["v"])
    print(f"transmissibility input fp64 {shape}", flush=True)
    ref = orc.evaluate_general(g, geo.fluid, p, trans=tr, want=("r", "J", "scale"))
    ref10 = orc.evaluate_general(g, geo.fluid, p, trans=tr, diag=diag, want=("r", "scale"))
    refbe = orc.evaluate_general(g, geo.fluid, p, trans=tr, accum=acc_h, v=be["v"],
                                 want=("r", "J", "jv", "scale"))
    first = None
    for tile in range(len(gpu.tile_shapes())):
        kw = dict(trans=trd, tile=tile)
        out = (host(gpu.residual(g, geo.fluid, None, pd, **kw)),
               *map(host, gpu.jacobian(g, geo.fluid, None, pd, **kw)),
               host(gpu.residual10(g, geo.fluid, None, pd, dev(diag[0]), dev(diag[1]), **kw)),
               host(gpu.residual_be(g, geo.fluid, None, pd, acc, **kw)),
               *map(host, gpu.jacobian_be(g, geo.fluid, None, pd, acc, **kw)),
               host(gpu.jvp(g, geo.fluid, None, pd, vd, accum=acc, **kw)[0]))
        r, rj, J, r10, rbe, rbej, Jbe, jv = out
        assert np.array_equal(r, rj) and np.array_equal(rbe, rbej)
        if first is None:
            check(r, ref["r"], ref["scale"][0], 1e-12, "r")
            check(J[0], ref["J"][0], ref["scale"][1], 1e-12, "J diag")
            for n in range(1, 7):
                check(J[n], ref["J"][n], np.abs(ref["J"][n]), 1e-12, f"J plane {n}")
            check(r10, ref10["r"], ref10["scale"][0], 1e-12, "r10")
            check(rbe, refbe["r"], refbe["scale"][0], 1e-12, "r be")
            check(Jbe[0], refbe["J"][0], refbe["scale"][1], 1e-12, "J be diag")
            scale = apply_J(np.abs(refbe["J"]), np.abs(be["v"]))
            assert np.all(np.abs(jv - refbe["jv"]) <= 1e-12 * scale + 1e-300)
            first = out
        else:
            for a, b in zip(out, first):
                assert np.array_equal(a, b), tile


@pytest.mark.parametrize("shape", SHAPES[:3], ids=lambda s: "x".join(map(str, s)))
def test_trans_fp32(gpu, orc, shape):
    geo, tr, diag, be = trans_case(shape, 70 + sum(shape))
    g = geo.grid
    pref = orc.hydrostatic(g, geo.fluid)
    dp = geo.dp32(0)
    tr32 = tuple(t.astype(np.float32) for t in tr)
    d32 = tuple(t.astype(np.float32) for t in diag)
    kw = dict(trans=tuple(dev(t) for t in tr32), pref=dev(pref))
    print(f"transmissibility input fp32 {shape}", flush=True)
    r = host(gpu.residual(g, geo.fluid, None, dev(dp), **kw))
    rj, J = map(host, gpu.jacobian(g, geo.fluid, None, dev(dp), **kw))
    r10 = host(gpu.residual10(g, geo.fluid, None, dev(dp), dev(d32[0]), dev(d32[1]), **kw))
    p_w = orc.widen_fp32(dp, pref)
    tw = tuple(t.astype(np.float64) for t in tr32)
    ref = orc.evaluate_general(g, geo.fluid, p_w, trans=tw, want=("r", "J", "scale"))
    ref10 = orc.evaluate_general(g, geo.fluid, p_w, trans=tw,
                                 diag=tuple(t.astype(np.float64) for t in d32),
                                 want=("r", "scale"))
    assert np.array_equal(r, rj)
    check(r, ref["r"], ref["scale"][0], 1e-5, "r")
    check(J[0], ref["J"][0], ref["scale"][1], 1e-5, "J diag")
    for n in range(1, 7):
        check(J[n], ref["J"][n], np.abs(ref["J"][n]), 1e-5, f"J plane {n}")
    check(r10, ref10["r"], ref10["scale"][0], 1e-5, "r10")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(3, 5, 7), (70, 9, 37), (129, 13, 3)],
                         ids=lambda s: "x".join(map(str, s)) if isinstance(s, tuple) else s)
def test_trans_vjp(gpu, orc, shape, prec):
    geo, tr, _, be = trans_case(shape, 90 + sum(shape))
    g = geo.grid
    w = be["v"]
    if prec == "fp64":
        p = orc.pressure(geo)
        kw = dict(trans=tuple(dev(t) for t in tr))
        pd, wd, p_w, tw, w_w, tol = dev(p), dev(w), p, tr, w, 1e-12
    else:
        pref = orc.hydrostatic(g, geo.fluid)
        dp = geo.dp32(0)
        tr32 = tuple(t.astype(np.float32) for t in tr)
        w32 = w.astype(np.float32)
        kw = dict(trans=tuple(dev(t) for t in tr32), pref=dev(pref))
        pd, wd = dev(dp), dev(w32)
        p_w, tw, w_w, tol = (orc.widen_fp32(dp, pref), tuple(t.astype(np.float64) for t in tr32),
                             w32.astype(np.float64), 1e-5)
    print(f"transmissibility-form vjp {prec} {shape}", flush=True)
    ref_gp, ref_gt, _ = orc.vjp_general(g, geo.fluid, p_w, w_w, trans=tw)
    ev = orc.evaluate_general(g, geo.fluid, p_w, trans=tw, want=("J", "scale"))
    from helpers import apply_JT, shift
    gp_scale = apply_JT(np.abs(ev["J"]), np.abs(w_w))
    # R16-style scale of the ln T gradient of a face: (|w_lo| + |w_hi|) times
    # the larger flux scale sum |F| of its two cells (the FP32 z-face potential
    # error, ~2e-3 Pa, is small against a cell's fluxes, not against a face
    # whose own potential difference is a few Pa)
    s, aw = ev["scale"][0], np.abs(w_w)
    gt_scale = [(aw + shift(aw, 2 * a + 1)) * np.maximum(s, shift(s, 2 * a + 1))
                for a in range(3)]
    first = None
    for tile in ((0, 3, 4) if prec == "fp64" else (None,)):
        gp, gt = gpu.residual_vjp(g, geo.fluid, None, pd, wd, tile=tile, **kw)
        gp, gt = host(gp), host(gt)
        assert gt.shape == (3,) + g.shape
        if first is None:
            check(gp, ref_gp, gp_scale, tol, "grad_p")
            for a in range(3):
                check(gt[a], ref_gt[a], gt_scale[a], tol, f"grad ln T axis {a}")
            first = (gp, gt)
        else:
            assert np.array_equal(gp, first[0]) and np.array_equal(gt, first[1]), tile


@pytest.mark.slow
def test_fullsize_paper10_given_transmissibilities(gpu, orc):
    """750 x 994 x 246, all ten transmissibilities given (the benchmark's
    paper10 transmissibility line, default launch): eight 24^3 crops against
    the oracle on the cells whose ten faces lie inside the crop, and
    conservation over the whole grid."""
    nx, ny, nz = geomodel.PAPER10_SHAPES[-1]
    g = geomodel.Grid(nx, ny, nz)
    tr = geomodel.paper10_trans(nx, ny, nz)
    dp = geomodel.paper10(nx, ny, nz).noise[0]
    fl = geomodel.Fluid()
    pref = orc.hydrostatic(g, fl)
    print(f"paper10 given transmissibilities {nx}x{ny}x{nz}", flush=True)
    r = gpu.residual10(g, fl, None, dev(dp), dev(tr["tne"]), dev(tr["tse"]), pref=dev(pref),
                       trans=(dev(tr["tx"]), dev(tr["ty"]), dev(tr["tz"])))
    torch.cuda.synchronize()
    r_sum = float(r.double().sum().item())
    r_abs = float(r.double().abs().sum().item())
    assert abs(r_sum) <= 1e-5 * r_abs
    r = r.cpu().numpy()
    c = 24
    for (i0, j0, k0) in [(0, 0, 0), (nx - c, ny - c, nz - c), (0, ny - c, 100), (nx - c, 0, 0),
                         (370, 500, 120), (63, 255, nz - c), (511, 0, 7), (0, 700, 200)]:
        sl = (slice(k0, k0 + c), slice(j0, j0 + c), slice(i0, i0 + c))
        sub = geomodel.Grid(c, c, c, g.dx, g.dy, g.dz, g.gk)
        mask = crop_mask(sub.shape, (i0, j0, k0), (i0 + c, j0 + c, k0 + c), (nx, ny, nz))
        w = {key: tr[key][sl].astype(np.float64) for key in tr}
        # a crop's last layer along each axis has faces leaving the crop: the
        # oracle closes them (the crop boundary), and the mask drops those cells
        ref = orc.evaluate_general(sub, fl, orc.widen_fp32(dp[sl], pref[k0:k0 + c]),
                                   trans=(w["tx"], w["ty"], w["tz"]), diag=(w["tne"], w["tse"]),
                                   want=("r", "scale"))
        e = np.where(mask, rel_err(r[sl], ref["r"], ref["scale"][0]), 0.0)
        assert e.max() <= 1e-5, ((i0, j0, k0), float(e.max()))
