"""tpfa_residual_and_vjp: the residual and the vector-Jacobian product in one
pass. r equals tpfa_residual's and the gradients equal tpfa_residual_vjp's,
bit for bit, in both precisions, on every tile, on pitched inputs and row
ranges; and the results meet the oracle's bound directly."""
import numpy as np
import pytest
import torch

import geomodel
from test_gpu_pitch import TOL32, TOL64, case, dev, pad

pytestmark = pytest.mark.gpu


def both(gpu, geo, d, pref, **kw):
    g = geo.grid
    base = dict(seal=d["seal"], ry=geo.ry, rz=geo.rz, pref=pref, **kw)
    r = gpu.residual(g, geo.fluid, d["kx"], d["p"], **base)
    gp, gm = gpu.residual_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], **base)
    rf, gpf, gmf = gpu.residual_and_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], **base)
    torch.cuda.synchronize()
    return (r, gp, gm), (rf, gpf, gmf)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tile", range(10))
def test_bitwise_equal_to_separate_calls(gpu, prec, tile):
    geo, f, pref, be = case(prec, seed=41)
    d = {k: dev(v) for k, v in f.items()}
    print(f"residual and vjp, {prec}, tile {tile}", flush=True)
    want, got = both(gpu, geo, d, None if pref is None else dev(pref), tile=tile)
    for name, w_, g_ in zip(("r", "grad_p", "grad_logk"), want, got):
        assert torch.equal(w_, g_), (prec, tile, name)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pitched_inputs_and_rows(gpu, prec):
    geo, f, pref, be = case(prec, seed=43)
    pr = None if pref is None else dev(pref)
    print(f"residual and vjp, pitched, rows, {prec}", flush=True)
    d = {k: pad(v, 96) for k, v in f.items()}
    want, got = both(gpu, geo, d, pr)
    for w_, g_ in zip(want, got):
        assert torch.equal(w_, g_)
    d = {k: dev(v) for k, v in f.items()}
    want, got = both(gpu, geo, d, pr, rows=(3, 11))
    for w_, g_ in zip(want, got):
        assert torch.equal(w_[:, 3:11], g_[:, 3:11])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_against_oracle(gpu, orc, prec):
    """r in the per-cell metric, the gradients against the oracle's (relative
    to their largest magnitude)."""
    geo = geomodel.random_small(45, 67, 21, 10, sigma=1.3, seal_prob=0.03, ry=1.0, rz=0.2)
    g = geo.grid
    w = np.random.default_rng(46).standard_normal(g.shape)
    print(f"residual and vjp vs oracle {prec}", flush=True)
    if prec == "fp64":
        p = orc.pressure(geo)
        r, gp, gm = gpu.residual_and_vjp(g, geo.fluid, dev(geo.kx), dev(p), dev(w),
                                         seal=dev(geo.seal), ry=geo.ry, rz=geo.rz)
        kx, pw, wv, tol = geo.kx, p, w, TOL64
    else:
        pref = orc.hydrostatic(g, geo.fluid, geo.p_top)
        dp, k32, w32 = geo.dp32(), geo.kx32(), w.astype(np.float32)
        r, gp, gm = gpu.residual_and_vjp(g, geo.fluid, dev(k32), dev(dp), dev(w32),
                                         seal=dev(geo.seal), pref=dev(pref), ry=geo.ry,
                                         rz=geo.rz)
        kx, pw, wv, tol = (k32.astype(np.float64), orc.widen_fp32(dp, pref),
                           w32.astype(np.float64), TOL32)
    torch.cuda.synchronize()
    ref = orc.evaluate(g, geo.fluid, kx, pw, ry=geo.ry, rz=geo.rz, seal=geo.seal, w=wv,
                       want=("r", "scale", "grad_p", "grad_logk"))
    r, gp, gm = (x.double().cpu().numpy() for x in (r, gp, gm))
    e_r = np.max(np.abs(r - ref["r"]) / np.where(ref["scale"][0] > 0, ref["scale"][0], 1.0))
    e_p = np.abs(gp - ref["grad_p"]).max() / np.abs(ref["grad_p"]).max()
    e_m = np.abs(gm - ref["grad_logk"]).max() / np.abs(ref["grad_logk"]).max()
    print(f"r {e_r:.2e} grad_p {e_p:.2e} grad_logk {e_m:.2e}", flush=True)
    assert e_r <= tol and e_p <= 10 * tol and e_m <= 10 * tol, (e_r, e_p, e_m)


def test_binding_checks(gpu):
    geo = geomodel.random_small(3, 40, 7, 5)
    g = geo.grid
    kx, p = dev(geo.kx), dev(np.full(g.shape, 1e7))
    print("residual_and_vjp binding checks", flush=True)
    with pytest.raises(ValueError, match="gradient"):
        gpu.residual_and_vjp(g, geo.fluid, kx, p, p, want_p=False, want_logk=False)
