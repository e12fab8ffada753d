"""GPU parity of the full backward-Euler residual of Eq. (2) (accumulation
term plus flux sum), its Jacobian, and the matrix-free Jacobian-vector
product, against the FP64 oracle (tpfa_residual_be, tpfa_jacobian_be,
tpfa_jvp through the C ABI):

* FP64 (1e-12) and the FP32 precision form (1e-5, inputs widened for the
  oracle), every tile shape bitwise equal;
* the residual of the three entry points bitwise equal to each other;
* J v against the oracle's J v and against the GPU's own stored J applied in
  FP64 on the host; the flux-only J v (no accumulation) against the oracle
  with zero porosity.

Metric: residual error over the oracle's per-cell scale (sum of |fluxes| plus
V/dt (|phi rho| + |phi_n rho_n|)), the Jacobian as in the flux tests, J v
over sum_L |J_KL| |v_L|.
"""
import numpy as np
import pytest
import torch

import geomodel
from helpers import apply_J, crop_mask, rel_err

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
SHAPES = [(3, 5, 7), (70, 9, 37), (17, 33, 5), (129, 13, 3), (1, 6, 4), (65, 3, 2)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def case(shape, seed=3):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed + 11 * nx + 7 * ny + nz, nx, ny, nz, sigma=1.3,
                                seal_prob=0.05)
    be = geomodel.be_fields(geo.grid, seed + nx + ny + nz)
    return geo, be


def oracle_be(orc, geo, p, phi, p_prev, be, v=None, want=("r", "J", "scale")):
    return orc.evaluate_be(geo.grid, geo.fluid, geo.kx, p, phi, p_prev, be["dt"], be["cr"],
                           ry=geo.ry, rz=geo.rz, seal=geo.seal, v=v, want=want)


def check_rJ(r, J, ref, tol):
    assert rel_err(r, ref["r"], ref["scale"][0]).max() <= tol
    if J is not None:
        assert rel_err(J[0], ref["J"][0], ref["scale"][1]).max() <= tol
        for n in range(1, 7):
            assert rel_err(J[n], ref["J"][n], np.abs(ref["J"][n])).max() <= tol


def check_jv(jv, J_ref, v, jv_ref, tol):
    scale = apply_J(np.abs(J_ref), np.abs(v))
    err = np.abs(np.asarray(jv, np.float64) - jv_ref)
    assert np.all(err <= tol * scale + 1e-300), float(np.max(err / np.maximum(scale, 1e-300)))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_be_fp64(gpu, orc, shape):
    geo, be = case(shape)
    p = orc.pressure(geo)
    p_prev = p - be["dp_step"]
    print(f"backward-Euler fp64 {shape}", flush=True)
    acc = dict(phi=dev(be["phi"]), p_prev=dev(p_prev), dt=be["dt"], cr=be["cr"])
    kw = dict(seal=dev(geo.seal), ry=geo.ry, rz=geo.rz)
    k, pd, vd = dev(geo.kx), dev(p), dev(be["v"])
    ref = oracle_be(orc, geo, p, be["phi"], p_prev, be, v=be["v"], want=("r", "J", "scale", "jv"))
    r0 = J0 = None
    for tile in range(len(gpu.tile_shapes())):
        r = host(gpu.residual_be(geo.grid, geo.fluid, k, pd, acc, tile=tile, **kw))
        rj, J = gpu.jacobian_be(geo.grid, geo.fluid, k, pd, acc, tile=tile, **kw)
        jv, rv = gpu.jvp(geo.grid, geo.fluid, k, pd, vd, accum=acc, want_r=True, tile=tile, **kw)
        rj, J, jv, rv = host(rj), host(J), host(jv), host(rv)
        assert np.array_equal(r, rj) and np.array_equal(r, rv), tile
        if r0 is None:
            check_rJ(r, J, ref, TOL64)
            check_jv(jv, ref["J"], be["v"], ref["jv"], TOL64)
            # J v of the stored J, applied on the host in FP64
            check_jv(jv, ref["J"], be["v"], apply_J(J, be["v"]), 1e-14)
            r0, J0, jv0 = r, J, jv
        else:
            assert np.array_equal(r, r0) and np.array_equal(J, J0) and np.array_equal(jv, jv0)


@pytest.mark.parametrize("shape", SHAPES[:4], ids=lambda s: "x".join(map(str, s)))
def test_be_fp32(gpu, orc, shape):
    geo, be = case(shape, seed=8)
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    dp = geo.dp32(0)
    dpn = (geo.noise[0] - be["dp_step"]).astype(np.float32)
    k32, phi32, v32 = geo.kx32(), be["phi"].astype(np.float32), be["v"].astype(np.float32)
    print(f"backward-Euler fp32 {shape}", flush=True)
    acc = dict(phi=dev(phi32), p_prev=dev(dpn), dt=be["dt"], cr=be["cr"])
    kw = dict(seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz)
    k, pd, vd = dev(k32), dev(dp), dev(v32)
    r = host(gpu.residual_be(geo.grid, geo.fluid, k, pd, acc, **kw))
    rj, J = gpu.jacobian_be(geo.grid, geo.fluid, k, pd, acc, **kw)
    jv, rv = gpu.jvp(geo.grid, geo.fluid, k, pd, vd, accum=acc, want_r=True, **kw)
    rj, J, jv, rv = host(rj), host(J), host(jv), host(rv)
    assert np.array_equal(r, rj) and np.array_equal(r, rv)
    p_w, pn_w = orc.widen_fp32(dp, pref), orc.widen_fp32(dpn, pref)
    ref = orc.evaluate_be(geo.grid, geo.fluid, k32.astype(np.float64), p_w,
                          phi32.astype(np.float64), pn_w, be["dt"], be["cr"], ry=geo.ry,
                          rz=geo.rz, seal=geo.seal, v=v32.astype(np.float64),
                          want=("r", "J", "scale", "jv"))
    check_rJ(r.astype(np.float64), J.astype(np.float64), ref, TOL32)
    check_jv(jv, ref["J"], v32.astype(np.float64), ref["jv"], TOL32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flux_jvp_without_accumulation(gpu, orc, prec):
    geo, be = case((70, 9, 37), seed=21)
    zero = np.zeros(geo.grid.shape)
    if prec == "fp64":
        p = orc.pressure(geo)
        k, pd, vd, pref = dev(geo.kx), dev(p), dev(be["v"]), None
        k_w, p_w, v_w, tol = geo.kx, p, be["v"], TOL64
    else:
        pref_h = orc.hydrostatic(geo.grid, geo.fluid)
        dp, k32, v32 = geo.dp32(0), geo.kx32(), be["v"].astype(np.float32)
        k, pd, vd, pref = dev(k32), dev(dp), dev(v32), dev(pref_h)
        k_w, p_w, v_w, tol = (k32.astype(np.float64), orc.widen_fp32(dp, pref_h),
                              v32.astype(np.float64), TOL32)
    kw = dict(seal=dev(geo.seal), pref=pref, ry=geo.ry, rz=geo.rz)
    jv, r = gpu.jvp(geo.grid, geo.fluid, k, pd, vd, want_r=True, **kw)
    r_flux = gpu.residual(geo.grid, geo.fluid, k, pd, **kw)
    torch.cuda.synchronize()
    assert torch.equal(r, r_flux)
    ref = orc.evaluate_be(geo.grid, geo.fluid, k_w, p_w, zero, p_w, 1.0, 0.0, ry=geo.ry,
                          rz=geo.rz, seal=geo.seal, v=v_w, want=("J", "jv"))
    check_jv(host(jv), ref["J"], v_w, ref["jv"], tol)


CROPS = [(0, 0, 0), (488, 488, 232), (0, 488, 100), (488, 0, 0), (250, 250, 120),
         (63, 255, 232), (301, 0, 7), (0, 400, 200)]


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fullsize_backward_euler(gpu, orc, prec):
    """512 x 512 x 256, the benchmark's backward-Euler inputs and default
    launches: the full residual (and in FP64 J v) on eight 24^3 crops against
    the oracle, on the crop cells whose faces all lie inside the crop."""
    geo = geomodel.big512(noise_seeds=(2,))
    g = geo.grid
    be = geomodel.be_fields(g, 9)
    pref = orc.hydrostatic(g, geo.fluid)
    print(f"512x512x256 backward Euler {prec}", flush=True)
    if prec == "fp64":
        p = pref[:, None, None] + geo.noise[0]
        pn = p - be["dp_step"]
        k, phi, v, tol = geo.kx, be["phi"], be["v"], TOL64
        kw = dict(seal=dev(geo.seal), ry=geo.ry, rz=geo.rz)
        p_in, pn_in = p, pn
    else:
        dp = geo.noise[0].astype(np.float32)
        dpn = (geo.noise[0] - be["dp_step"]).astype(np.float32)
        k, phi, v = (geo.kx32().astype(np.float64), be["phi"].astype(np.float32),
                     be["v"].astype(np.float32))
        p, pn = orc.widen_fp32(dp, pref), orc.widen_fp32(dpn, pref)
        kw = dict(seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz)
        p_in, pn_in, tol = dp, dpn, TOL32
    k_in = k if prec == "fp64" else k.astype(np.float32)
    acc = dict(phi=dev(phi), p_prev=dev(pn_in), dt=be["dt"], cr=be["cr"])
    jv, r = gpu.jvp(g, geo.fluid, dev(k_in), dev(p_in), dev(v), accum=acc, want_r=True, **kw)
    torch.cuda.synchronize()
    r, jv = r.cpu().numpy().astype(np.float64), jv.cpu().numpy().astype(np.float64)
    c = 24
    for (i0, j0, k0) in CROPS:
        sl = (slice(k0, k0 + c), slice(j0, j0 + c), slice(i0, i0 + c))
        sub = geomodel.Grid(c, c, c, g.dx, g.dy, g.dz, g.gk)
        mask = crop_mask(sub.shape, (i0, j0, k0), (i0 + c, j0 + c, k0 + c), (g.nx, g.ny, g.nz))
        ref = orc.evaluate_be(sub, geo.fluid, k[sl], p[sl], np.asarray(phi[sl], np.float64),
                              pn[sl], be["dt"], be["cr"], ry=geo.ry, rz=geo.rz,
                              seal=geo.seal[sl], v=np.asarray(v[sl], np.float64),
                              want=("r", "J", "scale", "jv"))
        e = np.where(mask, rel_err(r[sl], ref["r"], ref["scale"][0]), 0.0)
        assert e.max() <= tol, ((i0, j0, k0), float(e.max()))
        if prec == "fp64":
            scale = apply_J(np.abs(ref["J"]), np.abs(np.asarray(v[sl], np.float64)))
            ej = np.where(mask, np.abs(jv[sl] - ref["jv"]) / np.maximum(scale, 1e-300), 0.0)
            assert ej.max() <= tol, ((i0, j0, k0), float(ej.max()))
