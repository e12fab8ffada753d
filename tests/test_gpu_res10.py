"""GPU parity of the 10-flux stencil (six TPFA faces plus the four in-plane
diagonal faces the paper's kernel evaluates, Sec. 3) against the FP64 oracle:
odd shapes over every tile shape and several z-chunks (FP64 and the FP32
precision form), reduction to the 6-face residual when the diagonal
transmissibilities vanish, conservation, and the paper's own 750 x 994 x 246
FP32 workload checked on crops whose interior cells see the same neighbours
as in the full grid.

Tolerances: 1e-12 (FP64) and 1e-5 (FP32) in the per-cell relative metric
(residual error over the cell's flux scale sum |F|)."""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_res10, crop_mask

pytestmark = pytest.mark.gpu

TOL64, TOL32, TAU32 = 1e-12, 1e-5, 1e-4

SHAPES = [(1, 1, 5), (2, 2, 2), (3, 5, 7), (65, 3, 2), (70, 9, 37), (17, 33, 5),
          (130, 6, 70), (33, 17, 40), (129, 13, 3), (5, 1, 9), (1, 6, 4)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def small(shape, seed=17):
    nx, ny, nz = shape
    geo = geomodel.random_small(seed + 3 * nx + 5 * ny + 7 * nz, nx, ny, nz, sigma=1.5,
                                seal_prob=0.05)
    tne, tse = geomodel.diagonal_t(geo.grid, seed + nx + ny + nz)
    return geo, tne, tse


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_res10_fp64_all_tiles(gpu, orc, shape):
    geo, tne, tse = small(shape)
    p = orc.pressure(geo)
    print(f"res10 fp64 {shape}", flush=True)
    args = (geo.grid, geo.fluid, dev(geo.kx), dev(p), dev(tne), dev(tse))
    kw = dict(seal=dev(geo.seal), ry=geo.ry, rz=geo.rz)
    ref = None
    for tile in range(len(gpu.tile_shapes())):
        for kz in (0, 1, 3):
            r = host(gpu.residual10(*args, tile=tile, kz_chunk=kz, **kw))
            if ref is None:
                ref = r
                rep = compare_res10(orc, geo.grid, geo.fluid, geo.kx, p, tne, tse, r, tol=TOL64,
                                    tau=1e-9 * np.abs(p).max(), ry=geo.ry, rz=geo.rz,
                                    seal=geo.seal)
                assert rep["max_err"] <= TOL64, rep
            else:
                # every tile and chunk evaluates each cell with the same arithmetic
                assert np.array_equal(r, ref), (tile, kz)


@pytest.mark.parametrize("shape", SHAPES[2:8], ids=lambda s: "x".join(map(str, s)))
def test_res10_fp32_precision_form(gpu, orc, shape):
    geo, tne, tse = small(shape, seed=29)
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    dp, k32 = geo.dp32(0), geo.kx32()
    t32 = (tne.astype(np.float32), tse.astype(np.float32))
    print(f"res10 fp32 {shape}", flush=True)
    ref = None
    for tile in (0, 1, 3, 9):
        r = host(gpu.residual10(geo.grid, geo.fluid, dev(k32), dev(dp), dev(t32[0]), dev(t32[1]),
                                seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz,
                                tile=tile))
        if ref is None:
            ref = r
        assert np.array_equal(r, ref), tile
    p_w = orc.widen_fp32(dp, pref)
    rep = compare_res10(orc, geo.grid, geo.fluid, k32.astype(np.float64), p_w,
                        t32[0].astype(np.float64), t32[1].astype(np.float64), ref, tol=TOL32,
                        tau=TAU32, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    print(rep)
    assert rep["max_err"] <= TOL32, rep


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_res10_zero_diagonals_match_residual(gpu, orc, fp32):
    geo, _, _ = small((70, 9, 37), seed=41)
    z = np.zeros(geo.grid.shape)
    if fp32:
        pref = dev(orc.hydrostatic(geo.grid, geo.fluid))
        k, p, z = dev(geo.kx32()), dev(geo.dp32(0)), dev(z.astype(np.float32))
    else:
        pref = None
        k, p, z = dev(geo.kx), dev(orc.pressure(geo)), dev(z)
    kw = dict(seal=dev(geo.seal), pref=pref, ry=geo.ry, rz=geo.rz)
    # the Jacobian kernel evaluates each face from both sides (no shared fluxes)
    r_two_sided, _ = gpu.jacobian(geo.grid, geo.fluid, k, p, **kw)
    for tile in range(len(gpu.tile_shapes())):
        r10 = gpu.residual10(geo.grid, geo.fluid, k, p, z, z, tile=tile, **kw)
        r6 = gpu.residual(geo.grid, geo.fluid, k, p, tile=tile, **kw)
        torch.cuda.synchronize()
        assert torch.equal(r10, r6) and torch.equal(r10, r_two_sided), tile


def test_res10_conservation(gpu, orc):
    geo, tne, tse = small((130, 6, 70), seed=5)
    p = orc.pressure(geo)
    r = host(gpu.residual10(geo.grid, geo.fluid, dev(geo.kx), dev(p), dev(tne), dev(tse),
                            seal=dev(geo.seal), ry=geo.ry, rz=geo.rz))
    _, scale = orc.residual10(geo.grid, geo.fluid, geo.kx, p, tne, tse, ry=geo.ry, rz=geo.rz,
                              seal=geo.seal)
    assert abs(r.sum()) <= 16 * r.size * 1.2e-16 * scale.sum()


@pytest.mark.slow
def test_res10_paper_workload_fp32(gpu, orc):
    """750 x 994 x 246 (183,393,000 cells), FP32, default launch: eight crops
    (the domain's corners and edges and interior blocks) against the oracle,
    and conservation over the whole grid."""
    geo = geomodel.paper10()
    g = geo.grid
    print(f"paper10 {g.nx}x{g.ny}x{g.nz}", flush=True)
    pref = orc.hydrostatic(g, geo.fluid)
    kx, dp = geo.kx, geo.noise[0]
    tne, tse = geo.extra["tne"], geo.extra["tse"]
    r = gpu.residual10(g, geo.fluid, dev(kx), dev(dp), dev(tne), dev(tse), pref=dev(pref),
                       ry=geo.ry, rz=geo.rz)
    torch.cuda.synchronize()
    r_sum = float(r.double().sum().item())
    r_abs = float(r.double().abs().sum().item())
    r = r.cpu().numpy()
    assert abs(r_sum) <= 1e-5 * r_abs
    c = 24
    starts = [(0, 0, 0), (g.nx - c, g.ny - c, g.nz - c), (0, g.ny - c, 100), (g.nx - c, 0, 0),
              (370, 500, 120), (63, 255, g.nz - c), (511, 0, 7), (0, 700, 200)]
    for (i0, j0, k0) in starts:
        lo, hi = (i0, j0, k0), (i0 + c, j0 + c, k0 + c)
        sl = (slice(k0, k0 + c), slice(j0, j0 + c), slice(i0, i0 + c))
        sub = geomodel.Grid(c, c, c, g.dx, g.dy, g.dz, g.gk)
        p_w = orc.widen_fp32(dp[sl], pref[k0:k0 + c])
        mask = crop_mask(sub.shape, lo, hi, (g.nx, g.ny, g.nz))
        rep = compare_res10(orc, sub, geo.fluid, kx[sl].astype(np.float64), p_w,
                            tne[sl].astype(np.float64), tse[sl].astype(np.float64), r[sl],
                            tol=TOL32, tau=TAU32, ry=geo.ry, rz=geo.rz, seal=None, mask=mask)
        print(lo, rep)
        assert rep["max_err"] <= TOL32, (lo, rep)
