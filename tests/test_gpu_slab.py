"""The y-slab launch (a row range of the grid computed and written, the other
rows read as a halo): the kernel of one GPU in a y-slab decomposition. A
decomposition into uneven slabs is emulated on one GPU, each slab on its own
local arrays (its rows plus one halo row per side, copied from the global
arrays as the exchange would deliver them); every slab's outputs must equal
the owned rows of the full-grid launch bitwise, in every rock form and mode
(residual, Jacobian, VJP, 10-flux, backward Euler, J v; FP64 and FP32) and
for every tile shape. A range launch on the full arrays writes no other row."""
import numpy as np
import pytest
import torch

import geomodel

pytestmark = pytest.mark.gpu

SLABS = [(0, 9), (9, 20), (20, 21), (21, 37)]  # uneven, one of a single row


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def case(prec, seed=3):
    geo = geomodel.random_small(seed, 70, 37, 11, sigma=1.2, seal_prob=0.05)
    g = geo.grid
    k3 = geomodel.k3_fields(geo.kx, seed + 1)
    diag = geomodel.diagonal_t(g, seed + 2)
    be = geomodel.be_fields(g, seed + 3)
    pref = None
    if prec == "fp64":
        from oracle import pressure
        p = pressure(geo)
        cast = lambda a: a  # noqa: E731
    else:
        from oracle import hydrostatic
        pref = hydrostatic(g, geo.fluid)
        p = geo.dp32(0)
        cast = lambda a: np.asarray(a, np.float32)  # noqa: E731
    fields = dict(p=cast(p), kx=cast(geo.kx), ky=cast(k3[1]), kz=cast(k3[2]),
                  tne=cast(diag[0]), tse=cast(diag[1]), phi=cast(be["phi"]),
                  p_prev=cast(p - be["dp_step"]) if prec == "fp64" else cast(p),
                  v=cast(be["v"]), seal=geo.seal)
    return geo, fields, pref, be


def run_all(gpu, geo, g, f, pref, be, rows=None, tile=None):
    """Every output of every mode for fields f on grid g, as host arrays."""
    d = {k: dev(v) for k, v in f.items()}
    kw = dict(seal=d["seal"], ry=geo.ry, rz=geo.rz, rows=rows, tile=tile,
              pref=None if pref is None else dev(pref))
    acc = dict(phi=d["phi"], p_prev=d["p_prev"], dt=be["dt"], cr=be["cr"])
    out = {}
    out["res"] = gpu.residual(g, geo.fluid, d["kx"], d["p"], **kw)  # shared faces in FP64
    out["resbe"] = gpu.residual_be(g, geo.fluid, d["kx"], d["p"], acc, **kw)
    out["r"], out["J"] = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], **kw)
    out["gp"], out["gm"] = gpu.residual_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], **kw)
    out["r10"] = gpu.residual10(g, geo.fluid, d["kx"], d["p"], d["tne"], d["tse"], **kw)
    out["rbe"], out["Jbe"] = gpu.jacobian_be(g, geo.fluid, d["kx"], d["p"], acc, **kw)
    out["jv"], _ = gpu.jvp(g, geo.fluid, d["kx"], d["p"], d["v"], accum=acc, **kw)
    out["rk3"], out["Jk3"] = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], ky=d["ky"], kz=d["kz"],
                                          **kw)
    out["gk3"] = gpu.residual_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], ky=d["ky"], kz=d["kz"],
                                  **kw)[1]
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def rows_of(a, y0, y1):
    """Rows [y0, y1) of an output (the y axis is the second from last)."""
    return a[..., y0:y1, :]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_slab_decomposition_equals_full_grid(gpu, prec):
    geo, f, pref, be = case(prec)
    g = geo.grid
    print(f"slab decomposition {prec}", flush=True)
    full = run_all(gpu, geo, g, f, pref, be)
    for y0, y1 in SLABS:
        lo, hi = max(y0 - 1, 0), min(y1 + 1, g.ny)
        gl = geomodel.Grid(g.nx, hi - lo, g.nz, dx=g.dx, dy=g.dy, dz=g.dz, gk=g.gk)
        local = {k: rows_of(v, lo, hi) for k, v in f.items()}
        got = run_all(gpu, geo, gl, local, pref, be, rows=(y0 - lo, y1 - lo))
        for k, v in got.items():
            want = rows_of(full[k], y0, y1)
            assert np.array_equal(rows_of(v, y0 - lo, y1 - lo), want), (prec, y0, y1, k)


@pytest.mark.parametrize("tile", range(10))
def test_row_range_in_place_every_tile(gpu, tile):
    """On the full arrays: the owned rows equal the full launch (same tile),
    every other row keeps its previous contents."""
    geo, f, pref, be = case("fp64", seed=7)
    g = geo.grid
    d = {k: dev(v) for k, v in f.items()}
    print(f"row range in place, tile {tile}", flush=True)
    r_full, J_full = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], ry=geo.ry,
                                  rz=geo.rz, tile=tile)
    for y0, y1 in SLABS:
        r = torch.full_like(r_full, float("nan"))
        J = torch.full_like(J_full, float("nan"))
        gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], ry=geo.ry, rz=geo.rz,
                     tile=tile, rows=(y0, y1), r_out=r, J_out=J)
        torch.cuda.synchronize()
        assert torch.equal(r[:, y0:y1], r_full[:, y0:y1]), (tile, y0, y1)
        assert torch.equal(J[:, :, y0:y1], J_full[:, :, y0:y1]), (tile, y0, y1)
        assert torch.isnan(r[:, :y0]).all() and torch.isnan(r[:, y1:]).all()
        assert torch.isnan(J[:, :, :y0]).all() and torch.isnan(J[:, :, y1:]).all()
