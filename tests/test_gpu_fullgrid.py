"""Every cell of the benchmark's 512 x 512 x 256 grid against the oracle, in
the launch the benchmark times (library defaults, r and J in the sliced
layout, which equals the plane layout bitwise): the FP64 residual + Jacobian
at 1e-12 and the FP32 precision form of the same geomodel (on its widened
inputs) at 1e-5, in the per-cell relative metric of tests/helpers.py.

The oracle evaluates z slabs of 32 planes plus one halo plane on each side
(the halo planes are inputs only: the slab's own planes see all six
neighbours), so the whole grid is compared in bounded memory.
"""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_full

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SLAB = 32


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def big(orc):
    geo = geomodel.big512(noise_seeds=(2,))
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    return geo, pref


def headline(gpu, geo, k, p, **kw):
    """r, J of the sliced launch copied out to planes, checked bitwise against
    the plane layout's."""
    g = geo.grid
    rp, Jp = gpu.jacobian(g, geo.fluid, k, p, seal=dev(geo.seal), ry=geo.ry, rz=geo.rz, **kw)
    _, Js = gpu.jacobian(g, geo.fluid, k, p, seal=dev(geo.seal), ry=geo.ry, rz=geo.rz,
                         sliced=True, **kw)
    r, J = gpu.unslice(g, Js)
    torch.cuda.synchronize()
    assert torch.equal(r, rp) and torch.equal(J, Jp), "sliced and plane layouts differ"
    return r, J


def slabwise(orc, geo, k, p, r, J, tol, tau):
    """compare_full over z slabs [k0, k1) with halo planes; r, J on the device."""
    g = geo.grid
    worst = {"max_err": 0.0, "n_tie_faces": 0, "n_flipped_cells": 0}
    for k0 in range(0, g.nz, SLAB):
        k1 = min(g.nz, k0 + SLAB)
        lo, hi = max(0, k0 - 1), min(g.nz, k1 + 1)
        gs = geomodel.Grid(g.nx, g.ny, hi - lo, dx=g.dx, dy=g.dy, dz=g.dz, gk=g.gk)
        # the GPU's result of the slab's planes, halo planes included; only the
        # slab's own planes are compared (the halo planes lack a neighbour here)
        rs = r[lo:hi].double().cpu().numpy()
        Js = J[:, lo:hi].double().cpu().numpy()
        own = np.zeros(gs.shape, bool)
        own[k0 - lo:k1 - lo] = True
        rep = compare_full(orc, gs, geo.fluid, k[lo:hi], p[lo:hi], rs, Js, tol=tol, tau=tau,
                           ry=geo.ry, rz=geo.rz, seal=geo.seal[lo:hi], mask=own)
        worst["max_err"] = max(worst["max_err"], rep["max_err"])
        worst["n_tie_faces"] += rep["n_tie_faces"]
        worst["n_flipped_cells"] += rep["n_flipped_cells"]
        print(f"planes {k0}..{k1 - 1}: {rep}", flush=True)
    return worst


def test_every_cell_fp64(gpu, orc, big):
    geo, pref = big
    print("512x512x256 fp64, every cell", flush=True)
    p = pref[:, None, None] + geo.noise[0]
    r, J = headline(gpu, geo, dev(geo.kx), dev(p))
    rep = slabwise(orc, geo, geo.kx, p, r, J, 1e-12, 1e-9 * float(np.abs(p).max()))
    print("fp64 every cell:", rep)
    assert rep["max_err"] <= 1e-12


def test_every_cell_fp32(gpu, orc, big):
    geo, pref = big
    print("512x512x256 fp32, every cell", flush=True)
    dp, k32 = geo.dp32(0), geo.kx32()
    r, J = headline(gpu, geo, dev(k32), dev(dp), pref=dev(pref))
    p_w = orc.widen_fp32(dp, pref)
    rep = slabwise(orc, geo, k32.astype(np.float64), p_w, r, J, 1e-5, 1e-4)
    print("fp32 every cell:", rep)
    assert rep["max_err"] <= 1e-5
