"""Structured geomodels: spatially correlated ln k and planar fault / shale
barriers (seal bits on whole planes).

* Oracle pin: with complete barriers no flux crosses a sealed plane, so the
  residuals of every compartment the barriers cut off sum to zero (each
  compartment conserves mass on its own), while without the barriers they do
  not.
* GPU parity on the faulted geomodel: FP64 residual + Jacobian (1e-12), the
  FP32 precision form (1e-5) and the vector-Jacobian product, and the
  compartment invariant on the GPU's residual.
"""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_full, compare_vjp


def compartments(nx, ny, nz, xf, zb):
    """Boolean masks of the four compartments cut by the planes i = xf | xf+1
    and k = zb | zb+1."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    left, low = i <= xf, k <= zb
    return [left & low, left & ~low, ~left & low, ~left & ~low]


def sealed_model(seed=3, nx=17, ny=9, nz=12):
    g = geomodel.Grid(nx, ny, nz)
    geo = geomodel.draw("sealed", g, sigma=1.0, seed=seed, ry=1.0, rz=0.1)
    geo.logk = geomodel.correlated_logk(g, seed, corr_len=(3.0, 3.0, 1.0))
    geo.kx = np.exp(geo.logk)
    xf, zb = nx // 3, nz // 2
    geo.seal = geomodel.fault_seals(g, x_fault=xf, z_barrier=zb)
    return geo, xf, zb


def test_oracle_compartments_conserve_mass(orc):
    geo, xf, zb = sealed_model()
    p = orc.pressure(geo)
    out = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                       want=("r", "scale"))
    open_ = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz,
                         want=("r", "scale"))
    g = geo.grid
    crossing = 0.0
    for m in compartments(g.nx, g.ny, g.nz, xf, zb):
        tol = 16 * m.sum() * 1.2e-16 * out["scale"][0][m].sum()
        assert abs(out["r"][m].sum()) <= tol
        crossing = max(crossing, abs(open_["r"][m].sum()) / open_["scale"][0][m].sum())
    assert crossing > 1e-6  # without the barriers, flux does cross the planes


def test_correlated_field_statistics():
    g = geomodel.Grid(64, 48, 32)
    lk = geomodel.correlated_logk(g, 5, sigma=1.5, corr_len=(6.0, 6.0, 2.0))
    assert abs(lk.mean() - geomodel.LN_K_MEDIAN) < 0.5 and abs(lk.std() - 1.5) < 1e-9
    x = lk - lk.mean()
    cx = np.mean(x[:, :, :-1] * x[:, :, 1:]) / x.var()
    cz = np.mean(x[:-1] * x[1:]) / x.var()
    assert cx > 0.9 and 0.5 < cz < cx  # smooth along x, shorter correlation along z


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.gpu
def test_gpu_faulted_geomodel(gpu, orc):
    geo = geomodel.faulted()
    print("faulted geomodel", geo.grid, flush=True)
    p = orc.pressure(geo)
    r, J = gpu.jacobian(geo.grid, geo.fluid, dev(geo.kx), dev(p), seal=dev(geo.seal),
                        ry=geo.ry, rz=geo.rz)
    torch.cuda.synchronize()
    rep = compare_full(orc, geo.grid, geo.fluid, geo.kx, p, r.cpu().numpy(), J.cpu().numpy(),
                       tol=1e-12, tau=1e-9 * np.abs(p).max(), ry=geo.ry, rz=geo.rz,
                       seal=geo.seal)
    assert rep["max_err"] <= 1e-12, rep
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    dp, k32 = geo.dp32(0), geo.kx32()
    kw = dict(seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz)
    r32, J32 = gpu.jacobian(geo.grid, geo.fluid, dev(k32), dev(dp), **kw)
    w = np.random.default_rng(1).standard_normal(geo.grid.shape).astype(np.float32)
    gp, gm = gpu.residual_vjp(geo.grid, geo.fluid, dev(k32), dev(dp), dev(w), **kw)
    torch.cuda.synchronize()
    p_w, k_w = orc.widen_fp32(dp, pref), k32.astype(np.float64)
    rep = compare_full(orc, geo.grid, geo.fluid, k_w, p_w, r32.cpu().numpy(), J32.cpu().numpy(),
                       tol=1e-5, tau=1e-4, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert rep["max_err"] <= 1e-5, rep
    rep = compare_vjp(orc, geo.grid, geo.fluid, k_w, p_w, w.astype(np.float64),
                      gp.cpu().numpy(), gm.cpu().numpy(), tol=1e-5, tau=1e-4, ry=geo.ry,
                      rz=geo.rz, seal=geo.seal)
    assert rep["max_err"] <= 1e-5, rep


@pytest.mark.gpu
def test_gpu_compartments_conserve_mass(gpu, orc):
    geo, xf, zb = sealed_model(seed=9, nx=70, ny=9, nz=37)
    p = orc.pressure(geo)
    r = gpu.residual(geo.grid, geo.fluid, dev(geo.kx), dev(p), seal=dev(geo.seal),
                     ry=geo.ry, rz=geo.rz).cpu().numpy()
    scale = orc.evaluate(geo.grid, geo.fluid, geo.kx, p, ry=geo.ry, rz=geo.rz, seal=geo.seal,
                         want=("scale",))["scale"][0]
    g = geo.grid
    for m in compartments(g.nx, g.ny, g.nz, xf, zb):
        assert abs(r[m].sum()) <= 16 * m.sum() * 1.2e-16 * scale[m].sum()
