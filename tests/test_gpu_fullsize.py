"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (library defaults; autotuned tiles for the ensemble):

* 512 x 512 x 256 FP64 residual + Jacobian, and the FP32 precision form of the
  same geomodel: sampled cells (random, plus every domain face, edge and
  corner class) against the oracle evaluated cell by cell, and an invariant
  over the whole grid (the columns of J sum to zero);
* the same grid with per-direction permeability arrays (the benchmark's
  k_y, k_z recipe), FP64 and FP32, sampled cells against the oracle;
* its 500 x 500 x 256 crop (rows off 128-byte lines) in arrays of row pitch
  512, FP64 and FP32: bitwise equal to the contiguous launch, sampled cells
  against the oracle, the column-sum invariant;
* 256 x 256 x 128 FP32 residual and vector-Jacobian product against the full
  oracle evaluation;
* the 64-model uneven ensemble in one persistent launch: every model bitwise
  equal to its own single-grid launch, and sampled cells against the oracle.
"""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_full, compare_rows, compare_vjp

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL64, TOL32, TAU32 = 1e-12, 1e-5, 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def sample_cells(grid, n_random, seed):
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    rng = np.random.default_rng(seed)
    cells = [rng.integers(0, nx * ny * nz, n_random)]
    # every combination of low / interior / high position along each axis
    for i in (0, 1, nx // 2, nx - 2, nx - 1):
        for j in (0, 1, ny // 3, ny - 2, ny - 1):
            for k in (0, 1, nz // 2, nz - 2, nz - 1):
                cells.append(np.array([i + nx * (j + ny * k)]))
    # a full x row and a full y column on the bottom plane
    cells.append(np.arange(nx) + nx * (ny // 2))
    cells.append(nx // 2 + nx * np.arange(ny))
    return np.unique(np.concatenate(cells)).astype(np.int64)


def colsum_check(J, tol):
    """Columns of J sum to zero (sum_K r_K is identically zero) on the whole grid."""
    col = J[0].clone()
    col[:, :, 1:] += J[2][:, :, :-1]    # +x neighbour entries of cell i-1
    col[:, :, :-1] += J[1][:, :, 1:]    # -x neighbour entries of cell i+1
    col[:, 1:, :] += J[4][:, :-1, :]
    col[:, :-1, :] += J[3][:, 1:, :]
    col[1:, :, :] += J[6][:-1, :, :]
    col[:-1, :, :] += J[5][1:, :, :]
    scale = J.abs().sum(dim=0)
    bad = (col.abs() > tol * scale).sum().item()
    assert bad == 0, f"{bad} columns of J do not sum to zero"


@pytest.fixture(scope="module")
def big(orc):
    geo = geomodel.big512(noise_seeds=(2,))
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    return geo, pref


def test_fullsize_fp64_jacobian(gpu, orc, big):
    geo, pref = big
    print("512x512x256 fp64 jacobian", flush=True)
    p = pref[:, None, None] + geo.noise[0]
    r, J = gpu.jacobian(geo.grid, geo.fluid, dev(geo.kx), dev(p), seal=dev(geo.seal),
                        ry=geo.ry, rz=geo.rz)
    torch.cuda.synchronize()
    colsum_check(J, 1e-14)
    cells = sample_cells(geo.grid, 40000, 11)
    idx = torch.from_numpy(cells).cuda()
    r_s = r.view(-1)[idx].cpu().numpy()
    J_s = J.view(7, -1)[:, idx].cpu().numpy()
    del r, J
    rep = compare_rows(orc, geo.grid, geo.fluid, geo.kx, p, cells, r_s, J_s, tol=TOL64,
                       tau=1e-9 * np.abs(p).max(), ry=geo.ry, rz=geo.rz, seal=geo.seal)
    print("fp64 full size:", rep)
    assert rep["max_err"] <= TOL64


def test_fullsize_fp32_jacobian(gpu, orc, big):
    geo, pref = big
    print("512x512x256 fp32 jacobian", flush=True)
    dp, k32 = geo.dp32(0), geo.kx32()
    r, J = gpu.jacobian(geo.grid, geo.fluid, dev(k32), dev(dp), seal=dev(geo.seal),
                        pref=dev(pref), ry=geo.ry, rz=geo.rz)
    torch.cuda.synchronize()
    colsum_check(J.double(), 1e-6)
    cells = sample_cells(geo.grid, 40000, 12)
    idx = torch.from_numpy(cells).cuda()
    r_s = r.view(-1)[idx].double().cpu().numpy()
    J_s = J.view(7, -1)[:, idx].double().cpu().numpy()
    del r, J
    p_w = orc.widen_fp32(dp, pref)
    rep = compare_rows(orc, geo.grid, geo.fluid, k32.astype(np.float64), p_w, cells, r_s, J_s,
                       tol=TOL32, tau=TAU32, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    print("fp32 full size:", rep)
    assert rep["max_err"] <= TOL32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fullsize_per_direction_jacobian(gpu, orc, big, prec):
    geo, pref = big
    print(f"512x512x256 {prec} jacobian, per-direction k", flush=True)
    k3 = geomodel.k3_fields(geo.kx, 31)
    if prec == "fp64":
        p, ks, kw, tol = pref[:, None, None] + geo.noise[0], k3, {}, TOL64
        tau = 1e-9 * np.abs(p).max()
        p_dev = dev(p)
    else:
        dp = geo.dp32(0)
        ks = tuple(k.astype(np.float32) for k in k3)
        p, kw, tol, tau = orc.widen_fp32(dp, pref), dict(pref=dev(pref)), TOL32, TAU32
        p_dev = dev(dp)
    r, J = gpu.jacobian(geo.grid, geo.fluid, dev(ks[0]), p_dev, seal=dev(geo.seal),
                        ky=dev(ks[1]), kz=dev(ks[2]), **kw)
    torch.cuda.synchronize()
    colsum_check(J.double(), 1e-14 if prec == "fp64" else 1e-6)
    cells = sample_cells(geo.grid, 20000, 13 if prec == "fp64" else 14)
    idx = torch.from_numpy(cells).cuda()
    r_s = r.view(-1)[idx].double().cpu().numpy()
    J_s = J.view(7, -1)[:, idx].double().cpu().numpy()
    del r, J
    kw3 = tuple(k.astype(np.float64) for k in ks)
    rep = compare_rows(orc, geo.grid, geo.fluid, kw3[0], p, cells, r_s, J_s, tol=tol, tau=tau,
                       ry=1.0, rz=1.0, seal=geo.seal, ky=kw3[1], kz=kw3[2])
    print(f"{prec} per-direction full size:", rep)
    assert rep["max_err"] <= tol


def _pitched(a, ld):
    """Device copy of a (..., nz, ny, nx) array as a view of a buffer with row pitch ld."""
    t = dev(a)
    buf = torch.zeros(tuple(t.shape[:-1]) + (ld,), dtype=t.dtype, device=t.device)
    buf[..., :t.shape[-1]].copy_(t)
    return buf[..., :t.shape[-1]]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fullsize_pitched_jacobian(gpu, orc, big, prec):
    geo, pref = big
    nxp, nyp, ld = 500, 500, 512
    g = geomodel.Grid(nxp, nyp, geo.grid.nz, dx=geo.grid.dx, dy=geo.grid.dy, dz=geo.grid.dz,
                      gk=geo.grid.gk)
    print(f"500x500x256 {prec} jacobian, row pitch 512", flush=True)
    crop = lambda a: np.ascontiguousarray(a[:, :nyp, :nxp])  # noqa: E731
    seal = crop(geo.seal)
    if prec == "fp64":
        kx, p = crop(geo.kx), crop(pref[:, None, None] + geo.noise[0])
        p_dev, kw, tol, tau, pw, kwide = p, {}, TOL64, 1e-9 * np.abs(p).max(), p, kx
    else:
        kx, dp = crop(geo.kx32()), crop(geo.dp32(0))
        p_dev, kw, tol, tau = dp, dict(pref=dev(pref)), TOL32, TAU32
        pw, kwide = orc.widen_fp32(dp, pref), kx.astype(np.float64)
    r, J = gpu.jacobian(g, geo.fluid, _pitched(kx, ld), _pitched(p_dev, ld),
                        seal=_pitched(seal, ld), ry=geo.ry, rz=geo.rz, **kw)
    rc, Jc = gpu.jacobian(g, geo.fluid, dev(kx), dev(p_dev), seal=dev(seal), ry=geo.ry,
                          rz=geo.rz, **kw)
    torch.cuda.synchronize()
    assert r.stride(-2) == ld and J.stride(-2) == ld
    assert torch.equal(r, rc) and torch.equal(J, Jc)
    del rc, Jc
    colsum_check(J.double(), 1e-14 if prec == "fp64" else 1e-6)
    cells = sample_cells(g, 20000, 15 if prec == "fp64" else 16)
    kk, rem = np.divmod(cells, nxp * nyp)
    jj, ii = np.divmod(rem, nxp)
    ix = [torch.from_numpy(a).cuda() for a in (kk, jj, ii)]
    r_s = r[ix[0], ix[1], ix[2]].double().cpu().numpy()
    J_s = J[:, ix[0], ix[1], ix[2]].double().cpu().numpy()
    del r, J
    rep = compare_rows(orc, g, geo.fluid, kwide, pw, cells, r_s, J_s, tol=tol, tau=tau,
                       ry=geo.ry, rz=geo.rz, seal=seal)
    print(f"{prec} pitched full size:", rep)
    assert rep["max_err"] <= tol


def test_fullsize_adjoint(gpu, orc):
    geo = geomodel.adjoint256(n_sets=1)
    print("256x256x128 fp32 residual + vjp", flush=True)
    pref = orc.hydrostatic(geo.grid, geo.fluid)
    dp, k32 = geo.dp32(0), geo.kx32()
    w32 = geo.extra["w"][0].astype(np.float32)
    kw = dict(seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz)
    r = gpu.residual(geo.grid, geo.fluid, dev(k32), dev(dp), **kw)
    gp, gm = gpu.residual_vjp(geo.grid, geo.fluid, dev(k32), dev(dp), dev(w32), **kw)
    torch.cuda.synchronize()
    p_w = orc.widen_fp32(dp, pref)
    k_w = k32.astype(np.float64)
    rep = compare_full(orc, geo.grid, geo.fluid, k_w, p_w, r.cpu().numpy(), None, tol=TOL32,
                       tau=TAU32, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    print("adjoint forward:", rep)
    assert rep["max_err"] <= TOL32
    rep = compare_vjp(orc, geo.grid, geo.fluid, k_w, p_w, w32.astype(np.float64),
                      gp.cpu().numpy(), gm.cpu().numpy(), tol=TOL32, tau=TAU32, ry=geo.ry,
                      rz=geo.rz, seal=geo.seal)
    print("adjoint vjp:", rep)
    assert rep["max_err"] <= TOL32
    # the same workload in one pass (tpfa_residual_and_vjp, the bench's one_pass leg):
    # bitwise the two calls' results, so the comparisons above cover it
    r1, gp1, gm1 = gpu.residual_and_vjp(geo.grid, geo.fluid, dev(k32), dev(dp), dev(w32), **kw)
    torch.cuda.synchronize()
    assert torch.equal(r1, r) and torch.equal(gp1, gp) and torch.equal(gm1, gm)


def test_fullsize_ensemble(gpu, orc):
    from paper_2304_11274_amd import autotune
    models = geomodel.ensemble()
    print(f"ensemble of {len(models)} models", flush=True)
    members, prefs = [], []
    for geo in models:
        pref = orc.hydrostatic(geo.grid, geo.fluid)
        prefs.append(pref)
        members.append(dict(grid=geo.grid, fluid=geo.fluid, kx=dev(geo.kx32()), p=dev(geo.dp32()),
                            seal=dev(geo.seal), pref=dev(pref), ry=geo.ry, rz=geo.rz))
    (_, _, schedule), _ = autotune.tune_ensemble(members, reps=2)
    ens = gpu.Ensemble(members)
    ens.set_schedule(schedule)
    ens.run()
    torch.cuda.synchronize()
    for q, (m, geo) in enumerate(zip(members, models)):
        # the fitted tile (10) is for ensemble members only; results never depend on the tile
        r, J = gpu.jacobian(m["grid"], m["fluid"], m["kx"], m["p"], seal=m["seal"],
                            pref=m["pref"], ry=m["ry"], rz=m["rz"],
                            tile=None if m["tile"] == 10 else m["tile"],
                            kz_chunk=m["kz_chunk"])
        torch.cuda.synchronize()
        assert torch.equal(ens.r[q], r) and torch.equal(ens.J[q], J), q
        cells = sample_cells(geo.grid, 300, 100 + q)
        idx = torch.from_numpy(cells).cuda()
        r_s = ens.r[q].view(-1)[idx].double().cpu().numpy()
        J_s = ens.J[q].view(7, -1)[:, idx].double().cpu().numpy()
        p_w = orc.widen_fp32(geo.dp32(), prefs[q])
        rep = compare_rows(orc, geo.grid, geo.fluid, geo.kx32().astype(np.float64), p_w, cells,
                           r_s, J_s, tol=TOL32, tau=TAU32, ry=geo.ry, rz=geo.rz, seal=geo.seal)
        assert rep["max_err"] <= TOL32, (q, rep)
    ens.close()
