"""TPFA_LAUNCH_SLICED: r and J written into one array of 64-cell row slices
(8 runs of 64 values per slice: r, then the seven Jacobian planes). Unsliced,
every value is bitwise that of the plane layout, for every tile, precision,
rock form, the backward-Euler Jacobian, pitched inputs, row ranges and the
ensemble; the lanes of a row's last slice beyond nx hold zeros, rows outside
a row range stay untouched, and the sliced FP64 / FP32 results meet the
oracle bound directly."""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_full
from test_gpu_pitch import TAU32, TOL32, TOL64, case, dev, pad

pytestmark = pytest.mark.gpu


def nan_sliced(gpu, g, dtype):
    return torch.full(gpu.sliced_shape(g), float("nan"), dtype=dtype, device="cuda")


def check_whole(gpu, g, Js, rows=None):
    """Every value of the computed rows is finite, the lanes beyond nx zero;
    rows outside [y0, y1) still NaN."""
    nz, ny, S = gpu.sliced_shape(g)[:3]
    y0, y1 = (0, ny) if rows is None else rows
    flat = Js.permute(0, 1, 3, 2, 4).reshape(nz, ny, 8, S * 64)
    inside = flat[:, y0:y1]
    assert bool(torch.isfinite(inside).all()), "a computed slice was not written whole"
    assert bool((inside[..., g.nx:] == 0).all()), "lanes beyond nx are not zero"
    assert bool(torch.isnan(flat[:, :y0]).all()) and bool(torch.isnan(flat[:, y1:]).all()), \
        "rows outside the row range were written"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tile", range(10))
def test_every_tile_bitwise_equal_to_planes(gpu, prec, tile):
    """nx = 70 (two slices, the second one six cells deep) on every tile."""
    geo, f, pref, be = case(prec, seed=31)
    g = geo.grid
    d = {k: dev(v) for k, v in f.items()}
    dt = d["p"].dtype
    kw = dict(seal=d["seal"], ry=geo.ry, rz=geo.rz, tile=tile,
              pref=None if pref is None else dev(pref))
    print(f"sliced r + J, {prec}, tile {tile}", flush=True)
    r, J = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], **kw)
    Js = nan_sliced(gpu, g, dt)
    none, out = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], J_out=Js, sliced=True, **kw)
    torch.cuda.synchronize()
    assert none is None and out is Js
    rs, Jp = gpu.unslice(g, Js)
    assert torch.equal(rs, r) and torch.equal(Jp, J), (prec, tile)
    check_whole(gpu, g, Js)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_other_forms_and_backward_euler(gpu, prec):
    """Per-direction permeability, given transmissibilities and the
    backward-Euler Jacobian, on pitched inputs (ldx 96): sliced = planes."""
    geo, f, pref, be = case(prec, seed=33)
    g = geo.grid
    d = {k: pad(v, 96) for k, v in f.items()}
    dt = d["p"].dtype
    pr = None if pref is None else dev(pref)
    acc = dict(phi=d["phi"], p_prev=d["p_prev"], dt=be["dt"], cr=be["cr"])
    tr = (d["tx"], d["ty"], d["tz"])
    print(f"sliced r + J, other forms, {prec}", flush=True)
    calls = {
        "k3": lambda **o: gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], pref=pr,
                                      ky=d["ky"], kz=d["kz"], **o),
        "trans": lambda **o: gpu.jacobian(g, geo.fluid, None, d["p"], pref=pr, trans=tr, **o),
        "be": lambda **o: gpu.jacobian_be(g, geo.fluid, d["kx"], d["p"], acc, seal=d["seal"],
                                          pref=pr, ry=geo.ry, rz=geo.rz, **o),
    }
    for name, call in calls.items():
        r, J = call()
        Js = nan_sliced(gpu, g, dt)
        call(J_out=Js, sliced=True)
        torch.cuda.synchronize()
        rs, Jp = gpu.unslice(g, Js)
        assert torch.equal(rs, r) and torch.equal(Jp, J), (prec, name)
        check_whole(gpu, g, Js)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_row_range(gpu, prec):
    geo, f, pref, be = case(prec, seed=35)
    g = geo.grid
    d = {k: dev(v) for k, v in f.items()}
    kw = dict(seal=d["seal"], ry=geo.ry, rz=geo.rz, pref=None if pref is None else dev(pref))
    y0, y1 = 4, 15
    print(f"sliced r + J, rows ({y0}, {y1}), {prec}", flush=True)
    r, J = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], **kw)
    Js = nan_sliced(gpu, g, d["p"].dtype)
    gpu.jacobian(g, geo.fluid, d["kx"], d["p"], J_out=Js, sliced=True, rows=(y0, y1), **kw)
    torch.cuda.synchronize()
    check_whole(gpu, g, Js, (y0, y1))
    rs, Jp = gpu.unslice(g, Js)
    assert torch.equal(rs[:, y0:y1], r[:, y0:y1]) and torch.equal(Jp[:, :, y0:y1], J[:, :, y0:y1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sliced_against_oracle(gpu, orc, prec):
    """Direct parity of the sliced launch with the FP64 oracle (R16 bound) on
    a grid of three slices per row, the last one ragged (nx = 161)."""
    geo = geomodel.random_small(37, 161, 29, 11, sigma=1.5, seal_prob=0.02, ry=1.0, rz=0.1)
    g = geo.grid
    print(f"sliced jacobian vs oracle {prec}", flush=True)
    if prec == "fp64":
        p = orc.pressure(geo)
        _, Js = gpu.jacobian(g, geo.fluid, dev(geo.kx), dev(p), seal=dev(geo.seal), ry=geo.ry,
                             rz=geo.rz, sliced=True)
        kx, pw, tol, tau = geo.kx, p, TOL64, 1e-9 * np.abs(p).max()
    else:
        pref = orc.hydrostatic(g, geo.fluid, geo.p_top)
        dp, k32 = geo.dp32(), geo.kx32()
        _, Js = gpu.jacobian(g, geo.fluid, dev(k32), dev(dp), seal=dev(geo.seal),
                             pref=dev(pref), ry=geo.ry, rz=geo.rz, sliced=True)
        kx, pw, tol, tau = k32.astype(np.float64), orc.widen_fp32(dp, pref), TOL32, TAU32
    torch.cuda.synchronize()
    r, J = gpu.unslice(g, Js)
    rep = compare_full(orc, g, geo.fluid, kx, pw, r.cpu().numpy(), J.cpu().numpy(), tol=tol,
                       tau=tau, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert rep["max_err"] <= tol, rep


def test_ensemble_and_noalloc_members(gpu, orc):
    """Sliced members beside plane members in one ensemble (both schedules)
    and in the no-alloc run: every sliced member equals its single launch."""
    members = []
    for m, (shape, tile) in enumerate([((45, 20, 9), 0), ((130, 13, 6), 0), ((33, 31, 11), 1),
                                       ((64, 17, 7), 10)]):
        geo = geomodel.random_small(90 + m, *shape, sigma=1.0, seal_prob=0.03)
        pref = orc.hydrostatic(geo.grid, geo.fluid, geo.p_top)
        members.append(dict(grid=geo.grid, fluid=geo.fluid, kx=dev(geo.kx32()),
                            p=dev(geo.dp32(0)), seal=dev(geo.seal), pref=dev(pref),
                            ry=geo.ry, rz=geo.rz, tile=tile, sliced=m != 2))
    print("ensemble with sliced members", flush=True)
    want = []
    for d in members:
        kw = dict(seal=d["seal"], pref=d["pref"], ry=d["ry"], rz=d["rz"])
        want.append(gpu.jacobian(d["grid"], d["fluid"], d["kx"], d["p"], **kw))
    ens = gpu.Ensemble(members)
    for schedule in ("persistent", "grouped"):
        ens.set_schedule(schedule)
        for q in range(len(members)):
            if ens.J[q] is not None:
                ens.J[q].fill_(float("nan"))
        ens.run()
        torch.cuda.synchronize()
        for q, d in enumerate(members):
            r, J = want[q]
            if d["sliced"]:
                assert ens.r[q] is None
                check_whole(gpu, d["grid"], ens.J[q])
                rs, Jp = gpu.unslice(d["grid"], ens.J[q])
            else:
                rs, Jp = ens.r[q], ens.J[q]
            assert torch.equal(rs, r) and torch.equal(Jp, J), (schedule, q)
    outs = [(None, nan_sliced(gpu, d["grid"], torch.float32)) if d["sliced"] else
            (torch.empty_like(ens.r[q]), torch.empty_like(ens.J[q]))
            for q, d in enumerate(members)]
    gpu.ensemble_run_noalloc(members, outs)
    torch.cuda.synchronize()
    for q, d in enumerate(members):
        r, J = want[q]
        rs, Jp = gpu.unslice(d["grid"], outs[q][1]) if d["sliced"] else outs[q]
        assert torch.equal(rs, r) and torch.equal(Jp, J), ("noalloc", q)
    ens.close()


def test_binding_checks(gpu):
    geo = geomodel.random_small(3, 40, 7, 5)
    g = geo.grid
    kx, p = dev(geo.kx), dev(np.full(g.shape, 1e7))
    print("sliced binding checks", flush=True)
    with pytest.raises(ValueError, match="sliced"):
        gpu.jacobian(g, geo.fluid, kx, p, sliced=True, r_out=torch.empty_like(p))
    with pytest.raises(ValueError, match="elements"):
        gpu.jacobian(g, geo.fluid, kx, p, sliced=True,
                     J_out=torch.empty((7,) + tuple(p.shape), dtype=p.dtype, device="cuda"))
    assert gpu.resolve_launch(g, "jacobian", sliced=True)["sliced"]
