"""TPFA_LAUNCH_PAD_WRITES: with row-pitched outputs the tile lanes that fall in
a row's padding (nx <= i < ldx) store zeros there, so that rows are written in
whole lines. The real cells stay bitwise those of the launch without the flag
(and of the contiguous launch) in every mode and precision; padding outside
the lanes of the last tile of a row, and rows outside a row-range launch, are
left untouched; the binding refuses an output whose buffer ends inside the
padding of its last row."""
import numpy as np
import pytest
import torch

import geomodel

from test_gpu_pitch import case, dev, pad, run_all

pytestmark = pytest.mark.gpu


def padded_out(shape, lead, ldx, dtype):
    """NaN-filled (lead..., nz, ny, ldx) buffer and its view [..., :nx]."""
    nz, ny, nx = shape
    buf = torch.full(tuple(lead) + (nz, ny, ldx), float("nan"), dtype=dtype, device="cuda")
    return buf, buf[..., :nx]


def check_padding(buf, nx, covered):
    """Columns [nx, covered) of every row are zeros; columns [covered, ldx) NaN."""
    pad_ = buf[..., nx:covered]
    assert bool((pad_ == 0).all()), "padding lanes did not store zeros"
    assert bool(torch.isnan(buf[..., covered:]).all()), "padding beyond the tile was written"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ldx", [96, 128])
def test_every_mode_real_cells_unchanged(gpu, prec, ldx):
    """nx = 70: every default tile (64 or 128 cells wide) covers [70, 128)."""
    geo, f, pref, be = case(prec)
    print(f"pad writes, every mode, {prec}, ldx {ldx}", flush=True)
    want = run_all(gpu, geo, f, pref, be, dev)
    got = run_all(gpu, geo, f, pref, be, lambda a: pad(a, ldx), pad_writes=True)
    nx = geo.grid.nx
    bad = []
    for k, w in want.items():
        v = got[k]
        assert v.stride(-2) == ldx, k
        if not torch.equal(v, w):
            bad.append(("real cells differ", k))
        # the whole padding of each row is zeros (the binding's buffers hold it)
        base = v.as_strided(tuple(v.shape[:-1]) + (ldx,), v.stride())
        if not bool((base[..., nx:] == 0).all()):
            bad.append(("padding not zero", k))
    assert not bad, (prec, ldx, bad)


@pytest.mark.parametrize("tile", range(10))
def test_every_tile_covers_its_lanes_only(gpu, tile):
    geo, f, pref, be = case("fp32", seed=9)
    g = geo.grid
    ldx = 96
    shapes = gpu.tile_shapes()
    tx = shapes[tile][0]
    covered = min(ldx, (g.nx + tx - 1) // tx * tx)
    d = {k: pad(v, ldx) for k, v in f.items()}
    pref_d = dev(pref)
    print(f"pad writes, tile {tile} ({tx} wide): padding [{g.nx}, {covered}) written", flush=True)
    rc, Jc = gpu.jacobian(g, geo.fluid, dev(f["kx"]), dev(f["p"]), seal=dev(f["seal"]),
                          pref=pref_d, ry=geo.ry, rz=geo.rz, tile=tile)
    rb, r = padded_out(g.shape, (), ldx, torch.float32)
    Jb, J = padded_out(g.shape, (7,), ldx, torch.float32)
    gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], pref=pref_d, ry=geo.ry,
                 rz=geo.rz, tile=tile, r_out=r, J_out=J, pad_writes=True)
    torch.cuda.synchronize()
    assert torch.equal(r, rc) and torch.equal(J, Jc), tile
    check_padding(rb, g.nx, covered)
    check_padding(Jb, g.nx, covered)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_row_range_leaves_other_rows(gpu, prec):
    geo, f, pref, be = case(prec, seed=13)
    g = geo.grid
    ldx, y0, y1 = 128, 5, 17
    dt = torch.float64 if prec == "fp64" else torch.float32
    d = {k: pad(v, ldx) for k, v in f.items()}
    pref_d = None if pref is None else dev(pref)
    print(f"pad writes with rows ({y0}, {y1}), {prec}", flush=True)
    rb, r = padded_out(g.shape, (), ldx, dt)
    Jb, J = padded_out(g.shape, (7,), ldx, dt)
    gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], pref=pref_d, ry=geo.ry,
                 rz=geo.rz, rows=(y0, y1), r_out=r, J_out=J, pad_writes=True)
    rc, Jc = gpu.jacobian(g, geo.fluid, dev(f["kx"]), dev(f["p"]), seal=dev(f["seal"]),
                          pref=pref_d, ry=geo.ry, rz=geo.rz)
    torch.cuda.synchronize()
    assert torch.equal(r[:, y0:y1], rc[:, y0:y1]) and torch.equal(J[:, :, y0:y1], Jc[:, :, y0:y1])
    for b in (rb, Jb):
        assert bool((b[..., y0:y1, g.nx:] == 0).all())
        assert bool(torch.isnan(b[..., :y0, :]).all()) and bool(torch.isnan(b[..., y1:, :]).all())


def test_ensemble_members(gpu, orc):
    """Ensemble members with and without the flag: identical real cells, zeros
    in the padding of the flagged members, both schedules."""
    members, tiles = [], (0, 1, 10, 2)  # 10: the fitted tile
    for m, (shape, ldx) in enumerate([((45, 20, 9), 64), ((70, 13, 6), 96), ((33, 31, 11), 64),
                                      ((50, 17, 7), 64)]):
        geo = geomodel.random_small(60 + m, *shape, sigma=1.0, seal_prob=0.03)
        pref = orc.hydrostatic(geo.grid, geo.fluid, geo.p_top)
        members.append(dict(grid=geo.grid, fluid=geo.fluid, kx=pad(geo.kx32(), ldx),
                            p=pad(geo.dp32(0), ldx), seal=pad(geo.seal, ldx), pref=dev(pref),
                            ry=geo.ry, rz=geo.rz, tile=tiles[m]))
    print("ensemble members with pad writes", flush=True)
    plain = gpu.Ensemble(members)
    flagged = gpu.Ensemble([dict(d, pad_writes=True) for d in members])
    for schedule in ("persistent", "grouped"):
        plain.set_schedule(schedule)
        flagged.set_schedule(schedule)
        plain.run()
        flagged.run()
        torch.cuda.synchronize()
        for q, d in enumerate(members):
            nx = d["grid"].nx
            assert torch.equal(plain.r[q], flagged.r[q]) and torch.equal(plain.J[q], flagged.J[q])
            for t in (flagged.r[q], flagged.J[q]):
                full = t.as_strided(tuple(t.shape[:-1]) + (t.stride(-2),), t.stride())
                g_ = d["grid"]
                tx = (gpu.fit_tile_shape(g_.nx, g_.ny)[0] if tiles[q] == 10
                      else gpu.tile_shapes()[tiles[q]][0])
                covered = min(t.stride(-2), (nx + tx - 1) // tx * tx)
                assert bool((full[..., nx:covered] == 0).all()), (schedule, q)
    plain.close()
    flagged.close()


def test_binding_refuses_short_buffers(gpu, orc):
    """A view [..., off:off+nx] of a buffer of pitch ldx whose last row's
    padding runs past the buffer is refused with pad_writes (and accepted
    without it)."""
    geo = geomodel.random_small(3, 40, 7, 5)
    g = geo.grid
    ldx, off = 64, 10
    kx, p, s = (pad(a, ldx, off) for a in (geo.kx, orc.pressure(geo), geo.seal))
    print("pad writes: short output buffer refused", flush=True)
    buf = torch.zeros((g.nz, g.ny, ldx), dtype=torch.float64, device="cuda")
    out = buf[..., off:off + g.nx]
    with pytest.raises(ValueError, match="pad_writes"):
        gpu.residual(g, geo.fluid, kx, p, seal=s, out=out, pad_writes=True)
    gpu.residual(g, geo.fluid, kx, p, seal=s, out=out)
    torch.cuda.synchronize()


def test_noalloc_run_with_pad_writes(gpu, orc):
    """tpfa_ensemble_run_noalloc passes the members' flag to the same kernels:
    its outputs equal the batch's, padding zeros included."""
    members, outs = [], []
    for m, (shape, ldx) in enumerate([((45, 20, 9), 64), ((70, 13, 6), 96)]):
        geo = geomodel.random_small(80 + m, *shape, sigma=1.0, seal_prob=0.03)
        pref = orc.hydrostatic(geo.grid, geo.fluid, geo.p_top)
        members.append(dict(grid=geo.grid, fluid=geo.fluid, kx=pad(geo.kx32(), ldx),
                            p=pad(geo.dp32(0), ldx), seal=pad(geo.seal, ldx), pref=dev(pref),
                            ry=geo.ry, rz=geo.rz, tile=0, pad_writes=True))
        outs.append((padded_out(geo.grid.shape, (), ldx, torch.float32),
                     padded_out(geo.grid.shape, (7,), ldx, torch.float32)))
    print("noalloc ensemble run with pad writes", flush=True)
    ens = gpu.Ensemble(members)
    ens.run()
    gpu.ensemble_run_noalloc(members, [(r[1], J[1]) for r, J in outs])
    torch.cuda.synchronize()
    for q, ((rb, r), (Jb, J)) in enumerate(outs):
        nx = members[q]["grid"].nx
        assert torch.equal(r, ens.r[q]) and torch.equal(J, ens.J[q]), q
        check_padding(rb, nx, rb.shape[-1])
        check_padding(Jb, nx, Jb.shape[-1])
    ens.close()
