"""The library's default launch rules, read through tpfa_resolve_launch on the
host (no GPU): tile shape by mode, precision, rock form and row alignment; the
z chunk by mode and its re-chunking on small grids (the last round of
workgroups as full as possible); the XCD
band order by size, precision and form; row ranges; explicit launches taken as
given; argument errors."""
import ctypes as C
import math

import pytest
import torch

import geomodel
from paper_2304_11274_amd import _lib as L
from paper_2304_11274_amd import api

F64, F32 = torch.float64, torch.float32
G512 = geomodel.Grid(512, 512, 256)


def rl(grid, op, dtype=F64, **kw):
    return api.resolve_launch(grid, op, dtype, **kw)


def test_benchmark_launches():
    a = rl(G512, "jacobian")
    assert (a["shape"], a["threads"], a["kz_chunk"], a["xcd_remap"]) == ((64, 8), 512, 32, False)
    assert a["rows"] == (0, 512)
    b = rl(G512, "jacobian", F32)
    assert (b["shape"], b["kz_chunk"], b["xcd_remap"]) == ((64, 8), 32, True)
    assert rl(G512, "jacobian_be", F32)["kz_chunk"] == 16
    assert rl(G512, "residual")["shape"] == (64, 4)   # shared faces, more LDS
    assert rl(G512, "residual", F32)["shape"] == (64, 8)
    # the FP32 residual of the ratio form takes 64-plane chunks, the FP64 one 32
    # (a launch large enough that the small-grid re-chunking keeps the default)
    big_r = geomodel.Grid(512, 512, 2048)
    assert rl(big_r, "residual", F32)["kz_chunk"] == 64
    assert rl(big_r, "residual")["kz_chunk"] == 32
    for op in ("vjp", "jvp", "jvp_be"):
        r = rl(G512, op)
        assert (r["shape"], r["kz_chunk"], r["xcd_remap"]) == ((64, 4), 16, False), op
    k3 = rl(G512, "jacobian", form="k3")
    assert (k3["shape"], k3["kz_chunk"]) == ((64, 4), 32)   # 142 VGPRs: smaller workgroups
    assert rl(G512, "jacobian", F32, form="k3")["kz_chunk"] == 16


def test_rows_off_lines_and_row_pitch():
    g = geomodel.Grid(500, 500, 256)
    assert rl(g, "jacobian")["shape"] == (128, 4)          # halves the partial lines
    assert rl(g, "jacobian", ldx=512)["shape"] == (64, 8)  # pitched rows are on lines
    assert rl(g, "jacobian", F32)["shape"] == (64, 8)
    # 128-wide tiles would idle more lanes than 64-wide ones on 300-wide rows
    assert rl(geomodel.Grid(300, 700, 256), "jacobian")["shape"] == (64, 8)


def test_narrow_grids_and_the_10_flux_stencil():
    assert rl(geomodel.Grid(16, 40, 30), "jacobian")["shape"] == (16, 16)
    assert rl(geomodel.Grid(30, 40, 30), "jacobian")["shape"] == (32, 8)
    p10 = rl(geomodel.Grid(750, 994, 246), "residual10", F32)
    assert (p10["shape"], p10["kz_chunk"], p10["xcd_remap"]) == ((128, 4), 32, True)
    assert rl(geomodel.Grid(750, 994, 246), "residual10", F32, form="trans")["xcd_remap"] is False
    assert rl(geomodel.Grid(100, 100, 50), "residual10", F32)["shape"] == (64, 4)


def rounds_rule(grid, rows, shape, threads, default):
    """The documented chunk rule for small grids, with 8 waves per SIMD (what
    the library assumes where no device answers, as here): 256 CUs x 32 / waves
    per workgroup resident; the launch of the default chunk is kept when it
    fills the GPU four times over, otherwise L near-equal chunks maximise
    (T L / C) / ceil(T L / C) x kz / (kz + 2), L from nz / (2 default) to nz / 4."""
    tx, ty = shape
    tiles = -(-grid.nx // tx) * -(-rows // ty)
    cap = 256 * max(1, 32 // (threads // 64))
    nz = grid.nz
    if tiles * -(-nz // default) >= 4 * cap:
        return default
    best, best_kz = -1.0, default
    lo = max(1, -(-nz // (2 * default)))
    for L in range(lo, max(lo, -(-nz // 4)) + 1):
        k = -(-nz // L)
        chunks = -(-nz // k)
        rounds = tiles * chunks / cap
        score = rounds / math.ceil(rounds) * k / (k + 2)
        if score > best + 1e-9:
            best, best_kz = score, k
    return best_kz


@pytest.mark.parametrize("shape,op,dtype,default,kz", [
    ((256, 256, 128), "jacobian", F64, 32, 16),
    ((256, 256, 128), "vjp", F32, 16, 16),
    ((128, 128, 64), "residual", F32, 32, 4),
    ((128, 128, 64), "jacobian", F64, 32, 4),
    ((512, 512, 256), "jacobian", F64, 32, 32),
    ((300, 200, 90), "vjp", F32, 16, 12),
    ((64, 64, 200), "jacobian", F32, 32, 4),
])
def test_small_grids_get_round_filling_chunks(shape, op, dtype, default, kz):
    """Small grids: the chunk that fills the launch's last round best (the
    rule above, under the CPU's assumed occupancy); large grids keep the
    default."""
    g = geomodel.Grid(*shape)
    r = rl(g, op, dtype)
    assert r["kz_chunk"] == kz
    assert kz == rounds_rule(g, g.ny, r["shape"], r["threads"], default)


def test_band_order_by_size_precision_and_form():
    small = geomodel.Grid(256, 256, 128)        # 2^23 cells
    for op in ("residual", "jacobian", "vjp", "jvp", "residual_be", "jacobian_be"):
        for dt in (F64, F32):
            assert rl(small, op, dt)["xcd_remap"], (op, dt)
            assert rl(small, op, dt, form="k3")["xcd_remap"], (op, dt)
    assert not rl(small, "jacobian", form="trans")["xcd_remap"]
    big = geomodel.Grid(512, 512, 256)          # 2^26 cells
    assert not rl(big, "jacobian")["xcd_remap"] and not rl(big, "vjp", F32)["xcd_remap"]
    assert rl(big, "residual", F32)["xcd_remap"]
    # the rule counts the computed cells: one slab of 64 rows of the big grid is small
    slab = rl(geomodel.Grid(512, 66, 256), "jacobian", rows=(1, 65))
    assert slab["xcd_remap"] and slab["rows"] == (1, 65) and slab["kz_chunk"] == 16
    assert rl(geomodel.Grid(512, 4097, 16), "jacobian")["xcd_remap"] is False  # 2^25 cells


def test_explicit_launches_are_taken_as_given():
    r = rl(G512, "jacobian", F32, tile=0, kz_chunk=7)
    assert (r["tile"], r["kz_chunk"], r["xcd_remap"]) == (0, 7, False)
    r = rl(G512, "jacobian", tile=5, xcd_remap=True)
    assert (r["shape"], r["xcd_remap"], r["kz_chunk"]) == ((32, 16), True, 32)
    assert rl(geomodel.Grid(64, 64, 5), "jacobian", kz_chunk=64)["kz_chunk"] == 5  # at most nz


def test_pad_writes_flag_is_kept():
    """The caller's pad-writes bit survives the default launch's own flags."""
    g = geomodel.Grid(500, 64, 32)
    for tile, order in ((None, False), (0, False), (3, True)):
        r = rl(g, "jacobian", F32, tile=tile, xcd_remap=order, pad_writes=True, ldx=512)
        assert r["pad_writes"], (tile, order)
        assert not rl(g, "jacobian", F32, tile=tile, xcd_remap=order, ldx=512)["pad_writes"]
    assert api._launch(None, None, False, None, True).flags == L.TPFA_LAUNCH_PAD_WRITES
    assert api._launch(None, None, False) is None


def test_sliced_fp64_jacobian_defaults():
    """Sliced FP64 Jacobians on large grids: 128-plane chunks and the y-fast
    order where the tile rows are a multiple of 8; the plane layout keeps 32
    planes and the natural order. (1024 planes: a launch large enough that
    the small-grid re-chunking keeps the default with any residency.)"""
    s = rl(geomodel.Grid(512, 512, 1024), "jacobian", F64, sliced=True)
    assert (s["tile"], s["kz_chunk"], s["order"]) == (3, 128, "yfast"), s
    p = rl(G512, "jacobian", F64)
    assert (p["tile"], p["kz_chunk"], p["order"]) == (3, 32, "natural"), p
    odd = rl(geomodel.Grid(520, 500, 1024), "jacobian", F64, sliced=True)
    assert (odd["tile"], odd["kz_chunk"], odd["order"]) == (3, 128, "natural"), odd
    assert rl(G512, "jacobian", F32, sliced=True)["order"] == "bands"
    # the FP32 sliced Jacobian of the ratio form also takes 64-plane chunks,
    # its plane layout 32
    big32 = geomodel.Grid(512, 512, 512)
    assert rl(big32, "jacobian", F32, sliced=True)["kz_chunk"] == 64
    assert rl(big32, "jacobian", F32)["kz_chunk"] == 32
    assert rl(G512, "jacobian", F64, tile=3, sliced=True)["order"] == "natural"


def test_sliced_flag_is_kept():
    g = geomodel.Grid(500, 64, 32)
    for op in ("jacobian", "jacobian_be"):
        assert rl(g, op, F32, sliced=True)["sliced"]
        assert rl(g, op, F64, tile=3, sliced=True)["sliced"]
        assert not rl(g, op, F64)["sliced"]


def test_pad_writes_need_whole_last_rows():
    """The binding's host check: with pad_writes every output buffer must hold
    the padding of its last row (views at a column offset into a buffer of the
    same pitch do not)."""
    g = geomodel.Grid(40, 7, 5)
    lay = api._Layout(g)
    buf = torch.zeros((5, 7, 64))
    lay.take(buf[..., :40], "p")
    api._pad_ok(True, lay, out=buf[..., :40])
    api._pad_ok(False, lay, out=buf[..., 10:50])
    with pytest.raises(ValueError, match="pad_writes"):
        api._pad_ok(True, lay, out=buf[..., 10:50])
    J = torch.zeros((7, 5, 7, 64))
    api._pad_ok(True, lay, J_out=J[..., :40])
    with pytest.raises(ValueError, match="pad_writes"):
        api._pad_ok(True, lay, J_out=J[..., 10:50])


def test_errors():
    lib = L.load()
    g = api._grid(G512)
    rock = L.Rock(1, None, None, 1.0, 1.0, None)
    out = L.Launch()
    assert lib.tpfa_resolve_launch(C.byref(g), 8, L.TPFA_FP64, C.byref(rock), None,
                                   C.byref(out)) == L.TPFA_ERR_PARAM
    assert lib.tpfa_resolve_launch(C.byref(g), 1, 5, C.byref(rock), None,
                                   C.byref(out)) == L.TPFA_ERR_PARAM
    assert lib.tpfa_resolve_launch(C.byref(g), 1, L.TPFA_FP64, None, None,
                                   C.byref(out)) == L.TPFA_ERR_NULL
    assert lib.tpfa_resolve_launch(None, 1, L.TPFA_FP64, C.byref(rock), None,
                                   C.byref(out)) == L.TPFA_ERR_NULL
    bad_rows = L.Launch(-1, 0, 0, 3, 600)
    assert lib.tpfa_resolve_launch(C.byref(g), 1, L.TPFA_FP64, C.byref(rock), C.byref(bad_rows),
                                   C.byref(out)) == L.TPFA_ERR_PARAM
    bad_tile = L.Launch(10, 0, 0, 0, 0)
    assert lib.tpfa_resolve_launch(C.byref(g), 1, L.TPFA_FP64, C.byref(rock), C.byref(bad_tile),
                                   C.byref(out)) == L.TPFA_ERR_TILE
    g.ldx = 100
    assert lib.tpfa_resolve_launch(C.byref(g), 1, L.TPFA_FP64, C.byref(rock), None,
                                   C.byref(out)) == L.TPFA_ERR_SHAPE


@pytest.mark.parametrize("nz,most,want", [(34, 32, 17), (34, 48, 34), (128, 48, 43), (64, 32, 32),
                                          (1, 32, 1), (65, 32, 22), (96, 48, 48)])
def test_balanced_z_chunks(nz, most, want):
    """Per-model z chunks of the ensemble autotuner: the fewest chunks of at
    most `most` planes, of near-equal length, covering the column."""
    from paper_2304_11274_amd import autotune
    kz = autotune.balanced_kz(nz, most)
    assert kz == want and kz <= most
    chunks = -(-nz // kz)
    assert chunks == -(-nz // most) and (chunks - 1) * kz < nz <= chunks * kz


def test_fp32_chunks_hold_at_most_128_planes():
    """The FP32 kernels keep two constants per plane of their chunk in LDS, so
    an FP32 chunk runs as at most 128 planes; FP64 chunks are as given."""
    g = geomodel.Grid(64, 64, 300)
    assert rl(g, "jacobian", F32, tile=0, kz_chunk=200)["kz_chunk"] == 128
    assert rl(g, "vjp", F32, tile=0, kz_chunk=129)["kz_chunk"] == 128
    assert rl(g, "residual10", F32, tile=0, kz_chunk=128)["kz_chunk"] == 128
    assert rl(g, "jacobian", F64, tile=0, kz_chunk=200)["kz_chunk"] == 200
    assert rl(geomodel.Grid(64, 64, 90), "jacobian", F32, tile=0, kz_chunk=500)["kz_chunk"] == 90


@pytest.mark.parametrize("tile,want", [(6, L.TPFA_ERR_TILE), (7, L.TPFA_ERR_TILE),
                                       (3, L.TPFA_ERR_TILE), (9, L.TPFA_ERR_TILE)])
def test_batch_refuses_tiles_the_ensemble_kernels_do_not_hold(tile, want):
    """The ensemble kernels hold the tile bodies 0, 1, 2 only: any other
    explicit tile is refused on the host, before anything touches the device
    (the pointers below are never dereferenced)."""
    lib = L.load()
    g = geomodel.Grid(100, 40, 20)
    m = L.Model(api._grid(g), api._fluid(geomodel.Fluid()),
                L.Rock(16, None, None, 1.0, 0.1, None), L.State(16, None), 16, 16,
                L.Launch(tile, 0, 0, 0, 0))
    arr = (L.Model * 1)(m)
    h = C.c_void_p()
    assert lib.tpfa_batch_create(arr, 1, L.TPFA_FP64, 1, C.byref(h), None) == want
    assert not h.value
    assert b"tile 0, 1 or 2" in lib.tpfa_last_error()


def test_fitted_tile_shapes():
    """The ensemble's fitted tile: the fewest tiles of at most 64 cells per row,
    in near-equal parts of at least 8 cells; at most 256 cells and a halo ring
    one cell per thread covers; rows balanced."""
    from paper_2304_11274_amd import fit_tile_shape
    assert fit_tile_shape(100, 150) == (50, 5)
    assert fit_tile_shape(64, 64) == (64, 4)
    assert fit_tile_shape(200, 37) == (50, 5)
    assert fit_tile_shape(3, 10) == (8, 10)
    for nx in list(range(1, 300, 7)) + [256, 257, 512]:
        for rows in (1, 2, 7, 32, 33, 100, 255):
            tx, ty = fit_tile_shape(nx, rows)
            assert 8 <= tx <= 64 and 1 <= ty and tx * ty <= 256
            assert 2 * (tx + ty) + 4 <= 256
            assert -(-nx // tx) == max(1, -(-nx // 64)) or nx < 8
            assert ty <= rows or rows < 1
    lib = L.load()
    a, b = C.c_int(), C.c_int()
    assert lib.tpfa_fit_tile_shape(0, 5, C.byref(a), C.byref(b)) == L.TPFA_ERR_SHAPE
    assert lib.tpfa_fit_tile_shape(5, 5, None, C.byref(b)) == L.TPFA_ERR_NULL
