"""Launch-shape autotuner: picks the tile shape and the z-chunk length of the
march kernels per grid size class by timing the candidates on the GPU.

A size class groups grids whose (nx, ny, nz) round to the same buckets; one
representative per class is timed and the winner applies to the whole class.
Candidates whose lane utilisation (fraction of a tile's columns inside the
grid) is far below the best are skipped before timing. Results are returned
as {class: (tile, kz_chunk)} and can be cached in a JSON file.

Every tile and z-chunk computes each cell with the same arithmetic, so the
choice changes speed only, never results.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from . import api

TILE_IDS_256 = (0, 1, 2)          # the fixed tiles the ensemble kernels hold
FIT_TILE = 10                     # the ensemble kernels' tile fitted to each member
TILE_IDS_ALL = (0, 1, 2, 3, 4, 5)
KZ_CANDIDATES = (8, 16, 32, 64)


def size_class(nx: int, ny: int, nz: int) -> Tuple[int, int, int]:
    """Buckets of 16 cells in x and y, 32 planes in z."""
    return (int(math.ceil(nx / 16)), int(math.ceil(ny / 16)), int(math.ceil(nz / 32)))


def lane_utilisation(nx: int, ny: int, tile: int) -> float:
    """Share of a launch's threads that own a cell of the nx x ny plane."""
    if tile == FIT_TILE:
        tx, ty = api.fit_tile_shape(nx, ny)
        return nx * ny / (math.ceil(nx / tx) * math.ceil(ny / ty) * 256)
    tx, ty, th = api.tile_shapes()[tile]
    return nx * ny / (math.ceil(nx / tx) * math.ceil(ny / ty) * th)


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_member(m: dict, *, tiles: Sequence[int] = TILE_IDS_256,
                kz: Sequence[int] = KZ_CANDIDATES, mode: str = "jacobian", reps: int = 5,
                keep: float = 0.8) -> Tuple[int, int, float]:
    """Time every (tile, kz) candidate on one grid; returns (tile, kz, ms)."""
    g = m["grid"]
    util = {t: lane_utilisation(g.nx, g.ny, t) for t in tiles}
    best_u = max(util.values())
    cands = [(t, z) for t in tiles if util[t] >= keep * best_u for z in kz if z <= 2 * g.nz]
    p = m["p"]
    # outputs in the member's layout (its row pitch, or the sliced r + J array)
    sliced = mode == "jacobian" and m.get("sliced", False)
    ld = p.stride(-2) if g.ny > 1 else (p.stride(-3) if g.nz > 1 else g.nx)
    r = api.empty_pitched(g, p.dtype, p.device, (), ld)
    J = (api.empty_sliced(g, p.dtype, p.device) if sliced
         else api.empty_pitched(g, p.dtype, p.device, (7,), ld))
    best = None
    for t, z in cands:
        kw = dict(seal=m.get("seal"), pref=m.get("pref"), ry=m.get("ry", 1.0),
                  rz=m.get("rz", 1.0), tile=t, kz_chunk=z, pad_writes=m.get("pad_writes", False))
        if sliced:
            fn = lambda: api.jacobian(g, m["fluid"], m["kx"], p, J_out=J, sliced=True, **kw)  # noqa: E731
        elif mode == "jacobian":
            fn = lambda: api.jacobian(g, m["fluid"], m["kx"], p, r_out=r, J_out=J, **kw)  # noqa: E731
        else:
            fn = lambda: api.residual(g, m["fluid"], m["kx"], p, out=r, **kw)  # noqa: E731
        ms = _time(fn, reps)
        if best is None or ms < best[2]:
            best = (t, z, ms)
    return best


def tune_members(members: Sequence[dict], *, cache: Optional[str] = None, **kw
                 ) -> Dict[Tuple[int, int, int], Tuple[int, int]]:
    """Tune one representative per size class and assign ``tile`` and
    ``kz_chunk`` to every member in place. Returns the class table."""
    table: Dict[Tuple[int, int, int], Tuple[int, int]] = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            for k, v in json.load(f).items():
                table[tuple(int(x) for x in k.split(","))] = (int(v[0]), int(v[1]))
    reps: Dict[Tuple[int, int, int], dict] = {}
    for m in members:
        g = m["grid"]
        c = size_class(g.nx, g.ny, g.nz)
        if c not in table and c not in reps:
            reps[c] = m
    for c, m in reps.items():
        t, z, _ = tune_member(m, **kw)
        table[c] = (t, z)
    for m in members:
        g = m["grid"]
        m["tile"], m["kz_chunk"] = table[size_class(g.nx, g.ny, g.nz)]
    if cache:
        with open(cache, "w") as f:
            json.dump({",".join(map(str, k)): list(v) for k, v in sorted(table.items())}, f,
                      indent=1)
    return table


def ensemble_tile(nx: int, ny: int, tiles: Sequence[int] = (0, 1, FIT_TILE)) -> int:
    """The tile with the best lane utilisation among ``tiles``; ties go to the
    wider tile (longer contiguous rows per wave). 16-wide rows are left out by
    default: in FP32 they fill only half a 128-byte line per row."""
    best = None
    for t in tiles:
        u = lane_utilisation(nx, ny, t)
        if best is None or u > best[1] + 1e-12:
            best = (t, u)
    return best[0]


def balanced_kz(nz: int, most: int) -> int:
    """z chunk of a column of nz planes cut into the fewest chunks of at most
    ``most`` planes, of near-equal length (34 planes with most = 32: two
    chunks of 17 instead of 32 + 2; with most = 48: one of 34)."""
    chunks = -(-nz // most)
    return -(-nz // chunks)


def tune_ensemble(members: Sequence[dict], *, kz: Sequence[int] = (16, 32, 64),
                  tiles: Sequence[int] = TILE_IDS_256 + (FIT_TILE,),
                  schedules: Sequence[str] = ("persistent", "grouped"), reps: int = 5,
                  mode: str = "jacobian") -> Tuple[Tuple[str, int | str, str], Dict[str, float]]:
    """Chooses the launch shape of one ensemble launch by timing it: every
    uniform tile and a mixed assignment (per-model tile by lane utilisation),
    each with every uniform z chunk, per-model balanced chunks ('bal32',
    'bal48': see balanced_kz) and every schedule. Sets ``tile`` and
    ``kz_chunk`` on every member; returns ((assignment, kz, schedule),
    {label: ms})."""
    mixed = [ensemble_tile(m["grid"].nx, m["grid"].ny) for m in members]
    cands = [(f"tile{t}", [t] * len(members)) for t in tiles] + [("mixed", mixed)]
    # z chunks: uniform lengths, and per model balanced chunks of at most 32 or 48 planes
    zs = list(kz) + ["bal32", "bal48"]
    times, best = {}, None
    for label, assign in cands:
        for z in zs:
            for m, t in zip(members, assign):
                m["tile"] = t
                m["kz_chunk"] = (balanced_kz(m["grid"].nz, int(z[3:])) if isinstance(z, str)
                                 else z)
            ens = api.Ensemble(members, mode=mode)
            for sch in schedules:
                ens.set_schedule(sch)
                ms = _time(ens.run, reps)
                times[f"{label}/kz{z}/{sch}"] = ms
                if best is None or ms < best[0]:
                    best = (ms, label, assign, z, sch)
            ens.close()
            del ens
    _, label, assign, z, sch = best
    apply_ensemble_launch(members, (label, z, sch))
    return (label, z, sch), times


def apply_ensemble_launch(members: Sequence[dict], launch) -> None:
    """Sets ``tile`` and ``kz_chunk`` of every member from a launch returned by
    tune_ensemble: (assignment 'tile<t>' or 'mixed', z chunk or 'bal<n>',
    schedule)."""
    label, z = launch[0], launch[1]
    for m in members:
        nx, ny, nz = m["grid"].nx, m["grid"].ny, m["grid"].nz
        m["tile"] = ensemble_tile(nx, ny) if label == "mixed" else int(label[4:])
        m["kz_chunk"] = balanced_kz(nz, int(z[3:])) if isinstance(z, str) else int(z)
