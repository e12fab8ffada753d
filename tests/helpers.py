"""Test-side utilities: neighbour shifts, sparse Jacobians built from the seven
planes, the per-cell relative error metric and the upwind-tie tolerant check.

Plane order everywhere: [diag, -x, +x, -y, +y, -z, +z]; plane 1 + n holds
dr_K / dp_L for neighbour n of K. Arrays have shape (nz, ny, nx).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# neighbour n -> (numpy axis, side)
NB = [(2, -1), (2, +1), (1, -1), (1, +1), (0, -1), (0, +1)]


def shift(v: np.ndarray, n: int) -> np.ndarray:
    """u[K] = v[neighbour n of K], 0 where that neighbour does not exist."""
    ax, side = NB[n]
    u = np.zeros_like(v)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if side > 0:
        dst[ax] = slice(0, -1)
        src[ax] = slice(1, None)
    else:
        dst[ax] = slice(1, None)
        src[ax] = slice(0, -1)
    u[tuple(dst)] = v[tuple(src)]
    return u


def unshift(v: np.ndarray, n: int) -> np.ndarray:
    """Adjoint of shift(., n): u[L] = v[K] where L is neighbour n of K."""
    return shift(v, n ^ 1)  # the opposite neighbour


def apply_J(J: np.ndarray, v: np.ndarray) -> np.ndarray:
    out = J[0] * v
    for n in range(6):
        out = out + J[1 + n] * shift(v, n)
    return out


def apply_JT(J: np.ndarray, w: np.ndarray) -> np.ndarray:
    out = J[0] * w
    for n in range(6):
        out = out + unshift(J[1 + n] * w, n)
    return out


def sparse_J(J: np.ndarray) -> sp.csr_matrix:
    nz, ny, nx = J.shape[1:]
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [J[0].ravel()]
    for n in range(6):
        nb = shift(idx.astype(np.float64) + 1.0, n) - 1.0  # -1 where absent
        m = nb.ravel() >= 0
        rows.append(idx.ravel()[m])
        cols.append(nb.ravel()[m].astype(np.int64))
        vals.append(J[1 + n].ravel()[m])
        # an absent neighbour must carry an exact zero entry
        assert np.all(J[1 + n].ravel()[~m] == 0.0)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def face_neighbour_exists(shape, n: int) -> np.ndarray:
    ones = np.ones(shape)
    return shift(ones, n) > 0


# ---------------------------------------------------------------------------
# Per-cell relative error. A residual can vanish while its faces carry large
# fluxes, so r_K is compared against the flux scale s_K = sum_L |F_KL| and the
# diagonal against sum_L |dF_KL / dp_K|; an off-diagonal entry is a single
# face derivative and is compared against itself. Entries whose scale is 0
# must match exactly.
# ---------------------------------------------------------------------------

def rel_err(got: np.ndarray, ref: np.ndarray, scale: np.ndarray) -> np.ndarray:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.asarray(scale, np.float64)
    d = np.abs(got - ref)
    out = np.zeros_like(d)
    pos = scale > 0
    out[pos] = d[pos] / scale[pos]
    out[~pos] = np.where(d[~pos] == 0.0, 0.0, np.inf)
    return out


def errors_rJ(r, J, r_ref, J_ref, scale) -> dict:
    """Max per-cell relative errors of r, the diagonal and the off-diagonals."""
    e = {"r": float(rel_err(r, r_ref, scale[0]).max()) if r is not None else 0.0}
    if J is not None:
        e["diag"] = float(rel_err(J[0], J_ref[0], scale[1]).max())
        e["off"] = float(max(rel_err(J[1 + n], J_ref[1 + n], np.abs(J_ref[1 + n])).max()
                             for n in range(6)))
    return e


def cell_errors(r, J, r_ref, J_ref, scale) -> np.ndarray:
    """Per-cell max of the three relative errors (shape of r)."""
    e = rel_err(r, r_ref, scale[0])
    if J is not None:
        e = np.maximum(e, rel_err(J[0], J_ref[0], scale[1]))
        for n in range(6):
            e = np.maximum(e, rel_err(J[1 + n], J_ref[1 + n], np.abs(J_ref[1 + n])))
    return e


def tie_faces(dphi: np.ndarray, tau) -> np.ndarray:
    """Boolean [3, ...]: faces whose potential difference lies within tau of 0."""
    with np.errstate(invalid="ignore"):
        return np.abs(dphi) <= tau


def cells_touching(faces: np.ndarray) -> np.ndarray:
    """Cells adjacent to any marked face (faces indexed by their lower cell)."""
    # face (c, c + e_a) touches c and c + e_a; shift by the -a neighbour
    touch = faces[0] | faces[1] | faces[2]
    touch = touch | shift(faces[0].astype(np.float64), 0).astype(bool)
    touch = touch | shift(faces[1].astype(np.float64), 2).astype(bool)
    touch = touch | shift(faces[2].astype(np.float64), 4).astype(bool)
    return touch
