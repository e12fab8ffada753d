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


# ---------------------------------------------------------------------------
# GPU-vs-oracle comparison with upwind ties. Where a face's potential
# difference is within tau of 0, either upwind choice is a correct result;
# a cell that disagrees must touch such a face and must then agree with the
# oracle evaluated with the upwind choice of those faces flipped.
# ---------------------------------------------------------------------------

def _flip_force(dphi_faces, ties):
    force = np.zeros(dphi_faces.shape, np.int8)
    force[ties] = np.where(dphi_faces[ties] >= 0, -1, 1)  # the rule's opposite
    return force


def compare_full(orc, grid, fluid, kx, p, r_gpu, J_gpu, *, tol, tau, ry, rz, seal, ky=None,
                 kz=None, mask=None):
    """Full-grid comparison of r (and J if given); ky, kz: per-direction
    permeability arrays (then ry, rz are not used); only cells where ``mask``
    is set are compared, if given. Returns a report dict."""
    want = ("r", "J", "scale", "dphi")
    ref = orc.evaluate(grid, fluid, kx, p, ry=ry, rz=rz, seal=seal, ky=ky, kz=kz, want=want)
    r_gpu = None if r_gpu is None else np.asarray(r_gpu, np.float64).reshape(ref["r"].shape)
    J_gpu = None if J_gpu is None else np.asarray(J_gpu, np.float64).reshape(ref["J"].shape)
    err = _errs(r_gpu, J_gpu, ref)
    if mask is not None:
        err = np.where(mask, err, 0.0)
    ties = tie_faces(ref["dphi"], tau)
    rep = {"max_err": float(err.max()), "n_tie_faces": int(ties.sum()), "n_flipped_cells": 0}
    bad = err > tol
    if bad.any():
        touch = cells_touching(ties)
        assert not (bad & ~touch).any(), (
            f"{int((bad & ~touch).sum())} cells differ by up to {err[bad & ~touch].max():.3e} "
            "away from any upwind tie")
        alt = orc.evaluate(grid, fluid, kx, p, ry=ry, rz=rz, seal=seal, ky=ky, kz=kz,
                           force=_flip_force(ref["dphi"], ties), want=("r", "J", "scale"))
        err2 = _errs(r_gpu, J_gpu, alt)
        if mask is not None:
            err2 = np.where(mask, err2, 0.0)
        still = bad & (err2 > tol)
        assert not still.any(), f"{int(still.sum())} tie cells match neither upwind choice"
        rep["n_flipped_cells"] = int(bad.sum())
        rep["max_err"] = float(np.where(bad, err2, err).max())
    return rep


def _errs(r_gpu, J_gpu, ref):
    e = np.zeros(ref["r"].shape)
    if r_gpu is not None:
        e = np.maximum(e, rel_err(r_gpu, ref["r"], ref["scale"][0]))
    if J_gpu is not None:
        e = np.maximum(e, rel_err(J_gpu[0], ref["J"][0], ref["scale"][1]))
        for n in range(6):
            e = np.maximum(e, rel_err(J_gpu[1 + n], ref["J"][1 + n], np.abs(ref["J"][1 + n])))
    return e


def _row_errs(r_gpu, J_gpu, r, J, s):
    e = rel_err(r_gpu, r, s[0]) if r_gpu is not None else np.zeros(r.shape)
    if J_gpu is not None:
        e = np.maximum(e, rel_err(J_gpu[0], J[0], s[1]))
        for n in range(6):
            e = np.maximum(e, rel_err(J_gpu[1 + n], J[1 + n], np.abs(J[1 + n])))
    return e


def compare_rows(orc, grid, fluid, kx, p, cells, r_rows, J_rows, *, tol, tau, ry, rz, seal,
                 ky=None, kz=None):
    """Comparison of sampled cells (r_rows[n], J_rows[7, n] from the GPU); ky,
    kz: per-direction permeability arrays."""
    r, J, s, d = orc.rows(grid, fluid, kx, p, cells, ry=ry, rz=rz, seal=seal, ky=ky, kz=kz,
                          with_dphi=True)
    err = _row_errs(r_rows, J_rows, r, J, s)
    with np.errstate(invalid="ignore"):
        tie = np.abs(d) <= tau  # [6, n]
    rep = {"max_err": float(err.max()), "n_tie_faces": int(tie.sum()), "n_flipped_cells": 0}
    bad = err > tol
    if bad.any():
        assert tie[:, bad].any(axis=0).all(), (
            f"{int((bad & ~tie.any(axis=0)).sum())} sampled cells differ by up to "
            f"{err[bad & ~tie.any(axis=0)].max():.3e} away from any upwind tie")
        shape = (grid.nz, grid.ny, grid.nx)
        N = int(np.prod(shape))
        force = np.zeros((3, N), np.int8)
        strides = (1, grid.nx, grid.nx * grid.ny)
        for q in np.nonzero(bad)[0]:
            for n in np.nonzero(tie[:, q])[0]:
                axis, plus = n // 2, n % 2
                lower = cells[q] if plus else cells[q] - strides[axis]
                dlow = d[n, q] if plus else -d[n, q]  # potential seen from the lower cell
                force[axis, lower] = -1 if dlow >= 0 else 1
        r2, J2, s2 = orc.rows(grid, fluid, kx, p, cells[bad], ry=ry, rz=rz, seal=seal, ky=ky,
                              kz=kz, force=force.reshape((3,) + shape))
        e2 = _row_errs(None if r_rows is None else r_rows[bad],
                       None if J_rows is None else J_rows[:, bad], r2, J2, s2)
        assert np.all(e2 <= tol), f"{int((e2 > tol).sum())} tie cells match neither choice"
        rep["n_flipped_cells"] = int(bad.sum())
        rep["max_err"] = float(np.where(bad, 0, err).max())
    return rep


def vjp_scales(J_ref, scale, w):
    """Natural magnitudes of J^T w and of the log-permeability gradient at each
    cell: sums of the absolute values of their terms."""
    aw = np.abs(w)
    sp_ = apply_JT(np.abs(J_ref), aw)
    wmax = aw.copy()
    for n in range(6):
        wmax = np.maximum(wmax, shift(aw, n))
    sm = 2.0 * wmax * scale[0]
    return sp_, sm


def compare_vjp(orc, grid, fluid, kx, p, w, gp_gpu, gm_gpu, *, tol, tau, ry, rz, seal):
    want = ("J", "grad_p", "grad_logk", "scale", "dphi")
    ref = orc.evaluate(grid, fluid, kx, p, ry=ry, rz=rz, seal=seal, w=w, want=want)
    sp_, sm = vjp_scales(ref["J"], ref["scale"], w)
    shape = ref["grad_p"].shape

    def errs(o):
        e = np.zeros(shape)
        if gp_gpu is not None:
            e = np.maximum(e, rel_err(np.asarray(gp_gpu, np.float64).reshape(shape),
                                      o["grad_p"], sp_))
        if gm_gpu is not None:
            e = np.maximum(e, rel_err(np.asarray(gm_gpu, np.float64).reshape(shape),
                                      o["grad_logk"], sm))
        return e

    err = errs(ref)
    ties = tie_faces(ref["dphi"], tau)
    rep = {"max_err": float(err.max()), "n_tie_faces": int(ties.sum()), "n_flipped_cells": 0}
    bad = err > tol
    if bad.any():
        touch = cells_touching(ties)
        assert not (bad & ~touch).any(), (
            f"{int((bad & ~touch).sum())} cells differ by up to "
            f"{err[bad & ~touch].max():.3e} away from any upwind tie")
        alt = orc.evaluate(grid, fluid, kx, p, ry=ry, rz=rz, seal=seal, w=w,
                           force=_flip_force(ref["dphi"], ties), want=("grad_p", "grad_logk"))
        err2 = errs(alt)
        assert not (bad & (err2 > tol)).any()
        rep["n_flipped_cells"] = int(bad.sum())
        rep["max_err"] = float(np.where(bad, err2, err).max())
    return rep


# ---------------------------------------------------------------------------
# 10-flux stencil. A cell whose residual differs from the oracle beyond tol
# must touch an upwind tie (cardinal or diagonal face with |dPhi| <= tau) and
# must then agree with the oracle evaluated with the upwind choice of those
# faces flipped.
# ---------------------------------------------------------------------------

def diagonal_dphi(p: np.ndarray):
    """Potential differences p_lo - p_hi of the in-plane diagonal faces, each
    at the face's (i, j) end: [0] face (i,j)-(i+1,j+1), [1] face (i,j)-(i+1,j-1)
    (NaN where the face does not exist). The lower-index cell of the first is
    its (i, j) end, of the second its (i+1, j-1) end."""
    d = np.full((2,) + p.shape, np.nan)
    d[0][:, :-1, :-1] = p[:, :-1, :-1] - p[:, 1:, 1:]
    d[1][:, 1:, :-1] = p[:, :-1, 1:] - p[:, 1:, :-1]   # lower (i+1, j-1) minus upper (i, j)
    return d


def diagonal_ties(p: np.ndarray, tau) -> np.ndarray:
    """Cells touching an in-plane diagonal face with |p_K - p_L| <= tau."""
    t = np.zeros(p.shape, bool)
    ne = np.abs(p[:, :-1, :-1] - p[:, 1:, 1:]) <= tau     # (i,j)-(i+1,j+1)
    se = np.abs(p[:, 1:, :-1] - p[:, :-1, 1:]) <= tau     # (i,j)-(i+1,j-1)
    t[:, :-1, :-1] |= ne
    t[:, 1:, 1:] |= ne
    t[:, 1:, :-1] |= se
    t[:, :-1, 1:] |= se
    return t


def compare_res10(orc, grid, fluid, kx, p, tne, tse, r_gpu, *, tol, tau, ry, rz, seal,
                  mask=None):
    """Residual of the 10-flux stencil against the oracle, cell by cell (only
    where ``mask`` is set, if given). Returns a report dict."""
    r_ref, scale = orc.residual10(grid, fluid, kx, p, tne, tse, ry=ry, rz=rz, seal=seal)
    r_gpu = np.asarray(r_gpu, np.float64).reshape(r_ref.shape)
    err = rel_err(r_gpu, r_ref, scale)
    if mask is not None:
        err = np.where(mask, err, 0.0)
    bad = err > tol
    rep = {"max_err": float(err.max()), "n_cells": int(err.size if mask is None else mask.sum()),
           "n_tie_cells": 0}
    if bad.any():
        p = np.asarray(p, np.float64).reshape(r_ref.shape)
        dphi = orc.evaluate(grid, fluid, kx, p, ry=ry, rz=rz, seal=seal, want=("dphi",))["dphi"]
        dd = diagonal_dphi(p)
        ties = tie_faces(dphi, tau)
        dties = tie_faces(dd, tau)
        touch = cells_touching(ties) | diagonal_ties(p, tau)
        assert not (bad & ~touch).any(), (
            f"{int((bad & ~touch).sum())} cells differ by up to {err[bad & ~touch].max():.3e} "
            "away from any upwind tie")
        force = np.zeros((5,) + r_ref.shape, np.int8)
        force[:3] = _flip_force(dphi, ties)
        force[3:] = _flip_force(dd, dties)
        r_alt, _ = orc.residual10(grid, fluid, kx, p, tne, tse, ry=ry, rz=rz, seal=seal,
                                  force=force)
        err2 = rel_err(r_gpu, r_alt, scale)
        still = bad & (err2 > tol)
        assert not still.any(), f"{int(still.sum())} tie cells match neither upwind choice"
        rep["n_tie_cells"] = int(bad.sum())
        rep["max_err"] = float(np.where(bad, err2, err).max())
    return rep


def crop_mask(shape, lo, hi, full):
    """Cells of a crop whose ten neighbours in the full grid are all inside the
    crop (or outside the domain on both): crop faces on the domain boundary
    are exact, the others lose their outer layer."""
    m = np.ones(shape, bool)
    for ax, (a, b, n) in enumerate(zip(lo, hi, full)):
        sl = [slice(None)] * 3
        if a > 0:
            sl[2 - ax] = 0
            m[tuple(sl)] = False
        if b < n:
            sl[2 - ax] = -1
            m[tuple(sl)] = False
    return m
