"""Python binding of libtpfa.so: argument marshalling only.

Device memory comes from torch CUDA tensors (ROCm) and work is enqueued on
torch's current stream; every computation runs in the library's HIP kernels.
The precision is chosen by the dtype of ``p``: float64 -> the FP64 path,
float32 -> the precision form (``p`` holds offsets from ``pref``).
Tensors use the (nz, ny, nx) shape, x fastest. Per-cell arrays are either
contiguous or all views ``buf[..., :nx]`` of row-padded buffers of shape
(..., nz, ny, ldx) with one common row pitch ldx >= nx; outputs allocated here
take the layout of ``p``.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import torch

from . import _lib as L


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _grid(g, ld: int = 0) -> L.Grid:
    """ld: row pitch of the call's arrays (0 or nx: contiguous)."""
    return L.Grid(int(g.nx), int(g.ny), int(g.nz), float(g.dx), float(g.dy), float(g.dz),
                  float(g.gk), 0 if ld == int(g.nx) else int(ld))


def _fluid(f) -> L.Fluid:
    return L.Fluid(float(f.rho0), float(f.cf), float(f.p0), float(f.mu))


def _launch(tile: Optional[int], kz_chunk: Optional[int], xcd_remap, rows=None,
            pad_writes: bool = False, sliced: bool = False):
    """``xcd_remap``: True (or "bands") for the XCD band order, "yfast" for the
    y-fast tile order, False for the natural order. ``rows`` = (y_begin, y_end):
    compute and write only those rows (a y slab; the grid's other rows are read
    as its halo). ``pad_writes``: the outputs' row padding may be overwritten
    (zeros), so that rows of row-pitched outputs are written in whole lines.
    ``sliced``: r and J go to one array of 64-cell slices (see sliced_shape)."""
    if (tile is None and kz_chunk is None and not xcd_remap and rows is None and not pad_writes
            and not sliced):
        return None
    if xcd_remap == "yfast":
        flags = L.TPFA_LAUNCH_Y_FAST
    elif xcd_remap in (True, "bands"):
        flags = L.TPFA_LAUNCH_XCD_REMAP
    elif not xcd_remap:
        flags = 0
    else:
        raise ValueError(f"unknown workgroup order {xcd_remap!r}")
    if pad_writes:
        flags |= L.TPFA_LAUNCH_PAD_WRITES
    if sliced:
        flags |= L.TPFA_LAUNCH_SLICED
    y0, y1 = (0, 0) if rows is None else (int(rows[0]), int(rows[1]))
    return L.Launch(-1 if tile is None else int(tile), 0 if kz_chunk is None else int(kz_chunk),
                    flags, y0, y1)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _prec(p: torch.Tensor) -> int:
    if p.dtype == torch.float64:
        return L.TPFA_FP64
    if p.dtype == torch.float32:
        return L.TPFA_FP32
    raise TypeError(f"p must be float64 or float32, got {p.dtype}")


def _pitch(t, name, grid) -> Optional[int]:
    """Row pitch of a per-cell array of shape (nz, ny, nx) or (P, nz, ny, nx):
    nx when it is contiguous, ldx when it is a view ``buf[..., :nx]`` of a
    row-padded buffer (..., nz, ny, ldx); None when the array holds a single
    row, which every pitch addresses alike."""
    nx, ny, nz = int(grid.nx), int(grid.ny), int(grid.nz)
    if t.dim() in (3, 4) and tuple(t.shape[-3:]) == (nz, ny, nx):
        if nx > 1 and t.stride(-1) != 1:
            raise ValueError(f"{name} must be contiguous along x")
        # stride of each dimension in units of the pitch (dimensions of size 1 carry none)
        per = {-2: 1, -3: ny}
        if t.dim() == 4:
            per[0] = ny * nz
        fixed = [(d, f) for d, f in per.items() if t.shape[d] > 1]
        if not fixed:
            return None
        ld = t.stride(fixed[0][0]) // fixed[0][1]
        if ld < nx or any(t.stride(d) != f * ld for d, f in fixed):
            raise ValueError(f"{name}: strides {t.stride()} are not those of a row-padded "
                             f"(..., nz, ny, ldx) buffer")
        return ld
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous or a view [..., :nx] of a row-padded "
                         f"(..., nz, ny, ldx) buffer")
    return nx if t.numel() > nx else None


class _Layout:
    """The one row pitch of a call's per-cell arrays: set by the first array
    that fixes it (arrays of a single row fit any pitch), nx if none does."""

    def __init__(self, grid):
        self.grid = grid
        self.ld = None

    def take(self, t, name):
        got = _pitch(t, name, self.grid)
        if got is None:
            return
        if self.ld is None:
            self.ld = got
        elif got != self.ld:
            raise ValueError(f"{name} has row pitch {got}, the call's other arrays {self.ld}")

    @property
    def pitch(self) -> int:
        return int(self.grid.nx) if self.ld is None else self.ld


def _empty(p, lay, lead=(), dtype=None):
    """Output array in the call's layout: p's shape when the pitch is nx, else
    a view [..., :nx] of a new buffer with the call's row pitch."""
    dt = p.dtype if dtype is None else dtype
    grid, ld = lay.grid, lay.pitch
    if ld == int(grid.nx):
        return torch.empty(tuple(lead) + tuple(p.shape), dtype=dt, device=p.device)
    buf = torch.empty(tuple(lead) + (int(grid.nz), int(grid.ny), ld), dtype=dt, device=p.device)
    return buf[..., :int(grid.nx)]


def pitch_for(grid) -> int:
    """Row pitch for a grid's arrays: nx rounded up to a multiple of 32 cells,
    so that rows of float and double arrays start on 128-byte lines (with
    128-byte aligned buffers). One pitch serves every array of a call, the
    seal bytes included."""
    return (int(grid.nx) + 31) // 32 * 32


def empty_pitched(grid, dtype, device=None, lead=(), ldx: Optional[int] = None) -> torch.Tensor:
    """Uninitialised (lead..., nz, ny, nx) array with row pitch ``ldx``
    (default pitch_for(grid)): the view [..., :nx] of a (lead..., nz, ny, ldx)
    buffer. Outputs written into such arrays take whole lines at every tile
    edge."""
    ld = pitch_for(grid) if ldx is None else int(ldx)
    if ld < int(grid.nx):
        raise ValueError(f"row pitch {ld} is below nx = {grid.nx}")
    buf = torch.empty(tuple(lead) + (int(grid.nz), int(grid.ny), ld), dtype=dtype, device=device)
    return buf[..., :int(grid.nx)]


def sliced_shape(grid):
    """Shape (nz, ny, S, 8, 64) of the sliced r + J array, S = ceil(nx / 64):
    slice s of row j of plane k holds the residual (run 0) and the Jacobian
    planes diag, -x, +x, -y, +y, -z, +z (runs 1..7) of the cells
    64 s <= i < 64 s + 64; lanes beyond nx hold zeros."""
    return (int(grid.nz), int(grid.ny), (int(grid.nx) + 63) // 64, 8, 64)


def empty_sliced(grid, dtype, device=None) -> torch.Tensor:
    """Uninitialised sliced r + J array (sliced_shape)."""
    return torch.empty(sliced_shape(grid), dtype=dtype, device=device)


def unslice(grid, Js: torch.Tensor):
    """(r[nz, ny, nx], J[7, nz, ny, nx]) copied out of a sliced r + J array."""
    nz, ny, S = sliced_shape(grid)[:3]
    planes = Js.reshape(nz, ny, S, 8, 64).permute(3, 0, 1, 2, 4).reshape(8, nz, ny, S * 64)
    planes = planes[..., :int(grid.nx)].contiguous()
    return planes[0], planes[1:]


def _sliced_out(J_out, p, grid, want_r, r_out, dt, dev):
    """The sliced r + J array of a Jacobian call (allocated unless given)."""
    if want_r is not True or r_out is not None:
        raise ValueError("sliced=True writes the residual into J (run 0): leave want_r and r_out")
    J = J_out if J_out is not None else empty_sliced(grid, dt, dev)
    _need(J, "J_out", dt, math.prod(sliced_shape(grid)), dev)
    return J


def to_pitched(t: torch.Tensor, grid, ldx: Optional[int] = None) -> torch.Tensor:
    """Copy of a (lead..., nz, ny, nx) array in the layout of empty_pitched."""
    out = empty_pitched(grid, t.dtype, t.device, tuple(t.shape[:-3]), ldx)
    out.copy_(t)
    return out


def _need(t, name, dtype, n, device, lay=None):
    """Checks a tensor argument; a per-cell array (``lay`` given) must fit the
    call's row pitch."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor, got {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if lay is None:
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return
    lay.take(t, name)


def _pad_ok(pad_writes, lay, **outs):
    """With pad_writes the kernels write each output row up to the pitch, the
    last row of the last plane included: every output's buffer must hold it
    (a (..., nz, ny, ldx) buffer, as empty_pitched allocates)."""
    grid = lay.grid
    nx, ny, nz, ld = int(grid.nx), int(grid.ny), int(grid.nz), lay.pitch
    if not pad_writes or ld == nx:
        return
    for name, t in outs.items():
        if t is None:
            continue
        planes = t.numel() // (nx * ny * nz)
        need = t.storage_offset() + planes * nz * ny * ld
        have = t.untyped_storage().nbytes() // t.element_size()
        if need > have:
            raise ValueError(f"pad_writes: {name} ends inside the padding of its last row "
                             f"({need} elements from its storage start needed, {have} held); "
                             f"use (..., nz, ny, ldx) buffers such as empty_pitched")


def _kyz(ky, kz):
    if (ky is None) != (kz is None):
        raise ValueError("ky and kz go together (per-direction permeability arrays)")
    return None if ky is None else (ky, kz)


def _inputs(grid, kx, p, seal, pref, trans=None, kyz=None):
    n = int(grid.nx) * int(grid.ny) * int(grid.nz)
    prec = _prec(p)
    dt = p.dtype
    dev = p.device
    lay = _Layout(grid)
    _need(p, "p", dt, n, None, lay)
    if kyz is not None:
        if trans is not None:
            raise ValueError("give either permeabilities (kx, ky, kz) or trans, not both")
        _need(kyz[0], "ky", dt, n, dev, lay)
        _need(kyz[1], "kz", dt, n, dev, lay)
    if trans is not None:
        if kx is not None or seal is not None:
            raise ValueError("give either kx (and seal) or trans=(tx, ty, tz), not both")
        for name, t in zip(("tx", "ty", "tz"), trans):
            if t is None:
                raise ValueError(f"trans needs {name}")
            _need(t, name, dt, n, dev, lay)
    elif kx is None:
        raise ValueError("kx is required (or trans=(tx, ty, tz))")
    _need(kx, "kx", dt, n, dev, lay)
    _need(seal, "seal", torch.uint8, n, dev, lay)
    if prec == L.TPFA_FP32:
        if pref is None:
            raise ValueError("the FP32 precision form needs pref (float64[nz])")
        _need(pref, "pref", torch.float64, int(grid.nz), dev)
    return n, prec, dt, dev, lay


def _rock(kx, seal, ry, rz, trans=None, ky=None, kz=None) -> L.Rock:
    tx, ty, tz = trans if trans is not None else (None, None, None)
    return L.Rock(_ptr(kx), _ptr(ky), _ptr(kz), float(ry), float(rz), _ptr(seal), _ptr(tx),
                  _ptr(ty), _ptr(tz))


def residual(grid, fluid, kx, p, *, seal=None, pref=None, ry=1.0, rz=1.0, ky=None, kz=None,
             out=None, trans=None, tile=None, kz_chunk=None, xcd_remap=False,
             rows=None, pad_writes=False) -> torch.Tensor:
    """Flux residual r (paper Algorithm 1, Eqs. 3-5)."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    r = out if out is not None else _empty(p, lay)
    _need(r, "out", dt, n, dev, lay)
    _pad_ok(pad_writes, lay, out=r)
    lib = L.load()
    L.check(lib.tpfa_residual(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                              C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
                              C.byref(L.State(_ptr(p), _ptr(pref))), prec, _ptr(r),
                              _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes),
                              _stream(dev)), lib)
    return r


def _launch_ref(tile, kz_chunk, xcd_remap, rows=None, pad_writes=False, sliced=False):
    ln = _launch(tile, kz_chunk, xcd_remap, rows, pad_writes, sliced)
    return None if ln is None else C.byref(ln)


def jacobian(grid, fluid, kx, p, *, seal=None, pref=None, ry=1.0, rz=1.0, ky=None, kz=None,
             want_r=True, r_out=None, J_out=None, trans=None, tile=None, kz_chunk=None,
             xcd_remap=False, rows=None, pad_writes=False, sliced=False):
    """Residual (or None) and Jacobian J[7, nz, ny, nx], planes
    [diag, -x, +x, -y, +y, -z, +z]. With ``sliced``: (None, the sliced r + J
    array of sliced_shape), which unslice turns into planes."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    r = None
    if sliced:
        J = _sliced_out(J_out, p, grid, want_r, r_out, dt, dev)
    else:
        if want_r:
            r = r_out if r_out is not None else _empty(p, lay)
            _need(r, "r_out", dt, n, dev, lay)
        J = J_out if J_out is not None else _empty(p, lay, (7,))
        _need(J, "J_out", dt, 7 * n, dev, lay)
        _pad_ok(pad_writes, lay, r_out=r, J_out=J)
    lib = L.load()
    L.check(lib.tpfa_jacobian(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                              C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
                              C.byref(L.State(_ptr(p), _ptr(pref))), prec, _ptr(r), _ptr(J),
                              _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes, sliced),
                              _stream(dev)), lib)
    return r, J


def residual_vjp(grid, fluid, kx, p, w, *, seal=None, pref=None, ry=1.0, rz=1.0, ky=None, kz=None,
                 want_p=True, want_logk=True, gp_out=None, gm_out=None, trans=None, tile=None,
                 kz_chunk=None, xcd_remap=False, rows=None, pad_writes=False):
    """(grad_p, grad_logk) = (J^T w, d(w.r)/d ln kx); either may be None. With
    ``trans`` = (tx, ty, tz) the second output is grad_logt [3, nz, ny, nx]:
    d(w.r)/d ln T of each cell's +x, +y, +z face. With per-direction arrays
    ``ky``, ``kz`` it is [3, nz, ny, nx]: d(w.r)/d ln kx, ln ky, ln kz."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    _need(w, "w", dt, n, dev, lay)
    planes = 3 if trans is not None or ky is not None else 1
    gp = gm = None
    if want_p:
        gp = gp_out if gp_out is not None else _empty(p, lay)
        _need(gp, "gp_out", dt, n, dev, lay)
    if want_logk:
        gm = gm_out if gm_out is not None else _empty(p, lay, (3,) if planes == 3 else ())
        _need(gm, "gm_out", dt, planes * n, dev, lay)
    _pad_ok(pad_writes, lay, gp_out=gp, gm_out=gm)
    lib = L.load()
    fn = lib.tpfa_residual_vjp_trans if trans is not None else lib.tpfa_residual_vjp
    L.check(fn(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
               C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
               C.byref(L.State(_ptr(p), _ptr(pref))), prec, _ptr(w), _ptr(gp), _ptr(gm),
               _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes),
                              _stream(dev)), lib)
    return gp, gm


def residual_and_vjp(grid, fluid, kx, p, w, *, seal=None, pref=None, ry=1.0, rz=1.0,
                     want_p=True, want_logk=True, r_out=None, gp_out=None, gm_out=None,
                     tile=None, kz_chunk=None, xcd_remap=False, rows=None, pad_writes=False):
    """(r, grad_p, grad_logk) in one pass (tpfa_residual_and_vjp): the value and
    gradient of w.r. r equals residual(), the gradients residual_vjp(), bit
    for bit; permeability form with ratios only."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref)
    _need(w, "w", dt, n, dev, lay)
    if not (want_p or want_logk):
        raise ValueError("residual_and_vjp needs a gradient; use residual() for r alone")
    r = r_out if r_out is not None else _empty(p, lay)
    _need(r, "r_out", dt, n, dev, lay)
    gp = gm = None
    if want_p:
        gp = gp_out if gp_out is not None else _empty(p, lay)
        _need(gp, "gp_out", dt, n, dev, lay)
    if want_logk:
        gm = gm_out if gm_out is not None else _empty(p, lay)
        _need(gm, "gm_out", dt, n, dev, lay)
    _pad_ok(pad_writes, lay, r_out=r, gp_out=gp, gm_out=gm)
    lib = L.load()
    L.check(lib.tpfa_residual_and_vjp(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                                      C.byref(_rock(kx, seal, ry, rz)),
                                      C.byref(L.State(_ptr(p), _ptr(pref))), prec, _ptr(w),
                                      _ptr(r), _ptr(gp), _ptr(gm),
                                      _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes),
                                      _stream(dev)), lib)
    return r, gp, gm


def _accum(accum, dt_, n, dev, lay):
    """``accum`` = dict(phi=..., p_prev=..., dt=..., cr=...) -> L.Accum."""
    if accum is None:
        return None
    phi, p_prev = accum["phi"], accum["p_prev"]
    _need(phi, "phi", dt_, n, dev, lay)
    _need(p_prev, "p_prev", dt_, n, dev, lay)
    return L.Accum(_ptr(phi), _ptr(p_prev), float(accum["dt"]), float(accum.get("cr", 0.0)))


def residual_be(grid, fluid, kx, p, accum, *, seal=None, pref=None, ry=1.0, rz=1.0, ky=None,
                kz=None, out=None, trans=None, tile=None, kz_chunk=None, xcd_remap=False,
                rows=None, pad_writes=False) -> torch.Tensor:
    """Full backward-Euler residual of Eq. (2): V (phi rho - phi_n rho_n)/dt plus
    the flux sum. ``accum`` = dict(phi, p_prev, dt, cr)."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    acc = _accum(accum, dt, n, dev, lay)
    if acc is None:
        raise ValueError("residual_be needs accum")
    r = out if out is not None else _empty(p, lay)
    _need(r, "out", dt, n, dev, lay)
    _pad_ok(pad_writes, lay, out=r)
    lib = L.load()
    L.check(lib.tpfa_residual_be(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                                 C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
                                 C.byref(L.State(_ptr(p), _ptr(pref))), C.byref(acc), prec,
                                 _ptr(r), _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes),
                                 _stream(dev)), lib)
    return r


def jacobian_be(grid, fluid, kx, p, accum, *, seal=None, pref=None, ry=1.0, rz=1.0, ky=None,
                kz=None, want_r=True, r_out=None, J_out=None, trans=None, tile=None, kz_chunk=None,
                xcd_remap=False, rows=None, pad_writes=False, sliced=False):
    """Backward-Euler residual (or None) and its Jacobian J[7, nz, ny, nx]
    (with ``sliced``: None and the sliced r + J array, as for jacobian)."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    acc = _accum(accum, dt, n, dev, lay)
    if acc is None:
        raise ValueError("jacobian_be needs accum")
    r = None
    if sliced:
        J = _sliced_out(J_out, p, grid, want_r, r_out, dt, dev)
    else:
        if want_r:
            r = r_out if r_out is not None else _empty(p, lay)
            _need(r, "r_out", dt, n, dev, lay)
        J = J_out if J_out is not None else _empty(p, lay, (7,))
        _need(J, "J_out", dt, 7 * n, dev, lay)
        _pad_ok(pad_writes, lay, r_out=r, J_out=J)
    lib = L.load()
    L.check(lib.tpfa_jacobian_be(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                                 C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
                                 C.byref(L.State(_ptr(p), _ptr(pref))), C.byref(acc), prec,
                                 _ptr(r), _ptr(J),
                                 _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes, sliced),
                                 _stream(dev)), lib)
    return r, J


def jvp(grid, fluid, kx, p, v, *, accum=None, seal=None, pref=None, ry=1.0, rz=1.0, ky=None,
        kz=None, want_r=False, out=None, r_out=None, trans=None, tile=None, kz_chunk=None,
        xcd_remap=False, rows=None, pad_writes=False):
    """Matrix-free J v of the flux residual, or of the backward-Euler residual
    when ``accum`` is given; returns (jv, r or None)."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    _need(v, "v", dt, n, dev, lay)
    acc = _accum(accum, dt, n, dev, lay)
    jv = out if out is not None else _empty(p, lay)
    _need(jv, "out", dt, n, dev, lay)
    r = None
    if want_r:
        r = r_out if r_out is not None else _empty(p, lay)
        _need(r, "r_out", dt, n, dev, lay)
    _pad_ok(pad_writes, lay, out=jv, r_out=r)
    lib = L.load()
    L.check(lib.tpfa_jvp(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                         C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
                         C.byref(L.State(_ptr(p), _ptr(pref))),
                         None if acc is None else C.byref(acc), prec, _ptr(v), _ptr(jv),
                         _ptr(r), _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes),
                              _stream(dev)), lib)
    return jv, r


def residual10(grid, fluid, kx, p, tne, tse, *, seal=None, pref=None, ry=1.0, rz=1.0, ky=None,
               kz=None, out=None, trans=None, tile=None, kz_chunk=None, xcd_remap=False,
               rows=None, pad_writes=False) -> torch.Tensor:
    """Residual of the 10-flux stencil (six faces plus four in-plane diagonal
    faces with caller-supplied transmissibilities tne, tse)."""
    n, prec, dt, dev, lay = _inputs(grid, kx, p, seal, pref, trans, _kyz(ky, kz))
    _need(tne, "tne", dt, n, dev, lay)
    _need(tse, "tse", dt, n, dev, lay)
    r = out if out is not None else _empty(p, lay)
    _need(r, "out", dt, n, dev, lay)
    _pad_ok(pad_writes, lay, out=r)
    lib = L.load()
    L.check(lib.tpfa_residual10(C.byref(_grid(grid, lay.pitch)), C.byref(_fluid(fluid)),
                                C.byref(_rock(kx, seal, ry, rz, trans, ky, kz)),
                                C.byref(L.State(_ptr(p), _ptr(pref))), prec, _ptr(tne),
                                _ptr(tse), _ptr(r),
                                _launch_ref(tile, kz_chunk, xcd_remap, rows, pad_writes),
                                _stream(dev)), lib)
    return r


def hydrostatic(grid, fluid, p_top: Optional[float] = None, device=None) -> torch.Tensor:
    """Discrete hydrostatic reference column pref[nz] (float64, on the GPU)."""
    dev = torch.device(device) if device is not None else torch.device("cuda",
                                                                       torch.cuda.current_device())
    pref = torch.empty(int(grid.nz), dtype=torch.float64, device=dev)
    lib = L.load()
    top = float(fluid.p0 if p_top is None else p_top)
    L.check(lib.tpfa_hydrostatic(C.byref(_grid(grid)), C.byref(_fluid(fluid)), top, _ptr(pref),
                                 _stream(dev)), lib)
    return pref


def offset_pressure(grid, p: torch.Tensor, pref: torch.Tensor, out=None) -> torch.Tensor:
    """FP32 offsets dp = (float)(p - pref[k]) of an FP64 pressure field."""
    n = int(grid.nx) * int(grid.ny) * int(grid.nz)
    lay = _Layout(grid)
    _need(p, "p", torch.float64, n, None, lay)
    _need(pref, "pref", torch.float64, int(grid.nz), p.device)
    if out is not None:
        _need(out, "out", torch.float32, n, p.device, lay)
    dp = out if out is not None else _empty(p, lay, dtype=torch.float32)
    lib = L.load()
    L.check(lib.tpfa_offset_pressure(C.byref(_grid(grid, lay.pitch)), _ptr(p), _ptr(pref),
                                     _ptr(dp), _stream(p.device)), lib)
    return dp


def stream_probe(grid, p: torch.Tensor, k: torch.Tensor, seal: torch.Tensor,
                 out=None, sliced: bool = False) -> torch.Tensor:
    """Bandwidth probe with the Jacobian kernels' access pattern (tpfa_stream_probe):
    out[q] = p + (q + seal) * k for q = 0..7, from contiguous p, k (float64 or
    float32) and uint8 seal of the grid's shape (nz, ny, nx); returns out of
    shape (8, nz, ny, nx), or with ``sliced`` (tpfa_stream_probe_sliced) the
    array of sliced_shape with output q in run q (lanes beyond nx untouched)."""
    shape = (int(grid.nz), int(grid.ny), int(grid.nx))
    for t, name in ((p, "p"), (k, "k"), (seal, "seal")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous CUDA tensor")
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have the grid's shape {shape}")
    if k.dtype != p.dtype or p.dtype not in (torch.float64, torch.float32):
        raise ValueError("p and k must both be float64 or both float32")
    if seal.dtype != torch.uint8:
        raise ValueError("seal must be uint8")
    oshape = sliced_shape(grid) if sliced else (8,) + shape
    if out is None:
        out = torch.empty(oshape, dtype=p.dtype, device=p.device)
    elif not (out.is_contiguous() and out.dtype == p.dtype and tuple(out.shape) == oshape):
        raise ValueError(f"out must be contiguous, of p's dtype and of shape {oshape}")
    prec = L.TPFA_FP64 if p.dtype == torch.float64 else L.TPFA_FP32
    lib = L.load()
    fn = lib.tpfa_stream_probe_sliced if sliced else lib.tpfa_stream_probe
    L.check(fn(C.byref(_grid(grid)), prec, _ptr(p), _ptr(k), _ptr(seal), _ptr(out),
               _stream(p.device)), lib)
    return out


_OPS = {"residual": L.TPFA_OP_RESIDUAL, "jacobian": L.TPFA_OP_JACOBIAN, "vjp": L.TPFA_OP_VJP,
        "residual10": L.TPFA_OP_RESIDUAL10, "residual_be": L.TPFA_OP_RESIDUAL_BE,
        "jacobian_be": L.TPFA_OP_JACOBIAN_BE, "jvp": L.TPFA_OP_JVP, "jvp_be": L.TPFA_OP_JVP_BE}
_GIVEN = 1  # non-null marker for an array: tpfa_resolve_launch only reads which are given


def resolve_launch(grid, op: str, dtype=torch.float64, *, form: str = "k", tile=None,
                   kz_chunk=None, xcd_remap=False, rows=None, ldx: Optional[int] = None,
                   pad_writes: bool = False, sliced: bool = False) -> dict:
    """The launch a call of ``op`` ('residual', 'jacobian', 'vjp', 'residual10',
    'residual_be', 'jacobian_be', 'jvp', 'jvp_be') would make on this grid in
    this precision, rock form ('k': kx with ratios, 'k3': kx, ky, kz arrays,
    'trans': face transmissibilities), row pitch and launch arguments: tile
    id and shape, z planes per workgroup, XCD band order, row range. Nothing
    runs on the GPU."""
    prec = {torch.float64: L.TPFA_FP64, torch.float32: L.TPFA_FP32}[dtype]
    G = _GIVEN
    rock = {"k": L.Rock(G, None, None, 1.0, 1.0, None),
            "k3": L.Rock(G, G, G, 1.0, 1.0, None),
            "trans": L.Rock(None, None, None, 1.0, 1.0, None, G, G, G)}[form]
    ln = _launch(tile, kz_chunk, xcd_remap, rows, pad_writes, sliced)
    out = L.Launch()
    lib = L.load()
    L.check(lib.tpfa_resolve_launch(C.byref(_grid(grid, int(grid.nx) if ldx is None else ldx)),
                                    _OPS[op], prec, C.byref(rock),
                                    None if ln is None else C.byref(ln), C.byref(out)), lib)
    tx, ty, th = tile_shapes()[out.tile]
    return {"tile": out.tile, "shape": (tx, ty), "threads": th, "kz_chunk": out.kz_chunk,
            "xcd_remap": bool(out.flags & L.TPFA_LAUNCH_XCD_REMAP),
            "order": ("bands" if out.flags & L.TPFA_LAUNCH_XCD_REMAP else
                      "yfast" if out.flags & L.TPFA_LAUNCH_Y_FAST else "natural"),
            "rows": (out.y_begin, out.y_end),
            "pad_writes": bool(out.flags & L.TPFA_LAUNCH_PAD_WRITES),
            "sliced": bool(out.flags & L.TPFA_LAUNCH_SLICED)}


def fit_tile_shape(nx: int, rows: int):
    """(tx, ty) of the fitted tile (tile id TPFA_TILE_FIT = 10, ensemble members
    only) for rows of nx cells: 256 threads, tx ty <= 256 cells."""
    lib = L.load()
    tx, ty = C.c_int(), C.c_int()
    L.check(lib.tpfa_fit_tile_shape(int(nx), int(rows), C.byref(tx), C.byref(ty)), lib)
    return tx.value, ty.value


def tile_shapes():
    """[(tx, ty, threads)] of the compiled tiles, indexed by tile id."""
    lib = L.load()
    out = []
    for t in range(lib.tpfa_num_tiles()):
        tx, ty, th = C.c_int(), C.c_int(), C.c_int()
        L.check(lib.tpfa_tile_shape(t, C.byref(tx), C.byref(ty), C.byref(th)), lib)
        out.append((tx.value, ty.value, th.value))
    return out


def ensemble_run_noalloc(members: Sequence[dict], outputs: Sequence[tuple], *,
                         mode: str = "jacobian"):
    """One ensemble launch that allocates nothing (tpfa_ensemble_run_noalloc):
    ``members`` as for Ensemble, ``outputs`` one (r, J) pair per member,
    allocated by the caller in the layout of the member's p (r may be None in
    the Jacobian mode, J is ignored in the residual mode). The model table is
    written into the library's fixed-size device array: at most 256 members,
    and calls that overlap on one GPU race."""
    if not members or len(outputs) != len(members):
        raise ValueError("one (r, J) pair per member, at least one member")
    bm = {"jacobian": L.TPFA_BATCH_JACOBIAN, "residual": L.TPFA_BATCH_RESIDUAL}[mode]
    arr = (L.Model * len(members))()
    prec = device = None
    for m, (d, (r, J)) in enumerate(zip(members, outputs)):
        g, p = d["grid"], d["p"]
        n, pr, dt, dev, lay = _inputs(g, d["kx"], p, d.get("seal"), d.get("pref"))
        if prec is None:
            prec, device = pr, dev
        elif pr != prec or dev != device:
            raise ValueError("all ensemble members need the same precision and device")
        if d.get("sliced", False):
            if r is not None:
                raise ValueError("a sliced member takes r = None (the residual is in J)")
            _need(J, "J", dt, math.prod(sliced_shape(g)), dev)
        else:
            if bm == L.TPFA_BATCH_JACOBIAN:
                _need(J, "J", dt, 7 * n, dev, lay)
            if r is not None or bm == L.TPFA_BATCH_RESIDUAL:
                _need(r, "r", dt, n, dev, lay)
            _pad_ok(d.get("pad_writes", False), lay, r=r,
                    J=J if bm == L.TPFA_BATCH_JACOBIAN else None)
        arr[m] = L.Model(_grid(g, lay.pitch), _fluid(d["fluid"]),
                         _rock(d["kx"], d.get("seal"), d.get("ry", 1.0), d.get("rz", 1.0)),
                         L.State(_ptr(p), _ptr(d.get("pref"))), _ptr(r), _ptr(J),
                         _launch(d.get("tile"), d.get("kz_chunk"), False, d.get("rows"),
                                 d.get("pad_writes", False), d.get("sliced", False))
                         or L.Launch(-1, 0, 0, 0, 0))
    lib = L.load()
    L.check(lib.tpfa_ensemble_run_noalloc(arr, len(members), prec, bm, _stream(device)), lib)


class Ensemble:
    """Many independent grids run by one persistent kernel replayed from a
    HIP graph. ``members`` is a sequence of dicts with keys grid, fluid, kx,
    p, and optionally seal, pref, ry, rz, tile, kz_chunk, rows, pad_writes,
    sliced. Outputs are allocated here in the layout of the member's ``p``
    (``r[m]``, ``J[m]``; a sliced member: ``r[m]`` None and ``J[m]`` its sliced
    r + J array) and overwritten by every run."""

    def __init__(self, members: Sequence[dict], *, mode: str = "jacobian", want_r: bool = True):
        if not members:
            raise ValueError("an ensemble needs at least one member")
        self.mode = {"jacobian": L.TPFA_BATCH_JACOBIAN, "residual": L.TPFA_BATCH_RESIDUAL}[mode]
        self.members = list(members)
        self.r, self.J = [], []
        arr = (L.Model * len(members))()
        prec = None
        for m, d in enumerate(self.members):
            g, p = d["grid"], d["p"]
            n, pr, dt, dev, lay = _inputs(g, d["kx"], p, d.get("seal"), d.get("pref"))
            if prec is None:
                prec, self.device = pr, dev
            elif pr != prec or dev != self.device:
                raise ValueError("all ensemble members need the same precision and device")
            if d.get("sliced", False):
                r, J = None, empty_sliced(g, dt, dev)
            else:
                r = _empty(p, lay) if (
                    want_r or self.mode == L.TPFA_BATCH_RESIDUAL) else None
                J = _empty(p, lay, (7,)) if (
                    self.mode == L.TPFA_BATCH_JACOBIAN) else None
            self.r.append(r)
            self.J.append(J)
            arr[m] = L.Model(_grid(g, lay.pitch), _fluid(d["fluid"]),
                             _rock(d["kx"], d.get("seal"), d.get("ry", 1.0), d.get("rz", 1.0)),
                             L.State(_ptr(p), _ptr(d.get("pref"))), _ptr(r), _ptr(J),
                             _launch(d.get("tile"), d.get("kz_chunk"), False, d.get("rows"),
                                     d.get("pad_writes", False), d.get("sliced", False))
                             or L.Launch(-1, 0, 0, 0, 0))
        self.prec = prec
        self._handle = C.c_void_p()
        self._lib = L.load()
        L.check(self._lib.tpfa_batch_create(arr, len(self.members), prec, self.mode,
                                            C.byref(self._handle), _stream(self.device)),
                self._lib)
        self.schedule = "persistent"

    def set_schedule(self, schedule: str):
        """'persistent' (work counter) or 'grouped' (one workgroup per item)."""
        code = {"persistent": L.TPFA_SCHEDULE_PERSISTENT,
                "grouped": L.TPFA_SCHEDULE_GROUPED}[schedule]
        L.check(self._lib.tpfa_batch_set_schedule(self._handle, code), self._lib)
        self.schedule = schedule

    def run(self, graph: bool = True):
        fn = self._lib.tpfa_batch_run if graph else self._lib.tpfa_batch_run_eager
        L.check(fn(self._handle, _stream(self.device)), self._lib)

    def info(self):
        n = C.c_int64()
        wg = C.c_int()
        L.check(self._lib.tpfa_batch_info(self._handle, C.byref(n), C.byref(wg)), self._lib)
        return n.value, wg.value

    def close(self):
        if self._handle:
            self._lib.tpfa_batch_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TPFAResidual(torch.autograd.Function):
    """r(p, ln kx) with a hand-written adjoint.

    forward: kx = exp(logk) (the log-permeability parameterisation), then the
    residual kernel; backward: the vector-Jacobian kernel, which recomputes the
    upwind choices, returns (J^T w, d(w.r)/d ln kx). Non-tensor arguments:
    grid, fluid, seal, pref, ry, rz."""

    @staticmethod
    def forward(ctx, p, logk, grid, fluid, seal=None, pref=None, ry=1.0, rz=1.0):
        # one layout for every array of the calls (exp and the cotangents are contiguous)
        p, seal = p.contiguous(), None if seal is None else seal.contiguous()
        kx = torch.exp(logk).contiguous()
        r = residual(grid, fluid, kx, p, seal=seal, pref=pref, ry=ry, rz=rz)
        ctx.save_for_backward(p, kx)
        ctx.save_for_forward(p, kx)
        ctx.cfg = (grid, fluid, seal, pref, ry, rz)
        return r

    @staticmethod
    def backward(ctx, w):
        p, kx = ctx.saved_tensors
        grid, fluid, seal, pref, ry, rz = ctx.cfg
        gp, gm = residual_vjp(grid, fluid, kx, p, w.contiguous(), seal=seal, pref=pref, ry=ry,
                              rz=rz, want_p=ctx.needs_input_grad[0],
                              want_logk=ctx.needs_input_grad[1])
        return gp, gm, None, None, None, None, None, None

    @staticmethod
    def jvp(ctx, dp, dlogk, *_):
        """Forward mode with respect to p: the matrix-free Jacobian-vector
        product kernel. (A tangent in ln kx is not provided: use reverse mode.)"""
        if dlogk is not None and bool(dlogk.any()):  # zero tangents are passed too
            raise NotImplementedError("forward-mode derivative with respect to ln kx; "
                                      "use reverse mode (backward) for it")
        p, kx = ctx.saved_tensors
        grid, fluid, seal, pref, ry, rz = ctx.cfg
        if dp is None:
            return torch.zeros_like(p)
        jv, _ = jvp(grid, fluid, kx, p, dp.contiguous(), seal=seal, pref=pref, ry=ry, rz=rz)
        return jv


class TPFATransResidual(torch.autograd.Function):
    """r(p, ln T) in the transmissibility form, with a hand-written adjoint.

    forward: T = exp(logt), logt of shape [3, nz, ny, nx] (the +x, +y, +z face
    of every cell), then the residual kernel; backward: the vector-Jacobian
    kernel of that form returns (J^T w, d(w.r)/d ln T). Forward mode in p uses
    the Jacobian-vector product kernel. Non-tensor arguments: grid, fluid,
    pref."""

    @staticmethod
    def forward(ctx, p, logt, grid, fluid, pref=None):
        p = p.contiguous()
        t = torch.exp(logt).contiguous()
        trans = (t[0], t[1], t[2])
        r = residual(grid, fluid, None, p, pref=pref, trans=trans)
        ctx.save_for_backward(p, t)
        ctx.save_for_forward(p, t)
        ctx.cfg = (grid, fluid, pref)
        return r

    @staticmethod
    def backward(ctx, w):
        p, t = ctx.saved_tensors
        grid, fluid, pref = ctx.cfg
        gp, gt = residual_vjp(grid, fluid, None, p, w.contiguous(), pref=pref,
                              trans=(t[0], t[1], t[2]), want_p=ctx.needs_input_grad[0],
                              want_logk=ctx.needs_input_grad[1])
        return gp, gt, None, None, None

    @staticmethod
    def jvp(ctx, dp, dlogt, *_):
        if dlogt is not None and bool(dlogt.any()):  # zero tangents are passed too
            raise NotImplementedError("forward-mode derivative with respect to ln T; "
                                      "use reverse mode (backward) for it")
        p, t = ctx.saved_tensors
        grid, fluid, pref = ctx.cfg
        if dp is None:
            return torch.zeros_like(p)
        jv, _ = jvp(grid, fluid, None, p, dp.contiguous(), pref=pref, trans=(t[0], t[1], t[2]))
        return jv


class TPFAAnisoResidual(torch.autograd.Function):
    """r(p, ln k) in the per-direction permeability form, with a hand-written
    adjoint.

    forward: k = exp(logk3), logk3 of shape [3, nz, ny, nx] (ln kx, ln ky,
    ln kz of every cell), then the residual kernel; backward: the
    vector-Jacobian kernel returns (J^T w, d(w.r)/d ln k per direction).
    Forward mode in p uses the Jacobian-vector product kernel. Non-tensor
    arguments: grid, fluid, seal, pref."""

    @staticmethod
    def forward(ctx, p, logk3, grid, fluid, seal=None, pref=None):
        p, seal = p.contiguous(), None if seal is None else seal.contiguous()
        k = torch.exp(logk3).contiguous()
        r = residual(grid, fluid, k[0], p, seal=seal, pref=pref, ky=k[1], kz=k[2])
        ctx.save_for_backward(p, k)
        ctx.save_for_forward(p, k)
        ctx.cfg = (grid, fluid, seal, pref)
        return r

    @staticmethod
    def backward(ctx, w):
        p, k = ctx.saved_tensors
        grid, fluid, seal, pref = ctx.cfg
        gp, gk = residual_vjp(grid, fluid, k[0], p, w.contiguous(), seal=seal, pref=pref,
                              ky=k[1], kz=k[2], want_p=ctx.needs_input_grad[0],
                              want_logk=ctx.needs_input_grad[1])
        return gp, gk, None, None, None, None

    @staticmethod
    def jvp(ctx, dp, dlogk3, *_):
        if dlogk3 is not None and bool(dlogk3.any()):  # zero tangents are passed too
            raise NotImplementedError("forward-mode derivative with respect to ln k; "
                                      "use reverse mode (backward) for it")
        p, k = ctx.saved_tensors
        grid, fluid, seal, pref = ctx.cfg
        if dp is None:
            return torch.zeros_like(p)
        jv, _ = jvp(grid, fluid, k[0], p, dp.contiguous(), seal=seal, pref=pref, ky=k[1],
                    kz=k[2])
        return jv
