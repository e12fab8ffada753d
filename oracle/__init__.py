"""TPFA flux oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``libtpfa_oracle.so`` (built from ``tpfa_oracle.cpp``
with g++, no GPU code). Only the test suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this package; the GPU library
never does, and this package never imports the GPU library.

Everything is FP64 on host numpy arrays of shape (nz, ny, nx), x fastest.
``grid`` is any object with nx, ny, nz, dx, dy, dz, gk and ``fluid`` any object
with rho0, cf, p0, mu (the ``geomodel`` dataclasses fit).

See ``tpfa_oracle.cpp`` for the equations followed (paper Sec. 3, Eqs. 3-5,
Algorithm 1) and the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tpfa_oracle.cpp")
LIB = os.path.join(HERE, "libtpfa_oracle.so")

# Plain build: no fast-math, no FMA contraction, so every operation is the
# IEEE-rounded operation written in the source.
BUILD_CMD = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-Wextra", SRC, "-o", LIB]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = BUILD_CMD[:-1] + [tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("gk", C.c_double)]


class _Fluid(C.Structure):
    _fields_ = [("rho_ref", C.c_double), ("cf", C.c_double), ("p_ref", C.c_double),
                ("mu", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        lib = C.CDLL(LIB)
        vp = C.c_void_p
        lib.oracle_eval.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp, vp, vp,
                                    C.c_double, C.c_double, vp, vp, vp, vp, vp, vp, vp,
                                    vp, vp, vp]
        lib.oracle_rows.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp, vp, vp,
                                    C.c_double, C.c_double, vp, vp, vp, vp, C.c_int64,
                                    vp, vp, vp, vp]
        lib.oracle_eval_ld.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                       C.c_double, C.c_double, vp, vp, vp, vp]
        lib.oracle_eval_cs.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                       C.c_double, C.c_double, vp, vp, vp, vp,
                                       C.c_double, vp, vp]
        lib.oracle_hydrostatic.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid),
                                           C.c_double, vp]
        lib.oracle_residual10.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp, C.c_double,
                                          C.c_double, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_residual10_cs.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                             C.c_double, C.c_double, vp, vp, vp, vp, vp,
                                             C.c_double, vp]
        lib.oracle_eval_be.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp, C.c_double,
                                       C.c_double, vp, vp, vp, vp, C.c_double, C.c_double,
                                       vp, vp, vp, vp, vp]
        lib.oracle_eval_be_cs.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                          C.c_double, C.c_double, vp, vp, vp, vp, C.c_double,
                                          C.c_double, vp, C.c_double, vp]
        lib.oracle_eval_general.argtypes = ([C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                             C.c_double, C.c_double] + [vp] * 9 +
                                            [C.c_double, C.c_double] + [vp] * 5)
        lib.oracle_eval_general_cs.argtypes = ([C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                                C.c_double, C.c_double] + [vp] * 9 +
                                               [C.c_double, C.c_double, vp, C.c_double, vp])
        lib.oracle_vjp_general.argtypes = ([C.POINTER(_Grid), C.POINTER(_Fluid), vp,
                                            C.c_double, C.c_double] + [vp] * 9)
        lib.oracle_eval_k3.argtypes = ([C.POINTER(_Grid), C.POINTER(_Fluid)] + [vp] * 9 +
                                       [C.c_double, C.c_double] + [vp] * 9)
        lib.oracle_eval_k3_cs.argtypes = ([C.POINTER(_Grid), C.POINTER(_Fluid)] + [vp] * 9 +
                                          [C.c_double, C.c_double, vp, vp, C.c_double, vp])
        lib.oracle_eval_k3.restype = C.c_int
        lib.oracle_eval_k3_cs.restype = C.c_int
        lib.oracle_trans_cs.argtypes = [C.POINTER(_Grid), C.POINTER(_Fluid), vp, vp, vp, vp, vp,
                                        C.c_double, vp]
        lib.oracle_vjp_general.restype = C.c_int
        lib.oracle_trans_cs.restype = C.c_int
        lib.oracle_eval_general.restype = C.c_int
        lib.oracle_eval_general_cs.restype = C.c_int
        for fn in ("oracle_eval", "oracle_rows", "oracle_eval_ld", "oracle_eval_cs",
                   "oracle_hydrostatic", "oracle_residual10", "oracle_residual10_cs",
                   "oracle_eval_be", "oracle_eval_be_cs"):
            getattr(lib, fn).restype = C.c_int
        _lib = lib
    return _lib


def _g(grid) -> _Grid:
    return _Grid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.dx),
                 float(grid.dy), float(grid.dz), float(grid.gk))


def _f(fluid) -> _Fluid:
    return _Fluid(float(fluid.rho0), float(fluid.cf), float(fluid.p0), float(fluid.mu))


def _arr(a, dtype, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None and a.size != int(np.prod(shape)):
        raise ValueError(f"array of size {a.size} does not match {shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def evaluate(grid, fluid, kx, p, *, ry=1.0, rz=1.0, seal=None, ky=None, kz=None,
             w=None, force=None, want=("r", "J")) -> dict:
    """Residual and any of: J [7, nz, ny, nx], grad_p, grad_logk (need w),
    scale [2, ...] (sum |F|, sum |dF/dp_K|), dphi [3, ...] (face potential
    differences, NaN where no face). ``force`` is an int8 [3, ...] upwind
    override per face (+1 lower cell, -1 upper cell, 0 rule)."""
    shape = (grid.nz, grid.ny, grid.nx)
    n = int(np.prod(shape))
    kx = _arr(kx, np.float64, shape)
    p = _arr(p, np.float64, shape)
    ky = _arr(ky, np.float64, shape)
    kz = _arr(kz, np.float64, shape)
    seal = _arr(seal, np.uint8, shape)
    w = _arr(w, np.float64, shape)
    force = _arr(force, np.int8, (3,) + shape)
    out = {}
    bufs = {}
    for key, sh in (("r", shape), ("J", (7,) + shape), ("grad_p", shape),
                    ("grad_logk", shape), ("scale", (2,) + shape), ("dphi", (3,) + shape)):
        bufs[key] = np.empty(sh, np.float64) if key in want else None
    rc = _load().oracle_eval(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx), _ptr(ky),
                             _ptr(kz), float(ry), float(rz), _ptr(seal), _ptr(p),
                             _ptr(force), _ptr(w), _ptr(bufs["r"]), _ptr(bufs["J"]),
                             _ptr(bufs["grad_p"]), _ptr(bufs["grad_logk"]),
                             _ptr(bufs["scale"]), _ptr(bufs["dphi"]))
    if rc != 0:
        raise ValueError("oracle_eval rejected its arguments")
    for key in want:
        out[key] = bufs[key]
    assert n > 0
    return out


def rows(grid, fluid, kx, p, cells, *, ry=1.0, rz=1.0, seal=None, ky=None, kz=None,
         force=None, with_dphi=False):
    """(r[n], J[7, n], scale[2, n]) for the listed linear cell indices, plus
    dphi[6, n] (face potential differences seen from each cell, NaN where no
    face) when ``with_dphi``."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx = _arr(kx, np.float64, shape)
    p = _arr(p, np.float64, shape)
    ky = _arr(ky, np.float64, shape)
    kz = _arr(kz, np.float64, shape)
    seal = _arr(seal, np.uint8, shape)
    force = _arr(force, np.int8, (3,) + shape)
    cells = np.ascontiguousarray(cells, dtype=np.int64).ravel()
    n = cells.size
    r = np.empty(n)
    J = np.empty((7, n))
    s = np.empty((2, n))
    d = np.empty((6, n)) if with_dphi else None
    rc = _load().oracle_rows(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx), _ptr(ky),
                             _ptr(kz), float(ry), float(rz), _ptr(seal), _ptr(p),
                             _ptr(force), _ptr(cells), n, _ptr(r), _ptr(J), _ptr(s), _ptr(d))
    if rc != 0:
        raise ValueError("oracle_rows rejected its arguments")
    if with_dphi:
        return r, J, s, d
    return r, J, s


def evaluate_ld(grid, fluid, kx, p, *, ry=1.0, rz=1.0, seal=None):
    """Residual and Jacobian in long double (x87 80-bit on x86-64)."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx = _arr(kx, np.float64, shape)
    p = _arr(p, np.float64, shape)
    seal = _arr(seal, np.uint8, shape)
    r = np.empty(shape, np.longdouble)
    J = np.empty((7,) + shape, np.longdouble)
    rc = _load().oracle_eval_ld(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx),
                                float(ry), float(rz), _ptr(seal), _ptr(p), _ptr(r), _ptr(J))
    if rc != 0:
        raise ValueError("oracle_eval_ld rejected its arguments")
    return r, J


def evaluate_cs(grid, fluid, kx, p, *, ry=1.0, rz=1.0, seal=None, vp=None, vm=None,
                h=1e-20):
    """Complex-step residual: returns (Re r, Im r / h) for the perturbation
    p + i h vp, ln kx + i h vm."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx = _arr(kx, np.float64, shape)
    p = _arr(p, np.float64, shape)
    seal = _arr(seal, np.uint8, shape)
    vp = _arr(vp, np.float64, shape)
    vm = _arr(vm, np.float64, shape)
    re = np.empty(shape)
    im = np.empty(shape)
    rc = _load().oracle_eval_cs(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx),
                                float(ry), float(rz), _ptr(seal), _ptr(p), _ptr(vp),
                                _ptr(vm), float(h), _ptr(re), _ptr(im))
    if rc != 0:
        raise ValueError("oracle_eval_cs rejected its arguments")
    return re, im / h


def residual10(grid, fluid, kx, p, tne, tse, *, ry=1.0, rz=1.0, seal=None, force=None):
    """Residual of the 10-flux stencil (six TPFA faces plus the four in-plane
    diagonal faces with given transmissibilities) and its flux scale sum |F|.
    ``force`` is an int8 [5, ...] upwind override per face (+1 lower cell, -1
    upper cell, 0 rule): x, y, z faces by their lower cell, then the faces
    (i,j)-(i+1,j+1) and (i,j)-(i+1,j-1) by their (i, j) end."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx, p = _arr(kx, np.float64, shape), _arr(p, np.float64, shape)
    tne, tse = _arr(tne, np.float64, shape), _arr(tse, np.float64, shape)
    seal = _arr(seal, np.uint8, shape)
    force = _arr(force, np.int8, (5,) + shape)
    r = np.empty(shape)
    scale = np.empty((2,) + shape)
    rc = _load().oracle_residual10(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx), float(ry),
                                   float(rz), _ptr(seal), _ptr(tne), _ptr(tse), _ptr(p),
                                   _ptr(force), _ptr(r), _ptr(scale))
    if rc != 0:
        raise ValueError("oracle_residual10 rejected its arguments")
    return r, scale[0]


def residual10_cs(grid, fluid, kx, p, tne, tse, vp, *, ry=1.0, rz=1.0, seal=None, h=1e-20):
    """Complex-step directional derivative of the 10-flux residual along vp."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx, p = _arr(kx, np.float64, shape), _arr(p, np.float64, shape)
    tne, tse = _arr(tne, np.float64, shape), _arr(tse, np.float64, shape)
    vp, seal = _arr(vp, np.float64, shape), _arr(seal, np.uint8, shape)
    im = np.empty(shape)
    rc = _load().oracle_residual10_cs(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx),
                                      float(ry), float(rz), _ptr(seal), _ptr(tne), _ptr(tse),
                                      _ptr(p), _ptr(vp), float(h), _ptr(im))
    if rc != 0:
        raise ValueError("oracle_residual10_cs rejected its arguments")
    return im / h


def evaluate_be(grid, fluid, kx, p, phi, p_prev, dt, cr, *, ry=1.0, rz=1.0, seal=None,
                v=None, want=("r", "J")) -> dict:
    """Full backward-Euler residual of Eq. (2) (accumulation + flux sum) and any
    of: J [7, ...] (with the accumulation derivative on the diagonal), jv = J v
    (needs v), scale [2, ...] (sum of |terms| of r and of the diagonal)."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx, p = _arr(kx, np.float64, shape), _arr(p, np.float64, shape)
    phi, p_prev = _arr(phi, np.float64, shape), _arr(p_prev, np.float64, shape)
    seal, v = _arr(seal, np.uint8, shape), _arr(v, np.float64, shape)
    bufs = {}
    for key, sh in (("r", shape), ("J", (7,) + shape), ("jv", shape), ("scale", (2,) + shape)):
        bufs[key] = np.empty(sh, np.float64) if key in want else None
    rc = _load().oracle_eval_be(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx), float(ry),
                                float(rz), _ptr(seal), _ptr(p), _ptr(phi), _ptr(p_prev),
                                float(dt), float(cr), _ptr(v), _ptr(bufs["r"]),
                                _ptr(bufs["J"]), _ptr(bufs["jv"]), _ptr(bufs["scale"]))
    if rc != 0:
        raise ValueError("oracle_eval_be rejected its arguments")
    return {k: bufs[k] for k in want}


def evaluate_be_cs(grid, fluid, kx, p, phi, p_prev, dt, cr, vp, *, ry=1.0, rz=1.0, seal=None,
                   h=1e-20) -> np.ndarray:
    """Complex-step J vp of the full backward-Euler residual."""
    shape = (grid.nz, grid.ny, grid.nx)
    kx, p = _arr(kx, np.float64, shape), _arr(p, np.float64, shape)
    phi, p_prev = _arr(phi, np.float64, shape), _arr(p_prev, np.float64, shape)
    seal, vp = _arr(seal, np.uint8, shape), _arr(vp, np.float64, shape)
    im = np.empty(shape)
    rc = _load().oracle_eval_be_cs(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx), float(ry),
                                   float(rz), _ptr(seal), _ptr(p), _ptr(phi), _ptr(p_prev),
                                   float(dt), float(cr), _ptr(vp), float(h), _ptr(im))
    if rc != 0:
        raise ValueError("oracle_eval_be_cs rejected its arguments")
    return im / h


def _general_args(grid, p, kx, trans, seal, diag, accum, ry, rz):
    shape = (grid.nz, grid.ny, grid.nx)
    tx, ty, tz = (None, None, None) if trans is None else trans
    tne, tse = (None, None) if diag is None else diag
    acc = accum or {}
    arrs = [_arr(a, np.float64, shape) for a in (kx, tx, ty, tz, tne, tse, p,
                                                   acc.get("phi"), acc.get("p_prev"))]
    seal = _arr(seal, np.uint8, shape)
    kx, tx, ty, tz, tne, tse, p, phi, pn = arrs
    head = [_ptr(kx), float(ry), float(rz), _ptr(seal), _ptr(tx), _ptr(ty), _ptr(tz), _ptr(tne),
            _ptr(tse), _ptr(p), _ptr(phi), _ptr(pn), float(acc.get("dt", 1.0)),
            float(acc.get("cr", 0.0))]
    return shape, head, arrs + [seal]


def evaluate_general(grid, fluid, p, *, kx=None, trans=None, ry=1.0, rz=1.0, seal=None,
                     diag=None, accum=None, v=None, want=("r",)) -> dict:
    """The residual in any input form: permeability (kx, ry, rz, seal) or face
    transmissibilities ``trans`` = (tx, ty, tz); optional diagonal faces
    ``diag`` = (tne, tse); optional accumulation ``accum`` = dict(phi, p_prev,
    dt, cr). Outputs any of r, J, jv (needs v), scale."""
    shape, head, keep = _general_args(grid, p, kx, trans, seal, diag, accum, ry, rz)
    v = _arr(v, np.float64, shape)
    bufs = {}
    for key, sh in (("r", shape), ("J", (7,) + shape), ("jv", shape), ("scale", (2,) + shape)):
        bufs[key] = np.empty(sh, np.float64) if key in want else None
    rc = _load().oracle_eval_general(C.byref(_g(grid)), C.byref(_f(fluid)), *head, _ptr(v),
                                     _ptr(bufs["r"]), _ptr(bufs["J"]), _ptr(bufs["jv"]),
                                     _ptr(bufs["scale"]))
    if rc != 0:
        raise ValueError("oracle_eval_general rejected its arguments")
    return {k: bufs[k] for k in want}


def evaluate_general_cs(grid, fluid, p, vp, *, kx=None, trans=None, ry=1.0, rz=1.0, seal=None,
                        diag=None, accum=None, h=1e-20) -> np.ndarray:
    """Complex-step J vp of the general residual."""
    shape, head, keep = _general_args(grid, p, kx, trans, seal, diag, accum, ry, rz)
    vp = _arr(vp, np.float64, shape)
    im = np.empty(shape)
    rc = _load().oracle_eval_general_cs(C.byref(_g(grid)), C.byref(_f(fluid)), *head, _ptr(vp),
                                        float(h), _ptr(im))
    if rc != 0:
        raise ValueError("oracle_eval_general_cs rejected its arguments")
    return im / h


def vjp_general(grid, fluid, p, w, *, kx=None, trans=None, ry=1.0, rz=1.0, seal=None):
    """grad_p = J^T w in either rock form; with ``trans`` also grad_t [3, ...]
    (gradient with respect to ln T of each cell's +x, +y, +z face) and its
    scale (sum of |terms|). Returns (grad_p, grad_t, grad_t_scale)."""
    shape = (grid.nz, grid.ny, grid.nx)
    tx, ty, tz = (None, None, None) if trans is None else trans
    kx, tx, ty, tz, p, w = (_arr(a, np.float64, shape) for a in (kx, tx, ty, tz, p, w))
    seal = _arr(seal, np.uint8, shape)
    gp = np.empty(shape)
    gt = np.empty((3,) + shape) if trans is not None else None
    gs = np.empty((3,) + shape) if trans is not None else None
    rc = _load().oracle_vjp_general(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(kx), float(ry),
                                    float(rz), _ptr(seal), _ptr(tx), _ptr(ty), _ptr(tz), _ptr(p),
                                    _ptr(w), _ptr(gp), _ptr(gt), _ptr(gs))
    if rc != 0:
        raise ValueError("oracle_vjp_general rejected its arguments")
    return gp, gt, gs


def trans_cs(grid, fluid, p, trans, d, h=1e-20) -> np.ndarray:
    """Complex-step derivative of the transmissibility-form residual along the
    ln T direction d [3, ...]: returns d r / d(ln T) . d."""
    shape = (grid.nz, grid.ny, grid.nx)
    tx, ty, tz = (_arr(a, np.float64, shape) for a in trans)
    p = _arr(p, np.float64, shape)
    d = np.ascontiguousarray(d, np.float64)
    im = np.empty(shape)
    rc = _load().oracle_trans_cs(C.byref(_g(grid)), C.byref(_f(fluid)), _ptr(tx), _ptr(ty),
                                 _ptr(tz), _ptr(p), _ptr(d), float(h), _ptr(im))
    if rc != 0:
        raise ValueError("oracle_trans_cs rejected its arguments")
    return im / h


def _k3_args(grid, p, kx, ky, kz, seal, diag, accum):
    shape = (grid.nz, grid.ny, grid.nx)
    tne, tse = (None, None) if diag is None else diag
    acc = accum or {}
    arrs = [_arr(a, np.float64, shape) for a in (kx, ky, kz, tne, tse, p, acc.get("phi"),
                                                   acc.get("p_prev"))]
    seal = _arr(seal, np.uint8, shape)
    kx, ky, kz, tne, tse, p, phi, pn = arrs
    head = [_ptr(kx), _ptr(ky), _ptr(kz), _ptr(seal), _ptr(tne), _ptr(tse), _ptr(p), _ptr(phi),
            _ptr(pn), float(acc.get("dt", 1.0)), float(acc.get("cr", 0.0))]
    return shape, head, arrs + [seal]


def evaluate_k3(grid, fluid, p, kx, ky, kz, *, seal=None, diag=None, accum=None, v=None,
                w=None, want=("r",)) -> dict:
    """Per-direction permeability form (kx, ky, kz per cell, no ratios), with
    seal bits, optional diagonal faces ``diag`` = (tne, tse) and accumulation
    ``accum`` = dict(phi, p_prev, dt, cr). Outputs any of r, J, jv (needs v),
    scale, and with the cotangent w: grad_p = J^T w, grad_k3 [3, ...] =
    d(w.r)/d ln k_a for a = x, y, z, grad_k3_scale (sum of |terms|)."""
    shape, head, keep = _k3_args(grid, p, kx, ky, kz, seal, diag, accum)
    v = _arr(v, np.float64, shape)
    w = _arr(w, np.float64, shape)
    bufs = {}
    for key, sh in (("r", shape), ("J", (7,) + shape), ("jv", shape), ("scale", (2,) + shape),
                    ("grad_p", shape), ("grad_k3", (3,) + shape),
                    ("grad_k3_scale", (3,) + shape)):
        bufs[key] = np.empty(sh, np.float64) if key in want else None
    rc = _load().oracle_eval_k3(C.byref(_g(grid)), C.byref(_f(fluid)), *head, _ptr(v), _ptr(w),
                                *(_ptr(bufs[k]) for k in ("r", "J", "jv", "scale", "grad_p",
                                                          "grad_k3", "grad_k3_scale")))
    if rc != 0:
        raise ValueError("oracle_eval_k3 rejected its arguments")
    return {k: bufs[k] for k in want}


def evaluate_k3_cs(grid, fluid, p, kx, ky, kz, *, seal=None, diag=None, accum=None, vp=None,
                   dk=None, h=1e-20) -> np.ndarray:
    """Complex-step directional derivative of the per-direction form along
    vp (pressure) and dk [3, ...] (ln kx, ln ky, ln kz): Im r / h."""
    shape, head, keep = _k3_args(grid, p, kx, ky, kz, seal, diag, accum)
    vp = _arr(vp, np.float64, shape)
    dk = _arr(dk, np.float64, (3,) + shape)
    im = np.empty(shape)
    rc = _load().oracle_eval_k3_cs(C.byref(_g(grid)), C.byref(_f(fluid)), *head, _ptr(vp),
                                   _ptr(dk), float(h), _ptr(im))
    if rc != 0:
        raise ValueError("oracle_eval_k3_cs rejected its arguments")
    return im / h


def hydrostatic(grid, fluid, p_top: Optional[float] = None) -> np.ndarray:
    """Discrete hydrostatic reference profile pref[nz] (FP64)."""
    pref = np.empty(int(grid.nz))
    top = float(fluid.p0 if p_top is None else p_top)
    rc = _load().oracle_hydrostatic(C.byref(_g(grid)), C.byref(_f(fluid)), top, _ptr(pref))
    if rc != 0:
        raise ValueError("oracle_hydrostatic rejected its arguments")
    return pref


def pressure(geo, r: int = 0) -> np.ndarray:
    """Pressure field r of a geomodel: hydrostatic reference plus noise."""
    pref = hydrostatic(geo.grid, geo.fluid, geo.p_top)
    return pref[:, None, None] + geo.noise[r]


def widen_fp32(dp32: np.ndarray, pref: np.ndarray) -> np.ndarray:
    """FP64 pressure seen by the precision form: pref[k] + (double) dp."""
    return pref[:, None, None] + dp32.astype(np.float64)
