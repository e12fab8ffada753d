"""C-ABI checks that need no GPU: libtpfa.so loads, exports every function
declared in include/tpfa.h, and rejects invalid arguments on the host with the
documented error codes before anything is enqueued."""
import ctypes as C
import math
import os
import re

import pytest

import paper_2304_11274_amd as tp
from paper_2304_11274_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpfa.h")
DUMMY = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpfa_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding signatures out of sync with the header"


def test_constants_match_the_header():
    """Every #define and enumerator value of include/tpfa.h that the binding
    mirrors equals the binding's constant."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    found = {}
    for name, val in re.findall(r"#define\s+(TPFA_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text):
        found[name] = int(val)
    for name, val in re.findall(r"\b(TPFA_[A-Z0-9_]+)\s*=\s*(-?\d+)", text):
        found[name] = int(val)
    mirrored = {n: getattr(L, n) for n in dir(L) if n.startswith("TPFA_") and n in found}
    assert len(mirrored) >= 25, sorted(mirrored)
    for n, v in mirrored.items():
        assert found[n] == v, (n, found[n], v)
    missing = sorted(n for n in found if n.startswith(("TPFA_LAUNCH_", "TPFA_ERR_", "TPFA_OP_"))
                     and not hasattr(L, n))
    assert not missing, missing


def test_introspection(lib):
    assert lib.tpfa_version() // 10000 == L.ABI_MAJOR
    # the header's version is the one the library was built with
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "tpfa.h")).read()
    assert f"#define TPFA_VERSION {lib.tpfa_version()}" in hdr
    shapes = tp.tile_shapes()
    assert len(shapes) == lib.tpfa_num_tiles()
    for tx, ty, th in shapes:
        assert tx * ty == th and th in (256, 512)
    assert lib.tpfa_tile_shape(-1, None, None, None) == L.TPFA_ERR_TILE
    assert lib.tpfa_tile_shape(lib.tpfa_num_tiles(), None, None, None) == L.TPFA_ERR_TILE
    for code in range(0, -7, -1):
        assert lib.tpfa_strerror(code)
    assert b"unknown" in lib.tpfa_strerror(-99)


def good():
    g = L.Grid(8, 8, 8, 10.0, 10.0, 2.0, 9.81)
    f = L.Fluid(1000.0, 1e-9, 1e7, 1e-3)
    rk = L.Rock(DUMMY, None, None, 1.0, 0.1, None)
    st = L.State(DUMMY, None)
    return g, f, rk, st


def call_res(lib, g, f, rk, st, prec=L.TPFA_FP64, r=DUMMY, launch=None):
    return lib.tpfa_residual(None if g is None else C.byref(g), None if f is None else C.byref(f),
                             None if rk is None else C.byref(rk),
                             None if st is None else C.byref(st), prec, r,
                             None if launch is None else C.byref(launch), None)


def case(name, code, **mut):
    return pytest.param(mut, code, id=name)


@pytest.mark.parametrize("mut,code", [
    case("grid-null", L.TPFA_ERR_NULL, grid=None),
    case("fluid-null", L.TPFA_ERR_NULL, fluid=None),
    case("rock-null", L.TPFA_ERR_NULL, rock=None),
    case("state-null", L.TPFA_ERR_NULL, state=None),
    case("nx-zero", L.TPFA_ERR_SHAPE, nx=0),
    case("nz-negative", L.TPFA_ERR_SHAPE, nz=-3),
    case("nx-over-int32", L.TPFA_ERR_SHAPE, nx=2**31),
    case("ncell-overflow", L.TPFA_ERR_SHAPE, nx=2**31 - 1, ny=2**31 - 1, nz=2**31 - 1),
    case("ldx-below-nx", L.TPFA_ERR_SHAPE, ldx=7),
    case("ldx-negative", L.TPFA_ERR_SHAPE, ldx=-8),
    case("ldx-over-int32", L.TPFA_ERR_SHAPE, ldx=2**31),
    case("pitched-overflow", L.TPFA_ERR_SHAPE, ldx=2**31 - 1, ny=2**31 - 1, nz=2**31 - 1),
    case("pitched-r-null", L.TPFA_ERR_NULL, ldx=40, r=None),
    case("dx-zero", L.TPFA_ERR_PARAM, dx=0.0),
    case("dz-nan", L.TPFA_ERR_PARAM, dz=math.nan),
    case("gk-inf", L.TPFA_ERR_PARAM, gk=math.inf),
    case("mu-zero", L.TPFA_ERR_PARAM, mu=0.0),
    case("mu-negative", L.TPFA_ERR_PARAM, mu=-1e-3),
    case("cf-nan", L.TPFA_ERR_PARAM, cf=math.nan),
    case("ry-negative", L.TPFA_ERR_PARAM, ry=-1.0),
    case("rz-nan", L.TPFA_ERR_PARAM, rz=math.nan),
    case("kx-null", L.TPFA_ERR_NULL, kx=None),
    case("ky-without-kz", L.TPFA_ERR_NULL, ky=DUMMY),
    case("kz-without-ky", L.TPFA_ERR_NULL, kz=DUMMY),
    case("p-null", L.TPFA_ERR_NULL, p=None),
    case("fp32-no-pref", L.TPFA_ERR_UNSUPPORTED, prec=L.TPFA_FP32),
    case("unknown-precision", L.TPFA_ERR_PARAM, prec=7),
    case("r-null", L.TPFA_ERR_NULL, r=None),
    case("tile-unknown", L.TPFA_ERR_TILE, launch=(99, 0, 0)),
    case("tile-below", L.TPFA_ERR_TILE, launch=(-2, 0, 0)),
    case("kz-negative", L.TPFA_ERR_TILE, launch=(0, -1, 0)),
    case("rows-begin-negative", L.TPFA_ERR_PARAM, launch=(-1, 0, 0, -1, 4)),
    case("rows-past-ny", L.TPFA_ERR_PARAM, launch=(-1, 0, 0, 0, 9)),
    case("rows-empty", L.TPFA_ERR_PARAM, launch=(-1, 0, 0, 4, 4)),
    case("rows-end-missing", L.TPFA_ERR_PARAM, launch=(-1, 0, 0, 3, 0)),
])
def test_residual_validation(lib, mut, code):
    g, f, rk, st = good()
    prec, r, launch = L.TPFA_FP64, DUMMY, None
    for k, v in mut.items():
        if k == "grid":
            g = v
        elif k == "fluid":
            f = v
        elif k == "rock":
            rk = v
        elif k == "state":
            st = v
        elif k in ("nx", "ny", "nz", "dx", "dy", "dz", "gk", "ldx"):
            setattr(g, k, v)
        elif k in ("mu", "cf", "rho0", "p0"):
            setattr(f, k, v)
        elif k in ("kx", "ky", "kz", "ry", "rz"):
            setattr(rk, k, v if not isinstance(v, C.c_void_p) else v.value)
        elif k == "p":
            st.p = v
        elif k == "prec":
            prec = v
        elif k == "r":
            r = v
        elif k == "launch":
            launch = L.Launch(*v)
    rc = call_res(lib, g, f, rk, st, prec=prec, r=r, launch=launch)
    assert rc == code, lib.tpfa_last_error()
    assert lib.tpfa_last_error()  # a detail message is always set


def test_jacobian_and_vjp_validation(lib):
    g, f, rk, st = good()
    args = (C.byref(g), C.byref(f), C.byref(rk), C.byref(st), L.TPFA_FP64)
    assert lib.tpfa_jacobian(*args, DUMMY, None, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual_vjp(*args, None, DUMMY, DUMMY, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual_vjp(*args, DUMMY, None, None, None, None) == L.TPFA_ERR_NULL
    rk2 = L.Rock(DUMMY.value, DUMMY.value, None, 1.0, 1.0, None)  # ky without kz
    assert lib.tpfa_residual_vjp(C.byref(g), C.byref(f), C.byref(rk2), C.byref(st),
                                 L.TPFA_FP64, DUMMY, DUMMY, DUMMY, None,
                                 None) == L.TPFA_ERR_NULL
    g.nz = 0
    assert lib.tpfa_jacobian(*args, DUMMY, DUMMY, None, None) == L.TPFA_ERR_SHAPE


def test_sliced_validation(lib):
    """TPFA_LAUNCH_SLICED: Jacobian calls only, r NULL, one z plane of the
    sliced array below 2^32 bytes."""
    g, f, rk, st = good()
    args = (C.byref(g), C.byref(f), C.byref(rk), C.byref(st), L.TPFA_FP64)
    ln = L.Launch(-1, 0, L.TPFA_LAUNCH_SLICED, 0, 0)
    assert lib.tpfa_jacobian(*args, DUMMY, DUMMY, C.byref(ln), None) == L.TPFA_ERR_PARAM
    assert b"r = NULL" in lib.tpfa_last_error()
    assert lib.tpfa_residual(*args, DUMMY, C.byref(ln), None) == L.TPFA_ERR_UNSUPPORTED
    assert lib.tpfa_residual_vjp(*args, DUMMY, DUMMY, DUMMY, C.byref(ln),
                                 None) == L.TPFA_ERR_UNSUPPORTED
    # 2^16 cells per row (1024 slices) and 1024 rows in FP64: 2^32 bytes per plane
    big = L.Grid(65536, 1024, 2, 10.0, 10.0, 2.0, 9.81)
    assert lib.tpfa_jacobian(C.byref(big), C.byref(f), C.byref(rk), C.byref(st), L.TPFA_FP64,
                             None, DUMMY, C.byref(ln), None) == L.TPFA_ERR_SHAPE


def test_residual_and_vjp_validation(lib):
    g, f, rk, st = good()
    args = (C.byref(g), C.byref(f), C.byref(rk), C.byref(st), L.TPFA_FP64)
    fn = lib.tpfa_residual_and_vjp
    assert fn(*args, None, DUMMY, DUMMY, DUMMY, None, None) == L.TPFA_ERR_NULL  # w
    assert fn(*args, DUMMY, None, DUMMY, DUMMY, None, None) == L.TPFA_ERR_NULL  # r
    assert fn(*args, DUMMY, DUMMY, None, None, None, None) == L.TPFA_ERR_NULL  # both grads
    k3 = L.Rock(DUMMY.value, DUMMY.value, DUMMY.value, 1.0, 1.0, None)
    assert fn(C.byref(g), C.byref(f), C.byref(k3), C.byref(st), L.TPFA_FP64, DUMMY, DUMMY,
              DUMMY, DUMMY, None, None) == L.TPFA_ERR_UNSUPPORTED
    tr = L.Rock(None, None, None, 1.0, 1.0, None, DUMMY.value, DUMMY.value, DUMMY.value)
    assert fn(C.byref(g), C.byref(f), C.byref(tr), C.byref(st), L.TPFA_FP64, DUMMY, DUMMY,
              DUMMY, DUMMY, None, None) == L.TPFA_ERR_UNSUPPORTED
    ln = L.Launch(-1, 0, L.TPFA_LAUNCH_SLICED, 0, 0)
    assert fn(*args, DUMMY, DUMMY, DUMMY, DUMMY, C.byref(ln), None) == L.TPFA_ERR_UNSUPPORTED


def test_helpers_validation(lib):
    g, f, _, _ = good()
    assert lib.tpfa_hydrostatic(C.byref(g), C.byref(f), 1e7, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_hydrostatic(C.byref(g), C.byref(f), math.inf, DUMMY, None) == L.TPFA_ERR_PARAM
    assert lib.tpfa_hydrostatic(None, C.byref(f), 1e7, DUMMY, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_offset_pressure(C.byref(g), None, DUMMY, DUMMY, None) == L.TPFA_ERR_NULL
    g.ny = 0
    assert lib.tpfa_offset_pressure(C.byref(g), DUMMY, DUMMY, DUMMY, None) == L.TPFA_ERR_SHAPE


def test_stream_probe_validation(lib):
    g, _, _, _ = good()
    assert lib.tpfa_stream_probe(None, L.TPFA_FP64, DUMMY, DUMMY, DUMMY, DUMMY, None) == \
        L.TPFA_ERR_NULL
    assert lib.tpfa_stream_probe(C.byref(g), 7, DUMMY, DUMMY, DUMMY, DUMMY, None) == \
        L.TPFA_ERR_PARAM
    for q in range(4):
        ptrs = [DUMMY] * 4
        ptrs[q] = None
        assert lib.tpfa_stream_probe(C.byref(g), L.TPFA_FP32, *ptrs, None) == L.TPFA_ERR_NULL
    g.nz = 0
    assert lib.tpfa_stream_probe(C.byref(g), L.TPFA_FP64, DUMMY, DUMMY, DUMMY, DUMMY, None) == \
        L.TPFA_ERR_SHAPE
    assert lib.tpfa_stream_probe_sliced(C.byref(g), L.TPFA_FP64, DUMMY, DUMMY, DUMMY, DUMMY,
                                        None) == L.TPFA_ERR_SHAPE
    g.nz = 8
    assert lib.tpfa_stream_probe_sliced(C.byref(g), 7, DUMMY, DUMMY, DUMMY, DUMMY,
                                        None) == L.TPFA_ERR_PARAM
    assert lib.tpfa_stream_probe_sliced(C.byref(g), L.TPFA_FP64, None, DUMMY, DUMMY, DUMMY,
                                        None) == L.TPFA_ERR_NULL
    big = L.Grid(65536, 1024, 2, 10.0, 10.0, 2.0, 9.81)  # 2^32 bytes per sliced FP64 plane
    assert lib.tpfa_stream_probe_sliced(C.byref(big), L.TPFA_FP64, DUMMY, DUMMY, DUMMY, DUMMY,
                                        None) == L.TPFA_ERR_SHAPE
    import torch
    import geomodel
    t = torch.zeros((2, 2, 2), dtype=torch.float64)
    with pytest.raises(ValueError):
        tp.stream_probe(geomodel.Grid(2, 2, 2), t, t, t.to(torch.uint8))   # host tensors


def test_noalloc_run_validation(lib):
    g, f, rk, st = good()
    m = (L.Model * 257)()
    for q in range(257):
        m[q] = L.Model(g, f, rk, st, DUMMY.value, DUMMY.value, L.Launch(-1, 0, 0))
    J = L.TPFA_BATCH_JACOBIAN
    assert lib.tpfa_ensemble_run_noalloc(m, 257, L.TPFA_FP64, J, None) == L.TPFA_ERR_SHAPE
    assert b"at most 256" in lib.tpfa_last_error()
    assert lib.tpfa_ensemble_run_noalloc(None, 2, L.TPFA_FP64, J, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_ensemble_run_noalloc(m, 0, L.TPFA_FP64, J, None) == L.TPFA_ERR_SHAPE
    assert lib.tpfa_ensemble_run_noalloc(m, 2, L.TPFA_FP64, 5, None) == L.TPFA_ERR_PARAM
    m[1].launch = L.Launch(6, 0, 0)  # a tile the ensemble kernels do not hold
    assert lib.tpfa_ensemble_run_noalloc(m, 2, L.TPFA_FP64, J, None) == L.TPFA_ERR_TILE
    m[1].launch = L.Launch(-1, 0, 0)
    m[1].J = None
    assert lib.tpfa_ensemble_run_noalloc(m, 2, L.TPFA_FP64, J, None) == L.TPFA_ERR_NULL
    assert b"model 1" in lib.tpfa_last_error()


def test_batch_validation(lib):
    g, f, rk, st = good()
    out = C.c_void_p()
    m = (L.Model * 2)()
    for q in range(2):
        m[q] = L.Model(g, f, rk, st, DUMMY.value, DUMMY.value, L.Launch(-1, 0, 0))
    J = L.TPFA_BATCH_JACOBIAN
    assert lib.tpfa_batch_create(m, 2, L.TPFA_FP64, J, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_batch_create(None, 2, L.TPFA_FP64, J, C.byref(out), None) == L.TPFA_ERR_NULL
    assert lib.tpfa_batch_create(m, 0, L.TPFA_FP64, J, C.byref(out), None) == L.TPFA_ERR_SHAPE
    assert lib.tpfa_batch_create(m, 2, L.TPFA_FP64, 5, C.byref(out), None) == L.TPFA_ERR_PARAM
    m[1].launch = L.Launch(3, 0, 0)  # a 512-thread tile
    assert lib.tpfa_batch_create(m, 2, L.TPFA_FP64, J, C.byref(out), None) == L.TPFA_ERR_TILE
    m[1].launch = L.Launch(-1, 0, 0)
    m[1].J = None
    assert lib.tpfa_batch_create(m, 2, L.TPFA_FP64, J, C.byref(out), None) == L.TPFA_ERR_NULL
    assert b"model 1" in lib.tpfa_last_error()
    m[1].grid.nx = 0
    m[1].J = DUMMY.value
    assert lib.tpfa_batch_create(m, 2, L.TPFA_FP64, J, C.byref(out), None) == L.TPFA_ERR_SHAPE
    assert not out.value
    assert lib.tpfa_batch_run(None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_batch_run_eager(None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_batch_info(None, None, None) == L.TPFA_ERR_NULL
    lib.tpfa_batch_destroy(None)


def test_python_binding_rejects_host_tensors():
    import torch
    import geomodel
    g = geomodel.Grid(4, 4, 4)
    t = torch.zeros(64, dtype=torch.float64)
    with pytest.raises(ValueError):
        tp.residual(g, geomodel.Fluid(), t, t)
    with pytest.raises(TypeError):
        tp.residual(g, geomodel.Fluid(), t, t.to(torch.int32))
    # per-direction arrays go together (checked before any tensor is used)
    with pytest.raises(ValueError, match="ky and kz"):
        tp.jacobian(g, geomodel.Fluid(), t, t, ky=t)
    with pytest.raises(ValueError, match="ky and kz"):
        tp.residual_vjp(g, geomodel.Fluid(), t, t, t, kz=t)


def test_residual10_validation(lib):
    g, f, rk, st = good()
    args = (C.byref(g), C.byref(f), C.byref(rk), C.byref(st), L.TPFA_FP64)
    assert lib.tpfa_residual10(*args, None, DUMMY, DUMMY, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual10(*args, DUMMY, None, DUMMY, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual10(*args, DUMMY, DUMMY, None, None, None) == L.TPFA_ERR_NULL
    bad = L.Launch(99, 0, 0)
    assert lib.tpfa_residual10(*args, DUMMY, DUMMY, DUMMY, C.byref(bad), None) == L.TPFA_ERR_TILE
    g.nx = 0
    assert lib.tpfa_residual10(*args, DUMMY, DUMMY, DUMMY, None, None) == L.TPFA_ERR_SHAPE


def test_backward_euler_and_jvp_validation(lib):
    g, f, rk, st = good()
    args = (C.byref(g), C.byref(f), C.byref(rk), C.byref(st))
    acc = L.Accum(DUMMY.value, DUMMY.value, 3600.0, 1e-10)
    P64 = L.TPFA_FP64
    assert lib.tpfa_residual_be(*args, None, P64, DUMMY, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual_be(*args, C.byref(acc), P64, None, None, None) == L.TPFA_ERR_NULL
    for bad in (L.Accum(None, DUMMY.value, 3600.0, 0.0), L.Accum(DUMMY.value, None, 3600.0, 0.0)):
        assert lib.tpfa_residual_be(*args, C.byref(bad), P64, DUMMY, None, None) == L.TPFA_ERR_NULL
    for dt, cr in ((0.0, 0.0), (-1.0, 0.0), (math.inf, 0.0), (math.nan, 0.0), (1.0, math.nan)):
        bad = L.Accum(DUMMY.value, DUMMY.value, dt, cr)
        assert lib.tpfa_residual_be(*args, C.byref(bad), P64, DUMMY, None, None) == L.TPFA_ERR_PARAM
    assert lib.tpfa_jacobian_be(*args, C.byref(acc), P64, DUMMY, None, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_jacobian_be(*args, None, P64, DUMMY, DUMMY, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_jvp(*args, None, P64, None, DUMMY, None, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_jvp(*args, None, P64, DUMMY, None, None, None, None) == L.TPFA_ERR_NULL
    bad = L.Accum(DUMMY.value, DUMMY.value, -5.0, 0.0)
    assert lib.tpfa_jvp(*args, C.byref(bad), P64, DUMMY, DUMMY, None, None, None) == L.TPFA_ERR_PARAM
    st.pref = None
    assert lib.tpfa_jvp(*args, None, L.TPFA_FP32, DUMMY, DUMMY, None, None,
                        None) == L.TPFA_ERR_UNSUPPORTED


def test_transmissibility_form_validation(lib):
    g, f, _, st = good()
    args = lambda rk: (C.byref(g), C.byref(f), C.byref(rk), C.byref(st))  # noqa: E731
    D = DUMMY.value
    ok = L.Rock(None, None, None, 1.0, 1.0, None, D, D, D)
    for rk, code in ((L.Rock(None, None, None, 1.0, 1.0, None, D, None, D), L.TPFA_ERR_NULL),
                     (L.Rock(D, None, None, 1.0, 1.0, None, D, D, D), L.TPFA_ERR_PARAM),
                     (L.Rock(None, None, None, 1.0, 1.0, D, D, D, D), L.TPFA_ERR_PARAM)):
        assert lib.tpfa_residual(*args(rk), L.TPFA_FP64, None, None, None) == code
    # valid rock, but the VJP and the batch need the permeability form
    assert lib.tpfa_residual_vjp(*args(ok), L.TPFA_FP64, DUMMY, DUMMY, DUMMY, None,
                                 None) == L.TPFA_ERR_UNSUPPORTED
    m = (L.Model * 1)()
    m[0] = L.Model(g, f, ok, st, DUMMY.value, DUMMY.value, L.Launch(-1, 0, 0))
    out = C.c_void_p()
    assert lib.tpfa_batch_create(m, 1, L.TPFA_FP64, L.TPFA_BATCH_JACOBIAN, C.byref(out),
                                 None) == L.TPFA_ERR_UNSUPPORTED


def test_per_direction_form_validation(lib):
    """ky and kz go together, the ratios are not checked in that form (a
    negative ry fails only without the arrays), and the batch rejects it."""
    g, f, _, st = good()
    args = lambda rk: (C.byref(g), C.byref(f), C.byref(rk), C.byref(st))  # noqa: E731
    D = DUMMY.value
    assert lib.tpfa_residual(*args(L.Rock(D, None, None, -1.0, 1.0, None, None, None, None)),
                             L.TPFA_FP64, None, None, None) == L.TPFA_ERR_PARAM
    # with the arrays the ratios are ignored: the next failure is the NULL output
    assert lib.tpfa_residual(*args(L.Rock(D, D, D, -1.0, math.nan, None, None, None, None)),
                             L.TPFA_FP64, None, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual(*args(L.Rock(D, D, D, 1.0, 1.0, None, D, D, D)), L.TPFA_FP64,
                             DUMMY, None, None) == L.TPFA_ERR_PARAM
    m = (L.Model * 1)()
    m[0] = L.Model(g, f, L.Rock(D, D, D, 1.0, 1.0, None, None, None, None), st, DUMMY.value,
                   DUMMY.value, L.Launch(-1, 0, 0))
    out = C.c_void_p()
    assert lib.tpfa_batch_create(m, 1, L.TPFA_FP64, L.TPFA_BATCH_JACOBIAN, C.byref(out),
                                 None) == L.TPFA_ERR_UNSUPPORTED


def test_plane_size_limit(lib):
    """A cell is addressed within its x-y plane by a 32-bit byte offset, so one
    plane of one array must hold fewer than 2^32 bytes."""
    g, f, rk, st = good()
    g.nx, g.ny, g.nz = 2 ** 15, 2 ** 14, 1  # 2^29 cells: 2^32 bytes in FP64, 2^31 in FP32
    args = (C.byref(g), C.byref(f), C.byref(rk), C.byref(st))
    assert lib.tpfa_residual(*args, L.TPFA_FP64, DUMMY, None, None) == L.TPFA_ERR_SHAPE
    st.pref = DUMMY.value
    # FP32 passes the shape check and stops at the missing output
    assert lib.tpfa_residual(*args, L.TPFA_FP32, None, None, None) == L.TPFA_ERR_NULL
    g.ny = 2 ** 15  # 2^30 cells: 2^32 bytes in FP32
    assert lib.tpfa_residual(*args, L.TPFA_FP32, DUMMY, None, None) == L.TPFA_ERR_SHAPE
    # the limit applies to the padded plane: 8 x 2^14 cells with a row pitch of 2^15
    g.nx, g.ny, g.ldx = 8, 2 ** 14, 2 ** 15
    assert lib.tpfa_residual(*args, L.TPFA_FP64, DUMMY, None, None) == L.TPFA_ERR_SHAPE
    assert lib.tpfa_residual(*args, L.TPFA_FP32, None, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_offset_pressure(C.byref(L.Grid(8, 8, 8, 1.0, 1.0, 1.0, 0.0, 4)), DUMMY,
                                    DUMMY, DUMMY, None) == L.TPFA_ERR_SHAPE


def test_vjp_trans_validation(lib):
    g, f, rk, st = good()
    D = DUMMY.value
    tr = L.Rock(None, None, None, 1.0, 1.0, None, D, D, D)
    args = lambda r: (C.byref(g), C.byref(f), C.byref(r), C.byref(st), L.TPFA_FP64)  # noqa: E731
    assert lib.tpfa_residual_vjp_trans(*args(rk), DUMMY, DUMMY, DUMMY, None,
                                       None) == L.TPFA_ERR_UNSUPPORTED
    assert lib.tpfa_residual_vjp_trans(*args(tr), None, DUMMY, DUMMY, None, None) == L.TPFA_ERR_NULL
    assert lib.tpfa_residual_vjp_trans(*args(tr), DUMMY, None, None, None, None) == L.TPFA_ERR_NULL
