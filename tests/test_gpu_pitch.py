"""Row-pitched arrays (every per-cell array a view buf[..., :nx] of a buffer
with row pitch ldx >= nx): every mode, rock form and precision gives outputs
bitwise equal to the contiguous launch, padding is never read (it holds NaN,
or 0xFF seal bytes, which would poison any result that read it) and never
written, and the FP32 and FP64 Jacobians on padded arrays meet the oracle
bound directly. Pitches: odd (rows off every line), 128-byte multiples in
FP32 and FP64, and one with a column offset into a wider buffer."""
import numpy as np
import pytest
import torch

import geomodel
from helpers import compare_full

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
TAU32 = 1e-4  # Pa: upwind tie band of the FP32 form (its |dPhi| error is below 1e-6 Pa)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pad(a, ldx, off=0):
    """Device copy of a (..., nz, ny, nx) array as the view [..., off:off+nx] of a
    buffer with row pitch ldx; padding holds NaN (0xFF for bytes)."""
    t = dev(a)
    nx = t.shape[-1]
    fill = 255 if t.dtype == torch.uint8 else float("nan")
    buf = torch.full(tuple(t.shape[:-1]) + (ldx,), fill, dtype=t.dtype, device=t.device)
    v = buf[..., off:off + nx]
    v.copy_(t)
    return v


def out_like(p, lead=(), ldx=None, off=0):
    """A NaN-filled output buffer in a padded layout, and its view."""
    nz, ny, nx = p.shape
    buf = torch.full(tuple(lead) + (nz, ny, ldx), float("nan"), dtype=p.dtype, device=p.device)
    return buf, buf[..., off:off + nx]


def padding_untouched(buf, off, nx):
    """Every element of buf outside columns [off, off + nx) is still NaN."""
    mask = torch.ones(buf.shape[-1], dtype=torch.bool, device=buf.device)
    mask[off:off + nx] = False
    return bool(torch.isnan(buf[..., mask]).all())


def case(prec, seed=5, shape=(70, 23, 9)):
    geo = geomodel.random_small(seed, *shape, sigma=1.2, seal_prob=0.05)
    g = geo.grid
    k3 = geomodel.k3_fields(geo.kx, seed + 1)
    diag = geomodel.diagonal_t(g, seed + 2)
    be = geomodel.be_fields(g, seed + 3)
    tr = geomodel.diagonal_t(g, seed + 4, zero_prob=0.05) + geomodel.diagonal_t(g, seed + 5)[:1]
    pref = None
    if prec == "fp64":
        from oracle import pressure
        p = pressure(geo)
        cast = lambda a: a  # noqa: E731
    else:
        from oracle import hydrostatic
        pref = hydrostatic(g, geo.fluid)
        p = geo.dp32(0)
        cast = lambda a: np.asarray(a, np.float32)  # noqa: E731
    fields = dict(p=cast(p), kx=cast(geo.kx), ky=cast(k3[1]), kz=cast(k3[2]),
                  tne=cast(diag[0]), tse=cast(diag[1]), phi=cast(be["phi"]),
                  p_prev=cast(p - be["dp_step"]) if prec == "fp64" else cast(p),
                  v=cast(be["v"]), seal=geo.seal,
                  tx=cast(tr[0]), ty=cast(tr[1]), tz=cast(tr[2]))
    return geo, fields, pref, be


def run_all(gpu, geo, f, pref, be, put, tile=None, **extra):
    """Every output of every mode; `put` places a host array on the device;
    `extra` keyword arguments go to every call."""
    g = geo.grid
    d = {k: put(v) for k, v in f.items()}
    kw = dict(seal=d["seal"], ry=geo.ry, rz=geo.rz, tile=tile,
              pref=None if pref is None else dev(pref), **extra)
    acc = dict(phi=d["phi"], p_prev=d["p_prev"], dt=be["dt"], cr=be["cr"])
    tr = (d["tx"], d["ty"], d["tz"])
    pk = dict(pref=kw["pref"], tile=tile, **extra)
    o = {}
    o["res"] = gpu.residual(g, geo.fluid, d["kx"], d["p"], **kw)
    o["resbe"] = gpu.residual_be(g, geo.fluid, d["kx"], d["p"], acc, **kw)
    o["r"], o["J"] = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], **kw)
    o["gp"], o["gm"] = gpu.residual_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], **kw)
    o["r10"] = gpu.residual10(g, geo.fluid, d["kx"], d["p"], d["tne"], d["tse"], **kw)
    o["rbe"], o["Jbe"] = gpu.jacobian_be(g, geo.fluid, d["kx"], d["p"], acc, **kw)
    o["jv"], o["jvr"] = gpu.jvp(g, geo.fluid, d["kx"], d["p"], d["v"], accum=acc, want_r=True,
                                **kw)
    o["rk3"], o["Jk3"] = gpu.jacobian(g, geo.fluid, d["kx"], d["p"], ky=d["ky"], kz=d["kz"], **kw)
    o["gpk3"], o["gk3"] = gpu.residual_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], ky=d["ky"],
                                           kz=d["kz"], **kw)
    o["rT"], o["JT"] = gpu.jacobian(g, geo.fluid, None, d["p"], trans=tr, **pk)
    o["gpT"], o["gT"] = gpu.residual_vjp(g, geo.fluid, None, d["p"], d["v"], trans=tr, **pk)
    o["r10T"] = gpu.residual10(g, geo.fluid, None, d["p"], d["tne"], d["tse"], trans=tr, **pk)
    torch.cuda.synchronize()
    return o


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ldx,off", [(71, 0), (96, 0), (128, 0), (131, 33)])
def test_every_mode_bitwise_equal_to_contiguous(gpu, prec, ldx, off):
    geo, f, pref, be = case(prec)
    print(f"pitched layout {prec} ldx={ldx} off={off}", flush=True)
    want = run_all(gpu, geo, f, pref, be, dev)
    got = run_all(gpu, geo, f, pref, be, lambda a: pad(a, ldx, off))
    for k, w in want.items():
        v = got[k]
        assert v.stride(-2) == ldx, k  # outputs take the pitch of p
        assert torch.equal(v, w), (prec, ldx, off, k)


@pytest.mark.parametrize("tile", range(10))
def test_padding_never_written_every_tile(gpu, tile):
    geo, f, pref, be = case("fp32", seed=9)
    g = geo.grid
    ldx, off = 96, 0
    d = {k: pad(v, ldx, off) for k, v in f.items()}
    pref_d = dev(pref)
    print(f"pitched outputs, tile {tile}", flush=True)
    rc, Jc = gpu.jacobian(g, geo.fluid, dev(f["kx"]), dev(f["p"]), seal=dev(f["seal"]),
                          pref=pref_d, ry=geo.ry, rz=geo.rz, tile=tile)
    rb, r = out_like(d["p"], (), ldx, off)
    Jb, J = out_like(d["p"], (7,), ldx, off)
    gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], pref=pref_d, ry=geo.ry,
                 rz=geo.rz, tile=tile, r_out=r, J_out=J)
    gb, gm = out_like(d["p"], (3,), ldx, off)
    gpu.residual_vjp(g, geo.fluid, d["kx"], d["p"], d["v"], seal=d["seal"], pref=pref_d,
                     ky=d["ky"], kz=d["kz"], tile=tile, want_p=False, gm_out=gm)
    torch.cuda.synchronize()
    assert torch.equal(r, rc) and torch.equal(J, Jc), tile
    assert not torch.isnan(gm).any()
    for b in (rb, Jb, gb):
        assert padding_untouched(b, off, g.nx), tile


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_padded_jacobian_against_oracle(gpu, orc, prec):
    """Direct parity of the padded launch with the FP64 oracle (R16 bound)."""
    geo = geomodel.random_small(21, 97, 41, 13, sigma=1.5, seal_prob=0.02, ry=1.0, rz=0.1)
    g = geo.grid
    ldx = 128
    print(f"padded jacobian vs oracle {prec}", flush=True)
    if prec == "fp64":
        p = orc.pressure(geo)
        r, J = gpu.jacobian(g, geo.fluid, pad(geo.kx, ldx), pad(p, ldx), seal=pad(geo.seal, ldx),
                            ry=geo.ry, rz=geo.rz)
        kx, pw, tol, tau = geo.kx, p, TOL64, 1e-9 * np.abs(p).max()
    else:
        pref = orc.hydrostatic(g, geo.fluid, geo.p_top)
        dp, k32 = geo.dp32(), geo.kx32()
        r, J = gpu.jacobian(g, geo.fluid, pad(k32, ldx), pad(dp, ldx), seal=pad(geo.seal, ldx),
                            pref=dev(pref), ry=geo.ry, rz=geo.rz)
        kx, pw, tol, tau = k32.astype(np.float64), orc.widen_fp32(dp, pref), TOL32, TAU32
    assert r.stride(-2) == ldx and J.stride(-2) == ldx
    torch.cuda.synchronize()
    rep = compare_full(orc, g, geo.fluid, kx, pw, r.cpu().numpy(), J.cpu().numpy(), tol=tol,
                       tau=tau, ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert rep["max_err"] <= tol, rep


def test_offset_pressure_pitched(gpu, orc):
    geo = geomodel.random_small(4, 37, 6, 5)
    g = geo.grid
    p = orc.pressure(geo)
    pref = dev(orc.hydrostatic(g, geo.fluid))
    want = gpu.offset_pressure(g, dev(p), pref)
    pp = pad(p, 64)
    got = gpu.offset_pressure(g, pp, pref)
    buf, out = out_like(pp.float(), (), 64, 0)
    gpu.offset_pressure(g, pp, pref, out=out)
    torch.cuda.synchronize()
    assert got.stride(-2) == 64 and torch.equal(got, want) and torch.equal(out, want)
    assert padding_untouched(buf, 0, g.nx)


def test_ensemble_with_padded_members(gpu, orc):
    """Members with different pitches (and one contiguous) in one persistent
    launch: bitwise equal to their single launches."""
    members, singles = [], []
    for m, (shape, ldx) in enumerate([((45, 20, 9), 64), ((70, 13, 6), 70), ((33, 31, 11), 40)]):
        geo = geomodel.random_small(60 + m, *shape, sigma=1.0, seal_prob=0.03)
        pref = orc.hydrostatic(geo.grid, geo.fluid, geo.p_top)
        d = dict(grid=geo.grid, fluid=geo.fluid, kx=pad(geo.kx32(), ldx), p=pad(geo.dp32(0), ldx),
                 seal=pad(geo.seal, ldx), pref=dev(pref), ry=geo.ry, rz=geo.rz, tile=m % 3)
        members.append(d)
        singles.append(gpu.jacobian(d["grid"], d["fluid"], dev(geo.kx32()), dev(geo.dp32(0)),
                                    seal=dev(geo.seal), pref=d["pref"], ry=geo.ry, rz=geo.rz,
                                    tile=m % 3))
    print("ensemble with padded members", flush=True)
    ens = gpu.Ensemble(members)
    for schedule in ("persistent", "grouped"):
        ens.set_schedule(schedule)
        for q in range(len(members)):
            ens.r[q].fill_(float("nan"))
            ens.J[q].fill_(float("nan"))
        ens.run()
        torch.cuda.synchronize()
        for q, (r, J) in enumerate(singles):
            assert torch.equal(ens.r[q], r) and torch.equal(ens.J[q], J), (schedule, q)
    ens.close()


def test_mixed_pitches_are_refused(gpu):
    geo = geomodel.random_small(2, 20, 5, 4)
    g = geo.grid
    p = pad(geo.kx * 0 + 1e7, 32)
    with pytest.raises(ValueError, match="row pitch"):
        gpu.residual(g, geo.fluid, pad(geo.kx, 24), p)
    with pytest.raises(ValueError, match="row pitch"):
        gpu.residual(g, geo.fluid, pad(geo.kx, 32), p, out=torch.empty(g.shape, device="cuda",
                                                                       dtype=torch.float64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_row_range_on_pitched_arrays(gpu, prec):
    """A y-slab launch on row-pitched arrays writes exactly the owned rows of
    the real columns (equal to the full contiguous launch there) and leaves
    every other row and all padding untouched."""
    geo, f, pref, be = case(prec, seed=13)
    g = geo.grid
    ldx = 80
    pref_d = None if pref is None else dev(pref)
    kw = dict(ry=geo.ry, rz=geo.rz, pref=pref_d)
    rc, Jc = gpu.jacobian(g, geo.fluid, dev(f["kx"]), dev(f["p"]), seal=dev(f["seal"]), **kw)
    d = {k: pad(f[k], ldx) for k in ("kx", "p", "seal", "v")}
    for y0, y1 in ((0, 7), (7, 8), (8, 23)):
        print(f"row range {y0}:{y1} on pitch {ldx}, {prec}", flush=True)
        rb, r = out_like(d["p"], (), ldx)
        Jb, J = out_like(d["p"], (7,), ldx)
        gpu.jacobian(g, geo.fluid, d["kx"], d["p"], seal=d["seal"], rows=(y0, y1), r_out=r,
                     J_out=J, **kw)
        torch.cuda.synchronize()
        assert torch.equal(r[:, y0:y1], rc[:, y0:y1]) and torch.equal(J[:, :, y0:y1],
                                                                      Jc[:, :, y0:y1])
        for b in (rb, Jb):
            assert torch.isnan(b[..., :y0, :]).all() and torch.isnan(b[..., y1:, :]).all()
            assert padding_untouched(b, 0, g.nx)


def test_autograd_functions_accept_pitched_inputs(gpu):
    """The autograd Functions take row-pitched p / ln k (they work on
    contiguous copies): values and gradients equal the contiguous case."""
    geo, f, pref, be = case("fp64", seed=17)
    g = geo.grid
    w = dev(f["v"])
    res = []
    for put in (dev, lambda a: pad(a, 96)):
        p = put(f["p"]).requires_grad_(True)
        logk = put(np.log(f["kx"])).requires_grad_(True)
        logk3 = put(np.log(np.stack([f["kx"], f["ky"], f["kz"]]))).requires_grad_(True)
        r = gpu.TPFAResidual.apply(p, logk, g, geo.fluid, put(f["seal"]), None, geo.ry, geo.rz)
        ra = gpu.TPFAAnisoResidual.apply(p, logk3, g, geo.fluid, put(f["seal"]), None)
        gp, gk, gk3 = torch.autograd.grad((r * w).sum() + (ra * w).sum(), (p, logk, logk3))
        res.append((r.detach(), ra.detach(), gp, gk, gk3))
    torch.cuda.synchronize()
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_pitched_helpers(gpu):
    """Inputs copied with to_pitched and outputs from empty_pitched (rows on
    128-byte lines): the same results as the contiguous launch."""
    geo, f, pref, be = case("fp32", seed=19, shape=(45, 20, 7))
    g = geo.grid
    kw = dict(ry=geo.ry, rz=geo.rz, pref=dev(pref))
    rc, Jc = gpu.jacobian(g, geo.fluid, dev(f["kx"]), dev(f["p"]), seal=dev(f["seal"]), **kw)
    k, p, s = (gpu.to_pitched(dev(f[n]), g) for n in ("kx", "p", "seal"))
    r = gpu.empty_pitched(g, torch.float32, "cuda")
    J = gpu.empty_pitched(g, torch.float32, "cuda", (7,))
    gpu.jacobian(g, geo.fluid, k, p, seal=s, r_out=r, J_out=J, **kw)
    torch.cuda.synchronize()
    assert p.stride(-2) == 64 and s.stride(-2) == 64 and J.stride(-2) == 64
    assert torch.equal(r, rc) and torch.equal(J, Jc)
