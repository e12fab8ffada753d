"""Randomised parity (hypothesis, derandomised so every run draws the same
cases): small grids of any shape, seal density, precision, tile shape, z chunk,
workgroup order (natural, XCD bands, y fastest) and row pitch. The full-grid Jacobian launch meets the oracle
bound (R16 metric, either one-sided derivative at upwind ties); a launch over a
random row range on NaN-filled outputs equals it bitwise on the owned rows and
leaves every other row and all padding untouched. The same random launches
drive the VJP, the 10-flux residual, the per-direction and transmissibility
forms and the backward-Euler J and J v against the oracle, and random uneven
ensembles (either schedule, graph or direct launch) against the members'
single-grid launches, bitwise. The row-range launch is repeated with the
outputs' padding writable (pad_writes): equal owned rows, zeros in the padding
under the tile's lanes, everything else untouched; and with r and J in the
sliced layout: equal owned rows, zeros in the owned rows' lanes beyond nx,
everything else untouched. The one-pass residual + VJP equals the residual and
VJP calls bitwise under the same random launches."""
import numpy as np
import pytest
import torch
from hypothesis import given, settings, strategies as st

import geomodel
from helpers import compare_full

pytestmark = pytest.mark.gpu

TOL64, TOL32, TAU32 = 1e-12, 1e-5, 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pad(a, ldx):
    t = dev(a)
    fill = 255 if t.dtype == torch.uint8 else float("nan")
    buf = torch.full(tuple(t.shape[:-1]) + (ldx,), fill, dtype=t.dtype, device=t.device)
    buf[..., :t.shape[-1]].copy_(t)
    return buf[..., :t.shape[-1]]


@st.composite
def cases(draw):
    nx, ny, nz = draw(st.integers(1, 70)), draw(st.integers(1, 20)), draw(st.integers(1, 12))
    y0 = draw(st.integers(0, ny - 1))
    y1 = draw(st.integers(y0 + 1, ny))
    return dict(shape=(nx, ny, nz), seed=draw(st.integers(0, 10 ** 6)),
                seal=draw(st.sampled_from([0.0, 0.05, 0.3])),
                prec=draw(st.sampled_from(["fp64", "fp32"])),
                tile=draw(st.sampled_from([None] + list(range(10)))),
                kz=draw(st.sampled_from([None, 1, 3, 8])),
                remap=draw(st.sampled_from([False, True, "yfast"])),
                extra=draw(st.sampled_from([0, 1, 13])), rows=(y0, y1))


@settings(derandomize=True, max_examples=60, deadline=None)
@given(c=cases())
def test_random_launches_against_oracle(gpu, orc, c):
    print("case", c, flush=True)
    geo = geomodel.random_small(c["seed"] % 9973, *c["shape"], sigma=1.5, seal_prob=c["seal"])
    g = geo.grid
    ldx = g.nx + c["extra"]
    launch = dict(tile=c["tile"], kz_chunk=c["kz"], xcd_remap=c["remap"])
    if c["prec"] == "fp64":
        p = orc.pressure(geo)
        k, pin, kw, tol, tau = geo.kx, p, {}, TOL64, 1e-9 * float(np.abs(p).max())
        pw, kwide = p, geo.kx
    else:
        pref = orc.hydrostatic(g, geo.fluid, geo.p_top)
        k, pin = geo.kx32(), geo.dp32()
        kw, tol, tau = dict(pref=dev(pref)), TOL32, TAU32
        pw, kwide = orc.widen_fp32(pin, pref), k.astype(np.float64)
    kp, pp, sp = pad(k, ldx), pad(pin, ldx), pad(geo.seal, ldx)
    r, J = gpu.jacobian(g, geo.fluid, kp, pp, seal=sp, ry=geo.ry, rz=geo.rz, **launch, **kw)
    rb = torch.full(g.shape[:2] + (ldx,), float("nan"), dtype=r.dtype, device="cuda")
    Jb = torch.full((7,) + g.shape[:2] + (ldx,), float("nan"), dtype=r.dtype, device="cuda")
    y0, y1 = c["rows"]
    gpu.jacobian(g, geo.fluid, kp, pp, seal=sp, ry=geo.ry, rz=geo.rz, rows=(y0, y1),
                 r_out=rb[..., :g.nx], J_out=Jb[..., :g.nx], **launch, **kw)
    torch.cuda.synchronize()
    assert torch.equal(rb[:, y0:y1, :g.nx], r[:, y0:y1]) and torch.equal(Jb[..., y0:y1, :g.nx],
                                                                     J[..., y0:y1, :])
    assert torch.isnan(rb[:, :y0]).all() and torch.isnan(rb[:, y1:]).all()
    assert torch.isnan(Jb[..., :y0, :]).all() and torch.isnan(Jb[..., y1:, :]).all()
    assert torch.isnan(rb[..., g.nx:]).all() and torch.isnan(Jb[..., g.nx:]).all()
    # the same row-range launch with the outputs' padding writable: the owned
    # rows' padding under the tile's lanes is zeros, the rest untouched
    rp = torch.full_like(rb, float("nan"))
    Jp = torch.full_like(Jb, float("nan"))
    gpu.jacobian(g, geo.fluid, kp, pp, seal=sp, ry=geo.ry, rz=geo.rz, rows=(y0, y1),
                 r_out=rp[..., :g.nx], J_out=Jp[..., :g.nx], pad_writes=True, **launch, **kw)
    tx = gpu.resolve_launch(g, "jacobian", r.dtype, rows=(y0, y1), ldx=ldx, **launch)["shape"][0]
    cov = min(ldx, -(-g.nx // tx) * tx)
    torch.cuda.synchronize()
    assert torch.equal(rp[:, y0:y1, :g.nx], rb[:, y0:y1, :g.nx])
    assert torch.equal(Jp[..., y0:y1, :g.nx], Jb[..., y0:y1, :g.nx])
    assert bool((rp[:, y0:y1, g.nx:cov] == 0).all()) and bool((Jp[..., y0:y1, g.nx:cov] == 0).all())
    assert torch.isnan(rp[:, y0:y1, cov:]).all() and torch.isnan(Jp[..., y0:y1, cov:]).all()
    assert torch.isnan(rp[:, :y0]).all() and torch.isnan(rp[:, y1:]).all()
    # the same row-range launch with r and J in the sliced layout: the owned
    # rows' values bitwise, their lanes beyond nx zero, other rows untouched
    nz_, ny_, S = gpu.sliced_shape(g)[:3]
    Js = torch.full(gpu.sliced_shape(g), float("nan"), dtype=r.dtype, device="cuda")
    gpu.jacobian(g, geo.fluid, kp, pp, seal=sp, ry=geo.ry, rz=geo.rz, rows=(y0, y1), J_out=Js,
                 sliced=True, **launch, **kw)
    torch.cuda.synchronize()
    flat = Js.permute(3, 0, 1, 2, 4).reshape(8, nz_, ny_, S * 64)
    assert torch.equal(flat[0, :, y0:y1, :g.nx], r[:, y0:y1])
    assert torch.equal(flat[1:, :, y0:y1, :g.nx], J[:, :, y0:y1])
    assert bool((flat[:, :, y0:y1, g.nx:] == 0).all())
    assert torch.isnan(flat[:, :, :y0]).all() and torch.isnan(flat[:, :, y1:]).all()
    rep = compare_full(orc, g, geo.fluid, kwide, pw, r.double().cpu().numpy(),
                       J.double().cpu().numpy(), tol=tol, tau=tau, ry=geo.ry, rz=geo.rz,
                       seal=geo.seal)
    assert rep["max_err"] <= tol, (c, rep)


@settings(derandomize=True, max_examples=40, deadline=None)
@given(c=cases(), op=st.sampled_from(["vjp", "residual10"]))
def test_random_vjp_and_10_flux_against_oracle(gpu, orc, c, op):
    """The vector-Jacobian product (grad p, grad ln k) and the 10-flux residual
    under random launches and row pitches, against the oracle."""
    from helpers import compare_res10, compare_vjp
    print("case", op, c, flush=True)
    geo = geomodel.random_small(c["seed"] % 9973, *c["shape"], sigma=1.5, seal_prob=c["seal"])
    g = geo.grid
    ldx = g.nx + c["extra"]
    launch = dict(tile=c["tile"], kz_chunk=c["kz"], xcd_remap=c["remap"])
    rng = np.random.default_rng(c["seed"])
    w = rng.standard_normal(g.shape)
    tne, tse = geomodel.diagonal_t(g, c["seed"] % 9973 + 1)
    if c["prec"] == "fp64":
        p = orc.pressure(geo)
        k, pin, kw, tol, tau = geo.kx, p, {}, TOL64, 1e-9 * float(np.abs(p).max())
        pw, kwide, wq, tq = p, geo.kx, w, (tne, tse)
    else:
        pref = orc.hydrostatic(g, geo.fluid, geo.p_top)
        k, pin = geo.kx32(), geo.dp32()
        kw, tol, tau = dict(pref=dev(pref)), TOL32, TAU32
        pw, kwide = orc.widen_fp32(pin, pref), k.astype(np.float64)
        wq, tq = w.astype(np.float32), (tne.astype(np.float32), tse.astype(np.float32))
    args = (g, geo.fluid, pad(k, ldx), pad(pin, ldx))
    kw.update(seal=pad(geo.seal, ldx), ry=geo.ry, rz=geo.rz, **launch)
    if op == "vjp":
        wd = pad(wq, ldx)
        gp, gm = gpu.residual_vjp(*args, wd, **kw)
        # one pass: bitwise the residual and VJP calls
        r1, gp1, gm1 = gpu.residual_and_vjp(*args, wd, **kw)
        r0 = gpu.residual(*args, **kw)
        torch.cuda.synchronize()
        assert torch.equal(r1, r0) and torch.equal(gp1, gp) and torch.equal(gm1, gm)
        rep = compare_vjp(orc, g, geo.fluid, kwide, pw, np.asarray(wq, np.float64),
                          gp.double().cpu().numpy(), gm.double().cpu().numpy(), tol=tol, tau=tau,
                          ry=geo.ry, rz=geo.rz, seal=geo.seal)
    else:
        r = gpu.residual10(*args, pad(tq[0], ldx), pad(tq[1], ldx), **kw)
        torch.cuda.synchronize()
        rep = compare_res10(orc, g, geo.fluid, kwide, pw, tq[0].astype(np.float64),
                            tq[1].astype(np.float64), r.double().cpu().numpy(), tol=tol, tau=tau,
                            ry=geo.ry, rz=geo.rz, seal=geo.seal)
    assert rep["max_err"] <= tol, (op, c, rep)


def _check_rJ(r, J, ref, tol):
    from helpers import rel_err
    assert rel_err(r, ref["r"], ref["scale"][0]).max() <= tol
    assert rel_err(J[0], ref["J"][0], ref["scale"][1]).max() <= tol
    for n in range(1, 7):
        assert rel_err(J[n], ref["J"][n], np.abs(ref["J"][n])).max() <= tol, n


@settings(derandomize=True, max_examples=40, deadline=None)
@given(c=cases(), op=st.sampled_from(["k3", "trans", "be"]))
def test_random_other_forms_against_oracle(gpu, orc, c, op):
    """Per-direction permeability and face-transmissibility Jacobians, and the
    backward-Euler Jacobian with J v, under random launches and row pitches."""
    from helpers import apply_J, compare_full
    print("case", op, c, flush=True)
    s = c["seed"] % 9973
    geo = geomodel.random_small(s, *c["shape"], sigma=1.5, seal_prob=c["seal"])
    g = geo.grid
    ldx = g.nx + c["extra"]
    launch = dict(tile=c["tile"], kz_chunk=c["kz"], xcd_remap=c["remap"])
    fp64 = c["prec"] == "fp64"
    cast = (lambda a: a) if fp64 else (lambda a: np.asarray(a, np.float32))  # noqa: E731
    wide = lambda a: np.asarray(a, np.float64)  # noqa: E731
    if fp64:
        p = orc.pressure(geo)
        pin, pw, kw, tol, tau = p, p, {}, TOL64, 1e-9 * float(np.abs(p).max())
    else:
        pref = orc.hydrostatic(g, geo.fluid, geo.p_top)
        pin = geo.dp32()
        pw, kw, tol, tau = orc.widen_fp32(pin, pref), dict(pref=dev(pref)), TOL32, TAU32
    kw.update(launch)
    P = lambda a: pad(a, ldx)  # noqa: E731
    if op == "k3":
        k3 = [cast(a) for a in geomodel.k3_fields(geo.kx, s + 1)]
        r, J = gpu.jacobian(g, geo.fluid, P(k3[0]), P(pin), seal=P(geo.seal), ky=P(k3[1]),
                            kz=P(k3[2]), **kw)
        torch.cuda.synchronize()
        rep = compare_full(orc, g, geo.fluid, wide(k3[0]), pw, r.double().cpu().numpy(),
                           J.double().cpu().numpy(), tol=tol, tau=tau, ry=1.0, rz=1.0,
                           seal=geo.seal, ky=wide(k3[1]), kz=wide(k3[2]))
        assert rep["max_err"] <= tol, (op, c, rep)
    elif op == "trans":
        t = geomodel.diagonal_t(g, s + 2, zero_prob=0.05) + geomodel.diagonal_t(g, s + 3)[:1]
        tq = [cast(a) for a in t]
        r, J = gpu.jacobian(g, geo.fluid, None, P(pin), trans=tuple(P(a) for a in tq), **kw)
        torch.cuda.synchronize()
        ref = orc.evaluate_general(g, geo.fluid, pw, trans=tuple(wide(a) for a in tq),
                                   want=("r", "J", "scale"))
        _check_rJ(r.double().cpu().numpy(), J.double().cpu().numpy(), ref, tol)
    else:
        be = geomodel.be_fields(g, s + 4)
        if fp64:
            pn, pnw = p - be["dp_step"], p - be["dp_step"]
        else:
            pn = (geo.noise[0] - be["dp_step"]).astype(np.float32)
            pnw = orc.widen_fp32(pn, pref)
        phi, v = cast(be["phi"]), cast(be["v"])
        acc = dict(phi=P(phi), p_prev=P(pn), dt=be["dt"], cr=be["cr"])
        kx = cast(geo.kx)
        args = (g, geo.fluid, P(kx), P(pin))
        r, J = gpu.jacobian_be(*args, acc, seal=P(geo.seal), ry=geo.ry, rz=geo.rz, **kw)
        jv, _ = gpu.jvp(*args, P(v), accum=acc, seal=P(geo.seal), ry=geo.ry, rz=geo.rz, **kw)
        torch.cuda.synchronize()
        ref = orc.evaluate_be(g, geo.fluid, wide(kx), pw, wide(phi), pnw, be["dt"], be["cr"],
                              ry=geo.ry, rz=geo.rz, seal=geo.seal, v=wide(v),
                              want=("r", "J", "scale", "jv"))
        _check_rJ(r.double().cpu().numpy(), J.double().cpu().numpy(), ref, tol)
        scale = apply_J(np.abs(ref["J"]), np.abs(wide(v)))
        err = np.abs(jv.double().cpu().numpy() - ref["jv"])
        assert np.all(err <= tol * scale + 1e-300), (op, c)


@st.composite
def ensembles(draw):
    n = draw(st.integers(1, 12))
    members = []
    for _ in range(n):
        members.append(dict(shape=(draw(st.integers(1, 80)), draw(st.integers(1, 24)),
                                   draw(st.integers(1, 20))),
                            seed=draw(st.integers(0, 9999)), tile=draw(st.sampled_from([0, 1, 2, 10])),
                            kz=draw(st.sampled_from([1, 4, 16, 64])), extra=draw(st.sampled_from([0, 5]))))
    return dict(members=members, prec=draw(st.sampled_from(["fp64", "fp32"])),
                mode=draw(st.sampled_from(["jacobian", "residual"])),
                schedule=draw(st.sampled_from(["persistent", "grouped"])),
                graph=draw(st.booleans()))


@settings(derandomize=True, max_examples=25, deadline=None)
@given(e=ensembles())
def test_random_ensembles_equal_single_launches(gpu, orc, e):
    """Uneven ensembles of 1..12 members (tile, the fitted tile included, z
    chunk and row pitch per member), either schedule, graph replay or direct launch, repeated: every
    member's outputs bitwise equal to its own single-grid launch."""
    print("ensemble", e, flush=True)
    members, singles = [], []
    for m in e["members"]:
        geo = geomodel.random_small(m["seed"], *m["shape"], sigma=1.2, seal_prob=0.05)
        g = geo.grid
        ldx = g.nx + m["extra"]
        if e["prec"] == "fp64":
            k, pin, kw = geo.kx, orc.pressure(geo), {}
        else:
            k, pin = geo.kx32(), geo.dp32()
            kw = dict(pref=dev(orc.hydrostatic(g, geo.fluid, geo.p_top)))
        d = dict(grid=g, fluid=geo.fluid, kx=pad(k, ldx), p=pad(pin, ldx), seal=pad(geo.seal, ldx),
                 ry=geo.ry, rz=geo.rz, tile=m["tile"], kz_chunk=m["kz"], **kw)
        members.append(d)
        # the fitted tile (10) exists for ensemble members only; results never depend on the tile
        launch = dict(seal=dev(geo.seal), ry=geo.ry, rz=geo.rz,
                      tile=None if m["tile"] == 10 else m["tile"], kz_chunk=m["kz"], **kw)
        if e["mode"] == "jacobian":
            singles.append(gpu.jacobian(g, geo.fluid, dev(k), dev(pin), **launch))
        else:
            singles.append((gpu.residual(g, geo.fluid, dev(k), dev(pin), **launch), None))
    ens = gpu.Ensemble(members, mode=e["mode"])
    ens.set_schedule(e["schedule"])
    try:
        for rep in range(2):
            for q in range(len(members)):
                ens.r[q].fill_(float("nan"))
                if ens.J[q] is not None:
                    ens.J[q].fill_(float("nan"))
            ens.run(graph=e["graph"])
            torch.cuda.synchronize()
            for q, (r, J) in enumerate(singles):
                assert torch.equal(ens.r[q], r), (rep, q)
                if J is not None:
                    assert torch.equal(ens.J[q], J), (rep, q)
    finally:
        ens.close()
