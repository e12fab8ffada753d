#!/usr/bin/env python3
"""Benchmark of the TPFA flux residual + 7-point Jacobian on one MI355X.

One step = one application of the whole path (residual and Jacobian, i.e.
density, transmissibility, potential difference, upwinding, flux, derivatives
and the stores) to the 512 x 512 x 256 geomodel in FP64, with the pressure
vector changing every call as in the paper's protocol (Sec. 3: the flux
computation is applied 1000 times with a different pressure vector each time);
four pre-generated pressure fields rotate so that nothing is served from the
256 MB last-level cache. Inputs are resident in HBM before the timed region.
r and J are written in the library's sliced layout (TPFA_LAUNCH_SLICED: one
array of 64-cell row slices, each holding r and the seven Jacobian values of
its cells as eight runs of 64, the sliced ELLPACK order a matrix-vector product
reads); the same call with r and the seven Jacobian planes in eight separate
arrays is timed beside it (``--layouts``).

The same run also times, as extra fields of the JSON line:
  fp32     - the precision form (FP32 storage, FP64 potential/accumulation) on the same grid
  residual - the residual-only kernels (FP64 and FP32)
  batched  - the 64-model uneven ensemble: one persistent kernel replayed from a
             HIP graph vs one launch per model
  adjoint  - FP32 forward residual + vector-Jacobian product on 256 x 256 x 128 (two
             calls), and the same results from one call (tpfa_residual_and_vjp)
  newton   - the backward-Euler residual of Eq. (2) and the matrix-free J v (the
             operator of a Newton-Krylov step) on 512 x 512 x 256, FP64 and FP32
  aniso    - residual + Jacobian with per-direction permeability arrays (kx, ky,
             kz) on 512 x 512 x 256, FP64 and FP32
  slab     - one GPU's share of an 8-GPU y-slab decomposition of the same grid:
             a 512 x 66 x 256 local grid (64 owned rows + one halo row per side),
             FP64 residual + Jacobian of the owned rows (row-range launch)
  pitched  - residual + Jacobian on 500 x 500 x 256, whose rows are off 128-byte
             lines, with contiguous arrays vs arrays of row pitch 512 (FP64, FP32)
  paper10  - the paper's own workload (Sec. 7): 1000 applications of the FP32
             10-flux residual on Nx x Ny x 246 meshes up to 750 x 994 x 246
  copy_ceiling - the library's bandwidth probe: the Jacobian kernels' loads and
             stores without their arithmetic, FP64 and FP32, on the same cell count
  cpu_baseline, cpu_baselines, parity - the FP64 CPU oracle on each workload
             (16^3; 512 x 512 x 256 in FP64 and on the FP32 form's widened inputs;
             the 64-model ensemble; 256 x 256 x 128 forward + VJP), timed on the
             host, and its outputs compared with one GPU application of each
             (launched as timed): the per-cell relative error of every result
The roofline object is for the dominant kernel, the FP64 Jacobian kernel.

    python bench.py [--steps K] [--warmup W] [--sections fp64,fp32,res,newton,aniso,slab,
                                                   pitched,probe,batched,adjoint,paper10,cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells/s (residual+Jacobian) and % of HBM roofline, FP64 vs FP32 vs batched"
HBM_PEAK_GBS = 8000.0
LAYOUTS = {"sliced": "sliced (TPFA_LAUNCH_SLICED): one array of 64-cell row slices, each "
                     "holding r and the 7 Jacobian values of its cells as 8 runs of 64",
           "planes": "r and the 7 Jacobian planes in 8 separate (nz, ny, nx) arrays"}
# algorithmic bytes per cell: each input read once, each output written once
BYTES_FP64_RJ = 8 + 8 + 1 + 8 + 7 * 8      # p, kx, seal -> r, J  = 81
BYTES_FP32_RJ = 4 + 4 + 1 + 4 + 7 * 4      # dp, kx, seal -> r, J = 41
BYTES_FP64_R = 8 + 8 + 1 + 8               # 25
BYTES_FP32_R = 4 + 4 + 1 + 4               # 13
BYTES_FP32_VJP = 4 + 4 + 1 + 4 + 4 + 4     # dp, kx, seal, w -> grad_p, grad_logk = 21
BYTES_FP32_R_VJP = 4 + 4 + 1 + 4 + 3 * 4   # dp, kx, seal, w -> r, grad_p, grad_logk = 25
BYTES_FP32_R10 = 4 + 4 + 4 + 4 + 4         # dp, kx, tne, tse -> r (no seals) = 20
BYTES_FP32_R10T = 4 + 5 * 4 + 4            # dp, tx, ty, tz, tne, tse -> r = 28
# backward-Euler forms: + phi_ref, p_prev (and v in, J v out for the product)
BYTES_FP64_RBE = 8 + 8 + 1 + 8 + 8 + 8      # p, kx, seal, phi, p_prev -> r = 41
BYTES_FP64_JVP = BYTES_FP64_RBE + 8 + 8     # + v -> J v = 57
BYTES_FP32_JVP = 4 + 4 + 1 + 4 + 4 + 4 + 4 + 4  # = 29
BYTES_SPMV_FP64 = 7 * 8 + 8 + 8             # stored J, v -> J v = 72
BYTES_FP64_RJ_K3 = BYTES_FP64_RJ + 8 + 8    # + ky, kz arrays = 97
BYTES_FP32_RJ_K3 = BYTES_FP32_RJ + 4 + 4    # + ky, kz arrays = 49
# the paper's wall times for 1000 applications on 750 x 994 x 246 (Sec. 7, Table 1)
PAPER10_CONTEXT = {"cs2_s": 0.0823, "a100_raja_s": 16.8378, "a100_cuda_s": 14.6573}
# the kernels and the host code that picks their launches: a change to either
# invalidates the committed counter summaries
KERNEL_SRCS = [os.path.join(ROOT, "paper_2304_11274_amd", "csrc", f)
               for f in ("tpfa_tile.h", "tpfa_kernels.hip", "tpfa_march_f64.hip",
                         "tpfa_march_f32.hip", "tpfa_march_f32_plain.hip", "tpfa_api.cpp",
                         "tpfa_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tpfa_jacobian_fp64_512x512x256_traffic.txt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch of the FP64 Jacobian kernel from the committed
    rocprofv3 counter summary, or None if absent or taken on other source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_src_sha") != kernel_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Timer:
    """HIP events on torch's current stream (the stream the kernels run on)."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


# ---------------------------------------------------------------------------
# Per-cell relative error of a GPU result against the FP64 oracle (the metric
# every parity test uses): r against the cell's flux scale sum |F_KL|, the
# Jacobian diagonal against sum |dF_KL/dp_K|, an off-diagonal entry against
# itself, grad p against sum |J_rc| |w_r|, grad ln k against 2 max|w| sum |F|;
# an entry whose scale is 0 must be exactly 0 (else the error is infinite).
# Faces whose potential difference lies within tau of zero may take either
# upwind choice; the errors of cells away from such faces are reported apart.
# ---------------------------------------------------------------------------

def ensemble_members(tp, models, up, padded):
    """Members of the uneven ensemble (FP32 form) on the device: contiguous
    arrays, or rows padded to 128-byte lines (tpfa.pitch_for) with the outputs'
    row padding writable (pad_writes), so that every row is stored in whole
    lines."""
    members = []
    for geo_m in models:
        g = geo_m.grid
        arrs = [up(geo_m.kx32()), up(geo_m.dp32()), up(geo_m.seal)]
        if padded:
            arrs = [tp.to_pitched(a, g) for a in arrs]
        members.append(dict(grid=g, fluid=geo_m.fluid, kx=arrs[0], p=arrs[1], seal=arrs[2],
                            pref=tp.hydrostatic(g, geo_m.fluid), ry=geo_m.ry, rz=geo_m.rz,
                            pad_writes=padded))
    return members


def _rel(np, got, ref, scale):
    d = np.abs(np.asarray(got, np.float64) - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d == 0, 0.0, np.inf))
    return e


def _shift(np, v, axis, side):
    """u[c] = v[c + side e_axis] (0 outside); axis 0/1/2 = x/y/z."""
    u = np.zeros_like(v)
    ax = 2 - axis
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if side > 0:
        dst[ax], src[ax] = slice(0, -1), slice(1, None)
    else:
        dst[ax], src[ax] = slice(1, None), slice(0, -1)
    u[tuple(dst)] = v[tuple(src)]
    return u


def _tie_cells(np, dphi, tau):
    """Cells touching a face (indexed by its lower cell) with |dPhi| <= tau."""
    with np.errstate(invalid="ignore"):
        ties = np.abs(dphi) <= tau
    touch = ties[0] | ties[1] | ties[2]
    for a in range(3):
        touch |= _shift(np, ties[a].astype(np.uint8), a, -1).astype(bool)
    return ties, touch


def _report(np, e, dphi, tau, tol, extra=None):
    ties, touch = _tie_cells(np, dphi, tau)
    away = e[~touch]
    rep = {"max_rel_err": float(e.max()),
           "max_rel_err_away_from_ties": float(away.max()) if away.size else 0.0,
           "tie_faces": int(ties.sum()), "cells": int(e.size), "tol": tol, "tau_Pa": tau,
           "within_tol": bool(e.max() <= tol)}
    if extra:
        rep.update(extra)
    return rep


def rj_errors(np, r, J, ref):
    """Per-cell max of the residual and Jacobian errors."""
    e = _rel(np, r, ref["r"], ref["scale"][0])
    e = np.maximum(e, _rel(np, J[0], ref["J"][0], ref["scale"][1]))
    for q in range(1, 7):
        e = np.maximum(e, _rel(np, J[q], ref["J"][q], np.abs(ref["J"][q])))
    return e


def vjp_errors(np, gp, gm, w, ref):
    """Per-cell max of the grad p and grad ln k errors."""
    J, aw = ref["J"], np.abs(w)
    sp_ = np.abs(J[0]) * aw
    wmax = aw.copy()
    for n in range(6):
        a, side = n // 2, 1 if n % 2 else -1
        # (J^T |w|)_c gains |J_{L,c}| |w_L| from the row of neighbour L = c + side e_a,
        # whose plane for its neighbour c is the opposite one
        sp_ += _shift(np, np.abs(J[1 + (n ^ 1)]) * aw, a, side)
        wmax = np.maximum(wmax, _shift(np, aw, a, side))
    e = _rel(np, gp, ref["grad_p"], sp_)
    return np.maximum(e, _rel(np, gm, ref["grad_logk"], 2.0 * wmax * ref["scale"][0]))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f_:
            return next(l.split(":", 1)[1].strip() for l in f_ if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown CPU"


def oracle_leg(out, args, tp, torch, np, dev, geo, pref):
    """The FP64 oracle on the host (single-threaded, as it stands), timed on each
    workload, and its outputs compared cell by cell with one GPU application of
    the same inputs in the launch the timed sections use."""
    import geomodel
    import oracle
    cpu = _cpu_model()
    cores = len(os.sched_getaffinity(0))
    want = ("r", "J", "scale", "dphi")
    layout = args.layouts.split(",")[0]  # the fp64 / fp32 sections' headline output layout
    base = {"unit": "cells/s", "cores": 1, "kind": "oracle", "host_cores_available": cores}
    out["cpu_baselines"], out["parity"] = {}, {}

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def host(t):
        torch.cuda.synchronize()
        return t.cpu().numpy()

    def timed(fn):
        t0 = time.time()
        res = fn()
        return res, time.time() - t0

    # config 1: 16^3, FP64
    t16 = geomodel.tiny16()
    g1 = t16.grid
    p1 = oracle.pressure(t16)
    ref1, dt1 = timed(lambda: oracle.evaluate(g1, t16.fluid, t16.kx, p1, ry=t16.ry, rz=t16.rz,
                                              seal=t16.seal, want=want))
    reps = max(1, int(0.5 / max(dt1, 1e-4)))
    _, dtr = timed(lambda: [oracle.evaluate(g1, t16.fluid, t16.kx, p1, ry=t16.ry, rz=t16.rz,
                                            seal=t16.seal, want=("r", "J"))
                            for _ in range(reps)])
    k1, pd1, s1 = up(t16.kx), up(p1), up(t16.seal)
    r1, J1 = tp.jacobian(g1, t16.fluid, k1, pd1, seal=s1, ry=t16.ry, rz=t16.rz)
    e1 = rj_errors(np, host(r1), host(J1), ref1)
    for _ in range(10):
        tp.jacobian(g1, t16.fluid, k1, pd1, seal=s1, ry=t16.ry, rz=t16.rz, r_out=r1, J_out=J1)
    with Timer(torch) as tm:
        for _ in range(200):
            tp.jacobian(g1, t16.fluid, k1, pd1, seal=s1, ry=t16.ry, rz=t16.rz, r_out=r1,
                        J_out=J1)
    out["tiny16"] = {"workload": "16x16x16 FP64 residual + Jacobian (latency-bound; no "
                                 "roofline fraction: it fits in cache)",
                     "cells": g1.ncell, "ms_per_step": tm.ms / 200,
                     "cells_per_s": g1.ncell / (tm.ms / 200 / 1e3)}
    out["cpu_baselines"]["tiny16_fp64_rj"] = dict(
        base, value=g1.ncell * reps / dtr,
        sample=f"16x16x16, {reps} evaluations of r + J, {dtr:.2f} s on {cpu}")
    out["parity"]["tiny16_fp64_rj"] = _report(np, e1, ref1["dphi"], 1e-9 * np.abs(p1).max(),
                                              1e-12)
    log(f"oracle leg 16^3: {out['parity']['tiny16_fp64_rj']}")
    del k1, pd1, s1, r1, J1

    # config 2: 512 x 512 x 256 FP64, pressure field 0 (the p the GPU builds)
    g, fl = geo.grid, geo.fluid
    N = g.ncell
    pref_h = pref.cpu().numpy()
    p2 = pref_h[:, None, None] + geo.noise[0]
    ref2, dt2 = timed(lambda: oracle.evaluate(g, fl, geo.kx, p2, ry=geo.ry, rz=geo.rz,
                                              seal=geo.seal, want=want))
    out["cpu_baseline"] = dict(
        base, value=N / dt2,
        sample=f"the whole 512x512x256 workload, pressure field 0: FP64 r + J with the error "
               f"scales and face potentials, single-threaded plain oracle, {dt2:.1f} s on {cpu}")
    kx64, sl = up(geo.kx), up(geo.seal)

    def rj(kx_, p_, **kw):
        """r, J of one application in the headline layout (planes copied out of
        the sliced array), and whether they equal the plane layout's bitwise."""
        rp, Jp = tp.jacobian(g, fl, kx_, p_, seal=sl, ry=geo.ry, rz=geo.rz, **kw)
        if layout != "sliced":
            return rp, Jp, True
        _, Js = tp.jacobian(g, fl, kx_, p_, seal=sl, ry=geo.ry, rz=geo.rz, sliced=True, **kw)
        rs, Js_ = tp.unslice(g, Js)
        del Js
        return rs, Js_, bool(torch.equal(rs, rp) and torch.equal(Js_, Jp))

    r2, J2, same2 = rj(kx64, up(p2))
    rep2 = _report(np, rj_errors(np, host(r2), host(J2), ref2), ref2["dphi"],
                   1e-9 * float(np.abs(p2).max()), 1e-12,
                   {"output_layout": layout, "equal_to_planes_layout_bitwise": same2})
    out["parity"]["fp64_512"] = rep2
    del r2, J2
    log(f"oracle leg 512^2x256 FP64: {rep2} (oracle {dt2:.1f} s)")

    # config 3: the FP32 form on the same geomodel; informational error against
    # the unquantised FP64 inputs (the config-2 oracle), then against the oracle
    # on the widened FP32 inputs (the bound)
    k32 = geo.kx.astype(np.float32)
    dp32 = geo.noise[0].astype(np.float32)
    r3, J3, same3 = rj(up(k32), up(dp32), pref=pref)
    r3, J3 = host(r3), host(J3)
    info = float(rj_errors(np, r3, J3, ref2).max())
    del ref2, p2
    p3 = oracle.widen_fp32(dp32, pref_h)
    ref3, dt3 = timed(lambda: oracle.evaluate(g, fl, k32.astype(np.float64), p3, ry=geo.ry,
                                              rz=geo.rz, seal=geo.seal, want=want))
    rep3 = _report(np, rj_errors(np, r3, J3, ref3), ref3["dphi"], 1e-4, 1e-5,
                   {"max_rel_err_vs_unquantised_fp64_inputs": info, "output_layout": layout,
                    "equal_to_planes_layout_bitwise": same3})
    out["parity"]["fp32_512"] = rep3
    out["cpu_baselines"]["fp32_form_widened_inputs"] = dict(
        base, value=N / dt3,
        sample=f"512x512x256, the FP32 form's inputs widened to FP64 (k, pref[k] + dp): r + J "
               f"with error scales, {dt3:.1f} s on {cpu}")
    for sec, key in (("fp32", "fp32_512"),):
        if sec in out:
            out[sec]["max_rel_err"] = out["parity"][key]["max_rel_err"]
    del r3, J3, ref3, p3, kx64, sl
    torch.cuda.empty_cache()
    log(f"oracle leg 512^2x256 FP32: {rep3} (oracle {dt3:.1f} s)")

    # config 4: the 64-model ensemble (one graph-replayed launch), per model
    if "batched" in out:
        models = geomodel.ensemble()
        refs, t_or, worst = [], 0.0, None
        members = ensemble_members(tp, models, up, padded=True)  # the timed layout
        lt = out["batched"].get("ensemble_launch")
        if lt:
            from paper_2304_11274_amd import autotune
            autotune.apply_ensemble_launch(members, lt)
        ens = tp.Ensemble(members)
        if lt:
            ens.set_schedule(lt[2])
        ens.run()
        torch.cuda.synchronize()
        cells = 0
        for m, geo_m in enumerate(models):
            pw = oracle.widen_fp32(geo_m.dp32(), members[m]["pref"].cpu().numpy())
            ref, dtm = timed(lambda: oracle.evaluate(geo_m.grid, geo_m.fluid,
                                                     geo_m.kx32().astype(np.float64), pw,
                                                     ry=geo_m.ry, rz=geo_m.rz, seal=geo_m.seal,
                                                     want=want))
            t_or += dtm
            cells += geo_m.ncell
            rep = _report(np, rj_errors(np, host(ens.r[m]), host(ens.J[m]), ref), ref["dphi"],
                          1e-4, 1e-5)
            if worst is None or rep["max_rel_err"] > worst["max_rel_err"]:
                worst = dict(rep, model=m)
            tie = rep["tie_faces"]
            refs.append((rep["max_rel_err"], tie))
        ens.close()
        out["parity"]["ensemble"] = {
            "max_rel_err": max(e for e, _ in refs), "tie_faces": sum(t for _, t in refs),
            "tol": 1e-5, "cells": cells, "worst_model": worst,
            "within_tol": bool(max(e for e, _ in refs) <= 1e-5)}
        out["batched"]["max_rel_err"] = out["parity"]["ensemble"]["max_rel_err"]
        out["cpu_baselines"]["ensemble_64_models"] = dict(
            base, value=cells / t_or,
            sample=f"the 64-model ensemble, FP32 inputs widened, model by model, r + J with "
                   f"error scales, {t_or:.1f} s in total on {cpu}")
        del members, ens
        torch.cuda.empty_cache()
        log(f"oracle leg ensemble: {out['parity']['ensemble']}")

    # config 5: 256 x 256 x 128 FP32 forward residual + VJP, set 0
    if "adjoint" in out:
        geo_a = geomodel.adjoint256()
        ga = geo_a.grid
        pra = tp.hydrostatic(ga, geo_a.fluid)
        dpa = geo_a.noise[0].astype(np.float32)
        wa = geo_a.extra["w"][0].astype(np.float32)
        ka = geo_a.kx32()
        kw = dict(seal=up(geo_a.seal), pref=pra, ry=geo_a.ry, rz=geo_a.rz)
        ra = tp.residual(ga, geo_a.fluid, up(ka), up(dpa), **kw)
        gpa, gma = tp.residual_vjp(ga, geo_a.fluid, up(ka), up(dpa), up(wa), **kw)
        pw = oracle.widen_fp32(dpa, pra.cpu().numpy())
        ref, dta = timed(lambda: oracle.evaluate(ga, geo_a.fluid, ka.astype(np.float64), pw,
                                                 ry=geo_a.ry, rz=geo_a.rz, seal=geo_a.seal,
                                                 w=wa.astype(np.float64),
                                                 want=want + ("grad_p", "grad_logk")))
        e = np.maximum(_rel(np, host(ra), ref["r"], ref["scale"][0]),
                       vjp_errors(np, host(gpa), host(gma), wa.astype(np.float64), ref))
        out["parity"]["adjoint"] = _report(np, e, ref["dphi"], 1e-4, 1e-5)
        out["adjoint"]["max_rel_err"] = out["parity"]["adjoint"]["max_rel_err"]
        out["cpu_baselines"]["adjoint_fwd_vjp"] = dict(
            base, value=ga.ncell / dta,
            sample=f"256x256x128, FP32 inputs widened: r, J, grad p and grad ln k with error "
                   f"scales in one pass, {dta:.1f} s on {cpu}")
        log(f"oracle leg adjoint: {out['parity']['adjoint']}")
    out["max_rel_err"] = out["parity"]["fp64_512"]["max_rel_err"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sections",
                    default="fp64,fp32,res,newton,aniso,slab,pitched,probe,batched,adjoint,"
                            "paper10,cpu")
    ap.add_argument("--aux-steps", type=int, default=200,
                    help="steps of the fp32 / residual / batched / adjoint sections")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--paper10-steps", type=int, default=1000,
                    help="applications per mesh in the paper10 section (the paper uses 1000)")
    ap.add_argument("--layouts", default="sliced,planes",
                    help="output layouts of the fp64 and fp32 sections: the first is the "
                         "headline ('sliced' or 'planes'), the others are timed beside it")
    ap.add_argument("--ensemble-launch", default=None,
                    help="fixed ensemble launch 'assignment/kz/schedule' (e.g. tile0/16/grouped) "
                         "instead of the autotuner; per-model launches then take the library "
                         "defaults (for short profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the y-slab "
              "decomposition across GPUs is not implemented (the per-GPU slab launch is: "
              "see the 'slab' section).", file=sys.stderr)
        sys.exit(2)
    sections = set(args.sections.split(","))

    import numpy as np
    import torch

    import geomodel
    import paper_2304_11274_amd as tp

    tp.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    K, W, KA = args.steps, args.warmup, args.aux_steps
    out = {"metric": METRIC, "value": None, "unit": "cells/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    # ---------------------------------------------------------------- inputs
    t0 = time.time()
    geo = geomodel.big512()
    N = geo.ncell
    g, fl = geo.grid, geo.fluid
    pref = tp.hydrostatic(g, fl)
    kx64 = up(geo.kx)
    seal = up(geo.seal)
    noise = [up(nz_) for nz_ in geo.noise]
    del geo.logk
    log(f"inputs 512x512x256 generated and resident in {time.time() - t0:.1f} s")
    layouts = args.layouts.split(",")
    if not layouts or any(lo not in LAYOUTS for lo in layouts):
        ap.error(f"--layouts takes a list of {sorted(LAYOUTS)}")
    out["config"] = {"workload": "512x512x256 FP64 residual + 7-point Jacobian (6-face TPFA), "
                                 "4 rotating pressure fields",
                     "cells": N, "grid": [g.nx, g.ny, g.nz], "cell_m": [g.dx, g.dy, g.dz],
                     "sigma_lnk": 1.5, "ry": 1.0, "rz": 0.1, "seal_fraction": 0.01,
                     "output_layout": LAYOUTS[layouts[0]],
                     "launch": "library default: " + json.dumps(tp.resolve_launch(
                         g, "jacobian", torch.float64, sliced=layouts[0] == "sliced"))}

    def rj_call(prec_kx, pfields, layout, extra):
        """One r + J application per step in an output layout (buffers allocated here)."""
        if layout == "sliced":
            o = dict(J_out=tp.empty_sliced(g, prec_kx.dtype, dev), sliced=True)
        else:
            o = dict(r_out=torch.empty(g.shape, dtype=prec_kx.dtype, device=dev),
                     J_out=torch.empty((7,) + g.shape, dtype=prec_kx.dtype, device=dev))
        return lambda s: tp.jacobian(g, fl, prec_kx, pfields[s % 4], **extra, **o)

    def rate(ms, k, bytes_per_cell):
        t = ms / 1e3 / k
        return {"cells_per_s": N / t, "ms_per_step": ms / k,
                "algorithmic_GBps": bytes_per_cell * N / t / 1e9,
                "hbm_frac": bytes_per_cell * N / t / 1e9 / HBM_PEAK_GBS}

    # ------------------------------------------------------- FP64 r + J (value)
    if "fp64" in sections:
        ps = [(pref[:, None, None] + nz_).contiguous() for nz_ in noise]
        step = rj_call(kx64, ps, layouts[0], dict(seal=seal, ry=geo.ry, rz=geo.rz))
        for s in range(W):
            step(s)
        # five equal chunks of the K timed steps, each bracketed by events on the
        # same stream (no synchronisation inside the timed region): mean and
        # SD of the per-step time over the chunks
        n_chunks = 5 if K >= 5 else 1
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(n_chunks + 1)]
        bounds = [K * c // n_chunks for c in range(n_chunks + 1)]
        with Timer(torch) as tm:
            marks[0].record()
            for c in range(n_chunks):
                for s in range(bounds[c], bounds[c + 1]):
                    step(s)
                marks[c + 1].record()
        res = rate(tm.ms, K, BYTES_FP64_RJ)
        per = [marks[c].elapsed_time(marks[c + 1]) / (bounds[c + 1] - bounds[c])
               for c in range(n_chunks)]
        mean = sum(per) / len(per)
        sd = (sum((x - mean) ** 2 for x in per) / max(1, len(per) - 1)) ** 0.5
        out["ms_per_step_repeats"] = {"n": n_chunks, "mean": mean, "sd": sd, "chunks": per}
        out["value"] = res["cells_per_s"]
        out["ms_per_step"] = res["ms_per_step"]
        traffic = read_traffic()
        out["roofline"] = {"bound": "hbm", "achieved": res["algorithmic_GBps"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": res["hbm_frac"], "traffic": traffic,
                           "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + "
                                           "WRITE_SIZE, copy-calibrated)",
                           "algorithmic_bytes_per_launch": BYTES_FP64_RJ * N,
                           "kernel": "march_kernel<double, JACOBIAN, 64, 8>",
                           "bytes_per_cell": BYTES_FP64_RJ}
        log(f"fp64 r+J ({layouts[0]}): {res['ms_per_step']:.4f} ms/step, "
            f"{res['cells_per_s'] / 1e9:.2f} Gcell/s, {res['algorithmic_GBps']:.0f} GB/s "
            f"({100 * res['hbm_frac']:.1f}% of 8 TB/s)")
        del step
        out["fp64_layouts"] = {layouts[0]: res}
        for lo in layouts[1:]:
            other = rj_call(kx64, ps, lo, dict(seal=seal, ry=geo.ry, rz=geo.rz))
            for s in range(W):
                other(s)
            with Timer(torch) as tm:
                for s in range(K):
                    other(s)
            out["fp64_layouts"][lo] = rate(tm.ms, K, BYTES_FP64_RJ)
            del other
            log(f"fp64 r+J ({lo}): {out['fp64_layouts'][lo]}")
        r = torch.empty(g.shape, dtype=torch.float64, device=dev)
        if "res" in sections:
            for s in range(W):
                tp.residual(g, fl, kx64, ps[s % 4], seal=seal, ry=geo.ry, rz=geo.rz, out=r)
            with Timer(torch) as tm:
                for s in range(KA):
                    tp.residual(g, fl, kx64, ps[s % 4], seal=seal, ry=geo.ry, rz=geo.rz, out=r)
            out.setdefault("residual", {})["fp64"] = rate(tm.ms, KA, BYTES_FP64_R)
            log(f"fp64 residual: {out['residual']['fp64']}")
        del r, ps
        torch.cuda.empty_cache()

    # ------------------------------------------------- FP32 precision form r + J
    if "fp32" in sections:
        dps = [nz_.float() for nz_ in noise]
        kx32 = kx64.float()
        kw = dict(seal=seal, pref=pref, ry=geo.ry, rz=geo.rz)
        lay_res = {}
        for lo in layouts:
            step = rj_call(kx32, dps, lo, kw)
            for s in range(W):
                step(s)
            with Timer(torch) as tm:
                for s in range(KA):
                    step(s)
            lay_res[lo] = rate(tm.ms, KA, BYTES_FP32_RJ)
            del step
        res = dict(lay_res[layouts[0]], output_layout=layouts[0], layouts=lay_res)
        if out["value"]:
            res["speedup_vs_fp64"] = res["cells_per_s"] / out["value"]
        out["fp32"] = res
        log(f"fp32 r+J: {res}")
        r = torch.empty(g.shape, dtype=torch.float32, device=dev)
        if "res" in sections:
            for s in range(W):
                tp.residual(g, fl, kx32, dps[s % 4], seal=seal, pref=pref, ry=geo.ry,
                            rz=geo.rz, out=r)
            with Timer(torch) as tm:
                for s in range(KA):
                    tp.residual(g, fl, kx32, dps[s % 4], seal=seal, pref=pref, ry=geo.ry,
                                rz=geo.rz, out=r)
            out.setdefault("residual", {})["fp32"] = rate(tm.ms, KA, BYTES_FP32_R)
            log(f"fp32 residual: {out['residual']['fp32']}")
        del r, dps, kx32
        torch.cuda.empty_cache()

    # ----------------------- Newton step operators: backward-Euler r and J v
    if "newton" in sections:
        bf = geomodel.be_fields(g, 9)
        phi64, step = up(bf["phi"]), up(bf["dp_step"])
        v64 = up(bf["v"])
        p64 = (pref[:, None, None] + noise[0]).contiguous()
        pn64 = p64 - step
        acc64 = dict(phi=phi64, p_prev=pn64, dt=bf["dt"], cr=bf["cr"])
        kw = dict(seal=seal, ry=geo.ry, rz=geo.rz)
        r = torch.empty(g.shape, dtype=torch.float64, device=dev)
        jv = torch.empty_like(r)
        res = {}
        for name, fn, nbytes in (
                ("fp64_residual_be", lambda: tp.residual_be(g, fl, kx64, p64, acc64, out=r, **kw),
                 BYTES_FP64_RBE),
                ("fp64_jvp_be_with_r", lambda: tp.jvp(g, fl, kx64, p64, v64, accum=acc64,
                                                      want_r=True, out=jv, r_out=r, **kw),
                 BYTES_FP64_JVP + 8),
                ("fp64_jvp_be", lambda: tp.jvp(g, fl, kx64, p64, v64, accum=acc64, out=jv, **kw),
                 BYTES_FP64_JVP)):
            for _ in range(W):
                fn()
            with Timer(torch) as tm:
                for _ in range(KA):
                    fn()
            res[name] = rate(tm.ms, KA, nbytes)
        del r, jv, p64, pn64
        dp32, pn32 = noise[0].float(), (noise[0] - step).float()
        acc32 = dict(phi=phi64.float(), p_prev=pn32, dt=bf["dt"], cr=bf["cr"])
        k32, v32 = kx64.float(), v64.float()
        jv32 = torch.empty(g.shape, dtype=torch.float32, device=dev)
        for _ in range(W):
            tp.jvp(g, fl, k32, dp32, v32, accum=acc32, pref=pref, out=jv32, **kw)
        with Timer(torch) as tm:
            for _ in range(KA):
                tp.jvp(g, fl, k32, dp32, v32, accum=acc32, pref=pref, out=jv32, **kw)
        res["fp32_jvp_be"] = rate(tm.ms, KA, BYTES_FP32_JVP)
        res["stored_J_spmv_bytes_per_cell_fp64"] = BYTES_SPMV_FP64
        out["newton"] = res
        log(f"newton: {res}")
        del phi64, step, v64, dp32, pn32, acc32, k32, v32, jv32
        torch.cuda.empty_cache()

    # --------------- per-direction permeability arrays (kx, ky, kz), r + J
    if "aniso" in sections:
        _, ky_h, kz_h = geomodel.k3_fields(geo.kx, 31)
        ky64, kz64 = up(ky_h), up(kz_h)
        del ky_h, kz_h
        p64 = (pref[:, None, None] + noise[0]).contiguous()
        r = torch.empty(g.shape, dtype=torch.float64, device=dev)
        J = torch.empty((7,) + g.shape, dtype=torch.float64, device=dev)
        res = {"ky_kz": "ky = kx exp(0.3 N(0,1)), kz = 0.1 kx exp(0.5 N(0,1)), seed 31"}
        kw_ = dict(seal=seal, ky=ky64, kz=kz64, r_out=r, J_out=J)
        for _ in range(W):
            tp.jacobian(g, fl, kx64, p64, **kw_)
        with Timer(torch) as tm:
            for _ in range(KA):
                tp.jacobian(g, fl, kx64, p64, **kw_)
        res["fp64_rj"] = rate(tm.ms, KA, BYTES_FP64_RJ_K3)
        del r, J, p64
        torch.cuda.empty_cache()
        k3_32 = (kx64.float(), ky64.float(), kz64.float())
        del ky64, kz64
        dp32 = noise[0].float()
        r = torch.empty(g.shape, dtype=torch.float32, device=dev)
        J = torch.empty((7,) + g.shape, dtype=torch.float32, device=dev)
        kw_ = dict(seal=seal, pref=pref, ky=k3_32[1], kz=k3_32[2], r_out=r, J_out=J)
        for _ in range(W):
            tp.jacobian(g, fl, k3_32[0], dp32, **kw_)
        with Timer(torch) as tm:
            for _ in range(KA):
                tp.jacobian(g, fl, k3_32[0], dp32, **kw_)
        res["fp32_rj"] = rate(tm.ms, KA, BYTES_FP32_RJ_K3)
        out["aniso"] = res
        log(f"aniso: {res}")
        del r, J, k3_32, dp32
        torch.cuda.empty_cache()

    # ------------- one GPU's share of an 8-GPU y-slab decomposition (FP64 r + J)
    if "slab" in sections:
        n_gpu, owned = 8, g.ny // 8
        lo, hi = 3 * owned - 1, 4 * owned + 1  # an interior slab: one halo row per side
        gl = geomodel.Grid(g.nx, hi - lo, g.nz, dx=g.dx, dy=g.dy, dz=g.dz, gk=g.gk)
        # four rotating pressure fields, as on the full grid: one field of the
        # slab (69 MB) would otherwise be read from the 256 MB last-level cache
        pls = [(pref[:, None, None] + nz_[:, lo:hi, :]).contiguous() for nz_ in noise]
        kl = kx64[:, lo:hi, :].contiguous()
        sl = seal[:, lo:hi, :].contiguous()
        r = torch.empty(gl.shape, dtype=torch.float64, device=dev)
        J = torch.empty((7,) + gl.shape, dtype=torch.float64, device=dev)
        kw = dict(seal=sl, ry=geo.ry, rz=geo.rz, r_out=r, J_out=J, rows=(1, 1 + owned))
        for i in range(W):
            tp.jacobian(gl, fl, kl, pls[i % len(pls)], **kw)
        with Timer(torch) as tm:
            for i in range(KA):
                tp.jacobian(gl, fl, kl, pls[i % len(pls)], **kw)
        ms = tm.ms / KA
        cells = g.nx * owned * g.nz
        halo_bytes = g.nx * g.nz * (8 + 8 + 1)  # p, kx, seal of one halo row
        out["slab"] = {"workload": f"{g.nx}x{hi - lo}x{g.nz} local grid, rows 1..{owned} owned "
                                   f"(one GPU of {n_gpu}), FP64 residual + Jacobian",
                       "owned_cells": cells, "ms_per_step": ms,
                       "cells_per_s": cells / (ms / 1e3),
                       "algorithmic_GBps": BYTES_FP64_RJ * cells / (ms / 1e3) / 1e9,
                       "halo_bytes_per_side": halo_bytes,
                       "halo_exchange_us_one_xgmi_link": halo_bytes / 153e9 * 1e6,
                       "inputs": f"{len(pls)} rotating pressure fields with fixed k and seals "
                                 f"({(len(pls) * 8 + 8 + 1) * gl.nx * gl.ny * gl.nz / 1e6:.0f} MB, "
                                 "above the 256 MB last-level cache)"}
        log(f"slab: {out['slab']}")
        del r, J, pls, kl, sl
        torch.cuda.empty_cache()

    # -------- rows off 128-byte lines: contiguous vs row-pitched arrays (r + J)
    if "pitched" in sections:
        nxp, nyp, ldp = 500, 500, 512
        gp_ = geomodel.Grid(nxp, nyp, g.nz, dx=g.dx, dy=g.dy, dz=g.dz, gk=g.gk)
        cells = nxp * nyp * g.nz

        def layout(a, ld):
            """Crop of a 512 x 512 array to 500 x 500, contiguous or with row pitch ld."""
            c = a[..., :nyp, :nxp]
            if ld == nxp:
                return c.contiguous()
            buf = torch.zeros(tuple(c.shape[:-1]) + (ld,), dtype=c.dtype, device=dev)
            buf[..., :nxp].copy_(c)
            return buf[..., :nxp]

        res = {"workload": f"{nxp}x{nyp}x{g.nz} (rows of 4000 / 2000 bytes, off 128-byte "
                           f"lines), residual + Jacobian, contiguous vs row pitch {ldp} "
                           f"(and row pitch {ldp} with the outputs' padding written), and "
                           f"contiguous inputs with the sliced r + J output"}
        for prec in ("fp64", "fp32"):
            for ld, pw, sl_ in ((nxp, False, False), (ldp, False, False), (ldp, True, False),
                                (nxp, False, True)):
                sp = layout(seal, ld)
                if prec == "fp64":
                    kp = layout(kx64, ld)
                    pp = [layout(pref[:, None, None] + nz_[:, :nyp, :nxp], ld)
                          for nz_ in noise[:2]]
                    kw = dict(seal=sp, ry=geo.ry, rz=geo.rz)
                    bpc = BYTES_FP64_RJ
                else:
                    kp = layout(kx64[:, :nyp, :nxp].float(), ld)
                    pp = [layout(nz_[:, :nyp, :nxp].float(), ld) for nz_ in noise[:2]]
                    kw = dict(seal=sp, pref=pref, ry=geo.ry, rz=geo.rz)
                    bpc = BYTES_FP32_RJ
                kw["pad_writes"] = pw
                if sl_:
                    r_, J_ = tp.jacobian(gp_, fl, kp, pp[0], sliced=True, **kw)
                    kw.update(J_out=J_, sliced=True)
                else:
                    r_, J_ = tp.jacobian(gp_, fl, kp, pp[0], **kw)
                    kw.update(r_out=r_, J_out=J_)
                for s_ in range(W):
                    tp.jacobian(gp_, fl, kp, pp[s_ % 2], **kw)
                with Timer(torch) as tm:
                    for s_ in range(KA):
                        tp.jacobian(gp_, fl, kp, pp[s_ % 2], **kw)
                ms = tm.ms / KA
                key = "pitch_%d%s" % (ld, "_pad_writes" if pw else "_sliced" if sl_ else "")
                res.setdefault(prec, {})[key] = {
                    "ms_per_step": ms, "cells_per_s": cells / (ms / 1e3),
                    "algorithmic_GBps": bpc * cells / (ms / 1e3) / 1e9}
                del kp, sp, pp, r_, J_, kw
                torch.cuda.empty_cache()
            res[prec]["speedup_pitched"] = (res[prec]["pitch_%d" % nxp]["ms_per_step"]
                                            / res[prec]["pitch_%d" % ldp]["ms_per_step"])
        out["pitched"] = res
        log(f"pitched: {res}")

    # this device's bandwidth ceiling on the Jacobian kernels' access pattern: the
    # library's streaming probe (read p, k, seal; write eight outputs in the
    # output layout; coalesced, non-temporal), over the benchmark's cell count,
    # FP64 and FP32; the headline layout's probe is the ceiling
    if "probe" in sections:
        out["copy_ceiling"] = {}
        for name, t_, bpc in (("fp64", torch.float64, BYTES_FP64_RJ),
                              ("fp32", torch.float32, BYTES_FP32_RJ)):
            pp_ = noise[0].to(t_)
            kk_ = kx64.to(t_)
            for lo in layouts:
                sl_ = lo == "sliced"
                oo_ = (tp.empty_sliced(g, t_, dev) if sl_
                       else torch.empty((8,) + g.shape, dtype=t_, device=dev))
                for _ in range(3):
                    tp.stream_probe(g, pp_, kk_, seal, out=oo_, sliced=sl_)
                with Timer(torch) as tm:
                    for _ in range(20):
                        tp.stream_probe(g, pp_, kk_, seal, out=oo_, sliced=sl_)
                key = name if lo == layouts[0] else f"{name}_{lo}"
                out["copy_ceiling"][key] = {"bytes_per_cell": bpc, "cells": N,
                                            "output_layout": lo, "ms": tm.ms / 20,
                                            "GBps": bpc * N * 20 / (tm.ms / 1e3) / 1e9}
                del oo_
            del pp_, kk_
        out["copy_ceiling_GBps"] = out["copy_ceiling"]["fp64"]["GBps"]
        log(f"bandwidth probe: {out['copy_ceiling']}")
        # torch's device copy, for context
        src = torch.empty(2 ** 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        with Timer(torch) as tm:
            for _ in range(20):
                dst.copy_(src)
        out["copy_ceiling"]["torch_copy_GBps"] = 2 * src.numel() * 8 * 20 / (tm.ms / 1e3) / 1e9
        del src, dst
    del kx64, seal, noise
    torch.cuda.empty_cache()

    # ------------------------------------------------------- batched ensemble
    if "batched" in sections:
        t0 = time.time()
        models = geomodel.ensemble()
        # rows padded to 128-byte lines with writable output padding (whole-line
        # stores); the contiguous layout is timed below with the same launch
        members = ensemble_members(tp, models, up, padded=True)
        cells = sum(m.ncell for m in models)
        from paper_2304_11274_amd import autotune
        t1 = time.time()
        if args.ensemble_launch:
            lab, z_, sch_ = args.ensemble_launch.split("/")
            ens_best = (lab, z_ if z_.startswith("bal") else int(z_), sch_)
            ens_times = {}
            solo = [(None, None)] * len(members)
            autotune.apply_ensemble_launch(members, ens_best)
        else:
            # per-model launches: each model with its own tuned tile and z-chunk
            table = autotune.tune_members(members)
            solo = [(m["tile"], m["kz_chunk"]) for m in members]
            # one launch: tiles by lane utilisation, z chunk and schedule timed on the batch
            ens_best, ens_times = autotune.tune_ensemble(members)
            log(f"autotuned {len(table)} size classes for per-model launches; ensemble launch "
                f"{ens_best} ({ens_times}) in {time.time() - t1:.1f} s")
        ens = tp.Ensemble(members)
        ens.set_schedule(ens_best[2])
        n_items, n_wg = ens.info()
        log(f"ensemble of {len(members)} models, {cells} cells, {n_items} work items, "
            f"{n_wg} workgroups, set up in {time.time() - t0:.1f} s")
        for _ in range(W):
            ens.run()
        with Timer(torch) as tm:
            for _ in range(KA):
                ens.run()
        t_graph = tm.ms / KA
        # the same models, one launch per model on one stream
        outs = [(tp.empty_pitched(m["grid"], torch.float32, dev),
                 tp.empty_pitched(m["grid"], torch.float32, dev, (7,))) for m in members]
        ens_tiles = sorted({(m["tile"], m["kz_chunk"]) for m in members})
        ens_tiles_of = [(m["tile"], m["kz_chunk"]) for m in members]
        for m, (t_, z_) in zip(members, solo):
            m["tile"], m["kz_chunk"] = t_, z_

        def per_model():
            for m, (rr, JJ) in zip(members, outs):
                tp.jacobian(m["grid"], m["fluid"], m["kx"], m["p"], seal=m["seal"],
                            pref=m["pref"], ry=m["ry"], rz=m["rz"], r_out=rr, J_out=JJ,
                            tile=m["tile"], kz_chunk=m["kz_chunk"], pad_writes=True)
        for _ in range(W):
            per_model()
        with Timer(torch) as tm:
            for _ in range(KA):
                per_model()
        t_loop = tm.ms / KA
        pad_bytes = sum(m["p"].stride(-2) * m["grid"].ny * m["grid"].nz for m in members)
        out["batched"] = {"models": len(members), "cells": cells, "work_items": n_items,
                          "workgroups": n_wg, "schedule": ens_best[2], "dtype": "f32",
                          "layout": "rows padded to 128-byte lines (pitch_for), output "
                                    "padding written (pad_writes): whole-line stores",
                          "cells_with_padding": pad_bytes,
                          "cells_per_s": cells / (t_graph / 1e3), "ms_per_step": t_graph,
                          "algorithmic_GBps": BYTES_FP32_RJ * cells / (t_graph / 1e3) / 1e9,
                          "ensemble_launch": ens_best, "ensemble_tiles": ens_tiles,
                          "ensemble_autotune_ms": ens_times,
                          "per_model_launch_cells_per_s": cells / (t_loop / 1e3),
                          "per_model_launch_ms": t_loop,
                          "speedup_vs_per_model": t_loop / t_graph}
        out["batched"]["hbm_frac"] = out["batched"]["algorithmic_GBps"] / HBM_PEAK_GBS
        if out["value"]:
            out["batched"]["cells_per_s_vs_fp64"] = out["batched"]["cells_per_s"] / out["value"]
        ens.close()
        del ens, outs, members
        torch.cuda.empty_cache()
        # the same models in contiguous arrays (rows off 128-byte lines), same launch
        members = ensemble_members(tp, models, up, padded=False)
        for m, (t_, z_) in zip(members, ens_tiles_of):
            m["tile"], m["kz_chunk"] = t_, z_
        ens = tp.Ensemble(members)
        ens.set_schedule(ens_best[2])
        for _ in range(W):
            ens.run()
        with Timer(torch) as tm:
            for _ in range(KA):
                ens.run()
        t_con = tm.ms / KA
        out["batched"]["contiguous_rows_ms"] = t_con
        out["batched"]["contiguous_rows_cells_per_s"] = cells / (t_con / 1e3)
        log(f"batched: {out['batched']}")
        ens.close()
        del ens, members, models
        torch.cuda.empty_cache()

    # ---------------------------------------------------- adjoint fwd + VJP
    if "adjoint" in sections:
        geo_a = geomodel.adjoint256()
        ga = geo_a.grid
        Na = geo_a.ncell
        pra = tp.hydrostatic(ga, geo_a.fluid)
        ka = up(geo_a.kx32())
        sa = up(geo_a.seal)
        dpa = [up(n_.astype(np.float32)) for n_ in geo_a.noise]
        wa = [up(w_.astype(np.float32)) for w_ in geo_a.extra["w"]]
        ra = torch.empty(ga.shape, dtype=torch.float32, device=dev)
        gpa = torch.empty_like(ra)
        gma = torch.empty_like(ra)
        kw = dict(seal=sa, pref=pra, ry=geo_a.ry, rz=geo_a.rz)

        def fwd_bwd(s):
            tp.residual(ga, geo_a.fluid, ka, dpa[s % 4], out=ra, **kw)
            tp.residual_vjp(ga, geo_a.fluid, ka, dpa[s % 4], wa[s % 4], gp_out=gpa, gm_out=gma,
                            **kw)
        for s in range(W):
            fwd_bwd(s)
        with Timer(torch) as tm:
            for s in range(KA):
                fwd_bwd(s)
        t = tm.ms / KA
        out["adjoint"] = {"workload": "256x256x128 FP32 residual + VJP (grad p, grad ln k)",
                          "cells": Na, "cells_per_s": Na / (t / 1e3), "ms_per_step": t,
                          "algorithmic_GBps": (BYTES_FP32_R + BYTES_FP32_VJP) * Na / (t / 1e3)
                          / 1e9}
        out["adjoint"]["hbm_frac"] = out["adjoint"]["algorithmic_GBps"] / HBM_PEAK_GBS

        # the same results from tpfa_residual_and_vjp: r and the VJP in one pass
        # (value and gradient of w.r; r, grad p and grad ln k bitwise as above)
        def fused(s):
            tp.residual_and_vjp(ga, geo_a.fluid, ka, dpa[s % 4], wa[s % 4], r_out=ra,
                                gp_out=gpa, gm_out=gma, **kw)
        for s in range(W):
            fused(s)
        with Timer(torch) as tm:
            for s in range(KA):
                fused(s)
        t1 = tm.ms / KA
        out["adjoint"]["one_pass"] = {
            "call": "tpfa_residual_and_vjp", "ms_per_step": t1, "cells_per_s": Na / (t1 / 1e3),
            "speedup_vs_two_calls": t / t1,
            "algorithmic_GBps": BYTES_FP32_R_VJP * Na / (t1 / 1e3) / 1e9,
            "bytes_per_cell": BYTES_FP32_R_VJP}
        out["adjoint"]["one_pass"]["hbm_frac"] = (out["adjoint"]["one_pass"]["algorithmic_GBps"]
                                                  / HBM_PEAK_GBS)
        log(f"adjoint: {out['adjoint']}")
        del ka, sa, dpa, wa, ra, gpa, gma
        torch.cuda.empty_cache()

    # ------------------------------- the paper's workload: FP32 10-flux residual
    if "paper10" in sections:
        K10 = args.paper10_steps
        rows = []
        for (nx_, ny_, nz_) in geomodel.PAPER10_SHAPES:
            t0 = time.time()
            geo_p = geomodel.paper10(nx_, ny_, nz_)
            gp_ = geo_p.grid
            prp = tp.hydrostatic(gp_, geo_p.fluid)
            kp, dpp = up(geo_p.kx), up(geo_p.noise[0])
            tn, ts = up(geo_p.extra["tne"]), up(geo_p.extra["tse"])
            del geo_p
            rp = torch.empty(gp_.shape, dtype=torch.float32, device=dev)
            kw = dict(pref=prp, ry=1.0, rz=0.1, out=rp)
            for _ in range(W):
                tp.residual10(gp_, fl, kp, dpp, tn, ts, **kw)
            with Timer(torch) as tm:
                for _ in range(K10):
                    tp.residual10(gp_, fl, kp, dpp, tn, ts, **kw)
            Np = gp_.ncell
            t = tm.ms / K10
            rows.append({"grid": [nx_, ny_, nz_], "cells": Np, "ms_per_application": t,
                         "s_per_1000": t, "cells_per_s": Np / (t / 1e3),
                         "algorithmic_GBps": BYTES_FP32_R10 * Np / (t / 1e3) / 1e9,
                         "hbm_frac": BYTES_FP32_R10 * Np / (t / 1e3) / 1e9 / HBM_PEAK_GBS})
            log(f"paper10 {nx_}x{ny_}x{nz_}: {rows[-1]} (set up {time.time() - t0:.1f} s)")
            del kp, dpp, tn, ts, rp
            torch.cuda.empty_cache()
        # the paper's data model: all ten transmissibilities stored per face
        nx_, ny_, nz_ = geomodel.PAPER10_SHAPES[-1]
        gp_ = geomodel.Grid(nx_, ny_, nz_)
        tr = geomodel.paper10_trans(nx_, ny_, nz_)
        noise_p = geomodel.paper10(nx_, ny_, nz_).noise[0]
        prp = tp.hydrostatic(gp_, fl)
        dpp = up(noise_p)
        tdev = {k: up(v) for k, v in tr.items()}
        del tr, noise_p
        rp = torch.empty(gp_.shape, dtype=torch.float32, device=dev)
        kw = dict(pref=prp, out=rp, trans=(tdev["tx"], tdev["ty"], tdev["tz"]))
        for _ in range(W):
            tp.residual10(gp_, fl, None, dpp, tdev["tne"], tdev["tse"], **kw)
        with Timer(torch) as tm:
            for _ in range(K10):
                tp.residual10(gp_, fl, None, dpp, tdev["tne"], tdev["tse"], **kw)
        t = tm.ms / K10
        Np = gp_.ncell
        trans_row = {"grid": [nx_, ny_, nz_], "cells": Np, "ms_per_application": t,
                     "s_per_1000": t, "cells_per_s": Np / (t / 1e3),
                     "bytes_per_cell": BYTES_FP32_R10T,
                     "algorithmic_GBps": BYTES_FP32_R10T * Np / (t / 1e3) / 1e9,
                     "hbm_frac": BYTES_FP32_R10T * Np / (t / 1e3) / 1e9 / HBM_PEAK_GBS}
        log(f"paper10 with given transmissibilities: {trans_row}")
        del dpp, tdev, rp
        torch.cuda.empty_cache()
        out["paper10"] = {"workload": "FP32 10-flux residual (6 TPFA faces + 4 in-plane "
                                      "diagonal faces), 1000 applications per mesh, no seals",
                          "applications": K10, "bytes_per_cell": BYTES_FP32_R10,
                          "meshes": rows, "given_transmissibilities_750x994x246": trans_row,
                          "paper_750x994x246": PAPER10_CONTEXT}

    # ---------------- the FP64 oracle on the host: timings, and the GPU's errors
    if "cpu" in sections:
        oracle_leg(out, args, tp, torch, np, dev, geo, pref)

    rf = out.get("roofline")
    if rf is not None:
        # the same kernel against this device's own streaming-copy rate, and the
        # counter-measured HBM bytes per launch as a rate
        if out.get("copy_ceiling_GBps"):
            rf["frac_of_copy_ceiling"] = rf["achieved"] / out["copy_ceiling_GBps"]
        if rf.get("traffic") and out.get("ms_per_step"):
            rf["traffic_GBps"] = rf["traffic"] / (out["ms_per_step"] / 1e3) / 1e9
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
