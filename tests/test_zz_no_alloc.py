"""The allocation-free ensemble run (tpfa_ensemble_run_noalloc), called through
the C ABI, against the batch it is a variant of (tpfa_batch_create +
tpfa_batch_run, grouped schedule): two calls in a row, the second on a
smaller input (fewer, smaller models), each bitwise equal to the batch's
outputs for the same models, in FP32 and FP64, Jacobian and residual modes;
and more than 256 models refused on the host."""
import numpy as np
import pytest
import torch

import geomodel
from paper_2304_11274_amd import _lib as L

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def members_of(orc, prec, shapes, seed0):
    out = []
    for q, shape in enumerate(shapes):
        geo = geomodel.random_small(seed0 + q, *shape, sigma=1.3, seal_prob=0.05)
        g = geo.grid
        if prec == "fp64":
            k, pin, kw = geo.kx, orc.pressure(geo), {}
        else:
            k, pin = geo.kx32(), geo.dp32()
            kw = dict(pref=dev(orc.hydrostatic(g, geo.fluid, geo.p_top)))
        out.append(dict(grid=g, fluid=geo.fluid, kx=dev(k), p=dev(pin), seal=dev(geo.seal),
                        ry=geo.ry, rz=geo.rz, **kw))
    return out


def batch_outputs(gpu, members, mode):
    ens = gpu.Ensemble(members, mode=mode)
    ens.set_schedule("grouped")
    try:
        ens.run()
        torch.cuda.synchronize()
        return [(r.clone(), None if J is None else J.clone()) for r, J in zip(ens.r, ens.J)]
    finally:
        ens.close()


def fresh(members, mode):
    outs = []
    for m in members:
        r = torch.full_like(m["p"], float("nan"))
        J = (torch.full((7,) + tuple(m["p"].shape), float("nan"), dtype=m["p"].dtype,
                        device="cuda") if mode == "jacobian" else None)
        outs.append((r, J))
    return outs


BIG = [(70, 9, 13), (100, 20, 9), (16, 16, 5), (33, 7, 40), (1, 1, 1), (129, 3, 6), (40, 41, 3),
       (8, 30, 11), (65, 64, 2), (3, 100, 4), (90, 2, 17)]     # 11 models: two upload launches
SMALL = [(5, 4, 3), (100, 6, 2), (17, 9, 8)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("mode", ["jacobian", "residual"])
def test_noalloc_run_equals_the_batch(gpu, orc, prec, mode):
    print(f"noalloc {prec} {mode}", flush=True)
    for shapes, seed0 in ((BIG, 300), (SMALL, 500)):
        members = members_of(orc, prec, shapes, seed0)
        want = batch_outputs(gpu, members, mode)
        outs = fresh(members, mode)
        gpu.ensemble_run_noalloc(members, outs, mode=mode)
        torch.cuda.synchronize()
        for q, ((r, J), (rw, Jw)) in enumerate(zip(outs, want)):
            assert torch.equal(r, rw), (shapes[q], "r")
            if mode == "jacobian":
                assert torch.equal(J, Jw), (shapes[q], "J")


def test_noalloc_refuses_more_than_256_models(gpu):
    lib = gpu.load()
    arr = (L.Model * 257)()
    rc = lib.tpfa_ensemble_run_noalloc(arr, 257, L.TPFA_FP32, L.TPFA_BATCH_JACOBIAN, None)
    assert rc == L.TPFA_ERR_SHAPE and b"at most 256" in lib.tpfa_last_error()
