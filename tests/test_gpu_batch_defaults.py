"""Ensembles whose members give no tile: the batch takes each member's
single-grid default tile, or 64x4 where that default is a 512-thread tile the
ensemble kernels do not hold (64x8; 128x4 for FP64 Jacobians whose rows are
off 128-byte lines, e.g. nx = 100, 200, 500). Every member's outputs are
bitwise equal to its own single-grid launch (results never depend on the
tile), in both schedules."""
import numpy as np
import pytest
import torch

import geomodel

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_default_tiles_of_ensemble_members(gpu, orc, prec):
    shapes = [(100, 12, 7), (200, 5, 4), (500, 3, 3), (64, 64, 5), (20, 9, 6), (12, 40, 3)]
    members, singles = [], []
    for q, shape in enumerate(shapes):
        geo = geomodel.random_small(40 + q, *shape, sigma=1.2, seal_prob=0.05)
        g = geo.grid
        if prec == "fp64":
            k, pin, kw = geo.kx, orc.pressure(geo), {}
            assert gpu.resolve_launch(g, "jacobian")["threads"] == 512 or g.nx <= 32
        else:
            k, pin = geo.kx32(), geo.dp32()
            kw = dict(pref=dev(orc.hydrostatic(g, geo.fluid, geo.p_top)))
        members.append(dict(grid=g, fluid=geo.fluid, kx=dev(k), p=dev(pin), seal=dev(geo.seal),
                            ry=geo.ry, rz=geo.rz, **kw))
        singles.append(gpu.jacobian(g, geo.fluid, dev(k), dev(pin), seal=dev(geo.seal),
                                    ry=geo.ry, rz=geo.rz, **kw))
    ens = gpu.Ensemble(members)
    try:
        for schedule in ("persistent", "grouped"):
            ens.set_schedule(schedule)
            ens.run()
            torch.cuda.synchronize()
            for q, (r, J) in enumerate(singles):
                assert torch.equal(ens.r[q], r) and torch.equal(ens.J[q], J), (schedule, q)
    finally:
        ens.close()
