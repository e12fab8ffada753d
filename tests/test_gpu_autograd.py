"""torch.autograd integration: forward-mode derivatives with respect to p
through the Jacobian-vector product kernel (TPFAResidual and
TPFATransResidual), and the transmissibility-form Function (reverse mode
through its vector-Jacobian kernel): gradcheck in FP64 and agreement with the
oracle's J v and gradients."""
import numpy as np
import pytest
import torch
import torch.autograd.forward_ad as fwAD

import geomodel
from helpers import apply_J, apply_JT

pytestmark = pytest.mark.gpu


def dev(a, grad=False):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda",
                        requires_grad=grad)


def small(shape, seed):
    return geomodel.random_small(seed, *shape, sigma=1.0, seal_prob=0.05)


def test_forward_mode_permeability_form(gpu, orc):
    geo = small((17, 9, 6), 3)
    p = orc.pressure(geo)
    v = np.random.default_rng(2).standard_normal(p.shape)
    seal = torch.from_numpy(geo.seal).cuda()
    with fwAD.dual_level():
        pd = fwAD.make_dual(dev(p), dev(v))
        r = gpu.TPFAResidual.apply(pd, dev(geo.logk), geo.grid, geo.fluid, seal, None, geo.ry,
                                   geo.rz)
        jv = fwAD.unpack_dual(r).tangent
    # the Function forms kx = exp(ln kx) on the GPU; the kernel call gets the same kx
    ref_kernel, _ = gpu.jvp(geo.grid, geo.fluid, torch.exp(dev(geo.logk)), dev(p), dev(v),
                            seal=seal, ry=geo.ry, rz=geo.rz)
    torch.cuda.synchronize()
    assert torch.equal(jv, ref_kernel)
    J = orc.evaluate(geo.grid, geo.fluid, np.exp(geo.logk), p, ry=geo.ry, rz=geo.rz,
                     seal=geo.seal)["J"]
    scale = apply_J(np.abs(J), np.abs(v))
    assert np.all(np.abs(jv.cpu().numpy() - apply_J(J, v)) <= 1e-12 * scale)


def trans_inputs(shape, seed):
    g = geomodel.Grid(*shape)
    rng = np.random.default_rng(seed)
    a = (g.dy * g.dz / g.dx, g.dx * g.dz / g.dy, 0.1 * g.dx * g.dy / g.dz)
    logt = np.stack([np.log(a[d] * 1e-13) + rng.standard_normal(g.shape) for d in range(3)])
    return g, logt


def test_trans_function_gradcheck_fp64(gpu, orc):
    g, logt = trans_inputs((3, 3, 4), 5)
    geo = geomodel.random_small(6, 3, 3, 4)
    p = orc.pressure(geo)
    scale = 1e5

    def f(ps_, lt_):
        return gpu.TPFATransResidual.apply(ps_ * scale, lt_, g, geo.fluid)

    assert torch.autograd.gradcheck(f, (dev(p / scale, True), dev(logt, True)), eps=1e-6,
                                    atol=1e-9, rtol=1e-6)


def test_trans_function_matches_oracle(gpu, orc):
    g, logt = trans_inputs((33, 17, 9), 7)
    geo = geomodel.random_small(8, 33, 17, 9)
    p = orc.pressure(geo)
    w = np.random.default_rng(9).standard_normal(p.shape)
    v = np.random.default_rng(10).standard_normal(p.shape)
    pt, lt = dev(p, True), dev(logt, True)
    r = gpu.TPFATransResidual.apply(pt, lt, g, geo.fluid)
    r.backward(dev(w))
    tr = tuple(np.exp(logt[d]) for d in range(3))
    gp_ref, gt_ref, gt_scale = orc.vjp_general(g, geo.fluid, p, w, trans=tr)
    ev = orc.evaluate_general(g, geo.fluid, p, trans=tr, want=("r", "J", "scale"))
    assert np.all(np.abs(r.detach().cpu().numpy() - ev["r"]) <= 1e-12 * ev["scale"][0])
    gp_scale = apply_JT(np.abs(ev["J"]), np.abs(w))
    assert np.all(np.abs(pt.grad.cpu().numpy() - gp_ref) <= 1e-12 * gp_scale)
    assert np.all(np.abs(lt.grad.cpu().numpy() - gt_ref) <= 1e-12 * gt_scale + 1e-300)
    with fwAD.dual_level():
        pd = fwAD.make_dual(dev(p), dev(v))
        jv = fwAD.unpack_dual(gpu.TPFATransResidual.apply(pd, dev(logt), g, geo.fluid)).tangent
    scale = apply_J(np.abs(ev["J"]), np.abs(v))
    assert np.all(np.abs(jv.cpu().numpy() - apply_J(ev["J"], v)) <= 1e-12 * scale)
