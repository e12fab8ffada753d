"""The bandwidth probe (tpfa_stream_probe) writes what its header defines,
out[q][c] = p[c] + (q + seal[c]) k[c], bit for bit, in both precisions, on
grids whose sizes end inside a 64 x 8 column block and a 32-plane chunk; the
sliced variant writes the same values into the runs of the sliced layout and
nothing beyond nx."""
import numpy as np
import pytest
import torch

import geomodel
import paper_2304_11274_amd as tp

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", [(1, 1, 1), (64, 8, 32), (65, 9, 33), (100, 37, 70), (130, 5, 3),
                                   (500, 61, 40)])
def test_probe_values(gpu, dtype, shape):
    g = geomodel.Grid(*shape)
    rng = np.random.default_rng(sum(shape))
    p = rng.uniform(1e7, 1.1e7, g.shape).astype(dtype)
    k = rng.lognormal(np.log(1e-13), 1.0, g.shape).astype(dtype)
    s = rng.integers(0, 8, g.shape, dtype=np.uint8)
    out = tp.stream_probe(g, torch.from_numpy(p).cuda(), torch.from_numpy(k).cuda(),
                          torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for q in range(8):
        want = p + (q + s).astype(dtype) * k
        assert np.array_equal(got[q], want), q


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", [(1, 1, 1), (64, 8, 32), (65, 9, 33), (130, 5, 3), (100, 37, 70),
                                   (500, 61, 40)])
def test_probe_sliced_values(gpu, dtype, shape):
    g = geomodel.Grid(*shape)
    rng = np.random.default_rng(sum(shape) + 1)
    p = rng.uniform(1e7, 1.1e7, g.shape).astype(dtype)
    k = rng.lognormal(np.log(1e-13), 1.0, g.shape).astype(dtype)
    s = rng.integers(0, 8, g.shape, dtype=np.uint8)
    out = torch.full(tp.sliced_shape(g), float("nan"), dtype=torch.from_numpy(p).dtype,
                     device="cuda")
    tp.stream_probe(g, torch.from_numpy(p).cuda(), torch.from_numpy(k).cuda(),
                    torch.from_numpy(s).cuda(), out=out, sliced=True)
    torch.cuda.synchronize()
    nz, ny, S = tp.sliced_shape(g)[:3]
    flat = out.permute(3, 0, 1, 2, 4).reshape(8, nz, ny, S * 64).cpu().numpy()
    assert np.isnan(flat[..., g.nx:]).all()
    for q in range(8):
        want = p + (q + s).astype(dtype) * k
        assert np.array_equal(flat[q][..., :g.nx], want), q
