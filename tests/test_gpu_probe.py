"""The bandwidth probe (tpfa_stream_probe) writes what its header defines,
out[q][c] = p[c] + (q + seal[c]) k[c], bit for bit, in both precisions, for
sizes that end inside a workgroup's run and span several grid-stride passes."""
import numpy as np
import pytest
import torch

import paper_2304_11274_amd as tp

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [1, 1023, 1025, 300_001, 8_400_000])
def test_probe_values(gpu, dtype, n):
    rng = np.random.default_rng(n)
    p = rng.uniform(1e7, 1.1e7, n).astype(dtype)
    k = rng.lognormal(np.log(1e-13), 1.0, n).astype(dtype)
    s = rng.integers(0, 8, n, dtype=np.uint8)
    out = tp.stream_probe(torch.from_numpy(p).cuda(), torch.from_numpy(k).cuda(),
                          torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for q in range(8):
        want = p + (q + s).astype(dtype) * k
        assert np.array_equal(got[q], want), q
