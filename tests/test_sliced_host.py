"""The sliced r + J layout on the host: the binding's sliced_shape and unslice
follow the header's formula, element (((k ny + j) S + i / 64) 8 + q) 64 + i % 64
for output q (0 = r, 1..7 = the Jacobian planes) of cell (i, j, k), checked
element by element on CPU tensors."""
import itertools

import pytest
import torch

import geomodel
import paper_2304_11274_amd as tp


@pytest.mark.parametrize("shape", [(1, 1, 1), (64, 2, 3), (65, 3, 2), (130, 4, 2), (200, 1, 1)])
def test_unslice_follows_the_header_formula(shape):
    g = geomodel.Grid(*shape)
    nx, ny, nz = shape
    S = (nx + 63) // 64
    assert tp.sliced_shape(g) == (nz, ny, S, 8, 64)
    flat = torch.full((nz * ny * S * 512,), float("nan"), dtype=torch.float64)
    want_r = torch.empty((nz, ny, nx), dtype=torch.float64)
    want_J = torch.empty((7, nz, ny, nx), dtype=torch.float64)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        for q in range(8):
            v = float(((q * 1000 + k) * 1000 + j) * 1000 + i)
            flat[(((k * ny + j) * S + i // 64) * 8 + q) * 64 + i % 64] = v
            if q == 0:
                want_r[k, j, i] = v
            else:
                want_J[q - 1, k, j, i] = v
    r, J = tp.unslice(g, flat.view(tp.sliced_shape(g)))
    assert torch.equal(r, want_r) and torch.equal(J, want_J)
    assert r.is_contiguous() and J.is_contiguous()
