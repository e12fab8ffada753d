"""Host-side checks of the row-pitched layout in the Python binding: the row
pitch of an array is read from its strides (a contiguous array has pitch nx;
a view buf[..., :nx] of a (..., nz, ny, ldx) buffer has pitch ldx), every other
layout is refused, and outputs are allocated in the layout of p. No GPU is
used: these functions only read tensor metadata."""
import pytest
import torch

import geomodel
from paper_2304_11274_amd import api


G = geomodel.Grid(5, 4, 3)


def padded(lead=(), ldx=8, dtype=torch.float64):
    return torch.zeros(tuple(lead) + (G.nz, G.ny, ldx), dtype=dtype)[..., :G.nx]


def test_contiguous_arrays_have_pitch_nx():
    assert api._pitch(torch.zeros(G.nz, G.ny, G.nx), "a", G) == G.nx
    assert api._pitch(torch.zeros(G.nz * G.ny * G.nx), "a", G) == G.nx
    assert api._pitch(torch.zeros(7, G.nz, G.ny, G.nx), "a", G) == G.nx


@pytest.mark.parametrize("ldx", [6, 8, 32])
def test_padded_views_give_their_pitch(ldx):
    assert api._pitch(padded(ldx=ldx), "a", G) == ldx
    assert api._pitch(padded((7,), ldx=ldx), "J", G) == ldx
    assert api._pitch(padded((3,), ldx=ldx)[1], "t", G) == ldx
    # a view that starts at a later column of a wider buffer has the same pitch
    wide = torch.zeros(G.nz, G.ny, ldx + 3)[..., 2:2 + G.nx]
    assert api._pitch(wide, "a", G) == ldx + 3


def test_degenerate_dimensions():
    g = geomodel.Grid(5, 1, 3)
    t = torch.zeros(3, 1, 8)[..., :5]
    assert api._pitch(t, "a", g) == 8
    g = geomodel.Grid(5, 4, 1)
    t = torch.zeros(1, 4, 8)[..., :5]
    assert api._pitch(t, "a", g) == 8


@pytest.mark.parametrize("make", [
    lambda: torch.zeros(G.nz, 6, G.nx)[:, 1:5, :],          # a y slice: planes too far apart
    lambda: torch.zeros(G.nz, G.nx, G.ny).transpose(1, 2),  # x not fastest
    lambda: torch.zeros(G.nz, G.ny, 2 * G.nx)[..., ::2],    # x strided
    lambda: torch.zeros(7, G.nz, G.ny, 8)[:, :, :, :G.nx][::2],  # planes skipped
])
def test_other_layouts_are_refused(make):
    with pytest.raises(ValueError):
        api._pitch(make(), "a", G)


def test_outputs_follow_the_layout_of_p():
    p = padded(ldx=16)
    lay = api._Layout(G)
    lay.take(p, "p")
    r = api._empty(p, lay)
    J = api._empty(p, lay, (7,))
    assert tuple(r.shape) == (G.nz, G.ny, G.nx) and api._pitch(r, "r", G) == 16
    assert tuple(J.shape) == (7, G.nz, G.ny, G.nx) and api._pitch(J, "J", G) == 16
    q = torch.zeros(G.nz * G.ny * G.nx)
    lay = api._Layout(G)
    lay.take(q, "q")
    assert lay.pitch == G.nx and api._empty(q, lay).shape == q.shape
    assert api._empty(q, lay, dtype=torch.float32).dtype == torch.float32


def test_single_rows_fit_any_pitch():
    """A one-row grid's arrays fix no pitch: the call takes it from the
    arrays that do (here J's planes), or nx when none does."""
    g = geomodel.Grid(5, 1, 1)
    p = torch.zeros(1, 1, 8)[..., :5]
    J = torch.zeros(7, 1, 1, 8)[..., :5]
    assert api._pitch(p, "p", g) is None and api._pitch(J, "J", g) == 8
    lay = api._Layout(g)
    lay.take(p, "p")
    assert lay.pitch == 5
    lay.take(J, "J")
    lay.take(torch.zeros(1, 1, 5), "r")
    assert lay.pitch == 8
    with pytest.raises(ValueError, match="row pitch"):
        lay.take(torch.zeros(3, 1, 1, 6)[..., :5], "gm")
    assert api._empty(p, lay, (7,)).stride()[0] == 8



@pytest.mark.parametrize("nx,want", [(500, 512), (512, 512), (17, 32), (33, 64), (750, 768)])
def test_pitch_for_rounds_rows_to_lines(nx, want):
    g = geomodel.Grid(nx, 3, 2)
    assert api.pitch_for(g) == want
    for dtype in (torch.float32, torch.float64, torch.uint8):
        t = api.empty_pitched(g, dtype, "cpu", (7,))
        assert tuple(t.shape) == (7, 2, 3, nx) and api._pitch(t, "t", g) == want
        if dtype != torch.uint8:
            assert (want * t.element_size()) % 128 == 0
    with pytest.raises(ValueError):
        api.empty_pitched(g, torch.float32, "cpu", ldx=nx - 1)


def test_to_pitched_copies_values():
    src = torch.arange(G.nz * G.ny * G.nx, dtype=torch.float64).reshape(G.nz, G.ny, G.nx)
    t = api.to_pitched(src, G)
    assert torch.equal(t, src) and api._pitch(t, "t", G) == 32
    t3 = api.to_pitched(torch.stack([src, -src, 2 * src]), G, ldx=8)
    assert torch.equal(t3[1], -src) and api._pitch(t3, "t3", G) == 8


from hypothesis import given, settings, strategies as st  # noqa: E402


@st.composite
def strided_views(draw):
    """A view of a buffer with strides near those of a row-padded layout:
    each stride is the padded one or, with some probability, another value."""
    nx, ny, nz = draw(st.integers(1, 9)), draw(st.integers(1, 5)), draw(st.integers(1, 4))
    lead = draw(st.sampled_from([0, 1, 3]))
    ld = draw(st.integers(nx, nx + 6))
    exact = (1, ld, ld * ny, ld * ny * nz)
    strides = [e if draw(st.booleans()) or draw(st.booleans()) else draw(st.integers(1, 300))
               for e in exact]
    off = draw(st.integers(0, 5))
    return nx, ny, nz, lead, strides, off


@settings(max_examples=400, deadline=None)
@given(v=strided_views())
def test_accepted_views_have_the_kernel_layout(v):
    """Whatever strides a tensor has, if the binding accepts it with pitch ld,
    element (q, k, j, i) lies at storage offset q*ld*ny*nz + i + ld*(j + ny*k)
    from its first element: the addressing the kernels use."""
    nx, ny, nz, lead, (sx, sy, sz, sp), off = v
    g = geomodel.Grid(nx, ny, nz)
    shape = ((lead,) if lead else ()) + (nz, ny, nx)
    strides = ((sp,) if lead else ()) + (sz, sy, sx)
    need = off + sum((n - 1) * s for n, s in zip(shape, strides)) + 1
    t = torch.arange(need, dtype=torch.float64).as_strided(shape, strides, off)
    try:
        ld = api._pitch(t, "t", g)
    except ValueError:
        return
    t4 = t if lead else t.unsqueeze(0)
    q, k, j, i = torch.meshgrid(*(torch.arange(n) for n in t4.shape), indexing="ij")
    if ld is None:  # a single row: every pitch addresses it as off + i
        assert t4.shape[0] * nz * ny == 1 or t.numel() <= nx
        ld = nx
    assert ld >= nx
    want = off + q * ld * ny * nz + i + ld * (j + ny * k)
    assert torch.equal(t4.to(torch.int64), want.to(torch.int64))


def test_layout_property_sees_accepted_padded_views():
    """The generator above reaches accepted padded layouts (pitch > nx)."""
    t = torch.arange(2 * 3 * 4 * 10, dtype=torch.float64).as_strided((2, 3, 4, 7), (120, 40, 10, 1))
    assert api._pitch(t, "t", geomodel.Grid(7, 4, 3)) == 10
