"""Host-side cell orders of the particle sort (md_cell_order): row-major,
Morton and Hilbert ranks of an nd^3 cell grid.  The Hilbert curve of
Sec. 2.2 is pinned by its defining property: consecutive cells along it
are face neighbours."""
import numpy as np
import pytest

import md_inputs as I
from paper_0912_3824_amd import mdx


def _coords(nd):
    c = np.arange(nd ** 3)
    return np.stack([c % nd, (c // nd) % nd, c // (nd * nd)], axis=1)


def _path(nd, order):
    """Cells in rank order, as coordinates."""
    rank = mdx.cell_order_ranks(nd, order)
    assert sorted(rank.tolist()) == list(range(nd ** 3))  # a permutation
    inv = np.empty_like(rank)
    inv[rank] = np.arange(nd ** 3)
    return _coords(nd)[inv]


@pytest.mark.parametrize("nd", [1, 2, 3, 7])
def test_row_order_is_the_identity(nd):
    assert np.array_equal(mdx.cell_order_ranks(nd, "row"), np.arange(nd ** 3))


@pytest.mark.parametrize("nd", [2, 4, 8, 16])
def test_morton_rank_interleaves_the_coordinate_bits(nd):
    bits = nd.bit_length() - 1
    xyz = _coords(nd)
    want = np.zeros(nd ** 3, dtype=np.int64)
    for l in range(bits):  # bit l of x, y, z -> bits 3l, 3l+1, 3l+2
        for d in range(3):
            want |= ((xyz[:, d] >> l) & 1) << (3 * l + d)
    assert np.array_equal(mdx.cell_order_ranks(nd, "morton"), want)


@pytest.mark.parametrize("nd", [2, 4, 8, 16, 32])
def test_hilbert_steps_are_face_neighbours(nd):
    p = _path(nd, "hilbert")
    step = np.abs(np.diff(p, axis=0)).sum(axis=1)
    assert np.all(step == 1)
    assert np.array_equal(p[0], [0, 0, 0])
    # Morton, in contrast, jumps
    assert np.abs(np.diff(_path(nd, "morton"), axis=0)).sum(axis=1).max() > 1 or nd == 2


@pytest.mark.parametrize("nd", [3, 5, 12, 33])
def test_curves_on_other_grids_follow_the_enclosing_power_of_two(nd):
    big = 1 << (nd - 1).bit_length()
    for order in ("morton", "hilbert"):
        full = _path(big, order)
        inside = full[(full < nd).all(axis=1)]
        assert np.array_equal(_path(nd, order), inside), order


def test_bad_arguments_are_rejected():
    with pytest.raises(mdx.MdError):
        mdx.cell_order_ranks(0, "row")
    with pytest.raises(mdx.MdError):
        mdx.cell_order_ranks(4, 3)
    c = mdx.make_config(I.ka_table(), "ds", 0.001, 0.3, 1, 1000)
    assert mdx.md_validate(c) == 0
    c.cell_order = 3
    assert mdx.md_validate(c) == -1
