"""Placement of 2D grid rows in the population buffers, on the host (no GPU).

The step kernels store march step i of whole band b at buffer row
i * nfull + b: odd MHD bands march down and count their steps from the top,
and the rows of a last, partial band keep their place. Checkpoint blobs hold
the rows in grid order. These tests check the row map and the blob
reordering through the host check library, which compiles the same header
functions (vklb_host.hpp, vklb_kernels.hpp) the library uses.
"""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CC = os.path.join(ROOT, "paper_2608_04283_amd", "_cellcheck.so")
BLOCK = 256  # cells per storage block


@pytest.fixture(scope="module")
def cc():
    if not os.path.exists(CC):
        from paper_2608_04283_amd import build
        build.build_cellcheck()
    L = ctypes.CDLL(CC)
    L.vklb_cc_mem_row.restype = ctypes.c_longlong
    L.vklb_cc_mem_row.argtypes = [ctypes.c_int] * 4
    L.vklb_cc_reorder_rows.restype = None
    L.vklb_cc_reorder_rows.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 8
    return L


def march_order(b, band, down_odd):
    """Grid rows of whole band b in the order its workgroup marches them."""
    rows = list(range(b * band, (b + 1) * band))
    return rows[::-1] if down_odd and b % 2 else rows


@pytest.mark.parametrize("down_odd", [0, 1])
def test_mem_row_is_the_march_order_permutation(cc, down_odd):
    for ny in (1, 2, 3, 7, 8, 64, 96, 100, 170, 257):
        for band in (1, 2, 3, 4, 5, 7, 8, 16, 17, 32, 40, 64, 300):
            nfull = ny // band
            m = [cc.vklb_cc_mem_row(r, band, nfull, down_odd) for r in range(ny)]
            assert sorted(m) == list(range(ny)), (ny, band)
            for b in range(nfull):
                for i, r in enumerate(march_order(b, band, down_odd)):
                    assert m[r] == i * nfull + b, (ny, band, b, i)
            assert m[nfull * band:] == list(range(nfull * band, ny))
            # nfull = 0: rows in grid order
            assert [cc.vklb_cc_mem_row(r, band, 0, down_odd) for r in range(ny)] == list(range(ny))


def pidx(cell, plane, planes):
    """Element index of (cell, plane) in the blocked layout."""
    return (cell // BLOCK * planes + plane) * BLOCK + cell % BLOCK


@pytest.mark.parametrize("elem", [4, 8])
def test_checkpoint_rows_round_trip_in_grid_order(cc, elem):
    rng = np.random.default_rng(5)
    dt = np.float32 if elem == 4 else np.float64
    for sx, ny, band, down_odd, planes in ((64, 40, 8, 1, 45), (128, 48, 16, 0, 20), (320, 37, 5, 1, 3)):
        nfull = ny // band
        stride = -(-sx * ny // BLOCK) * BLOCK
        dev = rng.standard_normal(stride * planes).astype(dt)
        grid = np.zeros_like(dev)
        cc.vklb_cc_reorder_rows(dev.ctypes.data, grid.ctypes.data, sx, ny, band, nfull, down_odd, planes, elem, 1)
        back = np.zeros_like(dev)
        cc.vklb_cc_reorder_rows(grid.ctypes.data, back.ctypes.data, sx, ny, band, nfull, down_odd, planes, elem, 0)
        cols = np.arange(sx)
        for r in range(ny):
            m = cc.vklb_cc_mem_row(r, band, nfull, down_odd)
            for pl in range(planes):
                g = pidx(r * sx + cols, pl, planes)
                d = pidx(m * sx + cols, pl, planes)
                assert np.array_equal(grid[g], dev[d]), (sx, ny, band, r, pl)  # the blob: grid row r
                assert np.array_equal(back[d], dev[d]), (sx, ny, band, r, pl)  # and back in place
