"""Host check of the 3-D stage's face-tile fill (``dma_tile`` and its callers
in ``k3_stage``, ``csrc/sacx3.hip``).

The fill reads the face arrays without clamping positions into the ghost
layers: lane ``l`` of wave instruction ``c`` moves the 16-byte pair
``p = 64 c + l`` of a tile of ``NQ`` quantities x ``H`` rows x ``GW``
columns, at x = X0 - 2 + 2 (p mod GW/2) and y = Y0 - 1 + row, row =
p div (GW/2) mod H.  That is safe only if every address it forms lies inside
its face array, every LDS write inside its padded tile, and every position
a valid cell reads back lies within the ghost layers (where the unclamped
value is the stored face).  This test restates that index arithmetic and the
workspace layout (read from the sources' constants) and checks all three for
the grids the GPU tests run, 512^3, and a sweep of small and ragged grids
(any launch shape stages the same planes overall).
"""

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "paper_1710_06423_amd", "csrc", "sacx3.hip")).read()
HDR = open(os.path.join(ROOT, "include", "sacx.h")).read()


def _const(pattern, text):
    m = re.search(pattern, text)
    assert m, pattern
    return int(m.group(1))


G = _const(r"#define\s+SACX_GHOST\s+(\d+)", HDR)
NQF = _const(r"constexpr int NQF = (\d+);", SRC)
ALIGN = _const(r"constexpr int kAlign = (\d+);", SRC)
TX = _const(r"constexpr int TXF = (\d+), TYF", SRC)
TY = _const(r"constexpr int TXF = \d+, TYF = (\d+);", SRC)
GW = TX + 4
ZSEL = (2, 5, 3, 6)   # G_z tile slots: v_x, B_x, v_y, B_y (GVX, GB1, GVY, GB2)


def _ru(a, b):
    return (a + b - 1) // b * b


def _layout(nx, ny, nz):
    """Layout3 of plan3: pitch, plane and field length in doubles."""
    xoff = ALIGN // 8
    pitch = _ru(xoff + nx + G, ALIGN // 8)
    plane = pitch * (ny + 2 * G)
    fs = _ru(plane * (nz + 2 * G), ALIGN // 8)
    return xoff, pitch, plane, fs


def _tile(nq, h):
    """Quantity, row and pair of every lane of every instruction of a tile fill."""
    pr = GW // 2
    npairs = nq * h * pr
    nch = -(-npairs // 64)
    p = np.minimum(np.arange(nch * 64), npairs - 1)
    row, pair = p // pr, p % pr
    q, j = row // h, row % h
    lds_end = nch * 128                      # doubles written from the tile's start
    padded = -(-nq * h * GW // 128) * 128 + 2   # the tile plus its padding member
    return q, j, pair, lds_end, padded


TILES = [  # (direction, quantities, rows, first plane relative to zb)
    (0, NQF, TY + 2, 0),
    (1, NQF, TY + 1, 0),
    (2, 4, TY + 2, -1),
]


def check(nx, ny, nz):
    """All blocks of a grid at once.  Offsets grow with the plane, and over
    any launch shape the staged planes of a tile run from its first plane
    relative to the block start (0, or -1 for G_z) to n_z - 1, so those two
    planes bound every address."""
    xoff, pitch, plane, fs = _layout(nx, ny, nz)
    ntx, nty = -(-nx // TX), -(-ny // TY)
    for d, nq, h, zfirst in TILES:
        q, j, pair, lds_end, padded = _tile(nq, h)
        assert lds_end <= padded, "a fill writes past its tile's padding"
        slot = np.array([ZSEL[k] for k in q]) if d == 2 else q
        x = (np.arange(ntx) * TX)[:, None, None] - 2 + 2 * pair[None, None, :]
        y = (np.arange(nty) * TY)[None, :, None] - 1 + j[None, None, :]
        xy = xoff + x + (y + G) * pitch
        assert np.all(xy % 2 == 0), "a pair is not 16-byte aligned"
        lo = xy + (zfirst + G) * plane
        hi = xy + (nz - 1 + G) * plane
        assert lo.min() >= 0, (nx, ny, nz, d)
        assert hi.max() + 1 < fs, (nx, ny, nz, d)
        assert ((NQF * d + slot.max()) * fs + hi.max() + 1) < 3 * NQF * fs
    # positions read back by valid cells: staged columns tx+1..tx+3 (x-1..x+1)
    # and rows ty..ty+2 (y-1..y+1) of the cell's block
    for xx in (0, nx - 1):
        assert -G <= xx - 1 and xx + 1 <= nx + G - 1
    for yy in (0, ny - 1):
        assert -G <= yy - 1 and yy + 1 <= ny + G - 1


@pytest.mark.parametrize("shape", [(48, 48, 48), (160, 160, 160), (37, 21, 19), (40, 30, 1), (1, 24, 20),
                                   (26, 1, 17), (512, 512, 512)])
def test_tile_fill_in_bounds_on_tested_grids(shape):
    check(*shape)


def test_tile_fill_in_bounds_on_small_grids():
    for nx in (1, 2, 3, 31, 32, 33, 63, 65):
        for ny in (1, 2, 7, 8, 9, 17):
            for nz in (1, 2, 3):
                check(nx, ny, nz)


def test_layout_constants():
    # the fill's pairs rely on these: an even tile width and 256-byte rows
    assert GW % 2 == 0 and ALIGN % 16 == 0 and (ALIGN // 8) % 2 == 0
