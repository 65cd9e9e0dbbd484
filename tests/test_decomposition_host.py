"""Host logic of the decomposed driver (no GPU): why every subdomain takes
the whole domain's grid spacing explicitly, and the side kinds and
neighbours of a px x py split, which follow the domain's boundaries."""

import math

import pytest

import workloads as W
from paper_1710_06423_amd import EXCHANGE, OPEN, PERIODIC
from paper_1710_06423_amd.decomposed import DecomposedSolver, even_cuts


def test_subdomain_extent_alone_does_not_fix_the_spacing():
    """Why subdomains take the spacing explicitly: a subdomain's own extent
    over its cell count differs from the whole domain's spacing in the last
    bit for some cuts (here an Orszag-Tang grid on [0, 2 pi])."""
    x0, x1, n = 0.0, 2 * math.pi, 128
    d = (x1 - x0) / n
    off = [m for m in range(3, n) if ((x0 + m * d) - x0) / m != d or ((x0 + n * d) - (x0 + m * d)) / (n - m) != d]
    assert off, "every cut reproduces the spacing"


def test_even_cuts():
    assert even_cuts(10, 3) == [0, 3, 6, 10]
    assert even_cuts(8000, 2) == [0, 4000, 8000]


def _bare(prob, px, py):
    d = DecomposedSolver.__new__(DecomposedSolver)
    d.prob, d.px, d.py = prob, px, py
    return d


def test_sides_and_neighbours():
    ot = _bare(W.orszag_tang(64), 2, 3)
    for a in range(2):
        for b in range(3):
            assert ot._sides(a, b) == (EXCHANGE,) * 4   # periodic images are neighbours too
    assert ot._neighbour(0, 0, 0) == (1, 0) and ot._neighbour(1, 2, 3) == (1, 0)
    strips = _bare(W.orszag_tang(64), 1, 3)
    assert strips._sides(0, 1) == (PERIODIC, PERIODIC, EXCHANGE, EXCHANGE)
    bw = _bare(W.brio_wu(800), 3, 1)
    assert bw._sides(0, 0) == (OPEN, EXCHANGE, PERIODIC, PERIODIC)
    assert bw._sides(1, 0) == (EXCHANGE, EXCHANGE, PERIODIC, PERIODIC)
    assert bw._sides(2, 0) == (EXCHANGE, OPEN, PERIODIC, PERIODIC)
    # the exchange is symmetric: the side a subdomain unpacks is the one its neighbour packs
    for a in range(2):
        for b in range(3):
            for side in range(4):
                na, nb = ot._neighbour(a, b, side)
                assert ot._neighbour(na, nb, side ^ 1) == (a, b)
