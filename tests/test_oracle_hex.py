"""Hex pins of the oracle (rules: App. C, a parallelogram of hexagons,
player 1 joins top and bottom, player 2 left and right, no draws; the
connection function of the App. B grammar).

Pins: full game trees of the 1x1, 2x2 and 3x3 boards (1; 24 with 12 won by
each player; 257760 with 165600 / 92160 and no draw), the perft closed form
(N^2)!/(N^2-d)! while no chain can yet cross (d <= 2N-1), the no-draw
theorem (a full board has exactly one connected player), and the board's
symmetries (180 degree rotation keeps each player's goal; transposition
and anti-transposition swap the goals, so they map player 1's connection to
player 2's).
"""
import math

import numpy as np
import pytest

from oracle import ref


def hexg(N):
    return ref.Game(ref.HEX, N, N)


def test_tiny_full_trees():
    ref.set_checks(True)
    before = ref.check_failures()
    tot, tab, tr = ref.count_games(hexg(1), ref.init(hexg(1), 1), 1)
    assert tot == 1 and tab[1, 1] == 1
    tot, tab, tr = ref.count_games(hexg(2), ref.init(hexg(2), 1), 4)
    assert tot == 24 and tr == 0
    assert tab[3, 1] == 12 and tab[4, 2] == 12 and tab.sum() == 24
    tot, tab, tr = ref.count_games(hexg(3), ref.init(hexg(3), 1), 9)
    assert tot == 257760 and tr == 0
    assert tab[:, 1].sum() == 165600 and tab[:, 2].sum() == 92160 and tab[:, 0].sum() == 0
    assert list(tab.sum(1)) == [0, 0, 0, 0, 0, 1440, 5760, 43200, 86400, 120960]
    assert ref.check_failures() == before


@pytest.mark.parametrize("N,dmax", [(3, 5), (4, 5), (5, 4), (11, 2)])
def test_perft_closed_form(N, dmax):
    s = ref.init(hexg(N), 1)
    for d in range(1, dmax + 1):
        assert d <= 2 * N - 1
        assert ref.perft(hexg(N), s, d) == math.factorial(N * N) // math.factorial(N * N - d)


def test_no_draw_theorem():
    rng = np.random.default_rng(11)
    for N in (2, 3, 5, 8, 11, 19):
        g = hexg(N)
        for _ in range(3000 if N == 11 else 300):
            b = rng.integers(1, 3, size=N * N).astype(np.int8)
            w1, w2 = ref.holds_win(g, b, 1), ref.holds_win(g, b, 2)
            assert w1 + w2 == 1, (N, b)


def test_symmetries():
    rng = np.random.default_rng(5)
    N = 7
    g = hexg(N)
    hits = 0
    for _ in range(2000):
        dens = rng.uniform(0.3, 0.9)
        b = np.where(rng.random(N * N) < dens, rng.integers(1, 3, N * N), 0).astype(np.int8)
        B = b.reshape(N, N)
        sw = np.where(B == 0, 0, 3 - B).astype(np.int8)
        for p in (1, 2):
            base = ref.holds_win(g, b, p)
            hits += base
            assert ref.holds_win(g, B[::-1, ::-1].copy(), p) == base  # 180 degrees
            assert ref.holds_win(g, sw.T.copy(), 3 - p) == base  # transpose
            assert ref.holds_win(g, sw[::-1, ::-1].T.copy(), 3 - p) == base  # anti-transpose
    assert hits > 100  # the sample exercises connected boards


def test_neighbourhood_orientation():
    """(0,1)-(1,0) touch, (0,0)-(1,1) do not: the parallelogram leans so
    that (r, c) touches (r+1, c-1)."""
    g = hexg(2)
    assert ref.holds_win(g, [0, 1, 1, 0], 1) == 1
    assert ref.holds_win(g, [1, 0, 0, 1], 1) == 0
    assert ref.holds_win(g, [0, 2, 2, 0], 2) == 1
    assert ref.holds_win(g, [2, 0, 0, 2], 2) == 0


def test_random_playouts_always_end_with_a_winner():
    ref.set_checks(True)
    before = ref.check_failures()
    for N, n in ((11, 600), (5, 2000), (1, 10)):
        s = ref.init(hexg(N), n)
        rew, term, stats = ref.playout(hexg(N), s, 3, 100, threads=8)
        assert (s.status == ref.TERMINAL).all()
        assert (s.winner > 0).all()
        assert s.ply.min() >= 2 * N - 1 and s.ply.max() <= N * N
        assert stats[3] == 0 and stats[1] + stats[2] == n
        assert ((s.ply % 2 == 1) == (s.winner == 1)).all()
        assert (rew.sum(1) == 0).all() and (np.abs(rew) == 1).all()
    assert ref.check_failures() == before
