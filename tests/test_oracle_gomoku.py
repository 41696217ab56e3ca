"""Gomoku pins of the oracle (rules: App. C: a line of exactly five wins,
six or more does not count; full board is a draw).

Pins: perft closed form (no win is possible before ply 9), hand-built
positions whose answer the rule text fixes (a five wins, against the edge
too; an overline of six does not; a five beside an overline still wins),
and the dihedral symmetry of the square board.
"""
import math

import numpy as np
import pytest

from oracle import ref
from tests.oracle_util import apply_seq


def gom(N):
    return ref.Game(ref.GOMOKU, N, N)


@pytest.mark.parametrize("N,dmax", [(15, 2), (5, 4)])
def test_perft_closed_form(N, dmax):
    s = ref.init(gom(N), 1)
    for d in range(1, dmax + 1):
        assert ref.perft(gom(N), s, d) == math.factorial(N * N) // math.factorial(N * N - d)


def _board(N, stones):
    b = np.zeros((N, N), np.int8)
    for (r, c), v in stones.items():
        b[r, c] = v
    return b


def test_exactly_five():
    N, g = 15, gom(15)
    row = lambda cols, r=7, v=1: {(r, c): v for c in cols}
    assert ref.holds_win(g, _board(N, row(range(3, 8))), 1) == 1  # five
    assert ref.holds_win(g, _board(N, row(range(3, 7))), 1) == 0  # four
    assert ref.holds_win(g, _board(N, row(range(3, 9))), 1) == 0  # six
    assert ref.holds_win(g, _board(N, row(range(3, 10))), 1) == 0  # seven
    assert ref.holds_win(g, _board(N, row(range(0, 5))), 1) == 1  # against the left edge
    assert ref.holds_win(g, _board(N, row(range(10, 15))), 1) == 1  # against the right edge
    # a five blocked by the opponent on both ends is still a five
    st = row(range(3, 8))
    st[(7, 2)] = 2
    st[(7, 8)] = 2
    assert ref.holds_win(g, _board(N, st), 1) == 1
    # the other player's stones do not count
    assert ref.holds_win(g, _board(N, row(range(3, 8))), 2) == 0
    # columns and both diagonals
    assert ref.holds_win(g, _board(N, {(r, 4): 2 for r in range(10, 15)}), 2) == 1
    assert ref.holds_win(g, _board(N, {(k, k): 1 for k in range(5)}), 1) == 1
    assert ref.holds_win(g, _board(N, {(k, k): 1 for k in range(6)}), 1) == 0
    assert ref.holds_win(g, _board(N, {(2 + k, 12 - k): 1 for k in range(5)}), 1) == 1
    # overline in one direction and a five in another
    st = row(range(3, 9))
    st.update({(r, 5): 1 for r in range(3, 8)})
    assert ref.holds_win(g, _board(N, st), 1) == 1


def test_step_through_a_five_and_an_overline():
    g, N = gom(15), 15
    idx = lambda r, c: r * N + c
    # player 1 builds c3..c6 on row 7, player 2 answers on row 0; the fifth
    # stone wins at ply 9
    p1 = [idx(7, c) for c in (3, 4, 5, 6, 7)]
    p2 = [idx(0, c) for c in (0, 2, 4, 6)]
    seq = [x for pair in zip(p1, p2) for x in pair] + [p1[-1]]
    seq = seq[:9]
    s, tr = apply_seq(g, seq)
    assert s.status[0] == ref.TERMINAL and s.winner[0] == 1 and s.ply[0] == 9
    # filling the gap of 2 + gap + 3 makes six: no win, the game goes on
    p1 = [idx(7, c) for c in (3, 4, 6, 7, 8, 5)]
    p2 = [idx(0, c) for c in (0, 2, 4, 6, 8)]
    seq = [x for pair in zip(p1, p2) for x in pair] + [p1[-1]]
    s, tr = apply_seq(g, seq[:11])
    assert s.status[0] == ref.RUNNING and s.ply[0] == 11


def test_dihedral_symmetry():
    rng = np.random.default_rng(9)
    N, g = 9, gom(9)
    hits = 0
    for _ in range(1500):
        dens = rng.uniform(0.2, 0.8)
        B = np.where(rng.random((N, N)) < dens, rng.integers(1, 3, (N, N)), 0).astype(np.int8)
        for p in (1, 2):
            base = ref.holds_win(g, B, p)
            hits += base
            for k in range(4):
                R = np.rot90(B, k)
                assert ref.holds_win(g, R.copy(), p) == base
                assert ref.holds_win(g, R.T.copy(), p) == base
    assert hits > 50


def test_random_playouts():
    ref.set_checks(True)
    before = ref.check_failures()
    for N, n in ((15, 300), (5, 3000)):
        s = ref.init(gom(N), n)
        rew, term, stats = ref.playout(gom(N), s, 5, 0, threads=8)
        assert (s.status == ref.TERMINAL).all()
        won = s.winner > 0
        assert (s.ply[won] >= 9).all()
        assert (s.ply[s.winner == 0] == N * N).all()
        assert stats[1] + stats[2] + stats[3] == n
        for i in np.flatnonzero(won)[:50]:
            assert ref.holds_win(gom(N), s.board[i], int(s.winner[i])) == 1
    assert ref.check_failures() == before
