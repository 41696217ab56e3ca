"""Pins of the oracle's Yavalath (App. C: a regular hexagon of diameter 9;
four in a row wins, three in a row without four loses; full board draws).

Cell numbering (the reading stated in the oracle's header): rows top to
bottom, row r of a hexagon with side S holding D - |r - (S-1)| cells, left
to right; axial q = i + max(0, S-1-r) for cell i of row r."""
import math

import numpy as np
import pytest

from oracle import ref
from tests.oracle_util import random_states


def geometry(D):
    """(r, q) of every cell in the numbering above, and the inverse map."""
    S = (D + 1) // 2
    rq = []
    for r in range(D):
        n = D - abs(r - (S - 1))
        q0 = max(0, S - 1 - r)
        rq += [(r, q0 + i) for i in range(n)]
    return rq, {x: i for i, x in enumerate(rq)}


def test_cell_counts():
    for D, cells in ((3, 7), (5, 19), (7, 37), (9, 61)):
        g = ref.Game(ref.YAVALATH, D, D)
        assert g.cells == cells == 3 * ((D + 1) // 2) * ((D - 1) // 2) + 1
        assert g.num_actions == cells
        assert len(geometry(D)[0]) == cells
    with pytest.raises(Exception):
        ref.Game(ref.YAVALATH, 8, 8).info()


@pytest.mark.parametrize("D", [5, 9])
def test_perft_before_any_line(D):
    """Nobody can hold three stones before ply 5, so every sequence of up
    to 4 plies is legal: perft(d) = N!/(N-d)!."""
    g = ref.Game(ref.YAVALATH, D, D)
    s = ref.init(g, 1)
    N = g.cells
    for d in range(1, 5 if D == 5 else 4):
        assert ref.perft(g, s, d) == math.factorial(N) // math.factorial(N - d)


@pytest.mark.slow
def test_perft6_counts_the_losing_threes():
    """Side 3 (19 cells): a game ends at ply 5 exactly when player 1's three
    stones fill one of the 27 straight windows of three cells (9 in each of
    the three directions: rows of 3, 4, 5, 4, 3 cells hold 1, 2, 3, 2, 1),
    in any of 3! orders, with player 2's two stones elsewhere (16 then 15
    choices).  perft(6) = (19!/14! - 27 * 6 * 16 * 15) * 14."""
    g = ref.Game(ref.YAVALATH, 5, 5)
    s = ref.init(g, 1)
    ended5 = 27 * 6 * 16 * 15
    p5 = math.factorial(19) // math.factorial(14)
    assert ref.perft(g, s, 5) == p5
    assert ref.perft(g, s, 6) == (p5 - ended5) * 14


def _play(D, p1, p2, move, mover=1):
    """A position with the given stones ((r, q) lists), mover to play, then
    the move; returns (status, winner)."""
    rq, idx = geometry(D)
    g = ref.Game(ref.YAVALATH, D, D)
    s = ref.init(g, 1)
    for x in p1:
        s.board[0, idx[x]] = 1
    for x in p2:
        s.board[0, idx[x]] = 2
    s.to_move[0] = mover
    s.ply[0] = len(p1) + len(p2)
    ref.step(g, s, np.array([idx[move]], np.int32), want_mask=False)
    return int(s.status[0]), int(s.winner[0])


def test_hand_positions():
    T, R = ref.TERMINAL, ref.RUNNING
    # along (0, 1) on the middle row (r = 4, q = 0..8)
    assert _play(9, [(4, 0), (4, 1), (4, 2)], [(0, 4), (0, 5), (0, 6)], (4, 3)) == (T, 1)  # four wins
    assert _play(9, [(4, 0), (4, 1)], [(0, 4), (0, 5)], (4, 2)) == (T, 2)  # three loses
    assert _play(9, [(4, 0), (4, 1), (4, 3)], [(0, 4), (0, 5), (0, 6)], (4, 2)) == (T, 1)  # gap filled: four
    assert _play(9, [(4, 0), (4, 1), (4, 3), (4, 4)], [(0, 4), (0, 5), (0, 6), (0, 7)], (4, 2)) == (T, 1)  # five
    assert _play(9, [(4, 0), (4, 2)], [(0, 4), (0, 5)], (4, 4)) == (R, -1)  # no line
    # along (1, 0) and (1, -1)
    assert _play(9, [(2, 4), (3, 4), (4, 4)], [(0, 4), (0, 5), (0, 6)], (5, 4)) == (T, 1)
    assert _play(9, [(2, 6), (3, 5)], [(0, 4), (0, 5)], (4, 4)) == (T, 2)
    assert _play(9, [(2, 6), (3, 5), (4, 4)], [(0, 4), (0, 5), (0, 6)], (5, 3)) == (T, 1)
    # (1, 1) is not a line of this board: no loss
    assert _play(9, [(2, 2), (3, 3)], [(0, 4), (0, 5)], (4, 4)) == (R, -1)
    # a move that makes a three in one direction and a four in another wins
    assert _play(9, [(4, 0), (4, 1), (4, 2), (5, 3), (6, 3)],
                 [(0, 4), (0, 5), (0, 6), (0, 7), (1, 3)], (4, 3)) == (T, 1)
    # the opponent's three does not end the game: only the mover's lines count
    assert _play(9, [(8, 0), (8, 2)], [(4, 0), (4, 1), (4, 2)], (0, 4)) == (R, -1)
    # player 2's three loses for player 2
    assert _play(9, [(8, 0), (8, 2), (0, 4)], [(4, 0), (4, 1)], (4, 2), mover=2) == (T, 1)


def _symmetries(D):
    """The 12 symmetries of the hexagon as cell permutations (cube
    coordinates x = q - (S-1), z = r - (S-1), y = -x - z: rotation by 60
    degrees (x, y, z) -> (-z, -x, -y), reflection (x, y, z) -> (x, z, y))."""
    S = (D + 1) // 2
    rq, idx = geometry(D)

    def rot(c):
        x, y, z = c
        return (-z, -x, -y)

    def ref_(c):
        x, y, z = c
        return (x, z, y)

    perms = []
    for m in range(2):
        for k in range(6):
            p = []
            for (r, q) in rq:
                c = (q - (S - 1), None, r - (S - 1))
                c = (c[0], -c[0] - c[2], c[2])
                if m:
                    c = ref_(c)
                for _ in range(k):
                    c = rot(c)
                p.append(idx[(c[2] + S - 1, c[0] + S - 1)])
            perms.append(np.array(p))
    return perms


def test_rules_are_invariant_under_the_twelve_symmetries():
    """Stepping a mapped position with the mapped action gives the same
    status, winner and rewards, and the mapped board: a wrong line
    direction or a wrong row offset breaks this."""
    D = 9
    g = ref.Game(ref.YAVALATH, D, D)
    perms = _symmetries(D)
    assert len({tuple(p) for p in perms}) == 12
    rng = np.random.default_rng(5)
    s = random_states(g, 300, 40, rng)
    m = ref.legal_mask(g, s)
    a = np.array([rng.choice(np.flatnonzero(r)) if r.any() else 0 for r in m], np.int32)
    base = s.copy()
    rew, term, _ = ref.step(g, base, a, want_mask=False)
    for p in perms:
        t = s.copy()
        t.board = np.ascontiguousarray(np.zeros_like(s.board))
        t.board[:, p] = s.board
        r2, t2, _ = ref.step(g, t, p[a].astype(np.int32), want_mask=False)
        assert np.array_equal(r2, rew) and np.array_equal(t2, term)
        assert np.array_equal(t.status, base.status) and np.array_equal(t.winner, base.winner)
        mapped = np.zeros_like(base.board)
        mapped[:, p] = base.board
        assert np.array_equal(t.board, mapped)


def test_random_games_end_legally():
    """Full random games: every game ends by a line (or a full board), the
    oracle's own consistency checks (the opponent never holds three or
    four after the mover's ply) raise nothing, and lengths are at least 5."""
    g = ref.Game(ref.YAVALATH, 9, 9)
    ref.lib().ludax_ref_set_checks(1)
    try:
        before = ref.lib().ludax_ref_check_failures()
        s = ref.init(g, 2000)
        _, _, st = ref.playout(g, s, 7, 0, threads=8)
        assert ref.lib().ludax_ref_check_failures() == before
    finally:
        ref.lib().ludax_ref_set_checks(0)
    assert (s.status == ref.TERMINAL).all()
    assert s.ply.min() >= 5
    assert st[1] + st[2] + st[3] == 2000
