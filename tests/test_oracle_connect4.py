"""Connect Four pins of the oracle (rules: App. C; cell action space with
gravity expressed as a placement constraint, Sec. 3.4).

Pins: the published perft counts of Connect Four for depths 1..8 (found by
exhaustive enumeration; 7^d for d <= 6, 7^7 - 7 at d = 7 because a single
column fills after 6 plies), the 69 winning windows of the 6x7 board, and
the left-right mirror equivariance of the rules.
"""
import itertools

import numpy as np

from oracle import ref
from tests.oracle_util import random_legal_actions

C4 = ref.Game(ref.CONNECT_FOUR, 6, 7)


def test_perft():
    s = ref.init(C4, 1)
    got = [ref.perft(C4, s, d) for d in range(1, 9)]
    assert got == [7, 49, 343, 2401, 16807, 117649, 823536, 5673234]


def test_winning_windows():
    """Exactly 69 sets of four stones are a line of four (24 horizontal,
    21 vertical, 24 diagonal)."""
    n = 0
    b = np.zeros(42, np.int8)
    for cells in itertools.combinations(range(42), 4):
        b[:] = 0
        b[list(cells)] = 1
        n += ref.holds_win(C4, b, 1)
    assert n == 69


def test_first_legal_moves_and_gravity():
    s = ref.init(C4, 1)
    m = ref.legal_mask(C4, s)[0]
    assert list(np.flatnonzero(m)) == [35, 36, 37, 38, 39, 40, 41]  # bottom row
    ref.step(C4, s, [38], want_mask=False)
    m = ref.legal_mask(C4, s)[0]
    assert list(np.flatnonzero(m)) == [31, 35, 36, 37, 39, 40, 41]


def _mirror_action(a):
    r, c = divmod(a, 7)
    return r * 7 + (6 - c)


def test_mirror_equivariance():
    rng = np.random.default_rng(3)
    n = 400
    s = ref.init(C4, n)
    t = ref.init(C4, n)
    for _ in range(42):
        m = ref.legal_mask(C4, s)
        a = random_legal_actions(m, rng)
        b = np.array([_mirror_action(x) for x in a], np.int32)
        rs, ts, _ = ref.step(C4, s, a, want_mask=False)
        rt, tt, _ = ref.step(C4, t, b, want_mask=False)
        assert (rs == rt).all() and (ts == tt).all()
        assert (s.board.reshape(n, 6, 7)[:, :, ::-1] == t.board.reshape(n, 6, 7)).all()
        assert (s.status == t.status).all() and (s.winner == t.winner).all()


def test_random_playouts_shape():
    ref.set_checks(True)
    before = ref.check_failures()
    s = ref.init(C4, 4000)
    rew, term, stats = ref.playout(C4, s, 1, 0, threads=8)
    assert (s.status == ref.TERMINAL).all() and term.all()
    assert s.ply.min() >= 7 and s.ply.max() <= 42
    # a win at ply p belongs to the player who moved at p
    won = s.winner > 0
    assert ((s.ply[won] % 2 == 1) == (s.winner[won] == 1)).all()
    # draws only on a full board
    assert (s.ply[s.winner == 0] == 42).all()
    assert stats[1] + stats[2] + stats[3] == 4000
    assert stats[0] == s.ply.astype(np.int64).sum()
    assert ref.check_failures() == before
