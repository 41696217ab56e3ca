"""Pins of the oracle's Pente (App. C: 19x19, five or more in a row wins,
custodial capture of exactly two opponent stones, 10 captured stones win,
the first move at the exact centre).  The state's `passes` byte holds the
captured pairs (player 1 low four bits, player 2 high four bits)."""
import math

import numpy as np
import pytest

from oracle import ref
from tests.oracle_util import random_states

DIR8 = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def test_sizes_and_bound():
    g = ref.Game(ref.PENTE, 19, 19)
    assert g.info() == (361, 361, 377)
    for bad in (4, 6, 21):
        with pytest.raises(Exception):
            ref.Game(ref.PENTE, bad, bad).info()


@pytest.mark.parametrize("N", [5, 19])
def test_centre_first_and_perft_before_any_capture(N):
    """The empty board allows only the centre, and no capture is possible
    before player 2's second stone (ply 4), so perft(d) = (N^2-1)!/(N^2-d)!
    up to d = 4 (a capture at ply 4 does not change how many 4-ply
    sequences exist)."""
    g = ref.Game(ref.PENTE, N, N)
    s = ref.init(g, 1)
    m = ref.legal_mask(g, s)[0]
    assert np.flatnonzero(m).tolist() == [(N // 2) * N + N // 2]
    for d in range(1, 5 if N == 5 else 4):
        assert ref.perft(g, s, d) == math.factorial(N * N - 1) // math.factorial(N * N - d)


def _captures_at_ply4(N):
    """Independent count (by positions, not the oracle's step) of the 4-ply
    sequences on an empty N x N board whose fourth stone captures: player 1
    holds the centre C and X, player 2 holds A; player 2's second stone Y
    brackets C and X (Y + d and Y + 2d are C and X in either order) with A at
    Y + 3d, along some direction d."""
    C = (N // 2, N // 2)
    cells = [(r, c) for r in range(N) for c in range(N)]
    count = 0
    for A in cells:
        if A == C:
            continue
        for X in cells:
            if X in (C, A):
                continue
            for Y in cells:
                if Y in (C, A, X):
                    continue
                for dr, dc in DIR8:
                    pair = {(Y[0] + dr, Y[1] + dc), (Y[0] + 2 * dr, Y[1] + 2 * dc)}
                    if pair == {C, X} and (Y[0] + 3 * dr, Y[1] + 3 * dc) == A:
                        count += 1
                        break
    return count


@pytest.mark.parametrize("N", [5, 7])
def test_perft5_counts_the_captures_at_ply4(N):
    """perft(5) = (N^2 - 4) * perft(4) + 2 * K: each 4-ply sequence leaves
    N^2 - 4 empty cells for the fifth stone, two more when its fourth stone
    captured; K is counted independently."""
    g = ref.Game(ref.PENTE, N, N)
    s = ref.init(g, 1)
    p4 = ref.perft(g, s, 4)
    K = _captures_at_ply4(N)
    assert K > 0
    assert ref.perft(g, s, 5) == (N * N - 4) * p4 + 2 * K


def _state(N, p1, p2, mover, pairs=(0, 0)):
    g = ref.Game(ref.PENTE, N, N)
    s = ref.init(g, 1)
    for r, c in p1:
        s.board[0, r * N + c] = 1
    for r, c in p2:
        s.board[0, r * N + c] = 2
    s.to_move[0] = mover
    s.ply[0] = len(p1) + len(p2)
    s.passes[0] = np.int8(np.uint8(pairs[0] | (pairs[1] << 4)).view(np.int8))
    return g, s


def _move(N, p1, p2, move, mover=1, pairs=(0, 0)):
    g, s = _state(N, p1, p2, mover, pairs)
    ref.step(g, s, np.array([move[0] * N + move[1]], np.int32), want_mask=False)
    b = s.board[0].reshape(N, N)
    pb = int(np.uint8(s.passes[0]))
    return int(s.status[0]), int(s.winner[0]), b, (pb & 15, pb >> 4)


@pytest.mark.parametrize("d", DIR8)
def test_capture_in_every_direction(d):
    N = 19
    Y = (9, 9)
    a, b, x = [(Y[0] + k * d[0], Y[1] + k * d[1]) for k in (1, 2, 3)]
    st, w, board, pairs = _move(N, [x, (0, 0)], [a, b, (18, 18)], Y)
    assert st == ref.RUNNING and pairs == (1, 0)
    assert board[a] == 0 and board[b] == 0 and board[x] == 1 and board[Y] == 1


def test_capture_rules():
    N, T, R = 19, ref.TERMINAL, ref.RUNNING
    # one or three bracketed stones are not captured
    _, _, b, pairs = _move(N, [(9, 11), (0, 0)], [(9, 10), (18, 18)], (9, 9))
    assert pairs == (0, 0) and b[9, 10] == 2
    _, _, b, pairs = _move(N, [(9, 13), (0, 0)], [(9, 10), (9, 11), (9, 12), (18, 18)], (9, 9))
    assert pairs == (0, 0) and b[9, 11] == 2
    # placing into the opponent's bracket captures nothing (player 2 moves into X . O O X? no: into X O . X)
    _, _, b, pairs = _move(N, [(9, 9), (9, 12), (0, 0)], [(9, 10), (18, 18)], (9, 11), mover=2)
    assert pairs == (0, 0) and b[9, 10] == 2 and b[9, 11] == 2
    # two pairs in one move, in two directions
    st, w, b, pairs = _move(N, [(9, 12), (12, 9), (0, 0)], [(9, 10), (9, 11), (10, 9), (11, 9), (18, 18)], (9, 9))
    assert st == R and pairs == (2, 0) and b[9, 10] == b[9, 11] == b[10, 9] == b[11, 9] == 0
    # the fifth pair (10 stones) wins; player 2's count lives in the high bits
    st, w, _, pairs = _move(N, [(9, 12), (0, 0)], [(9, 10), (9, 11), (18, 18)], (9, 9), pairs=(4, 3))
    assert (st, w, pairs) == (T, 1, (5, 3))
    st, w, _, pairs = _move(N, [(9, 10), (9, 11), (18, 18)], [(9, 12), (0, 0), (0, 1)], (9, 9), mover=2,
                            pairs=(2, 4))
    assert (st, w, pairs) == (T, 2, (2, 5))
    # five and six in a row win; four does not
    st, w, _, _ = _move(N, [(5, 1), (5, 2), (5, 3), (5, 4)], [(0, 0), (0, 2), (0, 4)], (5, 5))
    assert (st, w) == (T, 1)
    st, w, _, _ = _move(N, [(5, 1), (5, 2), (5, 4), (5, 5), (5, 6)], [(0, 0), (0, 2), (0, 4), (0, 6)], (5, 3))
    assert (st, w) == (T, 1)
    st, w, _, _ = _move(N, [(5, 1), (5, 2), (5, 3)], [(0, 0), (0, 2)], (5, 4))
    assert (st, w) == (R, -1)
    # a capture on the edge: the bracketing stone must be on the board
    _, _, b, pairs = _move(N, [(0, 5)], [(0, 1), (0, 2)], (0, 3))
    assert pairs == (0, 0)


def _d4(N):
    idx = np.arange(N * N).reshape(N, N)
    maps = []
    for k in range(4):
        for flip in (False, True):
            m = np.rot90(idx, k)
            if flip:
                m = m.T
            maps.append(m.ravel())
    return maps


def test_rules_are_invariant_under_the_square_symmetries():
    N = 19
    g = ref.Game(ref.PENTE, N, N)
    rng = np.random.default_rng(8)
    s = random_states(g, 200, 120, rng)
    m = ref.legal_mask(g, s)
    a = np.array([rng.choice(np.flatnonzero(r)) if r.any() else 0 for r in m], np.int32)
    base = s.copy()
    rew, term, _ = ref.step(g, base, a, want_mask=False)
    inv = lambda p: np.argsort(p)
    for p in _d4(N):
        # p maps new index -> old index; the action moves to where its cell goes
        t = s.copy()
        t.board = np.ascontiguousarray(s.board[:, p])
        r2, t2, _ = ref.step(g, t, inv(p)[a].astype(np.int32), want_mask=False)
        assert np.array_equal(r2, rew) and np.array_equal(t2, term)
        assert np.array_equal(t.status, base.status) and np.array_equal(t.passes, base.passes)
        assert np.array_equal(t.board, base.board[:, p])


def test_random_games_end_legally():
    g = ref.Game(ref.PENTE, 19, 19)
    ref.lib().ludax_ref_set_checks(1)
    try:
        before = ref.lib().ludax_ref_check_failures()
        s = ref.init(g, 1000)
        _, _, st = ref.playout(g, s, 9, 0, threads=8)
        assert ref.lib().ludax_ref_check_failures() == before
    finally:
        ref.lib().ludax_ref_set_checks(0)
    assert (s.status == ref.TERMINAL).all()
    pairs = np.asarray(s.passes).view(np.uint8)
    caps_won = ((s.winner == 1) & ((pairs & 15) >= 5)) | ((s.winner == 2) & ((pairs >> 4) >= 5))
    assert caps_won.any() and (~caps_won).any()  # both ways of winning occur
    assert s.ply.min() >= 9
