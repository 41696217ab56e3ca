"""Reversi pins of the oracle (rules: App. C; start rules, Sec. 3.1; flip
effect, Sec. 3.2; forced pass and the end after both players pass).

Pins: the published perft counts of Othello from the standard start
(4, 12, 56, 244, 1396, 8200, 55092 for depths 1..7), the symmetry group of
the start position, and disc accounting (a placement that flips f discs
changes the mover's count by 1+f and the opponent's by -f; passes change
nothing).
"""
import numpy as np

from oracle import ref
from tests.oracle_util import apply_seq, random_legal_actions

REV = ref.Game(ref.REVERSI, 8, 8)
PASS = 64


def test_start_position():
    s = ref.init(REV, 1)
    B = s.board[0].reshape(8, 8)
    assert B[3, 3] == 2 and B[4, 4] == 2 and B[3, 4] == 1 and B[4, 3] == 1
    assert (B != 0).sum() == 4
    # the start is symmetric under transposition, anti-transposition and
    # the half turn, and not under a quarter turn (colours would swap)
    assert (B == B.T).all() and (B == B[::-1, ::-1].T).all() and (B == B[::-1, ::-1]).all()
    assert not (B == np.rot90(B)).all()
    m = ref.legal_mask(REV, s)[0]
    assert list(np.flatnonzero(m)) == [19, 26, 37, 44]


def test_perft():
    s = ref.init(REV, 1)
    assert [ref.perft(REV, s, d) for d in range(1, 8)] == [4, 12, 56, 244, 1396, 8200, 55092]


def test_disc_accounting_and_passes():
    rng = np.random.default_rng(2)
    n = 300
    s = ref.init(REV, n)
    placements = np.zeros(n, np.int64)
    saw_pass = False
    for _ in range(130):
        m = ref.legal_mask(REV, s)
        run = s.status == ref.RUNNING
        if not run.any():
            break
        a = random_legal_actions(m, rng)
        mover = s.to_move.copy()
        c1 = (s.board == 1).sum(1)
        c2 = (s.board == 2).sum(1)
        passes_before = s.passes.copy()
        ref.step(REV, s, a, want_mask=False)
        d1 = (s.board == 1).sum(1) - c1
        d2 = (s.board == 2).sum(1) - c2
        for i in np.flatnonzero(run):
            if a[i] == PASS:
                saw_pass = True
                assert m[i, :64].sum() == 0  # only forced
                assert d1[i] == 0 and d2[i] == 0
                assert s.passes[i] == passes_before[i] + 1
            else:
                assert m[i, PASS] == 0
                placements[i] += 1
                dm, do = (d1[i], d2[i]) if mover[i] == 1 else (d2[i], d1[i])
                f = -do
                assert f >= 1 and dm == 1 + f
                assert s.passes[i] == 0
    assert saw_pass
    assert (s.status == ref.TERMINAL).all()
    assert ((s.board != 0).sum(1) == 4 + placements).all()
    # every game ends with two passes in a row
    assert (s.passes == 2).all() and (s.last_action == PASS).all()
    assert s.ply.max() <= 121
    n1, n2 = (s.board == 1).sum(1), (s.board == 2).sum(1)
    exp = np.where(n1 > n2, 1, np.where(n2 > n1, 2, 0))
    assert (s.winner == exp).all()


def test_forced_pass_then_double_pass():
    """Hand-made position: player 1 on a1 (cell 0), player 2 on b1 (cell 1),
    player 2 to move has no flank, so it must pass."""
    s = ref.init(REV, 1)
    s.board[:] = 0
    s.board[0, 0], s.board[0, 1] = 1, 2
    s.to_move[0] = 2
    m = ref.legal_mask(REV, s)[0]
    assert list(np.flatnonzero(m)) == [PASS]
    rew, term, nm = ref.step(REV, s, [PASS])
    assert s.passes[0] == 1 and s.to_move[0] == 1 and term[0] == 0
    assert list(np.flatnonzero(nm[0])) == [2]  # c1 flanks b1
    ref.step(REV, s, [2])
    assert s.passes[0] == 0 and list(s.board[0, :3]) == [1, 1, 1]
    rew, term, nm = ref.step(REV, s, [PASS])  # player 2 has no disc left
    assert term[0] == 0 and list(np.flatnonzero(nm[0])) == [PASS]
    rew, term, nm = ref.step(REV, s, [PASS])  # neither can move: game over
    assert term[0] == 1 and s.status[0] == ref.TERMINAL and s.winner[0] == 1
    assert tuple(rew[0]) == (1, -1) and nm.sum() == 0


def test_multi_direction_flip():
    """Hand-made position: player 1 to move at d4 (3, 3); every neighbour is
    player 2's and player 1 holds the cell two steps out in six of the eight
    directions, so exactly those six discs flip."""
    s = ref.init(REV, 1)
    B = np.zeros((8, 8), np.int8)
    dirs = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
    for dr, dc in dirs:
        B[3 + dr, 3 + dc] = 2
    anchored = dirs[:6]
    for dr, dc in anchored:
        B[3 + 2 * dr, 3 + 2 * dc] = 1
    s.board[0] = B.reshape(-1)
    m = ref.legal_mask(REV, s)[0]
    assert m[27] == 1 and m[PASS] == 0
    ref.step(REV, s, [27], want_mask=False)
    A = s.board[0].reshape(8, 8)
    for dr, dc in dirs:
        assert A[3 + dr, 3 + dc] == (1 if (dr, dc) in anchored else 2)
    assert A[3, 3] == 1 and (A == 1).sum() == 1 + 6 + 6
