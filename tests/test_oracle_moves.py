"""Pins of the oracle's movement games (Sec. 3.2 move mechanic: step and
hop; App. A English Draughts listing; App. C rule texts): Wolf and Sheep
and English Draughts, 8 x 8, action = src * 64 + dst.

Independent pins: move counts worked out by hand (Wolf and Sheep), the
start cells printed in the paper's Draughts listing, the perft counts of
English draughts published by checkers programmers (a multi-capture is one
turn), and hand-built positions for every rule (hop priority, extra turn
with the same piece, promotion before the extra-turn test, the wolf on the
bottom row, a blocked player losing)."""
import os

import numpy as np
import pytest

from oracle import ref

HERE = os.path.dirname(os.path.abspath(__file__))
WS = ref.Game(ref.WOLF_SHEEP, 8, 8)
DR = ref.Game(ref.DRAUGHTS, 8, 8)


def cell(r, c):
    return 8 * r + c


def act(src, dst):
    return 64 * cell(*src) + cell(*dst)


def position(game, pieces, to_move=1, passes=0):
    """One RUNNING env with the given {(r, c): value} pieces."""
    s = ref.init(game, 1)
    s.board[0] = 0
    for (r, c), v in pieces.items():
        s.board[0, cell(r, c)] = v
    s.to_move[0] = to_move
    s.passes[0] = passes
    s.ply[0] = 10
    return s


def moves(game, s):
    m = ref.legal_mask(game, s)[0]
    return sorted((int(a) // 64, int(a) % 64) for a in np.flatnonzero(m))


def play(game, s, src, dst):
    rew, term, _ = ref.step(game, s, [act(src, dst)], want_mask=False)
    return tuple(rew[0]), int(term[0])


# ---------------------------------------------------------------- Wolf and Sheep

def test_wolf_sheep_shapes_and_start():
    assert WS.info() == (64, 4096, 56)
    s = ref.init(WS, 1)
    b = s.board[0]
    assert np.flatnonzero(b == 1).tolist() == [56, 58, 60, 62]  # the dark cells of the bottom row
    assert np.flatnonzero(b == 2).tolist() == [3]               # a central dark cell of the top row
    for i in np.flatnonzero(b):
        assert (i // 8 + i % 8) % 2 == 1
    for bad in ((7, 7), (8, 9), (9, 9)):
        with pytest.raises(Exception):
            ref.Game(ref.WOLF_SHEEP, *bad).info()


def test_wolf_sheep_first_moves_and_perft():
    """The sheep step up-left / up-right: (7,0) has one move, the others two
    (7 moves); the wolf on (0,3) then has (1,2) and (1,4) (14).  At ply 3 the
    sheep have 7 moves if the first move was (7,0)->(6,1) and 6 after each of
    the other six first moves (43 * 2 = 86); at ply 4 the wolf, on row 1,
    has all four diagonal cells free (344)."""
    s = ref.init(WS, 1)
    assert moves(WS, s) == [(56, 49), (58, 49), (58, 51), (60, 51), (60, 53), (62, 53), (62, 55)]
    assert [ref.perft(WS, s, d) for d in (1, 2, 3, 4)] == [7, 14, 86, 344]
    assert ref.perft_turns(WS, s, 4) == 344


def test_wolf_reaching_the_bottom_row_wins():
    s = position(WS, {(6, 1): 2, (7, 4): 1, (5, 6): 1, (3, 3): 1, (2, 0): 1}, to_move=2)
    assert moves(WS, s) == [(49, 40), (49, 42), (49, 56), (49, 58)]
    assert play(WS, s, (6, 1), (7, 0)) == ((-1, 1), 1)
    assert s.winner[0] == 2 and s.status[0] == ref.TERMINAL


def test_sheep_win_by_blocking_the_wolf():
    s = position(WS, {(0, 7): 2, (2, 7): 1, (7, 0): 1, (7, 2): 1, (7, 4): 1}, to_move=1)
    assert play(WS, s, (2, 7), (1, 6)) == ((1, -1), 1)
    assert s.winner[0] == 1


def test_stuck_sheep_lose():
    """Sheep that can no longer move lose once the wolf has moved (the mover
    wins when the next player has no legal action)."""
    s = position(WS, {(0, 1): 1, (0, 3): 1, (0, 5): 1, (0, 7): 1, (3, 4): 2}, to_move=2)
    assert play(WS, s, (3, 4), (4, 5)) == ((-1, 1), 1)
    assert s.winner[0] == 2


def test_wolf_sheep_random_play_invariants():
    n = 400
    s = ref.init(WS, n)
    rng = np.random.default_rng(8)
    row_sum = np.full(n, 28)
    for _ in range(60):
        m = ref.legal_mask(WS, s)
        a = np.array([np.flatnonzero(r)[rng.integers(0, r.sum())] if r.any() else 0 for r in m], np.int32)
        live = s.status == ref.RUNNING
        if not live.any():
            break
        mover = s.to_move.copy()
        ref.step(WS, s, np.where(live, a, 0), want_mask=False)
        for i in range(n):
            assert (s.board[i] == 1).sum() == 4 and (s.board[i] == 2).sum() == 1
            rs = int((np.flatnonzero(s.board[i] == 1) // 8).sum())
            # a sheep ply moves one sheep one row up; a wolf ply moves no sheep
            assert rs == row_sum[i] - (1 if live[i] and mover[i] == 1 else 0)
            row_sum[i] = rs
    assert (s.status == ref.TERMINAL).all()
    assert set(np.unique(s.winner)) <= {1, 2}
    assert s.ply.max() <= 56


# ---------------------------------------------------------------- English Draughts

def test_draughts_start_matches_the_listing():
    golden = {}
    with open(os.path.join(HERE, "golden", "draughts_start.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                golden[k] = [int(x) for x in v]
    assert DR.info() == (64, 4096, 200)
    b = ref.init(DR, 1).board[0]
    assert np.flatnonzero(b == 1).tolist() == golden["P1"]
    assert np.flatnonzero(b == 2).tolist() == golden["P2"]
    # the dark cells (r + c odd) of rows 5-7 and 0-2
    dark = [i for i in range(64) if (i // 8 + i % 8) % 2 == 1]
    assert golden["P1"] == [i for i in dark if i // 8 >= 5]
    assert golden["P2"] == [i for i in dark if i // 8 <= 2]


def test_draughts_perft_published_counts():
    """Published perft counts of 8x8 English draughts, where a multiple
    capture is one move: 7, 49, 302, 1469, 7361, 36768, 179740, 845931.
    Counting plies instead, the extra turns of multiple captures split some
    moves, which first happens at depth 7."""
    s = ref.init(DR, 1)
    expect = [7, 49, 302, 1469, 7361, 36768, 179740, 845931]
    assert [ref.perft_turns(DR, s, d) for d in range(1, 9)] == expect
    assert [ref.perft(DR, s, d) for d in range(1, 7)] == expect[:6]
    assert ref.perft(DR, s, 7) != expect[6]


def test_hop_has_priority_over_steps():
    s = position(DR, {(5, 2): 1, (5, 6): 1, (4, 3): 2, (0, 7): 2}, to_move=1)
    assert moves(DR, s) == [(cell(5, 2), cell(3, 4))]
    assert play(DR, s, (5, 2), (3, 4)) == ((0, 0), 0)
    assert s.board[0, cell(4, 3)] == 0 and s.board[0, cell(3, 4)] == 1 and s.to_move[0] == 2


def test_double_hop_is_an_extra_turn_of_the_same_piece():
    s = position(DR, {(6, 1): 1, (7, 6): 1, (5, 2): 2, (3, 4): 2, (3, 0): 2, (0, 7): 2}, to_move=1)
    assert moves(DR, s) == [(cell(6, 1), cell(4, 3))]
    assert play(DR, s, (6, 1), (4, 3)) == ((0, 0), 0)
    # player 1 moves again, only with the piece on (4, 3), and only hopping
    assert s.to_move[0] == 1 and s.passes[0] == cell(4, 3) + 1
    assert moves(DR, s) == [(cell(4, 3), cell(2, 5))]
    assert play(DR, s, (4, 3), (2, 5)) == ((0, 0), 0)
    assert s.to_move[0] == 2 and s.passes[0] == 0 and s.ply[0] == 12
    assert (s.board[0] == 2).sum() == 2


def test_promotion_then_backward_king_moves():
    s = position(DR, {(1, 2): 1, (6, 5): 2, (7, 0): 1}, to_move=1)
    play(DR, s, (1, 2), (0, 1))
    assert s.board[0, cell(0, 1)] == 5 and s.to_move[0] == 2
    play(DR, s, (6, 5), (7, 4))   # player 2's pawn on its far row becomes a king
    assert s.board[0, cell(7, 4)] == 6
    assert moves(DR, s) == [(cell(0, 1), cell(1, 0)), (cell(0, 1), cell(1, 2)), (cell(7, 0), cell(6, 1))]


def test_promotion_by_a_hop_continues_as_a_king():
    """The listing promotes before it tests for another hop, so a pawn
    crowned by a capture goes on capturing backwards as a king."""
    s = position(DR, {(2, 1): 1, (1, 2): 2, (1, 4): 2, (5, 0): 2}, to_move=1)
    assert play(DR, s, (2, 1), (0, 3)) == ((0, 0), 0)
    assert s.board[0, cell(0, 3)] == 5
    assert s.to_move[0] == 1 and s.passes[0] == cell(0, 3) + 1
    assert moves(DR, s) == [(cell(0, 3), cell(2, 5))]


def test_capturing_the_last_piece_or_blocking_wins():
    s = position(DR, {(5, 2): 1, (4, 3): 2}, to_move=1)
    assert play(DR, s, (5, 2), (3, 4)) == ((1, -1), 1)
    # player 2 still has a pawn, but it cannot move: blocked on (6, 7) by (7, 6)?
    s = position(DR, {(6, 7): 2, (7, 6): 1, (5, 4): 1, (6, 1): 1}, to_move=1)
    assert moves(DR, s)[0][0] in (cell(5, 4), cell(6, 1), cell(7, 6))
    assert play(DR, s, (5, 4), (4, 5)) == ((1, -1), 1)


def test_draughts_random_play_invariants():
    n = 200
    s = ref.init(DR, n)
    rng = np.random.default_rng(5)
    count = np.full(n, 24)
    for _ in range(200):
        live = s.status == ref.RUNNING
        if not live.any():
            break
        m = ref.legal_mask(DR, s)
        a = np.array([np.flatnonzero(r)[rng.integers(0, r.sum())] if r.any() else 0 for r in m], np.int32)
        prev = s.copy()
        ref.step(DR, s, np.where(live, a, 0), want_mask=False)
        for i in np.flatnonzero(live):
            c = int((s.board[i] != 0).sum())
            src, dst = divmod(int(a[i]), 64)
            hop = abs(src // 8 - dst // 8) == 2
            assert c == count[i] - (1 if hop else 0)
            count[i] = c
            # a pawn becomes a king only by moving onto its far row
            if prev.board[i, src] < 5 and s.board[i, dst] >= 5:
                assert dst // 8 == (0 if prev.to_move[i] == 1 else 7)
            assert (s.board[i] >= 5).sum() <= (prev.board[i] >= 5).sum() + 1
            assert set(np.unique(s.board[i])) <= {0, 1, 2, 5, 6}
    assert (s.status != ref.RUNNING).all()
    assert set(np.unique(s.status)) <= {ref.TERMINAL, ref.TRUNCATED}
    assert ((s.status == ref.TRUNCATED) == (s.ply == 200)).all()
