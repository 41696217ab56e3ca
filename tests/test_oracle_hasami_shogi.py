"""Pins of the oracle's Dai Hasami Shogi (App. C; Sec. 3.2 move mechanic
with slide and hop): 9 x 9, player 1 on rows 7-8 and player 2 on rows 0-1,
rook slides, hops over any adjacent piece, custodial captures of runs
enclosed by the moved piece, corner captures, and five in a row or column
outside the mover's start rows.  Action = src * 81 + dst.

Independent pins: move counts worked out by hand (plies 1 and 2), a
brute-force count of the 3-ply sequences and of their captures by a
separate move generator written here, and hand-built positions for every
rule."""
import numpy as np
import pytest

from oracle import ref

G = ref.Game(ref.HASAMI_SHOGI, 9, 9)
ORTH = [(-1, 0), (0, -1), (0, 1), (1, 0)]


def cell(r, c):
    return 9 * r + c


def act(src, dst):
    return 81 * cell(*src) + cell(*dst)


def position(pieces, to_move=1):
    s = ref.init(G, 1)
    s.board[0] = 0
    for (r, c), v in pieces.items():
        s.board[0, cell(r, c)] = v
    s.to_move[0] = to_move
    s.ply[0] = 10
    return s


def play(s, src, dst):
    rew, term, _ = ref.step(G, s, [act(src, dst)], want_mask=False)
    return tuple(rew[0]), int(term[0])


def test_shapes_and_start():
    assert G.info() == (81, 6561, 200)
    b = ref.init(G, 1).board[0].reshape(9, 9)
    assert (b[:2] == 2).all() and (b[7:] == 1).all() and (b[2:7] == 0).all()
    for bad in ((8, 8), (9, 8), (11, 11)):
        with pytest.raises(Exception):
            ref.Game(ref.HASAMI_SHOGI, *bad).info()


def test_perft_by_hand():
    """Ply 1: each row-7 piece slides up 1-5 cells (45), each row-8 piece
    hops its row-7 neighbour to row 6 (9): 54.  Ply 2: if player 1's piece
    went to row r >= 3 of column c, player 2's (1, c) slides r - 2 cells, the
    other eight row-1 pieces 5 each, the nine row-0 pieces hop to row 2:
    47 + r moves; a piece on (2, c) leaves (1, c) one hop to (3, c) and blocks
    the hop from (0, c): 49.  Sum over the 54 first moves: 9 x (50 + 51 + 52
    + 53 + 49) + 9 x 53 = 2772."""
    s = ref.init(G, 1)
    assert ref.perft(G, s, 1) == 54
    assert ref.perft(G, s, 2) == 2772


def _gen(board, me):
    """Independent move generator: (src, dst) pairs of `me` on a dict board."""
    out = []
    for (r, c), v in board.items():
        if v != me:
            continue
        for dr, dc in ORTH:
            k = 1
            while 0 <= r + k * dr < 9 and 0 <= c + k * dc < 9 and board.get((r + k * dr, c + k * dc), 0) == 0:
                out.append(((r, c), (r + k * dr, c + k * dc)))
                k += 1
            if k == 1 and 0 <= r + dr < 9 and 0 <= c + dc < 9:
                t = (r + 2 * dr, c + 2 * dc)
                if 0 <= t[0] < 9 and 0 <= t[1] < 9 and board.get(t, 0) == 0:
                    out.append(((r, c), t))
    return out


def _apply(board, me, src, dst):
    """Independent move application: move, enclosed runs, corners."""
    b = dict(board)
    del b[src]
    b[dst] = me
    opp = 3 - me
    for dr, dc in ORTH:
        run, k = [], 1
        while b.get((dst[0] + k * dr, dst[1] + k * dc), 0) == opp:
            run.append((dst[0] + k * dr, dst[1] + k * dc))
            k += 1
        if run and b.get((dst[0] + k * dr, dst[1] + k * dc), 0) == me:
            for p in run:
                del b[p]
    for cr, cc in ((0, 0), (0, 8), (8, 0), (8, 8)):
        nb = [(cr + (1 if cr == 0 else -1), cc), (cr, cc + (1 if cc == 0 else -1))]
        if b.get((cr, cc), 0) == opp and all(b.get(x, 0) == me for x in nb) and dst in nb:
            del b[(cr, cc)]
    return b


def _expand(state):
    """Every legal ply from every env of `state` (the oracle's mask and
    step): the batch of resulting states."""
    m = ref.legal_mask(G, state)
    rows, acts = np.nonzero(m)
    nxt = state.subset(rows)
    ref.step(G, nxt, acts.astype(np.int32), want_mask=False)
    return nxt


def test_three_plies_against_an_independent_generator():
    """All 3-ply sequences: their number (perft 3) and how many of them
    capture on the third ply (the earliest ply a capture can happen: a
    hop at ply 2 vacates the cell it would need), by the oracle and by a
    separate move generator written here."""
    start = {(r, c): (2 if r < 2 else 1) for r in (0, 1, 7, 8) for c in range(9)}
    total, captures = 0, 0
    for m1 in _gen(start, 1):
        b1 = _apply(start, 1, *m1)
        for m2 in _gen(b1, 2):
            b2 = _apply(b1, 2, *m2)
            assert len(b2) == 36
            for m3 in _gen(b2, 1):
                total += 1
                captures += len(_apply(b2, 1, *m3)) < 36
    assert captures > 0
    s3 = _expand(_expand(_expand(ref.init(G, 1))))
    assert s3.n == total == ref.perft(G, ref.init(G, 1), 3)
    assert int(((s3.board != 0).sum(1) < 36).sum()) == captures


def test_custodial_captures():
    # one piece, enclosed by the moved piece from the right
    s = position({(4, 2): 1, (4, 3): 2, (7, 4): 1, (0, 0): 2})
    play(s, (7, 4), (4, 4))
    assert s.board[0, cell(4, 3)] == 0 and s.to_move[0] == 2
    # a run of three, from a slide along the row
    s = position({(4, 2): 1, (4, 3): 2, (4, 4): 2, (4, 5): 2, (4, 8): 1, (0, 0): 2})
    play(s, (4, 8), (4, 6))
    assert (s.board[0, [cell(4, 3), cell(4, 4), cell(4, 5)]] == 0).all()
    # vertically, and in two directions at once
    s = position({(2, 4): 1, (3, 4): 2, (5, 4): 2, (6, 4): 1, (4, 0): 1, (0, 8): 2})
    play(s, (4, 0), (4, 4))
    assert s.board[0, cell(3, 4)] == 0 and s.board[0, cell(5, 4)] == 0
    # not enclosed: a gap, the board edge, or the mover's piece not at the end
    s = position({(4, 0): 2, (4, 1): 2, (4, 5): 1, (6, 2): 1, (0, 8): 2})
    play(s, (6, 2), (4, 2))
    assert s.board[0, cell(4, 1)] == 2 and s.board[0, cell(4, 0)] == 2
    # moving between two opponent pieces is safe
    s = position({(4, 2): 2, (4, 4): 2, (6, 3): 1, (0, 8): 2})
    play(s, (6, 3), (4, 3))
    assert s.board[0, cell(4, 3)] == 1


def test_hops_capture_nothing():
    s = position({(4, 4): 1, (3, 4): 2, (4, 5): 1, (0, 8): 2})
    play(s, (4, 4), (2, 4))   # over the opponent's piece
    assert s.board[0, cell(3, 4)] == 2
    s = position({(4, 4): 1, (4, 5): 1, (0, 8): 2})
    play(s, (4, 4), (4, 6))   # over its own piece
    assert s.board[0, cell(4, 5)] == 1 and s.board[0, cell(4, 6)] == 1


def test_corner_capture():
    s = position({(0, 0): 2, (1, 0): 1, (5, 1): 1, (0, 8): 2})
    play(s, (5, 1), (0, 1))
    assert s.board[0, cell(0, 0)] == 0
    # both neighbours already the mover's: a move elsewhere captures nothing
    s = position({(8, 8): 2, (7, 8): 1, (8, 7): 1, (4, 4): 1, (0, 0): 2})
    play(s, (4, 4), (4, 5))
    assert s.board[0, cell(8, 8)] == 2


def test_five_outside_the_start_rows_wins():
    s = position({(4, 0): 1, (4, 1): 1, (4, 2): 1, (4, 3): 1, (6, 4): 1, (0, 8): 2, (0, 6): 2})
    assert play(s, (6, 4), (4, 4)) == ((1, -1), 1)
    # five on player 1's start row 7 do not count
    s = position({(7, 0): 1, (7, 1): 1, (7, 2): 1, (7, 3): 1, (5, 4): 1, (0, 8): 2, (0, 6): 2})
    assert play(s, (5, 4), (7, 4)) == ((0, 0), 0)
    # a column: rows 2-6 win for player 1; rows 3-7 touch its start rows
    s = position({(2, 0): 1, (3, 0): 1, (4, 0): 1, (5, 0): 1, (6, 5): 1, (0, 8): 2, (0, 6): 2})
    assert play(s, (6, 5), (6, 0)) == ((1, -1), 1)
    s = position({(7, 0): 1, (3, 0): 1, (4, 0): 1, (5, 0): 1, (6, 5): 1, (0, 8): 2, (0, 6): 2})
    assert play(s, (6, 5), (6, 0)) == ((0, 0), 0)
    # player 2: rows 2-8 are outside its start rows
    s = position({(8, 0): 2, (8, 1): 2, (8, 2): 2, (8, 3): 2, (5, 4): 2, (4, 8): 1}, to_move=2)
    assert play(s, (5, 4), (8, 4)) == ((-1, 1), 1)


def test_blocked_player_loses():
    s = position({(0, 0): 2, (0, 1): 1, (0, 2): 1, (1, 0): 1, (5, 0): 1})
    assert play(s, (5, 0), (2, 0)) == ((1, -1), 1)
    assert s.board[0, cell(0, 0)] == 2


def test_random_play_invariants():
    n = 150
    s = ref.init(G, n)
    rng = np.random.default_rng(9)
    for _ in range(200):
        live = s.status == ref.RUNNING
        if not live.any():
            break
        m = ref.legal_mask(G, s)
        a = np.array([np.flatnonzero(r)[rng.integers(0, r.sum())] if r.any() else 0 for r in m], np.int32)
        prev = s.copy()
        ref.step(G, s, np.where(live, a, 0), want_mask=False)
        for i in np.flatnonzero(live):
            me = prev.to_move[i]
            assert (s.board[i] == me).sum() == (prev.board[i] == me).sum()        # the mover loses nothing
            assert (s.board[i] == 3 - me).sum() <= (prev.board[i] == 3 - me).sum()
            src, dst = divmod(int(a[i]), 81)
            assert s.board[i, dst] == me and s.board[i, src] == 0
    assert (s.status != ref.RUNNING).all()
    assert ((s.status == ref.TRUNCATED) == (s.ply == 200)).all()
