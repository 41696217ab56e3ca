"""Step and playout semantics of the oracle that hold for every game:
illegal actions, stepping an ended env, truncation, determinism, resume,
thread-count independence, argument errors."""
import numpy as np
import pytest

from oracle import ref
from tests.oracle_util import random_legal_actions

GAMES = [ref.Game(ref.TICTACTOE, 3, 3), ref.Game(ref.CONNECT_FOUR, 6, 7), ref.Game(ref.HEX, 11, 11),
         ref.Game(ref.REVERSI, 8, 8), ref.Game(ref.GOMOKU, 15, 15)]
IDS = ["ttt", "c4", "hex11", "reversi", "gomoku15"]


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_illegal_actions(g):
    rng = np.random.default_rng(1)
    n = 64
    s = ref.init(g, n)
    for _ in range(3):
        ref.step(g, s, random_legal_actions(ref.legal_mask(g, s), rng), want_mask=False)
    m = ref.legal_mask(g, s)
    before = s.copy()
    bad = np.zeros(n, np.int32)
    for i in range(n):
        kind = i % 3
        if kind == 0:
            bad[i] = -1 - i
        elif kind == 1:
            bad[i] = g.num_actions + i
        else:
            ill = np.flatnonzero(m[i] == 0)
            bad[i] = ill[rng.integers(0, ill.size)]
    rew, term, nm = ref.step(g, s, bad)
    assert (s.status == ref.ILLEGAL).all() and term.all() and (rew == 0).all()
    assert (s.board == before.board).all() and (s.ply == before.ply).all()
    assert (s.to_move == before.to_move).all() and (s.last_action == before.last_action).all()
    assert nm.sum() == 0


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_ended_env_is_a_noop(g):
    s = ref.init(g, 32)
    ref.playout(g, s, 9, 0)
    before = s.copy()
    m = ref.legal_mask(g, s)
    assert m.sum() == 0
    rew, term, nm = ref.step(g, s, np.zeros(32, np.int32))
    for f in ref.State.FIELDS:
        assert (getattr(s, f) == getattr(before, f)).all()
    assert term.all() and (rew == 0).all() and nm.sum() == 0
    rew, term, stats = ref.playout(g, s, 9, 0)
    assert (rew == 0).all() and term.all() and (stats == 0).all()


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_truncation_and_resume(g):
    """Stop every game after k plies with max_plies = k, reopen it, and the
    rest of the playout equals the uninterrupted one (the random stream is
    keyed by game and ply, not by call)."""
    n, seed, k = 200, 77, 5
    full = ref.init(g, n)
    r_full, _, st_full = ref.playout(g, full, seed, 1000)
    gk = ref.Game(g.kind, g.rows, g.cols, k)
    part = ref.init(gk, n)
    r_part, t_part, st_part = ref.playout(gk, part, seed, 1000)
    assert t_part.all()
    trunc = part.status == ref.TRUNCATED
    assert (part.ply[trunc] == k).all() and (part.winner[trunc] == -1).all()
    assert (r_part[trunc] == 0).all()
    ended = part.status == ref.TERMINAL
    assert (part.ply[ended] <= k).all()
    # reopen the truncated games and finish them under the natural bound
    part.status[trunc] = ref.RUNNING
    r2, _, st2 = ref.playout(g, part, seed, 1000)
    for f in ref.State.FIELDS:
        assert (getattr(part, f) == getattr(full, f)).all(), f
    assert (r2[trunc] == r_full[trunc]).all()
    assert st_part[0] + st2[0] == st_full[0]


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_determinism_ids_and_threads(g):
    n = 300
    a = ref.init(g, n)
    ra, ta, sa = ref.playout(g, a, 5, 40)
    b = ref.init(g, n)
    rb, tb, sb = ref.playout(g, b, 5, 0, game_id=np.arange(40, 40 + n), threads=8)
    for f in ref.State.FIELDS:
        assert (getattr(a, f) == getattr(b, f)).all()
    assert (ra == rb).all() and (sa == sb).all()
    c = ref.init(g, n)
    ref.playout(g, c, 6, 40)
    assert (c.board != a.board).any()
    # a game depends on its id only, not on its slot
    perm = np.random.default_rng(0).permutation(n)
    d = ref.init(g, n)
    ref.playout(g, d, 5, 0, game_id=40 + perm)
    assert (d.board == a.board[perm]).all() and (d.ply == a.ply[perm]).all()


def test_argument_errors():
    with pytest.raises(ref.OracleError):
        ref.Game(ref.CONNECT_FOUR, 7, 6).info()
    with pytest.raises(ref.OracleError):
        ref.Game(ref.HEX, 20, 20).info()
    with pytest.raises(ref.OracleError):
        ref.Game(ref.GOMOKU, 4, 4).info()
    with pytest.raises(ref.OracleError):
        ref.Game(9, 3, 3).info()
    assert ref.Game(ref.REVERSI, 8, 8).info() == (64, 65, 121)
    assert ref.Game(ref.HEX, 11, 11).info() == (121, 121, 121)
    assert ref.Game(ref.TICTACTOE, 3, 3, 4).info() == (9, 9, 4)
