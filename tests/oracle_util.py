"""Small helpers the oracle tests share: single-env stepping and seeded
action choices.  No rule logic lives here; every rule question goes to the
oracle."""
import numpy as np

from oracle import ref


def single(game, state, i=0):
    return state.subset([i])


def apply_seq(game, actions, state=None):
    """Play a list of actions from the start position (or `state`) on one env.
    Returns the state and the per-ply (reward, terminal)."""
    s = ref.init(game, 1) if state is None else state.copy()
    trace = []
    for a in actions:
        rew, term, _ = ref.step(game, s, [a], want_mask=False)
        trace.append((tuple(rew[0]), int(term[0])))
    return s, trace


def random_legal_actions(mask, rng):
    """One uniformly chosen legal action per row (rows without any legal
    action get 0)."""
    out = np.zeros(mask.shape[0], np.int32)
    for i, row in enumerate(mask):
        idx = np.flatnonzero(row)
        if idx.size:
            out[i] = idx[rng.integers(0, idx.size)]
    return out


def board2d(game, s, i=0):
    return s.board[i].reshape(game.rows, game.cols)


def random_states(game, n, plies, rng, illegal_every=0):
    """Reachable states: the oracle's start position plus up to `plies`
    uniformly chosen legal plies per env (a different count per env)."""
    s = ref.init(game, n)
    target = rng.integers(0, plies + 1, size=n)
    for p in range(plies):
        m = ref.legal_mask(game, s)
        a = np.zeros(n, np.int32)
        for i in range(n):
            idx = np.flatnonzero(m[i])
            if idx.size:
                a[i] = idx[rng.integers(0, idx.size)]
        live = (target > p) & (s.status == ref.RUNNING)
        if not live.any():
            break
        sub = np.flatnonzero(live)
        ss = s.subset(sub)
        ref.step(game, ss, a[sub], want_mask=False)
        for f in ref.State.FIELDS:
            getattr(s, f)[sub] = getattr(ss, f)
    return s
