"""Helpers for the GPU parity tests: move states between the oracle
(numpy, host) and the GPU library (torch, device), and compare them."""
import numpy as np
import torch

from oracle import ref
from paper_2506_22609_amd import ludax

FIELDS = ("board", "to_move", "status", "winner", "passes", "ply", "last_action")


def pair(kind, rows, cols, max_plies=0):
    return ref.Game(kind, rows, cols, max_plies), ludax.Game(kind, rows, cols, max_plies)


def to_device(game, s: "ref.State") -> "ludax.State":
    t = {f: torch.from_numpy(np.ascontiguousarray(getattr(s, f))).cuda() for f in FIELDS}
    return ludax.State.from_tensors(game, **t)


def from_device(d: "ludax.State") -> "ref.State":
    s = ref.State(d.n, d.cells)
    for f in FIELDS:
        setattr(s, f, np.ascontiguousarray(getattr(d, f).cpu().numpy()))
    return s


def assert_same_state(a: "ref.State", b: "ref.State", where=""):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        if not np.array_equal(x, y):
            bad = np.argwhere(x != y)
            i = bad[0][0]
            raise AssertionError(f"{where}: field {f} differs at env {i} "
                                 f"(oracle {x[i]}, gpu {y[i]}); {len(bad)} mismatches")


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
        for f in FIELDS:
            getattr(s, f)[sub] = getattr(ss, f)
    return s
