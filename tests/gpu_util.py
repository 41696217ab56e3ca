"""Helpers for the GPU parity tests: move states between the oracle
(numpy, host) and the GPU library (torch, device), and compare them."""
import numpy as np
import torch

from oracle import ref
from tests.oracle_util import random_states  # noqa: F401 (re-exported)
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
