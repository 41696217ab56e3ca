"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration the benchmark times: every env for the small cases, a
sampled subset (re-run one by one on the oracle by game id) plus
whole-batch invariants for the 65536-env batches."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2506_22609_amd import workloads as W
from tests.gpu_util import assert_same_state, from_device, pair

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu_batch(b, seed, base):
    _, dg = pair(b.kind, b.rows, b.cols)
    d = ludax.State(dg, b.n)
    ludax.init(dg, d)
    rew, term, stats = ludax.playout(dg, d, seed, base)
    return from_device(d), rew.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("seed", W.SEEDS)
def test_tictactoe_1024_every_env(seed):
    b = W.TTT_1024
    og, _ = pair(b.kind, b.rows, b.cols)
    s = ref.init(og, b.n)
    rew, term, stats = ref.playout(og, s, seed, 0)
    g, grew, gstats = _gpu_batch(b, seed, 0)
    assert_same_state(s, g)
    assert np.array_equal(rew, grew) and np.array_equal(stats, gstats)


def test_connect4_65536_every_env():
    b = W.C4_65536
    og, _ = pair(b.kind, b.rows, b.cols)
    base = W.game_id_base(3, b)
    s = ref.init(og, b.n)
    rew, term, stats = ref.playout(og, s, 1, base, threads=16)
    g, grew, gstats = _gpu_batch(b, 1, base)
    assert_same_state(s, g)
    assert np.array_equal(rew, grew) and np.array_equal(stats, gstats)


@pytest.mark.parametrize("b", [W.HEX11_65536, W.REVERSI_65536, W.GOMOKU15_65536],
                         ids=lambda b: b.name)
def test_65536_sampled(b):
    og, _ = pair(b.kind, b.rows, b.cols)
    seed, base = 2, W.game_id_base(5, b)
    g, grew, gstats = _gpu_batch(b, seed, base)
    rng = np.random.default_rng(b.kind)
    idx = np.sort(rng.choice(b.n, size=1536, replace=False))
    idx[0], idx[-1] = 0, b.n - 1
    s = ref.init(og, len(idx))
    rew, term, _ = ref.playout(og, s, seed, 0, game_id=base + idx, threads=16)
    assert_same_state(s, g.subset(idx))
    assert np.array_equal(rew, grew[idx])
    # whole-batch invariants
    assert (g.status == ref.TERMINAL).all()
    assert gstats[0] == g.ply.astype(np.int64).sum()
    assert gstats[1] == (g.winner == 1).sum() and gstats[2] == (g.winner == 2).sum()
    assert gstats[3] == (g.winner == 0).sum()
    assert gstats[1] + gstats[2] + gstats[3] == b.n
    if b.kind == ref.HEX:
        assert gstats[3] == 0
