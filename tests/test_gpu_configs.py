"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration the benchmark times: every env (every game, for the mixed
batches) of every batch is compared with the oracle playing the same game
ids, on the host's cores.  Only the per-ply loop over 1,048,576 Hex 19x19
envs (the state above the Infinity Cache) is checked on a sample plus
whole-batch invariants; the same kernel is compared on every env of the
524288-env loop."""
import os

import numpy as np
import pytest
import torch

from oracle import ref
from paper_2506_22609_amd import workloads as W
from tests.gpu_util import assert_same_state, from_device, pair

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")

THREADS = max(1, min(16, os.cpu_count() or 1))


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


def _oracle_batch(b, seed, base):
    og, _ = pair(b.kind, b.rows, b.cols)
    s = ref.init(og, b.n)
    rew, term, stats = ref.playout(og, s, seed, base, threads=THREADS)
    return og, s, rew, stats


def _check_whole_batch(b, og, g, gstats):
    """Counter invariants: every game ended; only the unbounded Draughts and
    Dai Hasami Shogi are ever cut at max_plies."""
    cut = g.status == ref.TRUNCATED
    assert ((g.status == ref.TERMINAL) | cut).all()
    assert (g.ply[cut] == og.info()[2]).all() and (b.kind in (ref.DRAUGHTS, ref.HASAMI_SHOGI) or not cut.any())
    assert gstats[0] == g.ply.astype(np.int64).sum()
    assert gstats[1] == ((g.status == ref.TERMINAL) & (g.winner == 1)).sum()
    assert gstats[2] == ((g.status == ref.TERMINAL) & (g.winner == 2)).sum()
    assert gstats[1] + gstats[2] + gstats[3] == b.n - int(cut.sum())
    if b.kind == ref.HEX:
        assert gstats[3] == 0


@pytest.mark.parametrize("seed", W.SEEDS)
def test_tictactoe_1024_every_env(seed):
    b = W.TTT_1024
    og, s, rew, stats = _oracle_batch(b, seed, 0)
    g, grew, gstats = _gpu_batch(b, seed, 0)
    assert_same_state(s, g)
    assert np.array_equal(rew, grew) and np.array_equal(stats, gstats)


@pytest.mark.parametrize("b", [W.C4_65536, W.HEX11_65536, W.REVERSI_65536, W.GOMOKU15_65536],
                         ids=lambda b: b.name)
def test_65536_every_env(b):
    """The headline batches (Connect Four, Hex 11x11) and the other members
    of the mixed batch at 65536 envs."""
    seed, base = 2, W.game_id_base(5, b)
    print(f"configs: {b.name} seed {seed} base {base}", flush=True)
    g, grew, gstats = _gpu_batch(b, seed, base)
    og, s, rew, stats = _oracle_batch(b, seed, base)
    assert_same_state(s, g)
    assert np.array_equal(rew, grew) and np.array_equal(stats, gstats)
    _check_whole_batch(b, og, g, gstats)


@pytest.mark.parametrize("b", list(W.LARGE_BATCHES) + list(W.MORE_GAMES), ids=lambda b: b.name)
def test_large_and_more_games_every_env(b):
    """The 19x19 batches of 524288 envs, and the Yavalath, Pente, Wolf and
    Sheep, Draughts and Dai Hasami Shogi batches of 65536 envs."""
    seed, base = 3, W.game_id_base(2, b)
    print(f"configs: {b.name} seed {seed} base {base}", flush=True)
    g, grew, gstats = _gpu_batch(b, seed, base)
    og, s, rew, stats = _oracle_batch(b, seed, base)
    assert_same_state(s, g)
    assert np.array_equal(rew, grew) and np.array_equal(stats, gstats)
    _check_whole_batch(b, og, g, gstats)


_ORACLE = {}


def _oracle_batch_cached(b, seed, base):
    key = (b.name, seed, base)
    if key not in _ORACLE:
        _ORACLE.clear()
        _ORACLE[key] = _oracle_batch(b, seed, base)
    return _ORACLE[key]


def _per_ply_loop(b, seed, base, aux=False):
    """ludax_random_step launched max_plies times (the benchmark's per-ply
    loop), with the counters around it; aux: with Hex's component cache."""
    _, dg = pair(b.kind, b.rows, b.cols)
    d = ludax.State(dg, b.n, aux=aux)
    ludax.init(dg, d)
    st = torch.zeros(4, dtype=torch.int64, device="cuda")
    ludax.state_stats(dg, d, -1, st)
    r = torch.empty((b.n, 2), dtype=torch.int8, device="cuda")
    t = torch.empty(b.n, dtype=torch.uint8, device="cuda")
    for _ in range(dg.max_plies):
        ludax.random_step(dg, d, seed, base, reward=r, terminal=t)
    ludax.state_stats(dg, d, +1, st)
    return from_device(d), st.cpu().numpy()


@pytest.mark.parametrize("aux", [False, True], ids=["flood", "union_find"])
def test_per_ply_loop_at_full_size_every_env(aux):
    """The per-ply loop over the Hex 19x19 batch of 524288 envs, with the
    end test by flood (aux = NULL) and by the component cache, ends every
    game exactly where the oracle's playout of the same game id ends."""
    b = W.HEX19_524288
    seed, base = 4, 7 * b.n
    print(f"configs: per-ply {b.name} aux {aux} seed {seed} base {base}", flush=True)
    g, gstats = _per_ply_loop(b, seed, base, aux)
    og, s, _, stats = _oracle_batch_cached(b, seed, base)
    assert_same_state(s, g)
    assert np.array_equal(stats, gstats)


@pytest.mark.parametrize("aux", [False, True], ids=["flood", "union_find"])
def test_per_ply_loop_above_infinity_cache_sampled(aux):
    """The per-ply loop over 1,048,576 Hex 19x19 envs: a sample of 8192
    envs replayed one by one on the oracle by game id, and the whole-batch
    counter invariants."""
    b = W.HEX19_1M
    seed, base = 5, 3 * b.n
    print(f"configs: per-ply {b.name} aux {aux} seed {seed} base {base}", flush=True)
    g, gstats = _per_ply_loop(b, seed, base, aux)
    og, _ = pair(b.kind, b.rows, b.cols)
    rng = np.random.default_rng(23)
    idx = np.sort(rng.choice(b.n, size=8192, replace=False))
    idx[0], idx[-1] = 0, b.n - 1
    s = ref.init(og, len(idx))
    ref.playout(og, s, seed, 0, game_id=base + idx, threads=THREADS)
    assert_same_state(s, g.subset(idx))
    _check_whole_batch(b, og, g, gstats)


@pytest.mark.parametrize("mb_name", ["MIXED4", "LARGE_MIXED"])
def test_mixed_full_size_every_game(mb_name):
    """The mixed persistent batches at their benchmark sizes: 4 x 262144
    game ids through 262144 slots, and 1048576 Hex / Gomoku 19x19 ids;
    every game's winner, length and last action against the oracle."""
    if mb_name == "MIXED4":
        kinds = [(b.kind, b.rows, b.cols) for b in W.MIXED4.kinds]
        n_games, total = W.MIXED4.n_games, W.MIXED4.slots
    else:
        kinds = [(b.kind, b.rows, b.cols) for b in W.LARGE_BATCHES]
        n_games, total = sum(b.n for b in W.LARGE_BATCHES), 262144
    games = [ludax.Game(k, r, c) for k, r, c in kinds]
    m = ludax.Mixed(games)
    m.slots = [total // len(games) // 64 * 64] * len(games)
    seed, base = 6, 12345
    print(f"configs: {mb_name} seed {seed} base {base} games {n_games}", flush=True)
    out, stats = m.playout(seed, base, n_games)
    torch.cuda.synchronize()
    w, p, l = (x.cpu().numpy() for x in (out.winner, out.plies, out.last_action))
    st = stats.cpu().numpy()
    js = np.arange(n_games, dtype=np.int64)
    for k, (kind, r, c) in enumerate(kinds):
        sel = js[(base + js) % len(kinds) == k]
        og = ref.Game(kind, r, c)
        s = ref.init(og, len(sel))
        _, _, ost = ref.playout(og, s, seed, 0, game_id=base + sel, threads=THREADS)
        assert np.array_equal(w[sel], np.where(s.status == ref.TERMINAL, s.winner, -1)), kind
        assert np.array_equal(p[sel], s.ply) and np.array_equal(l[sel], s.last_action), kind
        assert np.array_equal(st[k], ost), kind
