"""GPU parity: every call of the C ABI (through the Python binding) against
the CPU oracle, byte for byte, on the same seeded inputs.

Sizes span several 64-env workgroups plus a ragged tail; states come from
the start position and from reachable mid-game positions (some already
ended); actions include illegal and out-of-range ones.
"""
import numpy as np
import pytest
import torch

from oracle import ref
from tests.gpu_util import assert_same_state, from_device, pair, random_states, to_device

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")

GAMES = [
    (ref.TICTACTOE, 3, 3),
    (ref.CONNECT_FOUR, 6, 7),
    (ref.HEX, 11, 11),
    (ref.REVERSI, 8, 8),
    (ref.GOMOKU, 15, 15),
    (ref.HEX, 19, 19),
    (ref.GOMOKU, 19, 19),
    (ref.YAVALATH, 9, 9),
    (ref.YAVALATH, 5, 5),
    (ref.PENTE, 19, 19),
    (ref.PENTE, 7, 7),
    (ref.WOLF_SHEEP, 8, 8),
    (ref.DRAUGHTS, 8, 8),
    (ref.HASAMI_SHOGI, 9, 9),
]
IDS = ["ttt", "c4", "hex11", "reversi", "gomoku15", "hex19", "gomoku19", "yavalath9", "yavalath5", "pente19",
       "pente7", "wolf_sheep", "draughts", "hasami_shogi"]
MOVES = GAMES[-3:]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("g", GAMES, ids=IDS)
@pytest.mark.parametrize("n", [1, 63, 64, 65, 517])
def test_init(g, n):
    og, dg = pair(*g)
    d = ludax.State(dg, n)
    ludax.init(dg, d)
    assert_same_state(ref.init(og, n), from_device(d), f"init n={n}")


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_legal_mask(g):
    og, dg = pair(*g)
    rng = np.random.default_rng(100 + g[0] * 31 + g[1])
    n = 333
    s = random_states(og, n, og.cells if g[0] != ref.REVERSI else 70, rng)
    d = to_device(dg, s)
    got = ludax.legal_mask(dg, d).cpu().numpy()
    exp = ref.legal_mask(og, s)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_step_sequences(g):
    """Drive both sides with the same per-ply actions: mostly legal, some
    illegal or out of range; compare everything after every ply."""
    og, dg = pair(*g)
    rng = np.random.default_rng(7 + g[0] * 13 + g[1])
    n = 200
    s = ref.init(og, n)
    d = ludax.State(dg, n)
    ludax.init(dg, d)
    plies = min(og.cells + 6, 140)
    for p in range(plies):
        m = ref.legal_mask(og, s)
        a = np.zeros(n, np.int32)
        for i in range(n):
            r = rng.random()
            idx = np.flatnonzero(m[i])
            if r < 0.01:
                a[i] = -1 - int(rng.integers(0, 5))
            elif r < 0.02:
                a[i] = og.num_actions + int(rng.integers(0, 5))
            elif r < 0.04 or idx.size == 0:
                a[i] = int(rng.integers(0, og.num_actions))
            else:
                a[i] = idx[rng.integers(0, idx.size)]
        rew, term, nm = ref.step(og, s, a)
        grew, gterm, gnm = ludax.step(dg, d, torch.from_numpy(a).cuda())
        assert np.array_equal(rew, grew.cpu().numpy()), f"reward at ply {p}"
        assert np.array_equal(term, gterm.cpu().numpy()), f"terminal at ply {p}"
        assert np.array_equal(nm, gnm.cpu().numpy()), f"next mask at ply {p}"
        assert_same_state(s, from_device(d), f"ply {p}")
        if (s.status != ref.RUNNING).all():
            break


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_step_without_mask(g):
    og, dg = pair(*g)
    rng = np.random.default_rng(3)
    n = 130
    s = random_states(og, n, 10, rng)
    d = to_device(dg, s)
    m = ref.legal_mask(og, s)
    a = np.array([np.flatnonzero(r)[0] if r.any() else 0 for r in m], np.int32)
    rew, term, _ = ref.step(og, s, a, want_mask=False)
    grew, gterm, _ = ludax.step(dg, d, torch.from_numpy(a).cuda(), want_mask=False)
    assert np.array_equal(rew, grew.cpu().numpy()) and np.array_equal(term, gterm.cpu().numpy())
    assert_same_state(s, from_device(d))


@pytest.mark.parametrize("g", GAMES, ids=IDS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_playout_from_start(g, seed):
    og, dg = pair(*g)
    n = 1000 if og.cells <= 121 else 300
    s = ref.init(og, n)
    rew, term, stats = ref.playout(og, s, seed, 5000, threads=8)
    d = ludax.State(dg, n)
    ludax.init(dg, d)
    grew, gterm, gstats = ludax.playout(dg, d, seed, 5000)
    assert_same_state(s, from_device(d), "playout")
    assert np.array_equal(rew, grew.cpu().numpy())
    assert np.array_equal(term, gterm.cpu().numpy())
    assert np.array_equal(stats, gstats.cpu().numpy())


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_playout_from_midgame_with_ids(g):
    """Mid-game states (some ended, some ILLEGAL) and explicit game ids."""
    og, dg = pair(*g)
    rng = np.random.default_rng(11)
    n = 257
    s = random_states(og, n, min(og.cells, 40), rng)
    s.status[::17] = ref.ILLEGAL
    gid = rng.integers(-(2**62), 2**62, size=n, dtype=np.int64)
    d = to_device(dg, s)
    rew, term, stats = ref.playout(og, s, 0xDEADBEEFCAFEF00D, 0, game_id=gid)
    grew, gterm, gstats = ludax.playout(dg, d, 0xDEADBEEFCAFEF00D, 0,
                                        game_id=torch.from_numpy(gid).cuda())
    assert_same_state(s, from_device(d), "playout")
    assert np.array_equal(rew, grew.cpu().numpy())
    assert np.array_equal(term, gterm.cpu().numpy())
    assert np.array_equal(stats, gstats.cpu().numpy())


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_truncation(g):
    og, dg = pair(g[0], g[1], g[2], 7)
    n = 190
    s = ref.init(og, n)
    rew, term, stats = ref.playout(og, s, 9, 0)
    d = ludax.State(dg, n)
    ludax.init(dg, d)
    grew, gterm, gstats = ludax.playout(dg, d, 9, 0)
    assert_same_state(s, from_device(d))
    assert np.array_equal(stats, gstats.cpu().numpy())


@pytest.mark.parametrize("kind,sizes", [(ref.HEX, range(1, 20)), (ref.GOMOKU, range(5, 20)),
                                        (ref.YAVALATH, (3, 5, 7, 9)), (ref.PENTE, (7, 9, 19))],
                         ids=["hex", "gomoku", "yavalath", "pente"])
def test_every_board_size(kind, sizes):
    for N in sizes:
        og, dg = pair(kind, N, N)
        n = 130
        s = ref.init(og, n)
        rew, term, stats = ref.playout(og, s, N, 0, threads=8)
        d = ludax.State(dg, n)
        ludax.init(dg, d)
        grew, gterm, gstats = ludax.playout(dg, d, N, 0)
        assert_same_state(s, from_device(d), f"N={N}")
        assert np.array_equal(stats, gstats.cpu().numpy()), f"N={N}"
        # step parity on a few plies from mid-game
        rng = np.random.default_rng(N)
        s = random_states(og, 70, min(N * N, 30), rng)
        d = to_device(dg, s)
        for _ in range(3):
            m = ref.legal_mask(og, s)
            a = np.array([np.flatnonzero(r)[rng.integers(0, r.sum())] if r.any() else 0 for r in m],
                         np.int32)
            rew, term, nm = ref.step(og, s, a)
            grew, gterm, gnm = ludax.step(dg, d, torch.from_numpy(a).cuda())
            assert np.array_equal(nm, gnm.cpu().numpy()) and np.array_equal(rew, grew.cpu().numpy())
            assert_same_state(s, from_device(d), f"step N={N}")


def test_zero_envs():
    og, dg = pair(ref.HEX, 11, 11)
    d = ludax.State(dg, 0)
    ludax.init(dg, d)
    ludax.legal_mask(dg, d)
    ludax.step(dg, d, torch.zeros(0, dtype=torch.int32, device="cuda"))
    _, _, st = ludax.playout(dg, d, 1, 0)
    assert st.cpu().numpy().tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("g", GAMES[:5], ids=IDS[:5])
def test_state_stats_brackets_equal_playout_stats(g):
    """ludax_state_stats(-1) ... ludax_state_stats(+1) around a playout adds
    what the playout's own stats argument adds."""
    og, dg = pair(*g)
    rng = np.random.default_rng(21)
    s = random_states(og, 300, 12, rng)
    s.status[::9] = ref.ILLEGAL
    d1, d2 = to_device(dg, s), to_device(dg, s)
    _, _, st1 = ludax.playout(dg, d1, 4, 77)
    st2 = torch.full((4,), 5, dtype=torch.int64, device="cuda")
    ludax.state_stats(dg, d2, -1, st2)
    ludax.playout(dg, d2, 4, 77, stats=None)
    ludax.state_stats(dg, d2, +1, st2)
    assert (st2.cpu() - 5).tolist() == st1.cpu().tolist()
    assert_same_state(from_device(d1), from_device(d2))


def _oracle_random_step(og, s, seed, gid):
    """One ply of the oracle's uniform-random policy: the ply's Philox word,
    k = (w * n_legal) >> 32, the k-th legal action, then the oracle's step
    (an env with no legal action gets action -1, i.e. ILLEGAL)."""
    m = ref.legal_mask(og, s)
    a = np.full(s.n, -1, np.int32)
    for i in np.flatnonzero(s.status == ref.RUNNING):
        idx = np.flatnonzero(m[i])
        if idx.size:
            w = ref.draw(seed, int(gid[i]), int(s.ply[i]))
            a[i] = idx[(w * idx.size) >> 32]
    rew, term, _ = ref.step(og, s, a, want_mask=False)
    return rew, term


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_random_step_sequences(g):
    """ludax_random_step ply by ply against the oracle's draw + step, from
    mid-game states (whole blocks of ended envs, ILLEGAL ones, a ragged
    tail) with explicit game ids, until every env has ended."""
    og, dg = pair(*g)
    rng = np.random.default_rng(31 + g[0] * 7 + g[1])
    n = 333
    s = random_states(og, n, min(og.cells, 30), rng)
    s.status[:128] = ref.ILLEGAL  # two workgroups with nothing to play
    s.status[200::13] = ref.ILLEGAL
    gid = rng.integers(0, 2**62, size=n, dtype=np.int64)
    d = to_device(dg, s)
    dgid = torch.from_numpy(gid).cuda()
    seed = 0x1234_5678_9ABC_DEF0 + g[0]
    for p in range(og.info()[2] + 5):
        rew, term = _oracle_random_step(og, s, seed, gid)
        grew, gterm = ludax.random_step(dg, d, seed, game_id=dgid)
        assert np.array_equal(rew, grew.cpu().numpy()), f"reward at ply {p}"
        assert np.array_equal(term, gterm.cpu().numpy()), f"terminal at ply {p}"
        assert_same_state(s, from_device(d), f"random step {p}")
        if (s.status != ref.RUNNING).all():
            break
    assert (s.status != ref.RUNNING).all()


@pytest.mark.parametrize("g", GAMES, ids=IDS)
def test_random_step_loop_equals_playout(g):
    """Repeating ludax_random_step until nothing runs reproduces the
    oracle's whole playout with the same seed and game ids."""
    og, dg = pair(*g)
    n = 517 if og.cells <= 121 else 150
    s = ref.init(og, n)
    _, _, stats = ref.playout(og, s, 5, 1000, threads=8)
    d = ludax.State(dg, n)
    ludax.init(dg, d)
    st = torch.zeros(4, dtype=torch.int64, device="cuda")
    ludax.state_stats(dg, d, -1, st)
    for _ in range(og.info()[2] + 5):
        _, term = ludax.random_step(dg, d, 5, 1000)
        if bool(term.all()):
            break
    ludax.state_stats(dg, d, +1, st)
    assert_same_state(s, from_device(d), "random-step loop")
    assert np.array_equal(stats, st.cpu().numpy())


@pytest.mark.parametrize("g", GAMES[:5], ids=IDS[:5])
def test_step_blocks_without_running_env(g):
    """ludax_step on a batch whose first workgroups hold only ended envs
    (the kernel skips their boards): rewards, terminal flags, the next
    mask and the states still match the oracle."""
    og, dg = pair(*g)
    rng = np.random.default_rng(41)
    n = 300
    s = random_states(og, n, 8, rng)
    s.status[:192] = ref.ILLEGAL
    s.status[256:] = ref.ILLEGAL
    d = to_device(dg, s)
    m = ref.legal_mask(og, s)
    a = np.array([np.flatnonzero(r)[0] if r.any() else 0 for r in m], np.int32)
    rew, term, nm = ref.step(og, s, a)
    grew, gterm, gnm = ludax.step(dg, d, torch.from_numpy(a).cuda())
    assert np.array_equal(rew, grew.cpu().numpy()) and np.array_equal(term, gterm.cpu().numpy())
    assert np.array_equal(nm, gnm.cpu().numpy())
    assert_same_state(s, from_device(d))


@pytest.mark.parametrize("g", [GAMES[2], GAMES[3], GAMES[4], GAMES[7], GAMES[9], GAMES[12], GAMES[13]],
                         ids=["hex11", "reversi", "gomoku15", "yavalath9", "pente19", "draughts", "hasami_shogi"])
def test_policy_step_sequences(g):
    """ludax_policy_step ply by ply against the oracle's draw + step, with
    random logits: every action equals the oracle's, except where the
    oracle's threshold lies within float32 rounding of a running sum (then
    the GPU's action must be one of the two legal actions at that boundary)."""
    from oracle import net_ref as R
    og, dg = pair(*g)
    rng = np.random.default_rng(51 + g[0])
    n = 150
    s = random_states(og, n, min(og.cells, 20), rng)
    s.status[:64] = ref.ILLEGAL
    gid = rng.integers(0, 2**62, size=n, dtype=np.int64)
    d = to_device(dg, s)
    dgid = torch.from_numpy(gid).cuda()
    seed = 77
    close_calls = 0
    P = og.num_actions - (1 if g[0] == ref.REVERSI else 0)  # the actions that are not PASS
    for p in range(og.info()[2] + 5):
        lg = (rng.standard_normal((n, og.num_actions)) * 2.0).astype(np.float32)
        m = ref.legal_mask(og, s)
        a = np.full(n, -1, np.int32)
        near = np.zeros(n, bool)
        for i in np.flatnonzero(s.status == ref.RUNNING):
            legal = m[i, :P].astype(bool)
            if legal.any():
                a[i], margin = R.policy_action(lg[i, :P], legal, ref.draw(seed, int(gid[i]), int(s.ply[i])))
                near[i] = margin < 1e-5
            elif m[i].any():
                a[i] = og.num_actions - 1  # forced pass
        s_before = s.copy()
        rew, term, _ = ref.step(og, s, a, want_mask=False)
        grew, gterm = ludax.policy_step(dg, d, torch.from_numpy(lg).cuda(), seed, game_id=dgid)
        got = from_device(d)
        ga = got.last_action
        for i in np.flatnonzero(near & (ga != s.last_action)):
            # a draw at a boundary: accept the neighbouring legal action, replay it on the oracle
            close_calls += 1
            legal = np.flatnonzero(m[i, :P])
            k = np.searchsorted(legal, s.last_action[i])
            assert ga[i] in legal[max(0, k - 1):k + 2]
            one = s_before.subset([i])
            r1, t1, _ = ref.step(og, one, np.array([ga[i]], np.int32), want_mask=False)
            for f in ref.State.FIELDS:
                getattr(s, f)[i] = getattr(one, f)[0]
            rew[i], term[i] = r1[0], t1[0]
        assert np.array_equal(rew, grew.cpu().numpy()), f"reward at ply {p}"
        assert np.array_equal(term, gterm.cpu().numpy()), f"terminal at ply {p}"
        assert_same_state(s, got, f"policy step {p}")
        if (s.status != ref.RUNNING).all():
            break
    assert close_calls <= 2


@pytest.mark.parametrize("g", MOVES, ids=["wolf_sheep", "draughts", "hasami_shogi"])
def test_moves_deep_positions(g):
    """Movement games from positions deep into the game (Draughts: kings,
    pending extra turns): mask, stepped plies with next masks, then the
    playout to the end."""
    og, dg = pair(*g)
    rng = np.random.default_rng(61)
    n = 300
    s = random_states(og, n, 50 if g[0] == ref.WOLF_SHEEP else 150, rng)
    if g[0] == ref.DRAUGHTS:
        assert (s.board >= 5).any() and ((s.passes > 0) & (s.status == ref.RUNNING)).any()
    d = to_device(dg, s)
    assert np.array_equal(ludax.legal_mask(dg, d).cpu().numpy(), ref.legal_mask(og, s))
    for p in range(40):
        m = ref.legal_mask(og, s)
        a = np.array([np.flatnonzero(r)[rng.integers(0, r.sum())] if r.any() else 0 for r in m], np.int32)
        rew, term, nm = ref.step(og, s, a)
        grew, gterm, gnm = ludax.step(dg, d, torch.from_numpy(a).cuda())
        assert np.array_equal(rew, grew.cpu().numpy()) and np.array_equal(term, gterm.cpu().numpy()), p
        assert np.array_equal(nm, gnm.cpu().numpy()), f"next mask at ply {p}"
        assert_same_state(s, from_device(d), f"ply {p}")
    rew, term, stats = ref.playout(og, s, 3, 70, threads=8)
    grew, gterm, gstats = ludax.playout(dg, d, 3, 70)
    assert_same_state(s, from_device(d), "playout")
    assert np.array_equal(rew, grew.cpu().numpy()) and np.array_equal(stats, gstats.cpu().numpy())
