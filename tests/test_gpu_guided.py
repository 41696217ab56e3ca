"""The fused network-guided step (ludax_net_guided_step: the forward pass,
then the policy draw and the ply, with the logits kept on chip) against
(1) the same composition through memory on the GPU -- ludax_net_forward
then ludax_policy_step -- which must agree bit for bit, and (2) the
oracle's composition: the float64 network with the same bfloat16 rounding
points (oracle/net_ref.py), its policy draw and the rules oracle's step."""
import numpy as np
import pytest
import torch

from oracle import net_ref as R
from oracle import ref
from paper_2506_22609_amd.workloads import init_net_params
from tests.gpu_util import FIELDS, assert_same_state, from_device, pair, random_states, to_device

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("kind", [ref.HEX, ref.GOMOKU], ids=["hex11", "gomoku11"])
def test_guided_step_equals_forward_then_policy_step(kind):
    """Mid-game states (whole ended blocks, ILLEGAL envs, a ragged tail of a
    4-board block), explicit 64-bit game ids; every field, reward and
    terminal flag equal after every ply until every game has ended."""
    og, dg = pair(kind, 11, 11)
    rng = np.random.default_rng(60 + kind)
    n = 1031
    s = random_states(og, n, 40, rng)
    s.status[:256] = ref.ILLEGAL
    s.status[300::17] = ref.ILLEGAL
    a = to_device(dg, s)
    b = ludax.State.from_tensors(dg, **{f: getattr(a, f).clone() for f in FIELDS})
    gid = torch.from_numpy(rng.integers(0, 2**62, size=n, dtype=np.int64)).cuda()
    net = ludax.Net(11, 11, params=torch.from_numpy(init_net_params(21)).cuda())
    seed = 0xABCDEF0123
    for p in range(og.cells + 2):
        ra, ta = net.guided_step(dg, a, seed, game_id=gid)
        logits, _ = net.forward(b.board, b.to_move)
        rb, tb = ludax.policy_step(dg, b, logits, seed, game_id=gid)
        assert torch.equal(ra, rb) and torch.equal(ta, tb), f"reward / terminal at ply {p}"
        for f in FIELDS:
            assert torch.equal(getattr(a, f), getattr(b, f)), f"{f} at ply {p}"
        if bool(ta.all()):
            break
    assert bool(ta.all())


def test_guided_step_matches_oracle_composition():
    """Eight guided plies from Hex 11x11 mid-game states against the
    oracle: net_ref.forward's logits, net_ref.policy_action with the ply's
    Philox word, the rules oracle's step.  The GPU's logits differ from the
    float64 network's by float32 rounding (and the bfloat16 flips it moves),
    so a draw whose threshold lies within 2 (exp(d) - 1) of a running sum
    (relative to the total, d = that board's largest logit difference) may
    pick the neighbouring legal action; every other draw, and every rule
    outcome, must be exact."""
    og, dg = pair(ref.HEX, 11, 11)
    rng = np.random.default_rng(71)
    n = 160
    s = random_states(og, n, 30, rng)
    d = to_device(dg, s)
    gid = rng.integers(0, 2**62, size=n, dtype=np.int64)
    dgid = torch.from_numpy(gid).cuda()
    p64 = init_net_params(22).astype(np.float64)
    net = ludax.Net(11, 11, params=torch.from_numpy(init_net_params(22)).cuda())
    seed = 99
    near_calls = 0
    for ply in range(8):
        glog, _ = net.forward(d.board, d.to_move)
        glog = glog.cpu().numpy()
        f = R.forward(p64, s.board, s.to_move, 11, bf16=True)
        m = ref.legal_mask(og, s)
        a = np.zeros(n, np.int32)
        tol = np.zeros(n)
        for i in np.flatnonzero(s.status == ref.RUNNING):
            legal = m[i].astype(bool)
            w = ref.draw(seed, int(gid[i]), int(s.ply[i]))
            a[i], margin = R.policy_action(f["logits"][i], legal, w)
            dmax = float(np.abs(glog[i][legal] - f["logits"][i][legal]).max())
            tol[i] = margin if margin < 2.0 * np.expm1(dmax) + 1e-6 else -1.0
        s_before = s.copy()
        rew, term, _ = ref.step(og, s, a, want_mask=False)
        grew, gterm = net.guided_step(dg, d, seed, game_id=dgid)
        got = from_device(d)
        for i in np.flatnonzero((tol >= 0) & (got.last_action != s.last_action)):
            near_calls += 1
            legal = np.flatnonzero(m[i])
            k = np.searchsorted(legal, s.last_action[i])
            assert got.last_action[i] in legal[max(0, k - 1):k + 2], (ply, i)
            one = s_before.subset([i])
            r1, t1, _ = ref.step(og, one, np.array([got.last_action[i]], np.int32), want_mask=False)
            for fld in ref.State.FIELDS:
                getattr(s, fld)[i] = getattr(one, fld)[0]
            rew[i], term[i] = r1[0], t1[0]
        assert np.array_equal(rew, grew.cpu().numpy()), f"reward at ply {ply}"
        assert np.array_equal(term, gterm.cpu().numpy()), f"terminal at ply {ply}"
        assert_same_state(s, got, f"guided ply {ply}")
    assert near_calls <= n * 8 // 50


def test_guided_step_rejects_unsupported():
    net = ludax.Net(11, 11)
    g = ludax.Game(ref.REVERSI, 8, 8)
    s = ludax.State(g, 4)
    ludax.init(g, s)
    with pytest.raises(ludax.LudaxError):
        net.guided_step(g, s, 1)
    net19 = ludax.Net(19, 19)
    g19 = ludax.Game(ref.HEX, 19, 19)
    s19 = ludax.State(g19, 4)
    ludax.init(g19, s19)
    with pytest.raises(ludax.LudaxError):
        net19.guided_step(g19, s19, 1)


@pytest.mark.parametrize("kind,plies", [(ref.HEX, 20), (ref.GOMOKU, 7), (ref.HEX, 0)],
                         ids=["hex11-20", "gomoku11-7", "hex11-0"])
def test_guided_playout_equals_steps_then_estimate(kind, plies):
    """ludax_net_guided_playout (one kernel: every ply's forward pass, draw
    and step on chip, then the value cutoff) against `plies` calls of
    ludax_net_forward + ludax_policy_step and then ludax_net_estimate:
    identical states and estimates bit for bit, with ended and ILLEGAL envs,
    a ragged last 4-board group and explicit game ids."""
    og, dg = pair(kind, 11, 11)
    rng = np.random.default_rng(90 + kind + plies)
    n = 2051
    s = random_states(og, n, 60, rng)
    s.status[:300:7] = ref.ILLEGAL
    a = to_device(dg, s)
    b = ludax.State.from_tensors(dg, **{f: getattr(a, f).clone() for f in FIELDS})
    gid = torch.from_numpy(rng.integers(0, 2**62, size=n, dtype=np.int64)).cuda()
    net = ludax.Net(11, 11, params=torch.from_numpy(init_net_params(23)).cuda())
    seed = 0x5EED
    est_a = net.guided_playout(dg, a, plies, seed, game_id=gid)
    for _ in range(plies):
        logits, _ = net.forward(b.board, b.to_move)
        ludax.policy_step(dg, b, logits, seed, game_id=gid)
    est_b = net.estimate(b)
    for f in FIELDS:
        assert torch.equal(getattr(a, f), getattr(b, f)), f
    assert torch.equal(est_a, est_b)
    st = a.status.cpu().numpy()
    assert (st == ref.TERMINAL).any() or plies < 10


def test_guided_playout_value_matches_oracle():
    """With no plies the guided playout is the value cutoff of the given
    positions: against the float64 oracle network (relative L2 1e-3) on
    running envs, the exact outcome on ended ones."""
    og, dg = pair(ref.HEX, 11, 11)
    rng = np.random.default_rng(95)
    n = 203
    s = random_states(og, n, 80, rng)
    d = to_device(dg, s)
    p = init_net_params(24)
    net = ludax.Net(11, 11, params=torch.from_numpy(p).cuda())
    est = net.guided_playout(dg, d, 0, 1).cpu().numpy()
    v = R.forward(p.astype(np.float64), s.board, s.to_move, 11)["value"]
    exp = np.where(s.status == ref.TERMINAL, np.where(s.winner == 1, 1.0, np.where(s.winner == 2, -1.0, 0.0)),
                   np.where(s.status == ref.RUNNING, np.where(s.to_move == 1, v, -v), 0.0))
    run = s.status == ref.RUNNING
    assert np.array_equal(est[~run], exp[~run])
    err = np.linalg.norm(est[run] - exp[run]) / np.linalg.norm(exp[run])
    assert err < 1e-3, err


@pytest.mark.parametrize("kind", [ref.HEX, ref.GOMOKU], ids=["hex19", "gomoku19"])
def test_guided_budgeted_19x19(kind):
    """19x19 network-guided playouts (forward + policy step per ply, then the
    value cutoff) admitted in chunks under an HBM budget: the same states
    and estimates bit for bit whatever the chunk size (a budget of 3
    workgroups' workspace against one chunk for all 300 envs), and, on a
    sample, the oracle's composition (float64 network, its policy draw, the
    rules' step), exact except at draws within the logits' float32 error of
    a boundary (then a neighbouring legal action)."""
    from paper_2506_22609_amd import learn
    og, dg = pair(kind, 19, 19)
    rng = np.random.default_rng(120 + kind)
    n, plies, seed, base = 300, 3, 77, 5000
    s = random_states(og, n, 150, rng)
    p = init_net_params(25)
    net = ludax.Net(19, 19, params=torch.from_numpy(p).cuda())
    small = learn.ludax_ws_plus_logits(net, 3 * 64, og.cells) + 1000
    a = to_device(dg, s)
    b = ludax.State.from_tensors(dg, **{f: getattr(a, f).clone() for f in FIELDS})
    ea = learn.guided_budgeted(dg, net, a, plies, small, seed, base)
    eb = learn.guided_budgeted(dg, net, b, plies, 1 << 40, seed, base)
    for f in FIELDS:
        assert torch.equal(getattr(a, f), getattr(b, f)), f
    assert torch.equal(ea, eb)
    # the oracle's composition, ply by ply, on the first 12 and the last 12 envs
    p64 = p.astype(np.float64)
    near_calls = 0
    for lo in (0, n - 12):
        idx = np.arange(lo, lo + 12)
        so = s.subset(idx)
        c = to_device(dg, so)
        for ply in range(plies):
            glog, _ = net.forward(c.board, c.to_move)
            glog = glog.cpu().numpy()
            f = R.forward(p64, so.board, so.to_move, 19, bf16=True)
            m = ref.legal_mask(og, so)
            act = np.zeros(len(idx), np.int32)
            tol = np.full(len(idx), -1.0)
            for i in np.flatnonzero(so.status == ref.RUNNING):
                legal = m[i].astype(bool)
                act[i], margin = R.policy_action(f["logits"][i], legal, ref.draw(seed, base + lo + i, int(so.ply[i])))
                dmax = float(np.abs(glog[i][legal] - f["logits"][i][legal]).max())
                if margin < 2.0 * np.expm1(dmax) + 1e-6:
                    tol[i] = margin
            before = so.copy()
            ref.step(og, so, act, want_mask=False)
            est = learn.guided_budgeted(dg, net, c, 1, small, seed, base + lo)
            got = from_device(c)
            for i in np.flatnonzero((tol >= 0) & (got.last_action != so.last_action)):
                near_calls += 1
                legal = np.flatnonzero(m[i])
                k = np.searchsorted(legal, so.last_action[i])
                assert got.last_action[i] in legal[max(0, k - 1):k + 2]
                one = before.subset([i])
                ref.step(og, one, np.array([got.last_action[i]], np.int32), want_mask=False)
                for fld in ref.State.FIELDS:
                    getattr(so, fld)[i] = getattr(one, fld)[0]
            assert_same_state(so, got, f"guided 19x19 ply {ply}")
        v = R.forward(p64, so.board, so.to_move, 19)["value"]
        exp = np.where(so.status == ref.TERMINAL, np.where(so.winner == 1, 1.0, np.where(so.winner == 2, -1.0, 0.0)),
                       np.where(so.status == ref.RUNNING, np.where(so.to_move == 1, v, -v), 0.0))
        close_rel = np.linalg.norm(est.cpu().numpy() - exp) / max(np.linalg.norm(exp), 1e-30)
        assert close_rel < 1e-3, close_rel
    assert near_calls <= 2
