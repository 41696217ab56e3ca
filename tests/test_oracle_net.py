"""Pins of the float64 network oracle (oracle/net_ref.py) against things
that do not come from it: PyTorch's float64 convolution and its autograd,
PyTorch's bfloat16 conversion, central finite differences of the oracle's
own loss, the Hex transpose-with-colour-swap symmetry, closed forms of the
heads and of Adam's first step."""
import numpy as np
import pytest
import torch

from oracle import net_ref as R
from oracle import ref


def _params(seed, scale=1.0):
    from paper_2506_22609_amd.workloads import init_net_params
    return init_net_params(seed).astype(np.float64) * scale


def _hex_states(N, n, seed, plies=None):
    g = ref.Game(ref.HEX, N, N)
    rng = np.random.default_rng(seed)
    from tests.oracle_util import random_states
    return g, random_states(g, n, plies if plies is not None else N * N // 2, rng)


def test_param_count():
    assert R.n_params() == 64 * 27 + 64 + 3 * (64 * 576 + 64) + 64 + 1 + 64 + 1 == 112706


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        # exact ties between two bfloat16 neighbours
                        (np.arange(-500, 500) * 2 + 1).astype(np.float64) * 2.0 ** -8 + 1.0,
                        [0.0, -0.0, 1.0, -3.5]])
    x32 = x.astype(np.float32)
    exp = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(R.round_bf16(x32), exp)


def test_conv3x3_matches_torch_conv2d():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 5, 7, 7))
    w = rng.standard_normal((4, 5, 3, 3))
    b = rng.standard_normal(4)
    exp = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                     padding=1).numpy()
    assert np.allclose(R.conv3x3(x, w, b), exp, rtol=1e-12, atol=1e-12)


def test_conv3x3_backward_matches_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 6, 6))
    w = rng.standard_normal((5, 3, 3, 3))
    dz = rng.standard_normal((2, 5, 6, 6))
    tx = torch.from_numpy(x).requires_grad_()
    tw = torch.from_numpy(w).requires_grad_()
    tb = torch.zeros(5, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.conv2d(tx, tw, tb, padding=1).backward(torch.from_numpy(dz))
    dx, dw, db = R.conv3x3_backward(x, w, dz)
    assert np.allclose(dx, tx.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(dw, tw.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(db, tb.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_encode_hand_example():
    # 3x3 board: P1 at 0 and 4, P2 at 1; player 2 to move -> transposed, colours exchanged
    board = np.array([[1, 2, 0, 0, 1, 0, 0, 0, 0]], np.int8)
    x1 = R.encode(board, np.array([1]), 3)
    assert x1[0, 0].ravel().tolist() == [1, 0, 0, 0, 1, 0, 0, 0, 0]
    assert x1[0, 1].ravel().tolist() == [0, 1, 0, 0, 0, 0, 0, 0, 0]
    assert x1[0, 2].ravel().tolist() == [0, 0, 1, 1, 0, 1, 1, 1, 1]
    x2 = R.encode(board, np.array([2]), 3)
    assert x2[0, 0].ravel().tolist() == [0, 0, 0, 1, 0, 0, 0, 0, 0]  # P2's stone at (0,1) -> (1,0)
    assert x2[0, 1].ravel().tolist() == [1, 0, 0, 0, 1, 0, 0, 0, 0]
    assert R.frame_index(np.array([1, 5]), np.array([2, 2]), 3).tolist() == [3, 7]


def _transpose_swap(board, to_move, N):
    """Hex symmetry: transpose the board, exchange colours and the mover."""
    b = board.reshape(-1, N, N).transpose(0, 2, 1).reshape(-1, N * N)
    sw = np.where(b == 1, 2, np.where(b == 2, 1, 0)).astype(np.int8)
    return sw, (3 - to_move).astype(np.int8)


@pytest.mark.parametrize("N", [5, 11])
def test_encode_and_network_respect_hex_symmetry(N):
    """The planes of a position and of its transposed, colour-exchanged
    twin (mover exchanged too) are identical, so the network's value is
    equal and its action-order logits are transposed."""
    g, s = _hex_states(N, 40, 3)
    tb, tm = _transpose_swap(s.board, s.to_move.astype(np.int64), N)
    assert np.array_equal(R.encode(s.board, s.to_move, N), R.encode(tb, tm, N))
    p = _params(4)
    f1 = R.forward(p, s.board, s.to_move, N, bf16=False)
    f2 = R.forward(p, tb, tm, N, bf16=False)
    assert np.allclose(f1["value"], f2["value"], rtol=0, atol=1e-12)
    l2 = f2["logits"].reshape(-1, N, N).transpose(0, 2, 1).reshape(-1, N * N)
    assert np.allclose(f1["logits"], l2, rtol=0, atol=1e-12)


def test_heads_closed_form():
    """Zero conv weights: Y_4 = relu(b4) everywhere, so every logit is
    sum_c wp relu(b4) + bp and v = tanh(sum_c wv relu(b4) + bv)."""
    P = R.unpack(_params(5))
    for l in range(1, 5):
        P[f"W{l}"] = P[f"W{l}"] * 0.0
    flat = R.pack(P)
    board = np.zeros((2, 25), np.int8)
    f = R.forward(flat, board, np.array([1, 2]), 5, bf16=False)
    y = np.maximum(P["b4"], 0)
    assert np.allclose(f["logits"], y @ P["wp"] + P["bp"][0], atol=1e-12)
    assert np.allclose(f["value"], np.tanh(y @ P["wv"] + P["bv"][0]), atol=1e-12)


def test_masked_softmax_properties():
    rng = np.random.default_rng(6)
    lg = rng.standard_normal((10, 9)) * 5
    legal = rng.random((10, 9)) < 0.5
    legal[:, 0] = True
    p = R.masked_softmax(lg, legal)
    assert np.allclose(p.sum(1), 1.0) and (p[~legal] == 0).all() and (p[legal] > 0).all()


def _batch(N, n, seed):
    g, s = _hex_states(N, n, seed)
    rng = np.random.default_rng(seed + 100)
    act = np.array([rng.choice(np.flatnonzero(s.board[i] == 0)) for i in range(n)])
    z = rng.choice([-1.0, 1.0], size=n)
    return s.board, s.to_move, act, z


def test_backward_matches_finite_differences():
    """The oracle's gradient against central differences of its own
    float64 loss (advantages held at their value at the base point), along
    random directions: a dropped term, a wrong sign or a transposed operand
    anywhere in the backward shows up here."""
    N = 5
    board, tm, act, z = _batch(N, 6, 7)
    p = _params(8)
    f0 = R.forward(p, board, tm, N, bf16=False)
    adv = np.maximum(z - f0["value"], 0.0)

    def loss(q):
        f = R.forward(q, board, tm, N, bf16=False)
        pi = R.masked_softmax(f["logits_frame"], f["legal_frame"])
        a = R.frame_index(act, tm, N)
        return np.mean((f["value"] - z) ** 2) + np.mean(adv * -np.log(pi[np.arange(len(z)), a]))

    _, g = R.loss_and_grads(p, board, tm, act, z, N, bf16=False)
    rng = np.random.default_rng(9)
    for _ in range(6):
        d = rng.standard_normal(p.shape)
        h = 1e-7  # small enough that no pre-activation crosses the ReLU kink
        fd = (loss(p + h * d) - loss(p - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ d)
    # and per block of parameters (each layer's weights and biases, each head)
    o = 0
    for name, shape in R.param_shapes():
        k = int(np.prod(shape))
        d = np.zeros_like(p)
        d[o:o + k] = rng.standard_normal(k)
        fd = (loss(p + 1e-7 * d) - loss(p - 1e-7 * d)) / 2e-7
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd)), name
        o += k


def test_backward_matches_torch_autograd_with_bf16_rounding_points():
    """bf16 mode: the same network built from PyTorch float64 ops with the
    rounding applied at the same points as straight-through constants; its
    autograd gradient equals the oracle's."""
    N = 5
    board, tm, act, z = _batch(N, 5, 11)
    p = _params(12)
    (lv, lp), g = R.loss_and_grads(p, board, tm, act, z, N, bf16=True)
    P = {k: torch.from_numpy(v.copy()).requires_grad_() for k, v in R.unpack(p).items()}
    x = torch.from_numpy(R.encode(board, tm, N))

    def rb(t):  # forward value rounded, gradient passed straight through
        return t + (torch.from_numpy(R.round_bf16(t.detach().numpy())) - t).detach()

    class RoundGrad(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, gout):
            return torch.from_numpy(R.round_bf16(gout.numpy()))

    y = x
    for l in range(1, 5):
        zl = torch.nn.functional.conv2d(y, rb(P[f"W{l}"]), P[f"b{l}"], padding=1)
        y = RoundGrad.apply(rb(torch.relu(zl)))
    n = len(z)
    lf = torch.einsum("nchw,c->nhw", y, P["wp"]).reshape(n, N * N) + P["bp"][0]
    v = torch.tanh(y.mean(dim=(2, 3)) @ P["wv"] + P["bv"][0])
    legal = torch.from_numpy(x[:, 2].reshape(n, N * N).numpy() > 0)
    logp = torch.log_softmax(lf.masked_fill(~legal, -np.inf), dim=1)
    a = torch.from_numpy(R.frame_index(act, tm, N))
    zt = torch.from_numpy(z)
    adv = torch.clamp(zt - v, min=0.0).detach()
    L = torch.mean((v - zt) ** 2) + torch.mean(adv * -logp[torch.arange(n), a])
    L.backward()
    tg = np.concatenate([P[name].grad.numpy().ravel() for name, _ in R.param_shapes()])
    assert abs(L.item() - (lv + lp)) < 1e-12
    assert np.allclose(g, tg, rtol=1e-9, atol=1e-12)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(13)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    q, m, v = R.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # |g| / (|g| + eps) differs from 1 by at most eps / |g|
    assert (np.abs(q - (p - 1e-3 * np.sign(g))) <= 1e-3 * 1e-8 / np.abs(g) + 1e-15).all()
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def _grads_with_sum_dtype(dtype, p, board, tm, act, z, N):
    """The oracle's gradient with every convolution sum taken in `dtype`
    (the rounding points unchanged)."""
    orig_conv, orig_back = R.conv3x3, R.conv3x3_backward

    def conv(x, w, bias=None):
        return orig_conv(x.astype(dtype), w.astype(dtype), None if bias is None else bias.astype(dtype))

    def back(x, w, dz):
        return tuple(t.astype(dtype) for t in orig_back(x.astype(dtype), w.astype(dtype), dz.astype(dtype)))

    R.conv3x3, R.conv3x3_backward = conv, back
    try:
        return R.loss_and_grads(p, board, tm, act, z, N, beta=0.7, bf16=True)[1]
    finally:
        R.conv3x3, R.conv3x3_backward = orig_conv, orig_back


def test_float32_sums_move_the_gradient_by_less_than_the_gpu_tolerance():
    """The GPU sums in float32; with the same bfloat16 rounding points a sum
    that lands on the other side of a rounding boundary (or of the ReLU's
    zero) flips a value, and the backward pass carries such flips on.  The
    oracle's own arithmetic with float32 sums shows how large that is on 67
    Hex 11x11 positions: every parameter block stays within 1.1e-3 relative
    L2 of the float64 sums, below the 2e-3 the GPU gradient parity test
    allows on its small batches."""
    from tests.oracle_util import random_states
    N = 11
    g = ref.Game(ref.HEX, N, N)
    s = random_states(g, 67, N * N // 2, np.random.default_rng(3 + N))
    s = s.subset(np.flatnonzero(s.status == ref.RUNNING))
    rng = np.random.default_rng(4)
    act = np.array([rng.choice(np.flatnonzero(s.board[i] == 0)) for i in range(s.n)], np.int64)
    z = rng.choice([-1.0, 0.0, 1.0], size=s.n)
    p = _params(5)
    g64 = _grads_with_sum_dtype(np.float64, p, s.board, s.to_move, act, z, N)
    g32 = _grads_with_sum_dtype(np.float32, p, s.board, s.to_move, act, z, N)
    o = 0
    for name, shape in R.param_shapes():
        k = int(np.prod(shape))
        if name != "bp":
            e = np.linalg.norm(g32[o:o + k] - g64[o:o + k]) / np.linalg.norm(g64[o:o + k])
            assert e < 1.1e-3, (name, e)
        o += k


def test_adam_several_steps_match_torch_optim_adam():
    """Five Adam steps of the oracle (bias correction at every step, not
    only the first) against torch.optim.Adam in float64 on the same
    gradients: the two implementations put eps after the bias-corrected
    square root alike, so they agree to float64 rounding."""
    rng = np.random.default_rng(21)
    p0 = rng.standard_normal(300)
    grads = [rng.standard_normal(300) * 10.0 ** rng.integers(-4, 1) for _ in range(5)]
    t = torch.from_numpy(p0.copy()).requires_grad_()
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    q, m, v = p0.copy(), np.zeros(300), np.zeros(300)
    for k, g in enumerate(grads):
        t.grad = torch.from_numpy(g.copy())
        opt.step()
        q, m, v = R.adam(q, g, m, v, k + 1, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8)
        assert np.allclose(q, t.detach().numpy(), rtol=0, atol=1e-15), k
    st = opt.state[t]
    assert np.allclose(m, st["exp_avg"].numpy(), rtol=1e-14, atol=0)
    assert np.allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-14, atol=0)


def test_policy_action_boundaries():
    """Hand cases of the draw rule: a single legal action is always played;
    two equal logits split the unit interval at one half, u = 1/2 itself
    going to the second action (the first running sum must EXCEED u times
    the total); illegal actions are never played."""
    lg = np.array([0.3, 9.0, 0.3, -2.0], np.float32)
    legal = np.array([True, False, True, False])
    for w in (0, 1 << 31, 0xFFFFFFFF):
        assert R.policy_action(lg, np.array([False, False, True, False]), w)[0] == 2
    half = (1 << 23) << 8  # u = 2^23 / 2^24
    assert R.policy_action(lg, legal, half - 256)[0] == 0
    assert R.policy_action(lg, legal, half)[0] == 2
    assert R.policy_action(lg, legal, 0)[0] == 0
    assert R.policy_action(lg, legal, 0xFFFFFFFF)[0] == 2


def test_policy_action_draws_follow_masked_softmax():
    """The law of the policy draw over Philox words (the oracle's generator,
    pinned by the known-answer vectors) is the masked softmax of the
    logits: a chi-square test of 60000 draws over the legal actions of a
    row with logits spread over several units (1 % level)."""
    from scipy.stats import chisquare

    rng = np.random.default_rng(22)
    A = 12
    lg = (rng.standard_normal(A) * 1.5).astype(np.float32)
    legal = rng.random(A) < 0.7
    legal[[1, 7]] = True
    p = R.masked_softmax(lg[None].astype(np.float64), legal[None])[0]
    draws = 60000
    counts = np.zeros(A, np.int64)
    for j in range(draws // 4):
        for w in ref.philox([j, 0, 0, 0], [5, 0]):
            counts[R.policy_action(lg, legal, int(w))[0]] += 1
    assert counts[~legal].sum() == 0
    idx = np.flatnonzero(legal)
    assert chisquare(counts[idx], p[idx] * draws).pvalue > 0.01
