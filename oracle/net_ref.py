"""Plain float64 reference of the small convolutional policy/value network.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
benchmark's CPU leg, never by the GPU library or its binding.

The paper trains policy/value agents on its environments (Sec. 7, "Trained
Agents"; training batch 4096 and learning rate 0.001 in the appendix of
training hyperparameters) with a ResNet; this project's network is the small
one of its own benchmark configuration, written out here step by step:

  encode   (board, to_move) -> 3 planes in the mover's frame: the mover's
           stones, the opponent's stones, the empty cells.  For player 2 the
           board is transposed and the colours exchanged, which maps player
           2's left-right goal of Hex onto player 1's top-bottom goal (the
           transpose-with-colour-swap symmetry of Hex), so the network always
           sees the mover connecting top to bottom.
  trunk    4 layers Z_l = conv3x3(Y_{l-1}; W_l) + b_l (zero padding 1,
           cross-correlation, W_l[out][in][dr][dc]), Y_l = relu(Z_l),
           64 channels, Y_0 = the planes.
  policy   logit[p] = sum_c wp[c] Y_4[c][p] + bp over the cells of the
           mover's frame; a masked softmax over the empty cells.
  value    v = tanh(sum_c wv[c] mean_p Y_4[c][p] + bv): the expected final
           outcome for the mover (+1 win, -1 loss, 0 draw).

Loss of a batch of n samples (state s_i, action a_i played in s_i, final
outcome z_i for the mover of s_i) with policy weight beta:

  L = (1/n) sum_i [ (v_i - z_i)^2 + beta max(z_i - sg(v_i), 0) (-log pi_i[a_i]) ]

(sg = value held constant): value regression to the outcome, and the
log-likelihood of the move that was played, weighted by how much better
than predicted the mover did (clipped at zero: with negative weights the
objective has no lower bound, since it is minimised by driving the
probability of a losing move to zero), which raises the probability of
moves after which the mover did better than the value predicted.

bf16=True rounds, to bfloat16 (round to nearest, ties to even), exactly the
quantities the GPU kernels keep in bfloat16: the conv weights, each Y_l, and
each pre-activation gradient dZ_l before it multiplies anything; sums are
taken in float64 here (float32 on the GPU).  bf16=False is the plain float64
network (used by the finite-difference pin).

Flat parameter vector (float32 on the device, float64 here), in this order:
W1 [64][3][3][3], b1 [64], W2..W4 [64][64][3][3] with b2..b4 [64],
wp [64], bp [1], wv [64], bv [1].
"""
from __future__ import annotations

import numpy as np

CH = 64
LAYERS = 4


def param_shapes():
    shapes = [("W1", (CH, 3, 3, 3)), ("b1", (CH,))]
    for l in range(2, LAYERS + 1):
        shapes += [(f"W{l}", (CH, CH, 3, 3)), (f"b{l}", (CH,))]
    shapes += [("wp", (CH,)), ("bp", (1,)), ("wv", (CH,)), ("bv", (1,))]
    return shapes


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(flat):
    flat = np.asarray(flat, np.float64)
    assert flat.shape == (n_params(),)
    out, o = {}, 0
    for name, shape in param_shapes():
        k = int(np.prod(shape))
        out[name] = flat[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in param_shapes()])


def round_bf16(x):
    """Round to the nearest bfloat16 value, ties to even (finite inputs):
    through float32, then keep the top 16 bits after adding half an ulp of
    the kept part (plus one when the kept part is odd)."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def frame_index(action, to_move, N):
    """Cell index in the mover's frame of a board cell (transpose for
    player 2)."""
    a = np.asarray(action, np.int64)
    r, c = a // N, a % N
    return np.where(np.asarray(to_move) == 2, c * N + r, a)


def encode(board, to_move, N):
    """[n][N*N] int8 boards + to_move -> [n][3][N][N] planes."""
    b = np.asarray(board).reshape(-1, N, N)
    n = b.shape[0]
    x = np.zeros((n, 3, N, N))
    for i in range(n):
        if to_move[i] == 1:
            B, me, op = b[i], 1, 2
        else:
            B, me, op = b[i].T, 2, 1
        x[i, 0] = B == me
        x[i, 1] = B == op
        x[i, 2] = B == 0
    return x


def conv3x3(x, w, bias=None):
    """Zero-padded 3x3 cross-correlation: out[n][o][r][c] =
    sum_{i,dr,dc} w[o][i][dr][dc] x[n][i][r+dr-1][c+dc-1]."""
    n, ci, N, _ = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, w.shape[0], N, N))
    for dr in range(3):
        for dc in range(3):
            out += np.einsum("nihw,oi->nohw", xp[:, :, dr:dr + N, dc:dc + N], w[:, :, dr, dc], optimize=True)
    if bias is not None:
        out += bias[None, :, None, None]
    return out


def conv3x3_backward(x, w, dz):
    """Gradients of conv3x3(x, w) + b given dz = dL/d(out): (dx, dw, db)."""
    n, ci, N, _ = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dr in range(3):
        for dc in range(3):
            dxp[:, :, dr:dr + N, dc:dc + N] += np.einsum("nohw,oi->nihw", dz, w[:, :, dr, dc], optimize=True)
            dw[:, :, dr, dc] = np.einsum("nohw,nihw->oi", dz, xp[:, :, dr:dr + N, dc:dc + N], optimize=True)
    return dxp[:, :, 1:N + 1, 1:N + 1], dw, dz.sum(axis=(0, 2, 3))


def forward(params, board, to_move, N, bf16=True):
    """Returns a dict: logits [n][N*N] in ACTION order (board cells),
    logits_frame [n][N*N] in the mover's frame, legal_frame, value [n], and
    the activations (for backward)."""
    P = unpack(params)
    rnd = round_bf16 if bf16 else (lambda t: t)
    x = encode(board, to_move, N)
    ys = [x]
    for l in range(1, LAYERS + 1):
        z = conv3x3(ys[-1], rnd(P[f"W{l}"]), P[f"b{l}"])
        ys.append(rnd(np.maximum(z, 0.0)))
    y4 = ys[-1]
    n = x.shape[0]
    lf = np.einsum("nchw,c->nhw", y4, P["wp"]).reshape(n, N * N) + P["bp"][0]
    h = y4.mean(axis=(2, 3))
    u = h @ P["wv"] + P["bv"][0]
    v = np.tanh(u)
    # back to action order: the frame of player 2 is the transpose
    logits = lf.copy()
    t2 = np.asarray(to_move) == 2
    if t2.any():
        logits[t2] = lf[t2].reshape(-1, N, N).transpose(0, 2, 1).reshape(-1, N * N)
    return {"x": x, "ys": ys, "logits_frame": lf, "logits": logits, "h": h, "value": v,
            "legal_frame": x[:, 2].reshape(n, N * N) > 0}


def masked_softmax(logits, legal):
    z = np.where(legal, logits, -np.inf)
    m = z.max(axis=1, keepdims=True)
    e = np.where(legal, np.exp(z - m), 0.0)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grads(params, board, to_move, action, z, N, beta=1.0, bf16=True, fwd=None):
    """Loss of the batch (value part, policy part) and the gradient of L
    with respect to the flat parameter vector.  action: board cell played in
    each state (must be empty); z: final outcome for the mover."""
    P = unpack(params)
    rnd = round_bf16 if bf16 else (lambda t: t)
    f = fwd if fwd is not None else forward(params, board, to_move, N, bf16)
    n = f["value"].shape[0]
    z = np.asarray(z, np.float64)
    v = f["value"]
    pi = masked_softmax(f["logits_frame"], f["legal_frame"])
    a = frame_index(action, to_move, N)
    adv = np.maximum(z - v, 0.0)  # held constant
    logp = np.log(pi[np.arange(n), a])
    loss_v = np.mean((v - z) ** 2)
    loss_p = np.mean(beta * adv * (-logp))
    # head gradients
    dlog = beta * adv[:, None] * pi
    dlog[np.arange(n), a] -= beta * adv
    dlog /= n                                   # [n][PIX], zero off the legal cells
    du = (2.0 * (v - z) / n) * (1.0 - v * v)    # through tanh
    ys = f["ys"]
    y4 = ys[-1]
    g = {}
    g["wp"] = np.einsum("nchw,nhw->c", y4, dlog.reshape(n, N, N))
    g["bp"] = np.array([dlog.sum()])
    g["wv"] = f["h"].T @ du
    g["bv"] = np.array([du.sum()])
    dy = (np.einsum("nhw,c->nchw", dlog.reshape(n, N, N), P["wp"])
          + np.einsum("n,c->nc", du, P["wv"])[:, :, None, None] / (N * N))
    for l in range(LAYERS, 0, -1):
        dz = rnd(dy * (ys[l] > 0))
        dx, dw, db = conv3x3_backward(ys[l - 1], rnd(P[f"W{l}"]), dz)
        g[f"W{l}"], g[f"b{l}"] = dw, db
        dy = dx
    return (loss_v, loss_p), pack(g)


def adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, 2015) with bias correction; returns the
    new (params, m, v)."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def policy_action(logits, legal, w):
    """The move a policy step draws: over the legal actions in increasing
    order, the running float32 sum of exp(logit - max) is compared with
    u * total, u = (w >> 8) / 2^24 (w = the ply's 32-bit Philox word); the
    first action whose running sum exceeds it is played (the last legal one
    if none does).  Returns (action, margin): margin is the smallest distance
    between the threshold and a running sum, relative to the total, which
    says how close the draw was to picking a neighbour (an exp that differs
    in the last bit can move a running sum across the threshold only when
    the margin is of the order of float32 rounding)."""
    idx = np.flatnonzero(legal)
    lg = np.asarray(logits, np.float32)[idx]
    mx = lg.max()
    e = np.exp((lg - mx).astype(np.float32)).astype(np.float32)
    run = np.cumsum(e, dtype=np.float32)  # sequential float32 sums
    tot = run[-1]
    thr = np.float32(np.float32(w >> 8) * np.float32(2.0 ** -24)) * tot
    hit = np.flatnonzero(run > thr)
    a = int(idx[hit[0]]) if hit.size else int(idx[-1])
    margin = float(np.min(np.abs(run.astype(np.float64) - float(thr))) / float(tot))
    return a, margin
