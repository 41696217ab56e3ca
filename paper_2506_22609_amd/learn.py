"""Training data, training loop and value-cutoff evaluation of the
policy/value network, driven through the C ABI (every step of the game and
of the network runs in the library's kernels; PyTorch holds the buffers and
does the index bookkeeping).

Samples come from seeded uniform-random playouts (the paper's benchmark
policy, Sec. 6): every ply of every game gives one sample (position, the
move played there, the final outcome for the player who moved).  The
network learns the value (expected outcome under random play) and a policy
weighted towards moves after which the mover did better than predicted.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import torch

from . import ludax

RUNNING, TERMINAL = 0, 1


@dataclass
class Samples:
    board: torch.Tensor    # [m][cells] int8
    to_move: torch.Tensor  # [m] int8
    action: torch.Tensor   # [m] int16, the cell played
    z: torch.Tensor        # [m] float32, final outcome for the mover

    def __len__(self):
        return self.board.shape[0]

    def take(self, idx):
        return Samples(self.board[idx], self.to_move[idx], self.action[idx], self.z[idx])


def collect(game: ludax.Game, n_games: int, seed: int, id_base: int, batch: int = 65536) -> Samples:
    """Play n_games uniform-random games (ids id_base + i) ply by ply with
    ludax_random_step and keep every position before a move."""
    boards, tms, acts, zs = [], [], [], []
    for g0 in range(0, n_games, batch):
        n = min(batch, n_games - g0)
        s = ludax.State(game, n)
        ludax.init(game, s)
        r = torch.empty((n, 2), dtype=torch.int8, device="cuda")
        t = torch.empty(n, dtype=torch.uint8, device="cuda")
        rec = []
        for _ in range(game.max_plies):
            live = (s.status == RUNNING).nonzero().squeeze(1)
            if live.numel() == 0:
                break
            b, m = s.board[live].clone(), s.to_move[live].clone()
            ludax.random_step(game, s, seed, id_base + g0, reward=r, terminal=t)
            rec.append((live, b, m, s.last_action[live].clone()))
        w = s.winner.to(torch.float32)
        for live, b, m, a in rec:
            wl = w[live]
            mf = m.to(torch.float32)
            z = torch.where(wl == mf, 1.0, torch.where(wl == 3.0 - mf, -1.0, 0.0))
            boards.append(b)
            tms.append(m)
            acts.append(a)
            zs.append(z)
    return Samples(torch.cat(boards), torch.cat(tms), torch.cat(acts), torch.cat(zs))


def train(net: ludax.Net, data: Samples, steps: int, batch: int = 4096, lr: float = 1e-3, beta: float = 1.0,
          seed: int = 0, log_every: int = 0):
    """Adam on shuffled minibatches (the paper's training batch size 4096
    and learning rate 0.001).  Returns the per-step losses [steps][2]."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    m = len(data)
    perm = torch.randperm(m, generator=gen).cuda()
    losses = torch.empty((steps, 2), dtype=torch.float32, device="cuda")
    grads = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    pos = 0
    t0 = time.perf_counter()
    for k in range(steps):
        if pos + batch > m:
            perm = torch.randperm(m, generator=gen).cuda()
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        b = data.take(idx)
        net.loss_grad(b.board, b.to_move, b.action, b.z, beta=beta, grads=grads, loss=losses[k])
        net.adam(grads, lr=lr)
        if log_every and (k + 1) % log_every == 0:
            lv = losses[k - log_every + 1:k + 1].mean(0).tolist()
            print(f"step {k + 1}: value loss {lv[0]:.4f} policy term {lv[1]:.4f} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
    return losses


def replicate(game: ludax.Game, s: ludax.State, reps: int) -> ludax.State:
    """reps copies of every env (env i's copies are rows i*reps .. i*reps+reps-1)."""
    t = {f: getattr(s, f).repeat_interleave(reps, dim=0).contiguous() for f in ludax.State.FIELDS}
    return ludax.State.from_tensors(game, **t)


def outcome_p1(s: ludax.State) -> torch.Tensor:
    w = s.winner.to(torch.float32)
    return torch.where(s.status == TERMINAL, torch.where(w == 1, 1.0, torch.where(w == 2, -1.0, 0.0)),
                       torch.zeros_like(w))


def truth(game: ludax.Game, s: ludax.State, reps: int, seed: int, id_base: int) -> torch.Tensor:
    """Mean outcome for player 1 of `reps` full random playouts from each
    state (distinct game ids), the reference the estimates are judged by."""
    r = replicate(game, s, reps)
    ludax.playout(game, r, seed, id_base, stats=None)
    return outcome_p1(r).view(s.n, reps).mean(1)


def cutoff_estimate(game: ludax.Game, net: ludax.Net, s: ludax.State, k: int, seed: int, id_base: int):
    """k uniform-random plies (ludax_random_step), then the value cutoff
    (ludax_net_estimate).  Modifies s."""
    r = torch.empty((s.n, 2), dtype=torch.int8, device="cuda")
    t = torch.empty(s.n, dtype=torch.uint8, device="cuda")
    for _ in range(k):
        ludax.random_step(game, s, seed, id_base, reward=r, terminal=t)
    return net.estimate(s)


def play_vs_random(game: ludax.Game, net: ludax.Net, n: int, net_player: int, seed: int, id_base: int):
    """n games of the network's policy (ludax_policy_step on the logits of
    ludax_net_forward) against the uniform-random policy, the network moving
    for net_player (1 or 2).  All games start together and the mover of
    every running game at ply t is the same, so each ply is one call of one
    of the two steps.  Returns (net wins, opponent wins, draws)."""
    s = ludax.State(game, n)
    ludax.init(game, s)
    r = torch.empty((n, 2), dtype=torch.int8, device="cuda")
    t = torch.empty(n, dtype=torch.uint8, device="cuda")
    for ply in range(game.max_plies):
        if ply % 2 == net_player - 1:
            logits, _ = net.forward(s.board, s.to_move)
            ludax.policy_step(game, s, logits, seed, id_base, reward=r, terminal=t)
        else:
            ludax.random_step(game, s, seed, id_base, reward=r, terminal=t)
    w = s.winner
    return (int((w == net_player).sum()), int((w == 3 - net_player).sum()), int((w == 0).sum()))


def estimate_budgeted(game: ludax.Game, net: ludax.Net, s: ludax.State, budget_bytes: int,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """ludax_net_estimate over a batch of any size with the network's
    workspace held to budget_bytes of HBM: the envs are admitted in chunks
    of the largest batch whose workspace fits (ludax_net_max_batch)."""
    chunk = net.max_batch(budget_bytes) // 64 * 64  # whole workgroups; keeps every chunk's boards 16-byte aligned
    if chunk < 64:
        raise ValueError("the HBM budget does not hold the workspace of 64 positions")
    if out is None:
        out = torch.empty(s.n, dtype=torch.float32, device=s.board.device)
    for a in range(0, s.n, chunk):
        b = min(s.n, a + chunk)
        part = ludax.State.from_tensors(game, **{f: getattr(s, f)[a:b] for f in ludax.State.FIELDS})
        net.estimate(part, out=out[a:b])
    return out


def guided_budgeted(game: ludax.Game, net: ludax.Net, s: ludax.State, plies: int, budget_bytes: int, seed: int,
                    id_base: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Network-guided playouts with a value cutoff over a batch of any size,
    the network's workspace and logits held to budget_bytes of HBM: the envs
    are admitted in chunks (whole 64-env workgroups) of the largest batch
    whose inference workspace plus logits fit, and each chunk plays `plies`
    guided plies (ludax_net_forward, then ludax_policy_step; game ids
    id_base + env index, as for one call over the whole batch) before the
    value cutoff (ludax_net_estimate).  Modifies s; returns the estimates
    for player 1."""
    cells = game.cells
    chunk = guided_chunk(net, budget_bytes, cells)
    if chunk < 64:
        raise ValueError("the HBM budget does not hold the workspace of 64 positions")
    if out is None:
        out = torch.empty(s.n, dtype=torch.float32, device=s.board.device)
    logits = torch.empty((chunk, cells), dtype=torch.float32, device=s.board.device)
    value = torch.empty(chunk, dtype=torch.float32, device=s.board.device)
    r = torch.empty((chunk, 2), dtype=torch.int8, device=s.board.device)
    t = torch.empty(chunk, dtype=torch.uint8, device=s.board.device)
    for a in range(0, s.n, chunk):
        b = min(s.n, a + chunk)
        m = b - a
        part = ludax.State.from_tensors(game, **{f: getattr(s, f)[a:b] for f in ludax.State.FIELDS})
        for _ in range(plies):
            net.forward(part.board, part.to_move, logits=logits[:m], value=value[:m])
            ludax.policy_step(game, part, logits[:m], seed, id_base + a, reward=r[:m], terminal=t[:m])
        net.estimate(part, out=out[a:b])
    return out


def guided_chunk(net: ludax.Net, budget_bytes: int, cells: int) -> int:
    """The chunk guided_budgeted admits: the largest whole number of 64-env
    workgroups whose inference workspace plus logits fit the budget."""
    k = net.max_batch(budget_bytes)
    while k > 0 and ludax_ws_plus_logits(net, k, cells) > budget_bytes:
        k -= max(1, k // 64)
    return k // 64 * 64


def ludax_ws_plus_logits(net: ludax.Net, n: int, cells: int) -> int:
    """Inference workspace of n positions plus their float32 logits and
    values (bytes)."""
    return net.workspace_bytes(n) + n * (cells + 1) * 4
