#!/usr/bin/env python3
"""Throughput benchmark of the batched random-playout hot path on one MI355X.

Workload: single-game batches of 65536 environments each, Connect Four 6x7
and Hex 11x11 (int8 boards), uniform-random playouts from the start
position to the end of every game.  One benchmark step = both batches
reset to the start position and played out (legal mask, Philox draw, k-th
legal action, apply, end rules, repeated until every game has ended) with
the step/outcome counters, all in one launch (ludax_playout_batches);
the same step as six separate launches (ludax_init, ludax_playout,
ludax_state_stats per batch) is reported beside it.  Every step uses fresh
game ids, so no two steps play the same games.

Prints one JSON line: env-steps/s over the timed steps (all plies applied
by all environments / wall time between two device synchronisations), the
roofline figures of the dominant kernel (the one-grid playout kernel,
timed with events on its stream) and the CPU oracle's rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# The mixed persistent batches run one kernel per game kind on a stream of
# its own, concurrently.  HIP spreads a process's streams over
# GPU_MAX_HW_QUEUES hardware queues (4 by default) and kernels that share a
# queue run one after the other, so with torch's streams and two mixed
# handles alive the kinds would partly serialise (the 1M-game 19x19 mixed
# batch: 4.2 against 3.0 ms).  Sixteen queues give every stream of this
# process one of its own; the runtime reads the variable when it starts,
# before torch is imported.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer VALU work per env-step of the playout kernels (lane-operations):
# SQ_INSTS_VALU x 64 / env-steps of one launch, measured with rocprofv3 on
# this workload (profiles/playout_c4_hex11_n65536_sq_counters.txt): the
# separate Connect Four and Hex kernels, and the one-grid launch of both
# batches (env-steps of both).  Peak: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3 T lane-ops/s (the fp64 vector rate 78.6 TFLOP/s counts an
# FMA as two operations).
VALU_OPS_PER_STEP = {"connect4_6x7_n65536": 239, "hex11x11_n65536": 158, "group": 170}
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# the same count for the mixed persistent batch's one-grid kernel
# (k_persist_group over 4 x 262144 games, same profile)
MIXED_VALU_OPS_PER_STEP = 320
# HBM bytes of one launch of the dominant kernel: FETCH_SIZE and WRITE_SIZE
# scaled by a 1 GiB device copy in the same profiled run
# (profiles/playout_c4_hex11_n65536_hbm_bytes.txt): 0.41 MB read (no state:
# the kernel resets the envs itself) and 12.12 MB written (the final
# states, exactly their algorithmic bytes).
GROUP_TRAFFIC_BYTES = 12.53e6
HBM_PEAK_GBS = 8000.0
EVENT_EVERY = 8
# What the paper states about its own throughput (Sec. 6, Fig. 2): no
# absolute rate in the text (the figure is a plot), so vs_baseline is null.
PAPER_CONTEXT = {
    "absolute_env_steps_per_s": None,
    "figure": "Fig. 2: moves per second against batch size for 10 games (plot only)",
    "hardware": "one NVIDIA RTX 4090 (Ludax, PGX); Intel i9-9980XE, 18 cores / 36 threads (Ludii)",
    "protocol": "100 warm-up full-game episodes, then 500 measured, per batch size; std over episodes",
    "speedup_over_ludii": "about 3x (English Draughts) to about 450x (Hex), tensor playout regime",
}
# DRAM bytes (read + written) per env-step of the per-ply loop, from the
# FETCH_SIZE / WRITE_SIZE counters of every ludax_random_step dispatch of one
# loop, each scaled by what the counter reads for a 1 GiB device copy in the
# same profiled run (profiles/random_step_hex19_n1048576_hbm_bytes.txt).
DRAM_BYTES_PER_ENV_STEP = {"hex19x19_n1048576": 407.1 + 43.9, "hex19x19_n1048576_aux": 292.7 + 155.4}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(batches, budget_s: float):
    """The oracle as it stands on the host's cores: 3 warm-up and then at
    least 20 timed batches of the same workload (distinct game ids), with
    all the process's cores and with one thread; each batch's rate is
    recorded and the median and standard deviation reported.  The
    one-thread batches hold 4096 envs per game (a whole 65536-env batch
    takes seconds on one core; the oracle's per-env cost does not depend
    on the batch size).  budget_s bounds the timed batches of each leg."""
    import statistics

    from oracle import ref
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 64))

    def leg(threads: int, n_env: int, budget: float):
        rates, steps_total, el_total, k = [], 0, 0.0, 0
        while len(rates) < 20 or (el_total < budget and len(rates) < 200):
            steps, t0 = 0, time.perf_counter()
            for b in batches:
                g = ref.Game(b.kind, b.rows, b.cols)
                s = ref.init(g, n_env)
                _, _, st = ref.playout(g, s, 1, n_env * (1000 + k), threads=threads)
                steps += int(st[0])
            el = time.perf_counter() - t0
            if k >= 3:
                rates.append(steps / el)
                steps_total += steps
                el_total += el
            k += 1
        return {"median": statistics.median(rates), "std": statistics.pstdev(rates), "batches": len(rates),
                "envs_per_game": n_env, "threads": threads, "env_steps": steps_total, "seconds": el_total}

    full = leg(cores, batches[0].n, 0.5 * budget_s)
    one = leg(1, 4096, 0.5 * budget_s)
    names = " + ".join(b.name for b in batches)
    return {"value": full["median"], "unit": "env-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{full['batches']} timed batches of ({names}) after 3 warm-up batches, "
                      f"median of the per-batch rates",
            "cpu_model": _cpu_model(), "compiler": "gcc -O2 -std=c11 (oracle/ludax_ref.c), pthreads",
            "all_cores": full, "one_thread": one}


def _protocol(batches, games, states, rewards, terms, seeds=(1, 2, 3), warmup: int = 3, steps: int = 20):
    """The benchmark step repeated per seed: warm-up steps, then `steps`
    steps each bracketed by events on the stream (both batches reset and
    played out, with their counters, by one launch), fresh game ids every
    step; per seed the median and standard deviation of the per-step
    env-steps/s."""
    import statistics

    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    stream = torch.cuda.current_stream()
    group = ludax.BatchGroup([(g, s, r, t, None) for g, s, r, t in zip(games, states, rewards, terms)])
    out = {}
    for seed in seeds:
        st = torch.zeros((steps, len(batches), 4), dtype=torch.int64, device="cuda")
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for k in range(warmup + steps):
            rec = k >= warmup
            if rec:
                evs[k - warmup][0].record(stream)
            group.run(seed, [W.game_id_base(1000 + k, b) for b in batches], from_start=True, stream=stream,
                      stats=[st[k - warmup, j] if rec else None for j in range(len(batches))])
            if rec:
                evs[k - warmup][1].record(stream)
        torch.cuda.synchronize()
        env_steps = st[:, :, 0].sum(dim=1).cpu().tolist()
        ms = [a.elapsed_time(c) for a, c in evs]
        rates = [e / (m / 1e3) for e, m in zip(env_steps, ms)]
        out[f"seed{seed}"] = {"median_env_steps_per_s": statistics.median(rates),
                              "std_env_steps_per_s": statistics.pstdev(rates),
                              "median_ms_per_step": statistics.median(ms), "std_ms_per_step": statistics.pstdev(ms),
                              "steps": steps, "warmup": warmup}
    return out


def _separate_launches(batches, games, states, rewards, terms, seed: int, warmup: int = 3, steps: int = 20):
    """The same step as separate launches on one stream: per batch
    ludax_init, ludax_playout (its kernel bracketed by events) and
    ludax_state_stats(+1), six launches in all (right after ludax_init the
    counters' (-1) reduction adds zero, so one reduction after the playout
    gives them).  Reported beside the one-grid step."""
    import statistics

    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    stream = torch.cuda.current_stream()
    st = torch.zeros((len(batches), 4), dtype=torch.int64, device="cuda")
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
          for _ in batches]
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for k in range(warmup + steps):
        rec = k >= warmup
        if rec:
            step_ev[k - warmup][0].record(stream)
        for j, (b, g, s, r, t) in enumerate(zip(batches, games, states, rewards, terms)):
            ludax.init(g, s, stream=stream)
            if rec:
                ev[j][k - warmup][0].record(stream)
            ludax.playout(g, s, seed, W.game_id_base(2000 + k, b), reward=r, terminal=t, stats=None, stream=stream)
            if rec:
                ev[j][k - warmup][1].record(stream)
                ludax.state_stats(g, s, +1, st[j], stream=stream)
        if rec:
            step_ev[k - warmup][1].record(stream)
    torch.cuda.synchronize()
    ms = [a.elapsed_time(c) for a, c in step_ev]
    env_steps = int(st[:, 0].sum().item())
    return {"median_ms_per_step": statistics.median(ms),
            "env_steps_per_s": env_steps / (sum(ms) / 1e3),
            "playout_kernel_ms": {b.name: statistics.median(a.elapsed_time(c) for a, c in ev[j])
                                  for j, b in enumerate(batches)},
            "launches_per_step": 6, "steps": steps, "warmup": warmup}


def _mixed_equal_split_ms(m, kinds: int, total: int, seed: int, n: int, out, reps: int = 3) -> float:
    """Median event-timed batch of the mixed handle under the equal slot
    split (the plan before autotuning)."""
    import statistics

    import torch

    m.slots = [total // kinds // 64 * 64] * kinds
    m.playout(seed, 0, n, out=out, stats=None)
    ts = []
    for k in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        m.playout(seed, 0, n, out=out, stats=None)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def _mixed_section(seed: int, steps: int, warmup: int):
    """Mixed persistent batch (Reversi 8x8, Gomoku 15x15, Hex 11x11,
    Connect Four 6x7; game id g has kind g mod 4): 4 x 262144 game ids
    played through 262144 slots with refill, slot split autotuned, the call
    captured in a graph and replayed; beside it the same games as four
    plain single-kind batches of 262144 envs (init + playout each)."""
    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    mb = W.MIXED4
    games = [ludax.Game(b.kind, b.rows, b.cols) for b in mb.kinds]
    m = ludax.Mixed(games)
    n = mb.n_games
    out = ludax.MixedResult(n, len(games))
    # the equal split launched as one grid and as a kernel per kind
    equal_ms = {}
    for og in (True, False):
        m.one_grid = og
        equal_ms["one_grid" if og else "streams"] = _mixed_equal_split_ms(m, len(games), mb.slots, seed, n, out)
    tune_ms = m.autotune(seed, 0, n, mb.slots, out=out)
    stats = torch.zeros((len(games), 4), dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        m.playout(seed, 0, n, out=out, stats=stats)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.playout(seed, 0, n, out=out, stats=stats)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    stats.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    g_el = time.perf_counter() - t0
    per_kind = stats.cpu().tolist()
    g_steps = sum(r[0] for r in per_kind)
    # eager calls with fresh game ids every step
    stats.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        m.playout(seed, (k + 1) * n, n, out=out, stats=stats)
    torch.cuda.synchronize()
    e_el = time.perf_counter() - t0
    e_steps = int(stats[:, 0].sum().item())
    # the same games as four plain single-kind batches
    per = n // len(games)
    states = [ludax.State(g, per) for g in games]
    ids = [torch.arange(k, n, len(games), dtype=torch.int64, device="cuda") for k in range(len(games))]
    pst = torch.zeros(4, dtype=torch.int64, device="cuda")
    for g, s_, i in zip(games, states, ids):
        ludax.init(g, s_)
        ludax.playout(g, s_, seed, 0, game_id=i, stats=None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for g, s_, i in zip(games, states, ids):
            ludax.init(g, s_)
            ludax.playout(g, s_, seed, 0, game_id=i, stats=pst)
    torch.cuda.synchronize()
    p_el = time.perf_counter() - t0
    p_steps = int(pst[0].item())
    return {
        "workload": f"{mb.name}: {n} game ids, kind = id mod 4 "
                    f"({', '.join(b.name for b in mb.kinds)}), {mb.slots} slots with refill",
        "slots_per_kind": m.slots, "one_grid": m.one_grid, "autotuned_ms": tune_ms, "equal_split_ms": equal_ms,
        "mixed_graph_env_steps_per_s": g_steps / g_el,
        "mixed_graph_ms_per_batch": g_el / steps * 1e3,
        # VALU lane-ops per env-step (measured, one grid) x env-steps / time
        "valu_frac_graph": (MIXED_VALU_OPS_PER_STEP * g_steps / g_el / 1e12 / VALU_PEAK_TOPS
                            if m.one_grid else None),
        "mixed_eager_env_steps_per_s": e_steps / e_el,
        "plain_env_steps_per_s": p_steps / p_el,
        "plain_ms_per_batch": p_el / steps * 1e3,
        "env_steps_per_batch": g_steps // steps,
        "per_kind_env_steps_per_batch": [r[0] // steps for r in per_kind],
        "note": "graph replays repeat the captured game ids; eager calls use new ids each batch",
    }


def _copy_peak_gbs(mib: int = 1024, reps: int = 5) -> float:
    """Measured stream-copy rate of this GPU: a plain device-to-device copy
    of `mib` MiB, bytes read plus bytes written per second, event-timed."""
    import torch

    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * (mib << 20) / sec / 1e9


def _alg_bytes_per_env_step(game, aux: bool) -> int:
    """Algorithmic HBM bytes of one env-step of the per-ply loop.  Without
    the cache: the board and 8 B of scalars read; 8 B of scalars, 2 B
    reward, 1 B terminal and the 1-byte board delta written (cells + 20 B).
    With Hex's component cache: the two players' stones (8 B per 32 cells),
    the 4-byte tag and 8 B of scalars read; the scalars, reward, terminal,
    board delta, the changed 4-byte stone word, the tag and the new stone's
    2-byte parent entry written (the joins' parent reads and writes are
    data dependent and not counted)."""
    if not aux:
        return game.cells + 20
    nwc = (game.cells + 31) // 32
    return (8 * nwc + 4 + 8) + (8 + 3 + 1 + 4 + 4 + 2)


def _plain_step_section(cases, seed: int, reps: int):
    """The per-ply loop with the state in HBM between plies: ludax_init,
    then ludax_random_step launched max_plies times (the game's natural
    bound, so every game ends inside the loop), captured in one graph per
    batch and replayed.  cases: (batch, aux) pairs; aux = the Hex component
    cache (ludax_state.aux).  The replay time includes the launches of the
    tail, when few games are still running, and the gaps between graph
    nodes.  The achieved rate of algorithmic bytes is given as a fraction
    of the nominal HBM peak and of the measured stream-copy rate
    ("copy_peak_GBs"); where the profile of the per-ply kernels measured
    DRAM bytes per env-step (DRAM_BYTES_PER_ENV_STEP), their rate too
    ("hbm_frac_dram")."""
    import torch
    from paper_2506_22609_amd import ludax

    copy_gbs = _copy_peak_gbs()
    out = {"copy_peak_GBs": copy_gbs}
    for b, aux in cases:
        g = ludax.Game(b.kind, b.rows, b.cols)
        s = ludax.State(g, b.n, aux=aux)
        r = torch.empty((b.n, 2), dtype=torch.int8, device="cuda")
        t = torch.empty(b.n, dtype=torch.uint8, device="cuda")
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        base = 7 * b.n

        def loop():
            ludax.init(g, s)
            for _ in range(g.max_plies):
                ludax.random_step(g, s, seed, base, reward=r, terminal=t)

        # eager run bracketed by the counters: env-steps of one loop
        ludax.init(g, s)
        ludax.state_stats(g, s, -1, st)
        for _ in range(g.max_plies):
            ludax.random_step(g, s, seed, base, reward=r, terminal=t)
        ludax.state_stats(g, s, +1, st)
        torch.cuda.synchronize()
        steps = int(st[0].item())
        running_after = int((s.status == 0).sum().item())
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            loop()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            loop()
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        per = _alg_bytes_per_env_step(g, aux)
        init_bytes = b.n * (g.cells + 8) + (b.n * (16 + 8 * ((g.cells + 31) // 32)) if aux else 0)
        alg = steps * per + init_bytes
        name = b.name + ("_aux" if aux else "")
        res = {"launches": g.max_plies, "aux": bool(aux), "state_bytes": b.n * (g.cells + 8)
               + (b.n * g.aux_bytes if aux else 0), "env_steps": steps, "ms_per_loop": el * 1e3,
               "env_steps_per_s": steps / el, "alg_bytes_per_env_step": per,
               "alg_bytes_per_loop": alg, "achieved_GBs": alg / el / 1e9,
               "hbm_frac": alg / el / 1e9 / HBM_PEAK_GBS,
               "hbm_frac_of_copy": alg / el / 1e9 / copy_gbs,
               "still_running_after_loop": running_after}
        dram = DRAM_BYTES_PER_ENV_STEP.get(name)
        if dram is not None:
            res["dram_bytes_per_env_step"] = dram
            res["dram_GBs"] = dram * steps / el / 1e9
            res["hbm_frac_dram"] = dram * steps / el / 1e9 / HBM_PEAK_GBS
        out[name] = res
        del graph, s
        torch.cuda.synchronize()
    return out


def _large_section(batches, seed: int, reps: int):
    """Plain fused playouts (ludax_init + ludax_playout) of the large
    single-game batches, the playout kernel timed with events; and the
    same games through a one-kind persistent batch (refill)."""
    import torch
    from paper_2506_22609_amd import ludax

    out = {}
    for b in batches:
        g = ludax.Game(b.kind, b.rows, b.cols)
        s = ludax.State(g, b.n)
        r = torch.empty((b.n, 2), dtype=torch.int8, device="cuda")
        t = torch.empty(b.n, dtype=torch.uint8, device="cuda")
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        ludax.init(g, s)
        ludax.playout(g, s, seed, 0, reward=r, terminal=t, stats=None)
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for k in range(reps):
            ludax.init(g, s)
            ludax.state_stats(g, s, -1, st)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ludax.playout(g, s, seed, (k + 1) * b.n, reward=r, terminal=t, stats=None)
            e1.record()
            evs.append((e0, e1))
            ludax.state_stats(g, s, +1, st)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        kern = sum(a.elapsed_time(c) for a, c in evs) / reps / 1e3
        v = st.cpu().tolist()
        out[b.name] = {"env_steps_per_batch": v[0] // reps, "games_per_batch": b.n,
                       "ms_per_batch": el * 1e3, "playout_kernel_ms": kern * 1e3,
                       "env_steps_per_s": v[0] / reps / el, "playouts_per_s": b.n / el,
                       "mean_plies": v[0] / reps / b.n,
                       "p1_wins": v[1], "p2_wins": v[2], "draws": v[3]}
        del s
        torch.cuda.synchronize()
        # the same games through the persistent batch of this one kind
        # (ludax_mixed_*): 262144 lanes, a lane refilled as soon as its game
        # ends instead of waiting for the longest game of its wave; per-game
        # outputs (winner, plies, last action) instead of the final states
        m = ludax.Mixed([g])
        m.slots = [262144]
        res = ludax.MixedResult(b.n, 1)
        mst = torch.zeros((1, 4), dtype=torch.int64, device="cuda")
        m.playout(seed, 0, b.n, out=res, stats=None)
        torch.cuda.synchronize()
        ms = []
        for k in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            m.playout(seed, (k + 1) * b.n, b.n, out=res, stats=mst)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        ms.sort()
        med = ms[len(ms) // 2]
        psteps = int(mst[0, 0].item()) / reps
        out[b.name]["persistent"] = {"slots": 262144, "one_grid": m.one_grid, "ms_per_batch": med,
                                     "env_steps_per_s": psteps / (med / 1e3), "playouts_per_s": b.n / (med / 1e3)}
        del m, res
        torch.cuda.synchronize()
    return out


def _large_mixed_section(seed: int, reps: int, train_steps: int, budget_gb: float):
    """Large boards, mixed: 1,048,576 game ids, kind = id mod 2 (Hex 19x19,
    Gomoku 19x19), through the mixed persistent batch (slots autotuned) and
    as the two plain single-kind batches; then per game a network trained
    on its own random games, and 524288 held-out positions per game
    estimated by one full random playout and by the network's value with
    the network's workspace held to an HBM budget (positions admitted in
    chunks of ludax_net_max_batch), judged against the mean of 256 full
    random playouts on 2048 of them."""
    import torch
    from paper_2506_22609_amd import learn, ludax
    from paper_2506_22609_amd import workloads as W
    from paper_2506_22609_amd.workloads import init_net_params

    kinds = W.LARGE_BATCHES
    games = [ludax.Game(b.kind, b.rows, b.cols) for b in kinds]
    n_games = sum(b.n for b in kinds)
    m = ludax.Mixed(games)
    out = ludax.MixedResult(n_games, len(games))
    equal_ms = _mixed_equal_split_ms(m, len(games), 262144, seed, n_games, out)
    tune_ms = m.autotune(seed, 0, n_games, 262144, out=out)
    stats = torch.zeros((len(games), 4), dtype=torch.int64, device="cuda")
    m.playout(seed, 0, n_games, out=out, stats=stats)
    torch.cuda.synchronize()
    stats.zero_()
    t0 = time.perf_counter()
    for k in range(reps):
        m.playout(seed, (k + 1) * n_games, n_games, out=out, stats=stats)
    torch.cuda.synchronize()
    mixed_el = (time.perf_counter() - t0) / reps
    res = {"workload": f"{n_games} game ids, kind = id mod 2 (hex19x19, gomoku19x19)",
           "mixed": {"slots_per_kind": m.slots, "autotuned_ms": tune_ms, "equal_split_ms": equal_ms,
                     "ms_per_batch": mixed_el * 1e3,
                     "env_steps_per_s": int(stats[:, 0].sum()) / reps / mixed_el,
                     "playouts_per_s": n_games / mixed_el,
                     "per_kind_env_steps_per_batch": [int(x) // reps for x in stats[:, 0].tolist()]},
           "guided": {}}
    del out
    budget = int(budget_gb * 2**30)
    for b, g in zip(kinds, games):
        # about 10 M samples: Hex 19x19 games last ~332 plies, Gomoku 19x19 ~159
        data = learn.collect(g, 30000 if b.kind == W.HEX else 60000, seed=seed + 800, id_base=0)
        net = ludax.Net(b.rows, b.cols, params=torch.from_numpy(init_net_params(seed)).cuda())
        t0 = time.perf_counter()
        learn.train(net, data, train_steps, batch=4096, lr=1e-3, seed=seed)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        n_train = len(data)
        del data
        ev = learn.collect(g, 8000, seed=seed + 900, id_base=10**9)
        idx = torch.randperm(len(ev), generator=torch.Generator().manual_seed(seed))[:b.n].cuda()
        e = ev.take(idx)
        del ev
        n = e.board.shape[0]
        base = ludax.State(g, n)
        ludax.init(g, base)
        base.board.copy_(e.board)
        base.to_move.copy_(e.to_move)
        base.ply.copy_((e.board != 0).sum(1).to(torch.int16))
        sub = 2048
        held = ludax.State.from_tensors(g, **{f: getattr(base, f)[:sub].contiguous() for f in ludax.State.FIELDS})
        tr = learn.truth(g, held, 256, seed=seed + 950, id_base=2 * 10**9)
        est = torch.empty(n, dtype=torch.float32, device="cuda")
        timings = {}
        for name in ("plain_full_playout", "value_budgeted"):
            for rep in range(2):
                s = base.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if name == "plain_full_playout":
                    ludax.playout(g, s, seed + 960, 3 * 10**9, stats=None)
                    est = learn.outcome_p1(s)
                else:
                    learn.estimate_budgeted(g, net, s, budget, out=est)
                torch.cuda.synchronize()
                timings[name] = time.perf_counter() - t0
            timings[name + "_mse"] = ((est[:sub] - tr) ** 2).mean().item()
        # network-guided playouts: 20 plies proposed by the policy (forward +
        # policy step per ply) for both sides, then the value cutoff, in chunks
        # admitted by the same HBM budget
        s = base.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est = learn.guided_budgeted(g, net, s, 20, budget, seed + 980, 6 * 10**9)
        torch.cuda.synchronize()
        timings["policy20_budgeted"] = time.perf_counter() - t0
        timings["policy20_budgeted_mse"] = ((est[:sub] - tr) ** 2).mean().item()
        del s
        k, mse_k, pps = _averaged_playouts_at_error(g, held, tr, timings["value_budgeted_mse"], base, seed + 970,
                                                    5 * 10**9)
        res["guided"][b.name] = {
            "fixed_value_error": {"mse": timings["value_budgeted_mse"], "plain_playouts_averaged": k,
                                  "plain_average_mse": mse_k, "plain_positions_per_s": pps,
                                  "guided_positions_per_s": n / timings["value_budgeted"],
                                  "note": "k measured, as in the learned section"},
            "positions": n, "train_samples": n_train, "train_steps": train_steps, "train_s": t_train,
            "hbm_budget_bytes": budget, "admitted_chunk": net.max_batch(budget),
            "plain_full_playout": {"playouts_per_s": n / timings["plain_full_playout"],
                                   "mse_vs_256_playout_mean": timings["plain_full_playout_mse"]},
            "value_budgeted": {"playouts_per_s": n / timings["value_budgeted"],
                               "mse_vs_256_playout_mean": timings["value_budgeted_mse"]},
            "policy20_value_cutoff_budgeted": {"playouts_per_s": n / timings["policy20_budgeted"],
                                               "mse_vs_256_playout_mean": timings["policy20_budgeted_mse"],
                                               "chunk": learn.guided_chunk(net, budget, g.cells)}}
        del base, held, net
        torch.cuda.synchronize()
    return res


def _sweep_section(seed: int, reps: int):
    """Throughput against batch size (Sec. 6, Fig. 2): for each of the
    ten games of the paper's figure and batch sizes 2^10 .. 2^20, full-game
    episodes from the start position (ludax_init + ludax_playout, the
    movement games capped at 200 plies), two warm-up batches, then `reps`
    timed batches with fresh game ids, each bracketed by events; the median
    time and the mean env-steps of the timed batches (counted outside the
    timed region) give env-steps/s."""
    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    out = {}
    for b in W.SWEEP_GAMES:
        g = ludax.Game(b.kind, b.rows, b.cols)
        row = {}
        for n in W.SWEEP_SIZES:
            s = ludax.State(g, n)
            r = torch.empty((n, 2), dtype=torch.int8, device="cuda")
            t = torch.empty(n, dtype=torch.uint8, device="cuda")
            st = torch.zeros(4, dtype=torch.int64, device="cuda")
            for k in range(2):
                ludax.init(g, s)
                ludax.playout(g, s, seed, k * n, reward=r, terminal=t, stats=None)
            torch.cuda.synchronize()
            ms = []
            for k in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ludax.init(g, s)
                ludax.playout(g, s, seed, (k + 2) * n, reward=r, terminal=t, stats=None)
                e1.record()
                ludax.state_stats(g, s, +1, st)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            steps = int(st[0].item()) / reps  # env-steps of one batch (the mean over the timed ones)
            ms.sort()
            med = ms[len(ms) // 2]
            row[str(n)] = {"ms_per_batch": med, "min_ms": ms[0], "max_ms": ms[-1],
                           "env_steps_per_s": steps / (med / 1e3), "mean_plies": steps / n}
            del s, r, t
        out[b.name] = row
    return out


def _more_games_section(seed: int, reps: int):
    """Plain fused playouts of the paper's other games, 65536 envs each:
    Yavalath on the diameter-9 hexagon, Pente 19x19, and the movement games
    Wolf and Sheep and English Draughts (8x8)."""
    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    out = {}
    for b in W.MORE_GAMES:
        g = ludax.Game(b.kind, b.rows, b.cols)
        s = ludax.State(g, b.n)
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        ludax.init(g, s)
        ludax.playout(g, s, seed, 0, stats=None)
        torch.cuda.synchronize()
        ev = []
        for k in range(reps):
            ludax.init(g, s)
            ludax.state_stats(g, s, -1, st)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ludax.playout(g, s, seed, (k + 1) * b.n, stats=None)
            e1.record()
            ev.append((e0, e1))
            ludax.state_stats(g, s, +1, st)
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(c) for a, c in ev) / reps
        v = st.cpu().tolist()
        out[b.name] = {"playout_kernel_ms": ms, "env_steps_per_s": v[0] / reps / (ms / 1e3),
                       "mean_plies": v[0] / reps / b.n, "p1_wins": v[1], "p2_wins": v[2], "draws": v[3]}
    # the unbounded movement games: a few games run to the 200-ply cap, so a
    # plain batch waits for them; the persistent batch (ludax_mixed_*, one
    # kind) refills a lane as soon as its game ends
    for b in (W.DRAUGHTS_65536, W.HASAMI_SHOGI_65536):
        n_games, slots = 4 * b.n, b.n
        g = ludax.Game(b.kind, b.rows, b.cols)
        s = ludax.State(g, n_games)
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        m = ludax.Mixed([g])
        m.slots = [slots]
        res = ludax.MixedResult(n_games, 1)
        mst = torch.zeros((1, 4), dtype=torch.int64, device="cuda")
        ludax.init(g, s)
        ludax.playout(g, s, seed, 0, stats=None)
        m.playout(seed, 0, n_games, out=res, stats=None)
        torch.cuda.synchronize()
        p_ms, q_ms = [], []
        for k in range(reps):
            base = (k + 1) * n_games
            ludax.init(g, s)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            ludax.playout(g, s, seed, base, stats=st)
            e1.record()
            m.playout(seed, base, n_games, out=res, stats=mst)
            e2.record()
            p_ms.append((e0, e1))
            q_ms.append((e1, e2))
        torch.cuda.synchronize()
        pm = sum(a.elapsed_time(c) for a, c in p_ms) / reps
        qm = sum(a.elapsed_time(c) for a, c in q_ms) / reps
        steps = st[0].item() / reps
        assert mst[0, 0].item() == st[0].item()  # the same games, the same plies
        out[b.name.replace(f"_n{b.n}", f"_games{n_games}")] = {
            "plain_ms": pm, "plain_env_steps_per_s": steps / (pm / 1e3),
            "persistent_slots": slots, "persistent_ms": qm, "persistent_env_steps_per_s": steps / (qm / 1e3)}
    return out


def _averaged_playouts_at_error(g, held, tr, target_mse: float, base, seed: int, id_base: int):
    """Plain random playouts at a fixed value error, measured: average k full
    random playouts per held-out position (new game ids for each), k = 1,
    2, ..., judging each average against the 256-playout mean tr, until its
    squared error is no larger than target_mse (at most 128); then time k
    playouts of every position of base.  Returns (k, the k-average's
    squared error, positions per second)."""
    import torch
    from paper_2506_22609_amd import learn, ludax

    acc = torch.zeros(held.n, dtype=torch.float32, device="cuda")
    k, mse_k = 0, float("inf")
    while k < 128 and mse_k > target_mse:
        s = held.clone()
        ludax.playout(g, s, seed, id_base + k * held.n, stats=None)
        acc += learn.outcome_p1(s)
        k += 1
        mse_k = ((acc / k - tr) ** 2).mean().item()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(k):
        s = base.clone()
        ludax.playout(g, s, seed + 1, id_base + (128 + j) * base.n, stats=None)
    torch.cuda.synchronize()
    return k, mse_k, base.n / (time.perf_counter() - t0)


def _learned_section(seed: int, train_games: int, steps: int):
    """The learned policy/value network on Hex 11x11: samples from random
    playouts, training by the library's own forward/backward/Adam kernels,
    then 65536 held-out positions estimated four ways (one full random
    playout; the value alone; 20 random plies + value cutoff; 20 plies
    proposed by the policy for both sides + value cutoff), each timed and
    judged against the mean of 256 full random playouts (on 4096 of the
    positions); and the policy against the uniform-random mover."""
    import torch
    from paper_2506_22609_amd import learn, ludax
    from paper_2506_22609_amd.workloads import init_net_params

    g = ludax.Game(3, 11, 11)
    t0 = time.perf_counter()
    data = learn.collect(g, train_games, seed=seed + 100, id_base=0)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    net = ludax.Net(11, 11, params=torch.from_numpy(init_net_params(seed)).cuda())
    t0 = time.perf_counter()
    losses = learn.train(net, data, steps, batch=4096, lr=1e-3, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    flops_fwd = (27 * 64 * 2 + 3 * 576 * 64 * 2) * 121  # per board, the four convolutions
    lv = losses.cpu()
    del data

    ev = learn.collect(g, 12000, seed=seed + 200, id_base=10**9)
    idx = torch.randperm(len(ev), generator=torch.Generator().manual_seed(seed))[:65536].cuda()
    e = ev.take(idx)
    n = e.board.shape[0]
    base = ludax.State(g, n)
    ludax.init(g, base)
    base.board.copy_(e.board)
    base.to_move.copy_(e.to_move)
    base.ply.copy_((e.board != 0).sum(1).to(torch.int16))
    sub = 4096
    held = ludax.State.from_tensors(g, **{f: getattr(base, f)[:sub].contiguous() for f in ludax.State.FIELDS})
    tr = learn.truth(g, held, 256, seed=seed + 300, id_base=2 * 10**9)

    r = torch.empty((n, 2), dtype=torch.int8, device="cuda")
    t = torch.empty(n, dtype=torch.uint8, device="cuda")

    def plain(s):
        ludax.playout(g, s, seed + 400, 3 * 10**9, stats=None)
        return learn.outcome_p1(s)

    def value_only(s):
        return net.estimate(s)

    def value_one_kernel(s):
        # the value cutoff with no plies: the whole forward in one kernel
        return net.guided_playout(g, s, 0, seed + 600, 5 * 10**9)

    def cutoff(s):
        return learn.cutoff_estimate(g, net, s, 20, seed + 500, 4 * 10**9)

    def guided_unfused(s):
        # 20 plies through memory: forward to logits, then the policy step
        for _ in range(20):
            logits, _ = net.forward(s.board, s.to_move)
            ludax.policy_step(g, s, logits, seed + 600, 5 * 10**9, reward=r, terminal=t)
        return net.estimate(s)

    def guided_step(s):
        # the same plies, each by the forward's kernels with the draw and the
        # ply in the last one (logits on chip)
        for _ in range(20):
            net.guided_step(g, s, seed + 600, 5 * 10**9, reward=r, terminal=t)
        return net.estimate(s)

    def guided_one_kernel(s):
        # the same plies and the value cutoff in one persistent kernel
        return net.guided_playout(g, s, 20, seed + 600, 5 * 10**9)

    out = {"workload": f"hex11x11: training on {train_games} random games, {steps} Adam steps of 4096; "
                       f"{n} held-out positions (error measured on {sub} of them against 256 full random "
                       f"playouts each)",
           "collect_s": t_collect, "train_s": t_train, "train_ms_per_step": t_train / steps * 1e3,
           "train_tflops": 3 * 4096 * flops_fwd / (t_train / steps) / 1e12,
           "value_loss_first_last": [float(lv[:50, 0].mean()), float(lv[-50:, 0].mean())],
           "methods": {}}
    import statistics
    for name, fn in (("plain_full_playout", plain), ("value_only", value_only),
                     ("value_only_one_kernel", value_one_kernel), ("random20_value_cutoff", cutoff), ("policy20_value_cutoff_unfused", guided_unfused),
                     ("policy20_value_cutoff_guided_step", guided_step),
                     ("policy20_value_cutoff_one_kernel", guided_one_kernel)):
        s = base.clone()
        fn(s)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            s = base.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            est = fn(s)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        el = statistics.median(ts)
        mse = ((est[:sub] - tr) ** 2).mean().item()
        out["methods"][name] = {"playouts_per_s": n / el, "ms_per_65536": el * 1e3 * 65536 / n,
                                "mse_vs_256_playout_mean": mse, "timing": "median of 5"}
    # the three policy-guided paths give the same states and estimates bit for bit
    best = max(("policy20_value_cutoff_unfused", "policy20_value_cutoff_guided_step",
                "policy20_value_cutoff_one_kernel"), key=lambda k: out["methods"][k]["playouts_per_s"])
    out["methods"]["policy20_value_cutoff"] = dict(out["methods"][best], path=best)
    # at a fixed value error: the number of averaged full random playouts
    # that matches the value's squared error, measured
    # the faster of the two value paths (three kernels through memory, or
    # the one-kernel forward): the same network, the estimates equal to
    # float32 rounding order
    vpath = max(("value_only", "value_only_one_kernel"), key=lambda k: out["methods"][k]["playouts_per_s"])
    vm = out["methods"][vpath]
    k, mse_k, pps = _averaged_playouts_at_error(g, held, tr, vm["mse_vs_256_playout_mean"], base, seed + 800,
                                                7 * 10**9)
    out["fixed_value_error"] = {"mse": vm["mse_vs_256_playout_mean"], "plain_playouts_averaged": k,
                                "plain_average_mse": mse_k, "plain_positions_per_s": pps,
                                "guided_positions_per_s": vm["playouts_per_s"], "value_path": vpath,
                                "note": "k measured: the smallest number of averaged full random playouts "
                                        "whose squared error is no larger than the value's"}
    # the value forward alone, as a fraction of the bf16 MFMA peak
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        net.forward(base.board, base.to_move)
    e1.record()
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / 5 / 1e3
    out["forward_roofline"] = {"bound": "mfma", "achieved": n * flops_fwd / fwd_s / 1e12, "peak": 2500.0,
                               "unit": "TFLOP/s", "frac": n * flops_fwd / fwd_s / 1e12 / 2500.0,
                               "ms_per_65536": fwd_s * 1e3,
                               "note": "useful conv flops (121 cells, no padding) of the whole forward "
                                       "(encode, 4 conv layers, heads) over its event-timed duration"}
    out["policy_vs_random"] = {}
    for seat in (1, 2):
        w, l, d = learn.play_vs_random(g, net, 4096, seat, seed + 700, 6 * 10**9)
        out["policy_vs_random"][f"net_as_player{seat}"] = {"wins": w, "losses": l, "draws": d,
                                                           "win_rate": w / 4096}
    return out


def _hbm_probe(seed: int):
    """A short fixed sequence for hardware-counter runs (rocprofv3 --pmc):
    one plain device copy of 1 GiB (the known-size reference of the byte
    counters), one headline step (Connect Four and Hex 11x11 playouts of
    65536 envs), one mixed persistent batch (4 x 262144 game ids, equal
    split, one grid), and the per-ply loop over 1,048,576 Hex 19x19 envs (361
    ludax_random_step launches) without and then with the component cache.
    Prints the env-steps of each part, which the counters are divided by."""
    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    out = {}
    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    out["copy_bytes"] = 1 << 30
    for b in W.BENCH_BATCHES:
        g = ludax.Game(b.kind, b.rows, b.cols)
        s = ludax.State(g, b.n)
        ludax.init(g, s)
        _, _, st = ludax.playout(g, s, seed, 0)
        out[b.name] = {"env_steps": int(st[0].item())}
        del s
    # the headline step as bench.py times it: both batches in one launch
    games = [ludax.Game(b.kind, b.rows, b.cols) for b in W.BENCH_BATCHES]
    states = [ludax.State(g, b.n) for g, b in zip(games, W.BENCH_BATCHES)]
    res = ludax.playout_batches([(g, s, 0, None, None, torch.zeros(4, dtype=torch.int64, device="cuda"))
                                 for g, s in zip(games, states)], seed, from_start=True)
    out["group"] = {"env_steps": int(sum(r[2][0].item() for r in res))}
    del states, res
    # the mixed persistent batch (4 x 262144 game ids, equal slot split, one
    # grid): its kernel's instructions per env-step
    mb = W.MIXED4
    mgames = [ludax.Game(k.kind, k.rows, k.cols) for k in mb.kinds]
    mx = ludax.Mixed(mgames)
    mx.slots = [mb.slots // len(mgames) // 64 * 64] * len(mgames)
    mx.one_grid = True
    mres = ludax.MixedResult(mb.n_games, len(mgames))
    mst = torch.zeros((len(mgames), 4), dtype=torch.int64, device="cuda")
    mx.playout(seed, 0, mb.n_games, out=mres, stats=mst)
    torch.cuda.synchronize()
    out["mixed4"] = {"env_steps": int(mst[:, 0].sum().item()), "slots": mx.slots}
    del mx, mres
    b = W.HEX19_1M
    g = ludax.Game(b.kind, b.rows, b.cols)
    for aux in (False, True):
        s = ludax.State(g, b.n, aux=aux)
        r = torch.empty((b.n, 2), dtype=torch.int8, device="cuda")
        t = torch.empty(b.n, dtype=torch.uint8, device="cuda")
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        ludax.init(g, s)
        ludax.state_stats(g, s, -1, st)
        for _ in range(g.max_plies):
            ludax.random_step(g, s, seed, 7 * b.n, reward=r, terminal=t)
        ludax.state_stats(g, s, +1, st)
        torch.cuda.synchronize()
        out[b.name + ("_aux" if aux else "")] = {"env_steps": int(st[0].item()), "launches": g.max_plies}
        del s
        torch.cuda.synchronize()
    print(json.dumps({"hbm_probe": out}), flush=True)


def _net_probe(seed: int):
    """A short fixed sequence of the 11x11 network kernels for counter runs
    (rocprofv3 --pmc): twice the forward over 65536 mid-game Hex positions
    (ludax_net_forward, and ludax_net_guided_playout with no plies), then 5
    training steps at batch 4096 on random-play samples."""
    import torch
    from paper_2506_22609_amd import learn, ludax
    from paper_2506_22609_amd import workloads as W
    from paper_2506_22609_amd.workloads import init_net_params

    g = ludax.Game(W.HEX, 11, 11)
    net = ludax.Net(11, 11, params=torch.from_numpy(init_net_params(seed)).cuda())
    n = 65536
    s = ludax.State(g, n)
    ludax.init(g, s)
    r = torch.empty((n, 2), dtype=torch.int8, device="cuda")
    t = torch.empty(n, dtype=torch.uint8, device="cuda")
    for _ in range(30):
        ludax.random_step(g, s, seed + 2, 0, reward=r, terminal=t)
    for _ in range(2):
        net.forward(s.board, s.to_move)
        net.guided_playout(g, s.clone(), 0, seed + 4, 0)
    data = learn.collect(g, 2000, seed=seed + 3, id_base=0)
    learn.train(net, data, 5, batch=4096)
    torch.cuda.synchronize()
    print(json.dumps({"net_probe": {"positions": n, "train_steps": 5, "batch": 4096}}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-time budget of the CPU oracle baseline (0 = skip)")
    ap.add_argument("--sections", default="mixed,plain_step,large,more_games,learned,large_mixed",
                    help="comma-separated extra sections to run after the headline steps "
                         "(also: sweep, throughput against batch size for the paper's ten games)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed persistent batch section")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--no-plain-step", action="store_true",
                    help="skip the per-ply (ludax_random_step loop) section")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 19x19 large-board section")
    ap.add_argument("--section-reps", type=int, default=3)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned policy/value network section")
    ap.add_argument("--train-games", type=int, default=96000)
    ap.add_argument("--train-steps", type=int, default=2400)
    ap.add_argument("--large-train-steps", type=int, default=1200)
    ap.add_argument("--hbm-budget-gb", type=float, default=16.0,
                    help="HBM held by the network's workspace in the large-board guided estimate")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed steps, one plain device copy of this many MiB "
                         "(a known-size reference for HBM byte counters under a profiler)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="run only the short fixed sequence for hardware-counter runs and print its env-steps")
    ap.add_argument("--net-probe", action="store_true",
                    help="run only a short fixed sequence of the network kernels for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} asked for more): the playouts are independent "
              f"per game, and how the batch would shard over GPUs is described with the design, not run here",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_22609_amd import ludax
    from paper_2506_22609_amd import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.hbm_probe:
        _hbm_probe(args.seed)
        return
    if args.net_probe:
        _net_probe(args.seed)
        return
    batches = W.BENCH_BATCHES
    games = [ludax.Game(b.kind, b.rows, b.cols) for b in batches]
    states = [ludax.State(g, b.n) for g, b in zip(games, batches)]
    rewards = [torch.empty((b.n, 2), dtype=torch.int8, device="cuda") for b in batches]
    terms = [torch.empty(b.n, dtype=torch.uint8, device="cuda") for b in batches]
    stats = [torch.zeros(4, dtype=torch.int64, device="cuda") for _ in batches]
    stream = torch.cuda.current_stream()
    # an event pair costs the stream a few microseconds (10 % of a step), so
    # every EVENT_EVERY-th timed step is bracketed, not every step
    sampled = list(range(0, args.steps, EVENT_EVERY))
    timing = {j: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for j in sampled}

    group = ludax.BatchGroup(list(zip(games, states, rewards, terms, stats)))

    def one_step(k: int, record: bool):
        # both batches reset to the start and played out by one kernel
        # (ludax_playout_batches, from_start), then both batches' counters by
        # one reduction kernel; the events bracket the call, i.e. these two
        # kernels
        ev = timing.get(k - args.warmup) if record else None
        if ev:
            ev[0].record(stream)
        group.run(args.seed, [W.game_id_base(k, b) for b in batches], from_start=True, stream=stream)
        if ev:
            ev[1].record(stream)

    for k in range(args.warmup):
        one_step(k, False)
    torch.cuda.synchronize()
    for st in stats:
        st.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        one_step(k, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    per = {}
    total_steps = 0
    for b, st in zip(batches, stats):
        v = st.cpu().tolist()
        per[b.name] = {"env_steps": v[0], "p1_wins": v[1], "p2_wins": v[2], "draws": v[3]}
        total_steps += v[0]
    value = total_steps / elapsed
    kern_ms = sum(a.elapsed_time(c) for a, c in timing.values()) / len(timing)

    steps_per_launch = total_steps / args.steps
    kern_s = kern_ms / 1e3
    ops_per = VALU_OPS_PER_STEP["group"]
    achieved = ops_per * steps_per_launch / kern_s / 1e12 if ops_per else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS if achieved else None, "traffic": GROUP_TRAFFIC_BYTES,
                "kernel": "k_playout_group (connect4_6x7_n65536 + hex11x11_n65536 in one grid)",
                "kernel_ms": kern_ms,
                "timed": f"events around ludax_playout_batches (k_playout_group and the counters' k_stats_group) "
                         f"in {len(timing)} of the {args.steps} timed steps",
                "ops_per_env_step": ops_per,
                "env_steps_per_launch": steps_per_launch,
                "hbm_frac": GROUP_TRAFFIC_BYTES / kern_s / 1e9 / HBM_PEAK_GBS if GROUP_TRAFFIC_BYTES else None}

    out = {
        "metric": "env-steps/s (plain random playouts, single-game batches)",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic (start positions + Philox4x32-10 seeded uniform-random play)",
        "config": {"workload": " + ".join(b.name for b in batches),
                   "envs_per_batch": batches[0].n, "seed": args.seed, "per_game": per},
        "roofline": roofline,
    }
    out["paper_context"] = PAPER_CONTEXT
    out["protocol"] = _protocol(batches, games, states, rewards, terms)
    out["separate_launches"] = _separate_launches(batches, games, states, rewards, terms, args.seed)
    sec = set(x for x in args.sections.split(",") if x)
    if args.no_mixed:
        sec.discard("mixed")
    if args.no_plain_step:
        sec.discard("plain_step")
    if args.no_large:
        sec -= {"large", "large_mixed"}
    if args.no_learned:
        sec -= {"learned", "large_mixed"}
    if "mixed" in sec:
        out["mixed"] = _mixed_section(args.seed, args.mixed_steps, 1)
    if "sweep" in sec:
        out["sweep"] = _sweep_section(args.seed, args.section_reps)
    if "plain_step" in sec:
        cases = [(b, False) for b in batches] + [(W.HEX11_65536, True)]
        if "large" in sec:
            cases += [(b, False) for b in W.LARGE_BATCHES] + [(W.HEX19_524288, True), (W.HEX19_1M, False),
                                                            (W.HEX19_1M, True)]
        out["plain_step"] = _plain_step_section(cases, args.seed, args.section_reps)
    if "large" in sec:
        out["large"] = _large_section(W.LARGE_BATCHES, args.seed, args.section_reps)
    if "more_games" in sec:
        out["more_games"] = _more_games_section(args.seed, args.section_reps)
    if "learned" in sec:
        out["learned"] = _learned_section(args.seed, args.train_games, args.train_steps)
    if "large_mixed" in sec:
        out["large_mixed"] = _large_mixed_section(args.seed, args.section_reps, args.large_train_steps,
                                                  args.hbm_budget_gb)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = _cpu_baseline(batches, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
