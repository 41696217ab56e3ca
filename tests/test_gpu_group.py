"""GPU parity of ludax_playout_batches: several batches in one launch give
exactly the results of ludax_init (from the start) and ludax_playout per
batch, and the oracle's playouts of the same game ids; games outside the
group kernel take the per-batch path with the same results."""
import numpy as np
import pytest
import torch

from oracle import ref
from tests.gpu_util import assert_same_state, from_device, pair, random_states, to_device

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")

TTT, C4, HEX, REVERSI = ref.TICTACTOE, ref.CONNECT_FOUR, ref.HEX, ref.REVERSI
SIZES = {TTT: (3, 3), C4: (6, 7), HEX: (11, 11), REVERSI: (8, 8)}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _separate(games, states, bases, seed, from_start):
    """The reference call sequence: per batch ludax_init (from_start) and
    ludax_playout with counters."""
    out = []
    for g, s, base in zip(games, states, bases):
        if from_start:
            ludax.init(g, s)
        out.append(ludax.playout(g, s, seed, base))
    return out


def _run_group(games, states, bases, seed, from_start, with_stats=None):
    with_stats = with_stats or [True] * len(games)
    batch = [(g, s, base, None, None, torch.zeros(4, dtype=torch.int64, device="cuda") if w else None)
             for g, s, base, w in zip(games, states, bases, with_stats)]
    return ludax.playout_batches(batch, seed, from_start=from_start)


def _garbage_state(g, n, seed):
    """A state whose every field holds noise: from_start must not read it."""
    d = ludax.State(g, n)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    for f in ludax.State.FIELDS:
        t = getattr(d, f)
        t.copy_(torch.randint(-100, 100, t.shape, generator=gen, device="cuda").to(t.dtype))
    return d


@pytest.mark.parametrize("kinds,ns", [
    ((C4, HEX), (65536, 65536)),
    ((HEX, C4, TTT), (1000, 777, 64)),
    ((TTT, HEX, HEX, C4), (5, 130, 129, 3)),
    ((HEX,), (4097,)),
], ids=["headline", "ragged3", "four", "one"])
def test_group_from_start_equals_init_and_playout(kinds, ns):
    seed = 31
    bases = [10**6 * (k + 1) + 7 for k in range(len(kinds))]
    pairs = [pair(k, *SIZES[k]) for k in kinds]
    dg = [p[1] for p in pairs]
    print(f"group: kinds {kinds} n {ns}", flush=True)
    sep = [ludax.State(g, n) for g, n in zip(dg, ns)]
    ref_out = _separate(dg, sep, bases, seed, True)
    grp = [_garbage_state(g, n, 5 + k) for k, (g, n) in enumerate(zip(dg, ns))]
    out = _run_group(dg, grp, bases, seed, True)
    torch.cuda.synchronize()
    for k in range(len(kinds)):
        assert_same_state(from_device(sep[k]), from_device(grp[k]), f"batch {k}")
        for a, b in zip(ref_out[k], out[k]):
            assert torch.equal(a, b), f"batch {k}"
    # and the oracle's playouts of the same game ids
    for k, (og, _) in enumerate(pairs):
        s = ref.init(og, ns[k])
        rew, term, stats = ref.playout(og, s, seed, bases[k], threads=16)
        assert_same_state(s, from_device(grp[k]), f"oracle batch {k}")
        assert np.array_equal(rew, out[k][0].cpu().numpy())
        assert np.array_equal(stats, out[k][2].cpu().numpy())


@pytest.mark.parametrize("kinds,ns", [((C4, HEX, TTT), (300, 511, 70)), ((HEX, HEX), (64, 1))],
                         ids=["three", "hex2"])
def test_group_from_states_equals_playout(kinds, ns):
    """from_start = 0: mid-game states (some already ended) are played on."""
    seed = 8
    rng = np.random.default_rng(3)
    bases = [5000 * k for k in range(len(kinds))]
    pairs = [pair(k, *SIZES[k]) for k in kinds]
    dg = [p[1] for p in pairs]
    starts = [random_states(og, n, 12, rng) for (og, _), n in zip(pairs, ns)]
    print(f"group from states: kinds {kinds} n {ns}", flush=True)
    sep = [to_device(g, s) for g, s in zip(dg, starts)]
    grp = [to_device(g, s) for g, s in zip(dg, starts)]
    ref_out = _separate(dg, sep, bases, seed, False)
    out = _run_group(dg, grp, bases, seed, False)
    torch.cuda.synchronize()
    for k in range(len(kinds)):
        assert_same_state(from_device(sep[k]), from_device(grp[k]), f"batch {k}")
        for a, b in zip(ref_out[k], out[k]):
            assert torch.equal(a, b), f"batch {k}"
        s = starts[k].subset(np.arange(ns[k]))
        rew, term, stats = ref.playout(pairs[k][0], s, seed, bases[k], threads=16)
        assert_same_state(s, from_device(grp[k]), f"oracle batch {k}")
        assert np.array_equal(stats, out[k][2].cpu().numpy())


def test_group_outside_the_group_kernel_and_empty_batches():
    """Reversi is not in the group kernel: the batches run one after the
    other, with the same results; batches of no envs and batches without
    counters are accepted."""
    seed = 12
    kinds, ns = (REVERSI, HEX, C4), (200, 0, 65)
    bases = [1, 2, 3]
    dg = [pair(k, *SIZES[k])[1] for k in kinds]
    sep = [ludax.State(g, n) for g, n in zip(dg, ns)]
    ref_out = _separate(dg, sep, bases, seed, True)
    grp = [ludax.State(g, n) for g, n in zip(dg, ns)]
    out = _run_group(dg, grp, bases, seed, True, with_stats=[True, True, False])
    torch.cuda.synchronize()
    for k in range(len(kinds)):
        assert_same_state(from_device(sep[k]), from_device(grp[k]), f"batch {k}")
        assert torch.equal(ref_out[k][0], out[k][0]) and torch.equal(ref_out[k][1], out[k][1])
    assert torch.equal(ref_out[0][2], out[0][2]) and out[2][2] is None
    # the grouped path with an empty batch between two others
    grp2 = [ludax.State(g, n) for g, n in zip(dg[1:], ns[1:])]
    out2 = _run_group(dg[1:], grp2, bases[1:], seed, True)
    torch.cuda.synchronize()
    assert_same_state(from_device(sep[2]), from_device(grp2[1]))
    assert torch.equal(ref_out[2][2], out2[1][2]) and int(out2[0][2].abs().sum()) == 0


def test_group_from_start_leaves_hex_aux_on_the_final_boards():
    g = ludax.Game(HEX, 11, 11)
    n = 333
    s = ludax.State(g, n, aux=True)
    s.aux.fill_(0x5A)
    ludax.playout_batches([(g, s, 77, None, None, None)], 4, from_start=True)
    t = s.clone()
    ludax.aux_sync(g, t)
    torch.cuda.synchronize()
    assert torch.equal(s.aux, t.aux)


def test_batch_group_handle_repeats_the_call():
    """ludax.BatchGroup (arguments marshalled once) gives what
    playout_batches gives, call after call with new game ids and counters."""
    kinds, ns = (C4, HEX), (300, 257)
    dg = [pair(k, *SIZES[k])[1] for k in kinds]
    a = [ludax.State(g, n) for g, n in zip(dg, ns)]
    b = [ludax.State(g, n) for g, n in zip(dg, ns)]
    grp = ludax.BatchGroup([(g, s, None, None, None) for g, s in zip(dg, b)])
    for call in range(3):
        bases = [1000 * call + 1, 1000 * call + 2]
        ref_out = _run_group(dg, a, bases, 9, True)
        st = [torch.zeros(4, dtype=torch.int64, device="cuda") for _ in kinds]
        grp.run(9, bases, from_start=True, stats=st)
        torch.cuda.synchronize()
        for k in range(len(kinds)):
            assert_same_state(from_device(a[k]), from_device(b[k]), f"call {call} batch {k}")
            assert torch.equal(ref_out[k][0], grp.outputs[k][0]) and torch.equal(ref_out[k][2], st[k])


def test_batch_group_graph_replay():
    """The whole call (group kernel and counters) captured once and replayed:
    every replay equals the eager call with the same game ids."""
    kinds, ns = (C4, HEX), (1000, 777)
    dg = [pair(k, *SIZES[k])[1] for k in kinds]
    a = [ludax.State(g, n) for g, n in zip(dg, ns)]
    ref_out = _run_group(dg, a, [5, 6], 21, True)
    torch.cuda.synchronize()
    b = [ludax.State(g, n) for g, n in zip(dg, ns)]
    st = [torch.zeros(4, dtype=torch.int64, device="cuda") for _ in kinds]
    grp = ludax.BatchGroup([(g, s, None, None, x) for g, s, x in zip(dg, b, st)])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        grp.run(21, [5, 6], from_start=True, stream=side)  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        grp.run(21, [5, 6], from_start=True)
    for rep in range(3):
        for x in st:
            x.zero_()
        for s in b:
            s.board.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in range(len(kinds)):
            assert_same_state(from_device(a[k]), from_device(b[k]), f"replay {rep} batch {k}")
            assert torch.equal(ref_out[k][2], st[k]), rep
