"""GPU parity of the mixed persistent batch: every game's winner, length
and last action against the oracle playing that game id alone (kind =
id mod number of kinds), with slot counts small enough that every lane
plays many games (refill), ragged batch sizes and id bases, truncation,
and a captured-graph replay."""
import numpy as np
import pytest
import torch

from oracle import ref

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")

MIX4 = [(ref.REVERSI, 8, 8), (ref.GOMOKU, 15, 15), (ref.HEX, 11, 11), (ref.CONNECT_FOUR, 6, 7)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_batch(kinds, seed, id_base, n_games, max_plies=0):
    """Play every game id on the oracle; returns winner, plies, last, stats."""
    n = len(kinds)
    winner = np.zeros(n_games, np.int8)
    plies = np.zeros(n_games, np.int16)
    last = np.zeros(n_games, np.int16)
    stats = np.zeros((n, 4), np.int64)
    for k, (kind, r, c) in enumerate(kinds):
        g = ref.Game(kind, r, c, max_plies)
        j = np.array([x for x in range(n_games) if (id_base + x) % n == k], np.int64)
        if j.size == 0:
            continue
        s = ref.init(g, j.size)
        _, _, st = ref.playout(g, s, seed, 0, game_id=id_base + j, threads=16)
        winner[j] = np.where(s.status == ref.TERMINAL, s.winner, -1)
        plies[j] = s.ply
        last[j] = s.last_action
        stats[k] = st
    return winner, plies, last, stats


def run_mixed(kinds, seed, id_base, n_games, slots, max_plies=0, one_grid=None):
    games = [ludax.Game(kind, r, c, max_plies) for kind, r, c in kinds]
    m = ludax.Mixed(games)
    m.slots = slots
    if one_grid is not None:
        m.one_grid = one_grid
    out, stats = m.playout(seed, id_base, n_games)
    torch.cuda.synchronize()
    return out, stats, (m, games)


@pytest.mark.parametrize("one_grid", [True, False], ids=["one_grid", "streams"])
@pytest.mark.parametrize("id_base,n_games,slots", [
    (0, 4096, [128, 128, 64, 64]),
    (7, 3001, [64, 192, 128, 256]),
    (1 << 40, 777, [4096, 4096, 4096, 4096]),
])
def test_mixed_matches_oracle(id_base, n_games, slots, one_grid):
    out, stats, (m, _) = run_mixed(MIX4, 3, id_base, n_games, slots, one_grid=one_grid)
    assert m.one_grid == one_grid
    w, p, l, st = oracle_batch(MIX4, 3, id_base, n_games)
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)
    assert np.array_equal(out.last_action.cpu().numpy(), l)
    assert np.array_equal(stats.cpu().numpy(), st)


def test_mixed_other_kinds_and_truncation():
    """Kinds outside the one-grid kernel: a kernel per kind, and asking for
    one grid is refused."""
    kinds = [(ref.TICTACTOE, 3, 3), (ref.HEX, 5, 5), (ref.GOMOKU, 7, 7)]
    out, stats, (m, _) = run_mixed(kinds, 11, 5, 2000, [64, 128, 64], max_plies=20)
    assert not m.one_grid
    with pytest.raises(ludax.LudaxError):
        m.one_grid = True
    w, p, l, st = oracle_batch(kinds, 11, 5, 2000, max_plies=20)
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)
    assert np.array_equal(out.last_action.cpu().numpy(), l)
    assert np.array_equal(stats.cpu().numpy(), st)
    assert (w == -1).any()  # some games were truncated


def test_mixed_single_kind_equals_plain_playout():
    g = ludax.Game(ref.GOMOKU, 15, 15)
    m = ludax.Mixed([g])
    m.slots = [256]
    out, stats = m.playout(2, 100, 1500)
    d = ludax.State(g, 1500)
    ludax.init(g, d)
    _, _, pst = ludax.playout(g, d, 2, 100)
    w = torch.where(d.status == ref.TERMINAL, d.winner, torch.full_like(d.winner, -1))
    assert torch.equal(out.winner, w) and torch.equal(out.plies, d.ply)
    assert torch.equal(out.last_action, d.last_action)
    assert torch.equal(stats[0], pst)


@pytest.mark.parametrize("kind", [ref.HEX, ref.GOMOKU], ids=["hex19", "gomoku19"])
def test_mixed_single_kind_large_equals_plain_playout(kind):
    """The one-kind persistent batch as the large-board benchmark launches it
    (524288 games of a 19x19 game through 262144 refilled slots) gives every
    game the outcome, length and last action of the plain fused playout."""
    g = ludax.Game(kind, 19, 19)
    n = 524288
    m = ludax.Mixed([g])
    m.slots = [262144]
    out, stats = m.playout(5, 7 * n, n)
    d = ludax.State(g, n)
    ludax.init(g, d)
    _, _, pst = ludax.playout(g, d, 5, 7 * n)
    w = torch.where(d.status == ref.TERMINAL, d.winner, torch.full_like(d.winner, -1))
    assert torch.equal(out.winner, w) and torch.equal(out.plies, d.ply)
    assert torch.equal(out.last_action, d.last_action)
    assert torch.equal(stats[0], pst)


@pytest.mark.parametrize("one_grid", [True, False], ids=["one_grid", "streams"])
def test_mixed_graph_replay(one_grid):
    """The whole call (counter reset, the kinds' kernels -- one grid, or
    forked to the kinds' streams and joined -- and the counters) captured
    once and replayed; every replay equals the eager result."""
    games = [ludax.Game(kind, r, c) for kind, r, c in MIX4]
    m = ludax.Mixed(games)
    m.slots = [256, 256, 128, 128]
    m.one_grid = one_grid
    n = 2048
    ref_out, ref_stats = m.playout(9, 0, n)
    torch.cuda.synchronize()
    out = ludax.MixedResult(n, 4)
    stats = torch.zeros((4, 4), dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        m.playout(9, 0, n, out=out, stats=stats)  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.playout(9, 0, n, out=out, stats=stats)
    for rep in range(3):
        stats.zero_()
        out.winner.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.winner, ref_out.winner), rep
        assert torch.equal(out.plies, ref_out.plies), rep
        assert torch.equal(out.last_action, ref_out.last_action), rep
        assert torch.equal(stats, ref_stats), rep


def test_mixed_autotune_keeps_results():
    games = [ludax.Game(kind, r, c) for kind, r, c in MIX4]
    m = ludax.Mixed(games)
    n = 8192
    ms = m.autotune(5, 0, n, 4096)
    assert ms > 0
    sl = m.slots
    assert all(s % 64 == 0 and s >= 64 for s in sl)
    out, stats = m.playout(5, 0, n)
    w, p, l, st = oracle_batch(MIX4, 5, 0, n)
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)


def test_mixed_large_boards_match_oracle():
    """Hex 19x19 and Gomoku 19x19 in one mixed batch (the large-board
    configuration at a size the oracle replays quickly)."""
    kinds = [(ref.HEX, 19, 19), (ref.GOMOKU, 19, 19)]
    out, stats, _ = run_mixed(kinds, 19, 3, 1200, [128, 192])
    w, p, l, st = oracle_batch(kinds, 19, 3, 1200)
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)
    assert np.array_equal(out.last_action.cpu().numpy(), l)
    assert np.array_equal(stats.cpu().numpy(), st)


def test_mixed_with_yavalath_matches_oracle():
    kinds = [(ref.YAVALATH, 9, 9), (ref.HEX, 11, 11), (ref.YAVALATH, 7, 7)]
    out, stats, _ = run_mixed(kinds, 23, 11, 2500, [64, 128, 64])
    w, p, l, st = oracle_batch(kinds, 23, 11, 2500)
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)
    assert np.array_equal(out.last_action.cpu().numpy(), l)
    assert np.array_equal(stats.cpu().numpy(), st)


def test_mixed_with_pente_matches_oracle():
    kinds = [(ref.PENTE, 19, 19), (ref.GOMOKU, 19, 19), (ref.PENTE, 7, 7)]
    out, stats, _ = run_mixed(kinds, 29, 5, 1500, [128, 64, 64])
    w, p, l, st = oracle_batch(kinds, 29, 5, 1500)
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)
    assert np.array_equal(out.last_action.cpu().numpy(), l)
    assert np.array_equal(stats.cpu().numpy(), st)


def test_mixed_with_movement_games_matches_oracle():
    """Wolf and Sheep, English Draughts and Dai Hasami Shogi (Draughts and
    Dai Hasami Shogi games cut at 200 plies report winner -1) beside Hex,
    with few slots so that every lane plays several games."""
    kinds = [(ref.DRAUGHTS, 8, 8), (ref.WOLF_SHEEP, 8, 8), (ref.HASAMI_SHOGI, 9, 9), (ref.HEX, 11, 11)]
    out, stats, _ = run_mixed(kinds, 31, 9, 2201, [128, 64, 128, 64])
    w, p, l, st = oracle_batch(kinds, 31, 9, 2201)
    assert (w == -1).any()
    assert np.array_equal(out.winner.cpu().numpy(), w)
    assert np.array_equal(out.plies.cpu().numpy(), p)
    assert np.array_equal(out.last_action.cpu().numpy(), l)
    assert np.array_equal(stats.cpu().numpy(), st)
