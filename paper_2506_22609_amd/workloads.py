"""Seeded synthetic workloads: which games, batch sizes, seeds and game-id
ranges the tests and the benchmark run.  Holds no rule or sampling
arithmetic; both the GPU library and the CPU oracle take these as inputs.

The paper benchmarks its own rule sets under a uniformly random policy
(Sec. 6); no dataset is involved, so every input is a start position plus
(seed, game id) pairs.
"""
from dataclasses import dataclass

TICTACTOE, CONNECT_FOUR, HEX, REVERSI, GOMOKU, YAVALATH, PENTE, WOLF_SHEEP, DRAUGHTS, HASAMI_SHOGI = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10

SEEDS = (1, 2, 3)


@dataclass(frozen=True)
class Batch:
    name: str
    kind: int
    rows: int
    cols: int
    n: int


# 1024 Tic-Tac-Toe playouts (the small case the oracle finishes at once)
TTT_1024 = Batch("tictactoe3x3_n1024", TICTACTOE, 3, 3, 1024)
# single-game batches of 65536 envs: Connect Four 6x7 and Hex 11x11
C4_65536 = Batch("connect4_6x7_n65536", CONNECT_FOUR, 6, 7, 65536)
HEX11_65536 = Batch("hex11x11_n65536", HEX, 11, 11, 65536)
# the other rule sets at the same batch size (mixed-batch members)
REVERSI_65536 = Batch("reversi8x8_n65536", REVERSI, 8, 8, 65536)
GOMOKU15_65536 = Batch("gomoku15x15_n65536", GOMOKU, 15, 15, 65536)

BENCH_BATCHES = (C4_65536, HEX11_65536)
# the other placement games of the paper's benchmark list: Yavalath on the
# hexagon of diameter 9 (61 cells), Pente 19x19
YAVALATH9_65536 = Batch("yavalath9_n65536", YAVALATH, 9, 9, 65536)
PENTE19_65536 = Batch("pente19x19_n65536", PENTE, 19, 19, 65536)
# and the movement games: step and hop on the 8x8 board, slide and hop on 9x9
WOLF_SHEEP_65536 = Batch("wolf_sheep8x8_n65536", WOLF_SHEEP, 8, 8, 65536)
DRAUGHTS_65536 = Batch("draughts8x8_n65536", DRAUGHTS, 8, 8, 65536)
HASAMI_SHOGI_65536 = Batch("hasami_shogi9x9_n65536", HASAMI_SHOGI, 9, 9, 65536)
MORE_GAMES = (YAVALATH9_65536, PENTE19_65536, WOLF_SHEEP_65536, DRAUGHTS_65536, HASAMI_SHOGI_65536)

# the batch-size sweep of the paper's throughput figure (Sec. 6, Fig. 2:
# moves per second against batch size under uniform-random play): its ten
# games at batch sizes 2^10 .. 2^20
SWEEP_GAMES = (Batch("tictactoe3x3", TICTACTOE, 3, 3, 0), Batch("connect4_6x7", CONNECT_FOUR, 6, 7, 0),
               Batch("hex11x11", HEX, 11, 11, 0), Batch("reversi8x8", REVERSI, 8, 8, 0),
               Batch("gomoku15x15", GOMOKU, 15, 15, 0), Batch("yavalath9", YAVALATH, 9, 9, 0),
               Batch("pente19x19", PENTE, 19, 19, 0), Batch("wolf_sheep8x8", WOLF_SHEEP, 8, 8, 0),
               Batch("draughts8x8", DRAUGHTS, 8, 8, 0), Batch("hasami_shogi9x9", HASAMI_SHOGI, 9, 9, 0))
SWEEP_SIZES = (1024, 4096, 16384, 65536, 262144, 1048576)

# large boards: Hex 19x19 and Gomoku 19x19, 524288 envs each (1,048,576
# envs, 378.5 MB of int8 boards)
HEX19_524288 = Batch("hex19x19_n524288", HEX, 19, 19, 524288)
GOMOKU19_524288 = Batch("gomoku19x19_n524288", GOMOKU, 19, 19, 524288)
LARGE_BATCHES = (HEX19_524288, GOMOKU19_524288)
# the per-ply step's state above the 256 MB Infinity Cache: 1,048,576 Hex
# 19x19 envs (378.5 MB of boards), so every ply streams the boards from HBM
HEX19_1M = Batch("hex19x19_n1048576", HEX, 19, 19, 1048576)


def game_id_base(step: int, batch: Batch) -> int:
    """Distinct game ids per benchmark step: step * n."""
    return step * batch.n


@dataclass(frozen=True)
class MixedBatch:
    name: str
    kinds: tuple
    n_games: int
    slots: int


# the mixed persistent batch: 4 x 262144 game ids, kind = id mod 4
# (Reversi, Gomoku 15x15, Hex 11x11, Connect Four), 262144 slots
MIXED4 = MixedBatch("mixed4_n1048576_slots262144",
                    (Batch("reversi8x8", REVERSI, 8, 8, 0), Batch("gomoku15x15", GOMOKU, 15, 15, 0),
                     Batch("hex11x11", HEX, 11, 11, 0), Batch("connect4_6x7", CONNECT_FOUR, 6, 7, 0)),
                    4 * 262144, 262144)


# ---------------------------------------------------------------------------
# the policy/value network: seeded initial parameters and the training set
# ---------------------------------------------------------------------------
NET_CHANNELS = 64
NET_LAYERS = 4


def net_param_shapes():
    """Flat parameter order: W1 [64][3][3][3], b1, W2..W4 [64][64][3][3]
    with their biases, wp [64], bp [1], wv [64], bv [1]."""
    C = NET_CHANNELS
    shapes = [(C, 3, 3, 3), (C,)]
    for _ in range(NET_LAYERS - 1):
        shapes += [(C, C, 3, 3), (C,)]
    return shapes + [(C,), (1,), (C,), (1,)]


def init_net_params(seed: int):
    """He-uniform conv weights (bound sqrt(6 / fan_in)), small positive conv
    biases, small uniform head weights, zero head biases; float32."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for shape in net_param_shapes():
        if len(shape) == 4:
            a = float(np.sqrt(6.0 / (shape[1] * 9)))
            parts.append(rng.uniform(-a, a, shape))
        elif shape == (NET_CHANNELS,) and len(parts) < 2 * NET_LAYERS:
            parts.append(np.full(shape, 0.01))
        elif shape == (NET_CHANNELS,):
            parts.append(rng.uniform(-0.125, 0.125, shape))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
