// ludax_internal.hpp -- types shared by the kernel instantiations and the
// C-ABI host code of the GPU library (not part of the public header).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lx {

struct DevState {
    int8_t *board;
    int8_t *to_move;
    int8_t *status;
    int8_t *winner;
    int8_t *passes;
    int16_t *ply;
    int16_t *last_action;
};

// Kernel entry points of one (game, board size), filled in by the
// instantiation units.
struct GameOps {
    int kind, rows, cols, cells, num_actions;
    hipError_t (*init)(const DevState &, int64_t, hipStream_t);
    hipError_t (*mask)(const DevState &, int64_t, uint8_t *, hipStream_t);
    hipError_t (*step)(const DevState &, int64_t, int, const int32_t *, int8_t *, uint8_t *, uint8_t *,
                       hipStream_t);
    hipError_t (*playout)(const DevState &, int64_t, int, uint64_t, int64_t, const int64_t *, int8_t *,
                          uint8_t *, int64_t *, hipStream_t);
};

// Step and outcome counters: stats[0..3] += sign * (sum of ply, number of
// TERMINAL envs won by player 1, by player 2, drawn) over the n envs.
hipError_t launch_stats(const DevState &st, int64_t n, int sign, int64_t *stats, hipStream_t s);

// Lookup per game kind; NULL when the size is not supported.
const GameOps *ops_tictactoe(int rows, int cols);
const GameOps *ops_connect_four(int rows, int cols);
const GameOps *ops_hex(int rows, int cols);
const GameOps *ops_reversi(int rows, int cols);
const GameOps *ops_gomoku(int rows, int cols);

} // namespace lx
