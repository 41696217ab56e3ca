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

// One game kind of a mixed persistent batch (see k_persist_ply /
// k_persist_fill): its games are the global indices j0 + i * stride for
// i < count, game j has id id_base + j; results go to index j.
struct MixedArgs {
    int64_t id_base, j0, count, stride;
    int32_t max_plies;
    uint32_t key0, key1;
    int8_t *winner;
    int16_t *plies, *last;
    unsigned int *counter;
};

// Kernel entry points of one (game, board size), filled in by the
// instantiation units.
struct GameOps {
    int kind, rows, cols, cells, num_actions;
    hipError_t (*init)(const DevState &, int64_t, hipStream_t);
    hipError_t (*mask)(const DevState &, int64_t, uint8_t *, hipStream_t);
    hipError_t (*step)(const DevState &, int64_t, int, const int32_t *, int8_t *, uint8_t *, uint8_t *,
                       hipStream_t);
    hipError_t (*random_step)(const DevState &, int64_t, int, uint64_t, int64_t, const int64_t *, int8_t *,
                              uint8_t *, hipStream_t);
    hipError_t (*playout)(const DevState &, int64_t, int, uint64_t, int64_t, const int64_t *, int8_t *,
                          uint8_t *, int64_t *, hipStream_t);
    hipError_t (*persist)(const MixedArgs &, int, hipStream_t);
};

hipError_t launch_zero_counters(unsigned int *c, int n, hipStream_t s);
hipError_t launch_mixed_stats(const int8_t *winner, const int16_t *plies, int64_t n_games, int64_t id_base,
                              int n_kinds, int64_t *stats, hipStream_t s);

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
