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
    uint8_t *aux; // the game's per-env cache (Hex: hexaux.hpp), or NULL
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

// A batch group (k_playout_group): batch k of nb is served by blocks
// [first_block[k], first_block[k + 1]) and played with the group kernel's
// game slot[k]; game id of env i = gid_base[k] + i.
constexpr int GROUP_MAX = 4;

struct GroupArgs {
    DevState st[GROUP_MAX];
    int64_t n[GROUP_MAX];
    int64_t gid_base[GROUP_MAX];
    int8_t *reward[GROUP_MAX];
    uint8_t *terminal[GROUP_MAX];
    int32_t max_plies[GROUP_MAX];
    int32_t slot[GROUP_MAX];
    int32_t first_block[GROUP_MAX + 1];
    int32_t nb;
    uint32_t key0, key1;
};

// from_start: the envs are reset to the start position inside the kernel
hipError_t launch_playout_group(const GroupArgs &a, bool from_start, hipStream_t s);

// A mixed batch in one grid (k_persist_group): kind k of n runs on blocks
// [first_block[k], first_block[k + 1]) with the one-grid kernel's game
// slot[k] and its arguments k[k].
constexpr int MIXED_MAX = 8;

struct MixedGroupArgs {
    MixedArgs k[MIXED_MAX];
    int32_t slot[MIXED_MAX];
    int32_t first_block[MIXED_MAX + 1];
    int32_t n;
};

hipError_t launch_mixed_group(const MixedGroupArgs &a, hipStream_t s);

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
    hipError_t (*policy_step)(const DevState &, int64_t, int, const float *, uint64_t, int64_t, const int64_t *,
                              int8_t *, uint8_t *, hipStream_t);
    hipError_t (*playout)(const DevState &, int64_t, int, uint64_t, int64_t, const int64_t *, int8_t *,
                          uint8_t *, int64_t *, hipStream_t);
    hipError_t (*persist)(const MixedArgs &, int, hipStream_t); // NULL: no mixed batches of this game
    int aux_bytes;                                               // per-env cache size (0: no cache)
    hipError_t (*aux_sync)(const DevState &, int64_t, hipStream_t); // NULL when aux_bytes == 0
    int group_slot; // index in the batch-group kernel's game list, -1 if not in it
    int mixed_slot; // index in the one-grid mixed kernel's game list, -1 if not in it
};

hipError_t launch_zero_counters(unsigned int *c, int n, hipStream_t s);
hipError_t launch_mixed_stats(const int8_t *winner, const int16_t *plies, int64_t n_games, int64_t id_base,
                              int n_kinds, int64_t *stats, hipStream_t s);

// Step and outcome counters: stats[0..3] += sign * (sum of ply, number of
// TERMINAL envs won by player 1, by player 2, drawn) over the n envs.
hipError_t launch_stats(const DevState &st, int64_t n, int sign, int64_t *stats, hipStream_t s);
// the same for nb <= GROUP_MAX batches in one launch: stats[k] gets batch
// k's counters (batches with stats[k] NULL or n[k] = 0 are skipped)
hipError_t launch_stats_group(const DevState *st, const int64_t *n, int nb, int sign, int64_t *const *stats,
                              hipStream_t s);

// The policy/value network (net.hip); N = board side, 11 or 19.
int64_t net_n_params();
int64_t net_packed_bytes();
bool net_size_supported(int N);
int64_t net_forward_ws_bytes(int N, int64_t n);
int64_t net_train_ws_bytes(int N, int64_t n);
hipError_t net_pack(const float *params, void *packed, hipStream_t s);
hipError_t net_forward(int N, const float *params, const void *packed, const int8_t *board, const int8_t *to_move,
                       int64_t n, float *logits, float *value, void *ws, hipStream_t s);
hipError_t net_loss_grad(int N, const float *params, const void *packed, const int8_t *board,
                         const int8_t *to_move, const int16_t *action, const float *z, int64_t n, float beta,
                         float *loss, float *grads, void *ws, hipStream_t s);
// estimate [n] = outcome for player 1 (TERMINAL), +-value (RUNNING), 0 else;
// workspace: forward size plus n * (N * N + 1) floats
hipError_t net_estimate(int N, const float *params, const void *packed, const DevState &st, int64_t n,
                        float *estimate, void *ws, hipStream_t s);
// one guided ply (forward, policy draw from the logits on chip, step) of
// every env; N = 11, kind = Hex or Gomoku
hipError_t net_guided_step(int N, const float *params, const void *packed, const DevState &st, int kind, int64_t n,
                           int max_plies, uint64_t seed, int64_t gid_base, const int64_t *gid, int8_t *reward,
                           uint8_t *terminal, void *ws, hipStream_t s);
// `plies` guided plies of every env (11x11, Hex or Gomoku) in one kernel,
// then estimate [n] as net_estimate gives it; no workspace
hipError_t net_guided_playout(const float *params, const void *packed, const DevState &st, int kind, int64_t n,
                              int max_plies, int plies, uint64_t seed, int64_t gid_base, const int64_t *gid,
                              float *estimate, hipStream_t s);
hipError_t net_adam(float *params, const float *grads, float *m, float *v, int step, float lr, float b1, float b2,
                    float eps, void *packed, hipStream_t s);

// Lookup per game kind; NULL when the size is not supported.
const GameOps *ops_tictactoe(int rows, int cols);
const GameOps *ops_connect_four(int rows, int cols);
const GameOps *ops_hex(int rows, int cols);
const GameOps *ops_reversi(int rows, int cols);
const GameOps *ops_gomoku(int rows, int cols);
const GameOps *ops_yavalath(int rows, int cols);
const GameOps *ops_pente(int rows, int cols);
const GameOps *ops_wolf_sheep(int rows, int cols);
const GameOps *ops_draughts(int rows, int cols);
const GameOps *ops_hasami_shogi(int rows, int cols);

} // namespace lx
