// capi.cpp -- the extern "C" boundary of the GPU library (include/ludax.h).
//
// Host-side argument checks, then one kernel launch per call on the
// caller's stream.  Nothing here allocates device memory, frees it, or
// synchronises a stream.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>

#include "ludax.h"
#include "ludax_internal.hpp"

namespace lx {
const GameOps *ops_hex_a(int);
const GameOps *ops_hex_b(int);
const GameOps *ops_hex_c(int);
const GameOps *ops_hex_d(int);
const GameOps *ops_hex_e(int);
const GameOps *ops_gomoku_a(int);
const GameOps *ops_gomoku_b(int);
const GameOps *ops_gomoku_c(int);
const GameOps *ops_gomoku_d(int);
const GameOps *ops_gomoku_e(int);

const GameOps *ops_hex(int rows, int cols)
{
    if (rows != cols) return nullptr;
    const GameOps *(*parts[])(int) = {ops_hex_a, ops_hex_b, ops_hex_c, ops_hex_d, ops_hex_e};
    for (auto p : parts)
        if (const GameOps *o = p(rows)) return o;
    return nullptr;
}

const GameOps *ops_gomoku(int rows, int cols)
{
    if (rows != cols) return nullptr;
    const GameOps *(*parts[])(int) = {ops_gomoku_a, ops_gomoku_b, ops_gomoku_c, ops_gomoku_d,
                                      ops_gomoku_e};
    for (auto p : parts)
        if (const GameOps *o = p(rows)) return o;
    return nullptr;
}
} // namespace lx

struct ludax_game {
    ludax_game_desc desc;
    int32_t cells, num_actions, max_plies;
    const lx::GameOps *ops;
};

namespace {

thread_local char g_device_error[256] = "";

constexpr int64_t MAX_ENVS = 2147483647LL;

int device_error(hipError_t e)
{
    if (e == hipSuccess) return LUDAX_OK;
    std::snprintf(g_device_error, sizeof g_device_error, "%s (%d)", hipGetErrorString(e), (int)e);
    return LUDAX_E_DEVICE;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Common checks of a state argument; fills the device view.
int check_state(const ludax_state *s, lx::DevState *d)
{
    if (s == nullptr || s->board == nullptr || s->to_move == nullptr || s->status == nullptr ||
        s->winner == nullptr || s->passes == nullptr || s->ply == nullptr || s->last_action == nullptr)
        return LUDAX_E_INVALID;
    if (!aligned16(s->board)) return LUDAX_E_INVALID;
    d->board = s->board;
    d->to_move = s->to_move;
    d->status = s->status;
    d->winner = s->winner;
    d->passes = s->passes;
    d->ply = s->ply;
    d->last_action = s->last_action;
    return LUDAX_OK;
}

int natural_bound(int kind, int cells)
{
    // Reversi: 60 placements, at most 59 single passes between them, and
    // the two final passes.  Other games: one stone per ply, never removed.
    return kind == LUDAX_REVERSI ? (cells - 4) + (cells - 5) + 2 : cells;
}

} // namespace

extern "C" {

int ludax_game_create(const ludax_game_desc *desc, ludax_game **out)
{
    if (desc == nullptr || out == nullptr) return LUDAX_E_INVALID;
    *out = nullptr;
    if (desc->rows <= 0 || desc->cols <= 0 || desc->max_plies < 0 || desc->max_plies > 32767)
        return LUDAX_E_INVALID;
    const lx::GameOps *ops = nullptr;
    switch (desc->kind) {
    case LUDAX_TICTACTOE: ops = lx::ops_tictactoe(desc->rows, desc->cols); break;
    case LUDAX_CONNECT_FOUR: ops = lx::ops_connect_four(desc->rows, desc->cols); break;
    case LUDAX_HEX: ops = lx::ops_hex(desc->rows, desc->cols); break;
    case LUDAX_REVERSI: ops = lx::ops_reversi(desc->rows, desc->cols); break;
    case LUDAX_GOMOKU: ops = lx::ops_gomoku(desc->rows, desc->cols); break;
    default: return LUDAX_E_UNSUPPORTED;
    }
    if (ops == nullptr) return LUDAX_E_UNSUPPORTED;
    ludax_game *g = new (std::nothrow) ludax_game;
    if (g == nullptr) return LUDAX_E_INVALID;
    g->desc = *desc;
    g->cells = ops->cells;
    g->num_actions = ops->num_actions;
    g->max_plies = desc->max_plies ? desc->max_plies : natural_bound(desc->kind, ops->cells);
    g->ops = ops;
    *out = g;
    return LUDAX_OK;
}

int ludax_game_destroy(ludax_game *game)
{
    if (game == nullptr) return LUDAX_E_INVALID;
    delete game;
    return LUDAX_OK;
}

int ludax_game_info(const ludax_game *game, int32_t *cells, int32_t *num_actions, int32_t *aux_bytes,
                    int32_t *max_plies)
{
    if (game == nullptr) return LUDAX_E_INVALID;
    if (cells) *cells = game->cells;
    if (num_actions) *num_actions = game->num_actions;
    if (aux_bytes) *aux_bytes = 0;
    if (max_plies) *max_plies = game->max_plies;
    return LUDAX_OK;
}

int ludax_init(const ludax_game *game, ludax_state *state, int64_t n, hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    return device_error(game->ops->init(d, n, stream));
}

int ludax_legal_mask(const ludax_game *game, const ludax_state *state, uint8_t *mask, int64_t n,
                     hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (mask == nullptr || !aligned16(mask)) return LUDAX_E_INVALID;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    return device_error(game->ops->mask(d, n, mask, stream));
}

int ludax_step(const ludax_game *game, ludax_state *state, const int32_t *action, int8_t *reward,
               uint8_t *terminal, uint8_t *next_mask, int64_t n, hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (action == nullptr || reward == nullptr || terminal == nullptr ||
        (next_mask != nullptr && !aligned16(next_mask)))
        return LUDAX_E_INVALID;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    return device_error(
        game->ops->step(d, n, game->max_plies, action, reward, terminal, next_mask, stream));
}

int ludax_playout(const ludax_game *game, ludax_state *state, uint64_t seed, int64_t game_id_base,
                  const int64_t *game_id, int8_t *reward, uint8_t *terminal, int64_t *stats, int64_t n,
                  hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (reward == nullptr || terminal == nullptr) return LUDAX_E_INVALID;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    return device_error(game->ops->playout(d, n, game->max_plies, seed, game_id_base, game_id, reward,
                                           terminal, stats, stream));
}

int ludax_state_stats(const ludax_game *game, const ludax_state *state, int32_t sign, int64_t *stats,
                      int64_t n, hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS || (sign != 1 && sign != -1)) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (stats == nullptr) return LUDAX_E_INVALID;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    return device_error(lx::launch_stats(d, n, sign, stats, stream));
}

const char *ludax_strerror(int code)
{
    switch (code) {
    case LUDAX_OK: return "ok";
    case LUDAX_E_INVALID: return "invalid argument";
    case LUDAX_E_UNSUPPORTED: return "unsupported game or board size";
    case LUDAX_E_DEVICE: return "HIP device error";
    default: return "unknown error code";
    }
}

const char *ludax_last_device_error(void) { return g_device_error; }

} // extern "C"
