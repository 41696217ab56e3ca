// capi.cpp -- the extern "C" boundary of the GPU library (include/ludax.h).
//
// Host-side argument checks, then one kernel launch per call on the
// caller's stream.  Nothing here allocates device memory, frees it, or
// synchronises a stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

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

// Common checks of a state argument; fills the device view.  aux is kept
// only for a game with a per-env cache (aux_bytes > 0), and must then be
// 128-byte aligned (each env's row starts a cache line).
int check_state(const ludax_state *s, lx::DevState *d, int aux_bytes = 0)
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
    d->aux = aux_bytes > 0 ? static_cast<uint8_t *>(s->aux) : nullptr;
    if (d->aux != nullptr && (reinterpret_cast<uintptr_t>(d->aux) & 127u) != 0) return LUDAX_E_INVALID;
    return LUDAX_OK;
}

int natural_bound(int kind, int cells)
{
    // Reversi: 60 placements, at most 59 single passes between them, and
    // the two final passes.  Other games: one stone per ply, never removed.
    // Pente: a capture frees two cells, and after 16 removed stones somebody
    // has captured 10 and won, so the board is full by cells + 16 plies.
    // Wolf and Sheep: every other ply moves one of the four sheep a row up,
    // at most 7 rows each.  Draughts and Dai Hasami Shogi have no natural
    // end (pieces can move back and forth): the 200-ply cap for unbounded
    // games.
    if (kind == LUDAX_PENTE) return cells + 16;
    if (kind == LUDAX_WOLF_SHEEP) return 2 * 4 * 7;
    if (kind == LUDAX_DRAUGHTS || kind == LUDAX_HASAMI_SHOGI) return 200;
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
    case LUDAX_YAVALATH: ops = lx::ops_yavalath(desc->rows, desc->cols); break;
    case LUDAX_PENTE: ops = lx::ops_pente(desc->rows, desc->cols); break;
    case LUDAX_WOLF_SHEEP: ops = lx::ops_wolf_sheep(desc->rows, desc->cols); break;
    case LUDAX_DRAUGHTS: ops = lx::ops_draughts(desc->rows, desc->cols); break;
    case LUDAX_HASAMI_SHOGI: ops = lx::ops_hasami_shogi(desc->rows, desc->cols); break;
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
    if (aux_bytes) *aux_bytes = game->ops->aux_bytes;
    if (max_plies) *max_plies = game->max_plies;
    return LUDAX_OK;
}

int ludax_init(const ludax_game *game, ludax_state *state, int64_t n, hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    lx::DevState d;
    int rc = check_state(state, &d, game->ops->aux_bytes);
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
    int rc = check_state(state, &d, game->ops->aux_bytes);
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

int ludax_playout_batches(const ludax_batch *batches, int32_t n_batches, uint64_t seed, int32_t from_start,
                          hipStream_t stream)
{
    constexpr int NB = lx::GROUP_MAX;
    if (batches == nullptr || n_batches < 1 || n_batches > NB) return LUDAX_E_INVALID;
    lx::DevState d[NB], daux[NB];
    int64_t total = 0;
    bool grouped = true;
    for (int k = 0; k < n_batches; ++k) {
        const ludax_batch &b = batches[k];
        if (b.game == nullptr || b.n < 0 || b.n > MAX_ENVS) return LUDAX_E_INVALID;
        total += b.n;
        if (b.n == 0) continue;
        if (b.reward == nullptr || b.terminal == nullptr) return LUDAX_E_INVALID;
        int rc = check_state(b.state, &d[k]);
        if (rc == LUDAX_OK) rc = check_state(b.state, &daux[k], b.game->ops->aux_bytes);
        if (rc) return rc;
        if (b.game->ops->group_slot < 0) grouped = false;
    }
    if (total > MAX_ENVS) return LUDAX_E_INVALID; // one grid of at most 2^31 threads
    if (total == 0) return LUDAX_OK;
    hipError_t e = hipSuccess;
    if (!grouped) {
        // a game outside the group kernel: the batches one after another
        for (int k = 0; k < n_batches && e == hipSuccess; ++k) {
            const ludax_batch &b = batches[k];
            if (b.n == 0) continue;
            if (from_start) e = b.game->ops->init(daux[k], b.n, stream);
            if (e == hipSuccess)
                e = b.game->ops->playout(d[k], b.n, b.game->max_plies, seed, b.game_id_base, nullptr, b.reward,
                                         b.terminal, b.stats, stream);
        }
        return device_error(e);
    }
    // the longest-running games' blocks first (cells as the measure), so
    // that the shorter batches' waves fill in beside them
    int order[NB];
    for (int k = 0; k < n_batches; ++k) order[k] = k;
    std::stable_sort(order, order + n_batches, [&](int x, int y) {
        return batches[x].game->ops->cells > batches[y].game->ops->cells;
    });
    lx::GroupArgs a = {};
    lx::DevState ds[NB];
    int64_t ns[NB], *ss[NB];
    int m = 0;
    int64_t blocks = 0;
    for (int q = 0; q < n_batches; ++q) {
        const int k = order[q];
        const ludax_batch &b = batches[k];
        if (b.n == 0) continue;
        ds[m] = d[k];
        ns[m] = b.n;
        ss[m] = b.stats;
        a.st[m] = d[k];
        a.n[m] = b.n;
        a.gid_base[m] = b.game_id_base;
        a.reward[m] = b.reward;
        a.terminal[m] = b.terminal;
        a.max_plies[m] = b.game->max_plies;
        a.slot[m] = b.game->ops->group_slot;
        a.first_block[m] = (int32_t)blocks;
        blocks += (b.n + 63) / 64;
        ++m;
    }
    for (int k = m; k <= NB; ++k) a.first_block[k] = (int32_t)blocks;
    a.nb = m;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    // the counters as ludax_playout keeps them: after minus before, both
    // reductions over all batches in one launch each (from the start
    // positions the before part is zero and is not launched)
    if (!from_start) e = lx::launch_stats_group(ds, ns, m, -1, ss, stream);
    if (e == hipSuccess) e = lx::launch_playout_group(a, from_start != 0, stream);
    if (e == hipSuccess) e = lx::launch_stats_group(ds, ns, m, +1, ss, stream);
    // a cache that ludax_init would have reset now describes the final boards
    for (int k = 0; k < n_batches && e == hipSuccess && from_start; ++k)
        if (batches[k].n > 0 && daux[k].aux != nullptr)
            e = batches[k].game->ops->aux_sync(daux[k], batches[k].n, stream);
    return device_error(e);
}

int ludax_random_step(const ludax_game *game, ludax_state *state, uint64_t seed, int64_t game_id_base,
                      const int64_t *game_id, int8_t *reward, uint8_t *terminal, int64_t n,
                      hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (reward == nullptr || terminal == nullptr) return LUDAX_E_INVALID;
    lx::DevState d;
    int rc = check_state(state, &d, game->ops->aux_bytes);
    if (rc) return rc;
    return device_error(game->ops->random_step(d, n, game->max_plies, seed, game_id_base, game_id, reward,
                                               terminal, stream));
}

int ludax_policy_step(const ludax_game *game, ludax_state *state, const float *logits, uint64_t seed,
                      int64_t game_id_base, const int64_t *game_id, int8_t *reward, uint8_t *terminal,
                      int64_t n, hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (logits == nullptr || reward == nullptr || terminal == nullptr) return LUDAX_E_INVALID;
    lx::DevState d;
    int rc = check_state(state, &d, game->ops->aux_bytes);
    if (rc) return rc;
    return device_error(game->ops->policy_step(d, n, game->max_plies, logits, seed, game_id_base, game_id, reward,
                                               terminal, stream));
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

int ludax_aux_sync(const ludax_game *game, ludax_state *state, int64_t n, hipStream_t stream)
{
    if (game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0 || game->ops->aux_bytes == 0) return LUDAX_OK;
    lx::DevState d;
    int rc = check_state(state, &d, game->ops->aux_bytes);
    if (rc) return rc;
    if (d.aux == nullptr) return LUDAX_E_INVALID;
    return device_error(game->ops->aux_sync(d, n, stream));
}

struct ludax_mixed {
    int n;
    const ludax_game *games[8];
    int32_t slots[8];
    int one_grid; // 1: every kind in one launch (k_persist_group), 0: a kernel per kind on its stream
    hipStream_t streams[8];
    hipEvent_t fork, join[8];
};

namespace {

constexpr int MAX_KINDS = 8;
constexpr int64_t MAX_GAME_ID = (int64_t)1 << 62;

int check_slots(const int32_t *slots, int n)
{
    for (int k = 0; k < n; ++k)
        if (slots[k] < 64 || slots[k] > (1 << 24) || (slots[k] & 63) != 0) return LUDAX_E_INVALID;
    return LUDAX_OK;
}

// j0 and count of kind k among the ids id_base + j, j < n_games
void kind_range(int64_t id_base, int64_t n_games, int n, int k, int64_t *j0, int64_t *count)
{
    const int64_t first = ((int64_t)k - id_base % n + n) % n;
    *j0 = first;
    *count = first < n_games ? (n_games - 1 - first) / n + 1 : 0;
}

bool one_grid_ok(const ludax_mixed *m)
{
    for (int k = 0; k < m->n; ++k)
        if (m->games[k]->ops->mixed_slot < 0) return false;
    return true;
}

// Enqueue a batch under `slots` for the kinds whose bit is set in `mask`,
// in one grid or as one kernel per kind (one_grid).
int mixed_run(ludax_mixed *m, const int32_t *slots, unsigned mask, uint64_t seed, int64_t id_base,
              int64_t n_games, int8_t *winner, int16_t *plies, int16_t *last, int64_t *stats,
              uint32_t *workspace, hipStream_t stream, int one_grid)
{
    hipError_t e = lx::launch_zero_counters(workspace, m->n, stream);
    if (one_grid) {
        lx::MixedGroupArgs g = {};
        int q = 0, blocks = 0;
        for (int k = 0; k < m->n; ++k) {
            if (!((mask >> k) & 1u)) continue;
            lx::MixedArgs &a = g.k[q];
            kind_range(id_base, n_games, m->n, k, &a.j0, &a.count);
            if (a.count == 0) continue;
            a.id_base = id_base;
            a.stride = m->n;
            a.max_plies = m->games[k]->max_plies;
            a.key0 = (uint32_t)seed;
            a.key1 = (uint32_t)(seed >> 32);
            a.winner = winner;
            a.plies = plies;
            a.last = last;
            a.counter = workspace + k;
            const int64_t need = (a.count + 63) / 64 * 64;
            const int lanes = (int)std::min<int64_t>(slots[k], need);
            g.slot[q] = m->games[k]->ops->mixed_slot;
            g.first_block[q] = blocks;
            blocks += lanes / 64;
            ++q;
        }
        for (int k = q; k <= lx::MIXED_MAX; ++k) g.first_block[k] = blocks;
        g.n = q;
        if (e == hipSuccess && q > 0) e = lx::launch_mixed_group(g, stream);
        if (e == hipSuccess && stats != nullptr)
            e = lx::launch_mixed_stats(winner, plies, n_games, id_base, m->n, stats, stream);
        return device_error(e);
    }
    if (e == hipSuccess) e = hipEventRecord(m->fork, stream);
    for (int k = 0; k < m->n && e == hipSuccess; ++k) {
        if (!((mask >> k) & 1u)) continue;
        lx::MixedArgs a;
        kind_range(id_base, n_games, m->n, k, &a.j0, &a.count);
        if (a.count == 0) continue;
        a.id_base = id_base;
        a.stride = m->n;
        a.max_plies = m->games[k]->max_plies;
        a.key0 = (uint32_t)seed;
        a.key1 = (uint32_t)(seed >> 32);
        a.winner = winner;
        a.plies = plies;
        a.last = last;
        a.counter = workspace + k;
        // no more lanes than games
        const int64_t need = (a.count + 63) / 64 * 64;
        const int lanes = (int)std::min<int64_t>(slots[k], need);
        e = hipStreamWaitEvent(m->streams[k], m->fork, 0);
        if (e == hipSuccess) e = m->games[k]->ops->persist(a, lanes, m->streams[k]);
        if (e == hipSuccess) e = hipEventRecord(m->join[k], m->streams[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, m->join[k], 0);
    }
    if (e == hipSuccess && stats != nullptr)
        e = lx::launch_mixed_stats(winner, plies, n_games, id_base, m->n, stats, stream);
    return device_error(e);
}

int mixed_args_ok(const ludax_mixed *m, int64_t id_base, int64_t n_games, int8_t *winner, int16_t *plies,
                  int16_t *last, uint32_t *workspace)
{
    if (m == nullptr || id_base < 0 || n_games < 0 || id_base > MAX_GAME_ID - n_games ||
        n_games > MAX_ENVS)
        return LUDAX_E_INVALID;
    if (n_games > 0 && (winner == nullptr || plies == nullptr || last == nullptr || workspace == nullptr))
        return LUDAX_E_INVALID;
    return LUDAX_OK;
}

// wall time of one batch (ms), measured with events on the stream
int timed_run(ludax_mixed *m, const int32_t *slots, unsigned mask, uint64_t seed, int64_t id_base,
              int64_t n_games, int8_t *winner, int16_t *plies, int16_t *last, uint32_t *workspace,
              hipStream_t stream, float *ms, int one_grid)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return LUDAX_E_DEVICE;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return LUDAX_E_DEVICE;
    }
    int rc = device_error(hipEventRecord(a, stream));
    if (rc == LUDAX_OK)
        rc = mixed_run(m, slots, mask, seed, id_base, n_games, winner, plies, last, nullptr, workspace, stream,
                       one_grid);
    if (rc == LUDAX_OK) rc = device_error(hipEventRecord(b, stream));
    if (rc == LUDAX_OK) rc = device_error(hipEventSynchronize(b));
    if (rc == LUDAX_OK) rc = device_error(hipEventElapsedTime(ms, a, b));
    hipEventDestroy(a);
    hipEventDestroy(b);
    return rc;
}

// split `total` lanes in proportion to w (multiples of 64, at least 64 each)
void split(const double *w, int n, int32_t total, int32_t *out)
{
    double sum = 0;
    for (int k = 0; k < n; ++k) sum += w[k];
    for (int k = 0; k < n; ++k) {
        const double share = sum > 0 ? w[k] / sum : 1.0 / n;
        int32_t s = (int32_t)std::lround(share * total / 64.0) * 64;
        out[k] = std::max<int32_t>(64, std::min<int32_t>(s, 1 << 24));
    }
}

} // namespace

int ludax_mixed_create(const ludax_game *const *games, int32_t n_kinds, ludax_mixed **out)
{
    if (games == nullptr || out == nullptr || n_kinds < 1 || n_kinds > MAX_KINDS) return LUDAX_E_INVALID;
    *out = nullptr;
    for (int k = 0; k < n_kinds; ++k)
        if (games[k] == nullptr) return LUDAX_E_INVALID;
    for (int k = 0; k < n_kinds; ++k)
        if (games[k]->ops->persist == nullptr) return LUDAX_E_UNSUPPORTED;
    ludax_mixed *m = new (std::nothrow) ludax_mixed;
    if (m == nullptr) return LUDAX_E_INVALID;
    m->n = n_kinds;
    int created = 0;
    hipError_t e = hipEventCreateWithFlags(&m->fork, hipEventDisableTiming);
    for (int k = 0; k < n_kinds && e == hipSuccess; ++k) {
        m->games[k] = games[k];
        m->slots[k] = 65536;
        m->one_grid = 0;
        e = hipStreamCreateWithFlags(&m->streams[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->join[k], hipEventDisableTiming);
        if (e == hipSuccess) created = k + 1;
    }
    // one grid when every kind is in the one-grid kernel
    if (e == hipSuccess) m->one_grid = one_grid_ok(m) ? 1 : 0;
    if (e != hipSuccess) {
        for (int k = 0; k < created; ++k) {
            hipStreamDestroy(m->streams[k]);
            hipEventDestroy(m->join[k]);
        }
        delete m;
        return device_error(e);
    }
    *out = m;
    return LUDAX_OK;
}

int ludax_mixed_destroy(ludax_mixed *m)
{
    if (m == nullptr) return LUDAX_E_INVALID;
    for (int k = 0; k < m->n; ++k) {
        hipStreamDestroy(m->streams[k]);
        hipEventDestroy(m->join[k]);
    }
    hipEventDestroy(m->fork);
    delete m;
    return LUDAX_OK;
}

int ludax_mixed_set_slots(ludax_mixed *m, const int32_t *slots)
{
    if (m == nullptr || slots == nullptr || check_slots(slots, m->n) != LUDAX_OK) return LUDAX_E_INVALID;
    for (int k = 0; k < m->n; ++k) m->slots[k] = slots[k];
    return LUDAX_OK;
}

int ludax_mixed_get_slots(const ludax_mixed *m, int32_t *slots)
{
    if (m == nullptr || slots == nullptr) return LUDAX_E_INVALID;
    for (int k = 0; k < m->n; ++k) slots[k] = m->slots[k];
    return LUDAX_OK;
}

int ludax_mixed_set_one_grid(ludax_mixed *m, int32_t one_grid)
{
    if (m == nullptr || (one_grid != 0 && one_grid != 1)) return LUDAX_E_INVALID;
    if (one_grid && !one_grid_ok(m)) return LUDAX_E_UNSUPPORTED;
    m->one_grid = one_grid;
    return LUDAX_OK;
}

int ludax_mixed_get_one_grid(const ludax_mixed *m, int32_t *one_grid)
{
    if (m == nullptr || one_grid == nullptr) return LUDAX_E_INVALID;
    *one_grid = m->one_grid;
    return LUDAX_OK;
}

int ludax_mixed_playout(ludax_mixed *m, uint64_t seed, int64_t id_base, int64_t n_games, int8_t *winner,
                        int16_t *plies, int16_t *last_action, int64_t *stats, uint32_t *workspace,
                        hipStream_t stream)
{
    int rc = mixed_args_ok(m, id_base, n_games, winner, plies, last_action, workspace);
    if (rc) return rc;
    if (n_games == 0) return LUDAX_OK;
    return mixed_run(m, m->slots, 0xFFu, seed, id_base, n_games, winner, plies, last_action, stats, workspace,
                     stream, m->one_grid);
}

// ---------------------------------------------------------------------------
// ludax_mixed_playout_noalloc: the queue counters (one 32-bit word per kind)
// live in this file-scope device array instead of a caller workspace.  Each
// GPU holds its own copy; its device address is looked up once per device
// (host code never passes the array's name to a kernel: on the host that
// name is only a stand-in for the symbol, not a device address).
// ---------------------------------------------------------------------------
namespace {

constexpr int SCRATCH_WORDS = MAX_KINDS;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) uint32_t scratch[SCRATCH_WORDS];

std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
int scratch_for_current_device(uint32_t **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    if (dev < 0 || dev >= MAX_DEVICES) return LUDAX_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_error(e);
        g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LUDAX_OK;
}

} // namespace

int ludax_mixed_playout_noalloc(ludax_mixed *m, uint64_t seed, int64_t id_base, int64_t n_games, int8_t *winner,
                                int16_t *plies, int16_t *last_action, int64_t *stats, hipStream_t stream)
{
    // any non-null pointer passes mixed_args_ok's workspace test; the real
    // counters are the device's scratch words
    uint32_t dummy = 0;
    int rc = mixed_args_ok(m, id_base, n_games, winner, plies, last_action, &dummy);
    if (rc) return rc;
    if (m->n > SCRATCH_WORDS) return LUDAX_E_INVALID;
    if (n_games == 0) return LUDAX_OK;
    uint32_t *counters = nullptr;
    rc = scratch_for_current_device(&counters);
    if (rc) return rc;
    return mixed_run(m, m->slots, 0xFFu, seed, id_base, n_games, winner, plies, last_action, stats, counters,
                     stream, m->one_grid);
}

int ludax_mixed_autotune(ludax_mixed *m, uint64_t seed, int64_t id_base, int64_t n_games, int32_t total_slots,
                         int8_t *winner, int16_t *plies, int16_t *last_action, uint32_t *workspace,
                         hipStream_t stream, float *best_ms)
{
    int rc = mixed_args_ok(m, id_base, n_games, winner, plies, last_action, workspace);
    if (rc) return rc;
    if (n_games == 0 || total_slots < 64 * m->n) return LUDAX_E_INVALID;
    const int n = m->n;
    // 1. each kind alone at an equal share: its work in lane-milliseconds;
    //    and at half and twice that share, for how its time scales with its
    //    lanes (a kind bound by its longest games, or already filling the
    //    chip, gains little from more)
    int32_t eq[MAX_KINDS];
    double w[MAX_KINDS], root[MAX_KINDS], t_eq[MAX_KINDS], beta[MAX_KINDS];
    const double ones[MAX_KINDS] = {1, 1, 1, 1, 1, 1, 1, 1};
    split(ones, n, total_slots, eq);
    for (int k = 0; k < n; ++k) {
        float ms = 0.f;
        rc = timed_run(m, eq, 1u << k, seed, id_base, n_games, winner, plies, last_action, workspace, stream, &ms,
                       m->one_grid);
        if (rc) return rc;
        t_eq[k] = ms;
        w[k] = (double)ms * eq[k];
        root[k] = std::sqrt(w[k]);
        double slope = 0.0;
        int fits = 0;
        for (double f : {0.5, 2.0}) {
            int32_t alt[MAX_KINDS];
            for (int j = 0; j < n; ++j) alt[j] = eq[j];
            alt[k] = std::max<int32_t>(64, std::min<int32_t>((int32_t)(eq[k] * f) / 64 * 64, 1 << 24));
            if (alt[k] == eq[k]) continue;
            float ms2 = 0.f;
            rc = timed_run(m, alt, 1u << k, seed, id_base, n_games, winner, plies, last_action, workspace, stream,
                           &ms2, m->one_grid);
            if (rc) return rc;
            if (ms > 0.f && ms2 > 0.f) {
                slope += -std::log((double)ms2 / ms) / std::log((double)alt[k] / eq[k]);
                ++fits;
            }
        }
        // T_k(S) ~ t_eq (S / eq)^(-beta): beta = 1 for perfect scaling
        beta[k] = std::max(0.05, std::min(1.5, fits ? slope / fits : 1.0));
    }
    // 2. candidate splits of the whole batch
    std::vector<std::vector<int32_t>> plans;
    auto add = [&](const double *weights) {
        std::vector<int32_t> p(n);
        split(weights, n, total_slots, p.data());
        plans.push_back(p);
    };
    add(ones);
    add(w);
    add(root);
    int big = 0;
    for (int k = 1; k < n; ++k)
        if (w[k] > w[big]) big = k;
    for (double f : {0.75, 1.25}) {
        double v[MAX_KINDS];
        for (int k = 0; k < n; ++k) v[k] = k == big ? w[k] * f : w[k];
        add(v);
    }
    // the occupancy plan: the kinds run side by side and the batch ends with
    // the slowest, so give each kind the lanes that bring its fitted time to
    // a common T, with T such that the lanes add up to total_slots (bisection
    // on log T); and the same plan with the slowest-scaling kind's share
    // moved by -25 % and +25 %
    {
        double lo = 1e-6, hi = 1e6;
        double occ[MAX_KINDS];
        for (int it = 0; it < 100; ++it) {
            const double T = std::sqrt(lo * hi);
            double sum = 0.0;
            for (int k = 0; k < n; ++k) sum += eq[k] * std::pow(t_eq[k] / T, 1.0 / beta[k]);
            if (sum > total_slots) lo = T;
            else hi = T;
        }
        const double T = std::sqrt(lo * hi);
        for (int k = 0; k < n; ++k) occ[k] = eq[k] * std::pow(t_eq[k] / T, 1.0 / beta[k]);
        add(occ);
        int flat = 0;
        for (int k = 1; k < n; ++k)
            if (beta[k] < beta[flat]) flat = k;
        for (double f : {0.75, 1.25}) {
            double v[MAX_KINDS];
            for (int k = 0; k < n; ++k) v[k] = k == flat ? occ[k] * f : occ[k];
            add(v);
        }
    }
    // 3. keep the fastest (plan, launch) pair, each plan launched as one
    // grid (when every kind is in the one-grid kernel) and as a kernel per
    // kind (a warm-up run first)
    float best = 0.f;
    int best_i = -1, best_grid = 0;
    const int grids = one_grid_ok(m) ? 2 : 1;
    for (size_t i = 0; i < plans.size(); ++i) {
        for (int og = 0; og < grids; ++og) {
            float ms = 0.f;
            if (i == 0) {
                rc = timed_run(m, plans[i].data(), 0xFFu, seed, id_base, n_games, winner, plies, last_action,
                               workspace, stream, &ms, og);
                if (rc) return rc;
            }
            rc = timed_run(m, plans[i].data(), 0xFFu, seed, id_base, n_games, winner, plies, last_action,
                           workspace, stream, &ms, og);
            if (rc) return rc;
            // the better of two runs: one run's noise (a few percent) is as
            // large as the differences between the candidates
            float ms2 = 0.f;
            rc = timed_run(m, plans[i].data(), 0xFFu, seed, id_base, n_games, winner, plies, last_action,
                           workspace, stream, &ms2, og);
            if (rc) return rc;
            ms = std::min(ms, ms2);
            if (best_i < 0 || ms < best) {
                best = ms;
                best_i = (int)i;
                best_grid = og;
            }
        }
    }
    // 4. local refinement of the fastest plan in its launch mode: each
    //    kind's share moved by -30 % and +40 %, then by -15 % and +18 %
    //    (the other kinds keep their proportions), a move kept when the
    //    batch gets faster: the fitted model misses where kinds slow each
    //    other down by sharing the SIMDs
    std::vector<int32_t> cur = plans[best_i];
    for (double step : {1.4, 1.18}) {
        for (int k = 0; k < n; ++k) {
            for (double f : {1.0 / step, step}) {
                double v[MAX_KINDS];
                for (int j = 0; j < n; ++j) v[j] = (double)cur[j];
                v[k] *= f;
                std::vector<int32_t> p(n);
                split(v, n, total_slots, p.data());
                if (p == cur) continue;
                float ms = 0.f, ms2 = 0.f;
                rc = timed_run(m, p.data(), 0xFFu, seed, id_base, n_games, winner, plies, last_action, workspace,
                               stream, &ms, best_grid);
                if (rc) return rc;
                rc = timed_run(m, p.data(), 0xFFu, seed, id_base, n_games, winner, plies, last_action, workspace,
                               stream, &ms2, best_grid);
                if (rc) return rc;
                ms = std::min(ms, ms2);
                if (ms < best) {
                    best = ms;
                    cur = p;
                }
            }
        }
    }
    for (int k = 0; k < n; ++k) m->slots[k] = cur[k];
    m->one_grid = best_grid;
    if (best_ms) *best_ms = best;
    return LUDAX_OK;
}

struct ludax_net {
    int32_t n;
};

int ludax_net_create(int32_t rows, int32_t cols, ludax_net **out)
{
    if (out == nullptr) return LUDAX_E_INVALID;
    *out = nullptr;
    if (rows != cols || !lx::net_size_supported(rows)) return LUDAX_E_UNSUPPORTED;
    ludax_net *h = new (std::nothrow) ludax_net{rows};
    if (h == nullptr) return LUDAX_E_INVALID;
    *out = h;
    return LUDAX_OK;
}

int ludax_net_destroy(ludax_net *net)
{
    delete net;
    return LUDAX_OK;
}

int ludax_net_info(const ludax_net *net, int64_t *n_params, int64_t *packed_bytes)
{
    if (net == nullptr) return LUDAX_E_INVALID;
    if (n_params) *n_params = lx::net_n_params();
    if (packed_bytes) *packed_bytes = lx::net_packed_bytes();
    return LUDAX_OK;
}

int ludax_net_workspace_bytes(const ludax_net *net, int64_t n, int32_t training, int64_t *bytes)
{
    if (net == nullptr || bytes == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    *bytes = training ? lx::net_train_ws_bytes(net->n, n) : lx::net_forward_ws_bytes(net->n, n);
    return LUDAX_OK;
}

int ludax_net_max_batch(const ludax_net *net, int64_t budget_bytes, int32_t training, int64_t *n)
{
    if (net == nullptr || n == nullptr || budget_bytes < 0) return LUDAX_E_INVALID;
    auto bytes = [&](int64_t k) {
        return training ? lx::net_train_ws_bytes(net->n, k) : lx::net_forward_ws_bytes(net->n, k);
    };
    // the workspace grows with the batch: binary search of the largest fit
    int64_t lo = 0, hi = MAX_ENVS;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (bytes(mid) <= budget_bytes) lo = mid;
        else hi = mid - 1;
    }
    *n = lo > 0 && bytes(lo) <= budget_bytes ? lo : 0;
    return LUDAX_OK;
}

namespace {
bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }
} // namespace

int ludax_net_pack(const ludax_net *net, const float *params, void *packed, hipStream_t stream)
{
    if (net == nullptr || params == nullptr || packed == nullptr || !aligned16(packed)) return LUDAX_E_INVALID;
    return device_error(lx::net_pack(params, packed, stream));
}

int ludax_net_forward(const ludax_net *net, const float *params, const void *packed, const int8_t *board,
                      const int8_t *to_move, int64_t n, float *logits, float *value, void *workspace,
                      hipStream_t stream)
{
    if (net == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    if (params == nullptr || packed == nullptr || !aligned16(packed) || board == nullptr || to_move == nullptr ||
        logits == nullptr || value == nullptr || workspace == nullptr || !aligned256(workspace))
        return LUDAX_E_INVALID;
    return device_error(lx::net_forward(net->n, params, packed, board, to_move, n, logits, value, workspace, stream));
}

int ludax_net_loss_grad(const ludax_net *net, const float *params, const void *packed, const int8_t *board,
                        const int8_t *to_move, const int16_t *action, const float *z, int64_t n, float beta,
                        float *loss, float *grads, void *workspace, hipStream_t stream)
{
    if (net == nullptr || n < 1 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (params == nullptr || packed == nullptr || !aligned16(packed) || board == nullptr || to_move == nullptr ||
        action == nullptr || z == nullptr || loss == nullptr || grads == nullptr || workspace == nullptr ||
        !aligned256(workspace))
        return LUDAX_E_INVALID;
    return device_error(lx::net_loss_grad(net->n, params, packed, board, to_move, action, z, n, beta, loss, grads,
                                          workspace, stream));
}

int ludax_net_adam(const ludax_net *net, float *params, const float *grads, float *m, float *v, int32_t step,
                   float lr, float beta1, float beta2, float eps, void *packed, hipStream_t stream)
{
    if (net == nullptr || params == nullptr || grads == nullptr || m == nullptr || v == nullptr || step < 1 ||
        !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || (packed && !aligned16(packed)))
        return LUDAX_E_INVALID;
    return device_error(lx::net_adam(params, grads, m, v, step, lr, beta1, beta2, eps, packed, stream));
}

int ludax_net_estimate(const ludax_net *net, const float *params, const void *packed, const ludax_state *state,
                       int64_t n, float *estimate, void *workspace, hipStream_t stream)
{
    if (net == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (n == 0) return LUDAX_OK;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    if (params == nullptr || packed == nullptr || !aligned16(packed) || estimate == nullptr ||
        workspace == nullptr || !aligned256(workspace))
        return LUDAX_E_INVALID;
    return device_error(lx::net_estimate(net->n, params, packed, d, n, estimate, workspace, stream));
}

int ludax_net_guided_step(const ludax_net *net, const float *params, const void *packed, const ludax_game *game,
                          ludax_state *state, uint64_t seed, int64_t game_id_base, const int64_t *game_id,
                          int8_t *reward, uint8_t *terminal, int64_t n, void *workspace, hipStream_t stream)
{
    if (net == nullptr || game == nullptr || n < 0 || n > MAX_ENVS) return LUDAX_E_INVALID;
    if (net->n != 11 || game->desc.rows != 11 || game->desc.cols != 11 ||
        (game->desc.kind != LUDAX_HEX && game->desc.kind != LUDAX_GOMOKU))
        return LUDAX_E_UNSUPPORTED;
    if (n == 0) return LUDAX_OK;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    if (params == nullptr || packed == nullptr || !aligned16(packed) || reward == nullptr || terminal == nullptr ||
        workspace == nullptr || !aligned256(workspace))
        return LUDAX_E_INVALID;
    return device_error(lx::net_guided_step(net->n, params, packed, d, game->desc.kind, n, game->max_plies, seed,
                                            game_id_base, game_id, reward, terminal, workspace, stream));
}

int ludax_net_guided_playout(const ludax_net *net, const float *params, const void *packed, const ludax_game *game,
                             ludax_state *state, int32_t plies, uint64_t seed, int64_t game_id_base,
                             const int64_t *game_id, float *estimate, int64_t n, hipStream_t stream)
{
    if (net == nullptr || game == nullptr || n < 0 || n > MAX_ENVS || plies < 0) return LUDAX_E_INVALID;
    if (net->n != 11 || game->desc.rows != 11 || game->desc.cols != 11 ||
        (game->desc.kind != LUDAX_HEX && game->desc.kind != LUDAX_GOMOKU))
        return LUDAX_E_UNSUPPORTED;
    if (n == 0) return LUDAX_OK;
    lx::DevState d;
    int rc = check_state(state, &d);
    if (rc) return rc;
    if (params == nullptr || packed == nullptr || !aligned16(packed) || estimate == nullptr) return LUDAX_E_INVALID;
    return device_error(lx::net_guided_playout(params, packed, d, game->desc.kind, n, game->max_plies, plies, seed,
                                               game_id_base, game_id, estimate, stream));
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
