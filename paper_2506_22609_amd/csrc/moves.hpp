// moves.hpp -- the movement games (Sec. 3.2 move mechanic: step and hop) on
// the 8 x 8 board: Wolf and Sheep (kind 8) and English Draughts (kind 9).
//
// One env per lane; each player's pieces, and the pieces that move both ways
// (Draughts kings, the wolf), are 64-bit bitboards with bit = cell.  An
// action is an ordered cell pair src * 64 + dst.  Every move runs along a
// diagonal: up-left (-9 per cell), up-right (-7), down-left (+7) or
// down-right (+9).  So the legal moves of a position are four bitboards of
// SOURCE cells, one per direction, plus one move length for all of them
// (1 = step, 2 = hop: while any hop exists no step is legal).  For one source
// the four directions come in increasing destination order, so the k-th legal
// action in index order is found by a binary search over source prefixes
// and a pick among at most four directions.
//
//   k_mv_init     start positions
//   k_mv_mask     legal mask [n][4096]: each block writes its 64 rows
//                 cooperatively, 1 KB per wave store instruction
//   k_mv_step     one ply per env: caller's action, uniform random, or drawn
//                 from logits (MODE 0 / 1 / 2), optional next mask
//   k_mv_playout  the whole uniform-random game in registers
#pragma once

#include "kernels.hpp"

namespace lx {

namespace mv {
constexpr uint64_t COL0 = 0x0101010101010101ull;
constexpr uint64_t NOT_C0 = ~COL0, NOT_C7 = ~(COL0 << 7);                          // c >= 1, c <= 6
constexpr uint64_t NOT_C01 = ~(COL0 | (COL0 << 1)), NOT_C67 = ~((COL0 << 6) | (COL0 << 7)); // c >= 2, c <= 5
constexpr uint64_t ROW0 = 0xFFull, ROW7 = 0xFFull << 56;
} // namespace mv

// cell offset of one step in direction d (up-left, up-right, down-left, down-right)
__device__ __forceinline__ int diag_off(int d) { return d == 0 ? -9 : (d == 1 ? -7 : (d == 2 ? 7 : 9)); }

struct MoveSets {
    uint64_t s[4]; // sources with a legal move in direction d
    int dist;      // 1 = steps, 2 = hops
};

__device__ __forceinline__ uint64_t any_move(const MoveSets &m) { return m.s[0] | m.s[1] | m.s[2] | m.s[3]; }

__device__ __forceinline__ int count_moves(const MoveSets &m)
{
    return __popcll(m.s[0]) + __popcll(m.s[1]) + __popcll(m.s[2]) + __popcll(m.s[3]);
}

// legal moves from sources below cell x (1 <= x <= 63)
__device__ __forceinline__ int moves_below(const MoveSets &m, int x)
{
    const uint64_t b = (1ull << x) - 1ull;
    return __popcll(m.s[0] & b) + __popcll(m.s[1] & b) + __popcll(m.s[2] & b) + __popcll(m.s[3] & b);
}

// The k-th legal move (0 <= k < count_moves(m)) in increasing action order:
// its source cell and direction.
__device__ __forceinline__ void select_move(const MoveSets &m, int k, int &src, int &d)
{
    int lo = 0, hi = 64, below = 0; // moves_below(lo) = below <= k < moves_below(hi)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const int mid = (lo + hi) >> 1;
        const int c = moves_below(m, mid);
        if (c <= k) {
            lo = mid;
            below = c;
        } else {
            hi = mid;
        }
    }
    // the directions of source lo come in increasing action order: the r-th set one
    const int r = k - below;
    const int b0 = (int)((m.s[0] >> lo) & 1ull), b1 = (int)((m.s[1] >> lo) & 1ull),
              b2 = (int)((m.s[2] >> lo) & 1ull);
    src = lo;
    d = (b0 && r == 0) ? 0 : ((b1 && r == b0) ? 1 : ((b2 && r == b0 + b1) ? 2 : 3));
}

template <int KIND_>
struct DiagGame {
    static constexpr int KIND = KIND_, H = 8, W = 8, CELLS = 64, A = 64 * 64;
    static constexpr bool HOPS = KIND == 9; // Draughts; Wolf and Sheep only steps
    uint64_t p1, p2, both; // both: pieces that move in all four directions

    // Cell bytes (16 aligned dwords): owner in bits 0-1, bit 2 marks a
    // Draughts king.  The wolf (player 2's only piece) moves both ways.
    __device__ void load(const uint32_t (&v)[16])
    {
        uint32_t a[2] = {0u, 0u}, b[2] = {0u, 0u}, k[2] = {0u, 0u};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int w = j >> 3, sh = 4 * (j & 7);
            a[w] |= __builtin_amdgcn_udot4(v[j] & 0x01010101u, 0x08040201u, 0u, false) << sh;
            b[w] |= __builtin_amdgcn_udot4((v[j] >> 1) & 0x01010101u, 0x08040201u, 0u, false) << sh;
            k[w] |= __builtin_amdgcn_udot4((v[j] >> 2) & 0x01010101u, 0x08040201u, 0u, false) << sh;
        }
        p1 = ((uint64_t)a[1] << 32) | a[0];
        p2 = ((uint64_t)b[1] << 32) | b[0];
        both = HOPS ? ((uint64_t)k[1] << 32) | k[0] : p2;
    }

    __device__ void store(uint32_t (&v)[16]) const
    {
        const uint64_t k = HOPS ? both : 0ull;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            uint32_t x = 0u;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = 4 * j + i;
                const uint32_t cv = (uint32_t)((p1 >> c) & 1ull) | ((uint32_t)((p2 >> c) & 1ull) << 1) |
                                    ((uint32_t)((k >> c) & 1ull) << 2);
                x |= cv << (8 * i);
            }
            v[j] = x;
        }
    }

    __device__ void start()
    {
        if constexpr (HOPS) {
            // the dark cells of rows 5-7 (player 1) and of rows 0-2 (player 2)
            p1 = 0x55AA550000000000ull;
            p2 = 0x0000000000AA55AAull;
            both = 0ull;
        } else {
            p1 = 0x5500000000000000ull; // the dark cells of the bottom row
            p2 = 1ull << 3;
            both = p2;
        }
    }

    // Legal moves of `me`; cont = the extra-turn byte (Draughts: cell + 1 of
    // the only piece allowed to move, 0 = any piece).
    __device__ MoveSets moves(int me, int cont) const
    {
        const uint64_t own = me == 1 ? p1 : p2, opp = me == 1 ? p2 : p1;
        uint64_t movers = own;
        if (HOPS && cont > 0) movers &= cont <= 64 ? 1ull << (cont - 1) : 0ull;
        const uint64_t up = me == 1 ? movers : movers & both;
        const uint64_t down = me == 2 ? movers : movers & both;
        const uint64_t e = ~(p1 | p2);
        MoveSets m;
        if constexpr (HOPS) {
            m.s[0] = up & mv::NOT_C01 & (opp << 9) & (e << 18);
            m.s[1] = up & mv::NOT_C67 & (opp << 7) & (e << 14);
            m.s[2] = down & mv::NOT_C01 & (opp >> 7) & (e >> 14);
            m.s[3] = down & mv::NOT_C67 & (opp >> 9) & (e >> 18);
            m.dist = 2;
            if (any_move(m)) return m;
        }
        m.s[0] = up & mv::NOT_C0 & (e << 9);
        m.s[1] = up & mv::NOT_C7 & (e << 7);
        m.s[2] = down & mv::NOT_C0 & (e >> 7);
        m.s[3] = down & mv::NOT_C7 & (e >> 9);
        m.dist = 1;
        return m;
    }

    // Apply the legal move (src, d, dist) of `me` with its effects: capture
    // of the hopped piece, then promotion, then the extra-turn test (the
    // order of the Draughts description).  Returns the player to move next
    // and sets cont.
    __device__ int apply(int src, int d, int dist, int me, int &cont)
    {
        const int off = diag_off(d);
        const int dst = src + dist * off;
        const uint64_t bs = 1ull << src, bd = 1ull << dst, mv2 = bs | bd;
        p1 ^= me == 1 ? mv2 : 0ull;
        p2 ^= me == 2 ? mv2 : 0ull;
        if (both & bs) both ^= mv2;
        cont = 0;
        if constexpr (HOPS) {
            if (dist == 2) {
                const uint64_t keep = ~(1ull << (src + off)); // the hopped piece is captured
                p1 &= me == 2 ? keep : ~0ull;
                p2 &= me == 1 ? keep : ~0ull;
                both &= keep;
            }
            if (bd & (me == 1 ? mv::ROW0 : mv::ROW7)) both |= bd; // promotion
            if (dist == 2) {
                // can the same piece hop again?
                const uint64_t opp = me == 1 ? p2 : p1, e = ~(p1 | p2);
                const uint64_t up = me == 1 || (both & bd) ? bd : 0ull;
                const uint64_t down = me == 2 || (both & bd) ? bd : 0ull;
                const uint64_t again = (up & mv::NOT_C01 & (opp << 9) & (e << 18)) |
                                       (up & mv::NOT_C67 & (opp << 7) & (e << 14)) |
                                       (down & mv::NOT_C01 & (opp >> 7) & (e >> 14)) |
                                       (down & mv::NOT_C67 & (opp >> 9) & (e >> 18));
                if (again) {
                    cont = dst + 1;
                    return me;
                }
            }
        }
        return 3 - me;
    }

    // End rules after the mover's ply, given the next player's moves: the
    // wolf on the bottom row wins (Wolf and Sheep), then the mover wins if
    // the next player has no legal move.  -1 = the game goes on.
    __device__ int end_rules(int me, const MoveSets &next) const
    {
        if constexpr (!HOPS)
            if (me == 2 && (p2 & mv::ROW7)) return 2;
        return any_move(next) ? -1 : me;
    }
};

// Load / store one env's 64 cell bytes with 16-byte accesses.
__device__ __forceinline__ void load_cells(const int8_t *p, uint32_t (&v)[16])
{
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 x = q[i];
        v[4 * i] = x.x;
        v[4 * i + 1] = x.y;
        v[4 * i + 2] = x.z;
        v[4 * i + 3] = x.w;
    }
}

__device__ __forceinline__ void store_cells(int8_t *p, const uint32_t (&v)[16])
{
    uint4 *q = reinterpret_cast<uint4 *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = uint4{v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]};
}

// The block's legal-mask rows [nb][4096] from the move sets in LDS.  Store
// q (0..3) of lane t covers bytes 1024 q + 16 t .. +15 of a row: source
// 16 q + t / 4, destinations 16 (t % 4) .. +15, so each store instruction
// of the wave writes 1 KB of one row contiguously.
__device__ __forceinline__ void write_move_rows(uint8_t *__restrict__ rows, int nb, const MoveSets *sets)
{
    const int t = threadIdx.x;
    const int quarter = t & 3;
    for (int j = 0; j < nb; ++j) {
        const MoveSets m = sets[j];
        uint8_t *row = rows + (int64_t)j * 4096;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int src = 16 * q + (t >> 2);
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int dst = src + m.dist * diag_off(d);
                const bool on = ((m.s[d] >> src) & 1ull) && (dst >> 4) == quarter;
                const uint32_t byte = on ? 1u << (8 * (dst & 3)) : 0u;
                const int wi = (dst >> 2) & 3;
                w[0] |= wi == 0 ? byte : 0u;
                w[1] |= wi == 1 ? byte : 0u;
                w[2] |= wi == 2 ? byte : 0u;
                w[3] |= wi == 3 ? byte : 0u;
            }
            reinterpret_cast<uint4 *>(row)[64 * q + t] = uint4{w[0], w[1], w[2], w[3]};
        }
    }
}

__device__ __forceinline__ MoveSets no_moves()
{
    MoveSets m;
    m.s[0] = m.s[1] = m.s[2] = m.s[3] = 0ull;
    m.dist = 1;
    return m;
}

// ---------------------------------------------------------------------------
// a1: start positions
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_mv_init(DevState st, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    G g;
    g.start();
    uint32_t v[16];
    g.store(v);
    store_cells(st.board + e * 64, v);
    st.to_move[e] = 1;
    st.status[e] = RUNNING;
    st.winner[e] = -1;
    st.passes[e] = 0;
    st.ply[e] = 0;
    st.last_action[e] = -1;
}

// ---------------------------------------------------------------------------
// a2: legal mask
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_mv_mask(DevState st, int64_t n, uint8_t *__restrict__ mask)
{
    __shared__ MoveSets sets[BLOCK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    const bool valid = t < nb;
    const int64_t ec = valid ? e0 + t : e0;
    MoveSets m = no_moves();
    if (valid && st.status[ec] == RUNNING) {
        uint32_t v[16];
        load_cells(st.board + ec * 64, v);
        G g;
        g.load(v);
        m = g.moves(st.to_move[ec], st.passes[ec]);
    }
    sets[t] = m;
    __syncthreads();
    write_move_rows(mask + e0 * 4096, nb, sets);
}

// ---------------------------------------------------------------------------
// a3-a6 for one ply (MODE 0 caller's action, 1 uniform random, 2 drawn from
// the softmax of the logits over the legal actions), as k_step does for the
// placement games.  Boards are read and written with 16-byte accesses per
// lane; a block with no RUNNING env reads no board.
// ---------------------------------------------------------------------------
template <class G, int MODE>
__global__ __launch_bounds__(BLOCK) void k_mv_step(DevState st, int64_t n, int max_plies,
                                                   const int32_t *__restrict__ action,
                                                   const float *__restrict__ logits, uint32_t key0, uint32_t key1,
                                                   int64_t gid_base, const int64_t *__restrict__ gid,
                                                   int8_t *__restrict__ reward, uint8_t *__restrict__ terminal,
                                                   uint8_t *__restrict__ next_mask)
{
    __shared__ MoveSets sets[BLOCK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;
    const int64_t ec = valid ? e : e0;
    int status = valid ? (int)st.status[ec] : ILLEGAL;
    const bool was_running = status == RUNNING;

    if (!__syncthreads_or(was_running)) {
        if (valid) {
            reward[2 * e] = 0;
            reward[2 * e + 1] = 0;
            terminal[e] = 1;
        }
        if (next_mask != nullptr) {
            uint4 *dst = reinterpret_cast<uint4 *>(next_mask + e0 * 4096);
            for (int j = t; j < nb * 256; j += BLOCK) dst[j] = uint4{0u, 0u, 0u, 0u};
        }
        return;
    }

    G g;
    int me = 1, winner = -1, cont = 0, ply = 0, last = -1;
    int r1 = 0, r2 = 0;
    MoveSets next = no_moves();
    if (was_running) {
        uint32_t v[16];
        load_cells(st.board + ec * 64, v);
        g.load(v);
        me = st.to_move[ec];
        winner = st.winner[ec];
        cont = st.passes[ec];
        ply = st.ply[ec];
        last = st.last_action[ec];
        const MoveSets cur = g.moves(me, cont);
        const int nl = count_moves(cur);
        int src = 0, d = 0;
        bool legal = nl > 0;
        if constexpr (MODE == 0) {
            const int a = action[ec];
            legal = false;
            if (a >= 0 && a < G::A) {
                src = a >> 6;
#pragma unroll
                for (int dd = 0; dd < 4; ++dd)
                    if (((cur.s[dd] >> src) & 1ull) && src + cur.dist * diag_off(dd) == (a & 63)) {
                        legal = true;
                        d = dd;
                    }
            }
        } else {
            const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
            const Philox4 f = philox4x32_10((uint32_t)ply >> 2, (uint32_t)id, (uint32_t)(id >> 32), 0u, key0, key1);
            const int r = ply & 3;
            const uint32_t w = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
            if constexpr (MODE == 1) {
                if (legal) select_move(cur, (int)__umulhi(w, (uint32_t)nl), src, d);
            } else if (legal) {
                // softmax over the legal actions in increasing order (float32):
                // the first whose running sum of exp(logit - max) exceeds
                // u * total, u = (w >> 8) / 2^24; the last one if none does
                const float *lg = logits + ec * G::A;
                const uint64_t srcs = any_move(cur);
                float mx = -3.0e38f;
                for (uint64_t u = srcs; u; u &= u - 1ull) {
                    const int s = __builtin_ctzll(u);
                    for (int dd = 0; dd < 4; ++dd)
                        if ((cur.s[dd] >> s) & 1ull) mx = fmaxf(mx, lg[s * 64 + s + cur.dist * diag_off(dd)]);
                }
                float tot = 0.f;
                for (uint64_t u = srcs; u; u &= u - 1ull) {
                    const int s = __builtin_ctzll(u);
                    for (int dd = 0; dd < 4; ++dd)
                        if ((cur.s[dd] >> s) & 1ull) tot += expf(lg[s * 64 + s + cur.dist * diag_off(dd)] - mx);
                }
                const float thr = (float)(w >> 8) * 0x1p-24f * tot;
                float run = 0.f;
                bool picked = false;
                for (uint64_t u = srcs; u; u &= u - 1ull) {
                    const int s = __builtin_ctzll(u);
                    for (int dd = 0; dd < 4; ++dd)
                        if ((cur.s[dd] >> s) & 1ull) {
                            run += expf(lg[s * 64 + s + cur.dist * diag_off(dd)] - mx);
                            if (!picked) {
                                src = s;
                                d = dd;
                                picked = run > thr;
                            }
                        }
                }
            }
        }
        if (!legal) {
            status = ILLEGAL;
        } else {
            const int a = src * 64 + src + cur.dist * diag_off(d);
            const int nxt = g.apply(src, d, cur.dist, me, cont);
            ply += 1;
            last = a;
            next = g.moves(nxt, cont);
            const int outcome = g.end_rules(me, next);
            if (outcome >= 0) {
                status = TERMINAL;
                winner = outcome;
                r1 = outcome == 1 ? 1 : -1;
                r2 = -r1;
                next = no_moves();
            } else {
                me = nxt;
                if (ply >= max_plies) {
                    status = TRUNCATED;
                    winner = -1;
                    next = no_moves();
                }
            }
        }
    }
    if (valid) {
        if (was_running) {
            uint32_t v[16];
            g.store(v);
            store_cells(st.board + e * 64, v);
            st.to_move[e] = (int8_t)me;
            st.status[e] = (int8_t)status;
            st.winner[e] = (int8_t)winner;
            st.passes[e] = (int8_t)cont;
            st.ply[e] = (int16_t)ply;
            st.last_action[e] = (int16_t)last;
        }
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = status != RUNNING ? 1 : 0;
    }
    if (next_mask != nullptr) {
        sets[t] = next;
        __syncthreads();
        write_move_rows(next_mask + e0 * 4096, nb, sets);
    }
}

// One ply of a running game with Philox word w; cur holds the mover's legal
// moves on entry and the next mover's on return.  Returns whether the game
// goes on.
template <class G>
__device__ __forceinline__ bool move_ply(G &g, MoveSets &cur, int &me, int &cont, int &ply, int &last, int &status,
                                         int &winner, uint32_t w, int max_plies)
{
    const int nl = count_moves(cur);
    if (nl == 0) { // only on a hand-edited state
        status = ILLEGAL;
        return false;
    }
    int src, d;
    select_move(cur, (int)__umulhi(w, (uint32_t)nl), src, d);
    const int dist = cur.dist;
    last = src * 64 + src + dist * diag_off(d);
    const int nxt = g.apply(src, d, dist, me, cont);
    ply += 1;
    cur = g.moves(nxt, cont);
    const int outcome = g.end_rules(me, cur);
    if (outcome >= 0) {
        status = TERMINAL;
        winner = outcome;
        return false;
    }
    me = nxt;
    if (ply >= max_plies) {
        status = TRUNCATED;
        winner = -1;
        return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// a2-a8 fused: uniform-random playout to the end of every game
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_mv_playout(DevState st, int64_t n, int max_plies, uint32_t key0,
                                                      uint32_t key1, int64_t gid_base,
                                                      const int64_t *__restrict__ gid, int8_t *__restrict__ reward,
                                                      uint8_t *__restrict__ terminal)
{
    const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    int status = st.status[e];
    if (status != RUNNING) {
        reward[2 * e] = 0;
        reward[2 * e + 1] = 0;
        terminal[e] = 1;
        return;
    }
    uint32_t v[16];
    load_cells(st.board + e * 64, v);
    G g;
    g.load(v);
    int me = st.to_move[e], winner = st.winner[e], cont = st.passes[e], ply = st.ply[e], last = st.last_action[e];
    const uint64_t id = (uint64_t)(gid != nullptr ? gid[e] : gid_base + e);
    const uint32_t id_lo = (uint32_t)id, id_hi = (uint32_t)(id >> 32);
    MoveSets cur = g.moves(me, cont);
    // Philox words in order, w0 = the current ply's; a block serves plies
    // 4q .. 4q+3, the first one possibly entered part-way
    uint32_t w0, w1, w2, w3;
    {
        const Philox4 f = philox4x32_10((uint32_t)ply >> 2, id_lo, id_hi, 0u, key0, key1);
        const int r = ply & 3;
        w0 = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
        w1 = r == 0 ? f.v[1] : (r == 1 ? f.v[2] : f.v[3]);
        w2 = r == 0 ? f.v[2] : f.v[3];
        w3 = f.v[3];
    }
    bool running = true, first = true;
    while (running) {
        if ((ply & 3) == 0 && !first) {
            const Philox4 f = philox4x32_10((uint32_t)ply >> 2, id_lo, id_hi, 0u, key0, key1);
            w0 = f.v[0];
            w1 = f.v[1];
            w2 = f.v[2];
            w3 = f.v[3];
        }
        first = false;
        running = move_ply(g, cur, me, cont, ply, last, status, winner, w0, max_plies);
        w0 = w1;
        w1 = w2;
        w2 = w3;
    }
    const int r1 = status == TERMINAL ? (winner == 1 ? 1 : (winner == 2 ? -1 : 0)) : 0;
    g.store(v);
    store_cells(st.board + e * 64, v);
    st.to_move[e] = (int8_t)me;
    st.status[e] = (int8_t)status;
    st.winner[e] = (int8_t)winner;
    st.passes[e] = (int8_t)cont;
    st.ply[e] = (int16_t)ply;
    st.last_action[e] = (int16_t)last;
    reward[2 * e] = (int8_t)r1;
    reward[2 * e + 1] = (int8_t)-r1;
    terminal[e] = 1;
}

// Lane adapter of the mixed persistent batch (k_persist_lane).
template <class G>
struct DiagLane {
    struct Shared {
        int unused;
    };
    G g;
    MoveSets cur;
    int me, cont, ply, last, status, winner;
    __device__ void bind(Shared &, int) {}
    __device__ void start()
    {
        g.start();
        me = 1;
        cont = 0;
        ply = 0;
        last = -1;
        status = RUNNING;
        winner = -1;
        cur = g.moves(1, 0);
    }
    __device__ bool step(uint32_t w, int max_plies)
    {
        return move_ply(g, cur, me, cont, ply, last, status, winner, w, max_plies);
    }
};

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <class G>
struct MoveLaunch {
    static unsigned blocks(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }
    static hipError_t init(const DevState &st, int64_t n, hipStream_t s)
    {
        hipLaunchKernelGGL(k_mv_init<G>, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n);
        return hipGetLastError();
    }
    static hipError_t mask(const DevState &st, int64_t n, uint8_t *mask, hipStream_t s)
    {
        hipLaunchKernelGGL(k_mv_mask<G>, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, mask);
        return hipGetLastError();
    }
    static hipError_t step(const DevState &st, int64_t n, int max_plies, const int32_t *action, int8_t *reward,
                           uint8_t *terminal, uint8_t *next_mask, hipStream_t s)
    {
        hipLaunchKernelGGL((k_mv_step<G, 0>), dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies, action,
                           (const float *)nullptr, 0u, 0u, (int64_t)0, (const int64_t *)nullptr, reward, terminal,
                           next_mask);
        return hipGetLastError();
    }
    static hipError_t random_step(const DevState &st, int64_t n, int max_plies, uint64_t seed, int64_t gid_base,
                                  const int64_t *gid, int8_t *reward, uint8_t *terminal, hipStream_t s)
    {
        hipLaunchKernelGGL((k_mv_step<G, 1>), dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies,
                           (const int32_t *)nullptr, (const float *)nullptr, (uint32_t)seed, (uint32_t)(seed >> 32),
                           gid_base, gid, reward, terminal, (uint8_t *)nullptr);
        return hipGetLastError();
    }
    static hipError_t policy_step(const DevState &st, int64_t n, int max_plies, const float *logits, uint64_t seed,
                                  int64_t gid_base, const int64_t *gid, int8_t *reward, uint8_t *terminal,
                                  hipStream_t s)
    {
        hipLaunchKernelGGL((k_mv_step<G, 2>), dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies,
                           (const int32_t *)nullptr, logits, (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid,
                           reward, terminal, (uint8_t *)nullptr);
        return hipGetLastError();
    }
    static hipError_t playout(const DevState &st, int64_t n, int max_plies, uint64_t seed, int64_t gid_base,
                              const int64_t *gid, int8_t *reward, uint8_t *terminal, int64_t *stats, hipStream_t s)
    {
        hipError_t err = hipSuccess;
        if (stats != nullptr && (err = launch_stats(st, n, -1, stats, s)) != hipSuccess) return err;
        hipLaunchKernelGGL(k_mv_playout<G>, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies, (uint32_t)seed,
                           (uint32_t)(seed >> 32), gid_base, gid, reward, terminal);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (stats != nullptr) return launch_stats(st, n, +1, stats, s);
        return hipSuccess;
    }
    static hipError_t persist(const MixedArgs &a, int slots, hipStream_t s)
    {
        hipLaunchKernelGGL(k_persist_lane<DiagLane<G>>, dim3((unsigned)((slots + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                           s, a);
        return hipGetLastError();
    }
    static constexpr GameOps ops()
    {
        return GameOps{G::KIND, G::H, G::W, G::CELLS, G::A, &init, &mask, &step, &random_step, &policy_step,
                       &playout, &persist, 0, nullptr, -1, -1};
    }
};

} // namespace lx
