// kernels.hpp -- HIP kernels of the batched step and the fused random playout.
//
// One environment per lane, 64-lane workgroups (one wave).  A workgroup
// owns a contiguous run of 64 environments: their int8 boards are copied
// HBM -> LDS with 16-byte loads (the run starts 16-byte aligned because 64
// boards of any size are a multiple of 16 bytes), each lane then packs its
// own board into bitboards in VGPRs.  Scalars (to_move, status, ...) are
// read and written per lane, which is coalesced because they are
// structure-of-arrays.
//
//   k_init     start positions, 16-byte stores
//   k_mask     legal mask [n][A], staged through LDS for coalesced stores
//   k_step     one ply per env for a caller-chosen action; board delta
//              written in place, optional next mask
//   k_playout  the whole uniform-random game in registers: mask -> Philox
//              -> k-th legal action -> apply -> end rules, until every lane
//              of the wave has ended; final board written back through LDS
//   k_playout_hex  the same result for Hex by fill-then-resolve
//   k_stats    step and outcome counters (a difference of two reductions)
#pragma once

#include <type_traits>

#include "games.hpp"
#include "ludax_internal.hpp"

namespace lx {

constexpr int BLOCK = 64;

enum : int { RUNNING = 0, TERMINAL = 1, TRUNCATED = 2, ILLEGAL = 3 };

// Copy the boards of envs [e0, e0 + nb) from HBM to LDS (raw bytes).
template <int CELLS>
__device__ __forceinline__ void stage_in(const int8_t *__restrict__ board, int64_t e0, int nb,
                                         int8_t *lds)
{
    const int8_t *src = board + e0 * CELLS;
    const int bytes = nb * CELLS;
    const int full = bytes >> 4;
    for (int j = threadIdx.x; j < full; j += BLOCK)
        reinterpret_cast<uint4 *>(lds)[j] = reinterpret_cast<const uint4 *>(src)[j];
    for (int j = (full << 4) + threadIdx.x; j < bytes; j += BLOCK) lds[j] = src[j];
    __syncthreads();
}

// Copy `bytes` bytes from LDS to HBM at dst (16-byte aligned).
__device__ __forceinline__ void stage_out(int8_t *__restrict__ dst, int bytes, const int8_t *lds)
{
    __syncthreads();
    const int full = bytes >> 4;
    for (int j = threadIdx.x; j < full; j += BLOCK)
        reinterpret_cast<uint4 *>(dst)[j] = reinterpret_cast<const uint4 *>(lds)[j];
    for (int j = (full << 4) + threadIdx.x; j < bytes; j += BLOCK) dst[j] = lds[j];
}

// One lane's board bytes (LDS) -> cell-indexed bitboards of both players.
template <int CELLS, int NWC>
__device__ __forceinline__ void read_board(const int8_t *p, BB<NWC> &c1, BB<NWC> &c2)
{
    static_for<NWC>([&](auto I) {
        constexpr int i = I;
        uint32_t a = 0u, b = 0u;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const int c = 32 * i + j;
            if (c < CELLS) {
                const uint32_t v = (uint8_t)p[c];
                a |= (v & 1u) << j;
                b |= ((v >> 1) & 1u) << j;
            }
        }
        c1.w[i] = a;
        c2.w[i] = b;
    });
}

template <int CELLS, int NWC>
__device__ __forceinline__ void write_board(int8_t *p, const BB<NWC> &c1, const BB<NWC> &c2)
{
    static_for<NWC>([&](auto I) {
        constexpr int i = I;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const int c = 32 * i + j;
            if (c < CELLS) p[c] = (int8_t)(((c1.w[i] >> j) & 1u) | (((c2.w[i] >> j) & 1u) << 1));
        }
    });
}

// Legal mask row (A bytes) of one lane into LDS.
template <class G>
__device__ __forceinline__ void write_mask_row(int8_t *p, const typename G::M &m, bool pass_legal)
{
    const BB<G::NWC> c = G::to_canon(m);
    static_for<G::NWC>([&](auto I) {
        constexpr int i = I;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const int a = 32 * i + j;
            if (a < G::CELLS) p[a] = (int8_t)((c.w[i] >> j) & 1u);
        }
    });
    if constexpr (G::HAS_PASS) p[G::CELLS] = pass_legal ? 1 : 0;
}

// ---------------------------------------------------------------------------
// a1: start positions
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(256) void k_init(DevState st, int64_t n)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t bytes = n * G::CELLS;
    const int64_t chunks = bytes >> 4;
    for (int64_t j = tid; j < chunks; j += stride) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (G::KIND == 4) {
            // 64-byte boards; chunk j holds rows 2q and 2q+1, q = j % 4.  Row 3
            // (D4 = 2, E4 = 1) is bytes 8..15 of chunk 1, row 4 (D5 = 1, E5 = 2)
            // bytes 0..7 of chunk 2.
            const int q = (int)(j & 3);
            if (q == 1) { v.z = 0x02000000u; v.w = 0x00000001u; }
            if (q == 2) { v.x = 0x01000000u; v.y = 0x00000002u; }
        }
        reinterpret_cast<uint4 *>(st.board)[j] = v;
    }
    for (int64_t j = (chunks << 4) + tid; j < bytes; j += stride) st.board[j] = 0;
    for (int64_t e = tid; e < n; e += stride) {
        st.to_move[e] = 1;
        st.status[e] = RUNNING;
        st.winner[e] = -1;
        st.passes[e] = 0;
        st.ply[e] = 0;
        st.last_action[e] = -1;
    }
}

// ---------------------------------------------------------------------------
// a2: legal mask
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_mask(DevState st, int64_t n, uint8_t *__restrict__ mask)
{
    constexpr int LB = (G::CELLS > G::A ? G::CELLS : G::A);
    __shared__ __align__(16) int8_t lds[BLOCK * LB];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<G::CELLS>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const bool valid = t < nb;
    // every lane reads (lanes past the batch end read env e0 and an unused
    // LDS row, and are then ignored), which keeps the state in registers
    const int64_t ec = valid ? e0 + t : e0;
    BB<G::NWC> c1, c2;
    read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
    G g;
    g.load(c1, c2);
    const int me = st.to_move[ec];
    const bool running = valid && st.status[ec] == RUNNING;
    typename G::M m = bb_zero<G::NWI>();
    if (running) m = g.placements(me);
    const bool pass_legal = G::HAS_PASS && running && !any(m);
    __syncthreads();
    if (valid) write_mask_row<G>(lds + t * G::A, m, pass_legal);
    stage_out(reinterpret_cast<int8_t *>(mask) + e0 * G::A, nb * G::A, lds);
}

// ---------------------------------------------------------------------------
// a4-a6 for a given action: ludax_step
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_step(DevState st, int64_t n, int max_plies,
                                                const int32_t *__restrict__ action,
                                                int8_t *__restrict__ reward,
                                                uint8_t *__restrict__ terminal,
                                                uint8_t *__restrict__ next_mask)
{
    constexpr int LB = (G::CELLS > G::A ? G::CELLS : G::A);
    __shared__ __align__(16) int8_t lds[BLOCK * LB];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<G::CELLS>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    BB<G::NWC> c1, c2;
    read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
    G g;
    g.load(c1, c2);
    int me = st.to_move[ec], status = valid ? (int)st.status[ec] : ILLEGAL, winner = st.winner[ec];
    int passes = st.passes[ec], ply = st.ply[ec], last = st.last_action[ec];
    const int a = action[ec];
    int r1 = 0, r2 = 0;
    bool changed = false;
    if (valid && status == RUNNING) {
        const typename G::M m = g.placements(me);
        const bool is_pass = G::HAS_PASS && a == G::A - 1;
        bool legal;
        if (is_pass) legal = !any(m);
        else legal = a >= 0 && a < G::CELLS && test_bit(m, G::bit_of(a));
        if (!legal) {
            status = ILLEGAL;
        } else {
            int outcome;
            if (is_pass) {
                outcome = g.pass(passes);
            } else {
                outcome = g.place_step(G::bit_of(a), me);
                passes = 0;
                changed = true;
            }
            ply += 1;
            last = a;
            if (outcome >= 0) {
                status = TERMINAL;
                winner = outcome;
                r1 = outcome == 1 ? 1 : (outcome == 2 ? -1 : 0);
                r2 = -r1;
            } else {
                me = 3 - me;
                if (ply >= max_plies) {
                    status = TRUNCATED;
                    winner = -1;
                }
            }
        }
    }
    if (valid) {
        st.to_move[e] = (int8_t)me;
        st.status[e] = (int8_t)status;
        st.winner[e] = (int8_t)winner;
        st.passes[e] = (int8_t)passes;
        st.ply[e] = (int16_t)ply;
        st.last_action[e] = (int16_t)last;
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = status != RUNNING ? 1 : 0;
    }
    if constexpr (G::KIND == 4) {
        // flips can touch any cell: write whole boards (64 B per env) back
        __syncthreads();
        if (valid) {
            BB<G::NWC> c1, c2;
            g.store(c1, c2);
            write_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
        }
        stage_out(st.board + e0 * G::CELLS, nb * G::CELLS, lds);
    } else {
        // a placement changes one cell: the mover (to_move has advanced
        // unless the game ended) wrote its stone at the action's cell
        if (valid && changed) {
            const int mover = status == TERMINAL ? me : 3 - me;
            st.board[e * G::CELLS + a] = (int8_t)mover;
        }
    }
    if (next_mask != nullptr) {
        typename G::M m = bb_zero<G::NWI>();
        const bool running = valid && status == RUNNING;
        if (running) m = g.placements(me);
        const bool pass_legal = G::HAS_PASS && running && !any(m);
        __syncthreads();
        if (valid) write_mask_row<G>(lds + t * G::A, m, pass_legal);
        stage_out(reinterpret_cast<int8_t *>(next_mask) + e0 * G::A, nb * G::A, lds);
    }
}

// ---------------------------------------------------------------------------
// a2-a8 fused: uniform-random playout to the end of every game
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_playout(DevState st, int64_t n, int max_plies,
                                                   uint32_t key0, uint32_t key1, int64_t gid_base,
                                                   const int64_t *__restrict__ gid,
                                                   int8_t *__restrict__ reward,
                                                   uint8_t *__restrict__ terminal)
{
    __shared__ __align__(16) int8_t lds[BLOCK * G::CELLS];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<G::CELLS>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    BB<G::NWC> c1, c2;
    read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
    G g;
    g.load(c1, c2);
    int me = st.to_move[ec], status = valid ? (int)st.status[ec] : ILLEGAL, winner = st.winner[ec];
    int passes = st.passes[ec], ply = st.ply[ec], last = st.last_action[ec];
    const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
    const bool was_running = valid && status == RUNNING;
    if (was_running) g.prepare();
    const uint32_t id_lo = (uint32_t)id, id_hi = (uint32_t)(id >> 32);

    int r1 = 0, r2 = 0;
    // Philox words are consumed in order; w0 is the word of the current
    // ply.  A block serves plies 4q .. 4q+3; the first block may be entered
    // part-way when the starting ply is not a multiple of four.
    uint32_t w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
    if (was_running) {
        const Philox4 f = philox4x32_10((uint32_t)ply >> 2, id_lo, id_hi, 0u, key0, key1);
        const int r = ply & 3;
        w0 = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
        w1 = r == 0 ? f.v[1] : (r == 1 ? f.v[2] : f.v[3]);
        w2 = r == 0 ? f.v[2] : f.v[3];
        w3 = f.v[3];
    }
    bool running = was_running;
    bool first = true;
    while (running) {
        const typename G::M m = g.placements(me);
        const int np = popcount(m);
        const int nl = G::HAS_PASS ? (np > 0 ? np : 1) : np;
        if (nl == 0) { // only reachable from a hand-edited board
            status = ILLEGAL;
            break;
        }
        if ((ply & 3) == 0 && !first) {
            const Philox4 f = philox4x32_10((uint32_t)ply >> 2, id_lo, id_hi, 0u, key0, key1);
            w0 = f.v[0];
            w1 = f.v[1];
            w2 = f.v[2];
            w3 = f.v[3];
        }
        first = false;
        const int k = (int)__umulhi(w0, (uint32_t)nl);
        w0 = w1;
        w1 = w2;
        w2 = w3;
        int outcome, a;
        if (G::HAS_PASS && np == 0) {
            a = G::A - 1;
            outcome = g.pass(passes);
        } else {
            const int b = select_bit(m, k);
            a = G::action_of(b);
            outcome = g.place(b, me);
            passes = 0;
        }
        ply += 1;
        last = a;
        if (outcome >= 0) {
            status = TERMINAL;
            winner = outcome;
            r1 = outcome == 1 ? 1 : (outcome == 2 ? -1 : 0);
            r2 = -r1;
            running = false;
        } else {
            me = 3 - me;
            if (ply >= max_plies) {
                status = TRUNCATED;
                winner = -1;
                running = false;
            }
        }
    }
    if (valid) {
        BB<G::NWC> c1, c2;
        g.store(c1, c2);
        write_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
        st.to_move[e] = (int8_t)me;
        st.status[e] = (int8_t)status;
        st.winner[e] = (int8_t)winner;
        st.passes[e] = (int8_t)passes;
        st.ply[e] = (int16_t)ply;
        st.last_action[e] = (int16_t)last;
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = 1;
    }
    stage_out(st.board + e0 * G::CELLS, nb * G::CELLS, lds);
}

// ---------------------------------------------------------------------------
// The random sequence of a window of T plies, without any end test: ply j
// (from ply0) is played by the owner of `cur` for even j and of `oth` for
// odd j, on a uniformly drawn cell of G::open_cells, and its internal bit is
// recorded in moves[j * BLOCK + lane].  One Philox block serves the plies
// 4q .. 4q+3; the window is cut into a head (up to the next multiple of
// four), whole blocks of four plies and a tail, so that no ply tests
// whether it needs a new block.  On return cur / oth again hold the stones
// of the player who moved first / second.
// ---------------------------------------------------------------------------
template <class G, class E>
__device__ __forceinline__ void fill_window(typename G::M &cur, typename G::M &oth, int T, int ply0,
                                            uint32_t id_lo, uint32_t id_hi, uint32_t key0, uint32_t key1,
                                            E *moves, int t)
{
    using M = typename G::M;
    auto play = [&](M &mine, const M &theirs, int j, uint32_t w) {
        const int b = select_uniform(G::open_cells(mine, theirs), w);
        moves[j * BLOCK + t] = (E)b;
        mine = mine | onehot<G::NWI>(b);
    };
    auto swap_sides = [&]() {
        const M x = cur;
        cur = oth;
        oth = x;
    };
    int j = 0;
    const int r0 = ply0 & 3;
    const int head = r0 == 0 ? 0 : (T < 4 - r0 ? T : 4 - r0);
    if (head > 0) {
        const Philox4 f = philox4x32_10((uint32_t)ply0 >> 2, id_lo, id_hi, 0u, key0, key1);
        for (; j < head; ++j) {
            const int wi = r0 + j;
            play(cur, oth, j, wi == 1 ? f.v[1] : (wi == 2 ? f.v[2] : f.v[3]));
            swap_sides();
        }
    }
    for (; j + 4 <= T; j += 4) {
        const Philox4 f = philox4x32_10((uint32_t)(ply0 + j) >> 2, id_lo, id_hi, 0u, key0, key1);
        play(cur, oth, j, f.v[0]);
        play(oth, cur, j + 1, f.v[1]);
        play(cur, oth, j + 2, f.v[2]);
        play(oth, cur, j + 3, f.v[3]);
    }
    if (j < T) {
        const Philox4 f = philox4x32_10((uint32_t)(ply0 + j) >> 2, id_lo, id_hi, 0u, key0, key1);
        for (int i = 0; j < T; ++j, ++i) {
            play(cur, oth, j, i == 0 ? f.v[0] : (i == 1 ? f.v[1] : f.v[2]));
            swap_sides();
        }
    }
    // cur belongs to the player to move after the window; give it back to
    // the player who moved first
    if (T & 1) swap_sides();
}

// ---------------------------------------------------------------------------
// a2-a7 fused for Hex: fill, then resolve.
//
// Which cells get played does not depend on whether the game has already
// been won: the legal set is "every empty cell" either way.  So each lane
// first plays its random sequence until the board is full (or max_plies),
// with no end test at all, recording the cell of every ply in LDS.  Then it
// finds the ply at which the game really ended.  Connection of a player's
// stones only grows as stones are added, a full board has exactly one
// connected player, and two opposing chains cannot both cross, so: the
// winner W is the player connected at the end of the window, and the end
// ply is W's m*-th move for the smallest m* whose prefix of W's moves
// connects -- found by binary search, each probe a flood from W's first
// side that restarts from the largest prefix already known not to connect.
// Finally the moves after the end ply are taken off the board again.  The
// per-ply work drops to mask, draw, select and place; the connection floods
// run once per game instead of being the per-ply maximum over the 64 lanes.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(BLOCK) void k_playout_hex(DevState st, int64_t n, int max_plies,
                                                       uint32_t key0, uint32_t key1, int64_t gid_base,
                                                       const int64_t *__restrict__ gid,
                                                       int8_t *__restrict__ reward,
                                                       uint8_t *__restrict__ terminal)
{
    using G = Hex<N>;
    using M = typename G::M;
    constexpr int NW = G::NWI;
    using E = typename std::conditional<(G::CELLS <= 256), uint8_t, uint16_t>::type;
    constexpr int STAGE = BLOCK * G::CELLS;
    constexpr int LIST = BLOCK * G::CELLS * (int)sizeof(E);
    __shared__ __align__(16) int8_t lds[STAGE > LIST ? STAGE : LIST];
    E *moves = reinterpret_cast<E *>(lds); // moves[j * BLOCK + lane]: cell of window ply j

    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<G::CELLS>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    M b1, b2;
    read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, b1, b2);
    int me = st.to_move[ec], status = valid ? (int)st.status[ec] : ILLEGAL, winner = st.winner[ec];
    int passes = st.passes[ec], ply = st.ply[ec], last = st.last_action[ec];
    const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
    __syncthreads(); // the staging area becomes the move list

    const bool run = valid && status == RUNNING;
    const int empties = run ? G::CELLS - popcount(b1 | b2) : 0;
    const int room = max_plies - ply > 1 ? max_plies - ply : 1;
    const int T = empties < room ? empties : room; // plies in the window
    const int me0 = me, ply0 = ply;
    const uint32_t id_lo = (uint32_t)id, id_hi = (uint32_t)(id >> 32);

    // ---- fill: the random sequence, no end test ----
    M cur = pick(me0 == 1, b1, b2); // stones of the player to move at ply0
    M oth = pick(me0 == 1, b2, b1);
    fill_window<G>(cur, oth, T, ply0, id_lo, id_hi, key0, key1, moves, t);
    const M end1 = pick(me0 == 1, cur, oth); // boards after the window
    const M end2 = pick(me0 == 1, oth, cur);

    // ---- resolve: who connected, and at which ply ----
    int W = 0;
    if (T > 0) {
        if (G::joins(end1, 1)) W = 1;
        else if (empties == T || G::joins(end2, 2)) W = 2; // a full board always has a winner
    }
    const int jw0 = W == me0 ? 0 : 1;          // W's first ply in the window
    const int MW = W ? (T - jw0 + 1) >> 1 : 0; // W's moves in the window
    int jstar = -1;
    if (MW > 0) {
        M s_lo = pick(W == 1, b1, b2); // W's stones before its lo-th window move
        M r_lo = G::flood(G::first_side(s_lo, W), s_lo);
        int lo = 1, hi = MW, next = 1; // next = first move not yet in s_lo
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            M s = s_lo;
            for (int k = next; k <= mid; ++k) s = s | onehot<NW>((int)moves[(jw0 + 2 * (k - 1)) * BLOCK + t]);
            M r = r_lo | G::first_side(s, W);
            if (G::flood_to_far(r, s, W)) {
                hi = mid;
            } else {
                lo = mid + 1;
                s_lo = s;
                r_lo = r;
                next = mid + 1;
            }
        }
        jstar = jw0 + 2 * (lo - 1);
    }

    // ---- the final position ----
    const int played = jstar >= 0 ? jstar + 1 : T;
    M f1 = end1, f2 = end2;
    for (int j = played; j < T; ++j) { // take back the plies after the end
        const M x = onehot<NW>((int)moves[j * BLOCK + t]);
        const int who = ((j & 1) == 0) ? me0 : 3 - me0;
        if (who == 1) f1 = andnot(f1, x);
        else f2 = andnot(f2, x);
    }
    int r1 = 0, r2 = 0;
    if (run) {
        if (T == 0) {
            status = ILLEGAL; // RUNNING with no empty cell: only a hand-edited board
        } else {
            ply = ply0 + played;
            last = (int)moves[(played - 1) * BLOCK + t];
            if (jstar >= 0) {
                status = TERMINAL;
                winner = W;
                me = W;
                r1 = W == 1 ? 1 : -1;
                r2 = -r1;
            } else {
                me = (T & 1) ? 3 - me0 : me0;
                status = ply >= max_plies ? TRUNCATED : ILLEGAL;
            }
        }
    }
    __syncthreads(); // the move list becomes the staging area again
    if (valid) {
        write_board<G::CELLS, G::NWC>(lds + t * G::CELLS, f1, f2);
        st.to_move[e] = (int8_t)me;
        st.status[e] = (int8_t)status;
        st.winner[e] = (int8_t)winner;
        st.passes[e] = (int8_t)passes;
        st.ply[e] = (int16_t)ply;
        st.last_action[e] = (int16_t)last;
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = 1;
    }
    stage_out(st.board + e0 * G::CELLS, nb * G::CELLS, lds);
}

// ---------------------------------------------------------------------------
// a2-a7 fused for the line games (Tic-Tac-Toe, Connect Four): fill, then
// resolve.  As for Hex, the legal set does not depend on whether the game
// is over (empty cells; Connect Four: empty cells resting on the floor or a
// piece), so each lane plays its random sequence to the end of the window
// first.  "Some player holds a line of n or more" only becomes true by the
// owner's own placement and then stays true, so the ply that ended the
// game is the first prefix of the window at which it holds -- found by
// binary search over the window, each probe two shift-AND line tests.
// Without a line, a full board is a draw (wins are tested before draws).
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(BLOCK) void k_playout_lines(DevState st, int64_t n, int max_plies,
                                                         uint32_t key0, uint32_t key1, int64_t gid_base,
                                                         const int64_t *__restrict__ gid,
                                                         int8_t *__restrict__ reward,
                                                         uint8_t *__restrict__ terminal)
{
    using M = typename G::M;
    constexpr int NW = G::NWI;
    using E = uint8_t; // internal bit indices are below 64
    __shared__ __align__(16) int8_t lds[BLOCK * G::CELLS];
    E *moves = reinterpret_cast<E *>(lds); // moves[j * BLOCK + lane]: internal bit of window ply j

    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<G::CELLS>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    BB<G::NWC> c1, c2;
    read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
    const M b1 = G::from_canon(c1), b2 = G::from_canon(c2);
    int me = st.to_move[ec], status = valid ? (int)st.status[ec] : ILLEGAL, winner = st.winner[ec];
    int passes = st.passes[ec], ply = st.ply[ec], last = st.last_action[ec];
    const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
    __syncthreads(); // the staging area becomes the move list

    const bool run = valid && status == RUNNING;
    const int empties = run ? G::CELLS - popcount(b1 | b2) : 0;
    const int room = max_plies - ply > 1 ? max_plies - ply : 1;
    const int me0 = me, ply0 = ply;
    const uint32_t id_lo = (uint32_t)id, id_hi = (uint32_t)(id >> 32);
    // the window ends where the board is full, at max_plies, or where no
    // legal cell is left (Connect Four columns fill; equal to "full" here)
    const int T = empties < room ? empties : room;

    M cur = pick(me0 == 1, b1, b2);
    M oth = pick(me0 == 1, b2, b1);
    fill_window<G>(cur, oth, T, ply0, id_lo, id_hi, key0, key1, moves, t);
    const M end1 = pick(me0 == 1, cur, oth);
    const M end2 = pick(me0 == 1, oth, cur);

    // ---- resolve: the first prefix with a line ----
    int jstar = -1;
    if (T > 0 && (G::line(end1) | G::line(end2))) {
        M s1 = b1, s2 = b2; // stones before window ply lo
        int lo = 0, hi = T - 1, next = 0;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            M a1 = s1, a2 = s2;
            for (int j = next; j <= mid; ++j) {
                const M x = onehot<NW>((int)moves[j * BLOCK + t]);
                const bool p1 = ((j & 1) == 0) == (me0 == 1);
                a1 = pick(p1, a1 | x, a1);
                a2 = pick(p1, a2, a2 | x);
            }
            if (G::line(a1) | G::line(a2)) {
                hi = mid;
            } else {
                lo = mid + 1;
                s1 = a1;
                s2 = a2;
                next = mid + 1;
            }
        }
        jstar = lo;
    }

    // ---- the final position ----
    const int played = jstar >= 0 ? jstar + 1 : T;
    M f1 = end1, f2 = end2;
    for (int j = played; j < T; ++j) { // take back the plies after the end
        const M x = onehot<NW>((int)moves[j * BLOCK + t]);
        const bool p1 = ((j & 1) == 0) == (me0 == 1);
        f1 = pick(p1, andnot(f1, x), f1);
        f2 = pick(p1, f2, andnot(f2, x));
    }
    int r1 = 0, r2 = 0;
    if (run) {
        if (T == 0) {
            status = ILLEGAL; // RUNNING with no empty cell: only a hand-edited board
        } else {
            ply = ply0 + played;
            last = G::action_of((int)moves[(played - 1) * BLOCK + t]);
            const int mover = ((played - 1) & 1) == 0 ? me0 : 3 - me0; // of the last ply
            if (jstar >= 0) {
                status = TERMINAL;
                winner = mover;
                me = mover;
                r1 = mover == 1 ? 1 : -1;
                r2 = -r1;
            } else if (T == empties) {
                status = TERMINAL; // full board without a line: draw
                winner = 0;
                me = mover;
            } else {
                me = 3 - mover;
                status = TRUNCATED;
            }
        }
    }
    __syncthreads(); // the move list becomes the staging area again
    if (valid) {
        write_board<G::CELLS, G::NWC>(lds + t * G::CELLS, G::to_canon(f1), G::to_canon(f2));
        st.to_move[e] = (int8_t)me;
        st.status[e] = (int8_t)status;
        st.winner[e] = (int8_t)winner;
        st.passes[e] = (int8_t)passes;
        st.ply[e] = (int16_t)ply;
        st.last_action[e] = (int16_t)last;
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = 1;
    }
    stage_out(st.board + e0 * G::CELLS, nb * G::CELLS, lds);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <class G>
struct Launch {
    static hipError_t init(const DevState &st, int64_t n, hipStream_t s)
    {
        const int64_t work = (n * G::CELLS + 15) / 16 > n ? (n * G::CELLS + 15) / 16 : n;
        int64_t blocks = (work + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_init<G>, dim3((unsigned)blocks), dim3(256), 0, s, st, n);
        return hipGetLastError();
    }
    static hipError_t mask(const DevState &st, int64_t n, uint8_t *mask, hipStream_t s)
    {
        const int64_t blocks = (n + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL(k_mask<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n, mask);
        return hipGetLastError();
    }
    static hipError_t step(const DevState &st, int64_t n, int max_plies, const int32_t *action,
                           int8_t *reward, uint8_t *terminal, uint8_t *next_mask, hipStream_t s)
    {
        const int64_t blocks = (n + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL(k_step<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n, max_plies,
                           action, reward, terminal, next_mask);
        return hipGetLastError();
    }
    static hipError_t playout(const DevState &st, int64_t n, int max_plies, uint64_t seed,
                              int64_t gid_base, const int64_t *gid, int8_t *reward,
                              uint8_t *terminal, int64_t *stats, hipStream_t s)
    {
        const int64_t blocks = (n + BLOCK - 1) / BLOCK;
        hipError_t err = hipSuccess;
        if (stats != nullptr && (err = launch_stats(st, n, -1, stats, s)) != hipSuccess) return err;
        if constexpr (G::KIND == 3) {
            hipLaunchKernelGGL(k_playout_hex<G::H>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n,
                               max_plies, (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid, reward,
                               terminal);
        } else if constexpr (G::KIND == 1 || G::KIND == 2) {
            hipLaunchKernelGGL(k_playout_lines<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n,
                               max_plies, (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid, reward,
                               terminal);
        } else {
            hipLaunchKernelGGL(k_playout<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n, max_plies,
                               (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid, reward, terminal);
        }
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (stats != nullptr) return launch_stats(st, n, +1, stats, s);
        return hipSuccess;
    }
    static constexpr GameOps ops()
    {
        return GameOps{G::KIND, G::H, G::W, G::CELLS, G::A, &init, &mask, &step, &playout};
    }
};

} // namespace lx

namespace lx {

// Table of GameOps for the sizes N = LO .. HI of a size-templated game.
template <template <int> class G, int LO, int... I>
const GameOps *ops_in_range(int n, std::integer_sequence<int, I...>)
{
    static const GameOps table[] = {Launch<G<LO + I>>::ops()...};
    const int i = n - LO;
    return (i >= 0 && i < (int)sizeof...(I)) ? &table[i] : nullptr;
}

template <template <int> class G, int LO, int HI>
const GameOps *ops_range(int n)
{
    return ops_in_range<G, LO>(n, std::make_integer_sequence<int, HI - LO + 1>{});
}

} // namespace lx
