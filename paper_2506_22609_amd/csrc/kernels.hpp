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
//   k_step     one ply per env for a caller-chosen action, the uniform
//              random one, or one drawn from given logits; board delta
//              written in place, optional next mask
//   k_playout  the whole uniform-random game in registers: mask -> Philox
//              -> k-th legal action -> apply -> end rules, until every lane
//              of the wave has ended; final board written back through LDS
//   k_playout_fill  the same result for Hex, Tic-Tac-Toe and Connect Four by
//              fill-then-resolve (random fill, then a binary search of the end)
//   k_persist_ply / k_persist_fill  the mixed persistent batch (and
//              k_persist_lane for the movement games)
//   k_stats    step and outcome counters (a difference of two reductions)
#pragma once

#include <type_traits>

#include "games.hpp"
#include "hexaux.hpp"
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
// The lane's row starts at any byte offset, so it is read as the aligned
// dwords that cover it (one more than its length, hence the 16 bytes of
// slack behind every staging array) and each 4-cell group is realigned with
// v_alignbyte; a dot product of the group's low (high) bits with the byte
// weights 1, 2, 4, 8 packs the four cells of player 1 (player 2) into one
// nibble.
constexpr int STAGE_SLACK = 16;

template <int CELLS, int NWC>
__device__ __forceinline__ void read_board(const int8_t *p, BB<NWC> &c1, BB<NWC> &c2)
{
    constexpr int G4 = (CELLS + 3) / 4;                                    // 4-cell groups
    constexpr uint32_t LAST = CELLS % 4 == 0 ? 0xFFFFFFFFu : (1u << (8 * (CELLS % 4))) - 1u;
    const uint32_t off = (uint32_t)(uintptr_t)p & 3u;
    const uint32_t *q = reinterpret_cast<const uint32_t *>(p - off);
    uint32_t lo = q[0];
    static_for<NWC>([&](auto I) {
        constexpr int i = I;
        uint32_t a = 0u, b = 0u;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * i + j;
            if (k < G4) {
                const uint32_t hi = q[k + 1];
                uint32_t v = __builtin_amdgcn_alignbyte(hi, lo, off);
                if (k == G4 - 1) v &= LAST;
                lo = hi;
                a |= __builtin_amdgcn_udot4(v & 0x01010101u, 0x08040201u, 0u, false) << (4 * j);
                b |= (__builtin_amdgcn_udot4(v & 0x02020202u, 0x08040201u, 0u, false) >> 1) << (4 * j);
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
    __shared__ __align__(16) int8_t lds[BLOCK * LB + STAGE_SLACK];
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

// The action of one ply of a RUNNING env with legal placements m: the
// caller's (MODE 0), the uniform-random one of a3 (MODE 1), or the policy
// draw from the softmax of the env's logits (lg: its row, in action order)
// over the legal placements (MODE 2).  `legal` reports whether the action
// may be applied, `is_pass` whether it is Reversi's PASS.
template <class G, int MODE>
__device__ __forceinline__ int choose_action(const typename G::M &m, int ply, int64_t ec,
                                             const int32_t *__restrict__ action, const float *lg,
                                             uint32_t key0, uint32_t key1, int64_t gid_base,
                                             const int64_t *__restrict__ gid, bool &legal, bool &is_pass)
{
    int a = 0;
    if constexpr (MODE >= 1) {
        // the ply's word of the game's Philox stream
        const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
        const Philox4 f = philox4x32_10((uint32_t)ply >> 2, (uint32_t)id, (uint32_t)(id >> 32), 0u, key0, key1);
        const int r = ply & 3;
        const uint32_t w = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
        const int np = popcount(m);
        is_pass = G::HAS_PASS && np == 0;
        legal = np > 0 || is_pass; // a hand-edited board may leave no action
        if constexpr (MODE == 1) {
            // uniform: the k-th legal action, k = (w * n_legal) >> 32
            if (np > 0) a = G::action_of(select_bit(m, (int)__umulhi(w, (uint32_t)np)));
        } else {
            // softmax of the logits over the legal placements (float32,
            // in increasing action order): the first action whose running
            // sum of exp(logit - max) exceeds u * total, u = (w >> 8) / 2^24
            float mx = -3.0e38f;
            for (int c = 0; c < G::CELLS; ++c)
                if (test_bit(m, G::bit_of(c))) mx = fmaxf(mx, lg[c]);
            float tot = 0.f;
            for (int c = 0; c < G::CELLS; ++c)
                if (test_bit(m, G::bit_of(c))) tot += expf(lg[c] - mx);
            const float thr = (float)(w >> 8) * 0x1p-24f * tot;
            float run = 0.f;
            int pick = -1, lastc = -1;
            for (int c = 0; c < G::CELLS; ++c)
                if (test_bit(m, G::bit_of(c))) {
                    run += expf(lg[c] - mx);
                    lastc = c;
                    if (pick < 0 && run > thr) pick = c;
                }
            if (np > 0) a = pick >= 0 ? pick : lastc;
        }
        if (is_pass) a = G::A - 1;
    } else {
        a = action[ec];
        is_pass = G::HAS_PASS && a == G::A - 1;
        if (is_pass) legal = !any(m);
        else legal = a >= 0 && a < G::CELLS && test_bit(m, G::bit_of(a));
    }
    return a;
}

// ---------------------------------------------------------------------------
// a4-a6 for one ply: ludax_step (caller-chosen action, MODE 0),
// ludax_random_step (the uniform-random action of a3, MODE 1) and
// ludax_policy_step (an action drawn from the softmax of given logits over
// the legal actions with the same Philox word, MODE 2).  The
// state stays in HBM between launches, so this kernel is bound by its bytes:
// the block's statuses are read first and a block with no RUNNING env reads
// no board; only envs that were RUNNING write their scalars back, and a
// placement writes the one cell it changed (Reversi and Pente: the whole
// board, since flips and captures change other cells).
// ---------------------------------------------------------------------------
template <class G, int MODE>
__global__ __launch_bounds__(BLOCK) void k_step(DevState st, int64_t n, int max_plies,
                                                const int32_t *__restrict__ action,
                                                const float *__restrict__ logits, uint32_t key0,
                                                uint32_t key1, int64_t gid_base,
                                                const int64_t *__restrict__ gid,
                                                int8_t *__restrict__ reward,
                                                uint8_t *__restrict__ terminal,
                                                uint8_t *__restrict__ next_mask)
{
    constexpr int LB = (G::CELLS > G::A ? G::CELLS : G::A);
    __shared__ __align__(16) int8_t lds[BLOCK * LB + STAGE_SLACK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;
    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    int status = valid ? (int)st.status[ec] : ILLEGAL;
    const bool was_running = status == RUNNING;

    if (!__syncthreads_or(was_running)) {
        // nothing to play in this block: every env is a no-op
        if (valid) {
            reward[2 * e] = 0;
            reward[2 * e + 1] = 0;
            terminal[e] = 1;
        }
        if (next_mask != nullptr) {
            uint8_t *dst = next_mask + e0 * G::A;
            const int bytes = nb * G::A, full = bytes >> 4;
            for (int j = t; j < full; j += BLOCK) reinterpret_cast<uint4 *>(dst)[j] = uint4{0u, 0u, 0u, 0u};
            for (int j = (full << 4) + t; j < bytes; j += BLOCK) dst[j] = 0;
        }
        return;
    }

    stage_in<G::CELLS>(st.board, e0, nb, lds);
    BB<G::NWC> c1, c2;
    read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
    G g;
    g.load(c1, c2);
    int me = st.to_move[ec], winner = st.winner[ec];
    int passes = st.passes[ec], ply = st.ply[ec], last = st.last_action[ec];
    int r1 = 0, r2 = 0, a = 0;
    bool changed = false;
    if (was_running) {
        const typename G::M m = g.placements(me);
        bool legal, is_pass;
        a = choose_action<G, MODE>(m, ply, ec, action, MODE == 2 ? logits + ec * G::A : nullptr, key0, key1, gid_base,
                                   gid, legal, is_pass);
        if (!legal) {
            status = ILLEGAL;
        } else {
            int outcome;
            if (is_pass) {
                outcome = g.pass(passes);
            } else {
                outcome = g.place_step(G::bit_of(a), me, passes);
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
        if (was_running) {
            st.to_move[e] = (int8_t)me;
            st.status[e] = (int8_t)status;
            st.winner[e] = (int8_t)winner;
            st.passes[e] = (int8_t)passes;
            st.ply[e] = (int16_t)ply;
            st.last_action[e] = (int16_t)last;
        }
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = status != RUNNING ? 1 : 0;
    }
    if constexpr (G::KIND == 4 || G::KIND == 7) {
        // Reversi's flips and Pente's captures can touch any cell: write
        // whole boards back
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
// The per-ply step of Hex with the aux cache (hexaux.hpp): the same three
// modes and results as k_step, but a lane reads its env's two bitboards
// from aux instead of the board, and the end test is a union-find join of
// the new stone with its same-coloured neighbours.  The board still gets
// its one-byte delta, the aux its changed stone word, the union-find
// entries and the tag.  A block with a stale env (tag mismatch) stages its
// boards and rebuilds those envs' caches first.
// ---------------------------------------------------------------------------
template <int N, int MODE>
__global__ __launch_bounds__(BLOCK) void k_step_hexaux(DevState st, int64_t n, int max_plies,
                                                       const int32_t *__restrict__ action,
                                                       const float *__restrict__ logits, uint32_t key0,
                                                       uint32_t key1, int64_t gid_base,
                                                       const int64_t *__restrict__ gid,
                                                       int8_t *__restrict__ reward,
                                                       uint8_t *__restrict__ terminal,
                                                       uint8_t *__restrict__ next_mask)
{
    using G = Hex<N>;
    using X = HexAux<N>;
    constexpr int NW = X::NWC;
    // LDS only for the next mask's coalesced rows (dynamic: 0 bytes when no
    // mask is asked for, so the per-ply loop keeps its occupancy)
    extern __shared__ __align__(16) int8_t lds_mask[];
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
            uint8_t *dst = next_mask + e0 * G::A;
            const int bytes = nb * G::A, full = bytes >> 4;
            for (int j = t; j < full; j += BLOCK) reinterpret_cast<uint4 *>(dst)[j] = uint4{0u, 0u, 0u, 0u};
            for (int j = (full << 4) + t; j < bytes; j += BLOCK) dst[j] = 0;
        }
        return;
    }

    uint8_t *ax = st.aux + ec * X::BYTES;
    uint32_t *stones = reinterpret_cast<uint32_t *>(ax + X::STONES);
    uint16_t *par = reinterpret_cast<uint16_t *>(ax + X::PARENT);
    int me = st.to_move[ec], winner = st.winner[ec];
    int ply = st.ply[ec], last = st.last_action[ec];
    BB<NW> p1 = bb_zero<NW>(), p2 = bb_zero<NW>();
    bool stale = false;
    if (was_running) {
        // the tag and the stones in one round of loads
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            p1.w[i] = stones[i];
            p2.w[i] = stones[NW + i];
        }
        stale = *reinterpret_cast<const uint32_t *>(ax) != aux_tag(ply, last);
        if (stale) {
            p1 = bb_zero<NW>();
            p2 = bb_zero<NW>();
            // the state was changed without this cache: rebuild it from the
            // board (byte reads; a rare path)
            const int8_t *brow = st.board + ec * G::CELLS;
            static_for<NW>([&](auto I) {
                constexpr int i = I;
#pragma unroll 4
                for (int j = 0; j < 32 && 32 * i + j < G::CELLS; ++j) {
                    const int v = brow[32 * i + j];
                    p1.w[i] |= (v == 1 ? 1u : 0u) << j;
                    p2.w[i] |= (v == 2 ? 1u : 0u) << j;
                }
            });
            uf_build<N>(par, p1, 1);
            uf_build<N>(par, p2, 2);
        }
    }
    int r1 = 0, r2 = 0, a = 0;
    bool changed = false;
    if (was_running) {
        const BB<NW> m = G::open_cells(p1, p2);
        bool legal, is_pass;
        a = choose_action<G, MODE>(m, ply, ec, action, MODE == 2 ? logits + ec * G::A : nullptr, key0, key1, gid_base,
                                   gid, legal, is_pass);
        if (!legal) {
            status = ILLEGAL;
        } else {
            const bool me_was1 = me == 1;
            const bool won = uf_place<N>(par, me_was1 ? p1 : p2, a, me);
            if (me_was1) p1 = p1 | onehot<NW>(a);
            else p2 = p2 | onehot<NW>(a);
            changed = true;
            ply += 1;
            last = a;
            if (won) {
                status = TERMINAL;
                winner = me;
                r1 = me == 1 ? 1 : -1;
                r2 = -r1;
            } else {
                me = 3 - me;
                if (ply >= max_plies) {
                    status = TRUNCATED;
                    winner = -1;
                }
            }
            if (stale) {
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    stones[i] = p1.w[i];
                    stones[NW + i] = p2.w[i];
                }
            } else {
                // the changed word, selected from registers
                const BB<NW> &own = me_was1 ? p1 : p2;
                uint32_t wv = 0u;
#pragma unroll
                for (int i = 0; i < NW; ++i) wv |= (i == (a >> 5)) ? own.w[i] : 0u;
                stones[(me_was1 ? 0 : NW) + (a >> 5)] = wv;
            }
            *reinterpret_cast<uint32_t *>(ax) = aux_tag(ply, last);
        }
    }
    if (valid) {
        if (was_running) {
            st.to_move[e] = (int8_t)me;
            st.status[e] = (int8_t)status;
            st.winner[e] = (int8_t)winner;
            st.ply[e] = (int16_t)ply;
            st.last_action[e] = (int16_t)last;
        }
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)r2;
        terminal[e] = status != RUNNING ? 1 : 0;
        if (changed) st.board[e * G::CELLS + a] = (int8_t)(status == TERMINAL ? me : 3 - me);
    }
    if (next_mask != nullptr) {
        BB<NW> m = bb_zero<NW>();
        const bool running = valid && status == RUNNING;
        if (running) m = G::open_cells(p1, p2);
        if (valid) write_mask_row<G>(lds_mask + t * G::A, m, false);
        stage_out(reinterpret_cast<int8_t *>(next_mask) + e0 * G::A, nb * G::A, lds_mask);
    }
}

// The aux caches of envs [0, n) from their boards (ludax_init with aux: the
// start position; ludax_aux_sync: whatever the boards hold).  One env per
// lane, 64-env blocks.
template <int N, bool FROM_BOARD>
__global__ __launch_bounds__(BLOCK) void k_hexaux_sync(DevState st, int64_t n)
{
    using G = Hex<N>;
    using X = HexAux<N>;
    constexpr int NW = X::NWC;
    __shared__ __align__(16) int8_t lds[BLOCK * G::CELLS + STAGE_SLACK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    const bool valid = t < nb;
    const int64_t ec = valid ? e0 + t : e0;
    BB<NW> p1 = bb_zero<NW>(), p2 = bb_zero<NW>();
    if constexpr (FROM_BOARD) {
        stage_in<G::CELLS>(st.board, e0, nb, lds);
        read_board<G::CELLS, NW>(lds + t * G::CELLS, p1, p2);
    }
    if (!valid) return;
    uint8_t *ax = st.aux + ec * X::BYTES;
    uint32_t *stones = reinterpret_cast<uint32_t *>(ax + X::STONES);
    uint16_t *par = reinterpret_cast<uint16_t *>(ax + X::PARENT);
    if constexpr (FROM_BOARD) {
        uf_build<N>(par, p1, 1);
        uf_build<N>(par, p2, 2);
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        stones[i] = p1.w[i];
        stones[NW + i] = p2.w[i];
    }
    *reinterpret_cast<uint32_t *>(ax) = FROM_BOARD ? aux_tag(st.ply[ec], st.last_action[ec]) : aux_tag(0, -1);
}

// The draw of ludax_policy_step for one board by the 64 lanes of a wave
// (lg: its logits in action order, brow: its board bytes; cells <= 128, two
// per lane, the legal actions the empty cells).  The same float32 values in
// the same order as choose_action MODE 2: the maximum over the legal cells
// (a wave reduction, exact in any order), exp(logit - max) per cell, the
// running sum in increasing cell order (one uniform add per legal cell,
// the sum so far recorded at that cell's lane), the threshold u * total;
// the first legal cell whose running sum exceeds it, by a ballot (the last
// legal cell if none).  Uniform result; -1 when no cell is empty.
template <int CELLS>
__device__ __forceinline__ int wave_policy_draw(const float *lg, const int8_t *brow, uint32_t w)
{
    static_assert(CELLS <= 128, "two cells per lane");
    const int lane = threadIdx.x & 63;
    const bool l0 = lane < CELLS && brow[lane] == 0;
    const bool l1 = lane + 64 < CELLS && brow[lane + 64] == 0;
    const float g0 = l0 ? lg[lane] : -3.0e38f, g1 = l1 ? lg[lane + 64] : -3.0e38f;
    float mx = fmaxf(-3.0e38f, fmaxf(g0, g1));
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) mx = fmaxf(mx, __shfl_xor(mx, sft));
    const float e0 = l0 ? expf(g0 - mx) : 0.f, e1 = l1 ? expf(g1 - mx) : 0.f;
    const uint64_t m0 = __ballot(l0), m1 = __ballot(l1);
    if ((m0 | m1) == 0) return -1;
    float run = 0.f, r0 = 0.f, r1 = 0.f;
    for (int c = 0; c < CELLS; ++c) {
        const bool hi = c >= 64;
        const int k = hi ? c - 64 : c;
        if (((hi ? m1 : m0) >> k) & 1u) {
            const float ec = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hi ? e1 : e0), k));
            run += ec;
            if (lane == k) {
                if (hi) r1 = run;
                else r0 = run;
            }
        }
    }
    const float thr = (float)(w >> 8) * 0x1p-24f * run;
    const uint64_t h0 = __ballot(l0 && r0 > thr), h1 = __ballot(l1 && r1 > thr);
    if (h0) return __builtin_ctzll(h0);
    if (h1) return 64 + __builtin_ctzll(h1);
    return m1 ? 64 + 63 - __builtin_clzll(m1) : 63 - __builtin_clzll(m0);
}

// One ply of ludax_policy_step for env e by the 64 lanes of a wave (every
// lane computes the same values; lane 0 writes): the fused guided steps of
// the network, which keep the logits (lg) and the board bytes (brow, with
// readable slack behind it, as in read_board) on chip.  Same draw, rules
// and state as k_step MODE 2 for the placement games whose legal actions
// are the empty cells and whose ply changes one cell (Hex, Gomoku).
// reward / terminal may be NULL.  Returns the cell played (-1 if none), and
// the env's side to move and whether it still runs after the ply.
template <class G>
__device__ __forceinline__ int wave_policy_ply(const DevState &st, int64_t e, int max_plies, const float *lg,
                                               const int8_t *brow, uint32_t key0, uint32_t key1, int64_t gid_base,
                                               const int64_t *__restrict__ gid, int8_t *__restrict__ reward,
                                               uint8_t *__restrict__ terminal, int &to_move, bool &running)
{
    static_assert(G::KIND == 3 || G::KIND == 5, "legal actions = empty cells, one cell per ply");
    const int lane = threadIdx.x & 63;
    int status = st.status[e];
    int me = st.to_move[e];
    int r1 = 0, r2 = 0, played = -1;
    if (status == RUNNING) {
        int winner = st.winner[e], passes = st.passes[e], ply = st.ply[e];
        const uint64_t id = (uint64_t)(gid != nullptr ? gid[e] : gid_base + e);
        const Philox4 f = philox4x32_10((uint32_t)ply >> 2, (uint32_t)id, (uint32_t)(id >> 32), 0u, key0, key1);
        const int r = ply & 3;
        const uint32_t w = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
        const int a = wave_policy_draw<G::CELLS>(lg, brow, w);
        if (a < 0) {
            status = ILLEGAL;
        } else {
            BB<G::NWC> c1, c2;
            read_board<G::CELLS, G::NWC>(brow, c1, c2);
            G g;
            g.load(c1, c2);
            const int outcome = g.place_step(G::bit_of(a), me, passes);
            const int mover = me;
            ply += 1;
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
            if (lane == 0) {
                st.board[e * G::CELLS + a] = (int8_t)mover;
                st.to_move[e] = (int8_t)me;
                st.winner[e] = (int8_t)winner;
                st.passes[e] = (int8_t)passes;
                st.ply[e] = (int16_t)ply;
                st.last_action[e] = (int16_t)a;
            }
            played = a;
        }
        if (lane == 0) st.status[e] = (int8_t)status;
    }
    if (lane == 0) {
        if (reward != nullptr) {
            reward[2 * e] = (int8_t)r1;
            reward[2 * e + 1] = (int8_t)r2;
        }
        if (terminal != nullptr) terminal[e] = status != RUNNING ? 1 : 0;
    }
    to_move = me;
    running = status == RUNNING;
    return played;
}

// One ply of a running game with random word w: legal set, the k-th legal
// action for k = (w * n_legal) >> 32, apply, end rules, advance.  Returns
// whether the game goes on.  A RUNNING state with no legal action (only on
// a hand-edited board) becomes ILLEGAL without consuming the ply.
template <class G>
__device__ __forceinline__ bool random_ply(G &g, int &me, int &passes, int &ply, int &last, int &status,
                                           int &winner, uint32_t w, int max_plies)
{
    const typename G::M m = g.placements(me);
    const int np = popcount(m);
    const int nl = G::HAS_PASS ? (np > 0 ? np : 1) : np;
    if (nl == 0) {
        status = ILLEGAL;
        return false;
    }
    const int k = (int)__umulhi(w, (uint32_t)nl);
    int outcome, a;
    if (G::HAS_PASS && np == 0) {
        a = G::A - 1;
        outcome = g.pass(passes);
    } else {
        const int b = select_bit(m, k);
        a = G::action_of(b);
        if constexpr (G::KIND == 5) outcome = g.place_drawn(b, me, passes, np); // Gomoku: np empty cells
        else outcome = g.place(b, me, passes);
    }
    ply += 1;
    last = a;
    if (outcome >= 0) {
        status = TERMINAL;
        winner = outcome;
        return false;
    }
    me = 3 - me;
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
// Start position of a lane (Reversi: the four discs; the rest: empty).
template <class G>
__device__ __forceinline__ void start_position(G &g)
{
    if constexpr (G::KIND == 4) {
        // player 1 on E4 (row 3, col 4) and D5 (row 4, col 3); player 2 on D4 and E5
        g.p1 = onehot<G::NWI>(3 * 8 + 4) | onehot<G::NWI>(4 * 8 + 3);
        g.p2 = onehot<G::NWI>(3 * 8 + 3) | onehot<G::NWI>(4 * 8 + 4);
    } else {
        g.p1 = bb_zero<G::NWI>();
        g.p2 = bb_zero<G::NWI>();
    }
}

template <class G>
__global__ __launch_bounds__(BLOCK) void k_playout(DevState st, int64_t n, int max_plies,
                                                   uint32_t key0, uint32_t key1, int64_t gid_base,
                                                   const int64_t *__restrict__ gid,
                                                   int8_t *__restrict__ reward,
                                                   uint8_t *__restrict__ terminal)
{
    __shared__ __align__(16) int8_t lds[BLOCK * G::CELLS + STAGE_SLACK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    int me = st.to_move[ec], status = valid ? (int)st.status[ec] : ILLEGAL, winner = st.winner[ec];
    int passes = st.passes[ec], ply = st.ply[ec], last = st.last_action[ec];
    G g;
    // a block whose envs are all RUNNING at ply 0 holds start positions (the
    // ply counts the plies applied since ludax_init): its boards are not read
    if (__syncthreads_and(!valid || (status == RUNNING && ply == 0))) {
        start_position(g);
    } else {
        stage_in<G::CELLS>(st.board, e0, nb, lds);
        BB<G::NWC> c1, c2;
        read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
        g.load(c1, c2);
    }
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
        if ((ply & 3) == 0 && !first) {
            const Philox4 f = philox4x32_10((uint32_t)ply >> 2, id_lo, id_hi, 0u, key0, key1);
            w0 = f.v[0];
            w1 = f.v[1];
            w2 = f.v[2];
            w3 = f.v[3];
        }
        first = false;
        running = random_ply(g, me, passes, ply, last, status, winner, w0, max_plies);
        w0 = w1;
        w1 = w2;
        w2 = w3;
    }
    if (was_running && status == TERMINAL) {
        r1 = winner == 1 ? 1 : (winner == 2 ? -1 : 0);
        r2 = -r1;
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
// A block's move list in LDS: the internal bit index of window ply j of
// lane t.  Boards up to 256 bits: one byte per ply, at [j * BLOCK + t].
// Larger boards (Hex 17 .. 19): the low byte there, and the ninth bit in a
// word array behind it, word (j / 32) of lane t at [(j / 32) * BLOCK + t]
// (the lanes of a word row are consecutive: no bank conflicts), cleared per
// window and set with LDS atomics.  Two bytes per ply would take 46 KB at
// 19x19, three blocks (waves) per CU; this takes 26 KB, six.
// ---------------------------------------------------------------------------
template <class G>
struct Moves {
    static constexpr bool WIDE = G::NBITS > 256;
    static constexpr int HW = (G::CELLS + 31) / 32; // ninth-bit words per lane
    static constexpr int BYTES = BLOCK * G::CELLS + (WIDE ? BLOCK * HW * 4 : 0);
    int8_t *base;
    __device__ __forceinline__ uint8_t *lo() const { return reinterpret_cast<uint8_t *>(base); }
    __device__ __forceinline__ uint32_t *hi() const
    {
        return reinterpret_cast<uint32_t *>(base + BLOCK * G::CELLS);
    }
    __device__ __forceinline__ void clear(int t) const
    {
        if constexpr (WIDE) {
#pragma unroll
            for (int q = 0; q < HW; ++q) hi()[q * BLOCK + t] = 0u;
        }
    }
    __device__ __forceinline__ void put(int j, int t, int b) const
    {
        lo()[j * BLOCK + t] = (uint8_t)b;
        if constexpr (WIDE) {
            if (b & 256)
                __hip_atomic_fetch_or(&hi()[(j >> 5) * BLOCK + t], 1u << (j & 31), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __device__ __forceinline__ int get(int j, int t) const
    {
        int b = lo()[j * BLOCK + t];
        if constexpr (WIDE) b |= (int)((hi()[(j >> 5) * BLOCK + t] >> (j & 31)) & 1u) << 8;
        return b;
    }
};

// ---------------------------------------------------------------------------
// The random sequence of a window of T plies, without any end test: ply j
// (from ply0) is played by the owner of `cur` for even j and of `oth` for
// odd j, on a uniformly drawn cell of G::open_cells, and its internal bit is
// recorded in the move list (Moves).  One Philox block serves the plies
// 4q .. 4q+3; the window is cut into a head (up to the next multiple of
// four), whole blocks of four plies and a tail, so that no ply tests
// whether it needs a new block.  On return cur / oth again hold the stones
// of the player who moved first / second.
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ void fill_window(typename G::M &cur, typename G::M &oth, int T, int ply0,
                                            uint32_t id_lo, uint32_t id_hi, uint32_t key0, uint32_t key1,
                                            const Moves<G> &moves, int t)
{
    using M = typename G::M;
    // The legal set and its size are carried from ply to ply (the chosen
    // cell's bit leaves it and joins the mover's stones).  Hex and
    // Tic-Tac-Toe: the legal cells are the empty cells.  Connect Four: the
    // lowest empty cell of each column, so the cell above the chosen one
    // (one row stride up) joins the set, or the set shrinks when a column
    // fills.
    constexpr bool EMPTY_IS_LEGAL = G::KIND == 1 || G::KIND == 3;
    constexpr bool CARRY = EMPTY_IS_LEGAL || G::KIND == 2;
    M open = bb_zero<G::NWI>();
    int n_open = 0;
    if constexpr (CARRY) {
        open = G::open_cells(cur, oth);
        n_open = popcount(open);
    }
    moves.clear(t);
    auto play = [&](M &mine, const M &theirs, int j, uint32_t w) {
        if constexpr (CARRY) {
            int wi;
            uint32_t bit;
            select_bit_split(open, (int)__umulhi(w, (uint32_t)n_open), wi, bit);
            const int b = 32 * wi + __builtin_ctz(bit);
            moves.put(j, t, b);
            const int sel = word_sel(wi);
            static_for<G::NWI>([&](auto I) {
                constexpr int i = I;
                const uint32_t x = bit & word_mask(sel, i);
                mine.w[i] |= x;
                open.w[i] ^= x;
            });
            if constexpr (EMPTY_IS_LEGAL) {
                --n_open;
            } else {
                const int up = b - G::S; // the cell above (same column, one row up)
                static_for<G::NWI>([&](auto I) {
                    constexpr int i = I;
                    open.w[i] |= (up >= 0 && (up >> 5) == i) ? 1u << (up & 31) : 0u;
                });
                n_open -= up < 0 ? 1 : 0;
            }
        } else {
            const int b = select_uniform(G::open_cells(mine, theirs), w);
            moves.put(j, t, b);
            mine = mine | onehot<G::NWI>(b);
        }
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
//
// The line games (Tic-Tac-Toe, Connect Four) use the same scheme: their
// legal set is also independent of the game being over (Connect Four:
// empty cells resting on the floor or a piece), and "some player holds a
// line of n or more" only becomes true by the owner's own placement and
// then stays true, so the end ply is the first prefix of the window at
// which it holds -- again by binary search, each probe two shift-AND line
// tests.  Without a line, a full board is a draw (wins before draws).
// ---------------------------------------------------------------------------

// The outcome of one lane's window.
template <class G>
struct Window {
    typename G::M f1, f2; // final stones of players 1 and 2
    int status;           // TERMINAL, TRUNCATED, or ILLEGAL (no legal cell)
    int winner, me, ply, last;
};


// Play and resolve one window from stones b1 / b2, player me0 to move at
// ply0.  Only meaningful for run == true (otherwise T = 0 and nothing is
// played); `empties` legal cells remain at ply0.
template <class G>
__device__ __forceinline__ Window<G> play_window(const typename G::M &b1, const typename G::M &b2,
                                                 bool run, int me0, int ply0, int max_plies,
                                                 uint32_t id_lo, uint32_t id_hi, uint32_t key0,
                                                 uint32_t key1, const Moves<G> &moves, int t)
{
    using M = typename G::M;
    constexpr int NW = G::NWI;
    const int empties = run ? G::CELLS - popcount(b1 | b2) : 0;
    const int room = max_plies - ply0 > 1 ? max_plies - ply0 : 1;
    const int T = empties < room ? empties : room; // plies in the window

    // ---- fill: the random sequence, no end test ----
    M cur = pick(me0 == 1, b1, b2); // stones of the player to move at ply0
    M oth = pick(me0 == 1, b2, b1);
    fill_window<G>(cur, oth, T, ply0, id_lo, id_hi, key0, key1, moves, t);
    const M end1 = pick(me0 == 1, cur, oth); // boards after the window
    const M end2 = pick(me0 == 1, oth, cur);

    // ---- resolve: the ply that ended the game (-1: none in the window) ----
    int jstar = -1;
    if constexpr (G::KIND == 3) {
        int W = 0;
        if (T > 0) {
            if (G::joins(end1, 1)) W = 1;
            else if (empties == T || G::joins(end2, 2)) W = 2; // a full board always has a winner
        }
        const int jw0 = W == me0 ? 0 : 1;          // W's first ply in the window
        const int MW = W ? (T - jw0 + 1) >> 1 : 0; // W's moves in the window
        if (MW > 0) {
            const bool w1 = W == 1;
            M s_lo = pick(w1, b1, b2); // W's stones before its lo-th window move
            M r_lo = G::flood(G::first_side_sel(s_lo, w1), s_lo);
            int lo = 1, hi = MW, next = 1; // next = first move not yet in s_lo
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                M s = s_lo;
                // W's moves next..mid, four list reads in flight at a time
                // (an index past mid repeats mid's cell)
                for (int k = next; k <= mid; k += 4) {
                    int c[4];
                    static_for<4>([&](auto I) {
                        constexpr int i = I;
                        const int kk = k + i < mid ? k + i : mid;
                        c[i] = moves.get(jw0 + 2 * (kk - 1), t);
                    });
                    static_for<4>([&](auto I) { s = s | onehot<NW>(c[I]); });
                }
                M r = r_lo | G::first_side_sel(s, w1);
                if (G::flood_to_far_sel(r, s, w1)) {
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
    } else {
        if (T > 0 && (G::line(end1) | G::line(end2))) {
            M s1 = b1, s2 = b2; // stones before window ply lo
            int lo = 0, hi = T - 1, next = 0;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                M a1 = s1, a2 = s2;
                // plies next..mid, four list reads in flight at a time (an
                // index past mid repeats mid's cell, on the same board)
                for (int j = next; j <= mid; j += 4) {
                    int c[4], jj[4];
                    static_for<4>([&](auto I) {
                        constexpr int i = I;
                        jj[i] = j + i < mid ? j + i : mid;
                        c[i] = moves.get(jj[i], t);
                    });
                    static_for<4>([&](auto I) {
                        constexpr int i = I;
                        const M x = onehot<NW>(c[i]);
                        const bool p1 = ((jj[i] & 1) == 0) == (me0 == 1);
                        a1 = pick(p1, a1 | x, a1);
                        a2 = pick(p1, a2, a2 | x);
                    });
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
    }

    // ---- the final position ----
    Window<G> w;
    const int played = jstar >= 0 ? jstar + 1 : T;
    // take back the plies after the end: a cell holds one player's stone,
    // so the cells of those plies leave both boards; four list reads in
    // flight at a time (an index past the window repeats its last ply)
    M undo = bb_zero<NW>();
    for (int j = played; j < T; j += 4) {
        int c[4];
        static_for<4>([&](auto I) {
            constexpr int i = I;
            c[i] = moves.get(j + i < T - 1 ? j + i : T - 1, t);
        });
        static_for<4>([&](auto I) { undo = undo | onehot<NW>(c[I]); });
    }
    w.f1 = andnot(end1, undo);
    w.f2 = andnot(end2, undo);
    w.winner = -1;
    w.ply = ply0 + played;
    w.me = me0;
    w.last = -1;
    if (T == 0) {
        w.status = ILLEGAL; // RUNNING with no legal cell: only a hand-edited board
    } else {
        w.last = G::action_of(moves.get(played - 1, t));
        const int mover = ((played - 1) & 1) == 0 ? me0 : 3 - me0; // of the last ply
        if (jstar >= 0) {
            w.status = TERMINAL;
            w.winner = mover;
            w.me = mover;
        } else if (T == empties && G::KIND != 3) {
            w.status = TERMINAL; // full board without a line: draw
            w.winner = 0;
            w.me = mover;
        } else {
            w.me = 3 - mover;
            w.status = w.ply >= max_plies ? TRUNCATED : ILLEGAL;
        }
    }
    return w;
}

// LDS bytes of one block of a fill-then-resolve playout: the boards'
// staging area and, after it, the move list
template <class G>
constexpr int fill_lds_bytes()
{
    constexpr int STAGE = BLOCK * G::CELLS;
    constexpr int LIST = Moves<G>::BYTES;
    return (STAGE > LIST ? STAGE : LIST) + STAGE_SLACK;
}

// Fill-then-resolve playout of the envs [blk * BLOCK, blk * BLOCK + 64) of
// a batch of states (Hex, Tic-Tac-Toe, Connect Four); lds holds
// fill_lds_bytes<G>() bytes.  FROM_START: every env is first reset to the
// start position as ludax_init sets it (empty board, player 1 to move,
// RUNNING, ply 0, no last action), so no field of the state is read.
template <class G, bool FROM_START>
__device__ __forceinline__ void playout_fill_block(const DevState &st, int64_t n, int max_plies, uint32_t key0,
                                                   uint32_t key1, int64_t gid_base, const int64_t *__restrict__ gid,
                                                   int8_t *__restrict__ reward, uint8_t *__restrict__ terminal,
                                                   int64_t blk, int8_t *lds)
{
    using M = typename G::M;
    const Moves<G> moves{lds}; // the move list over the staging area

    const int64_t e0 = blk * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    const int64_t ec = valid ? e : e0; // lanes past the batch end mirror env e0, then are ignored
    int me = 1, status = valid ? RUNNING : ILLEGAL, winner = -1, passes = 0, ply = 0, last = -1;
    if constexpr (!FROM_START) {
        me = st.to_move[ec];
        status = valid ? (int)st.status[ec] : ILLEGAL;
        winner = st.winner[ec];
        passes = st.passes[ec];
        ply = st.ply[ec];
        last = st.last_action[ec];
    }
    const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
    // a block whose envs are all RUNNING at ply 0 holds start positions
    // (empty boards for these games; the ply counts the plies applied since
    // ludax_init): its boards are not read
    M b1 = bb_zero<G::NWI>(), b2 = bb_zero<G::NWI>();
    if constexpr (!FROM_START) {
        if (!__syncthreads_and(!valid || (status == RUNNING && ply == 0))) {
            stage_in<G::CELLS>(st.board, e0, nb, lds);
            BB<G::NWC> c1, c2;
            read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
            b1 = G::from_canon(c1);
            b2 = G::from_canon(c2);
        }
        __syncthreads(); // the staging area becomes the move list
    }

    const bool run = valid && status == RUNNING;
    const Window<G> w = play_window<G>(b1, b2, run, me, ply, max_plies, (uint32_t)id, (uint32_t)(id >> 32),
                                       key0, key1, moves, t);
    M f1 = b1, f2 = b2;
    int r1 = 0, r2 = 0;
    if (run) {
        f1 = w.f1;
        f2 = w.f2;
        status = w.status;
        winner = w.winner;
        me = w.me;
        ply = w.ply;
        last = w.last;
        r1 = winner == 1 ? 1 : (winner == 2 ? -1 : 0);
        r2 = -r1;
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

// Fill-then-resolve playout of a batch of states (Hex, Tic-Tac-Toe,
// Connect Four).
template <class G>
__global__ __launch_bounds__(BLOCK) void k_playout_fill(DevState st, int64_t n, int max_plies,
                                                        uint32_t key0, uint32_t key1, int64_t gid_base,
                                                        const int64_t *__restrict__ gid,
                                                        int8_t *__restrict__ reward,
                                                        uint8_t *__restrict__ terminal)
{
    __shared__ __align__(16) int8_t lds[fill_lds_bytes<G>()];
    playout_fill_block<G, false>(st, n, max_plies, key0, key1, gid_base, gid, reward, terminal, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Batch groups: several batches, each of its own game, in one launch.  The
// group's games are a fixed type list Gs (GroupGames); block b serves batch
// k for first_block[k] <= b < first_block[k + 1], and runs the body of that
// batch's game (slot[k], its index in Gs).  Kernels of one stream run one
// after the other, so separate launches leave the chip to the first
// batch's waves alone (65536 envs = one wave per SIMD) and the next batch
// waits for its tail; in one grid the batches' waves share the SIMDs.
// ---------------------------------------------------------------------------
template <class... Gs>
struct GroupGames {
    static constexpr int LDS = [] {
        int m = 0;
        for (int b : {fill_lds_bytes<Gs>()...}) m = b > m ? b : m;
        return m;
    }();
    template <class G>
    static constexpr int slot_of()
    {
        int i = 0, r = -1;
        for (bool same : {std::is_same_v<G, Gs>...}) {
            if (same && r < 0) r = i;
            ++i;
        }
        return r;
    }
};

// the fill-then-resolve games that share the group kernel
using PlayoutGroup = GroupGames<TicTacToe, ConnectFour, Hex<11>>;

// field k of a kernel-argument array, k wave-uniform: a chain of selects on
// constant indices keeps the arguments in scalar registers (an indexed
// access would copy the array to scratch memory)
template <class T, int N>
__device__ __forceinline__ T pick(const T (&v)[N], int k)
{
    T r = v[0];
#pragma unroll
    for (int j = 1; j < N; ++j) r = k == j ? v[j] : r;
    return r;
}

__device__ __forceinline__ DevState pick_state(const DevState (&v)[GROUP_MAX], int k)
{
    DevState r = v[0];
#pragma unroll
    for (int j = 1; j < GROUP_MAX; ++j)
        if (k == j) r = v[j];
    return r;
}

template <bool FROM_START, int I, class G, class... Rest>
__device__ __forceinline__ void group_body(const GroupArgs &a, int slot, int k, int64_t blk, int8_t *lds)
{
    if (slot == I) {
        playout_fill_block<G, FROM_START>(pick_state(a.st, k), pick(a.n, k), pick(a.max_plies, k), a.key0, a.key1,
                                          pick(a.gid_base, k), nullptr, pick(a.reward, k), pick(a.terminal, k),
                                          blk, lds);
    } else if constexpr (sizeof...(Rest) > 0) {
        group_body<FROM_START, I + 1, Rest...>(a, slot, k, blk, lds);
    }
}

template <bool FROM_START, class... Gs>
__device__ __forceinline__ void group_run(const GroupArgs &a, GroupGames<Gs...>, int slot, int k, int64_t blk,
                                          int8_t *lds)
{
    group_body<FROM_START, 0, Gs...>(a, slot, k, blk, lds);
}

template <bool FROM_START, class Group>
__global__ __launch_bounds__(BLOCK) void k_playout_group(GroupArgs a)
{
    __shared__ __align__(16) int8_t lds[Group::LDS];
    const int b = blockIdx.x;
    int k = 0;
#pragma unroll
    for (int j = 1; j < GROUP_MAX; ++j)
        if (j < a.nb && b >= a.first_block[j]) k = j;
    // The batches come longest-running first.  A SIMD runs a wave of the
    // longest batch next to waves of shorter ones: the longer the batch,
    // the higher its waves' issue priority, so the long pole runs at close
    // to its own speed and the short batches fill the cycles it leaves.
    group_run<FROM_START>(a, Group{}, pick(a.slot, k), k, (int64_t)(b - pick(a.first_block, k)), lds);
}

// ---------------------------------------------------------------------------
// Mixed persistent batch: one kernel per game kind, all kinds launched
// concurrently.  A kind's games are the global indices j0, j0 + stride,
// j0 + 2 stride, ... of the batch (count of them); game j has id
// id_base + j.  A wave takes its games from the kind's queue 64 at a time
// (one atomic per 64 games) and writes each game's winner (-1 if
// truncated), ply count and last action at its global index.
// ---------------------------------------------------------------------------

// next chunk of 64 games of this kind for the calling wave (wave-uniform)
__device__ __forceinline__ int64_t next_chunk(unsigned int *counter)
{
    unsigned int c = 0u;
    if (threadIdx.x == 0) c = atomicAdd(counter, 1u);
    return (int64_t)__shfl(c, 0, 64);
}

// Per-ply kinds (Reversi, Gomoku): every lane plays one game at a time and
// starts a new one as soon as its game has ended.  New games start only on
// wave steps s = 0 mod 4, so every lane's ply is then a multiple of four
// and one Philox block per lane serves the next four steps: the block
// refresh is uniform across the wave, and a finished lane idles at most
// three steps.
template <class G>
__device__ __forceinline__ void persist_ply_body(const MixedArgs &a)
{
    const int t = threadIdx.x;
    const uint64_t below = (1ull << t) - 1ull;
    G g;
    start_position(g);
    int me = 1, passes = 0, ply = 0, last = -1, status = RUNNING, winner = -1;
    int64_t i = -1; // game of this kind played by the lane, -1 = idle
    uint32_t id_lo = 0u, id_hi = 0u, w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
    int64_t pool = 0, pool_end = 0; // wave-uniform: unassigned games [pool, pool_end)
    bool exhausted = false;
    for (int s = 0;; ++s) {
        if ((s & 3) == 0) {
            uint64_t need = __ballot(i < 0);
            while (need != 0ull && !exhausted) {
                if (pool == pool_end) {
                    pool = next_chunk(a.counter) * BLOCK;
                    pool_end = pool + BLOCK < a.count ? pool + BLOCK : a.count;
                    if (pool >= a.count) {
                        exhausted = true;
                        break;
                    }
                }
                const int take = (int)(pool_end - pool) < __popcll(need) ? (int)(pool_end - pool) : __popcll(need);
                const int rank = __popcll(need & below);
                if (((need >> t) & 1ull) && rank < take) {
                    i = pool + rank;
                    const uint64_t id = (uint64_t)(a.id_base + a.j0 + i * a.stride);
                    id_lo = (uint32_t)id;
                    id_hi = (uint32_t)(id >> 32);
                    start_position(g);
                    me = 1;
                    passes = 0;
                    ply = 0;
                    last = -1;
                    status = RUNNING;
                    winner = -1;
                }
                pool += take;
                need = __ballot(i < 0);
            }
            if (__ballot(i >= 0) == 0ull) break;
            if (i >= 0) {
                const Philox4 f = philox4x32_10((uint32_t)ply >> 2, id_lo, id_hi, 0u, a.key0, a.key1);
                w0 = f.v[0];
                w1 = f.v[1];
                w2 = f.v[2];
                w3 = f.v[3];
            }
        }
        if (i >= 0) {
            const bool going = random_ply(g, me, passes, ply, last, status, winner, w0, a.max_plies);
            w0 = w1;
            w1 = w2;
            w2 = w3;
            if (!going) {
                const int64_t j = a.j0 + i * a.stride;
                a.winner[j] = (int8_t)(status == TERMINAL ? winner : -1);
                a.plies[j] = (int16_t)ply;
                a.last[j] = (int16_t)last;
                i = -1;
            }
        }
    }
}

template <class G>
__global__ __launch_bounds__(BLOCK) void k_persist_ply(MixedArgs a)
{
    persist_ply_body<G>(a);
}

// The same schedule for the movement games, over a lane adapter L:
// L::Shared is the block's LDS the adapter needs, bind(shared, lane) sets
// it up, start() begins a game at the start position, step(w, max_plies)
// plays one ply with Philox word w and returns whether the game goes on,
// and ply / last / status / winner report it.  Every ply is one wave step,
// so the Philox blocks stay aligned exactly as in k_persist_ply.
template <class L>
__global__ __launch_bounds__(BLOCK) void k_persist_lane(MixedArgs a)
{
    __shared__ typename L::Shared shared;
    const int t = threadIdx.x;
    const uint64_t below = (1ull << t) - 1ull;
    L lane;
    lane.bind(shared, t);
    int64_t i = -1; // game of this kind played by the lane, -1 = idle
    uint32_t id_lo = 0u, id_hi = 0u, w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
    int64_t pool = 0, pool_end = 0; // wave-uniform: unassigned games [pool, pool_end)
    bool exhausted = false;
    for (int s = 0;; ++s) {
        if ((s & 3) == 0) {
            uint64_t need = __ballot(i < 0);
            while (need != 0ull && !exhausted) {
                if (pool == pool_end) {
                    pool = next_chunk(a.counter) * BLOCK;
                    pool_end = pool + BLOCK < a.count ? pool + BLOCK : a.count;
                    if (pool >= a.count) {
                        exhausted = true;
                        break;
                    }
                }
                const int take = (int)(pool_end - pool) < __popcll(need) ? (int)(pool_end - pool) : __popcll(need);
                const int rank = __popcll(need & below);
                if (((need >> t) & 1ull) && rank < take) {
                    i = pool + rank;
                    const uint64_t id = (uint64_t)(a.id_base + a.j0 + i * a.stride);
                    id_lo = (uint32_t)id;
                    id_hi = (uint32_t)(id >> 32);
                    lane.start();
                }
                pool += take;
                need = __ballot(i < 0);
            }
            if (__ballot(i >= 0) == 0ull) break;
            if (i >= 0) {
                const Philox4 f = philox4x32_10((uint32_t)lane.ply >> 2, id_lo, id_hi, 0u, a.key0, a.key1);
                w0 = f.v[0];
                w1 = f.v[1];
                w2 = f.v[2];
                w3 = f.v[3];
            }
        }
        if (i >= 0) {
            const bool going = lane.step(w0, a.max_plies);
            w0 = w1;
            w1 = w2;
            w2 = w3;
            if (!going) {
                const int64_t j = a.j0 + i * a.stride;
                a.winner[j] = (int8_t)(lane.status == TERMINAL ? lane.winner : -1);
                a.plies[j] = (int16_t)lane.ply;
                a.last[j] = (int16_t)lane.last;
                i = -1;
            }
        }
    }
}

// Fill-then-resolve kinds (Hex, Tic-Tac-Toe, Connect Four): every game of
// a chunk fills the same number of plies from the start position, so the
// 64 lanes of a wave play 64 games in lockstep and then take the next chunk.
template <class G>
__device__ __forceinline__ void persist_fill_body(const MixedArgs &a, int8_t *lds)
{
    using M = typename G::M;
    const int t = threadIdx.x;
    const M zero = bb_zero<G::NWI>();
    const Moves<G> moves{lds};
    for (;;) {
        const int64_t c = next_chunk(a.counter) * BLOCK;
        if (c >= a.count) break;
        const int64_t i = c + t;
        const bool valid = i < a.count;
        const int64_t j = a.j0 + (valid ? i : c) * a.stride;
        const uint64_t id = (uint64_t)(a.id_base + j);
        const Window<G> w = play_window<G>(zero, zero, valid, 1, 0, a.max_plies, (uint32_t)id,
                                           (uint32_t)(id >> 32), a.key0, a.key1, moves, t);
        if (valid) {
            a.winner[j] = (int8_t)(w.status == TERMINAL ? w.winner : -1);
            a.plies[j] = (int16_t)w.ply;
            a.last[j] = (int16_t)w.last;
        }
        __syncthreads(); // the move list is reused by the next chunk
    }
}

template <class G>
__global__ __launch_bounds__(BLOCK) void k_persist_fill(MixedArgs a)
{
    __shared__ __align__(16) int8_t lds[Moves<G>::BYTES];
    persist_fill_body<G>(a, lds);
}

// A mixed batch in one grid: the kinds' persistent loops side by side in
// one launch, block b serving kind k for first_block[k] <= b <
// first_block[k + 1] with the body of its game (slot[k] in the type list
// Gs).  No stream per kind: the kinds overlap whatever the queues, as long
// as the grid is resident at once (the register footprint is the largest
// body's, the LDS the largest move list).
template <class... Gs>
struct PersistGames {
    template <class G>
    static constexpr int lds_of()
    {
        return (G::KIND == 1 || G::KIND == 2 || G::KIND == 3) ? Moves<G>::BYTES : 0;
    }
    static constexpr int LDS = [] {
        int m = 16;
        for (int b : {lds_of<Gs>()...}) m = b > m ? b : m;
        return m;
    }();
    template <class G>
    static constexpr int slot_of()
    {
        int i = 0, r = -1;
        for (bool same : {std::is_same_v<G, Gs>...}) {
            if (same && r < 0) r = i;
            ++i;
        }
        return r;
    }
};

// the small-board kinds that share the one-grid mixed kernel
using PersistGroup = PersistGames<TicTacToe, ConnectFour, Reversi, Hex<11>, Gomoku<15>>;

template <int I, class G, class... Rest>
__device__ __forceinline__ void persist_group_body(const MixedArgs &a, int slot, int8_t *lds)
{
    if (slot == I) {
        if constexpr (G::KIND == 1 || G::KIND == 2 || G::KIND == 3)
            persist_fill_body<G>(a, lds);
        else
            persist_ply_body<G>(a);
    } else if constexpr (sizeof...(Rest) > 0) {
        persist_group_body<I + 1, Rest...>(a, slot, lds);
    }
}

template <class... Gs>
__device__ __forceinline__ void persist_group_run(const MixedArgs &a, PersistGames<Gs...>, int slot, int8_t *lds)
{
    persist_group_body<0, Gs...>(a, slot, lds);
}

template <class Group>
__global__ __launch_bounds__(BLOCK) void k_persist_group(MixedGroupArgs g)
{
    __shared__ __align__(16) int8_t lds[Group::LDS];
    const int b = blockIdx.x;
    int k = 0;
#pragma unroll
    for (int j = 1; j < MIXED_MAX; ++j)
        if (j < g.n && b >= g.first_block[j]) k = j;
    // the kind's arguments by constant-index selects (scalar registers)
    MixedArgs a = g.k[0];
    int slot = g.slot[0];
#pragma unroll
    for (int j = 1; j < MIXED_MAX; ++j)
        if (k == j) {
            a = g.k[j];
            slot = g.slot[j];
        }
    persist_group_run(a, Group{}, slot, lds);
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
        if constexpr (G::KIND == 3) {
            if (st.aux != nullptr)
                hipLaunchKernelGGL((k_hexaux_sync<G::H, false>), dim3((unsigned)((n + BLOCK - 1) / BLOCK)),
                                   dim3(BLOCK), 0, s, st, n);
        }
        return hipGetLastError();
    }
    static hipError_t aux_sync(const DevState &st, int64_t n, hipStream_t s)
    {
        if constexpr (G::KIND == 3) {
            hipLaunchKernelGGL((k_hexaux_sync<G::H, true>), dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK),
                               0, s, st, n);
            return hipGetLastError();
        } else {
            return hipSuccess;
        }
    }
    // the step kernel of MODE: Hex with an aux cache takes k_step_hexaux
    // (whose LDS, dynamic, holds only the next mask's rows)
    template <int MODE>
    static auto step_kernel(const DevState &st)
    {
        if constexpr (G::KIND == 3) {
            if (st.aux != nullptr) return &k_step_hexaux<G::H, MODE>;
        }
        return &k_step<G, MODE>;
    }
    static unsigned step_lds(const DevState &st, const uint8_t *next_mask)
    {
        if constexpr (G::KIND == 3) {
            if (st.aux != nullptr && next_mask != nullptr) return BLOCK * G::A + STAGE_SLACK;
        }
        return 0u;
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
        hipLaunchKernelGGL(step_kernel<0>(st), dim3((unsigned)blocks), dim3(BLOCK), step_lds(st, next_mask), s, st, n,
                           max_plies,
                           action, (const float *)nullptr, 0u, 0u, (int64_t)0, (const int64_t *)nullptr, reward,
                           terminal, next_mask);
        return hipGetLastError();
    }
    static hipError_t random_step(const DevState &st, int64_t n, int max_plies, uint64_t seed,
                                  int64_t gid_base, const int64_t *gid, int8_t *reward, uint8_t *terminal,
                                  hipStream_t s)
    {
        const int64_t blocks = (n + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL(step_kernel<1>(st), dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n, max_plies,
                           (const int32_t *)nullptr, (const float *)nullptr, (uint32_t)seed, (uint32_t)(seed >> 32),
                           gid_base, gid, reward, terminal, (uint8_t *)nullptr);
        return hipGetLastError();
    }
    static hipError_t policy_step(const DevState &st, int64_t n, int max_plies, const float *logits,
                                  uint64_t seed, int64_t gid_base, const int64_t *gid, int8_t *reward,
                                  uint8_t *terminal, hipStream_t s)
    {
        const int64_t blocks = (n + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL(step_kernel<2>(st), dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n, max_plies,
                           (const int32_t *)nullptr, logits, (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid,
                           reward, terminal, (uint8_t *)nullptr);
        return hipGetLastError();
    }
    static hipError_t playout(const DevState &st, int64_t n, int max_plies, uint64_t seed,
                              int64_t gid_base, const int64_t *gid, int8_t *reward,
                              uint8_t *terminal, int64_t *stats, hipStream_t s)
    {
        const int64_t blocks = (n + BLOCK - 1) / BLOCK;
        hipError_t err = hipSuccess;
        if (stats != nullptr && (err = launch_stats(st, n, -1, stats, s)) != hipSuccess) return err;
        if constexpr (G::KIND == 1 || G::KIND == 2 || G::KIND == 3) {
            hipLaunchKernelGGL(k_playout_fill<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n,
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
    static hipError_t persist(const MixedArgs &a, int slots, hipStream_t s)
    {
        const int blocks = (slots + BLOCK - 1) / BLOCK;
        if constexpr (G::KIND == 1 || G::KIND == 2 || G::KIND == 3) {
            hipLaunchKernelGGL(k_persist_fill<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, a);
        } else {
            hipLaunchKernelGGL(k_persist_ply<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, a);
        }
        return hipGetLastError();
    }
    static constexpr GameOps ops()
    {
        if constexpr (G::KIND == 3)
            return GameOps{G::KIND,     G::H,         G::W,     G::CELLS, G::A,
                           &init,       &mask,        &step,    &random_step,
                           &policy_step, &playout,    &persist, HexAux<G::H>::BYTES,
                           &aux_sync,   PlayoutGroup::slot_of<G>(), PersistGroup::slot_of<G>()};
        else
            return GameOps{G::KIND, G::H, G::W, G::CELLS, G::A, &init, &mask, &step, &random_step, &policy_step,
                           &playout, &persist, 0, nullptr, PlayoutGroup::slot_of<G>(), PersistGroup::slot_of<G>()};
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
