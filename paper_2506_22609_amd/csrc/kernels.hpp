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
//              of the wave has ended; final board written back through LDS,
//              step and outcome counters reduced per wave, one atomic each
#pragma once

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

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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
    G g;
    int me = 1;
    bool running = false;
    if (valid) {
        BB<G::NWC> c1, c2;
        read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
        g.load(c1, c2);
        me = st.to_move[e0 + t];
        running = st.status[e0 + t] == RUNNING;
    }
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

    G g;
    int me = 1, status = ILLEGAL, winner = -1, passes = 0, ply = 0, last = -1, a = 0;
    if (valid) {
        BB<G::NWC> c1, c2;
        read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
        g.load(c1, c2);
        me = st.to_move[e];
        status = st.status[e];
        winner = st.winner[e];
        passes = st.passes[e];
        ply = st.ply[e];
        last = st.last_action[e];
        a = action[e];
    }
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
                                                   uint8_t *__restrict__ terminal,
                                                   unsigned long long *__restrict__ stats)
{
    __shared__ __align__(16) int8_t lds[BLOCK * G::CELLS];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<G::CELLS>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;

    G g;
    int me = 1, status = ILLEGAL, winner = -1, passes = 0, ply = 0, last = -1;
    uint64_t id = 0;
    if (valid) {
        BB<G::NWC> c1, c2;
        read_board<G::CELLS, G::NWC>(lds + t * G::CELLS, c1, c2);
        g.load(c1, c2);
        me = st.to_move[e];
        status = st.status[e];
        winner = st.winner[e];
        passes = st.passes[e];
        ply = st.ply[e];
        last = st.last_action[e];
        id = (uint64_t)(gid != nullptr ? gid[e] : gid_base + e);
    }
    const bool was_running = valid && status == RUNNING;
    if (was_running) g.prepare();
    const uint32_t id_lo = (uint32_t)id, id_hi = (uint32_t)(id >> 32);

    int r1 = 0, r2 = 0, steps = 0;
    uint32_t blk_q = 0xFFFFFFFFu;
    Philox4 blk;
    blk.v[0] = blk.v[1] = blk.v[2] = blk.v[3] = 0u;
    bool running = was_running;
    while (running) {
        const typename G::M m = g.placements(me);
        const int np = popcount(m);
        const int nl = G::HAS_PASS ? (np > 0 ? np : 1) : np;
        if (nl == 0) { // only reachable from a hand-edited board
            status = ILLEGAL;
            break;
        }
        const uint32_t q = (uint32_t)ply >> 2;
        if (q != blk_q) {
            blk = philox4x32_10(q, id_lo, id_hi, 0u, key0, key1);
            blk_q = q;
        }
        const int j = ply & 3;
        const uint32_t w = j == 0 ? blk.v[0] : (j == 1 ? blk.v[1] : (j == 2 ? blk.v[2] : blk.v[3]));
        const int k = (int)__umulhi(w, (uint32_t)nl);
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
        steps += 1;
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
    if (stats != nullptr) {
        const bool ended = was_running && status == TERMINAL;
        const int s = wave_sum(steps);
        const int w1 = __popcll(__ballot(ended && winner == 1));
        const int w2 = __popcll(__ballot(ended && winner == 2));
        const int d = __popcll(__ballot(ended && winner == 0));
        if (t == 0) {
            atomicAdd(&stats[0], (unsigned long long)s);
            atomicAdd(&stats[1], (unsigned long long)w1);
            atomicAdd(&stats[2], (unsigned long long)w2);
            atomicAdd(&stats[3], (unsigned long long)d);
        }
    }
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
        hipLaunchKernelGGL(k_playout<G>, dim3((unsigned)blocks), dim3(BLOCK), 0, s, st, n, max_plies,
                           (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid, reward, terminal,
                           reinterpret_cast<unsigned long long *>(stats));
        return hipGetLastError();
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
