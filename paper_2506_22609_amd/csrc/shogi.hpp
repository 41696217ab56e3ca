// shogi.hpp -- Dai Hasami Shogi (kind 10): the slide and hop mechanics of
// Sec. 3.2 on the 9 x 9 board, with custodial and corner captures and the
// five-in-a-row win outside the start rows (App. C).
//
// One env per lane.  Each player's pieces are an 81-bit board twice over:
// row-major (bit r*9 + c) and column-major (bit c*9 + r), so that the
// occupancy of a piece's row and of its column are both one 9-bit field.
// From those two fields a piece's moves are four numbers: per direction
// (up, left, right, down) the length of its slide (the run of empty cells
// next to it, found with one leading / trailing zero count), or a hop over
// the neighbour when that neighbour is a piece and the cell beyond is
// empty.  For one source the destinations in increasing cell order are the
// up cells (farthest first), the left cells, the right cells and the down
// cells, so the j-th move of a piece is arithmetic on the four numbers and
// the k-th legal action is a walk over the pieces in increasing order.
//
//   k_sh_init, k_sh_mask (rows of 6561 bytes written as one contiguous
//   stream per block), k_sh_step (MODE 0 / 1 / 2), k_sh_playout
#pragma once

#include "kernels.hpp"

namespace lx {

typedef unsigned __int128 u128;

namespace hs {

constexpr int N = 9, CELLS = 81, A = 81 * 81;

constexpr u128 cols_0_4()
{
    u128 m = 0;
    for (int r = 0; r < N; ++r) m |= (u128)0x1F << (N * r);
    return m;
}
constexpr u128 ALL = ((u128)1 << CELLS) - 1;
constexpr u128 ROWS_0_6 = ((u128)1 << (7 * N)) - 1;         // player 1's rows outside its start rows
constexpr u128 ROWS_2_8 = ALL ^ (((u128)1 << (2 * N)) - 1); // player 2's
constexpr u128 COLS_0_4 = cols_0_4();                      // where a row window of five can start

__host__ __device__ __forceinline__ u128 bit(int c) { return (u128)1 << c; }
__host__ __device__ __forceinline__ int div9(int c) { return (c * 57) >> 9; } // exact for 0 <= c < 81
__host__ __device__ __forceinline__ int tpos(int c)
{
    const int r = div9(c);
    return (c - N * r) * N + r;
}
__host__ __device__ __forceinline__ uint32_t field9(u128 x, int pos) { return (uint32_t)(x >> pos) & 0x1FFu; }
__host__ __device__ __forceinline__ int high_bit(uint32_t x) { return 31 - __builtin_clz(x); } // x != 0
__host__ __device__ __forceinline__ int low_bit(uint32_t x) { return __builtin_ctz(x); }        // x != 0
// lowest set bit of a nonzero board (below bit 96), without a branch: the
// lowest nonzero 32-bit word picked by two selects
__host__ __device__ __forceinline__ uint32_t first_set(uint32_t w) { return (uint32_t)__builtin_ffs((int)w) - 1u; }
__host__ __device__ __forceinline__ int low_bit128(u128 x)
{
    const uint32_t w0 = (uint32_t)x, w1 = (uint32_t)(x >> 32), w2 = (uint32_t)(x >> 64);
    uint32_t r = first_set(w2) + 64u;
    r = w1 ? first_set(w1) + 32u : r;
    r = w0 ? first_set(w0) : r;
    return (int)r;
}

// Moves of the piece on (r, c) given the occupancy of its row (bit =
// column) and of its column (bit = row): per direction a slide length 0..8
// or 9 for a hop, packed 4 bits each: up, left, right, down.
__host__ __device__ __forceinline__ uint32_t piece_moves(uint32_t row, uint32_t col, int r, int c)
{
    const uint32_t ux = col & ((1u << r) - 1u), dx = col >> (r + 1);
    const uint32_t lx = row & ((1u << c) - 1u), rx = row >> (c + 1);
    uint32_t U = ux ? (uint32_t)(r - 1 - high_bit(ux)) : (uint32_t)r;
    uint32_t L = lx ? (uint32_t)(c - 1 - high_bit(lx)) : (uint32_t)c;
    uint32_t R = rx ? (uint32_t)low_bit(rx) : (uint32_t)(8 - c);
    uint32_t D = dx ? (uint32_t)low_bit(dx) : (uint32_t)(8 - r);
    // no slide but a piece next to it: a hop if the cell beyond is on the board and empty
    if (U == 0 && r >= 2 && !((col >> (r - 2)) & 1u)) U = 9;
    if (L == 0 && c >= 2 && !((row >> (c - 2)) & 1u)) L = 9;
    if (R == 0 && c <= 6 && !((row >> (c + 2)) & 1u)) R = 9;
    if (D == 0 && r <= 6 && !((col >> (r + 2)) & 1u)) D = 9;
    return U | (L << 4) | (R << 8) | (D << 12);
}

__host__ __device__ __forceinline__ int dir_moves(uint32_t v) { return v == 9u ? 1 : (int)v; }

__host__ __device__ __forceinline__ int n_moves(uint32_t pm)
{
    return dir_moves(pm & 15u) + dir_moves((pm >> 4) & 15u) + dir_moves((pm >> 8) & 15u) + dir_moves(pm >> 12);
}

// destination of the j-th move (0 <= j < n_moves(pm)) of the piece on src
__host__ __device__ __forceinline__ int nth_dst(uint32_t pm, int src, int j)
{
    const uint32_t U = pm & 15u, L = (pm >> 4) & 15u, R = (pm >> 8) & 15u, D = pm >> 12;
    const int cu = dir_moves(U), cl = dir_moves(L), cr = dir_moves(R);
    if (j < cu) return U == 9u ? src - 2 * N : src - N * ((int)U - j);
    j -= cu;
    if (j < cl) return L == 9u ? src - 2 : src - ((int)L - j);
    j -= cl;
    if (j < cr) return R == 9u ? src + 2 : src + 1 + j;
    j -= cr;
    return D == 9u ? src + 2 * N : src + N * (1 + j);
}

// is dst one of the moves pm of the piece on src?
__host__ __device__ __forceinline__ bool has_dst(uint32_t pm, int src, int dst)
{
    const int r = div9(src), c = src - N * r, rd = div9(dst), cd = dst - N * rd;
    const int U = (int)(pm & 15u), L = (int)((pm >> 4) & 15u), R = (int)((pm >> 8) & 15u), D = (int)(pm >> 12);
    if (cd == c && rd < r) return U == 9 ? rd == r - 2 : rd >= r - U;
    if (cd == c && rd > r) return D == 9 ? rd == r + 2 : rd <= r + D;
    if (rd == r && cd < c) return L == 9 ? cd == c - 2 : cd >= c - L;
    if (rd == r && cd > c) return R == 9 ? cd == c + 2 : cd <= c + R;
    return false;
}

} // namespace hs

struct Shogi {
    static constexpr int KIND = 10, H = 9, W = 9, CELLS = 81, A = 81 * 81, NWC = 3;
    u128 p1, p2; // row-major
    u128 t1, t2; // column-major

    __host__ __device__ void set(u128 a, u128 b)
    {
        p1 = a;
        p2 = b;
        t1 = t2 = 0;
        for (u128 x = a; x; x &= x - 1) t1 |= hs::bit(hs::tpos(hs::low_bit128(x)));
        for (u128 x = b; x; x &= x - 1) t2 |= hs::bit(hs::tpos(hs::low_bit128(x)));
    }

    __host__ __device__ void start()
    {
        // player 2 on rows 0-1, player 1 on rows 7-8
        set(((u128)1 << 81) - ((u128)1 << 63), ((u128)1 << 18) - 1);
    }

    __host__ __device__ uint32_t moves_of(int src) const
    {
        const int r = hs::div9(src), c = src - 9 * r;
        return hs::piece_moves(hs::field9(p1 | p2, 9 * r), hs::field9(t1 | t2, 9 * c), r, c);
    }

    __host__ __device__ int count(int me) const
    {
        int n = 0;
        for (u128 x = me == 1 ? p1 : p2; x; x &= x - 1) n += hs::n_moves(moves_of(hs::low_bit128(x)));
        return n;
    }

    // the k-th legal move of `me` in increasing action order
    __host__ __device__ void select(int me, int k, int &src, int &dst) const
    {
        src = 0;
        dst = 0;
        for (u128 x = me == 1 ? p1 : p2; x; x &= x - 1) {
            const int s = hs::low_bit128(x);
            const uint32_t pm = moves_of(s);
            const int m = hs::n_moves(pm);
            if (k < m) {
                src = s;
                dst = hs::nth_dst(pm, s, k);
                return;
            }
            k -= m;
        }
    }

    __host__ __device__ bool legal(int me, int src, int dst) const
    {
        if (src < 0 || src >= 81 || dst < 0 || dst >= 81) return false;
        if (!(((me == 1 ? p1 : p2) >> src) & 1)) return false;
        return hs::has_dst(moves_of(src), src, dst);
    }

    // Move the piece of `me` from src to dst, then the captures; returns me
    // if the mover now has five in a row or column outside its start rows,
    // else -1 (the next end rule, an opponent left without a legal move,
    // needs the opponent's move count: see shogi_outcome).
    __host__ __device__ int apply(int me, int src, int dst)
    {
        const u128 mv = hs::bit(src) | hs::bit(dst), mt = hs::bit(hs::tpos(src)) | hs::bit(hs::tpos(dst));
        u128 own = me == 1 ? p1 : p2, ownT = me == 1 ? t1 : t2;
        u128 opp = me == 1 ? p2 : p1, oppT = me == 1 ? t2 : t1;
        own ^= mv;
        ownT ^= mt;
        const int r = hs::div9(dst), c = dst - 9 * r;
        // runs of opponent pieces enclosed between dst and another own piece
        const uint32_t orow = hs::field9(opp, 9 * r), mrow = hs::field9(own, 9 * r);
        const uint32_t ocol = hs::field9(oppT, 9 * c), mcol = hs::field9(ownT, 9 * c);
        uint32_t cap_row = 0u, cap_col = 0u; // captured cells of row r (bit = column) / column c (bit = row)
        {
            const int run = hs::low_bit(~orow >> (c + 1)); // opponent cells right of c
            const int e = c + 1 + run;
            if (run > 0 && e <= 8 && ((mrow >> e) & 1u)) cap_row |= ((1u << run) - 1u) << (c + 1);
            const uint32_t other = ~orow & ((1u << c) - 1u); // cells left of c that are not the opponent's
            if (other) {
                const int e2 = hs::high_bit(other), run2 = c - 1 - e2;
                if (run2 > 0 && ((mrow >> e2) & 1u)) cap_row |= ((1u << run2) - 1u) << (e2 + 1);
            }
        }
        {
            const int run = hs::low_bit(~ocol >> (r + 1));
            const int e = r + 1 + run;
            if (run > 0 && e <= 8 && ((mcol >> e) & 1u)) cap_col |= ((1u << run) - 1u) << (r + 1);
            const uint32_t other = ~ocol & ((1u << r) - 1u);
            if (other) {
                const int e2 = hs::high_bit(other), run2 = r - 1 - e2;
                if (run2 > 0 && ((mcol >> e2) & 1u)) cap_col |= ((1u << run2) - 1u) << (e2 + 1);
            }
        }
        for (uint32_t x = cap_row; x; x &= x - 1u) {
            const int cc = hs::low_bit(x);
            opp &= ~hs::bit(9 * r + cc);
            oppT &= ~hs::bit(9 * cc + r);
        }
        for (uint32_t x = cap_col; x; x &= x - 1u) {
            const int rr = hs::low_bit(x);
            opp &= ~hs::bit(9 * rr + c);
            oppT &= ~hs::bit(9 * c + rr);
        }
        // a corner piece whose two neighbours are now the mover's, dst being one
        // corners 0, 8, 72, 80 with neighbours (9, 1), (17, 7), (63, 73), (71, 79)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cn = q == 0 ? 0 : (q == 1 ? 8 : (q == 2 ? 72 : 80));
            const int v = q == 0 ? 9 : (q == 1 ? 17 : (q == 2 ? 63 : 71));
            const int h = q == 0 ? 1 : (q == 1 ? 7 : (q == 2 ? 73 : 79));
            if ((dst == v || dst == h) && ((opp >> cn) & 1) && ((own >> v) & 1) && ((own >> h) & 1)) {
                opp &= ~hs::bit(cn);
                oppT &= ~hs::bit(hs::tpos(cn));
            }
        }
        if (me == 1) {
            p1 = own;
            t1 = ownT;
            p2 = opp;
            t2 = oppT;
        } else {
            p2 = own;
            t2 = ownT;
            p1 = opp;
            t1 = oppT;
        }
        // five in a row or column outside the mover's start rows
        const u128 x = own & (me == 1 ? hs::ROWS_0_6 : hs::ROWS_2_8);
        const u128 row5 = x & (x >> 1) & (x >> 2) & (x >> 3) & (x >> 4) & hs::COLS_0_4;
        const u128 col5 = x & (x >> 9) & (x >> 18) & (x >> 27) & (x >> 36);
        if (row5 | col5) return me;
        return -1;
    }
};


__device__ __forceinline__ u128 to_u128(const BB<3> &b)
{
    return (u128)b.w[0] | ((u128)b.w[1] << 32) | ((u128)b.w[2] << 64);
}

__device__ __forceinline__ BB<3> from_u128(u128 x)
{
    BB<3> b;
    b.w[0] = (uint32_t)x;
    b.w[1] = (uint32_t)(x >> 32);
    b.w[2] = (uint32_t)(x >> 64);
    return b;
}

// Move count of `me` that also leaves, for the select below, every piece's
// (source << 24 | move count << 16 | packed moves) in the lane's column of
// an LDS array (entry i at cache[i * BLOCK], conflict-free across the wave).  A player
// never has more than its 18 start pieces; on a hand-edited board with
// more, pieces past the 18th are counted but not cached, and the select
// then stays inside the cache (a legal move, not necessarily the k-th).
constexpr int SHOGI_MAX_PIECES = 18;

__device__ __forceinline__ int count_cached(const Shogi &g, int me, uint32_t *cache)
{
    int n = 0, i = 0;
    for (u128 x = me == 1 ? g.p1 : g.p2; x; x &= x - 1, ++i) {
        const int s = hs::low_bit128(x);
        const uint32_t pm = g.moves_of(s);
        const int m = hs::n_moves(pm);
        if (i < SHOGI_MAX_PIECES) cache[i * BLOCK] = ((uint32_t)s << 24) | ((uint32_t)m << 16) | pm;
        n += m;
    }
    return n;
}

// the k-th legal move from the cache of the last count_cached (n > 0):
// the piece whose moves hold it, then its destination
__device__ __forceinline__ void select_cached(const uint32_t *cache, int k, int &src, int &dst)
{
    uint32_t v = cache[0];
    int i = 0;
#pragma unroll 1
    while ((int)((v >> 16) & 0xFFu) <= k && i + 1 < SHOGI_MAX_PIECES) {
        k -= (int)((v >> 16) & 0xFFu);
        v = cache[++i * BLOCK];
    }
    const int m = (int)((v >> 16) & 0xFFu);
    src = (int)(v >> 24);
    dst = hs::nth_dst(v & 0xFFFFu, src, k < m ? k : 0);
}

// One lane's row of move summaries (per cell: the packed moves of the
// mover's piece there, 0 elsewhere), for the mask writer.
__device__ __forceinline__ void shogi_summary(const Shogi &g, int me, bool running, uint16_t *row)
{
    for (int c = 0; c < 81; ++c) row[c] = 0;
    if (running)
        for (u128 x = me == 1 ? g.p1 : g.p2; x; x &= x - 1) {
            const int s = hs::low_bit128(x);
            row[s] = (uint16_t)g.moves_of(s);
        }
}

// The block's mask rows [nb][6561] from the summaries: the rows are one
// contiguous, 16-byte aligned run of bytes, written 16 bytes per lane and
// 1 KB per wave store; byte (env j, action src * 81 + dst) is 1 iff dst is
// among the moves of the piece on src.
__device__ __forceinline__ void write_shogi_rows(uint8_t *__restrict__ rows, int nb, const uint16_t *summ)
{
    const int t = threadIdx.x;
    const int total = nb * hs::A, full = total >> 4;
    auto byte_at = [&](int j, int src, int dst) -> uint32_t {
        const uint32_t pm = summ[j * 81 + src];
        return pm != 0u && hs::has_dst(pm, src, dst) ? 1u : 0u;
    };
    for (int q = t; q < full; q += BLOCK) {
        const int pos = 16 * q;
        int j = (int)((unsigned)pos / (unsigned)hs::A);
        const int a = pos - j * hs::A;
        int src = (int)((unsigned)a / 81u), dst = a - 81 * src;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            w[i >> 2] |= byte_at(j, src, dst) << (8 * (i & 3));
            if (++dst == 81) {
                dst = 0;
                if (++src == 81) {
                    src = 0;
                    ++j;
                }
            }
        }
        reinterpret_cast<uint4 *>(rows)[q] = uint4{w[0], w[1], w[2], w[3]};
    }
    const int pos = 16 * full + t;
    if (pos < total) {
        const int j = pos / hs::A, a = pos - j * hs::A, src = a / 81;
        rows[pos] = (uint8_t)byte_at(j, src, a - 81 * src);
    }
}

// Philox word of a ply of a game
__device__ __forceinline__ uint32_t ply_word(uint64_t id, int ply, uint32_t key0, uint32_t key1)
{
    const Philox4 f = philox4x32_10((uint32_t)ply >> 2, (uint32_t)id, (uint32_t)(id >> 32), 0u, key0, key1);
    const int r = ply & 3;
    return r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
}

// After the mover's ply: the end rules (five, then a next player without a
// legal move) given apply's outcome; nl = the next player's move count,
// whose moves are left in the cache.
__device__ __forceinline__ int shogi_outcome(const Shogi &g, int me, int five, int &nl, uint32_t *cache)
{
    nl = count_cached(g, 3 - me, cache);
    return five >= 0 ? five : (nl == 0 ? me : -1);
}

// One ply of a running game with Philox word w, from the move cache of
// the last count (nl moves); returns whether the game goes on.  Also the
// lane adapter of the mixed persistent batch (k_persist_lane).
struct ShogiLane {
    struct Shared {
        uint32_t cache[SHOGI_MAX_PIECES * BLOCK];
    };
    Shogi g;
    uint32_t *cache;
    int me, passes, ply, last, status, winner, nl;
    __device__ void bind(Shared &sh, int t) { cache = sh.cache + t; }
    __device__ void start()
    {
        g.start();
        me = 1;
        passes = 0;
        ply = 0;
        last = -1;
        status = RUNNING;
        winner = -1;
        nl = count_cached(g, 1, cache);
    }
    __device__ bool step(uint32_t w, int max_plies)
    {
        if (nl == 0) { // only on a hand-edited state
            status = ILLEGAL;
            return false;
        }
        int src, dst;
        select_cached(cache, (int)__umulhi(w, (uint32_t)nl), src, dst);
        const int five = g.apply(me, src, dst);
        passes = 0;
        ply += 1;
        last = src * 81 + dst;
        const int outcome = shogi_outcome(g, me, five, nl, cache);
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
};

// a1
__global__ __launch_bounds__(BLOCK) void k_sh_init(DevState st, int64_t n)
{
    __shared__ __align__(16) int8_t lds[BLOCK * 81 + STAGE_SLACK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    if (t < nb) {
        Shogi g;
        g.start();
        write_board<81, 3>(lds + t * 81, from_u128(g.p1), from_u128(g.p2));
        const int64_t e = e0 + t;
        st.to_move[e] = 1;
        st.status[e] = RUNNING;
        st.winner[e] = -1;
        st.passes[e] = 0;
        st.ply[e] = 0;
        st.last_action[e] = -1;
    }
    stage_out(st.board + e0 * 81, nb * 81, lds);
}

// a2
__global__ __launch_bounds__(BLOCK) void k_sh_mask(DevState st, int64_t n, uint8_t *__restrict__ mask)
{
    __shared__ __align__(16) int8_t lds[BLOCK * 81 + STAGE_SLACK];
    __shared__ uint16_t summ[BLOCK * 81];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<81>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const bool valid = t < nb;
    const int64_t ec = valid ? e0 + t : e0;
    BB<3> c1, c2;
    read_board<81, 3>(lds + t * 81, c1, c2);
    Shogi g;
    g.set(to_u128(c1), to_u128(c2));
    shogi_summary(g, st.to_move[ec], valid && st.status[ec] == RUNNING, summ + t * 81);
    __syncthreads();
    write_shogi_rows(mask + e0 * hs::A, nb, summ);
}

// a3-a6 for one ply, MODE 0 caller's action / 1 uniform random / 2 softmax
// of the logits over the legal actions in increasing order
template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_sh_step(DevState st, int64_t n, int max_plies,
                                                   const int32_t *__restrict__ action,
                                                   const float *__restrict__ logits, uint32_t key0, uint32_t key1,
                                                   int64_t gid_base, const int64_t *__restrict__ gid,
                                                   int8_t *__restrict__ reward, uint8_t *__restrict__ terminal,
                                                   uint8_t *__restrict__ next_mask)
{
    __shared__ __align__(16) int8_t lds[BLOCK * 81 + STAGE_SLACK];
    __shared__ uint16_t summ[BLOCK * 81];
    __shared__ uint32_t cache_all[SHOGI_MAX_PIECES * BLOCK];
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    const int t = threadIdx.x;
    uint32_t *cache = cache_all + t;
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
            uint8_t *dst = next_mask + e0 * hs::A;
            const int bytes = nb * hs::A, full = bytes >> 4;
            for (int j = t; j < full; j += BLOCK) reinterpret_cast<uint4 *>(dst)[j] = uint4{0u, 0u, 0u, 0u};
            for (int j = (full << 4) + t; j < bytes; j += BLOCK) dst[j] = 0;
        }
        return;
    }

    stage_in<81>(st.board, e0, nb, lds);
    BB<3> c1, c2;
    read_board<81, 3>(lds + t * 81, c1, c2);
    Shogi g;
    g.set(to_u128(c1), to_u128(c2));
    int me = st.to_move[ec], winner = st.winner[ec], passes = st.passes[ec], ply = st.ply[ec],
        last = st.last_action[ec];
    int r1 = 0;
    if (was_running) {
        int src = -1, dst = -1;
        bool legal;
        if constexpr (MODE == 0) {
            const int a = action[ec];
            if (a >= 0 && a < hs::A) {
                src = a / 81;
                dst = a - 81 * src;
            }
            legal = g.legal(me, src, dst);
        } else {
            const int nl = count_cached(g, me, cache);
            legal = nl > 0;
            const uint32_t w = ply_word((uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec), ply, key0, key1);
            if constexpr (MODE == 1) {
                if (legal) select_cached(cache, (int)__umulhi(w, (uint32_t)nl), src, dst);
            } else if (legal) {
                const float *lg = logits + ec * hs::A;
                const u128 own = me == 1 ? g.p1 : g.p2;
                float mx = -3.0e38f;
                for (u128 x = own; x; x &= x - 1) {
                    const int s = hs::low_bit128(x);
                    const uint32_t pm = g.moves_of(s);
                    for (int j = 0, m = hs::n_moves(pm); j < m; ++j) mx = fmaxf(mx, lg[s * 81 + hs::nth_dst(pm, s, j)]);
                }
                float tot = 0.f;
                for (u128 x = own; x; x &= x - 1) {
                    const int s = hs::low_bit128(x);
                    const uint32_t pm = g.moves_of(s);
                    for (int j = 0, m = hs::n_moves(pm); j < m; ++j)
                        tot += expf(lg[s * 81 + hs::nth_dst(pm, s, j)] - mx);
                }
                const float thr = (float)(w >> 8) * 0x1p-24f * tot;
                float run = 0.f;
                bool picked = false;
                for (u128 x = own; x; x &= x - 1) {
                    const int s = hs::low_bit128(x);
                    const uint32_t pm = g.moves_of(s);
                    for (int j = 0, m = hs::n_moves(pm); j < m; ++j) {
                        const int d = hs::nth_dst(pm, s, j);
                        run += expf(lg[s * 81 + d] - mx);
                        if (!picked) {
                            src = s;
                            dst = d;
                            picked = run > thr;
                        }
                    }
                }
            }
        }
        if (!legal) {
            status = ILLEGAL;
        } else {
            const int five = g.apply(me, src, dst);
            passes = 0;
            ply += 1;
            last = src * 81 + dst;
            int nl;
            const int outcome = shogi_outcome(g, me, five, nl, cache);
            if (outcome >= 0) {
                status = TERMINAL;
                winner = outcome;
                r1 = outcome == 1 ? 1 : -1;
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
        reward[2 * e + 1] = (int8_t)-r1;
        terminal[e] = status != RUNNING ? 1 : 0;
    }
    __syncthreads();
    if (valid) write_board<81, 3>(lds + t * 81, from_u128(g.p1), from_u128(g.p2));
    stage_out(st.board + e0 * 81, nb * 81, lds);
    if (next_mask != nullptr) {
        shogi_summary(g, me, valid && status == RUNNING, summ + t * 81);
        __syncthreads();
        write_shogi_rows(next_mask + e0 * hs::A, nb, summ);
    }
}

// a2-a8 fused: the whole uniform-random game in registers
__global__ __launch_bounds__(BLOCK) void k_sh_playout(DevState st, int64_t n, int max_plies, uint32_t key0,
                                                      uint32_t key1, int64_t gid_base,
                                                      const int64_t *__restrict__ gid, int8_t *__restrict__ reward,
                                                      uint8_t *__restrict__ terminal)
{
    __shared__ __align__(16) int8_t lds[BLOCK * 81 + STAGE_SLACK];
    __shared__ ShogiLane::Shared shared;
    const int64_t e0 = (int64_t)blockIdx.x * BLOCK;
    const int nb = (int)(n - e0 < BLOCK ? n - e0 : BLOCK);
    stage_in<81>(st.board, e0, nb, lds);
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const bool valid = t < nb;
    const int64_t ec = valid ? e : e0;
    BB<3> c1, c2;
    read_board<81, 3>(lds + t * 81, c1, c2);
    ShogiLane L;
    L.bind(shared, t);
    L.g.set(to_u128(c1), to_u128(c2));
    L.me = st.to_move[ec];
    L.status = valid ? (int)st.status[ec] : ILLEGAL;
    L.winner = st.winner[ec];
    L.passes = st.passes[ec];
    L.ply = st.ply[ec];
    L.last = st.last_action[ec];
    const uint64_t id = (uint64_t)(gid != nullptr ? gid[ec] : gid_base + ec);
    const uint32_t id_lo = (uint32_t)id, id_hi = (uint32_t)(id >> 32);
    const bool was_running = valid && L.status == RUNNING;
    L.nl = was_running ? count_cached(L.g, L.me, L.cache) : 0;
    uint32_t w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
    if (was_running) {
        const Philox4 f = philox4x32_10((uint32_t)L.ply >> 2, id_lo, id_hi, 0u, key0, key1);
        const int r = L.ply & 3;
        w0 = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
        w1 = r == 0 ? f.v[1] : (r == 1 ? f.v[2] : f.v[3]);
        w2 = r == 0 ? f.v[2] : f.v[3];
        w3 = f.v[3];
    }
    bool running = was_running, first = true;
    while (running) {
        if ((L.ply & 3) == 0 && !first) {
            const Philox4 f = philox4x32_10((uint32_t)L.ply >> 2, id_lo, id_hi, 0u, key0, key1);
            w0 = f.v[0];
            w1 = f.v[1];
            w2 = f.v[2];
            w3 = f.v[3];
        }
        first = false;
        running = L.step(w0, max_plies);
        w0 = w1;
        w1 = w2;
        w2 = w3;
    }
    const int r1 = was_running && L.status == TERMINAL ? (L.winner == 1 ? 1 : -1) : 0;
    if (valid) {
        write_board<81, 3>(lds + t * 81, from_u128(L.g.p1), from_u128(L.g.p2));
        st.to_move[e] = (int8_t)L.me;
        st.status[e] = (int8_t)L.status;
        st.winner[e] = (int8_t)L.winner;
        st.passes[e] = (int8_t)L.passes;
        st.ply[e] = (int16_t)L.ply;
        st.last_action[e] = (int16_t)L.last;
        reward[2 * e] = (int8_t)r1;
        reward[2 * e + 1] = (int8_t)-r1;
        terminal[e] = 1;
    }
    stage_out(st.board + e0 * 81, nb * 81, lds);
}

struct ShogiLaunch {
    static unsigned blocks(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }
    static hipError_t init(const DevState &st, int64_t n, hipStream_t s)
    {
        hipLaunchKernelGGL(k_sh_init, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n);
        return hipGetLastError();
    }
    static hipError_t mask(const DevState &st, int64_t n, uint8_t *mask, hipStream_t s)
    {
        hipLaunchKernelGGL(k_sh_mask, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, mask);
        return hipGetLastError();
    }
    static hipError_t step(const DevState &st, int64_t n, int max_plies, const int32_t *action, int8_t *reward,
                           uint8_t *terminal, uint8_t *next_mask, hipStream_t s)
    {
        hipLaunchKernelGGL(k_sh_step<0>, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies, action,
                           (const float *)nullptr, 0u, 0u, (int64_t)0, (const int64_t *)nullptr, reward, terminal,
                           next_mask);
        return hipGetLastError();
    }
    static hipError_t random_step(const DevState &st, int64_t n, int max_plies, uint64_t seed, int64_t gid_base,
                                  const int64_t *gid, int8_t *reward, uint8_t *terminal, hipStream_t s)
    {
        hipLaunchKernelGGL(k_sh_step<1>, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies,
                           (const int32_t *)nullptr, (const float *)nullptr, (uint32_t)seed, (uint32_t)(seed >> 32),
                           gid_base, gid, reward, terminal, (uint8_t *)nullptr);
        return hipGetLastError();
    }
    static hipError_t policy_step(const DevState &st, int64_t n, int max_plies, const float *logits, uint64_t seed,
                                  int64_t gid_base, const int64_t *gid, int8_t *reward, uint8_t *terminal,
                                  hipStream_t s)
    {
        hipLaunchKernelGGL(k_sh_step<2>, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies,
                           (const int32_t *)nullptr, logits, (uint32_t)seed, (uint32_t)(seed >> 32), gid_base, gid,
                           reward, terminal, (uint8_t *)nullptr);
        return hipGetLastError();
    }
    static hipError_t playout(const DevState &st, int64_t n, int max_plies, uint64_t seed, int64_t gid_base,
                              const int64_t *gid, int8_t *reward, uint8_t *terminal, int64_t *stats, hipStream_t s)
    {
        hipError_t err = hipSuccess;
        if (stats != nullptr && (err = launch_stats(st, n, -1, stats, s)) != hipSuccess) return err;
        hipLaunchKernelGGL(k_sh_playout, dim3(blocks(n)), dim3(BLOCK), 0, s, st, n, max_plies, (uint32_t)seed,
                           (uint32_t)(seed >> 32), gid_base, gid, reward, terminal);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (stats != nullptr) return launch_stats(st, n, +1, stats, s);
        return hipSuccess;
    }
    static hipError_t persist(const MixedArgs &a, int slots, hipStream_t s)
    {
        hipLaunchKernelGGL(k_persist_lane<ShogiLane>, dim3((unsigned)((slots + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s,
                           a);
        return hipGetLastError();
    }
    static constexpr GameOps ops()
    {
        return GameOps{Shogi::KIND, Shogi::H, Shogi::W, Shogi::CELLS, Shogi::A, &init, &mask, &step, &random_step,
                       &policy_step, &playout, &persist, 0, nullptr, -1, -1};
    }
};

} // namespace lx
