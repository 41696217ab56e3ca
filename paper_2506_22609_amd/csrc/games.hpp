// games.hpp -- the rule sets as env-per-lane bitboard state machines.
//
// Every game keeps the two players' stones as bitboards in registers, in an
// internal bit layout chosen so that line and neighbour tests are shifts:
//   Tic-Tac-Toe   bit = cell (9 bits)
//   Connect Four  row stride 8 (a zero guard column stops horizontal and
//                 diagonal shifts from wrapping), 48 bits
//   Reversi       bit = cell (64 bits); column masks stop wrapping
//   Hex N         bit = cell (N*N bits); column masks stop wrapping
//   Gomoku N      row stride N+1 (zero guard column), N*(N+1) bits
//   Pente N       row stride N+1 (zero guard column), N*(N+1) bits
//   Yavalath D    axial (r, q) at bit r*(D+1) + q inside a D x (D+1)
//                 rhombus; the guard column and the corners outside the
//                 hexagon stay zero
// Every internal layout is increasing in the cell index, so "the k-th legal
// cell in index order" is the k-th set bit of the internal legal mask.
//
// Interface of a game type G (used by the kernels):
//   KIND, H, W, CELLS, A, NWC (words of a cell-indexed bitboard), NWI (words
//   of the internal layout), HAS_PASS
//   from_canon / to_canon: cell-indexed <-> internal layout
//   load(c1, c2) / store(c1, c2): whole state from / to cell-indexed boards
//   placements(me): internal mask of legal placements for player `me`
//   action_of(bit) / bit_of(action)
//   place(bit, me, extra): apply a legal placement, return the end-rule
//                   outcome: -1 the game goes on, 0 draw, 1 or 2 the winner;
//                   extra is the state's per-game byte (Reversi: consecutive
//                   passes, reset by a placement; Pente: captured pairs)
//   pass(passes): Reversi's forced pass
#pragma once

#include "bitboard.hpp"

namespace lx {

// ---------------------------------------------------------------------------
// generic cell-layout helpers
// ---------------------------------------------------------------------------

// Read LEN <= 32 bits starting at compile-time bit position POS.
template <int POS, int LEN, int NW>
__device__ __forceinline__ uint32_t get_field(const BB<NW> &x)
{
    constexpr int q = POS / 32, s = POS % 32;
    constexpr uint32_t m = LEN == 32 ? 0xFFFFFFFFu : ((1u << LEN) - 1u);
    uint32_t v = x.w[q] >> s;
    if constexpr (s + LEN > 32 && q + 1 < NW) v |= x.w[q + 1 < NW ? q + 1 : 0] << (32 - s);
    return v & m;
}

// OR a LEN-bit value into compile-time bit position POS.
template <int POS, int LEN, int NW>
__device__ __forceinline__ void or_field(BB<NW> &x, uint32_t v)
{
    constexpr int q = POS / 32, s = POS % 32;
    x.w[q] |= v << s;
    if constexpr (s + LEN > 32 && q + 1 < NW) x.w[q + 1 < NW ? q + 1 : 0] |= v >> (32 - s);
}

// Re-stride rows: cell (r, c) at bit r*FROM + c -> bit r*TO + c, c < W.
template <int H, int W, int FROM, int TO, int NWF, int NWT>
__device__ __forceinline__ BB<NWT> restride(const BB<NWF> &x)
{
    BB<NWT> r = bb_zero<NWT>();
    static_for<H>([&](auto R) {
        constexpr int row = R;
        or_field<row * TO, W>(r, get_field<row * FROM, W>(x));
    });
    return r;
}

// ---------------------------------------------------------------------------
// Tic-Tac-Toe (App. C): a line of three wins, then a full board draws.
// ---------------------------------------------------------------------------
struct TicTacToe {
    static constexpr int KIND = 1, H = 3, W = 3, CELLS = 9, A = 9, NWC = 1, NWI = 1, NBITS = 9;
    static constexpr bool HAS_PASS = false;
    using M = BB<1>;
    M p1, p2;

    __device__ static M from_canon(const BB<NWC> &c) { return c; }
    __device__ static BB<NWC> to_canon(const M &m) { return m; }
    __device__ static int action_of(int b) { return b; }
    __device__ static int bit_of(int a) { return a; }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = c1; p2 = c2; }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = p1; c2 = p2; }
    __device__ void prepare() {}

    __device__ M placements(int) const
    {
        M m;
        m.w[0] = ~(p1.w[0] | p2.w[0]) & 0x1FFu;
        return m;
    }

    // legal placements for either player given both stone sets, and the
    // win predicate of one player's stones (both monotone in the stones)
    __device__ static M open_cells(const M &a, const M &b)
    {
        M m;
        m.w[0] = ~(a.w[0] | b.w[0]) & 0x1FFu;
        return m;
    }
    __device__ static bool line(const M &x) { return three(x.w[0]); }

    __device__ static bool three(uint32_t x)
    {
        // rows, columns, diagonals of the 3x3 board
        constexpr uint32_t L[8] = {0x007u, 0x038u, 0x1C0u, 0x049u, 0x092u, 0x124u, 0x111u, 0x054u};
        bool w = false;
#pragma unroll
        for (int i = 0; i < 8; ++i) w = w | ((x & L[i]) == L[i]);
        return w;
    }

    __device__ int place(int b, int me, int &extra)
    {
        const uint32_t bit = 1u << b;
        uint32_t own = (me == 1 ? p1.w[0] : p2.w[0]) | bit;
        if (me == 1) p1.w[0] = own;
        else p2.w[0] = own;
        if (three(own)) return me;
        if ((p1.w[0] | p2.w[0]) == 0x1FFu) return 0;
        return -1;
    }
    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }
    __device__ int pass(int &) { return -1; }
};

// ---------------------------------------------------------------------------
// Connect Four 6x7 (App. C; Sec. 3.4): a placement must rest on the floor
// or on a piece; four or more in a line wins; then a full board draws.
// Internal bit of (r, c) = 8r + c; column 7 is an always-empty guard.
// ---------------------------------------------------------------------------
struct ConnectFour {
    static constexpr int KIND = 2, H = 6, W = 7, CELLS = 42, A = 42, NWC = 2, NWI = 2;
    static constexpr int S = 8, NBITS = H * S;
    static constexpr bool HAS_PASS = false;
    using M = BB<NWI>;
    M p1, p2;

    struct Valid {
        constexpr bool operator()(int b) const { return (b % S) < W; }
    };
    struct Floor {
        constexpr bool operator()(int b) const { return b / S == H - 1 && (b % S) < W; }
    };

    __device__ static M from_canon(const BB<NWC> &c) { return restride<H, W, W, S, NWC, NWI>(c); }
    __device__ static BB<NWC> to_canon(const M &m) { return restride<H, W, S, W, NWI, NWC>(m); }
    __device__ static int action_of(int b) { return (b >> 3) * W + (b & 7); }
    __device__ static int bit_of(int a) { return (a / W) * S + (a % W); }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = from_canon(c1); p2 = from_canon(c2); }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = to_canon(p1); c2 = to_canon(p2); }
    __device__ void prepare() {}

    // legal placements for either player given both stone sets: empty
    // cells whose lower neighbour (bit + 8) is occupied, or on the floor
    __device__ static M open_cells(const M &a, const M &b)
    {
        const M occ = a | b;
        const M support = shr<S>(occ) | const_mask<Floor, NBITS, NWI>();
        return and_mask<Valid, NBITS, NWI>(andnot(support, occ));
    }
    __device__ M placements(int) const { return open_cells(p1, p2); }

    // the win predicate of one player's stones: four or more in a line
    __device__ static bool line(const M &x)
    {
        return four_along<1>(x) | four_along<S>(x) | four_along<S - 1>(x) | four_along<S + 1>(x);
    }

    template <int D>
    __device__ static bool four_along(const M &x)
    {
        const M a = x & shr<D>(x);
        return any(a & shr<2 * D>(a));
    }

    __device__ int place(int b, int me, int &extra)
    {
        M own = pick(me == 1, p1, p2) | onehot<NWI>(b);
        p1 = pick(me == 1, own, p1);
        p2 = pick(me == 1, p2, own);
        if (line(own)) return me;
        const M occ = p1 | p2;
        if (same(occ, const_mask<Valid, NBITS, NWI>())) return 0;
        return -1;
    }
    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }
    __device__ int pass(int &) { return -1; }
};

// ---------------------------------------------------------------------------
// Hex NxN (App. C): parallelogram board; (r, c) touches (r-1, c), (r-1, c+1),
// (r, c-1), (r, c+1), (r+1, c-1), (r+1, c).  Player 1 joins row 0 to row
// N-1, player 2 column 0 to column N-1.  No draws (every full board has
// exactly one connected player), so the only end rule is the mover's
// connection.
//
// The single-step kernel floods the new stone's group (6-neighbour
// dilation by shifts, repeated until it stops growing) and checks both
// sides.  The playout kernel does not test connection ply by ply at all:
// see k_playout_fill in kernels.hpp.
// ---------------------------------------------------------------------------
template <int N>
struct Hex {
    static constexpr int KIND = 3, H = N, W = N, CELLS = N * N, A = N * N;
    static constexpr int NWC = (CELLS + 31) / 32, NWI = NWC, NBITS = CELLS;
    static constexpr bool HAS_PASS = false;
    using M = BB<NWI>;
    M p1, p2;

    struct Col0 {
        constexpr bool operator()(int b) const { return b % N == 0; }
    };
    struct ColL {
        constexpr bool operator()(int b) const { return b % N == N - 1; }
    };
    struct NotCol0 {
        constexpr bool operator()(int b) const { return b % N != 0; }
    };
    struct NotColL {
        constexpr bool operator()(int b) const { return b % N != N - 1; }
    };
    struct Row0 {
        constexpr bool operator()(int b) const { return b < N; }
    };
    struct RowL {
        constexpr bool operator()(int b) const { return b >= N * (N - 1); }
    };

    __device__ static M from_canon(const BB<NWC> &c) { return c; }
    __device__ static BB<NWC> to_canon(const M &m) { return m; }
    __device__ static int action_of(int b) { return b; }
    __device__ static int bit_of(int a) { return a; }

    // stones of player p on p's first / far side
    __device__ static M first_side(const M &x, int p)
    {
        return p == 1 ? and_mask<Row0, NBITS, NWI>(x) : and_mask<Col0, NBITS, NWI>(x);
    }
    __device__ static bool meets_far_side(const M &x, int p)
    {
        return p == 1 ? any(and_mask<RowL, NBITS, NWI>(x)) : any(and_mask<ColL, NBITS, NWI>(x));
    }
    // first_side / meets_far_side for a per-lane player (p1: player 1)
    // without a branch on it: both sides' tests, then a select
    __device__ static M first_side_sel(const M &x, bool p1)
    {
        return pick(p1, and_mask<Row0, NBITS, NWI>(x), and_mask<Col0, NBITS, NWI>(x));
    }
    __device__ static bool meets_far_side_sel(const M &x, bool p1)
    {
        const bool row = any(and_mask<RowL, NBITS, NWI>(x));
        const bool col = any(and_mask<ColL, NBITS, NWI>(x));
        return (p1 & row) | (!p1 & col);
    }
    // do p's stones `x` join p's two sides?
    __device__ static bool joins(const M &x, int p)
    {
        M r = first_side(x, p);
        return flood_to_far(r, x, p);
    }

    // x plus its six neighbours, clipped to the board.  With y = x plus the
    // right neighbours (r, c+1) and z = x plus the left neighbours (r, c-1),
    // the row above contributes (r-1, c), (r-1, c+1) = y shifted up and the
    // row below (r+1, c), (r+1, c-1) = z shifted down: four shifts in all.
    __device__ static M dilate(const M &x)
    {
        if constexpr (N == 1) {
            return x;
        } else {
            // a wrap lands in column 0 (or past the last cell) / in column N-1
            const M y = x | and_mask<NotCol0, NBITS, NWI>(shl<1>(x));
            const M z = x | and_mask<NotColL, NBITS, NWI>(shr<1>(x));
            return and_mask<AllBits, NBITS, NWI>(y | z | shr<N>(y) | shl<N>(z));
        }
    }

    // grow `seed` inside `allowed` to its connected closure (seed within
    // allowed); two dilations per convergence test
    __device__ static M flood(M seed, const M &allowed)
    {
        for (;;) {
            const M n1 = dilate(seed) & allowed;
            const M n2 = dilate(n1) & allowed;
            seed = n2;
            if (same(n2, n1)) return seed;
        }
    }

    // grow `r` inside `allowed` until it stops growing or meets p's far
    // side (growth is monotone, so testing every second dilation is
    // enough); returns whether it met the far side
    __device__ static bool flood_to_far(M &r, const M &allowed, int p)
    {
        for (;;) {
            const M n1 = dilate(r) & allowed;
            const M n2 = dilate(n1) & allowed;
            r = n2;
            if (same(n2, n1) | meets_far_side(n2, p)) return meets_far_side(n2, p);
        }
    }

    // flood_to_far for a per-lane player (p1: player 1): the same rounds
    // without a branch on the player
    __device__ static bool flood_to_far_sel(M &r, const M &allowed, bool p1)
    {
        for (;;) {
            const M n1 = dilate(r) & allowed;
            const M n2 = dilate(n1) & allowed;
            r = n2;
            const bool hit = meets_far_side_sel(n2, p1);
            if (hit | same(n2, n1)) return hit;
        }
    }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = c1; p2 = c2; }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = p1; c2 = p2; }
    __device__ void prepare() {}

    __device__ static M open_cells(const M &a, const M &b) { return and_mask<AllBits, NBITS, NWI>(~(a | b)); }
    __device__ M placements(int) const { return open_cells(p1, p2); }

    // place and test the new stone's group against both sides
    __device__ int place(int b, int me, int &extra)
    {
        const M s = onehot<NWI>(b);
        const M own = pick(me == 1, p1, p2) | s;
        p1 = pick(me == 1, own, p1);
        p2 = pick(me == 1, p2, own);
        const M g = flood(s, own);
        const bool won = any(first_side(g, me)) && meets_far_side(g, me);
        return won ? me : -1;
    }
    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }
    __device__ int pass(int &) { return -1; }
};

// ---------------------------------------------------------------------------
// Reversi 8x8 (App. C): a placement must sandwich at least one line of the
// opponent's discs between the new disc and one of the mover's; every such
// line flips.  With no placement the mover must pass (PASS = action 64).
// Two passes in a row end the game; most discs wins, equal counts draw.
// ---------------------------------------------------------------------------
struct Reversi {
    static constexpr int KIND = 4, H = 8, W = 8, CELLS = 64, A = 65, NWC = 2, NWI = 2, NBITS = 64;
    static constexpr bool HAS_PASS = true;
    using M = BB<2>;
    M p1, p2;

    struct Col0 {
        constexpr bool operator()(int b) const { return b % 8 == 0; }
    };
    struct Col7 {
        constexpr bool operator()(int b) const { return b % 8 == 7; }
    };

    __device__ static M from_canon(const BB<NWC> &c) { return c; }
    __device__ static BB<NWC> to_canon(const M &m) { return m; }
    __device__ static int action_of(int b) { return b; }
    __device__ static int bit_of(int a) { return a; }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = c1; p2 = c2; }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = p1; c2 = p2; }
    __device__ void prepare() {}

    // one step in direction D (0..7): E, W, S, N, SE, SW, NE, NW
    template <int D>
    __device__ static M step(const M &x)
    {
        if constexpr (D == 0) return andnot_mask<Col0, 64, 2>(shl<1>(x));
        else if constexpr (D == 1) return andnot_mask<Col7, 64, 2>(shr<1>(x));
        else if constexpr (D == 2) return shl<8>(x);
        else if constexpr (D == 3) return shr<8>(x);
        else if constexpr (D == 4) return andnot_mask<Col0, 64, 2>(shl<9>(x));
        else if constexpr (D == 5) return andnot_mask<Col7, 64, 2>(shl<7>(x));
        else if constexpr (D == 6) return andnot_mask<Col0, 64, 2>(shr<7>(x));
        else return andnot_mask<Col7, 64, 2>(shr<9>(x));
    }

    template <int D, int K>
    __device__ static M shift_k(const M &x)
    {
        // K steps along D at once: the shift amount times K
        if constexpr (D == 0) return shl<K>(x);
        else if constexpr (D == 1) return shr<K>(x);
        else if constexpr (D == 2) return shl<8 * K>(x);
        else if constexpr (D == 3) return shr<8 * K>(x);
        else if constexpr (D == 4) return shl<9 * K>(x);
        else if constexpr (D == 5) return shl<7 * K>(x);
        else if constexpr (D == 6) return shr<7 * K>(x);
        else return shr<9 * K>(x);
    }
    // the cells where a step along D may land (a step that wraps around a
    // row edge lands in the first or the last column)
    template <int D>
    __device__ static M landing(const M &x)
    {
        if constexpr (D == 0 || D == 4 || D == 6) return andnot_mask<Col0, 64, 2>(x);
        else if constexpr (D == 1 || D == 5 || D == 7) return andnot_mask<Col7, 64, 2>(x);
        else return x;
    }

    // `gen` extended along D over the cells of `pro` (already restricted to
    // landing cells) by doubling steps: runs of up to seven cells, three
    // shifts of the growing set and two of the propagator
    template <int D>
    __device__ static M fill(M gen, M pro)
    {
        gen = gen | (pro & shift_k<D, 1>(gen));
        pro = pro & shift_k<D, 1>(pro);
        gen = gen | (pro & shift_k<D, 2>(gen));
        pro = pro & shift_k<D, 2>(pro);
        return gen | (pro & shift_k<D, 4>(gen));
    }

    __device__ M placements(int me) const
    {
        const M own = pick(me == 1, p1, p2);
        const M opp = pick(me == 1, p2, p1);
        const M empty = ~(p1 | p2);
        // walking from the mover's discs over a run of the opponent's along
        // D lands on exactly the empty cells that flank along -D; all eight
        // directions together give every legal placement
        M m = bb_zero<2>();
        static_for<8>([&](auto Dc) {
            constexpr int D = Dc;
            const M run = andnot(fill<D>(own, landing<D>(opp)), own); // opponent's discs reached
            m = m | (shift_k<D, 1>(run) & landing<D>(empty));
        });
        return m;
    }

    __device__ int place(int b, int me, int &extra)
    {
        const M s = onehot<2>(b);
        M own = pick(me == 1, p1, p2);
        M opp = pick(me == 1, p2, p1);
        // opponent discs flipped along D: the run of them from s, when a
        // disc of the mover closes it
        M f = bb_zero<2>();
        static_for<8>([&](auto Dc) {
            constexpr int D = Dc;
            const M run = fill<D>(s, landing<D>(opp)); // s and the run after it
            const bool closed = any(shift_k<D, 1>(run) & landing<D>(own));
            f = f | (closed ? andnot(run, s) : bb_zero<2>());
        });
        own = own | f | s;
        opp = andnot(opp, f);
        p1 = pick(me == 1, own, opp);
        p2 = pick(me == 1, opp, own);
        extra = 0; // a placement ends a run of passes
        return -1;
    }

    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }

    __device__ int pass(int &passes)
    {
        passes += 1;
        if (passes < 2) return -1;
        const int n1 = popcount(p1), n2 = popcount(p2);
        return n1 > n2 ? 1 : (n2 > n1 ? 2 : 0);
    }
};

// ---------------------------------------------------------------------------
// Gomoku NxN (App. C): a maximal line of exactly five wins (six or more does
// not count), then a full board draws.  Internal bit of (r, c) = r(N+1) + c;
// column N is an always-empty guard.
// ---------------------------------------------------------------------------
template <int N>
struct Gomoku {
    static constexpr int KIND = 5, H = N, W = N, CELLS = N * N, A = N * N;
    static constexpr int S = N + 1, NBITS = N * S;
    static constexpr int NWC = (CELLS + 31) / 32, NWI = (NBITS + 31) / 32;
    static constexpr bool HAS_PASS = false;
    using M = BB<NWI>;
    M p1, p2;

    struct Valid {
        constexpr bool operator()(int b) const { return (b % S) < N; }
    };

    __device__ static M from_canon(const BB<NWC> &c) { return restride<N, N, N, S, NWC, NWI>(c); }
    __device__ static BB<NWC> to_canon(const M &m) { return restride<N, N, S, N, NWI, NWC>(m); }
    __device__ static int action_of(int b) { return (b / S) * N + (b % S); }
    __device__ static int bit_of(int a) { return (a / N) * S + (a % N); }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = from_canon(c1); p2 = from_canon(c2); }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = to_canon(p1); c2 = to_canon(p2); }
    __device__ void prepare() {}

    __device__ M placements(int) const { return and_mask<Valid, NBITS, NWI>(~(p1 | p2)); }

    // starts i of runs of five or more along step D (i .. i+4D all set)
    template <int D>
    __device__ static M five_plus(const M &x)
    {
        const M a1 = x & shr<D>(x);       // i, i+D
        const M a2 = a1 & shr<2 * D>(a1); // i .. i+3D
        return a2 & shr<4 * D>(x);        // i .. i+4D
    }
    // among those, a run of exactly five: neither i-D nor i+5D set
    template <int D>
    __device__ static bool exact_five(const M &x, const M &a3)
    {
        return any(andnot(andnot(a3, shl<D>(x)), shr<5 * D>(x)));
    }
    // a run of exactly five in some direction; the exactness shifts run only
    // where some run of five or more exists (in a game, at its last ply)
    __device__ static bool any_exact_five(const M &x)
    {
        const M h = five_plus<1>(x), v = five_plus<S>(x), d1 = five_plus<S - 1>(x), d2 = five_plus<S + 1>(x);
        if (!any(h | v | d1 | d2)) return false;
        return exact_five<1>(x, h) | exact_five<S>(x, v) | exact_five<S - 1>(x, d1) | exact_five<S + 1>(x, d2);
    }

    // place player me's stone on cell b: me's win, else a draw when `full`
    // (the board is full after this stone), else -1.  The stone's word is
    // picked by word masks, per player (no select between whole boards).
    __device__ int place_full(int b, int me, bool full)
    {
        const uint32_t bit = 1u << (b & 31);
        const int sel = word_sel(b >> 5);
        const int s1 = me == 1 ? sel : 0, s2 = sel ^ s1;
#pragma unroll
        for (int i = 0; i < NWI; ++i) {
            p1.w[i] |= bit & word_mask(s1, i);
            p2.w[i] |= bit & word_mask(s2, i);
        }
        if (any_exact_five(pick(me == 1, p1, p2))) return me;
        return full ? 0 : -1;
    }
    __device__ int place(int b, int me, int &extra)
    {
        const int r = place_full(b, me, false);
        if (r >= 0) return r;
        return popcount(p1 | p2) == CELLS ? 0 : -1;
    }
    // a random ply knows the number of empty cells before its stone
    __device__ int place_drawn(int b, int me, int &extra, int n_legal) { return place_full(b, me, n_legal == 1); }
    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }
    __device__ int pass(int &) { return -1; }
};

// ---------------------------------------------------------------------------
// Yavalath (App. C) on a regular hexagon of diameter D (odd, side
// SIDE = (D+1)/2): four or more in a row wins, else three in a row (no
// four) loses, else a full board draws.  Cells are numbered row by row from
// the top, row r holding D - |r - (SIDE-1)| cells; cell i of row r has axial
// q = i + max(0, SIDE-1-r).  Straight lines run along (0, 1), (1, 0) and
// (1, -1), which in the internal layout are the shifts 1, D + 1 and D.  Only
// the mover's stones can form a new line, and a mover who already had a line
// would have ended the game, so full-board tests of the mover's stones are
// exact: some four -> win, else some three -> every run is at most three
// long, so any three is an exact three -> loss.
// ---------------------------------------------------------------------------
template <int D>
struct Yavalath {
    static_assert(D % 2 == 1 && D >= 3, "odd diameter");
    static constexpr int KIND = 6, H = D, W = D, SIDE = (D + 1) / 2;
    static constexpr int CELLS = 3 * SIDE * (SIDE - 1) + 1, A = CELLS;
    static constexpr int S = D + 1, NBITS = D * S;
    static constexpr int NWC = (CELLS + 31) / 32, NWI = (NBITS + 31) / 32;
    static constexpr bool HAS_PASS = false;
    using M = BB<NWI>;
    M p1, p2;

    __host__ __device__ static constexpr int rlen(int r) { return D - (r > SIDE - 1 ? r - (SIDE - 1) : SIDE - 1 - r); }
    __host__ __device__ static constexpr int q0(int r) { return r < SIDE - 1 ? SIDE - 1 - r : 0; }
    // first cell of row r (closed forms: rows grow by one to the middle row, then shrink)
    __host__ __device__ static constexpr int rstart(int r)
    {
        if (r <= SIDE - 1) return r * SIDE + r * (r - 1) / 2;
        const int mid = (SIDE - 1) * SIDE + (SIDE - 1) * (SIDE - 2) / 2, k = r - SIDE;
        return mid + D + k * D - k * (k + 1) / 2;
    }
    static_assert(rstart(D) == CELLS, "row starts");

    struct Valid {
        constexpr bool operator()(int b) const
        {
            const int r = b / S, q = b % S;
            return r < D && q >= q0(r) && q < q0(r) + rlen(r);
        }
    };

    __device__ static M from_canon(const BB<NWC> &c)
    {
        M m = bb_zero<NWI>();
        static_for<D>([&](auto R) {
            constexpr int r = R;
            or_field<r * S + q0(r), rlen(r)>(m, get_field<rstart(r), rlen(r)>(c));
        });
        return m;
    }
    __device__ static BB<NWC> to_canon(const M &m)
    {
        BB<NWC> c = bb_zero<NWC>();
        static_for<D>([&](auto R) {
            constexpr int r = R;
            or_field<rstart(r), rlen(r)>(c, get_field<r * S + q0(r), rlen(r)>(m));
        });
        return c;
    }
    __device__ static int action_of(int b)
    {
        const int r = b / S;
        return rstart(r) + (b % S) - q0(r);
    }
    __device__ static int bit_of(int a)
    {
        int r = 0;
#pragma unroll
        for (int k = 1; k < D; ++k) r += a >= rstart(k) ? 1 : 0;
        return r * S + q0(r) + (a - rstart(r));
    }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = from_canon(c1); p2 = from_canon(c2); }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = to_canon(p1); c2 = to_canon(p2); }
    __device__ void prepare() {}

    __device__ M placements(int) const { return and_mask<Valid, NBITS, NWI>(~(p1 | p2)); }

    template <int K>
    __device__ static M runs3(const M &x) { return x & shr<K>(x) & shr<2 * K>(x); }
    template <int K>
    __device__ static M runs4(const M &x) { const M a = x & shr<K>(x); return a & shr<2 * K>(a); }

    __device__ int place(int b, int me, int &extra)
    {
        M own = pick(me == 1, p1, p2) | onehot<NWI>(b);
        p1 = pick(me == 1, own, p1);
        p2 = pick(me == 1, p2, own);
        if (any(runs4<1>(own) | runs4<S>(own) | runs4<D>(own))) return me;
        if (any(runs3<1>(own) | runs3<S>(own) | runs3<D>(own))) return 3 - me;
        if (popcount(p1 | p2) == CELLS) return 0;
        return -1;
    }
    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }
    __device__ int pass(int &) { return -1; }
};

// ---------------------------------------------------------------------------
// Pente (App. C) on N x N, N odd: while the board is empty the only legal
// placement is the centre; a placement that brackets exactly two opponent
// stones between itself and one of the mover's stones on a straight line
// removes them (any of the 8 directions, several at once); five or more in
// a row, or 5 captured pairs (10 stones), wins; a full board draws.  The
// state's per-game byte holds the captured pairs (player 1 in the low four
// bits, player 2 in the high four bits).  Layout as Gomoku (row stride
// N + 1): walking from the new stone, the zero guard column ends every
// horizontal or diagonal chain before it can wrap to the next row, so the
// bracket test needs no bounds test.
// ---------------------------------------------------------------------------
template <int N>
struct Pente {
    static_assert(N % 2 == 1, "odd side: the centre is a cell");
    static constexpr int KIND = 7, H = N, W = N, CELLS = N * N, A = N * N;
    static constexpr int S = N + 1, NBITS = N * S;
    static constexpr int NWC = (CELLS + 31) / 32, NWI = (NBITS + 31) / 32;
    static constexpr int CENTRE = (N / 2) * S + N / 2;
    static constexpr bool HAS_PASS = false;
    using M = BB<NWI>;
    M p1, p2;

    struct Valid {
        constexpr bool operator()(int b) const { return (b % S) < N; }
    };

    __device__ static M from_canon(const BB<NWC> &c) { return restride<N, N, N, S, NWC, NWI>(c); }
    __device__ static BB<NWC> to_canon(const M &m) { return restride<N, N, S, N, NWI, NWC>(m); }
    __device__ static int action_of(int b) { return (b / S) * N + (b % S); }
    __device__ static int bit_of(int a) { return (a / N) * S + (a % N); }

    __device__ void load(const BB<NWC> &c1, const BB<NWC> &c2) { p1 = from_canon(c1); p2 = from_canon(c2); }
    __device__ void store(BB<NWC> &c1, BB<NWC> &c2) const { c1 = to_canon(p1); c2 = to_canon(p2); }
    __device__ void prepare() {}

    __device__ M placements(int) const
    {
        const M occ = p1 | p2;
        return pick(any(occ), and_mask<Valid, NBITS, NWI>(~occ), onehot<NWI>(CENTRE));
    }

    // the new stone at b brackets two opponent stones along step D: read
    // from the views of the mover's and the opponent's stones around b; a
    // capture marks the two cells in the view of captured stones
    template <int D>
    __device__ __forceinline__ static uint32_t brackets(const uint32_t (&vo)[4], const uint32_t (&vp)[4],
                                                        uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3)
    {
        const uint32_t hit = view_bit<D>(vp) & view_bit<2 * D>(vp) & view_bit<3 * D>(vo);
        constexpr int p1 = 64 + D, p2 = 64 + 2 * D;
        static_assert(p1 >= 0 && p2 >= 0 && p1 < 128 && p2 < 128, "inside the view");
        const uint32_t m1 = hit << (p1 & 31), m2 = hit << (p2 & 31);
        // the capture view's words as separate scalars (no indexed array)
        if constexpr ((p1 >> 5) == 0) c0 |= m1; else if constexpr ((p1 >> 5) == 1) c1 |= m1;
        else if constexpr ((p1 >> 5) == 2) c2 |= m1; else c3 |= m1;
        if constexpr ((p2 >> 5) == 0) c0 |= m2; else if constexpr ((p2 >> 5) == 1) c1 |= m2;
        else if constexpr ((p2 >> 5) == 2) c2 |= m2; else c3 |= m2;
        return hit;
    }
    // starts of runs of five or more along step K
    template <int K>
    __device__ static M runs5(const M &x)
    {
        const M a = x & shr<K>(x);    // i, i+K
        const M b = a & shr<2 * K>(a); // i .. i+3K
        return b & shr<4 * K>(x);      // i .. i+4K
    }

    __device__ int place(int b, int me, int &extra)
    {
        const M s = onehot<NWI>(b);
        const M own = pick(me == 1, p1, p2) | s;
        M opp = pick(me == 1, p2, p1);
        // the captures: the cells within three steps of b in the eight
        // directions, read from 128-bit views of both players' stones
        // around b (three steps span at most 3 (S + 1) <= 63 bits)
        static_assert(3 * (S + 1) < 64, "captures inside the view");
        uint32_t vo[4], vp[4];
        view128(own, b, vo);
        view128(opp, b, vp);
        uint32_t c0 = 0u, c1 = 0u, c2 = 0u, c3 = 0u;
        int pairs = 0;
        pairs += brackets<1>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<-1>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<S>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<-S>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<S + 1>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<-(S + 1)>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<S - 1>(vo, vp, c0, c1, c2, c3);
        pairs += brackets<-(S - 1)>(vo, vp, c0, c1, c2, c3);
        if (__any(pairs != 0)) {
            const uint32_t cv[4] = {c0, c1, c2, c3};
            opp = andnot(opp, unview128<NWI>(cv, b));
        }
        p1 = pick(me == 1, own, opp);
        p2 = pick(me == 1, opp, own);
        int lo = extra & 15, hi = (extra >> 4) & 15;
        lo += me == 1 ? pairs : 0;
        hi += me == 1 ? 0 : pairs;
        extra = lo | (hi << 4);
        const int mine = me == 1 ? lo : hi;
        if (any(runs5<1>(own) | runs5<S>(own) | runs5<S - 1>(own) | runs5<S + 1>(own)) || mine >= 5) return me;
        if (popcount(p1 | p2) == CELLS) return 0;
        return -1;
    }
    __device__ int place_step(int b, int me, int &extra) { return place(b, me, extra); }
    __device__ int pass(int &) { return -1; }
};

} // namespace lx
