// bitboard.hpp -- device primitives for env-per-lane board games on gfx950.
//
// A board of up to 19x19 cells is a multiword bitboard of 32-bit words held
// in VGPRs (one environment per lane).  Shifts by compile-time amounts become
// v_alignbit_b32 funnel shifts; masks are compile-time immediates expanded
// word by word with static_for, so no table is read from memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace lx {

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Word `word` of the mask whose bit b (0 <= b < nbits) is set iff pred(b).
template <class P>
constexpr uint32_t mask_word(P pred, int nbits, int word)
{
    uint32_t m = 0;
    for (int j = 0; j < 32; ++j) {
        const int b = 32 * word + j;
        if (b < nbits && pred(b)) m |= 1u << j;
    }
    return m;
}

template <int NW>
struct BB {
    uint32_t w[NW];
};

template <int NW>
__device__ __forceinline__ BB<NW> bb_zero()
{
    BB<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = 0u;
    return r;
}

template <int NW>
__device__ __forceinline__ BB<NW> operator|(const BB<NW> &a, const BB<NW> &b)
{
    BB<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = a.w[i] | b.w[i];
    return r;
}

template <int NW>
__device__ __forceinline__ BB<NW> operator&(const BB<NW> &a, const BB<NW> &b)
{
    BB<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = a.w[i] & b.w[i];
    return r;
}

template <int NW>
__device__ __forceinline__ BB<NW> andnot(const BB<NW> &a, const BB<NW> &b) // a & ~b
{
    BB<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = a.w[i] & ~b.w[i];
    return r;
}

template <int NW>
__device__ __forceinline__ BB<NW> operator~(const BB<NW> &a)
{
    BB<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = ~a.w[i];
    return r;
}

// c ? a : b, word by word (a whole-struct select would go through memory;
// so would a select between the addresses of two boards, which is what
// reference arguments invite: the boards are taken by value)
template <int NW>
__device__ __forceinline__ BB<NW> pick(bool c, BB<NW> a, BB<NW> b)
{
    BB<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = c ? a.w[i] : b.w[i];
    return r;
}

template <int NW>
__device__ __forceinline__ bool any(const BB<NW> &a)
{
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) o |= a.w[i];
    return o != 0u;
}

template <int NW>
__device__ __forceinline__ bool same(const BB<NW> &a, const BB<NW> &b)
{
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) o |= a.w[i] ^ b.w[i];
    return o == 0u;
}

template <int NW>
__device__ __forceinline__ int popcount(const BB<NW> &a)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) c += __popc(a.w[i]);
    return c;
}

// a & M, a & ~M and M itself, where M = {b < NBITS : P{}(b)} for a
// default-constructible constexpr predicate type P.
template <class P, int NBITS, int NW>
__device__ __forceinline__ BB<NW> and_mask(const BB<NW> &a)
{
    BB<NW> r;
    static_for<NW>([&](auto I) {
        constexpr int i = I;
        constexpr uint32_t m = mask_word(P{}, NBITS, i);
        r.w[i] = a.w[i] & m;
    });
    return r;
}

template <class P, int NBITS, int NW>
__device__ __forceinline__ BB<NW> andnot_mask(const BB<NW> &a)
{
    BB<NW> r;
    static_for<NW>([&](auto I) {
        constexpr int i = I;
        constexpr uint32_t m = mask_word(P{}, NBITS, i);
        r.w[i] = a.w[i] & ~m;
    });
    return r;
}

template <class P, int NBITS, int NW>
__device__ __forceinline__ BB<NW> const_mask()
{
    BB<NW> r;
    static_for<NW>([&](auto I) {
        constexpr int i = I;
        r.w[i] = mask_word(P{}, NBITS, i);
    });
    return r;
}

struct AllBits {
    constexpr bool operator()(int) const { return true; }
};

// Logical shift towards higher bit indices by a compile-time amount.
template <int S, int NW>
__device__ __forceinline__ BB<NW> shl(const BB<NW> &x)
{
    static_assert(S > 0, "shift amount");
    constexpr int q = S / 32, s = S % 32;
    BB<NW> r;
    static_for<NW>([&](auto I) {
        constexpr int i = I;
        constexpr int j = i - q;
        uint32_t hi = 0u, lo = 0u;
        if constexpr (j >= 0) hi = x.w[j >= 0 ? j : 0];
        if constexpr (j - 1 >= 0) lo = x.w[j - 1 >= 0 ? j - 1 : 0];
        if constexpr (s == 0) r.w[i] = hi;
        else r.w[i] = __builtin_amdgcn_alignbit(hi, lo, 32 - s);
    });
    return r;
}

// Logical shift towards lower bit indices by a compile-time amount.
template <int S, int NW>
__device__ __forceinline__ BB<NW> shr(const BB<NW> &x)
{
    static_assert(S > 0, "shift amount");
    constexpr int q = S / 32, s = S % 32;
    BB<NW> r;
    static_for<NW>([&](auto I) {
        constexpr int i = I;
        constexpr int j = i + q;
        uint32_t hi = 0u, lo = 0u;
        if constexpr (j < NW) lo = x.w[j < NW ? j : 0];
        if constexpr (j + 1 < NW) hi = x.w[j + 1 < NW ? j + 1 : 0];
        if constexpr (s == 0) r.w[i] = lo;
        else r.w[i] = __builtin_amdgcn_alignbit(hi, lo, s);
    });
    return r;
}

// Shift by a signed compile-time amount (positive = towards higher bits).
template <int S, int NW>
__device__ __forceinline__ BB<NW> shift(const BB<NW> &x)
{
    if constexpr (S > 0) return shl<S>(x);
    else return shr<-S>(x);
}

// All ones when x < 0, else zero, as a byte permute in which every byte
// takes the sign of x's top byte: a select on it is a bit-field insert,
// where a compare would write a scalar lane mask that the select reading it
// waits a few cycles for.
__device__ __forceinline__ int sign_mask(int x)
{
    return (int)__builtin_amdgcn_perm(0u, (uint32_t)x, 0x09090909u);
}

// A 128-bit view of a bitboard around a per-lane cell b: v bit (64 + o) is
// x bit (b + o) for every offset o in [-64, 64), zero off the board.  The
// five words q - 2 .. q + 2 (q = b / 32) are picked by a barrel shift over
// q's bits (a few selects per stage instead of a select chain per word),
// then funnel-shifted by b mod 32.  Tests at constant offsets from b then
// read constant bit positions of the view.
template <int NW>
__device__ __forceinline__ void view128(const BB<NW> &x, int b, uint32_t (&v)[4])
{
    static_assert(NW <= 16, "q fits four selector bits");
    const int q = b >> 5, off = b & 31;
    // y[i] = x word i - 2, zero outside the board
    uint32_t y[20];
    static_for<20>([&](auto I) {
        constexpr int i = I;
        y[i] = (i >= 2 && i - 2 < NW) ? x.w[(i >= 2 && i - 2 < NW) ? i - 2 : 0] : 0u;
    });
    // y[j] <- y[j + step] where q has the step's bit, for the entries the
    // later stages read.  The choice is a bit-field insert under an opaque
    // all-ones mask: as selects on q the stages are recognised as an
    // indexed read and the words go to private memory.
    auto stage = [&](auto STEP, auto KEEP) {
        constexpr int step = STEP, keep = KEEP;
        const uint32_t on = (uint32_t)sign_mask(q << (31 - __builtin_ctz(step)));
        static_for<keep>([&](auto J) {
            constexpr int j = J;
            y[j] = (on & y[j + step]) | (~on & y[j]);
        });
    };
    if constexpr (NW > 8) stage(std::integral_constant<int, 8>{}, std::integral_constant<int, 12>{});
    if constexpr (NW > 4) stage(std::integral_constant<int, 4>{}, std::integral_constant<int, 8>{});
    if constexpr (NW > 2) stage(std::integral_constant<int, 2>{}, std::integral_constant<int, 6>{});
    if constexpr (NW > 1) stage(std::integral_constant<int, 1>{}, std::integral_constant<int, 5>{});
    static_for<4>([&](auto J) {
        constexpr int j = J;
        v[j] = __builtin_amdgcn_alignbit(y[j + 1], y[j], (unsigned)off);
    });
}

// bit 64 + O of a view: x bit (b + O)
template <int O>
__device__ __forceinline__ uint32_t view_bit(const uint32_t (&v)[4])
{
    static_assert(O >= -64 && O < 64, "offset inside the view");
    constexpr int p = 64 + O;
    return (v[p >> 5] >> (p & 31)) & 1u;
}

// The inverse of view128: the board whose bit b + o is view bit 64 + o
// (offsets that fall off the board are dropped).
template <int NW>
__device__ __forceinline__ BB<NW> unview128(const uint32_t (&c)[4], int b)
{
    const int q = b >> 5, off = b & 31;
    // the view shifted up by b mod 32: window words 0..4 (window word j is
    // board word q - 2 + j); funnel shifts, b mod 32 = 0 taking the words
    // as they are
    uint32_t t[20];
    static_for<20>([&](auto I) { t[(int)I] = 0u; });
    const unsigned back = (unsigned)(32 - off) & 31u;
    t[0] = c[0] << off;
    static_for<3>([&](auto J) {
        constexpr int j = J + 1;
        t[j] = off == 0 ? c[j] : __builtin_amdgcn_alignbit(c[j], c[j - 1], back);
    });
    t[4] = off == 0 ? 0u : __builtin_amdgcn_alignbit(0u, c[3], back);
    // window word j to board word q - 2 + j: t[k] <- t[k - step] where q has
    // the step's bit (t index k is board word k - 2)
    auto stage = [&](auto STEP, auto TOP) {
        constexpr int step = STEP, top = TOP;
        const uint32_t on = (uint32_t)sign_mask(q << (31 - __builtin_ctz(step)));
        static_for<top>([&](auto K) {
            constexpr int k = top - 1 - K; // from the top down: reads the unshifted entries
            const uint32_t below = k >= step ? t[k >= step ? k - step : 0] : 0u;
            t[k] = (on & below) | (~on & t[k]);
        });
    };
    constexpr int TOPN = NW + 2 < 20 ? NW + 2 : 20;
    if constexpr (NW > 1) stage(std::integral_constant<int, 1>{}, std::integral_constant<int, (6 < TOPN ? 6 : TOPN)>{});
    if constexpr (NW > 2) stage(std::integral_constant<int, 2>{}, std::integral_constant<int, (8 < TOPN ? 8 : TOPN)>{});
    if constexpr (NW > 4) stage(std::integral_constant<int, 4>{}, std::integral_constant<int, (12 < TOPN ? 12 : TOPN)>{});
    if constexpr (NW > 8) stage(std::integral_constant<int, 8>{}, std::integral_constant<int, TOPN>{});
    BB<NW> r;
    static_for<NW>([&](auto I) { r.w[(int)I] = t[(int)I + 2]; });
    return r;
}

// Word i of a bitboard picked by a per-lane word index q without a compare
// (whose lane mask in a scalar register costs wait states before the
// select that reads it): sel = word_sel(q) has bit q set, and
// word_mask(sel, i) sign-extends bit i of it, all ones in word q and zero
// elsewhere.  A q outside [0, 31) selects no word of a board of fewer
// than 31 words.
__device__ __forceinline__ int word_sel(int q) { return (int)(1u << (q & 31)); }
__device__ __forceinline__ uint32_t word_mask(int sel, int i)
{
    return (uint32_t)__builtin_amdgcn_sbfe(sel, (unsigned)i, 1u);
}

// Bitboard with only bit b set (b in range).
template <int NW>
__device__ __forceinline__ BB<NW> onehot(int b)
{
    static_assert(NW < 32, "the word selector is a 32-bit mask");
    BB<NW> r;
    const uint32_t bit = 1u << (b & 31);
    const int sel = word_sel(b >> 5);
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = bit & word_mask(sel, i);
    return r;
}

template <int NW>
__device__ __forceinline__ uint32_t test_bit(const BB<NW> &x, int b)
{
    // OR of masked words: a select chain here is turned into a private-memory
    // table lookup by the compiler
    const int q = b >> 5;
    uint32_t w = 0u;
#pragma unroll
    for (int i = 0; i < NW; ++i) w |= x.w[i] & (0u - (uint32_t)(q == i));
    return (w >> (b & 31)) & 1u;
}

// Position of the k-th (from 0) set bit of a 32-bit word; k < popcount(w).
// Binary search over halves with the position as a bit offset into the
// unshifted word: the lower half of the current window [off, off + 2s)
// holds c set bits; when k >= c the bit is in the upper half.  The
// "k >= c" choice is taken from the sign of k - c (sign_mask).
__device__ __forceinline__ int select_in_word(uint32_t w, int k)
{
    int off = 0;
#pragma unroll
    for (int s = 16; s >= 1; s >>= 1) {
        const int c = __popc(__builtin_amdgcn_ubfe(w, (unsigned)off, (unsigned)s));
        const int d = k - c;
        const int lower = sign_mask(d);
        k = (lower & k) | (~lower & d);
        off |= ~lower & s;
    }
    return off;
}

// The word holding the k-th (from 0) set bit: its value, index and the
// count of set bits in the words before it; k < popcount(m).  Up to four
// words, the last word whose prefix count is <= k, by a chain of selects.
// Longer boards first pick a group of four words the same way, then the
// word within the group: about half the selects of one chain over all
// the words.
template <int NW>
__device__ __forceinline__ void select_word(const BB<NW> &m, int k, uint32_t &wsel, int &wi, int &off)
{
    if constexpr (NW <= 4) {
        wsel = m.w[0];
        wi = 0;
        off = 0;
        int pre = __popc(m.w[0]);
#pragma unroll
        for (int i = 1; i < NW; ++i) {
            const bool ge = k >= pre;
            wsel = ge ? m.w[i] : wsel;
            wi = ge ? i : wi;
            off = ge ? pre : off;
            pre += __popc(m.w[i]);
        }
    } else {
        constexpr int NG = (NW + 3) / 4;
        BB<4> q;
        q.w[0] = m.w[0], q.w[1] = m.w[1], q.w[2] = m.w[2], q.w[3] = m.w[3];
        int g = 0, goff = 0;
        int gpre = __popc(m.w[0]) + __popc(m.w[1]) + __popc(m.w[2]) + __popc(m.w[3]);
        static_for<NG - 1>([&](auto I) {
            constexpr int G = I + 1;
            const int start = gpre; // set bits before group G
            const bool ge = k >= start;
            static_for<4>([&](auto J) {
                constexpr int j = J;
                constexpr int i = 4 * G + j;
                const uint32_t x = i < NW ? m.w[i < NW ? i : 0] : 0u;
                q.w[j] = ge ? x : q.w[j];
                if constexpr (G + 1 < NG) gpre += __popc(x);
            });
            g = ge ? G : g;
            goff = ge ? start : goff;
        });
        int j;
        select_word<4>(q, k - goff, wsel, j, off);
        wi = 4 * g + j;
        off += goff;
    }
}

// Index of the k-th (from 0) set bit in increasing bit order; k < popcount(m).
template <int NW>
__device__ __forceinline__ int select_bit(const BB<NW> &m, int k)
{
    uint32_t wsel;
    int wi, off;
    select_word(m, k, wsel, wi, off);
    return 32 * wi + select_in_word(wsel, k - off);
}

// The same search returning the word index of the k-th set bit and that bit
// within its word.
template <int NW>
__device__ __forceinline__ void select_bit_split(const BB<NW> &m, int k, int &word, uint32_t &bit)
{
    uint32_t wsel;
    int off;
    select_word(m, k, wsel, word, off);
    bit = 1u << select_in_word(wsel, k - off);
}

// The legal action of a uniform draw: with n = popcount(m) set bits and a
// 32-bit random word w, the k-th set bit for k = (w * n) >> 32.
template <int NW>
__device__ __forceinline__ int select_uniform(const BB<NW> &m, uint32_t w)
{
    return select_bit(m, (int)__umulhi(w, (uint32_t)popcount(m)));
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4x32 Philox S-box.  Each round multiplies counter words 0 and 2 by the two
// Philox multipliers; the high halves are xored with the other two words and
// the round key, the low halves move into place; the key advances by the two
// Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-way xors, one bitwise-ternary instruction each (0x96: odd
        // parity of the three inputs)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96u);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96u);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

// Pack four 0/1/2 cell bytes (one dword, little endian) into 4-bit fields:
// player-1 flags and player-2 flags, cell j at bit j.
__device__ __forceinline__ uint32_t pack4_p1(uint32_t v) { return ((v & 0x01010101u) * 0x00204081u) >> 21 & 0xFu; }
__device__ __forceinline__ uint32_t pack4_p2(uint32_t v) { return (((v >> 1) & 0x01010101u) * 0x00204081u) >> 21 & 0xFu; }
// Inverse: 4-bit fields of both players -> four cell bytes.
__device__ __forceinline__ uint32_t unpack4(uint32_t b1, uint32_t b2)
{
    return ((b1 * 0x00204081u) & 0x01010101u) | (((b2 * 0x00204081u) & 0x01010101u) << 1);
}

} // namespace lx
