// hexaux.hpp -- Hex's connected components kept from ply to ply in the
// state's aux bytes (Sec. 4, "Dynamic State Attributes": the `connected`
// end rule of Hex is served by a component structure that each move updates
// locally instead of a recomputation from scratch).
//
// The per-ply step without aux reads the whole int8 board, packs it into
// bitboards and floods the mover's group from the new stone.  With aux it
// reads the two players' bitboards (8 * NWC bytes) instead of the board
// (N * N bytes) and joins the new stone to the components of its at most
// six neighbours of the same colour with a union-find, so the end test is a
// few parent reads instead of a flood.
//
// Per environment, BYTES bytes (a multiple of 128, rows 128-byte aligned,
// so that the part every ply reads is one 128-byte cache line):
//   [0, 4)              tag: the (ply, last_action) the cache belongs to
//   [16, 16 + 4 NWC)    player 1's stones, bit c = cell c
//   [.., 16 + 8 NWC)    player 2's stones (16 + 8 NWC <= 128 up to 19x19)
//   [128, 128 + 2 N^2)  uint16 parent[c] for every occupied cell c: a root
//                       holds ROOT | side flags of its component (bit 0: it
//                       touches its owner's first side, bit 1: the far
//                       side), any other cell the index of its parent.
//                       Entries of empty cells are unused.
// A step whose tag does not match the env's (ply, last_action) -- the state
// was changed by a call without this aux, or by a playout -- rebuilds the
// cache from the board first.
#pragma once

#include "games.hpp"

namespace lx {

template <int N>
struct HexAux {
    static constexpr int CELLS = N * N, NWC = (CELLS + 31) / 32;
    static constexpr int STONES = 16, PARENT = 128;
    static constexpr int BYTES = PARENT + (2 * CELLS + 127) / 128 * 128;
    static_assert(STONES + 8 * NWC <= PARENT, "tag and stones share one cache line");
    static constexpr uint16_t ROOT = 0x8000u;
};

__device__ __forceinline__ uint32_t aux_tag(int ply, int last)
{
    return ((uint32_t)(uint16_t)ply | ((uint32_t)(uint16_t)last << 16)) ^ 0xA5C3A5C3u;
}

// side flags of cell b for player p (bit 0: p's first side, bit 1: p's far
// side); a corner belongs to both sides that meet there
template <int N>
__device__ __forceinline__ uint16_t hex_sides(int b, int p)
{
    const int r = b / N, c = b - (b / N) * N;
    const int k = p == 1 ? r : c;
    return (uint16_t)((k == 0 ? 1u : 0u) | (k == N - 1 ? 2u : 0u));
}

// Place player me's stone on cell b, whose stones before the move are
// `own`: join b to the components of its same-coloured neighbours and
// return whether the joined component touches both of me's sides.  The
// neighbours' roots are found together: their parent entries are loaded at
// once, then each chain climbs one level per round (independent loads in
// flight together instead of one find after another).  The other roots
// are linked under the first neighbour's root r0, and every neighbour and
// b itself point straight at r0 (their entries share b's cache lines), so
// chains stay short.
template <int N>
__device__ __forceinline__ bool uf_place(uint16_t *par, const BB<HexAux<N>::NWC> &own, int b, int me)
{
    constexpr uint16_t ROOT = HexAux<N>::ROOT;
    const int r = b / N, c = b - (b / N) * N;
    // the six neighbours (r-1,c), (r-1,c+1), (r,c-1), (r,c+1), (r+1,c-1), (r+1,c)
    const int nb[6] = {b - N, b - N + 1, b - 1, b + 1, b + N - 1, b + N};
    const bool ok[6] = {r > 0, r > 0 && c < N - 1, c > 0, c < N - 1, r < N - 1 && c > 0, r < N - 1};
    bool in[6];
    int x[6];
    uint16_t e[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        in[k] = ok[k] && test_bit(own, nb[k]);
        x[k] = nb[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = in[k] ? par[x[k]] : ROOT;
    for (;;) {
        bool more = false;
#pragma unroll
        for (int k = 0; k < 6; ++k) more |= !(e[k] & ROOT);
        if (!more) break;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (!(e[k] & ROOT)) {
                x[k] = e[k];
                e[k] = par[x[k]];
            }
    }
    uint16_t flags = hex_sides<N>(b, me), f0 = 0;
    int r0 = -1;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (in[k]) {
            flags |= e[k] & 3u;
            if (r0 < 0) {
                r0 = x[k];
                f0 = e[k] & 3u;
            }
        }
    if (r0 < 0) {
        par[b] = (uint16_t)(ROOT | flags);
        return flags == 3u;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (in[k] && x[k] != r0) par[x[k]] = (uint16_t)r0;   // another component's root
        if (in[k] && nb[k] != r0) par[nb[k]] = (uint16_t)r0; // the neighbour itself
    }
    par[b] = (uint16_t)r0;
    if (flags != f0) par[r0] = (uint16_t)(ROOT | flags);
    return flags == 3u;
}

// Label every component of player p's stones `own` from scratch: the
// lowest cell of a component is its root.
template <int N>
__device__ __forceinline__ void uf_build(uint16_t *par, BB<HexAux<N>::NWC> own, int p)
{
    using G = Hex<N>;
    constexpr uint16_t ROOT = HexAux<N>::ROOT;
    constexpr int NW = HexAux<N>::NWC;
    while (any(own)) {
        int s = 0;
#pragma unroll
        for (int i = NW - 1; i >= 0; --i)
            if (own.w[i]) s = 32 * i + __builtin_ctz(own.w[i]);
        const BB<NW> g = G::flood(onehot<NW>(s), own);
        const uint16_t flags = (uint16_t)((any(G::first_side(g, p)) ? 1u : 0u) | (G::meets_far_side(g, p) ? 2u : 0u));
        own = andnot(own, g);
        static_for<NW>([&](auto I) {
            constexpr int i = I;
            uint32_t w = g.w[i];
            while (w) {
                const int cell = 32 * i + __builtin_ctz(w);
                w &= w - 1u;
                par[cell] = cell == s ? (uint16_t)(ROOT | flags) : (uint16_t)s;
            }
        });
    }
}

} // namespace lx
