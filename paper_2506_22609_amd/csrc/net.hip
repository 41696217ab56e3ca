// net.hip -- the small convolutional policy/value network on bf16 MFMA.
//
// Network (the model of the paper's "Trained Agents" section made small):
// 3 mover-frame planes -> 4 x (conv3x3, 64 channels, ReLU) -> a policy head
// (a 1x1 convolution to one logit per cell) and a value head (tanh of a
// linear map of the channel means).  Conv weights and activations are
// bfloat16, every sum is float32; the heads are float32.
//
// Activation layout: NHWC with a zero ring, [n][N+2][N+2][C] bf16, so a 3x3
// tap is a plain pointer offset and needs no bounds test.  The first layer's
// input has C = 4 (mover, opponent, empty, zero).
//
// Convolution = implicit GEMM on v_mfma_f32_16x16x32_bf16: M = 64 output
// channels (4 tiles), N = the cells of one board (16-cell tiles, up to 8
// tiles per wave), K = 9 taps x C input channels; with the channels as M a
// lane's results are consecutive channels of one cell, written 16 bytes at a
// time.  A wave owns one (board, group of
// 8 cell tiles) and keeps 8 x 4 accumulator tiles in registers; the block's
// weights ([64][K] bf16, rows padded by 8 elements) sit in LDS and are
// shared by the block's four waves.  The same kernel computes the gradient
// with respect to the input (the transposed convolution is a convolution of
// dZ with the weights flipped in space and with input and output channels
// exchanged), masked by the ReLU of the layer below.
//
// Weight gradients: dW[o][i][t] = sum over boards and cells of dZ[p][o] x
// X[p + tap t][i]: M = 64 output channels, N = (tap, input channel), K =
// cells, on the same MFMA; each block stages one board at a time in LDS
// (dZ transposed so a fragment is one 16-byte read) and accumulates over its
// share of the batch; per-block partial sums are added by a second kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "kernels.hpp"
#include "ludax_internal.hpp"

namespace lx {
namespace net {

constexpr int C = 64;
constexpr int WAVE = 64;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest, ties to even (finite values)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Two floats to bf16 by the hardware conversion (v_cvt_pk_bf16_f32: round
// to nearest, ties to even, as f2bf; one instruction for the pair where
// f2bf takes four per value), lo in the low half.
typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));
typedef float f32x2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_v){lo, hi}, bf16x2_v));
}
// y = bf16(relu(a)), bf16(relu(b)) as floats: a layer's output as the next
// layer reads it
__device__ __forceinline__ void relu_bf16_pair(float a, float b, float &ya, float &yb)
{
    const uint32_t p = pack_bf16(fmaxf(a, 0.f), fmaxf(b, 0.f));
    ya = __uint_as_float(p << 16);
    yb = __uint_as_float(p & 0xFFFF0000u);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// pointers of the memory-to-LDS load builtin
typedef __attribute__((address_space(1))) void glb_void;
typedef __attribute__((address_space(3))) void lds_void;

// ---------------------------------------------------------------------------
// parameter offsets in the flat float32 vector
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int64_t w_off(int l) // l = 1..4
{
    return l == 1 ? 0 : (int64_t)(C * 27 + C) + (int64_t)(l - 2) * (C * C * 9 + C);
}
__host__ __device__ constexpr int64_t b_off(int l) { return w_off(l) + (l == 1 ? C * 27 : C * C * 9); }
constexpr int64_t WP_OFF = (int64_t)(C * 27 + C) + 3 * (int64_t)(C * C * 9 + C);
constexpr int64_t BP_OFF = WP_OFF + C;
constexpr int64_t WV_OFF = BP_OFF + 1;
constexpr int64_t BV_OFF = WV_OFF + C;
constexpr int64_t N_PARAMS = BV_OFF + 1;
static_assert(N_PARAMS == 112706, "parameter count");

// Packed bf16 weights: forward [64 out][K] with k = tap * C_in + in (layer 1:
// C_in = 4, the fourth channel zero, K padded to 64), then for layers 2..4
// the data-gradient weights [64 in][576] with k = tap' * 64 + out and
// tap' = 8 - tap.
constexpr int K1 = 64, K2 = 576;
__host__ __device__ constexpr int64_t pf_off(int l) { return l == 1 ? 0 : (int64_t)C * K1 + (int64_t)(l - 2) * C * K2; }
__host__ __device__ constexpr int64_t pb_off(int l) { return (int64_t)C * K1 + 3 * (int64_t)C * K2 + (int64_t)(l - 2) * C * K2; }
constexpr int64_t PACKED_ELEMS = (int64_t)C * K1 + 6 * (int64_t)C * K2;
// 16 zero bytes inside the packed weights: layer 1's row 0 at k = 40 .. 47
// (taps 10 and 11, past the 9 taps, are packed as zeros)
__host__ __device__ inline const uint16_t *zero16(const uint16_t *packed) { return packed + pf_off(1) + 40; }

__global__ void k_pack(const float *__restrict__ p, uint16_t *__restrict__ out)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < PACKED_ELEMS;
         j += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        if (j < C * K1) {
            const int o = (int)(j / K1), k = (int)(j % K1), t = k >> 2, i = k & 3;
            if (t < 9 && i < 3) v = p[w_off(1) + (o * 3 + i) * 9 + t];
        } else if (j < pb_off(2)) {
            const int64_t r = j - C * K1;
            const int l = 2 + (int)(r / (C * K2));
            const int q = (int)(r % (C * K2)), o = q / K2, k = q % K2, t = k >> 6, i = k & 63;
            v = p[w_off(l) + (o * C + i) * 9 + t];
        } else {
            const int64_t r = j - pb_off(2);
            const int l = 2 + (int)(r / (C * K2));
            const int q = (int)(r % (C * K2)), i = q / K2, k = q % K2, tp = k >> 6, o = k & 63;
            v = p[w_off(l) + (o * C + i) * 9 + (8 - tp)];
        }
        out[j] = f2bf(v);
    }
}

// ---------------------------------------------------------------------------
// encode: boards -> layer-1 input planes [n][NP][NP][4] (ring zero)
// ---------------------------------------------------------------------------
template <int N>
__global__ void k_encode(const int8_t *__restrict__ board, const int8_t *__restrict__ to_move, int64_t n,
                         uint2 *__restrict__ a0)
{
    constexpr int NP = N + 2, PP = NP * NP;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n * PP) return;
    const int64_t b = j / PP;
    const int q = (int)(j % PP), R = q / NP, Q = q % NP;
    uint2 v = {0u, 0u};
    if (R >= 1 && R <= N && Q >= 1 && Q <= N) {
        const int r = R - 1, c = Q - 1, me = to_move[b];
        const int cell = me == 2 ? c * N + r : r * N + c; // player 2 sees the transpose
        const int x = board[b * (N * N) + cell];
        const uint32_t one = 0x3F80u; // bf16 1.0
        const uint32_t c0 = x == me ? one : 0u, c1 = (x != 0 && x != me) ? one : 0u, c2 = x == 0 ? one : 0u;
        v.x = c0 | (c1 << 16);
        v.y = c2;
    }
    a0[j] = v;
}

// ring cell j (0 <= j < 4 * (NP - 1)) of a padded NP x NP frame
template <int NP>
__device__ __forceinline__ int ring_cell(int j)
{
    if (j < NP) return j;                               // top row
    if (j < 2 * NP) return (NP - 1) * NP + (j - NP);    // bottom row
    const int k = j - 2 * NP;                           // sides, rows 1 .. NP-2
    return (1 + (k >> 1)) * NP + ((k & 1) ? NP - 1 : 0);
}

// zero the ring of one board's [NP][NP][64] bf16 activation (one wave)
template <int N>
__device__ __forceinline__ void zero_ring(uint16_t *act_b, int lane)
{
    constexpr int NP = N + 2, RING = 4 * (NP - 1);
    for (int j = lane; j < RING * 8; j += WAVE) {
        const int cell = ring_cell<NP>(j >> 3);
        reinterpret_cast<uint4 *>(act_b + (int64_t)cell * C)[j & 7] = uint4{0u, 0u, 0u, 0u};
    }
}

// ---------------------------------------------------------------------------
// Output-channel placement.  The convolutions multiply the weights (M = the
// output channels) by the activations (N = the cells of a tile), so a lane
// of a 16 x 16 product holds four M rows of one cell.  A row m of the wave's
// channel tile nt is given the weight row of channel
//   half * 16 NTW + 4 NTW (m / 4) + 4 nt + m % 4,
// which makes a lane's rows over all its NTW tiles 4 NTW consecutive
// channels of its cell, stored with 16-byte writes.  w_slot is the inverse:
// the LDS row that holds output channel o.
// ---------------------------------------------------------------------------
// the output channel whose weights sit in LDS row s (inverse of w_slot)
template <int NTW>
__device__ __forceinline__ int w_channel(int s)
{
    const int half = s / (16 * NTW), nt = (s / 16) % NTW, m = s % 16;
    return half * 16 * NTW + 4 * NTW * (m >> 2) + 4 * nt + (m & 3);
}

template <int NTW>
__device__ __forceinline__ int w_slot(int o)
{
    constexpr int SPAN = 16 * NTW; // output channels of one wave
    const int half = o / SPAN, r = o % SPAN;
    const int m = 4 * (r / (4 * NTW)) + (r & 3), nt = (r >> 2) % NTW;
    return (half * NTW + nt) * 16 + m;
}

// Epilogue of one cell: acc[nt][k] is channel c0 + 4 nt + k of the cell
// whose output row starts at orow (mrow: the same row of the mask).
//   MODE 0: bf16(relu(acc)); the accumulators started at the bias
//   MODE 1: bf16(acc) where the mask is positive, else 0
template <int NTW, int MODE>
__device__ __forceinline__ void store_cell(const f32x4 (&acc)[NTW], const uint16_t *mrow, uint16_t *orow)
{
    float v[4 * NTW];
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[4 * nt + k] = acc[nt][k];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int j = 0; j < 4 * NTW; ++j) v[j] = fmaxf(v[j], 0.f);
    } else {
#pragma unroll
        for (int q = 0; q < NTW / 2; ++q) {
            const uint4 mv = reinterpret_cast<const uint4 *>(mrow)[q];
            const uint32_t mw[4] = {mv.x, mv.y, mv.z, mv.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t m = (mw[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                v[8 * q + j] = (m != 0 && (m & 0x8000u) == 0) ? v[8 * q + j] : 0.f;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NTW / 2; ++q) {
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            w[j] = pack_bf16(v[8 * q + 2 * j], v[8 * q + 2 * j + 1]);
        reinterpret_cast<uint4 *>(orow)[q] = uint4{w[0], w[1], w[2], w[3]};
    }
}

// ---------------------------------------------------------------------------
// 3x3 convolution, implicit GEMM on MFMA.
//   MODE 0 (forward):  out = bf16(relu(conv(X, W) + bias))
//   MODE 1 (data gradient): out = bf16(conv(X, W) * [mask > 0]), X = dZ of the
//          layer above, W = its flipped, transposed weights, mask = the
//          forward activation of the layer below.
// CIN = 4 (layer-1 planes) or 64.  Grid: 4 waves per block, one wave per
// (board, group of up to 8 cell tiles).
// ---------------------------------------------------------------------------
template <int N, int CIN, int MODE>
__global__ __launch_bounds__(256, 2) void k_conv(const uint16_t *__restrict__ x, const uint16_t *__restrict__ w,
                                              const float *__restrict__ bias,
                                              const uint16_t *__restrict__ mask, uint16_t *__restrict__ out,
                                              int64_t n)
{
    constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    constexpr int MT = (PIX + 15) / 16, NG = (MT + 7) / 8;
    constexpr int K = CIN == 4 ? K1 : K2, KS = K + 8;
    __shared__ __align__(16) uint16_t ws[C * KS];

    // stage the weights (all 256 threads), 16 bytes at a time
    for (int j = threadIdx.x; j < C * K / 8; j += 256) {
        const int o = j / (K / 8), k8 = j % (K / 8);
        reinterpret_cast<uint4 *>(ws + w_slot<4>(o) * KS)[k8] = reinterpret_cast<const uint4 *>(w + (int64_t)o * K)[k8];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= n * NG) return;
    const int64_t b = item / NG;
    const int g = (int)(item % NG);
    const uint16_t *xb = x + b * (int64_t)PP * CIN;
    uint16_t *ob = out + b * (int64_t)PP * C;
    if (g == 0) zero_ring<N>(ob, lane);

    const int row = lane & 15, quad = lane >> 4;
    // the A rows (cells) of this lane in each tile, as offsets of the
    // top-left tap in the padded frame; cells past the board read cell 0
    int cell_off[8];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        const int p = (g * 8 + mt) * 16 + row;
        const int pc = p < PIX ? p : 0;
        cell_off[mt] = ((pc / N) * NP + (pc % N)) * CIN;
    }
    // accumulators start at the bias of their channels 16 quad + 4 nt + k
    f32x4 acc[8][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 b0 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k) b0[k] = bias[16 * quad + 4 * nt + k];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt][nt] = b0;
    }

    // A fragments of K-step ks: this lane's 8 consecutive k of each tile row
    auto load_a = [&](int ks, bf16x8 (&a)[8]) {
        const int k0 = ks * 32 + quad * 8;
        int off0, off1;
        if constexpr (CIN == 4) {
            // k = tap * 4 + channel: two taps per lane; taps >= 9 read tap 0
            // (their weights are zero)
            const int t0 = k0 >> 2, t1 = t0 + 1;
            const int u0 = t0 < 9 ? t0 : 0, u1 = t1 < 9 ? t1 : 0;
            off0 = ((u0 / 3) * NP + (u0 % 3)) * CIN;
            off1 = ((u1 / 3) * NP + (u1 % 3)) * CIN;
        } else {
            const int t = k0 >> 6;
            off0 = ((t / 3) * NP + (t % 3)) * CIN + (k0 & 63);
            off1 = 0;
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            if (g * 8 + mt >= MT) break;
            if constexpr (CIN == 4) {
                const uint2 lo = *reinterpret_cast<const uint2 *>(xb + cell_off[mt] + off0);
                const uint2 hi = *reinterpret_cast<const uint2 *>(xb + cell_off[mt] + off1);
                a[mt] = as_bf16x8(uint4{lo.x, lo.y, hi.x, hi.y});
            } else {
                a[mt] = as_bf16x8(*reinterpret_cast<const uint4 *>(xb + cell_off[mt] + off0));
            }
        }
    };
    // software pipeline: the next K-step's A fragments load while this
    // step's MFMAs run
    constexpr int KSTEPS = K / 32;
    bf16x8 a_cur[8], a_nxt[8];
    load_a(0, a_cur);
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const int k0 = ks * 32 + quad * 8;
        bf16x8 bfr[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            bfr[nt] = as_bf16x8(*reinterpret_cast<const uint4 *>(ws + (nt * 16 + row) * KS + k0));
        if (ks + 1 < KSTEPS) load_a(ks + 1, a_nxt);
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            if (g * 8 + mt >= MT) break;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[nt], a_cur[mt], acc[mt][nt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) a_cur[mt] = a_nxt[mt];
    }

    // epilogue: lane holds channels 16 quad .. 16 quad + 15 of cell row of each tile
    const int c0 = 16 * quad;
    const uint16_t *mb = MODE == 1 ? mask + b * (int64_t)PP * C : nullptr;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        if (g * 8 + mt >= MT) break;
        const int p = (g * 8 + mt) * 16 + row;
        if (p >= PIX) continue;
        const int64_t o = (int64_t)(((p / N) + 1) * NP + (p % N) + 1) * C + c0;
        store_cell<4, MODE>(acc[mt], MODE == 1 ? mb + o : nullptr, ob + o);
    }
}

// ---------------------------------------------------------------------------
// Cells of the 16-lane tiles of the LDS convolutions.  An activation
// fragment read takes 16 bytes of each of the tile's 16 cells, at a 64-byte
// cell pitch with the 16-byte chunks rotated by q / 4 (q = the cell's
// top-left tap in the padded frame): conflict-free exactly when the 16 q
// cover every residue mod 16, and a tap shifts all of them by one offset.
// Runs of 16 consecutive board cells cross a row wrap of the padded frame,
// where two residues repeat (a second pass over the banks).  So lane r of
// tile t takes the t-th cell in board order with q mod 16 = r.  Entry: q of
// the lane's cell, or -1 - q0 for a lane left without one (it reads the
// first filled lane's q0: the same addresses, served by broadcast).
// ---------------------------------------------------------------------------
template <int N>
struct TileCells {
    static constexpr int NP = N + 2, PIX = N * N, MT = (PIX + 15) / 16;
    int16_t v[MT * 16];
    bool ok; // every residue class fits in MT tiles
    constexpr TileCells() : v{}, ok(true)
    {
        int count[16] = {};
        for (int i = 0; i < MT * 16; ++i) v[i] = -32768;
        for (int p = 0; p < PIX; ++p) {
            const int q = (p / N) * NP + p % N, r = q % 16, t = count[r]++;
            if (t >= MT) ok = false;
            else v[t * 16 + r] = (int16_t)q;
        }
        for (int t = 0; t < MT; ++t) {
            int first = 0;
            for (int r = 15; r >= 0; --r)
                if (v[t * 16 + r] >= 0) first = v[t * 16 + r];
            for (int r = 0; r < 16; ++r)
                if (v[t * 16 + r] == -32768) v[t * 16 + r] = (int16_t)(-1 - first);
        }
    }
};
static_assert(TileCells<11>().ok && TileCells<19>().ok, "tile partition");
__constant__ TileCells<11> kTiles11 = TileCells<11>();
__constant__ TileCells<19> kTiles19 = TileCells<19>();

// the entry of lane `row` of tile `mt` (see TileCells)
template <int N>
__device__ __forceinline__ int tile_entry(int mt, int row)
{
    if constexpr (N == 11) return kTiles11.v[mt * 16 + row];
    else return kTiles19.v[mt * 16 + row];
}
__device__ __forceinline__ int entry_q(int e) { return e >= 0 ? e : -1 - e; }

// ---------------------------------------------------------------------------
// The 64-channel convolution with both operands in LDS.  Reading A (the
// activations) straight from memory re-reads every cell once per tap, which
// leaves the MFMA pipes waiting on the vector memory path; here a block
// stages its boards and the weights in LDS, half of the input channels at a
// time (two phases of 9 taps x 32 channels), so each activation byte comes
// from memory once per layer; the staging copies go from memory to LDS
// directly, all of a wave's copies in flight together.  N = 11: 4 boards
// per block, one wave per board with all 64 output channels; N = 19: 2
// boards per block, each board's cells in 3 groups of <= 8 tiles and its
// output channels split over 2 waves (12 waves).  Same MODEs as k_conv,
// plus MODE 2: the first two layers of the forward in one kernel.
// ---------------------------------------------------------------------------
template <int N, int SPLIT>
struct LdsConv {
    static constexpr int SIDE = N;
    static constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    static constexpr int MT = (PIX + 15) / 16, NG = (MT + 7) / 8;
    static constexpr int BPB = N <= 13 ? 4 : 2;        // boards per block
    static constexpr int NSPLIT = SPLIT;                // waves sharing a board's 64 output channels
    static constexpr int NTW = 4 / NSPLIT;              // output-channel tiles per wave
    static constexpr int THREADS = BPB * NG * NSPLIT * 64;
    static constexpr int WS = 9 * 32 + 8;               // weight row stride (bf16), one half of K
};
// the per-group kernel (k_conv_lds) gives each board's 64 output channels to
// one wave at 11x11 (each activation fragment then feeds four MFMAs instead
// of two: 0.81 against 0.94 ms per 65536-board layer) and to two at 19x19
// (measured 3 % faster there); the weights-resident one (k_conv_res) splits
// them over two (its register prefetch of the next group leaves no room for
// 128 accumulators)
template <int N>
using LdsL = LdsConv<N, N <= 13 ? 1 : 2>;
template <int N>
using LdsR = LdsConv<N, 2>;

// The board and head sides of the fused forward: the boards and sides to
// move, layer 1's packed weights and bias (MODE 2: layers 1 and 2 in one
// kernel), and the parameter vector and outputs of the heads (MODE 3: the
// last layer and the heads in one kernel).
struct FwdArgs {
    const int8_t *board, *to_move;
    const uint16_t *w1;
    const float *b1;
    const float *params;
    float *logits, *value;
    // Every LDS convolution takes the zero ring of its input from zero16 (16
    // zero bytes) instead of from memory, so an output's ring is written only
    // when ring != 0: the training forward, whose activations the weight
    // gradients read with their taps.
    const uint16_t *zero16;
    int ring;
    // MODE 4 (the fused guided step): the policy ply of each board's env,
    // drawn from the logits on chip (see guided_step below)
    DevState st;
    int kind, max_plies;
    uint32_t key0, key1;
    int64_t gid_base;
    const int64_t *gid;
    int8_t *reward;
    uint8_t *terminal;
};

// Cell codes of the fused forward: for each board of a block and each cell
// of its padded frame, 0 = the mover's stone, 1 = the opponent's, 2 = empty,
// 3 = the zero ring, in the mover's frame (player 2 sees the transpose of the
// board: frame cell (r, c) is board cell c N + r), so a layer-1 tap is one
// byte read.  These are the encoder's planes (mover, opponent, empty, 0).
// The raw inputs of one thread's cell codes (board byte and side to move of
// each of its cells; x = -1 for a ring cell or a board past the batch end),
// loaded ahead of the store so that the loads' latencies overlap.
template <class L>
struct CodeIn {
    static constexpr int R = (L::BPB * L::PP + L::THREADS - 1) / L::THREADS;
    int x[R], me[R];
};

template <class L>
__device__ __forceinline__ void code_load(const FwdArgs &a1, int64_t b0, int64_t n, CodeIn<L> &ci)
{
    constexpr int N = L::SIDE, NP = L::NP, PP = L::PP, PIX = L::PIX, ITEMS = L::BPB * PP;
#pragma unroll
    for (int k = 0; k < CodeIn<L>::R; ++k) {
        const int j = threadIdx.x + k * L::THREADS, bb = j / PP, q = j % PP, rr = q / NP - 1, c = q % NP - 1;
        const bool in = j < ITEMS && b0 + bb < n && (unsigned)rr < (unsigned)N && (unsigned)c < (unsigned)N;
        ci.me[k] = in ? (int)a1.to_move[b0 + bb] : 0;
        ci.x[k] = in ? (int)a1.board[(b0 + bb) * PIX + (ci.me[k] == 2 ? c * N + rr : rr * N + c)] : -1;
    }
}

template <class L>
__device__ __forceinline__ void code_store(const CodeIn<L> &ci, uint8_t *cc)
{
#pragma unroll
    for (int k = 0; k < CodeIn<L>::R; ++k) {
        const int j = threadIdx.x + k * L::THREADS;
        if (j < L::BPB * L::PP)
            cc[j] = (uint8_t)(ci.x[k] < 0 ? 3 : (ci.x[k] == ci.me[k] ? 0 : (ci.x[k] == 0 ? 2 : 1)));
    }
}

// Cell codes of the fused forward: for each board of a block and each cell
// of its padded frame, 0 = the mover's stone, 1 = the opponent's, 2 = empty,
// 3 = the zero ring, in the mover's frame (player 2 sees the transpose of the
// board: frame cell (r, c) is board cell c N + r), so a layer-1 tap is one
// byte read.  These are the encoder's planes (mover, opponent, empty, 0).
template <class L>
__device__ __forceinline__ void cell_codes(const FwdArgs &a1, int64_t b0, int64_t n, uint8_t *cc)
{
    CodeIn<L> ci;
    code_load<L>(a1, b0, n, ci);
    code_store<L>(ci, cc);
}

// Layer 1 (3 input planes, 64 output channels) for the output channels
// 32 h .. 32 h + 31 of the block's BPB boards, written bf16(relu) into the
// interior cells of the block's LDS tile in the layout layer 2 reads (cell q
// of board bb at xs + (bb PP + q) 32, chunk c8 at position (c8 + q / 4) mod 4).
// The input planes come from the cell codes (cc).  Work items (board,
// 16-cell tile, 16-channel tile) are spread over the block's waves (a wave
// always gets the same channel tile, so its weight fragments are loaded
// once); an item is two MFMAs (K = 9 taps x 4 planes, padded to 64) with the
// channels as M, so a lane ends with 4 consecutive channels of one cell: one
// 8-byte LDS write.
template <class L>
__device__ __forceinline__ void layer1_half(const FwdArgs &a1, int h, int64_t b0, int64_t n, const uint8_t *cc,
                                            uint16_t *xs)
{
    constexpr int N = L::SIDE, NP = L::NP, PP = L::PP, PIX = L::PIX, MT = L::MT, BPB = L::BPB;
    constexpr int NWAVES = L::THREADS / 64;
    static_assert(NWAVES % 2 == 0, "a wave keeps one channel tile");
    const int lane = threadIdx.x & 63, row = lane & 15, quad = lane >> 4;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int co = 32 * h + 16 * (wid & 1); // the wave's channel tile
    uint4 wa[K1 / 32];
#pragma unroll
    for (int ks = 0; ks < K1 / 32; ++ks)
        wa[ks] = *reinterpret_cast<const uint4 *>(a1.w1 + (co + row) * K1 + ks * 32 + quad * 8);
    const f32x4 bias = {a1.b1[co + 4 * quad], a1.b1[co + 4 * quad + 1], a1.b1[co + 4 * quad + 2],
                        a1.b1[co + 4 * quad + 3]};
    // frame offsets of this lane's taps 8 ks + 2 quad + e; taps >= 9 (zero
    // weights) read tap 0
    int toff[K1 / 32][2];
#pragma unroll
    for (int ks = 0; ks < K1 / 32; ++ks)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int t = 8 * ks + 2 * quad + e, u = t < 9 ? t : 0;
            toff[ks][e] = (u / 3) * NP + u % 3;
        }
    constexpr uint32_t ONE = 0x3F80u; // bf16 1.0
#pragma unroll 1
    for (int it = wid; it < BPB * MT * 2; it += NWAVES) {
        const int bb = it / (MT * 2), mt = (it % (MT * 2)) >> 1;
        if (b0 + bb >= n) continue; // a board past the batch end: its tile is never read
        const int p = mt * 16 + row, pc = p < PIX ? p : 0;
        const uint8_t *cb = cc + bb * PP + (pc / N) * NP + pc % N; // top-left tap of cell p
        f32x4 acc = bias;
#pragma unroll
        for (int ks = 0; ks < K1 / 32; ++ks) {
            uint32_t v[4];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint32_t code = cb[toff[ks][e]];
                v[2 * e] = code < 2 ? ONE << (16 * code) : 0u; // planes 0, 1
                v[2 * e + 1] = code == 2 ? ONE : 0u;           // planes 2, 3
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(wa[ks]), as_bf16x8(uint4{v[0], v[1], v[2], v[3]}),
                                                          acc, 0, 0, 0);
        }
        if (p < PIX) { // channels co + 4 quad + k, k < 4, of cell p
            const int q = (p / N + 1) * NP + p % N + 1, c = co - 32 * h + 4 * quad;
            const uint2 o = {pack_bf16(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f)),
                             pack_bf16(fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f))};
            *reinterpret_cast<uint2 *>(xs + (bb * PP + q) * 32 + (((c >> 3) + (q >> 2)) & 3) * 8 + (c & 7)) = o;
        }
    }
}

// The heads on the last layer's accumulators (k_conv_lds MODE 3), for a
// wave that holds all 64 channels (NTW = 4, lane channels c0 = 16 quad ..
// c0 + 15) of all cells of its board b (tiles mt < 8, cell_off / vmask as in
// k_conv_lds): the layer's output y = bf16(relu(acc)) as the next layer would
// read it, then per cell the policy logit wp . y + bp (written in action
// order: player 2's frame is transposed back) and the value
// tanh(wv . mean over cells of y + bv), the same sums as k_heads.
template <int N, int NTW>
__device__ __forceinline__ void heads_epilogue(const f32x4 (&acc)[8][NTW], const int (&cell_off)[8], unsigned vmask,
                                               int c0, int64_t b, const FwdArgs &a1)
{
    static_assert(NTW == 4, "one wave holds all channels of its cells");
    constexpr int NP = N + 2, PIX = N * N;
    const int lane = threadIdx.x & 63, quad = lane >> 4;
    float wp[16], wv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        wp[j] = a1.params[WP_OFF + c0 + j];
        wv[j] = a1.params[WV_OFF + c0 + j];
    }
    const float bp = a1.params[BP_OFF];
    const int me = a1.to_move[b];
    float sv = 0.f;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        const bool valid = (vmask >> mt) & 1u;
        float lp = 0.f, lv = 0.f;
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
            for (int k = 0; k < 4; k += 2) {
                float y0, y1;
                relu_bf16_pair(acc[mt][nt][k], acc[mt][nt][k + 1], y0, y1);
                lp += y0 * wp[4 * nt + k];
                lv += y0 * wv[4 * nt + k];
                lp += y1 * wp[4 * nt + k + 1];
                lv += y1 * wv[4 * nt + k + 1];
            }
        // the four quads hold the four 16-channel parts of the same cell
        lp += __shfl_xor(lp, 16);
        lp += __shfl_xor(lp, 32);
        lv += __shfl_xor(lv, 16);
        lv += __shfl_xor(lv, 32);
        if (valid) {
            sv += lv;
            if (quad == 0) {
                const int r = cell_off[mt] / NP, c = cell_off[mt] % NP;
                a1.logits[b * PIX + (me == 2 ? c * N + r : r * N + c)] = lp + bp;
            }
        }
    }
    // the 16 rows of a quad cover all cells of the board once
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) sv += __shfl_xor(sv, s);
    if (lane == 0) a1.value[b] = tanhf(sv / (float)PIX + a1.params[BV_OFF]);
}

// The policy logits of heads_epilogue, for the fused guided step: the same
// sums, written to the board's LDS row lg (action order) instead of memory;
// no value.
template <int N, int NTW>
__device__ __forceinline__ void heads_to_lds(const f32x4 (&acc)[8][NTW], const int (&cell_off)[8], unsigned vmask,
                                             int c0, int64_t b, const FwdArgs &a1, float *lg)
{
    static_assert(NTW == 4, "one wave holds all channels of its cells");
    constexpr int NP = N + 2;
    const int lane = threadIdx.x & 63, quad = lane >> 4;
    float wp[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) wp[j] = a1.params[WP_OFF + c0 + j];
    const float bp = a1.params[BP_OFF];
    const int me = a1.to_move[b];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        const bool valid = (vmask >> mt) & 1u;
        float lp = 0.f;
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
            for (int k = 0; k < 4; k += 2) {
                float y0, y1;
                relu_bf16_pair(acc[mt][nt][k], acc[mt][nt][k + 1], y0, y1);
                lp += y0 * wp[4 * nt + k];
                lp += y1 * wp[4 * nt + k + 1];
            }
        lp += __shfl_xor(lp, 16);
        lp += __shfl_xor(lp, 32);
        if (valid && quad == 0) {
            const int r = cell_off[mt] / NP, c = cell_off[mt] % NP;
            lg[me == 2 ? c * N + r : r * N + c] = lp + bp;
        }
    }
}

// MODE 2 (forward of the first two layers): each channel half of layer 1's
// output is computed by the block from its boards (a1) straight into the LDS
// tile that layer 2 reads, so layer 1's activations never go to memory; x is
// unused, w / bias are layer 2's and the output is layer 2's.
// MODE 3 (the last layer and the heads, 11x11): a forward layer whose output
// goes through the heads in registers (heads_epilogue) instead of to memory;
// out is unused, the logits and values go to a1.logits / a1.value.
template <int N, int MODE>
__global__ __launch_bounds__(LdsL<N>::THREADS, 2) void k_conv_lds(const uint16_t *__restrict__ x,
                                                                     const uint16_t *__restrict__ w,
                                                                     const float *__restrict__ bias,
                                                                     const uint16_t *__restrict__ mask,
                                                                     uint16_t *__restrict__ out, int64_t n,
                                                                     FwdArgs a1)
{
    using L = LdsL<N>;
    constexpr int NP = L::NP, PP = L::PP, MT = L::MT, NG = L::NG, BPB = L::BPB, WS = L::WS;
    constexpr int NTW = L::NTW;
    static_assert(MODE != 3 || (NG == 1 && MT <= 8 && NTW == 4), "MODE 3: one wave holds a whole board");
    __shared__ __align__(16) uint16_t ws[C * WS];
    __shared__ __align__(16) uint16_t xs[BPB * PP * 32];
    // MODE 2: the cell codes of the block's boards
    __shared__ uint8_t cc[MODE == 2 ? BPB * PP : 1];

    const int lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) / L::NSPLIT, half = (threadIdx.x >> 6) % L::NSPLIT;
    const int slot = wave / NG, g = wave % NG;
    const int64_t b0 = (int64_t)blockIdx.x * BPB;
    const int64_t b = b0 + slot;
    const bool live = b < n;
    const int row = lane & 15, quad = lane >> 4;
    // this lane's cell in each tile (see TileCells): its top-left tap in the
    // padded frame, and bit mt set if the lane has a cell in tile mt
    int cell_off[8];
    unsigned vmask = 0;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        const int e = g * 8 + mt < MT ? tile_entry<N>(g * 8 + mt, row) : -1;
        cell_off[mt] = entry_q(e);
        vmask |= (e >= 0 ? 1u : 0u) << mt;
    }
    // this lane's output channels are c0 .. c0 + 4 NTW - 1; the accumulators
    // start at their bias
    const int c0 = half * 16 * NTW + 4 * NTW * quad;
    f32x4 acc[8][NTW];
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
        f32x4 bv = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE != 1)
#pragma unroll
            for (int k = 0; k < 4; ++k) bv[k] = bias[c0 + 4 * nt + k];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt][nt] = bv;
    }

    if constexpr (MODE == 2) cell_codes<L>(a1, b0, n, cc); // read after the barrier below
    for (int h = 0; h < 2; ++h) { // input channels 32h .. 32h+31
        // the staging goes straight from memory to LDS (no registers), every
        // load of a wave in flight at once; a wave instruction fills 64
        // consecutive 16-byte chunks of the tile, one per lane, so each lane
        // picks the source of its chunk
        __syncthreads(); // the previous half's products are done
        {
            const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
            constexpr int NWAVES = L::THREADS / 64, WCH = C * (WS / 8); // 37 chunks a row, the last one padding
            for (int base = wid * 64; base < WCH; base += NWAVES * 64) {
                const int i = base + lane, srow = i / (WS / 8), col = i % (WS / 8);
                const int o = w_channel<NTW>(srow), t = col < 36 ? col >> 2 : 0, c8 = col < 36 ? col & 3 : 0;
                if (i < WCH)
                    __builtin_amdgcn_global_load_lds(
                        (glb_void *)(w + (int64_t)o * K2 + t * 64 + h * 32 + c8 * 8), (lds_void *)(ws + base * 8), 16,
                        0, 0);
            }
            if constexpr (MODE != 2) {
                constexpr int XCH = BPB * PP * 4;
                for (int base = wid * 64; base < XCH; base += NWAVES * 64) {
                    // chunk c8 of cell q sits at chunk position (c8 + q / 4) mod 4: the 16 cells
                    // a fragment read touches then fall on 16 different LDS bank groups
                    const int i = base + lane, bb = i / (PP * 4), q = (i % (PP * 4)) >> 2;
                    const int c8 = ((i & 3) - (q >> 2)) & 3, qr = q / NP, qc = q % NP;
                    const bool ring = qr == 0 || qr == NP - 1 || qc == 0 || qc == NP - 1;
                    const int64_t bsrc = b0 + bb < n ? b0 + bb : b0; // a board past the end: any valid one
                    const uint16_t *src = ring ? a1.zero16 : x + (bsrc * PP + q) * C + h * 32 + c8 * 8;
                    if (i < XCH)
                        __builtin_amdgcn_global_load_lds((glb_void *)src, (lds_void *)(xs + base * 8), 16, 0, 0);
                }
            }
        }
        if constexpr (MODE == 2) {
            if (h == 0) {
                // the ring of every board's tile stays zero for both halves
                for (int j = threadIdx.x; j < BPB * 4 * (NP - 1) * 4; j += L::THREADS) {
                    const int bb = j / (4 * (NP - 1) * 4), r = j % (4 * (NP - 1) * 4);
                    const int q = ring_cell<NP>(r >> 2);
                    *reinterpret_cast<uint4 *>(xs + (bb * PP + q) * 32 + (r & 3) * 8) = uint4{0u, 0u, 0u, 0u};
                }
            }
            layer1_half<L>(a1, h, b0, n, cc, xs);
        }
        __builtin_amdgcn_s_waitcnt(0); // this wave's memory-to-LDS loads have landed
        __syncthreads();
        if (!live) continue;
        const uint16_t *xb = xs + slot * PP * 32;
        // the 9 taps.  With all 64 channels in the wave (and registers to
        // spare: not MODE 2), unrolled, tap t + 1's fragments read from LDS
        // while tap t's products run; else one tap at a time.
        constexpr bool PIPE = NTW == 4 && MODE != 2;
        auto frag_b = [&](int t, bf16x8 (&bf)[NTW]) {
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt)
                bf[nt] = as_bf16x8(
                    *reinterpret_cast<const uint4 *>(ws + ((half * NTW + nt) * 16 + row) * WS + t * 32 + quad * 8));
        };
        auto frag_a = [&](int t, bf16x8 (&af)[8]) {
            const int toff = (t / 3) * NP + (t % 3);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                if (g * 8 + mt < MT) {
                    const int q = cell_off[mt] + toff;
                    af[mt] = as_bf16x8(*reinterpret_cast<const uint4 *>(xb + q * 32 + ((quad + (q >> 2)) & 3) * 8));
                }
        };
        if constexpr (PIPE) {
            bf16x8 bcur[NTW], acur[8], bnxt[NTW], anxt[8];
            frag_b(0, bcur);
            frag_a(0, acur);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                if (t + 1 < 9) {
                    frag_b(t + 1, bnxt);
                    frag_a(t + 1, anxt);
                }
#pragma unroll
                for (int mt = 0; mt < 8; ++mt)
                    if (g * 8 + mt < MT)
#pragma unroll
                        for (int nt = 0; nt < NTW; ++nt)
                            acc[mt][nt] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(bcur[nt], acur[mt], acc[mt][nt], 0, 0, 0);
                if (t + 1 < 9) {
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt) bcur[nt] = bnxt[nt];
#pragma unroll
                    for (int mt = 0; mt < 8; ++mt) acur[mt] = anxt[mt];
                }
            }
        } else {
#pragma unroll 1
            for (int t = 0; t < 9; ++t) {
                const int toff = (t / 3) * NP + (t % 3);
                bf16x8 bf[NTW];
                frag_b(t, bf);
#pragma unroll
                for (int mt = 0; mt < 8; ++mt) {
                    if (g * 8 + mt >= MT) break;
                    const int q = cell_off[mt] + toff;
                    const bf16x8 a =
                        as_bf16x8(*reinterpret_cast<const uint4 *>(xb + q * 32 + ((quad + (q >> 2)) & 3) * 8));
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[nt], a, acc[mt][nt], 0, 0, 0);
                }
            }
        }
    }
    if constexpr (MODE == 4) {
        // the fused guided step: the logits of each board go to LDS (the
        // activation tile is free once every wave's products are done), its
        // board bytes beside them, and one lane per board draws and plays
        // the policy ply (policy_ply_one)
        static_assert(NG == 1 && L::NSPLIT == 1, "MODE 4: one wave holds a whole board");
        constexpr int PIX = L::PIX;
        __syncthreads();
        constexpr int LGS = (PIX + 3) / 4 * 4, BRS = (PIX + 31) / 16 * 16;
        float *lg = reinterpret_cast<float *>(xs) + slot * LGS;
        int8_t *brow = reinterpret_cast<int8_t *>(xs) + BPB * LGS * 4 + slot * BRS;
        static_assert(BPB * LGS * 4 + BPB * BRS <= BPB * PP * 32 * 2, "logits and boards fit the tile");
        if (live) {
            heads_to_lds<N, NTW>(acc, cell_off, vmask, c0, b, a1, lg);
            for (int j = lane; j < PIX; j += 64) brow[j] = a1.board[b * PIX + j];
        }
        __syncthreads();
        if (live) {
            int tmv;
            bool run;
            if (a1.kind == 3)
                wave_policy_ply<Hex<N>>(a1.st, b, a1.max_plies, lg, brow, a1.key0, a1.key1, a1.gid_base, a1.gid,
                                        a1.reward, a1.terminal, tmv, run);
            else
                wave_policy_ply<Gomoku<N>>(a1.st, b, a1.max_plies, lg, brow, a1.key0, a1.key1, a1.gid_base, a1.gid,
                                           a1.reward, a1.terminal, tmv, run);
        }
        return;
    }
    if (!live) return;

    if constexpr (MODE == 3) {
        heads_epilogue<N, NTW>(acc, cell_off, vmask, c0, b, a1);
        return;
    }
    uint16_t *ob = out + b * (int64_t)PP * C;
    if (g == 0 && half == 0 && a1.ring) zero_ring<N>(ob, lane);
    const uint16_t *mb = MODE == 1 ? mask + b * (int64_t)PP * C : nullptr;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        if (g * 8 + mt >= MT) break;
        if (!((vmask >> mt) & 1u)) continue;
        const int64_t o = (int64_t)(cell_off[mt] + NP + 1) * C + c0; // the cell: one row and column in
        store_cell<NTW, MODE == 1 ? 1 : 0>(acc[mt], MODE == 1 ? mb + o : nullptr, ob + o);
    }
}

// ---------------------------------------------------------------------------
// The whole 11x11 forward in one persistent kernel, the activations never
// leaving the chip.  A block (one per CU: 4 waves, one per board) walks
// 4-board groups; a group's activations of both channel halves stay in LDS
// (86.5 KB) through all four layers, each layer's weights are staged half
// by half (37.9 KB, from L2), and layer 4 goes through the heads in
// registers.  Per layer a wave keeps its board's 64 channels x 8 cell tiles
// in accumulators; after the last half's products (and a barrier) it
// writes bf16(relu) back over the layer's input.  The layer-by-layer kernels
// write every activation to memory and read it back (37 KB per board and
// layer); this one moves the boards in and the heads out.
//   MODE 0: logits and values to memory (ludax_net_forward's results).
//   MODE 1: `plies` guided plies of every env, then the value cutoff: after
//           layer 4 each board's logits go to LDS and the board's first lane
//           draws and plays the policy ply (the board row and the side to
//           move stay in LDS between plies); after the last ply one more
//           forward gives estimate[b] (ludax_net_estimate's mapping).
// ---------------------------------------------------------------------------
struct FusedArgs {
    const float *params;
    const uint16_t *packed;
    int64_t n;
    // MODE 0
    const int8_t *board, *to_move;
    float *logits, *value;
    // MODE 1
    DevState st;
    int kind, max_plies, plies;
    uint32_t key0, key1;
    int64_t gid_base;
    const int64_t *gid;
    float *estimate;
};

// One guided ply of a board whose env state lives in LDS for the whole
// group (k_fwd11 MODE 1), by the 64 lanes of its wave: sc = {status, side
// to move, winner, passes, ply, last action}, brow = its board bytes, lg =
// its logits.  The draw and the rules are those of wave_policy_ply; lane 0
// updates sc and brow.  Returns the cell played, or -1.
template <class G>
__device__ __forceinline__ int lds_policy_ply(int *sc, uint64_t id, int max_plies, const float *lg, int8_t *brow,
                                              uint32_t key0, uint32_t key1)
{
    const int lane = threadIdx.x & 63;
    int status = sc[0];
    if (status != RUNNING) return -1;
    int me = sc[1], winner = sc[2], passes = sc[3], ply = sc[4];
    const Philox4 f = philox4x32_10((uint32_t)ply >> 2, (uint32_t)id, (uint32_t)(id >> 32), 0u, key0, key1);
    const int r = ply & 3;
    const uint32_t w = r == 0 ? f.v[0] : (r == 1 ? f.v[1] : (r == 2 ? f.v[2] : f.v[3]));
    const int a = wave_policy_draw<G::CELLS>(lg, brow, w);
    if (a < 0) {
        if (lane == 0) sc[0] = ILLEGAL;
        return -1;
    }
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
    } else {
        me = 3 - me;
        if (ply >= max_plies) {
            status = TRUNCATED;
            winner = -1;
        }
    }
    if (lane == 0) {
        brow[a] = (int8_t)mover;
        sc[0] = status;
        sc[1] = me;
        sc[2] = winner;
        sc[3] = passes;
        sc[4] = ply;
        sc[5] = a;
    }
    return a;
}

constexpr int FUSED_BLOCKS_PER_CU = 1;

// Geometry of the fused 11x11 forward: 4 boards per block, two waves per
// board (cell tiles 0-3 and 4-7), 8 waves.
struct Fused11 {
    static constexpr int SIDE = 11, NP = 13, PP = NP * NP, PIX = 121, MT = 8, BPB = 4, THREADS = 512;
    static constexpr int WS = 9 * 32 + 8;
};

// Stage weight half i (layer 2 + i / 2, input channels 32 (i % 2) ..) of
// the packed forward weights into an LDS buffer of [64][WS] rows, in the
// row permutation of w_channel (memory to LDS directly, the block's waves
// sharing the 37 chunks of each row).
__device__ __forceinline__ void stage_weight_half(const uint16_t *packed, int i, uint16_t *dst)
{
    constexpr int WS = Fused11::WS, WCH = C * (WS / 8), NWAVES = Fused11::THREADS / 64;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint16_t *w = packed + pf_off(2 + i / 2);
    const int h = i % 2;
    for (int base = wid * 64; base < WCH; base += NWAVES * 64) {
        const int j = base + lane, srow = j / (WS / 8), col = j % (WS / 8);
        const int o = w_channel<4>(srow), t = col < 36 ? col >> 2 : 0, c8 = col < 36 ? col & 3 : 0;
        if (j < WCH)
            __builtin_amdgcn_global_load_lds((glb_void *)(w + (int64_t)o * K2 + t * 64 + h * 32 + c8 * 8),
                                             (lds_void *)(dst + base * 8), 16, 0, 0);
    }
}

template <int MODE>
__global__ __launch_bounds__(512, 1) void k_fwd11(FusedArgs fa)
{
    using L = Fused11;
    constexpr int N = L::SIDE, NP = L::NP, PP = L::PP, PIX = L::PIX, BPB = L::BPB, WS = L::WS, NTW = 4, TPW = 4;
    constexpr int NT = L::THREADS;
    // two weight buffers: half i + 1 is staged while half i is multiplied
    __shared__ __align__(16) uint16_t ws[2][C * WS];
    __shared__ __align__(16) uint16_t xa[2][BPB * PP * 32];
    __shared__ __align__(16) int8_t brow[BPB][144];
    __shared__ uint8_t cc[BPB * PP];
    // each board's env state for the group: status, side to move, winner,
    // passes, ply, last action (MODE 0: only the side to move)
    __shared__ int scal[BPB][6];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, slot = wave >> 1, g = wave & 1;
    const int row = lane & 15, quad = lane >> 4;
    const int c0 = 16 * quad; // this lane's output channels c0 .. c0 + 15
    // this wave's cell tiles 4 g .. 4 g + 3; vmask8: which of all 8 tiles have a cell in this lane's row
    int cell_off[TPW];
    unsigned vmask = 0, vmask8 = 0;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) vmask8 |= (tile_entry<N>(mt, row) >= 0 ? 1u : 0u) << mt;
#pragma unroll
    for (int mt = 0; mt < TPW; ++mt) {
        const int e = tile_entry<N>(TPW * g + mt, row);
        cell_off[mt] = entry_q(e);
        vmask |= (e >= 0 ? 1u : 0u) << mt;
    }
    const float *params = fa.params;
    const uint16_t *packed = fa.packed;
    const int64_t n = fa.n;
    FwdArgs a1{};
    a1.w1 = packed + pf_off(1);
    a1.b1 = params + b_off(1);
    // the heads' scratch borrows the start of the first tile once every
    // wave's products are done: per board 128 logits and the value partials
    // of its 8 tiles x 16 rows; so the rings, zero in
    // every layer's input, are re-zeroed at the start of each round
    float *hs = reinterpret_cast<float *>(xa[0]);
    float *lgs = hs, *vps = hs + BPB * 128;
    auto zero_rings = [&]() {
        for (int j = threadIdx.x; j < 2 * BPB * 4 * (NP - 1) * 4; j += NT) {
            const int hh = j / (BPB * 4 * (NP - 1) * 4), r0 = j % (BPB * 4 * (NP - 1) * 4);
            const int bb = r0 / (4 * (NP - 1) * 4), r = r0 % (4 * (NP - 1) * 4);
            const int q = ring_cell<NP>(r >> 2);
            *reinterpret_cast<uint4 *>(xa[hh] + (bb * PP + q) * 32 + (r & 3) * 8) = uint4{0u, 0u, 0u, 0u};
        }
    };
    stage_weight_half(packed, 0, ws[0]);

    const int64_t stride = (int64_t)gridDim.x * BPB;
    for (int64_t b0 = (int64_t)blockIdx.x * BPB; b0 < n; b0 += stride) {
        const int64_t b = b0 + slot;
        const bool live = b < n;
        __syncthreads(); // the previous group is done with brow and scal
        for (int j = threadIdx.x; j < BPB * PIX; j += NT) {
            const int bb = j / PIX, c = j % PIX;
            const int8_t *src = MODE == 0 ? fa.board : fa.st.board;
            brow[bb][c] = b0 + bb < n ? src[(b0 + bb) * PIX + c] : (int8_t)0;
        }
        if (threadIdx.x < BPB) {
            const int64_t bt = b0 + threadIdx.x;
            const bool in = bt < n;
            int *sc = scal[threadIdx.x];
            if constexpr (MODE == 0) {
                sc[0] = ILLEGAL;
                sc[1] = in ? (int)fa.to_move[bt] : 1;
            } else {
                sc[0] = in ? (int)fa.st.status[bt] : ILLEGAL;
                sc[1] = in ? (int)fa.st.to_move[bt] : 1;
                sc[2] = in ? (int)fa.st.winner[bt] : -1;
                sc[3] = in ? (int)fa.st.passes[bt] : 0;
                sc[4] = in ? (int)fa.st.ply[bt] : 0;
                sc[5] = in ? (int)fa.st.last_action[bt] : -1;
            }
        }
        const int rounds = MODE == 0 ? 1 : fa.plies + 1;
        for (int ply = 0; ply < rounds; ++ply) {
            __syncthreads(); // brow / scal of the previous ply are written
            const bool last = ply == rounds - 1;
            if constexpr (MODE == 1) {
                // no env of the group running and no value left to compute
                if (!last && scal[0][0] != 0 && scal[1][0] != 0 && scal[2][0] != 0 && scal[3][0] != 0) continue;
            }
            // is another round coming (this group's next ply or a next group)?
            const bool more = !last || b0 + stride < n;
            for (int j = threadIdx.x; j < BPB * PP; j += NT) {
                const int bb = j / PP, q = j % PP, rr = q / NP - 1, c = q % NP - 1;
                const bool in = b0 + bb < n && (unsigned)rr < (unsigned)N && (unsigned)c < (unsigned)N;
                const int me = scal[bb][1];
                const int x = in ? (int)brow[bb][me == 2 ? c * N + rr : rr * N + c] : -1;
                cc[j] = (uint8_t)(x < 0 ? 3 : (x == me ? 0 : (x == 0 ? 2 : 1)));
            }
            zero_rings();
            __syncthreads();
            layer1_half<L>(a1, 0, b0, n, cc, xa[0]);
            layer1_half<L>(a1, 1, b0, n, cc, xa[1]);
            f32x4 acc[TPW][NTW];
#pragma unroll 1
            for (int i = 0; i < 6; ++i) {
                const int l = 2 + i / 2, h = i % 2;
                if (h == 0) {
                    const float *bias = params + b_off(l);
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt) {
                        const f32x4 bv = {bias[c0 + 4 * nt], bias[c0 + 4 * nt + 1], bias[c0 + 4 * nt + 2],
                                          bias[c0 + 4 * nt + 3]};
#pragma unroll
                        for (int mt = 0; mt < TPW; ++mt) acc[mt][nt] = bv;
                    }
                }
                // half i has landed (every wave's copies) and half i - 1's buffer is free
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (i < 5) stage_weight_half(packed, i + 1, ws[(i + 1) & 1]);
                else if (more) stage_weight_half(packed, 0, ws[0]);
                if (live) {
                    const uint16_t *wb = ws[i & 1];
                    const uint16_t *xb = xa[h] + slot * PP * 32;
                    auto frag_b = [&](int t, bf16x8 (&bf)[NTW]) {
#pragma unroll
                        for (int nt = 0; nt < NTW; ++nt)
                            bf[nt] = as_bf16x8(
                                *reinterpret_cast<const uint4 *>(wb + (nt * 16 + row) * WS + t * 32 + quad * 8));
                    };
                    auto frag_a = [&](int t, bf16x8 (&af)[TPW]) {
                        const int toff = (t / 3) * NP + (t % 3);
#pragma unroll
                        for (int mt = 0; mt < TPW; ++mt) {
                            const int q = cell_off[mt] + toff;
                            af[mt] = as_bf16x8(*reinterpret_cast<const uint4 *>(xb + q * 32 + ((quad + (q >> 2)) & 3) * 8));
                        }
                    };
                    bf16x8 bcur[NTW], acur[TPW], bnxt[NTW], anxt[TPW];
                    frag_b(0, bcur);
                    frag_a(0, acur);
#pragma unroll
                    for (int t = 0; t < 9; ++t) {
                        if (t + 1 < 9) {
                            frag_b(t + 1, bnxt);
                            frag_a(t + 1, anxt);
                        }
#pragma unroll
                        for (int mt = 0; mt < TPW; ++mt)
#pragma unroll
                            for (int nt = 0; nt < NTW; ++nt)
                                acc[mt][nt] =
                                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(bcur[nt], acur[mt], acc[mt][nt], 0, 0, 0);
                        if (t + 1 < 9) {
#pragma unroll
                            for (int nt = 0; nt < NTW; ++nt) bcur[nt] = bnxt[nt];
#pragma unroll
                            for (int mt = 0; mt < TPW; ++mt) acur[mt] = anxt[mt];
                        }
                    }
                }
                if (h == 1 && l < 4) {
                    __syncthreads(); // every wave is done reading the layer's input
                    if (live) {
                        // bf16(relu) of channels c0 .. c0 + 15 of each cell over the input: half
                        // quad / 2, 16-byte chunks 2 (quad & 1) and 2 (quad & 1) + 1
                        uint16_t *xo = xa[quad >> 1] + slot * PP * 32;
#pragma unroll
                        for (int mt = 0; mt < TPW; ++mt) {
                            if (!((vmask >> mt) & 1u)) continue;
                            const int q = cell_off[mt] + NP + 1;
#pragma unroll
                            for (int k8 = 0; k8 < 2; ++k8) {
                                uint32_t wv[4];
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    const int i0 = 8 * k8 + 2 * j, i1 = i0 + 1;
                                    const float v0 = fmaxf(acc[mt][i0 >> 2][i0 & 3], 0.f);
                                    const float v1 = fmaxf(acc[mt][i1 >> 2][i1 & 3], 0.f);
                                    wv[j] = pack_bf16(v0, v1);
                                }
                                const int c8 = 2 * (quad & 1) + k8;
                                *reinterpret_cast<uint4 *>(xo + q * 32 + ((c8 + (q >> 2)) & 3) * 8) =
                                    uint4{wv[0], wv[1], wv[2], wv[3]};
                            }
                        }
                    }
                }
            }
            // the heads on layer 4's accumulators (y = the layer's output as it
            // would be stored): per cell the policy logit, per tile the value
            // partial of each row; the same sums as heads_epilogue
            const bool policy = MODE == 0 || !last;
            const int me = scal[slot][1];
            __syncthreads(); // the tiles are free: the heads' scratch goes there
            if (live) {
                float wp[16], wv[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    wp[j] = params[WP_OFF + c0 + j];
                    wv[j] = params[WV_OFF + c0 + j];
                }
                const float bp = params[BP_OFF];
#pragma unroll
                for (int mt = 0; mt < TPW; ++mt) {
                    float lp = 0.f, lv = 0.f;
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
                        for (int k = 0; k < 4; k += 2) {
                            float y0, y1;
                            relu_bf16_pair(acc[mt][nt][k], acc[mt][nt][k + 1], y0, y1);
                            lp += y0 * wp[4 * nt + k];
                            lv += y0 * wv[4 * nt + k];
                            lp += y1 * wp[4 * nt + k + 1];
                            lv += y1 * wv[4 * nt + k + 1];
                        }
                    lp += __shfl_xor(lp, 16);
                    lp += __shfl_xor(lp, 32);
                    lv += __shfl_xor(lv, 16);
                    lv += __shfl_xor(lv, 32);
                    if (quad == 0) vps[(slot * 8 + TPW * g + mt) * 16 + row] = lv;
                    if (policy && ((vmask >> mt) & 1u) && quad == 0) {
                        const int r = cell_off[mt] / NP, c = cell_off[mt] % NP;
                        const int a = me == 2 ? c * N + r : r * N + c;
                        if (MODE == 0) fa.logits[b * PIX + a] = lp + bp;
                        else lgs[slot * 128 + a] = lp + bp;
                    }
                }
            }
            __syncthreads();
            // the value: the partials of all 8 tiles in tile order, then over the rows
            float v = 0.f;
            if (live && g == 0) {
                float sv = 0.f;
#pragma unroll
                for (int mt = 0; mt < 8; ++mt)
                    if ((vmask8 >> mt) & 1u) sv += vps[(slot * 8 + mt) * 16 + row];
#pragma unroll
                for (int sft = 8; sft >= 1; sft >>= 1) sv += __shfl_xor(sv, sft);
                v = tanhf(sv / (float)PIX + params[BV_OFF]);
            }
            if constexpr (MODE == 0) {
                if (live && g == 0 && lane == 0) fa.value[b] = v;
            } else if (last) {
                if (live && g == 0 && lane == 0) {
                    // the value cutoff: the network's value for RUNNING envs (for
                    // player 1), the outcome of ended ones
                    const int stt = scal[slot][0], wn = scal[slot][2];
                    fa.estimate[b] = stt == 1 ? (wn == 1 ? 1.f : (wn == 2 ? -1.f : 0.f))
                                              : (stt == 0 ? (me == 1 ? v : -v) : 0.f);
                }
            } else if (wave < BPB && b0 + wave < n) {
                // board `wave`'s ply by wave `wave`: the four plies on four SIMDs
                const int64_t bp = b0 + wave;
                const uint64_t id = (uint64_t)(fa.gid != nullptr ? fa.gid[bp] : fa.gid_base + bp);
                if (fa.kind == 3)
                    lds_policy_ply<Hex<N>>(scal[wave], id, fa.max_plies, lgs + wave * 128, brow[wave], fa.key0,
                                           fa.key1);
                else
                    lds_policy_ply<Gomoku<N>>(scal[wave], id, fa.max_plies, lgs + wave * 128, brow[wave], fa.key0,
                                              fa.key1);
            }
        }
        if constexpr (MODE == 1) {
            // the group's final states back to memory
            __syncthreads();
            for (int j = threadIdx.x; j < BPB * PIX; j += NT) {
                const int bb = j / PIX, c = j % PIX;
                if (b0 + bb < n) fa.st.board[(b0 + bb) * PIX + c] = brow[bb][c];
            }
            if (threadIdx.x < BPB && b0 + threadIdx.x < n) {
                const int64_t bt = b0 + threadIdx.x;
                const int *sc = scal[threadIdx.x];
                fa.st.status[bt] = (int8_t)sc[0];
                fa.st.to_move[bt] = (int8_t)sc[1];
                fa.st.winner[bt] = (int8_t)sc[2];
                fa.st.passes[bt] = (int8_t)sc[3];
                fa.st.ply[bt] = (int16_t)sc[4];
                fa.st.last_action[bt] = (int16_t)sc[5];
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0); // no copy to LDS outlives the block
}

// ---------------------------------------------------------------------------
// The same convolution with the weights resident: one block per CU keeps
// all 64 x 576 weights in LDS for the whole launch (staged once, instead of
// once per 4-board group) and walks its share of the BPB-board groups; a
// group's activations are staged half of the input channels at a time, and
// the next (group, half) is loaded into registers while the current one is
// multiplied.  Same wave mapping, MODEs and epilogue as k_conv_lds.  Used
// for the 19x19 forward, where it measured faster; at 11x11 one block per CU
// keeps too few bytes in flight and the per-group kernel wins.
// ---------------------------------------------------------------------------
constexpr int RES_BLOCKS = 256; // one per CU

// MODE 2 as in k_conv_lds: the first two layers, layer 1 computed per group
// from its cell codes; the next group's board bytes are loaded into
// registers while the current group is multiplied.
// MODE 3: the last layer and the heads (see heads_epilogue).  A board's
// channels and cells are spread over 2 x 3 waves: each wave adds its
// per-cell policy partials into LDS (float atomics: two adds onto zero per
// logit, the same sum in either order) and writes its value partial to its
// own LDS slot, the slots summed in a fixed order when the group is written
// out (after the next group's first barrier, the last one after the loop),
// so values are reproducible bit for bit; the logit sums are cleared there.
template <int N, int MODE>
__global__ __launch_bounds__(LdsR<N>::THREADS, 1) void k_conv_res(const uint16_t *__restrict__ x,
                                                                     const uint16_t *__restrict__ w,
                                                                     const float *__restrict__ bias,
                                                                     const uint16_t *__restrict__ mask,
                                                                     uint16_t *__restrict__ out, int64_t n,
                                                                     FwdArgs a1)
{
    using L = LdsR<N>;
    constexpr int NP = L::NP, PP = L::PP, MT = L::MT, NG = L::NG, BPB = L::BPB;
    constexpr int NTW = L::NTW, THREADS = L::THREADS;
    constexpr int WR = K2 + 8;                           // weight row stride (bf16)
    constexpr int XITEMS = BPB * PP * 4;                 // 16-byte chunks of one (group, half)
    constexpr int XR = MODE == 2 ? 1 : (XITEMS + THREADS - 1) / THREADS; // per thread
    __shared__ __align__(16) uint16_t wsr[C * WR];
    __shared__ __align__(16) uint16_t xs[BPB * PP * 32];
    __shared__ uint8_t cc[MODE == 2 ? BPB * PP : 1]; // MODE 2: the group's cell codes
    // MODE 3: head weights (wp, wv), the group's logit and value sums
    __shared__ float hw[MODE == 3 ? 2 * C : 1];
    __shared__ float hl[MODE == 3 ? BPB * L::PIX : 1];
    __shared__ float hv[MODE == 3 ? BPB * L::NSPLIT * NG : 1];

    const int lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) / L::NSPLIT, half = (threadIdx.x >> 6) % L::NSPLIT;
    const int slot = wave / NG, g = wave % NG;
    const int row = lane & 15, quad = lane >> 4;
    // this lane's cell in each tile (see TileCells): its top-left tap in the
    // padded frame, and bit mt set if the lane has a cell in tile mt
    int cell_off[8];
    unsigned vmask = 0;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        const int e = g * 8 + mt < MT ? tile_entry<N>(g * 8 + mt, row) : -1;
        cell_off[mt] = entry_q(e);
        vmask |= (e >= 0 ? 1u : 0u) << mt;
    }
    for (int j = threadIdx.x; j < C * (K2 / 8); j += THREADS) {
        const int o = j / (K2 / 8), r = j % (K2 / 8);
        *reinterpret_cast<uint4 *>(wsr + w_slot<NTW>(o) * WR + r * 8) =
            *reinterpret_cast<const uint4 *>(w + (int64_t)o * K2 + r * 8);
    }

    // this lane's output channels are c0 .. c0 + 4 NTW - 1; each group's
    // accumulators start at their bias
    const int c0 = half * 16 * NTW + 4 * NTW * quad;
    float bv[4 * NTW];
#pragma unroll
    for (int j = 0; j < 4 * NTW; ++j) bv[j] = MODE != 1 ? bias[c0 + j] : 0.f;

    const int64_t groups = (n + BPB - 1) / BPB;
    CodeIn<L> ci; // MODE 2: the next group's cell-code inputs
    if constexpr (MODE == 2) {
        if ((int64_t)blockIdx.x < groups) code_load<L>(a1, (int64_t)blockIdx.x * BPB, n, ci);
    }
    uint4 pre[XR];
    auto load = [&](int64_t grp, int h) { // chunks (board, cell, 8 channels) of half h
        // chunk j of a group is 16 bytes at element 8 j of its (board, cell) rows,
        // 4 chunks per cell and half
        const uint16_t *base = x + grp * BPB * (int64_t)PP * C + h * 32;
        const int64_t left = (n - grp * BPB) * (int64_t)PP * 4; // chunks of live boards
#pragma unroll
        for (int r = 0; r < XR; ++r) {
            const int j = threadIdx.x + r * THREADS, q = (j >> 2) % PP, qr = q / NP, qc = q % NP;
            const bool ring = qr == 0 || qr == NP - 1 || qc == 0 || qc == NP - 1; // zeros, not read
            pre[r] = j < XITEMS && j < left && !ring
                         ? *reinterpret_cast<const uint4 *>(base + (int64_t)(j >> 2) * C + (j & 3) * 8)
                         : uint4{0u, 0u, 0u, 0u};
        }
    };
    if constexpr (MODE == 3) { // ordered by the first barrier below
        for (int j = threadIdx.x; j < 2 * C; j += THREADS)
            hw[j] = a1.params[(j < C ? WP_OFF : WV_OFF) + (j & (C - 1))];
        for (int j = threadIdx.x; j < BPB * L::PIX; j += THREADS) hl[j] = 0.f;
    }
    // MODE 3: write out the sums of group pg and clear them (after a barrier)
    auto flush = [&](int64_t pg) {
        constexpr int PIX = L::PIX;
        const float bp = a1.params[BP_OFF], bvv = a1.params[BV_OFF];
        for (int j = threadIdx.x; j < BPB * PIX; j += THREADS) {
            const int bb = j / PIX, p = j % PIX;
            const int64_t bo = pg * BPB + bb;
            if (bo < n) {
                const int me = a1.to_move[bo], r = p / N, c = p % N;
                a1.logits[bo * PIX + (me == 2 ? c * N + r : p)] = hl[j] + bp;
            }
            hl[j] = 0.f;
        }
        if (threadIdx.x < BPB) {
            const int64_t bo = pg * BPB + threadIdx.x;
            float sv = 0.f;
            for (int k = 0; k < L::NSPLIT * NG; ++k) sv += hv[threadIdx.x * L::NSPLIT * NG + k];
            if (bo < n) a1.value[bo] = tanhf(sv / (float)PIX + bvv);
        }
    };
    if constexpr (MODE != 2) {
        if ((int64_t)blockIdx.x < groups) load(blockIdx.x, 0);
    } else {
        // layer 1 writes only the interior cells: the ring of the tile stays
        // zero for the whole launch (ordered by the first barrier below)
        for (int j = threadIdx.x; j < BPB * 4 * (NP - 1) * 4; j += THREADS) {
            const int bb = j / (4 * (NP - 1) * 4), r = j % (4 * (NP - 1) * 4);
            const int q = ring_cell<NP>(r >> 2);
            *reinterpret_cast<uint4 *>(xs + (bb * PP + q) * 32 + (r & 3) * 8) = uint4{0u, 0u, 0u, 0u};
        }
    }

    for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const int64_t b = grp * BPB + slot;
        const bool live = b < n;
        f32x4 acc[8][NTW];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) acc[mt][nt] = f32x4{bv[4 * nt], bv[4 * nt + 1], bv[4 * nt + 2], bv[4 * nt + 3]};
        for (int h = 0; h < 2; ++h) { // input channels 32h .. 32h+31
            __syncthreads();          // the weights are in; the previous half's products are done
            if constexpr (MODE == 3) {
                // the previous group's head sums are complete (its epilogue came before this barrier)
                if (h == 0 && grp != (int64_t)blockIdx.x) flush(grp - gridDim.x);
            }
            if constexpr (MODE == 2) {
                if (h == 0) {
                    code_store<L>(ci, cc);
                    __syncthreads();
                    const int64_t ng = grp + gridDim.x;
                    if (ng < groups) code_load<L>(a1, ng * BPB, n, ci);
                }
                layer1_half<L>(a1, h, grp * BPB, n, cc, xs);
                __syncthreads();
            } else {
#pragma unroll
                for (int r = 0; r < XR; ++r) {
                    const int j = threadIdx.x + r * THREADS;
                    if (j < XITEMS) {
                        const int bb = j / (PP * 4), rem = j % (PP * 4), q = rem >> 2, c8 = rem & 3;
                        // chunk c8 of cell q sits at chunk position (c8 + q / 4) mod 4 (bank spread)
                        *reinterpret_cast<uint4 *>(xs + (bb * PP + q) * 32 + ((c8 + (q >> 2)) & 3) * 8) = pre[r];
                    }
                }
                __syncthreads();
                {
                    // the next (group, half): this group's second half, or the next group's first
                    const int64_t ng = h == 0 ? grp : grp + gridDim.x;
                    if (ng < groups) load(ng, h ^ 1);
                }
            }
            if (!live) continue;
            const uint16_t *xb = xs + slot * PP * 32;
#pragma unroll 1
            for (int t = 0; t < 9; ++t) {
                const int toff = (t / 3) * NP + (t % 3);
                bf16x8 bfr[NTW];
#pragma unroll
                for (int nt = 0; nt < NTW; ++nt)
                    bfr[nt] = as_bf16x8(*reinterpret_cast<const uint4 *>(
                        wsr + ((half * NTW + nt) * 16 + row) * WR + t * 64 + h * 32 + quad * 8));
#pragma unroll
                for (int mt = 0; mt < 8; ++mt) {
                    if (g * 8 + mt >= MT) break;
                    const int q = cell_off[mt] + toff;
                    const bf16x8 a =
                        as_bf16x8(*reinterpret_cast<const uint4 *>(xb + q * 32 + ((quad + (q >> 2)) & 3) * 8));
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[nt], a, acc[mt][nt], 0, 0, 0);
                }
            }
        }
        if (!live) continue;
        if constexpr (MODE == 3) {
            // this lane's 4 NTW channels of each of its cells: policy and value dots
            float sv = 0.f;
#pragma unroll
            for (int mt = 0; mt < 8; ++mt) {
                if (g * 8 + mt >= MT) break;
                float lp = 0.f, lv = 0.f;
#pragma unroll
                for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
                    for (int k = 0; k < 4; k += 2) {
                        float y0, y1;
                        relu_bf16_pair(acc[mt][nt][k], acc[mt][nt][k + 1], y0, y1);
                        lp += y0 * hw[c0 + 4 * nt + k];
                        lv += y0 * hw[C + c0 + 4 * nt + k];
                        lp += y1 * hw[c0 + 4 * nt + k + 1];
                        lv += y1 * hw[C + c0 + 4 * nt + k + 1];
                    }
                lp += __shfl_xor(lp, 16); // the four quads: the same cell
                lp += __shfl_xor(lp, 32);
                lv += __shfl_xor(lv, 16);
                lv += __shfl_xor(lv, 32);
                if ((vmask >> mt) & 1u) {
                    sv += lv;
                    if (quad == 0) {
                        // at most two partials per cell onto a zeroed slot: the
                        // first lands exactly and float addition commutes, so
                        // the sum does not depend on which wave adds first
                        static_assert(L::NSPLIT <= 2, "order-independent policy sums");
                        const int r = cell_off[mt] / NP, c = cell_off[mt] % NP;
                        atomicAdd(&hl[slot * L::PIX + r * N + c], lp);
                    }
                }
            }
#pragma unroll
            for (int s2 = 8; s2 >= 1; s2 >>= 1) sv += __shfl_xor(sv, s2); // the 16 rows
            if (lane == 0) hv[(slot * L::NSPLIT + half) * NG + g] = sv;
            continue;
        }
        uint16_t *ob = out + b * (int64_t)PP * C;
        if (g == 0 && half == 0 && a1.ring) zero_ring<N>(ob, lane);
        const uint16_t *mb = MODE == 1 ? mask + b * (int64_t)PP * C : nullptr;
        // the output cells' offsets are formed per group from opaque copies:
        // the compiler would otherwise hold all of them across the launch
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            if (g * 8 + mt >= MT) break;
            if (!((vmask >> mt) & 1u)) continue;
            int co = cell_off[mt];
            asm volatile("" : "+v"(co));
            const int o = (co + NP + 1) * C + c0; // the cell itself
            store_cell<NTW, MODE == 1 ? 1 : 0>(acc[mt], MODE == 1 ? mb + o : nullptr, ob + o);
        }
    }
    if constexpr (MODE == 3) {
        // the block's last group
        const int64_t mine = (int64_t)blockIdx.x < groups ? (groups - 1 - blockIdx.x) / gridDim.x : -1;
        __syncthreads();
        if (mine >= 0) flush((int64_t)blockIdx.x + mine * gridDim.x);
    }
}

// ---------------------------------------------------------------------------
// heads, forward: one wave per board, lanes over cells.
// logits in action order (the frame of player 2 is transposed back), and
// optionally in the mover's frame; value = tanh(wv . mean + bv).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_heads(const uint16_t *__restrict__ y4, const float *__restrict__ p,
                                               const int8_t *__restrict__ to_move, int64_t n,
                                               float *__restrict__ logits, float *__restrict__ logits_frame,
                                               float *__restrict__ value)
{
    constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    __shared__ float hw[2 * C];
    if (threadIdx.x < C) hw[threadIdx.x] = p[WP_OFF + threadIdx.x];
    else if (threadIdx.x < 2 * C) hw[threadIdx.x] = p[WV_OFF + threadIdx.x - C];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n) return;
    const uint16_t *yb = y4 + b * (int64_t)PP * C;
    const int me = to_move[b];
    const float bp = p[BP_OFF];
    float sv = 0.f;
    for (int q = lane; q < PIX; q += WAVE) {
        const uint4 *src = reinterpret_cast<const uint4 *>(yb + (int64_t)(((q / N) + 1) * NP + (q % N) + 1) * C);
        float lp = 0.f, lv = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint4 v = src[j];
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const float y0 = __uint_as_float(wd[h] << 16), y1 = __uint_as_float(wd[h] & 0xFFFF0000u);
                const int c0 = j * 8 + 2 * h;
                lp += y0 * hw[c0] + y1 * hw[c0 + 1];
                lv += y0 * hw[C + c0] + y1 * hw[C + c0 + 1];
            }
        }
        const float l = lp + bp;
        const int r = q / N, c = q % N;
        const int cell = me == 2 ? c * N + r : q;
        logits[b * PIX + cell] = l;
        if (logits_frame) logits_frame[b * PIX + q] = l;
        sv += lv;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) sv += __shfl_xor(sv, s);
    if (lane == 0) value[b] = tanhf(sv / (float)PIX + p[BV_OFF]);
}

// ---------------------------------------------------------------------------
// heads, backward: one wave per sample.  Masked softmax over the empty cells
// of the mover's frame, d(loss)/d(logit), d(loss)/d(pre-tanh value), the
// per-sample loss terms, and dZ4 = bf16((dlogit wp + du wv / PIX) * [Y4 > 0])
// into the padded gradient buffer (ring zeroed).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_heads_bwd(const uint16_t *__restrict__ y4, const uint2 *__restrict__ a0,
                                                   const float *__restrict__ p,
                                                   const float *__restrict__ logits_frame,
                                                   const float *__restrict__ value,
                                                   const int8_t *__restrict__ to_move,
                                                   const int16_t *__restrict__ action, const float *__restrict__ z,
                                                   int64_t n, float beta, float inv_n, float *__restrict__ dlog,
                                                   float *__restrict__ du_out, float *__restrict__ loss_terms,
                                                   uint16_t *__restrict__ g4)
{
    constexpr int NP = N + 2, PP = NP * NP, PIX = N * N, QL = (PIX + 63) / 64;
    __shared__ float hw[2 * C];
    __shared__ float dsh[4][PIX]; // each wave's logit gradients, for the gradient pass
    if (threadIdx.x < C) hw[threadIdx.x] = p[WP_OFF + threadIdx.x];
    else if (threadIdx.x < 2 * C) hw[threadIdx.x] = p[WV_OFF + threadIdx.x - C];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * 4 + wave;
    if (b >= n) return;
    const int me = to_move[b];
    const int act = action[b];
    const int a = me == 2 ? (act % N) * N + act / N : act; // frame index of the move
    const float v = value[b], zb = z[b];

    float l[QL];
    bool legal[QL];
    float mx = -3.0e38f;
#pragma unroll
    for (int j = 0; j < QL; ++j) {
        const int q = lane + 64 * j;
        legal[j] = false;
        l[j] = 0.f;
        if (q < PIX) {
            const int R = q / N + 1, Q = q % N + 1;
            legal[j] = a0[(int64_t)b * PP + R * NP + Q].y != 0u; // the empty plane
            l[j] = logits_frame[b * PIX + q];
            if (legal[j]) mx = fmaxf(mx, l[j]);
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) mx = fmaxf(mx, __shfl_xor(mx, s));
    float e[QL], se = 0.f;
#pragma unroll
    for (int j = 0; j < QL; ++j) {
        e[j] = legal[j] ? expf(l[j] - mx) : 0.f;
        se += e[j];
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) se += __shfl_xor(se, s);
    const float adv = fmaxf(zb - v, 0.f); // weight of the move's log-likelihood, clipped at zero
    const float du = 2.f * (v - zb) * inv_n * (1.f - v * v);
    if (lane == 0) {
        du_out[b] = du;
        loss_terms[2 * b] = (v - zb) * (v - zb) * inv_n;
    }
    uint16_t *gb = g4 + b * (int64_t)PP * C;
    zero_ring<N>(gb, lane);
    const uint16_t *yb = y4 + b * (int64_t)PP * C;
    const float dv = du / (float)PIX;
#pragma unroll
    for (int j = 0; j < QL; ++j) {
        const int q = lane + 64 * j;
        if (q >= PIX) continue;
        const float pi = e[j] / se;
        float d = legal[j] ? beta * adv * pi : 0.f;
        if (q == a) {
            d -= beta * adv;
            loss_terms[2 * b + 1] = beta * adv * -(l[j] - mx - logf(se)) * inv_n;
        }
        d *= inv_n;
        dlog[b * PIX + q] = d;
        dsh[wave][q] = d;
    }
    // dZ4 = [y4 > 0] (d wp + dv wv), 8 cells at a time: lane = (cell, 16-byte
    // chunk of 8 channels), so each load and store covers whole 128-byte cells
    // (the wave's own LDS writes above come first in its instruction order)
    const int sub = lane >> 3, k = lane & 7;
    float wp8[8], wv8[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        wp8[i] = hw[8 * k + i];
        wv8[i] = hw[C + 8 * k + i];
    }
    for (int q = sub; q < PIX; q += 8) {
        const float d = dsh[wave][q];
        const int64_t o = (int64_t)((q / N + 1) * NP + (q % N) + 1) * C + 8 * k;
        const uint4 yv = *reinterpret_cast<const uint4 *>(yb + o);
        const uint32_t wd[4] = {yv.x, yv.y, yv.z, yv.w};
        uint32_t od[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint16_t y0 = (uint16_t)(wd[h] & 0xFFFFu), y1 = (uint16_t)(wd[h] >> 16);
            const float g0 = (y0 != 0 && (y0 & 0x8000u) == 0) ? d * wp8[2 * h] + dv * wv8[2 * h] : 0.f;
            const float g1 = (y1 != 0 && (y1 & 0x8000u) == 0) ? d * wp8[2 * h + 1] + dv * wv8[2 * h + 1] : 0.f;
            od[h] = pack_bf16(g0, g1);
        }
        *reinterpret_cast<uint4 *>(gb + o) = uint4{od[0], od[1], od[2], od[3]};
    }
}

// ---------------------------------------------------------------------------
// head weight gradients, per block partial sums over a share of the batch:
// in parameter order: part[blk][c] = sum dlog[b][q] Y4[b][q][c] (wp),
// part[blk][64] = sum dlog (bp), part[blk][65 + c] = sum du[b] Y4[b][q][c] /
// PIX (wv), part[blk][129] = sum du (bv)
// ---------------------------------------------------------------------------
constexpr int HEAD_PART = 2 * C + 2;

template <int N>
__global__ __launch_bounds__(256) void k_head_wgrad(const uint16_t *__restrict__ y4, const float *__restrict__ dlog,
                                                    const float *__restrict__ du, int64_t n,
                                                    float *__restrict__ part)
{
    // one wave per board, lane = channel; the block's four waves add up in LDS
    constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    __shared__ float red[4][HEAD_PART];
    const int c = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float ap = 0.f, av = 0.f, sp = 0.f, sv = 0.f;
    for (int64_t b = (int64_t)blockIdx.x * 4 + wave; b < n; b += (int64_t)gridDim.x * 4) {
        const uint16_t *yb = y4 + b * (int64_t)PP * C;
        const float *db = dlog + b * PIX;
        float mv = 0.f;
        for (int r = 0; r < N; ++r) { // cells in order, a row's loads issued together
            const uint16_t *yr = yb + (int64_t)((r + 1) * NP + 1) * C + c;
            const float *dr = db + r * N;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const float y = bf2f(yr[q * C]);
                const float d = dr[q];
                ap += d * y;
                mv += y;
                sp += d; // every lane adds the same sum; lane 0's is kept
            }
        }
        av += du[b] * mv / (float)PIX;
        sv += du[b];
    }
    red[wave][c] = ap;
    red[wave][C + 1 + c] = av;
    if (c == 0) {
        red[wave][C] = sp;
        red[wave][2 * C + 1] = sv;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < HEAD_PART; j += 256)
        part[(int64_t)blockIdx.x * HEAD_PART + j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
}

// ---------------------------------------------------------------------------
// conv weight gradient: dW[o][i][t] = sum_{b,p} dZ[b][p][o] X[b][p + tap t][i]
// and db[o] = sum dZ[b][p][o], per block partial sums.  M = 64 output
// channels (4 tiles), N = (tap, input channel) columns, K = cells (padded to
// 32 per board).  Four waves split the column tiles.  A block walks its
// boards one at a time: the next board's dZ and X are loaded into registers
// while the current one is multiplied, then transposed into LDS (cell-major
// rows per channel); the bias gradient is summed by wave 0 from the A
// fragments it already holds.  With 64 input channels wave w takes the
// channel tile w of every tap, so a lane's channel row is fixed and each
// tap is a constant offset: the eight 2-byte reads of a B fragment use
// eight per-K-step addresses with the tap in the instructions' offset
// field; X is transposed two cells at a time (32-bit writes).
// part layout per block: [64 * CR * 9] (param order o, i, t) then [64] db.
// ---------------------------------------------------------------------------
template <int N, int CIN>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t *__restrict__ dz, const uint16_t *__restrict__ x,
                                                    int64_t n, float *__restrict__ part)
{
    constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    constexpr int PIXP = (PIX + 31) / 32 * 32, DS = PIXP + 8; // dZ^T row stride
    // X^T row stride: room for every tap of every cell; with 64 channels
    // even (cell pairs are 32-bit writes) and an odd number of words (the 16
    // rows of a fragment read fall in 16 banks)
    constexpr int PPS = CIN == 64 ? (PP + 1) / 4 * 4 + 2 : PP + 8;
    static_assert(CIN != 64 || (PPS >= PP && PPS % 2 == 0 && (PPS / 2) % 2 == 1), "X^T stride");
    constexpr int CR = CIN == 4 ? 3 : CIN;                    // real input channels
    constexpr int NCOL = 9 * CIN, NT = (NCOL + 15) / 16;      // column tiles
    constexpr int NTW = (NT + 3) / 4;                         // column tiles per wave
    constexpr int PART = C * CR * 9 + C;
    // per-thread loads of one board.  dZ: an item is (channel pair, group of
    // 8 cells) -- the 32 lanes of a half-wave read one cell's 128 bytes --
    // written as two 16-byte rows of dZ^T (cells past the board are its zero
    // padding).  X: a (cell, 8 channels) item, 16 bytes (64 channels), or a
    // cell, 8 bytes (4 channels), written as single cells of X^T.
    constexpr int DZ_ITEMS = 32 * (PIXP / 8), DZ_R = (DZ_ITEMS + 255) / 256;
    // X items: a cell of 4 channels (8 bytes); with 64 channels a pair of
    // cells and 8 channels (two 16-byte loads)
    constexpr int X_ITEMS = CIN == 4 ? PP : (PP + 1) / 2 * 8, X_R = (X_ITEMS + 255) / 256;
    __shared__ __align__(16) uint16_t dzt[C * DS];
    __shared__ __align__(16) uint16_t xt[CIN * PPS];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, quad = lane >> 4;
    f32x4 acc[4][NTW];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < NTW; ++j) acc[mt][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dsum[4] = {0.f, 0.f, 0.f, 0.f}; // wave 0: bias-gradient partial sums of channels mt*16 + row
    // this lane's B column in each of its tiles: (tap offset, channel)
    int col_off[NTW], col_ch[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        const int col = (wave * NTW + j) * 16 + row;
        const int cc = col < NCOL ? col : 0;
        const int t = cc / CIN, i = cc % CIN;
        col_off[j] = (t / 3) * NP + (t % 3);
        col_ch[j] = i;
    }
    static_assert(CIN != 64 || NTW == 9, "64 channels: a wave's tiles are the 9 taps of its channel tile");
    uint32_t dzv[DZ_R][8]; // the next board: 8 cells of a channel pair per item
    uint4 xv[X_R], xv2[CIN == 64 ? X_R : 1];
    auto load_board = [&](int64_t b) {
        const uint16_t *db = dz + b * (int64_t)PP * C;
        const uint16_t *xb = x + b * (int64_t)PP * CIN;
#pragma unroll
        for (int r = 0; r < DZ_R; ++r) {
            const int j = threadIdx.x + 256 * r;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int q = (j >> 5) * 8 + i; // cells past PIX are the zero padding of dZ^T
                dzv[r][i] = j < DZ_ITEMS && q < PIX
                                ? *reinterpret_cast<const uint32_t *>(db + (int64_t)((q / N + 1) * NP + q % N + 1) * C +
                                                                      2 * (j & 31))
                                : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < X_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < X_ITEMS) {
                if constexpr (CIN == 4) {
                    const uint2 v = *reinterpret_cast<const uint2 *>(xb + (int64_t)j * 4);
                    xv[r] = uint4{v.x, v.y, 0u, 0u};
                } else {
                    const int q = 2 * (j >> 3), c8 = (j & 7) * 8;
                    xv[r] = *reinterpret_cast<const uint4 *>(xb + (int64_t)q * C + c8);
                    xv2[r] = q + 1 < PP ? *reinterpret_cast<const uint4 *>(xb + (int64_t)(q + 1) * C + c8)
                                        : uint4{0u, 0u, 0u, 0u};
                }
            }
        }
    };
    if ((int64_t)blockIdx.x < n) load_board(blockIdx.x);

    for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
        __syncthreads(); // the previous board's fragments are read
#pragma unroll
        for (int r = 0; r < DZ_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < DZ_ITEMS) {
                // channel 2cp: the low halves of the 8 cells, channel 2cp+1: the high halves
                uint32_t lo[4], hi[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    lo[d] = __builtin_amdgcn_perm(dzv[r][2 * d + 1], dzv[r][2 * d], 0x05040100u);
                    hi[d] = __builtin_amdgcn_perm(dzv[r][2 * d + 1], dzv[r][2 * d], 0x07060302u);
                }
                const int cp = j & 31, q0 = (j >> 5) * 8;
                *reinterpret_cast<uint4 *>(dzt + (2 * cp) * DS + q0) = uint4{lo[0], lo[1], lo[2], lo[3]};
                *reinterpret_cast<uint4 *>(dzt + (2 * cp + 1) * DS + q0) = uint4{hi[0], hi[1], hi[2], hi[3]};
            }
        }
#pragma unroll
        for (int r = 0; r < X_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < X_ITEMS) {
                if constexpr (CIN == 4) {
                    xt[0 * PPS + j] = (uint16_t)(xv[r].x & 0xFFFFu);
                    xt[1 * PPS + j] = (uint16_t)(xv[r].x >> 16);
                    xt[2 * PPS + j] = (uint16_t)(xv[r].y & 0xFFFFu);
                    xt[3 * PPS + j] = (uint16_t)(xv[r].y >> 16);
                } else {
                    // channel c0 + 2h: the low halves of both cells, c0 + 2h + 1: the high halves
                    const int q = 2 * (j >> 3), c0 = (j & 7) * 8;
                    const uint32_t a[4] = {xv[r].x, xv[r].y, xv[r].z, xv[r].w};
                    const uint32_t bq[4] = {xv2[r].x, xv2[r].y, xv2[r].z, xv2[r].w};
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        *reinterpret_cast<uint32_t *>(xt + (c0 + 2 * h) * PPS + q) =
                            __builtin_amdgcn_perm(bq[h], a[h], 0x05040100u);
                        *reinterpret_cast<uint32_t *>(xt + (c0 + 2 * h + 1) * PPS + q) =
                            __builtin_amdgcn_perm(bq[h], a[h], 0x07060302u);
                    }
                }
            }
        }
        __syncthreads();
        if (b + gridDim.x < n) load_board(b + gridDim.x); // in flight during the products
        for (int ks = 0; ks < PIXP / 32; ++ks) {
            const int p0 = ks * 32 + quad * 8; // this lane's 8 consecutive cells
            uint4 araw[4];
            bf16x8 afr[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                araw[mt] = *reinterpret_cast<const uint4 *>(dzt + (mt * 16 + row) * DS + p0);
                afr[mt] = as_bf16x8(araw[mt]);
            }
            if (wave == 0) {
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const uint32_t wd[4] = {araw[mt].x, araw[mt].y, araw[mt].z, araw[mt].w};
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        dsum[mt] += __uint_as_float(wd[h] << 16) + __uint_as_float(wd[h] & 0xFFFF0000u);
                }
            }
            int cq[8]; // top-left tap of each of the 8 cells in the padded frame
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int p = p0 + i < PIX ? p0 + i : 0;
                cq[i] = (p / N) * NP + p % N;
            }
            if constexpr (CIN == 64) {
                // this lane's channel row; tap t = j at a constant offset
                const uint16_t *xl[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) xl[i] = xt + (wave * 16 + row) * PPS + cq[i];
#pragma unroll
                for (int j = 0; j < NTW; ++j) {
                    const int off = (j / 3) * NP + (j % 3);
                    uint32_t u[4];
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        u[h] = (uint32_t)xl[2 * h][off] | ((uint32_t)xl[2 * h + 1][off] << 16);
                    const bf16x8 bfr = as_bf16x8(uint4{u[0], u[1], u[2], u[3]});
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mt], bfr, acc[mt][j], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int j = 0; j < NTW; ++j) {
                    if (wave * NTW + j >= NT) break;
                    const uint16_t *xrow = xt + col_ch[j] * PPS + col_off[j];
                    uint32_t u[4];
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        u[h] = (uint32_t)xrow[cq[2 * h]] | ((uint32_t)xrow[cq[2 * h + 1]] << 16);
                    const bf16x8 bfr = as_bf16x8(uint4{u[0], u[1], u[2], u[3]});
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mt], bfr, acc[mt][j], 0, 0, 0);
                }
            }
        }
    }
    float *o = part + (int64_t)blockIdx.x * PART;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        const int col = (wave * NTW + j) * 16 + row;
        if (wave * NTW + j >= NT || col >= NCOL) continue;
        // 64 channels: tile j of wave w is tap j, channels 16 w + row
        const int t = CIN == 64 ? j : col / CIN, i = CIN == 64 ? wave * 16 + row : col % CIN;
        if (i >= CR) continue;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = mt * 16 + quad * 4 + r;
                o[(co * CR + i) * 9 + t] = acc[mt][j][r];
            }
    }
    if (wave == 0) {
        // the four quads of a row held different cells of the same channel
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            dsum[mt] += __shfl_xor(dsum[mt], 16, 64);
            dsum[mt] += __shfl_xor(dsum[mt], 32, 64);
        }
        if (quad == 0) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) o[C * CR * 9 + mt * 16 + row] = dsum[mt];
        }
    }
}

// The same product for the 64-channel layers with the B operand read as
// whole fragments: both LDS frames use a row stride RS that is a multiple
// of 8 cells (dZ^T holds interior cell (r, c) at r * RS + c, X^T padded cell
// (r, c) at r * RS + c, zeros elsewhere), so K runs over dZ^T positions and
// the tap (tr, tc) of position q is X^T position q + tr * RS + tc.  The 16
// columns of a tile share one tap, so a lane's 8 B values are X^T positions
// q0 + off .. + 7 of its channel: two aligned 16-byte reads and a funnel
// shift by tc cells, instead of eight 2-byte gathers.  K grows from the
// cells padded to 32 to N * RS padded to 32 (the extra positions are
// zero in dZ^T).
template <int N>
__global__ __launch_bounds__(256) void k_conv_wgrad64(const uint16_t *__restrict__ dz, const uint16_t *__restrict__ x,
                                                      int64_t n, float *__restrict__ part)
{
    constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    constexpr int RS = (NP + 7) / 8 * 8;                      // frame row stride
    constexpr int KP = (N * RS + 31) / 32 * 32;               // dZ^T positions, whole k-steps
    constexpr int DS = KP + 8;                                // dZ^T row stride
    constexpr int XS = KP + 2 * RS + 16 + 8;                  // X^T row stride (reads reach KP + 2 RS + 10)
    constexpr int NCOL = 9 * C, NT = NCOL / 16, NTW = NT / 4; // 36 column tiles, 9 per wave
    constexpr int PART = C * C * 9 + C;
    constexpr int DZ_ITEMS = PIX * 8, DZ_R = (DZ_ITEMS + 255) / 256;
    constexpr int X_ITEMS = PP * 8, X_R = (X_ITEMS + 255) / 256;
    __shared__ __align__(16) uint16_t dzt[C * DS];
    __shared__ __align__(16) uint16_t xt[C * XS];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, quad = lane >> 4;
    f32x4 acc[4][NTW];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < NTW; ++j) acc[mt][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dsum[4] = {0.f, 0.f, 0.f, 0.f}; // wave 0: bias-gradient partial sums of channels mt*16 + row
    // every position that no board writes (frame padding, slack) stays zero
    for (int j = threadIdx.x; j < C * DS / 8; j += 256) reinterpret_cast<uint4 *>(dzt)[j] = uint4{0u, 0u, 0u, 0u};
    for (int j = threadIdx.x; j < C * XS / 8; j += 256) reinterpret_cast<uint4 *>(xt)[j] = uint4{0u, 0u, 0u, 0u};

    uint4 dzr[DZ_R], xr4[X_R];
    auto load_board = [&](int64_t b) {
        const uint16_t *db = dz + b * (int64_t)PP * C;
        const uint16_t *xb = x + b * (int64_t)PP * C;
#pragma unroll
        for (int r = 0; r < DZ_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < DZ_ITEMS) {
                const int q = j >> 3, c0 = (j & 7) * 8;
                dzr[r] = *reinterpret_cast<const uint4 *>(db + (int64_t)((q / N + 1) * NP + q % N + 1) * C + c0);
            }
        }
#pragma unroll
        for (int r = 0; r < X_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < X_ITEMS) xr4[r] = *reinterpret_cast<const uint4 *>(xb + (int64_t)(j >> 3) * C + (j & 7) * 8);
        }
    };
    if ((int64_t)blockIdx.x < n) load_board(blockIdx.x);

    for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
        __syncthreads(); // the zero fill, or the previous board's fragments, are done
#pragma unroll
        for (int r = 0; r < DZ_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < DZ_ITEMS) {
                const int q = j >> 3, c0 = (j & 7) * 8;
                const int pos = (q / N) * RS + q % N;
                const uint32_t wd[4] = {dzr[r].x, dzr[r].y, dzr[r].z, dzr[r].w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    dzt[(c0 + 2 * h) * DS + pos] = (uint16_t)(wd[h] & 0xFFFFu);
                    dzt[(c0 + 2 * h + 1) * DS + pos] = (uint16_t)(wd[h] >> 16);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < X_R; ++r) {
            const int j = threadIdx.x + 256 * r;
            if (j < X_ITEMS) {
                const int q = j >> 3, c0 = (j & 7) * 8;
                const int pos = (q / NP) * RS + q % NP;
                const uint32_t wd[4] = {xr4[r].x, xr4[r].y, xr4[r].z, xr4[r].w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    xt[(c0 + 2 * h) * XS + pos] = (uint16_t)(wd[h] & 0xFFFFu);
                    xt[(c0 + 2 * h + 1) * XS + pos] = (uint16_t)(wd[h] >> 16);
                }
            }
        }
        __syncthreads();
        if (b + gridDim.x < n) load_board(b + gridDim.x); // in flight during the products
        for (int ks = 0; ks < KP / 32; ++ks) {
            const int q0 = ks * 32 + quad * 8; // this lane's 8 consecutive positions
            uint4 araw[4];
            bf16x8 afr[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                araw[mt] = *reinterpret_cast<const uint4 *>(dzt + (mt * 16 + row) * DS + q0);
                afr[mt] = as_bf16x8(araw[mt]);
            }
            if (wave == 0) {
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const uint32_t wd[4] = {araw[mt].x, araw[mt].y, araw[mt].z, araw[mt].w};
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        dsum[mt] += __uint_as_float(wd[h] << 16) + __uint_as_float(wd[h] & 0xFFFF0000u);
                }
            }
#pragma unroll
            for (int j = 0; j < NTW; ++j) {
                const int tile = wave * NTW + j;     // columns tile*16 .. +15: tap t, channels
                const int t = tile >> 2;             // (tile & 3) * 16 .. +15
                const int tr = t / 3, tc = t - 3 * tr;
                const int base = ((tile & 3) * 16 + row) * XS + q0 + tr * RS; // 8-cell aligned
                const uint4 lo = *reinterpret_cast<const uint4 *>(xt + base);
                const uint4 hi = *reinterpret_cast<const uint4 *>(xt + base + 8);
                const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
                uint32_t u[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    // cells tc .. tc + 7 of the 16 read: dword d = cells tc + 2d, tc + 2d + 1
                    const uint32_t a0 = tc >= 2 ? w[d + 1] : w[d];
                    const uint32_t a1 = tc >= 2 ? w[d + 2] : w[d + 1];
                    u[d] = __builtin_amdgcn_alignbyte(a1, a0, (tc & 1) * 2);
                }
                const bf16x8 bfr = as_bf16x8(uint4{u[0], u[1], u[2], u[3]});
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mt], bfr, acc[mt][j], 0, 0, 0);
            }
        }
    }
    float *o = part + (int64_t)blockIdx.x * PART;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        const int col = (wave * NTW + j) * 16 + row;
        const int t = col / C, i = col % C;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = mt * 16 + quad * 4 + r;
                o[(co * C + i) * 9 + t] = acc[mt][j][r];
            }
    }
    if (wave == 0) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            dsum[mt] += __shfl_xor(dsum[mt], 16, 64);
            dsum[mt] += __shfl_xor(dsum[mt], 32, 64);
        }
        if (quad == 0) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) o[C * C * 9 + mt * 16 + row] = dsum[mt];
        }
    }
}

// out[j] = sum over rows r < rows of part[r * stride + j], j < cols: a block
// takes 32 columns, its 8 waves' worth of row groups add up in LDS
__global__ __launch_bounds__(256) void k_sum_rows(const float *__restrict__ part, int64_t rows, int stride, int cols,
                                                  float *__restrict__ out)
{
    __shared__ float red[8][32];
    const int cl = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int j = blockIdx.x * 32 + cl;
    float s = 0.f;
    if (j < cols)
        for (int64_t r = grp; r < rows; r += 64) { // 8 rows' loads in flight at a time
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = r + 8 * k < rows ? part[(r + 8 * k) * stride + j] : 0.f;
#pragma unroll
            for (int k = 0; k < 8; ++k) s += v[k];
        }
    red[grp][cl] = s;
    __syncthreads();
    if (grp == 0 && j < cols) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) t += red[k][cl];
        out[j] = t;
    }
}

// loss[j] = sum over rows r < n of terms[2 r + j], j = 0, 1 (one block)
__global__ __launch_bounds__(256) void k_sum_loss(const float *__restrict__ terms, int64_t n, float *__restrict__ loss)
{
    __shared__ float red[2][256];
    float a = 0.f, b = 0.f;
    for (int64_t r = threadIdx.x; r < n; r += 8 * 256) { // 8 pairs' loads in flight at a time
        float2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            v[k] = r + 256 * k < n ? reinterpret_cast<const float2 *>(terms)[r + 256 * k] : float2{0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a += v[k].x;
            b += v[k].y;
        }
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int k = 128; k >= 1; k >>= 1) {
        if (threadIdx.x < k) {
            red[0][threadIdx.x] += red[0][threadIdx.x + k];
            red[1][threadIdx.x] += red[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) loss[threadIdx.x] = red[threadIdx.x][0];
}

// value cutoff estimate for player 1
__global__ void k_estimate(const int8_t *__restrict__ status, const int8_t *__restrict__ winner,
                           const int8_t *__restrict__ to_move, const float *__restrict__ value, int64_t n,
                           float *__restrict__ est)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int st = status[i];
    float e = 0.f;
    if (st == 1) e = winner[i] == 1 ? 1.f : (winner[i] == 2 ? -1.f : 0.f);
    else if (st == 0) e = to_move[i] == 1 ? value[i] : -value[i];
    est[i] = e;
}

// Adam (Kingma & Ba) with bias correction, float32 master weights
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t np, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    p[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }
constexpr int WG_BLOCKS = 256;  // blocks of the conv weight-gradient reductions
// blocks of the first layer's weight gradient: its partial sums are small
// (64 x 27 + 64 floats) and its blocks light enough for two per CU, so more
// blocks (fewer boards each) keep more loads in flight; the partials still
// fit the 64-channel layers' buffer
constexpr int WG1_BLOCKS = 512;
static_assert((int64_t)WG1_BLOCKS * (C * 27 + C) <= (int64_t)WG_BLOCKS * (C * C * 9 + C), "partials");
constexpr int HW_BLOCKS = 1024; // blocks of the head weight-gradient reduction

int64_t blocks_min(int64_t n, int64_t cap) { return n < cap ? n : cap; }

struct Carve {
    char *base;
    int64_t off = 0;
    template <class T>
    T *take(int64_t bytes)
    {
        T *p = reinterpret_cast<T *>(base + off);
        off += align256(bytes);
        return p;
    }
};

template <int N>
struct Sizes {
    static constexpr int NP = N + 2, PP = NP * NP, PIX = N * N;
    static constexpr int64_t a0(int64_t n) { return n * PP * 8; }
    static constexpr int64_t act(int64_t n) { return n * PP * C * 2; }
    static constexpr int64_t forward_ws(int64_t n) { return align256(a0(n)) + 2 * align256(act(n)); }
    static constexpr int64_t train_ws(int64_t n)
    {
        return align256(a0(n)) + 6 * align256(act(n)) + 3 * align256(n * PIX * 4) + 3 * align256(n * 4) +
               align256(n * 8) + align256((int64_t)WG_BLOCKS * (C * C * 9 + C) * 4) +
               align256((int64_t)HW_BLOCKS * HEAD_PART * 4);
    }
};

template <int N>
hipError_t forward_t(const float *params, const uint16_t *packed, const int8_t *board, const int8_t *to_move,
                     int64_t n, float *logits, float *value, void *ws, hipStream_t s)
{
    using S = Sizes<N>;
    Carve cv{static_cast<char *>(ws)};
    cv.take<uint2>(S::a0(n)); // the input planes' share of the workspace (unused by the fused forward)
    uint16_t *ya = cv.take<uint16_t>(S::act(n));
    uint16_t *yb = cv.take<uint16_t>(S::act(n));
    using LC = LdsL<N>;
    using LR = LdsR<N>;
    const unsigned lb = (unsigned)((n + LC::BPB - 1) / LC::BPB);
    const unsigned rb = (unsigned)blocks_min((n + LR::BPB - 1) / LR::BPB, RES_BLOCKS);
    // Three kernels: layers 1 + 2 from the boards (layer 1's activations kept
    // in LDS), layer 3, layer 4 + the heads (layer 4's activations kept in
    // registers).  19x19: the weights-resident kernel (measured 9.8 against
    // 10.5 ms per 65536-board forward); 11x11: the per-group staging measured
    // faster (3.7 against 3.9 ms).
    const uint16_t *z = zero16(packed);
    const FwdArgs a1{board, to_move, packed + pf_off(1), params + b_off(1), nullptr, nullptr, nullptr, z, 0};
    const FwdArgs ah{nullptr, to_move, nullptr, nullptr, params, logits, value, z, 0};
    const FwdArgs a3{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, z, 0};
    if constexpr (N == 19) {
        hipLaunchKernelGGL((k_conv_res<N, 2>), dim3(rb), dim3(LR::THREADS), 0, s, (const uint16_t *)nullptr,
                           packed + pf_off(2), params + b_off(2), (const uint16_t *)nullptr, ya, n, a1);
        hipLaunchKernelGGL((k_conv_res<N, 0>), dim3(rb), dim3(LR::THREADS), 0, s, ya, packed + pf_off(3),
                           params + b_off(3), (const uint16_t *)nullptr, yb, n, a3);
        hipLaunchKernelGGL((k_conv_res<N, 3>), dim3(rb), dim3(LR::THREADS), 0, s, yb, packed + pf_off(4),
                           params + b_off(4), (const uint16_t *)nullptr, (uint16_t *)nullptr, n, ah);
    } else {
        hipLaunchKernelGGL((k_conv_lds<N, 2>), dim3(lb), dim3(LC::THREADS), 0, s, (const uint16_t *)nullptr,
                           packed + pf_off(2), params + b_off(2), (const uint16_t *)nullptr, ya, n, a1);
        hipLaunchKernelGGL((k_conv_lds<N, 0>), dim3(lb), dim3(LC::THREADS), 0, s, ya, packed + pf_off(3),
                           params + b_off(3), (const uint16_t *)nullptr, yb, n, a3);
        hipLaunchKernelGGL((k_conv_lds<N, 3>), dim3(lb), dim3(LC::THREADS), 0, s, yb, packed + pf_off(4),
                           params + b_off(4), (const uint16_t *)nullptr, (uint16_t *)nullptr, n, ah);
    }
    return hipGetLastError();
}

// One guided ply of every env: the forward's three kernels, the last one
// drawing and playing each env's policy ply from its logits on chip
// (k_conv_lds MODE 4); 11x11 only.
hipError_t guided_step_t(const float *params, const uint16_t *packed, const DevState &st, int kind, int64_t n,
                         int max_plies, uint64_t seed, int64_t gid_base, const int64_t *gid, int8_t *reward,
                         uint8_t *terminal, void *ws, hipStream_t s)
{
    constexpr int N = 11;
    using S = Sizes<N>;
    Carve cv{static_cast<char *>(ws)};
    cv.take<uint2>(S::a0(n));
    uint16_t *ya = cv.take<uint16_t>(S::act(n));
    uint16_t *yb = cv.take<uint16_t>(S::act(n));
    using LC = LdsL<N>;
    const unsigned lb = (unsigned)((n + LC::BPB - 1) / LC::BPB);
    const uint16_t *z = zero16(packed);
    const FwdArgs a1{st.board, st.to_move, packed + pf_off(1), params + b_off(1), nullptr, nullptr, nullptr, z, 0};
    const FwdArgs a3{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, z, 0};
    FwdArgs ah{st.board, st.to_move, nullptr, nullptr, params, nullptr, nullptr, z, 0};
    ah.st = st;
    ah.kind = kind;
    ah.max_plies = max_plies;
    ah.key0 = (uint32_t)seed;
    ah.key1 = (uint32_t)(seed >> 32);
    ah.gid_base = gid_base;
    ah.gid = gid;
    ah.reward = reward;
    ah.terminal = terminal;
    hipLaunchKernelGGL((k_conv_lds<N, 2>), dim3(lb), dim3(LC::THREADS), 0, s, (const uint16_t *)nullptr,
                       packed + pf_off(2), params + b_off(2), (const uint16_t *)nullptr, ya, n, a1);
    hipLaunchKernelGGL((k_conv_lds<N, 0>), dim3(lb), dim3(LC::THREADS), 0, s, ya, packed + pf_off(3),
                       params + b_off(3), (const uint16_t *)nullptr, yb, n, a3);
    hipLaunchKernelGGL((k_conv_lds<N, 4>), dim3(lb), dim3(LC::THREADS), 0, s, yb, packed + pf_off(4),
                       params + b_off(4), (const uint16_t *)nullptr, (uint16_t *)nullptr, n, ah);
    return hipGetLastError();
}

int cu_count()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

unsigned fused_grid(int64_t n)
{
    const int64_t groups = (n + Fused11::BPB - 1) / Fused11::BPB;
    const int64_t cap = (int64_t)cu_count() * FUSED_BLOCKS_PER_CU;
    return (unsigned)(groups < cap ? groups : cap);
}

// The 11x11 forward as one kernel (k_fwd11 MODE 0).
hipError_t forward_fused11(const float *params, const uint16_t *packed, const int8_t *board, const int8_t *to_move,
                           int64_t n, float *logits, float *value, hipStream_t s)
{
    FusedArgs fa{};
    fa.params = params;
    fa.packed = packed;
    fa.n = n;
    fa.board = board;
    fa.to_move = to_move;
    fa.logits = logits;
    fa.value = value;
    hipLaunchKernelGGL(k_fwd11<0>, dim3(fused_grid(n)), dim3(Fused11::THREADS), 0, s, fa);
    return hipGetLastError();
}

template <int N>
hipError_t loss_grad_t(const float *params, const uint16_t *packed, const int8_t *board, const int8_t *to_move,
                       const int16_t *action, const float *z, int64_t n, float beta, float *loss, float *grads,
                       void *ws, hipStream_t s)
{
    using S = Sizes<N>;
    constexpr int MT = (S::PIX + 15) / 16, NG = (MT + 7) / 8;
    Carve cv{static_cast<char *>(ws)};
    uint2 *a0 = cv.take<uint2>(S::a0(n));
    uint16_t *y[5];
    y[0] = reinterpret_cast<uint16_t *>(a0);
    for (int l = 1; l <= 4; ++l) y[l] = cv.take<uint16_t>(S::act(n));
    uint16_t *ga = cv.take<uint16_t>(S::act(n)), *gb = cv.take<uint16_t>(S::act(n));
    float *logits = cv.take<float>(n * S::PIX * 4);
    float *lframe = cv.take<float>(n * S::PIX * 4);
    float *dlog = cv.take<float>(n * S::PIX * 4);
    float *value = cv.take<float>(n * 4);
    float *du = cv.take<float>(n * 4);
    cv.take<float>(n * 4);
    float *lterms = cv.take<float>(n * 8);
    float *part = cv.take<float>((int64_t)WG_BLOCKS * (C * C * 9 + C) * 4);
    float *hpart = cv.take<float>((int64_t)HW_BLOCKS * HEAD_PART * 4);

    const unsigned eb = (unsigned)((n * S::PP + 255) / 256), cb = (unsigned)((n * NG + 3) / 4),
                   hb = (unsigned)((n + 3) / 4);
    const unsigned wb = (unsigned)blocks_min(n, WG_BLOCKS);
    hipLaunchKernelGGL(k_encode<N>, dim3(eb), dim3(256), 0, s, board, to_move, n, a0);
    hipLaunchKernelGGL((k_conv<N, 4, 0>), dim3(cb), dim3(256), 0, s, y[0], packed + pf_off(1), params + b_off(1),
                       (const uint16_t *)nullptr, y[1], n);
    using LC = LdsL<N>;
    using LR = LdsR<N>;
    const unsigned lb = (unsigned)((n + LC::BPB - 1) / LC::BPB);
    const unsigned rb = (unsigned)blocks_min((n + LR::BPB - 1) / LR::BPB, RES_BLOCKS);
    // forward layers write their rings (the weight gradients read them); the
    // data gradients' rings are never read from memory
    const FwdArgs fr{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, zero16(packed), 1};
    const FwdArgs fd{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, zero16(packed), 0};
    for (int l = 2; l <= 4; ++l) {
        if constexpr (N == 19)
            hipLaunchKernelGGL((k_conv_res<N, 0>), dim3(rb), dim3(LR::THREADS), 0, s, y[l - 1], packed + pf_off(l),
                               params + b_off(l), (const uint16_t *)nullptr, y[l], n, fr);
        else
            hipLaunchKernelGGL((k_conv_lds<N, 0>), dim3(lb), dim3(LC::THREADS), 0, s, y[l - 1], packed + pf_off(l),
                               params + b_off(l), (const uint16_t *)nullptr, y[l], n, fr);
    }
    hipLaunchKernelGGL(k_heads<N>, dim3(hb), dim3(256), 0, s, y[4], params, to_move, n, logits, lframe, value);
    hipLaunchKernelGGL(k_heads_bwd<N>, dim3(hb), dim3(256), 0, s, y[4], a0, params, lframe, value, to_move,
                       action, z, n, beta, 1.f / (float)n, dlog, du, lterms, ga);
    const unsigned hwb = (unsigned)blocks_min((n + 3) / 4, HW_BLOCKS);
    hipLaunchKernelGGL(k_head_wgrad<N>, dim3(hwb), dim3(256), 0, s, y[4], dlog, du, n, hpart);
    hipLaunchKernelGGL(k_sum_rows, dim3((HEAD_PART + 31) / 32), dim3(256), 0, s, hpart, (int64_t)hwb, HEAD_PART,
                       HEAD_PART, grads + WP_OFF);
    constexpr int PART64 = C * C * 9 + C, PART4 = C * 27 + C;
    for (int l = 4; l >= 2; --l) {
        // 19x19: aligned B fragments (K = 19 x 24 positions padded to 480
        // against 361 cells padded to 384); 11x11: the 2-byte gathers win,
        // since its K would grow by half (176 positions padded to 192
        // against 121 cells padded to 128)
        if constexpr (N == 19)
            hipLaunchKernelGGL((k_conv_wgrad64<N>), dim3(wb), dim3(256), 0, s, ga, y[l - 1], n, part);
        else
            hipLaunchKernelGGL((k_conv_wgrad<N, 64>), dim3(wb), dim3(256), 0, s, ga, y[l - 1], n, part);
        hipLaunchKernelGGL(k_sum_rows, dim3((PART64 + 31) / 32), dim3(256), 0, s, part, (int64_t)wb, PART64,
                           PART64, grads + w_off(l));
        hipLaunchKernelGGL((k_conv_lds<N, 1>), dim3(lb), dim3(LC::THREADS), 0, s, ga, packed + pb_off(l),
                           (const float *)nullptr, y[l - 1], gb, n, fd);
        uint16_t *t = ga;
        ga = gb;
        gb = t;
    }
    const unsigned wb1 = (unsigned)blocks_min(n, WG1_BLOCKS);
    hipLaunchKernelGGL((k_conv_wgrad<N, 4>), dim3(wb1), dim3(256), 0, s, ga, y[0], n, part);
    hipLaunchKernelGGL(k_sum_rows, dim3((PART4 + 31) / 32), dim3(256), 0, s, part, (int64_t)wb1, PART4, PART4,
                       grads + w_off(1));
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, lterms, n, loss);
    return hipGetLastError();
}

} // namespace
} // namespace net

int64_t net_n_params() { return net::N_PARAMS; }
int64_t net_packed_bytes() { return net::PACKED_ELEMS * 2; }
bool net_size_supported(int N) { return N == 11 || N == 19; }

int64_t net_forward_ws_bytes(int N, int64_t n)
{
    // the forward's buffers, then the logits and values of ludax_net_estimate
    const int64_t f = N == 11 ? net::Sizes<11>::forward_ws(n) : net::Sizes<19>::forward_ws(n);
    return f + net::align256(n * N * N * 4) + net::align256(n * 4);
}
int64_t net_train_ws_bytes(int N, int64_t n)
{
    return N == 11 ? net::Sizes<11>::train_ws(n) : net::Sizes<19>::train_ws(n);
}

hipError_t net_pack(const float *params, void *packed, hipStream_t s)
{
    hipLaunchKernelGGL(net::k_pack, dim3(256), dim3(256), 0, s, params, static_cast<uint16_t *>(packed));
    return hipGetLastError();
}

// 11x11: the one-kernel forward (activations on chip; the same products in
// the same order as the three-kernel forward, so the same logits and
// values); 19x19: the three kernels with the weights resident.
hipError_t net_forward(int N, const float *params, const void *packed, const int8_t *board, const int8_t *to_move,
                       int64_t n, float *logits, float *value, void *ws, hipStream_t s)
{
    const uint16_t *pk = static_cast<const uint16_t *>(packed);
    return N == 11 ? net::forward_fused11(params, pk, board, to_move, n, logits, value, s)
                   : net::forward_t<19>(params, pk, board, to_move, n, logits, value, ws, s);
}

hipError_t net_loss_grad(int N, const float *params, const void *packed, const int8_t *board,
                         const int8_t *to_move, const int16_t *action, const float *z, int64_t n, float beta,
                         float *loss, float *grads, void *ws, hipStream_t s)
{
    const uint16_t *pk = static_cast<const uint16_t *>(packed);
    return N == 11 ? net::loss_grad_t<11>(params, pk, board, to_move, action, z, n, beta, loss, grads, ws, s)
                   : net::loss_grad_t<19>(params, pk, board, to_move, action, z, n, beta, loss, grads, ws, s);
}

hipError_t net_guided_step(int N, const float *params, const void *packed, const DevState &st, int kind, int64_t n,
                           int max_plies, uint64_t seed, int64_t gid_base, const int64_t *gid, int8_t *reward,
                           uint8_t *terminal, void *ws, hipStream_t s)
{
    if (N != 11) return hipErrorInvalidValue;
    return net::guided_step_t(params, static_cast<const uint16_t *>(packed), st, kind, n, max_plies, seed, gid_base,
                              gid, reward, terminal, ws, s);
}

hipError_t net_guided_playout(const float *params, const void *packed, const DevState &st, int kind, int64_t n,
                              int max_plies, int plies, uint64_t seed, int64_t gid_base, const int64_t *gid,
                              float *estimate, hipStream_t s)
{
    net::FusedArgs fa{};
    fa.params = params;
    fa.packed = static_cast<const uint16_t *>(packed);
    fa.n = n;
    fa.st = st;
    fa.kind = kind;
    fa.max_plies = max_plies;
    fa.plies = plies;
    fa.key0 = (uint32_t)seed;
    fa.key1 = (uint32_t)(seed >> 32);
    fa.gid_base = gid_base;
    fa.gid = gid;
    fa.estimate = estimate;
    hipLaunchKernelGGL(net::k_fwd11<1>, dim3(net::fused_grid(n)), dim3(net::Fused11::THREADS), 0, s, fa);
    return hipGetLastError();
}

hipError_t net_estimate(int N, const float *params, const void *packed, const DevState &st, int64_t n,
                        float *estimate, void *ws, hipStream_t s)
{
    // 11x11: the guided playout kernel with no plies (value cutoff only,
    // nothing but the estimates written)
    if (N == 11) return net_guided_playout(params, packed, st, 3, n, 1, 0, 0, 0, nullptr, estimate, s);
    const int64_t f = N == 11 ? net::Sizes<11>::forward_ws(n) : net::Sizes<19>::forward_ws(n);
    float *logits = reinterpret_cast<float *>(static_cast<char *>(ws) + f);
    float *value = reinterpret_cast<float *>(static_cast<char *>(ws) + f + net::align256(n * N * N * 4));
    hipError_t e = net_forward(N, params, packed, st.board, st.to_move, n, logits, value, ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(net::k_estimate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, st.status, st.winner,
                       st.to_move, value, n, estimate);
    return hipGetLastError();
}

hipError_t net_adam(float *params, const float *grads, float *m, float *v, int step, float lr, float b1, float b2,
                    float eps, void *packed, hipStream_t s)
{
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(net::k_adam, dim3((unsigned)((net::N_PARAMS + 255) / 256)), dim3(256), 0, s, params, grads,
                       m, v, net::N_PARAMS, lr, b1, b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || packed == nullptr) return e;
    return net_pack(params, packed, s);
}

} // namespace lx
