// stats.hip -- the step and outcome counters of ludax_playout.
//
// Launched before (sign -1) and after (sign +1) a playout on the same
// stream: an env that was not RUNNING is unchanged by the playout and
// cancels out, so the difference counts the plies applied and the games
// ended by the playout.  Each thread reads 16 envs with 16-byte loads
// (all four loads in flight at once), a block reduces through wave
// shuffles and LDS, and adds its totals with four atomics; few blocks keep
// same-address atomics rare.
#include <algorithm>

#include "ludax_internal.hpp"

namespace lx {

namespace {

constexpr int SB = 256;      // threads per block
constexpr int PER = 16;      // envs per thread per pass
constexpr int TERMINAL_STATUS = 1;

__device__ __forceinline__ void tally(int st, int w, int &w1, int &w2, int &d)
{
    const bool term = st == TERMINAL_STATUS;
    w1 += term && w == 1;
    w2 += term && w == 2;
    d += term && w == 0;
}

// The counters of envs [0, n) (the first nvec groups of 16 by vector loads),
// this block's share of them for blocks blockIdx.x of gridDim.x.
__device__ __forceinline__ void stats_block(const int8_t *__restrict__ status, const int8_t *__restrict__ winner,
                                            const int16_t *__restrict__ ply, int64_t n, int64_t nvec, int sign,
                                            unsigned long long *__restrict__ stats)
{
    int64_t s = 0;
    int w1 = 0, w2 = 0, d = 0;
    const int64_t stride = (int64_t)gridDim.x * SB;
    // vector part: groups of 16 envs (pointers are 16-byte aligned when nvec > 0)
    for (int64_t g = (int64_t)blockIdx.x * SB + threadIdx.x; g < nvec; g += stride) {
        const uint4 sv = reinterpret_cast<const uint4 *>(status)[g];
        const uint4 wv = reinterpret_cast<const uint4 *>(winner)[g];
        const uint4 p0 = reinterpret_cast<const uint4 *>(ply)[2 * g];
        const uint4 p1 = reinterpret_cast<const uint4 *>(ply)[2 * g + 1];
        const uint32_t sw[4] = {sv.x, sv.y, sv.z, sv.w};
        const uint32_t ww[4] = {wv.x, wv.y, wv.z, wv.w};
        const uint32_t pw[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) s += (int16_t)(pw[k] & 0xFFFFu) + (int16_t)(pw[k] >> 16);
#pragma unroll
        for (int k = 0; k < 16; ++k)
            tally((int8_t)(sw[k >> 2] >> (8 * (k & 3))), (int8_t)(ww[k >> 2] >> (8 * (k & 3))), w1, w2, d);
    }
    // scalar tail
    for (int64_t i = nvec * PER + (int64_t)blockIdx.x * SB + threadIdx.x; i < n; i += stride) {
        s += ply[i];
        tally(status[i], winner[i], w1, w2, d);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        w1 += __shfl_xor(w1, o, 64);
        w2 += __shfl_xor(w2, o, 64);
        d += __shfl_xor(d, o, 64);
    }
    __shared__ long long part[SB / 64][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        part[wv][0] = s;
        part[wv][1] = w1;
        part[wv][2] = w2;
        part[wv][3] = d;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        long long v = 0;
#pragma unroll
        for (int k = 0; k < SB / 64; ++k) v += part[k][threadIdx.x];
        if (v != 0) atomicAdd(&stats[threadIdx.x], (unsigned long long)(sign * v));
    }
}

__global__ __launch_bounds__(SB) void k_stats(const int8_t *__restrict__ status,
                                              const int8_t *__restrict__ winner,
                                              const int16_t *__restrict__ ply, int64_t n, int64_t nvec,
                                              int sign, unsigned long long *__restrict__ stats)
{
    stats_block(status, winner, ply, n, nvec, sign, stats);
}

struct StatsGroup {
    const int8_t *status[GROUP_MAX];
    const int8_t *winner[GROUP_MAX];
    const int16_t *ply[GROUP_MAX];
    int64_t n[GROUP_MAX], nvec[GROUP_MAX];
    unsigned long long *stats[GROUP_MAX];
};

// blockIdx.y = the batch (a launch holds only batches with counters)
__global__ __launch_bounds__(SB) void k_stats_group(StatsGroup g, int sign)
{
    const int k = blockIdx.y;
    // constant-index selects keep the arguments in scalar registers
    const int8_t *status = g.status[0], *winner = g.winner[0];
    const int16_t *ply = g.ply[0];
    int64_t n = g.n[0], nvec = g.nvec[0];
    unsigned long long *stats = g.stats[0];
#pragma unroll
    for (int j = 1; j < GROUP_MAX; ++j)
        if (k == j) {
            status = g.status[j];
            winner = g.winner[j];
            ply = g.ply[j];
            n = g.n[j];
            nvec = g.nvec[j];
            stats = g.stats[j];
        }
    stats_block(status, winner, ply, n, nvec, sign, stats);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int64_t stats_blocks(int64_t work)
{
    int64_t blocks = (work + SB - 1) / SB;
    if (blocks < 1) blocks = 1;
    if (blocks > 128) blocks = 128;
    return blocks;
}

} // namespace

hipError_t launch_stats(const DevState &st, int64_t n, int sign, int64_t *stats, hipStream_t s)
{
    const bool vec = aligned16(st.status) && aligned16(st.winner) && aligned16(st.ply);
    const int64_t nvec = vec ? n / PER : 0;
    // one group of 16 envs per thread (latency, not bandwidth, is the
    // cost here), at most 128 blocks so that atomics stay few
    const int64_t blocks = stats_blocks(nvec > 0 ? nvec : n);
    hipLaunchKernelGGL(k_stats, dim3((unsigned)blocks), dim3(SB), 0, s, st.status, st.winner, st.ply, n,
                       nvec, sign, reinterpret_cast<unsigned long long *>(stats));
    return hipGetLastError();
}

hipError_t launch_stats_group(const DevState *st, const int64_t *n, int nb, int sign, int64_t *const *stats,
                              hipStream_t s)
{
    if (nb > GROUP_MAX) return hipErrorInvalidValue;
    StatsGroup g = {};
    int m = 0;
    int64_t blocks = 1;
    for (int k = 0; k < nb; ++k) {
        if (stats[k] == nullptr || n[k] <= 0) continue;
        const bool vec = aligned16(st[k].status) && aligned16(st[k].winner) && aligned16(st[k].ply);
        g.status[m] = st[k].status;
        g.winner[m] = st[k].winner;
        g.ply[m] = st[k].ply;
        g.n[m] = n[k];
        g.nvec[m] = vec ? n[k] / PER : 0;
        g.stats[m] = reinterpret_cast<unsigned long long *>(stats[k]);
        blocks = std::max<int64_t>(blocks, stats_blocks(g.nvec[m] > 0 ? g.nvec[m] : n[k]));
        ++m;
    }
    if (m == 0) return hipSuccess;
    // a block past a smaller batch's share finds no envs and adds nothing
    hipLaunchKernelGGL(k_stats_group, dim3((unsigned)blocks, (unsigned)m), dim3(SB), 0, s, g, sign);
    return hipGetLastError();
}

namespace {

// Zero the queue counters (a kernel, not a memset, so that a captured
// graph can replay it).
__global__ void k_zero_counters(unsigned int *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

// Per-kind counters of a mixed batch: block (x, k) reduces the games of
// kind k, i.e. the global indices j with (id_base + j) mod n_kinds == k.
__global__ __launch_bounds__(SB) void k_mixed_stats(const int8_t *__restrict__ winner,
                                                    const int16_t *__restrict__ plies, int64_t n_games,
                                                    int64_t id_base, int n_kinds,
                                                    unsigned long long *__restrict__ stats)
{
    const int k = blockIdx.y;
    const int64_t j0 = ((int64_t)k - id_base % n_kinds + n_kinds) % n_kinds;
    int64_t s = 0;
    int w1 = 0, w2 = 0, d = 0;
    for (int64_t j = j0 + ((int64_t)blockIdx.x * SB + threadIdx.x) * n_kinds; j < n_games;
         j += (int64_t)gridDim.x * SB * n_kinds) {
        s += plies[j];
        const int w = winner[j];
        w1 += w == 1;
        w2 += w == 2;
        d += w == 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        w1 += __shfl_xor(w1, o, 64);
        w2 += __shfl_xor(w2, o, 64);
        d += __shfl_xor(d, o, 64);
    }
    __shared__ long long part[SB / 64][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        part[wv][0] = s;
        part[wv][1] = w1;
        part[wv][2] = w2;
        part[wv][3] = d;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        long long v = 0;
#pragma unroll
        for (int q = 0; q < SB / 64; ++q) v += part[q][threadIdx.x];
        if (v != 0) atomicAdd(&stats[4 * k + threadIdx.x], (unsigned long long)v);
    }
}

} // namespace

hipError_t launch_zero_counters(unsigned int *c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, c, n);
    return hipGetLastError();
}

hipError_t launch_mixed_stats(const int8_t *winner, const int16_t *plies, int64_t n_games, int64_t id_base,
                              int n_kinds, int64_t *stats, hipStream_t s)
{
    const int64_t per_kind = (n_games + n_kinds - 1) / n_kinds;
    int64_t blocks = (per_kind + 4 * SB - 1) / (4 * SB);
    if (blocks < 1) blocks = 1;
    if (blocks > 128) blocks = 128;
    hipLaunchKernelGGL(k_mixed_stats, dim3((unsigned)blocks, (unsigned)n_kinds), dim3(SB), 0, s, winner, plies,
                       n_games, id_base, n_kinds, reinterpret_cast<unsigned long long *>(stats));
    return hipGetLastError();
}

} // namespace lx
