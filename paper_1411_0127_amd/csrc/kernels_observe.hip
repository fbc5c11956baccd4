// Observable kernels of libsg (gfx950): per-sample counts over bit-packed words.
//   unsatisfied bonds: bit j of J[d][i] ^ S[i] ^ S[i + d^] is 1 when bond (i, i+d^)
//   of sample j is unsatisfied (Sec. 4, bond bit e_ik); the energy of Eq. (1) is
//   E_j = 2 U_j - 3V;
//   replica difference: bit j of A[i] ^ B[i].
// Each thread adds its words into a bit-sliced ("vertical") count per sample --
// plane b holds bit b of 64 per-sample counts, kept as two 32-sample halves --
// then the block turns the planes into 64 integers and writes one row of partial
// sums; a second kernel adds the rows.  No atomics, so the result is
// deterministic.
//
// The count has two levels: a 4-plane counter takes the words of a few sites (at
// most 15 ones per sample) and is added into the 16-plane total only when full,
// so a word costs a short carry chain instead of a 16-plane one.  The bond count
// walks each thread's (x, y) column up z, so the +z neighbour word read for one
// site is the spin word of the next, and coordinates are found once per column.
#include <algorithm>

#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kThreads = 256;
constexpr int kPlanes = 16;  // a thread may add at most 2^16 - 1 ones per sample
constexpr int kLowMax = 15;  // ones per sample the 4-plane counter holds

struct Count2 {
    uint32_t lo[2][4];
    uint32_t tot[2][kPlanes];
    int held;  // ones per sample lo may hold (an upper bound)

    __device__ void clear()
    {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                lo[h][b] = 0;
#pragma unroll
            for (int b = 0; b < kPlanes; ++b)
                tot[h][b] = 0;
        }
        held = 0;
    }
    // lo into tot (ripple-carry add of a 4-bit vertical number), lo cleared
    __device__ void spill()
    {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t c = tot[h][0] & lo[h][0];
            tot[h][0] ^= lo[h][0];
#pragma unroll
            for (int b = 1; b < 4; ++b) {
                const uint32_t t = bop3<bop::kXor3>(tot[h][b], lo[h][b], c);
                c = bop3<bop::kMaj>(tot[h][b], lo[h][b], c);
                tot[h][b] = t;
            }
#pragma unroll
            for (int b = 4; b < kPlanes; ++b) {
                const uint32_t t = tot[h][b] & c;
                tot[h][b] ^= c;
                c = t;
            }
#pragma unroll
            for (int b = 0; b < 4; ++b)
                lo[h][b] = 0;
        }
        held = 0;
    }
    // one word: bit j adds 1 to sample j
    __device__ void add1(uint64_t w)
    {
        if (held + 1 > kLowMax)
            spill();
        const uint32_t v[2] = {(uint32_t)w, (uint32_t)(w >> 32)};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t c = v[h];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const uint32_t t = lo[h][b] & c;
                lo[h][b] ^= c;
                c = t;
            }
            lo[h][3] ^= c;
        }
        held += 1;
    }
    // three words: bit j of each adds 1 to sample j (a full adder first)
    __device__ void add3(uint64_t a, uint64_t b, uint64_t c)
    {
        if (held + 3 > kLowMax)
            spill();
        const uint32_t va[2] = {(uint32_t)a, (uint32_t)(a >> 32)};
        const uint32_t vb[2] = {(uint32_t)b, (uint32_t)(b >> 32)};
        const uint32_t vc[2] = {(uint32_t)c, (uint32_t)(c >> 32)};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t b0 = bop3<bop::kXor3>(va[h], vb[h], vc[h]);  // weight 1
            const uint32_t b1 = bop3<bop::kMaj>(va[h], vb[h], vc[h]);   // weight 2
            const uint32_t k0 = lo[h][0] & b0;
            lo[h][0] ^= b0;
            const uint32_t n1 = bop3<bop::kXor3>(lo[h][1], b1, k0);
            const uint32_t k1 = bop3<bop::kMaj>(lo[h][1], b1, k0);
            lo[h][1] = n1;
            const uint32_t k2 = lo[h][2] & k1;
            lo[h][2] ^= k1;
            lo[h][3] ^= k2;
        }
        held += 3;
    }
};

// Move the 64 counts of every thread of the block into partials[blockIdx.x][0..63],
// 32 samples at a time to keep the table within 33 KB of LDS.
__device__ void block_flush(Count2 &vc, uint64_t *__restrict__ partials)
{
    __shared__ uint32_t tab[32][kThreads + 1];
    vc.spill();
    const int tid = threadIdx.x;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll 4
        for (int jj = 0; jj < 32; ++jj) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < kPlanes; ++b)
                v |= ((vc.tot[half][b] >> jj) & 1u) << b;
            tab[jj][tid] = v;
        }
        __syncthreads();
        if (tid < 32) {
            uint64_t s = 0;
            for (int k = 0; k < kThreads; ++k)
                s += tab[tid][k];
            partials[(size_t)blockIdx.x * 64 + half * 32 + tid] = s;
        }
        __syncthreads();
    }
}

// Work item = one (x, y) column over one z range of zc planes; items are numbered
// x fastest, so a wave reads consecutive words of a row.
__global__ __launch_bounds__(kThreads) void k_count_unsat(const uint64_t *__restrict__ S,
                                                          const uint64_t *__restrict__ J, int L, int zc, int nzc,
                                                          uint64_t *__restrict__ partials)
{
    const int64_t LL = (int64_t)L * L;
    const int64_t Vj = coupling_stride(L);
    const int64_t items = LL * nzc;
    Count2 vc;
    vc.clear();
    for (int64_t it = blockIdx.x * (int64_t)kThreads + threadIdx.x; it < items; it += (int64_t)gridDim.x * kThreads) {
        const int64_t col = it % LL;
        const int z0 = (int)(it / LL) * zc;
        const int z1 = min(L, z0 + zc);
        const int y = (int)(col / L);
        const int x = (int)(col - (int64_t)y * L);
        const int64_t dx = (x + 1 == L) ? -(int64_t)(L - 1) : 1;
        const int64_t dy = (y + 1 == L) ? -(int64_t)(L - 1) * L : (int64_t)L;
        int64_t i = (int64_t)z0 * LL + col;
        uint64_t s = S[i];
#pragma unroll 4
        for (int z = z0; z < z1; ++z, i += LL) {
            // bond (i, i + d) of sample j is unsatisfied when bit j of J[d][i] ^ s_i ^ s_{i+d} is 1
            const uint64_t sz = S[(z + 1 == L) ? col : i + LL];
            const uint64_t wx = J[i] ^ s ^ S[i + dx];
            const uint64_t wy = J[Vj + i] ^ s ^ S[i + dy];
            const uint64_t wz = J[2 * Vj + i] ^ s ^ sz;
            vc.add3(wx, wy, wz);
            s = sz;
        }
    }
    block_flush(vc, partials);
}

__global__ __launch_bounds__(kThreads) void k_count_diff(const uint64_t *__restrict__ A,
                                                         const uint64_t *__restrict__ B, int64_t V,
                                                         uint64_t *__restrict__ partials)
{
    Count2 vc;
    vc.clear();
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < V; i += (int64_t)gridDim.x * kThreads)
        vc.add1(A[i] ^ B[i]);
    block_flush(vc, partials);
}

__global__ __launch_bounds__(1024) void k_reduce_partials(const uint64_t *__restrict__ partials, int nblocks,
                                                          uint64_t *__restrict__ out)
{
    __shared__ uint64_t part[16][64];
    const int j = threadIdx.x & 63;
    const int q = threadIdx.x >> 6;
    uint64_t s = 0;
#pragma unroll 8
    for (int b = q; b < nblocks; b += 16)
        s += partials[(size_t)b * 64 + j];
    part[q][j] = s;
    __syncthreads();
    if (q == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            t += part[k][j];
        out[j] = t;
    }
}

int blocks_for(int64_t words_per_site, int64_t V)
{
    // enough threads that no thread adds more than 2^16 - 1 words
    const int64_t max_sites = ((1 << kPlanes) - 1) / words_per_site;
    int64_t nb = (V + (int64_t)kThreads * 64 - 1) / ((int64_t)kThreads * 64);
    const int64_t need = (V + (int64_t)kThreads * max_sites - 1) / ((int64_t)kThreads * max_sites);
    if (nb < need)
        nb = need;
    if (nb > kMaxReduceBlocks)
        nb = kMaxReduceBlocks;
    if (nb < 1)
        nb = 1;
    return (int)nb;
}

}  // namespace

// Shape of the bond count with at most max_blocks blocks: a thread for every 16
// sites (short walks, for latency at small sides), at most max_blocks blocks; z range per work item
// (whole columns where one plane has an item for every thread, shorter ranges
// below that), items and blocks; false if a thread would add more than 2^16 - 1
// ones per sample.
static bool unsat_shape(int L, int max_blocks, int &zc, int &nzc, int &nblocks)
{
    const int64_t LL = (int64_t)L * L;
    const int64_t want = std::min<int64_t>((int64_t)max_blocks * kThreads, (LL * L + 15) / 16);
    const int64_t n = std::min<int64_t>(L, std::max<int64_t>(1, (want + LL - 1) / LL));
    zc = (int)((L + n - 1) / n);
    nzc = (L + zc - 1) / zc;
    const int64_t items = LL * nzc;
    nblocks = (int)std::min<int64_t>(max_blocks, (items + kThreads - 1) / kThreads);
    const int64_t per_thread = (items + (int64_t)nblocks * kThreads - 1) / ((int64_t)nblocks * kThreads);
    return 3 * (int64_t)zc * per_thread <= (1 << kPlanes) - 1;
}

hipError_t launch_count_unsat(const uint64_t *S, const uint64_t *J, int L, uint64_t *partials, int &nblocks,
                              hipStream_t s)
{
    if (L < 2)
        return hipErrorInvalidValue;
    // half the reduction rows where the count fits them (one resident round of
    // blocks; the rest of the reduction area then holds the totals of many sweeps),
    // all of them for the largest sides
    int zc = 0, nzc = 0;
    if (!unsat_shape(L, kMaxReduceBlocks / 2, zc, nzc, nblocks) && !unsat_shape(L, kMaxReduceBlocks, zc, nzc, nblocks))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_count_unsat, dim3(nblocks), dim3(kThreads), 0, s, S, J, L, zc, nzc, partials);
    return hipGetLastError();
}

hipError_t launch_count_diff(const uint64_t *A, const uint64_t *B, int64_t V, uint64_t *partials, int &nblocks,
                             hipStream_t s)
{
    nblocks = blocks_for(1, V);
    if ((int64_t)nblocks * kThreads * ((1 << kPlanes) - 1) < V)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_count_diff, dim3(nblocks), dim3(kThreads), 0, s, A, B, V, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const uint64_t *partials, int nblocks, uint64_t *out64, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, s, partials, nblocks, out64);
    return hipGetLastError();
}

}  // namespace sg
