// Observable kernels of libsg (gfx950): per-sample counts over bit-packed words.
//   unsatisfied bonds: bit j of J[d][i] ^ S[i] ^ S[i + d^] is 1 when bond (i, i+d^)
//   of sample j is unsatisfied (Sec. 4, bond bit e_ik); the energy of Eq. (1) is
//   E_j = 2 U_j - 3V;
//   replica difference: bit j of A[i] ^ B[i].
// Each thread adds its words into a 16-plane bit-sliced ("vertical") counter --
// plane b holds bit b of 64 per-sample counts -- then the block turns the planes
// into 64 integers and writes one row of partial sums; a second kernel adds the
// rows.  No atomics, so the result is deterministic.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kThreads = 256;
constexpr int kPlanes = 16;  // a thread may add at most 2^16 - 1 words

struct VCounter {
    uint64_t c[kPlanes];
    __device__ void clear()
    {
#pragma unroll
        for (int b = 0; b < kPlanes; ++b)
            c[b] = 0;
    }
    __device__ void add(uint64_t w)
    {
#pragma unroll
        for (int b = 0; b < kPlanes; ++b) {
            const uint64_t k = c[b] & w;
            c[b] ^= w;
            w = k;
        }
    }
};

// Move the 64 counts of every thread of the block into partials[blockIdx.x][0..63],
// 32 samples at a time to keep the table within 33 KB of LDS.
__device__ void block_flush(const VCounter &vc, uint64_t *__restrict__ partials)
{
    __shared__ uint32_t tab[32][kThreads + 1];
    const int tid = threadIdx.x;
    for (int half = 0; half < 2; ++half) {
#pragma unroll 4
        for (int jj = 0; jj < 32; ++jj) {
            const int j = half * 32 + jj;
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < kPlanes; ++b)
                v |= (uint32_t)((vc.c[b] >> j) & 1ull) << b;
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

__global__ __launch_bounds__(kThreads) void k_count_unsat(const uint64_t *__restrict__ S,
                                                          const uint64_t *__restrict__ J, int L,
                                                          uint64_t *__restrict__ partials)
{
    const int64_t V = (int64_t)L * L * L;
    const int64_t Vj = coupling_stride(L);
    const int64_t LL = (int64_t)L * L;
    VCounter vc;
    vc.clear();
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < V; i += (int64_t)gridDim.x * kThreads) {
        const int x = (int)(i % L);
        const int y = (int)((i / L) % L);
        const int64_t z = i / LL;
        const uint64_t s = S[i];
        const int64_t ix = (x + 1 == L) ? i - (L - 1) : i + 1;
        const int64_t iy = (y + 1 == L) ? i - (int64_t)(L - 1) * L : i + L;
        const int64_t iz = (z + 1 == L) ? i - (V - LL) : i + LL;
        vc.add(J[i] ^ s ^ S[ix]);
        vc.add(J[Vj + i] ^ s ^ S[iy]);
        vc.add(J[2 * Vj + i] ^ s ^ S[iz]);
    }
    block_flush(vc, partials);
}

__global__ __launch_bounds__(kThreads) void k_count_diff(const uint64_t *__restrict__ A,
                                                         const uint64_t *__restrict__ B, int64_t V,
                                                         uint64_t *__restrict__ partials)
{
    VCounter vc;
    vc.clear();
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < V; i += (int64_t)gridDim.x * kThreads)
        vc.add(A[i] ^ B[i]);
    block_flush(vc, partials);
}

// Sum the per-block rows: 16 threads per sample each add every 16th row, then
// the 16 partial sums of a sample are added in LDS.
__global__ __launch_bounds__(1024) void k_reduce_partials(const uint64_t *__restrict__ partials, int nblocks,
                                                          uint64_t *__restrict__ out)
{
    __shared__ uint64_t part[16][64];
    const int j = threadIdx.x & 63;
    const int q = threadIdx.x >> 6;
    uint64_t s = 0;
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

hipError_t launch_count_unsat(const uint64_t *S, const uint64_t *J, int L, uint64_t *partials, int &nblocks,
                              hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    nblocks = blocks_for(3, V);
    if ((int64_t)nblocks * kThreads * (((1 << kPlanes) - 1) / 3) < V)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_count_unsat, dim3(nblocks), dim3(kThreads), 0, s, S, J, L, partials);
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
