// Initialisation and random-stream kernels of libsg (gfx950).
//  - couplings and spins from the SplitMix64 keyed generator (MINSTD seeds are
//    a keyed hash of the site, evaluated where they are used);
//  - MT19937 (Matsumoto-Nishimura 1998) per-column streams: init_genrand, and a
//    per-sweep fill of the L draws every column needs (Sec. 3 of the paper: a
//    per-stream MT19937 whose state is laid out so that consecutive streams are
//    consecutive in memory, word k of stream c at k*ncols + c);
//  - Parisi-Rapuano per-column streams (Sec. 3): x_n = x_{n-24} + x_{n-55} mod
//    2^32, R_n = x_n ^ x_{n-61}, state x_n at word n mod 64 in the same strided
//    layout; the per-sweep fill keeps each column's 64 words in LDS.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int per_thread = 1)
{
    int64_t g = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    return (int)g;
}

__global__ void k_init_couplings(uint64_t *__restrict__ J, int64_t V, int64_t Vj, uint64_t key)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < V; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t n = 1ull + 3ull * (uint64_t)i;
        J[i] = sm_out(key, n);
        J[Vj + i] = sm_out(key, n + 1);
        J[2 * Vj + i] = sm_out(key, n + 2);
    }
}

__global__ void k_init_spins(uint64_t *__restrict__ S, int64_t V, uint64_t key)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < V; i += (int64_t)gridDim.x * blockDim.x)
        S[i] = sm_out(key, 1ull + (uint64_t)i);
}

// init_genrand of column c's stream with seed = low 32 bits of its keyed word.
__global__ void k_init_mt(uint32_t *__restrict__ st, int ncols, uint64_t key)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols)
        return;
    uint32_t v = (uint32_t)sm_out(key, 1ull + (uint64_t)c);
    st[c] = v;
    for (int k = 1; k < kMtN; ++k) {
        v = 1812433253u * (v ^ (v >> 30)) + (uint32_t)k;
        st[(size_t)k * ncols + c] = v;
    }
}

__device__ __forceinline__ uint32_t mt_temper(uint32_t y)
{
    y ^= y >> 11;
    y ^= (y << 7) & 0x9D2C5680u;
    y ^= (y << 15) & 0xEFC60000u;
    y ^= y >> 18;
    return y;
}

// Draws of sweeps t .. t+nsw-1: column c produces its outputs t*L .. (t+nsw)*L - 1
// and writes output t*L + u to R[u*L*L + c], so sweep t+s's draws fill
// R[s*L^3 .. (s+1)*L^3).  The twist is done one word at a time, right
// before the word is output: word i of a new block is computed from word i and
// i+1 of the previous block and word i+397 (already renewed when i+397 >= 624
// wraps), which is exactly the order of the sequential in-place twist.
//
// Steps go in groups of U: the words a group reads (i+1 .. i+U and i+397 ..
// i+397+U-1, mod 624) are loaded first, together.  None of them is renewed inside
// the group -- word i+1+u is renewed at step u+1, after it is read, and word
// i+397+u mod 624 is renewed 227 steps before or 397 steps after step u -- so the
// group sees the same values the sequential twist does, with U loads in flight.
// blockIdx.y selects one of up to two streams sets (replicas).
struct MtFillArgs {
    uint32_t *st[2];
    uint32_t *R[2];
};

constexpr int kMtGroup = 8;

__global__ __launch_bounds__(256) void k_mt_fill(MtFillArgs a, int L, int64_t t, int nsw)
{
    const int ncols = L * L;
    const int nz = nsw * L;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols)
        return;
    uint32_t *__restrict__ st = a.st[blockIdx.y];
    uint32_t *__restrict__ R = a.R[blockIdx.y];
    int i = (int)(((int64_t)t * L) % kMtN);
    uint32_t cur = st[(size_t)i * ncols + c];
    for (int z0 = 0; z0 < nz; z0 += kMtGroup) {
        const int n = min(kMtGroup, nz - z0);
        uint32_t nxt[kMtGroup], far[kMtGroup];
#pragma unroll
        for (int u = 0; u < kMtGroup; ++u) {
            if (u < n) {
                int i1 = i + 1 + u;
                i1 = i1 >= kMtN ? i1 - kMtN : i1;
                int im = i + 397 + u;
                im = im >= kMtN ? im - kMtN : im;
                im = im >= kMtN ? im - kMtN : im;
                nxt[u] = st[(size_t)i1 * ncols + c];
                far[u] = st[(size_t)im * ncols + c];
            }
        }
#pragma unroll
        for (int u = 0; u < kMtGroup; ++u) {
            if (u < n) {
                const uint32_t y = (cur & 0x80000000u) | (nxt[u] & 0x7FFFFFFFu);
                uint32_t v = far[u] ^ (y >> 1);
                v ^= (y & 1u) ? 0x9908B0DFu : 0u;
                st[(size_t)i * ncols + c] = v;
                R[(size_t)(z0 + u) * ncols + c] = mt_temper(v);
                // word i+1 is renewed next; its value before that is the one read
                cur = nxt[u];
                i = (i + 1 == kMtN) ? 0 : i + 1;
            }
        }
    }
}

// Parisi-Rapuano seed words x_{-61+k} = lo32(out(key, 1 + 61 c + k)), k = 0..60,
// word k = 0 made odd (a full-period start needs one odd word); x_n lives at word
// n mod 64, so the seeds go to words 3..63.
__global__ void k_init_pr(uint32_t *__restrict__ st, int ncols, uint64_t key)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols)
        return;
    for (int k = 0; k < 3; ++k)
        st[(size_t)k * ncols + c] = 0u;
    for (int k = 0; k < 61; ++k) {
        uint32_t w = (uint32_t)sm_out(key, 1ull + 61ull * (uint64_t)c + (uint64_t)k);
        if (k == 0)
            w |= 1u;
        st[(size_t)(k + 3) * ncols + c] = w;
    }
}

// The numbers of sweeps t .. t+nsw-1 (numbers t*L .. (t+nsw)*L - 1) of every
// column, laid out as for MT19937, for up to two stream sets (blockIdx.y).  A thread owns one column; its 64 state words sit
// in LDS at word k * kPrBlock + thread (no bank conflicts) while it steps the
// recurrence, and go back to HBM at the end.
constexpr int kPrBlock = 128;
struct PrFillArgs {
    uint32_t *st[2];
    uint32_t *R[2];
};
__global__ __launch_bounds__(kPrBlock) void k_pr_fill(PrFillArgs a, int L, int64_t t, int nsw)
{
    __shared__ uint32_t buf[64 * kPrBlock];
    const int ncols = L * L;
    const int c = blockIdx.x * kPrBlock + threadIdx.x;
    if (c >= ncols)
        return;
    uint32_t *__restrict__ st = a.st[blockIdx.y];
    uint32_t *__restrict__ R = a.R[blockIdx.y];
    uint32_t *b = buf + threadIdx.x;
    for (int k = 0; k < 64; ++k)
        b[k * kPrBlock] = st[(size_t)k * ncols + c];
    const int64_t n0 = t * (int64_t)L;
    for (int z = 0; z < nsw * L; ++z) {
        const int n = (int)((n0 + z) & 63);
        const uint32_t x = b[((n - 24) & 63) * kPrBlock] + b[((n - 55) & 63) * kPrBlock];
        R[(size_t)z * ncols + c] = x ^ b[((n - 61) & 63) * kPrBlock];
        b[n * kPrBlock] = x;
    }
    for (int k = 0; k < 64; ++k)
        st[(size_t)k * ncols + c] = b[k * kPrBlock];
}

// MINSTD number of every site in the sweep whose multiplier is a =
// 16807^(t+1) mod (2^31 - 1): out[i] for site i = x + L*(y + L*z), from the
// same seed and jump functions the sweep kernels evaluate.
__global__ void k_minstd_draws(uint32_t *__restrict__ out, int L, uint32_t a, uint32_t mk)
{
    const int64_t LL = (int64_t)L * L, V = LL * L;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < V; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t z = (uint32_t)(i / LL), xy = (uint32_t)(i - (int64_t)z * LL);
        out[i] = minstd_jump(a, minstd_seed(xy, minstd_plane_key(z, mk)));
    }
}

}  // namespace

hipError_t launch_init_couplings(uint64_t *J, int L, uint64_t key, hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_init_couplings, dim3(grid_for(V, 4)), dim3(kBlock), 0, s, J, V, coupling_stride(L), key);
    return hipGetLastError();
}

hipError_t launch_init_spins(uint64_t *S, int L, uint64_t key, hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_init_spins, dim3(grid_for(V, 4)), dim3(kBlock), 0, s, S, V, key);
    return hipGetLastError();
}

hipError_t launch_minstd_draws(uint32_t *out, int L, uint32_t a, uint32_t mk, hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_minstd_draws, dim3(grid_for(V, 4)), dim3(kBlock), 0, s, out, L, a, mk);
    return hipGetLastError();
}

hipError_t launch_init_mt(uint32_t *state, int L, uint64_t key, hipStream_t s)
{
    const int ncols = L * L;
    hipLaunchKernelGGL(k_init_mt, dim3((ncols + kBlock - 1) / kBlock), dim3(kBlock), 0, s, state, ncols, key);
    return hipGetLastError();
}

hipError_t launch_init_pr(uint32_t *state, int L, uint64_t key, hipStream_t s)
{
    const int ncols = L * L;
    hipLaunchKernelGGL(k_init_pr, dim3((ncols + kBlock - 1) / kBlock), dim3(kBlock), 0, s, state, ncols, key);
    return hipGetLastError();
}

hipError_t launch_pr_fill(uint32_t *const *state, uint32_t *const *rbuf, int n, int L, int64_t t, int nsw,
                          hipStream_t s)
{
    if (nsw < 1 || nsw > 2)
        return hipErrorInvalidValue;
    const int ncols = L * L;
    PrFillArgs a{};
    for (int r = 0; r < n && r < 2; ++r) {
        a.st[r] = state[r];
        a.R[r] = rbuf[r];
    }
    hipLaunchKernelGGL(k_pr_fill, dim3((ncols + kPrBlock - 1) / kPrBlock, n), dim3(kPrBlock), 0, s, a, L, t, nsw);
    return hipGetLastError();
}

hipError_t launch_mt_fill(uint32_t *const *state, uint32_t *const *rbuf, int n, int L, int64_t t, int nsw,
                          hipStream_t s)
{
    if (nsw < 1 || nsw > 2)
        return hipErrorInvalidValue;
    const int ncols = L * L;
    MtFillArgs a{};
    for (int r = 0; r < n && r < 2; ++r) {
        a.st[r] = state[r];
        a.R[r] = rbuf[r];
    }
    hipLaunchKernelGGL(k_mt_fill, dim3((ncols + kBlock - 1) / kBlock, n), dim3(kBlock), 0, s, a, L, t, nsw);
    return hipGetLastError();
}

}  // namespace sg
