// Small lattices in one workgroup: every sweep of a call in one launch, with the
// energy of Sec. 1, Eq. (1) counted after each sweep.
//
// A lattice of up to kSmallSites sites (L <= 16) keeps its spin words and its
// three coupling words per site in LDS (136 KB with the reduction table) for the
// whole call.  Each sweep is the checkerboard of Sec. 1, red sites (x + y + z
// even) then blue, sites of one colour updated in place with the bit-sliced rule
// of Sec. 4 and the same keyed numbers as every other kernel, so the spins equal
// theirs bit for bit.  A thread owns fixed sites of each colour (as the two-pass
// kernel numbers them: x = 2 xh + parity), so no lane idles in a colour pass, and
// keeps their neighbour indices and MINSTD seeds in registers.  After each sweep
// the workgroup counts the unsatisfied bonds of the lattice's samples and writes
// them to out[sweep][64].  At these sizes a sweep is a few microseconds of work,
// so one launch per call instead of three per sweep is what sets the time.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kSmallThreads = 1024;
constexpr int kPerThread = kSmallSites / 2 / kSmallThreads;  // sites of one colour per thread
constexpr int kCountPlanes = 4;  // a thread adds at most 3 * 4 = 12 bond words per count
constexpr int kWavePlanes = 10;  // a wave's count is at most 64 * 12 = 768 < 2^10
constexpr int kBallotSamples = 16;  // up to this many samples the counts are read by ballots
constexpr int kDirectSamples = 4;   // up to this many, counted per sample directly

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int d)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Per-sample totals of the wave's bit-sliced counts (planes cnt[0..3], bit j of
// plane b = bit b of lane's count of sample j), for every sample: a butterfly of
// bit-sliced additions across the lanes, after which every lane holds the wave's
// ten planes, and lane j reads sample j's total out of them.
__device__ __forceinline__ uint64_t wave_counts(const uint64_t (&cnt)[kCountPlanes], int lane)
{
    uint64_t w[kWavePlanes];
#pragma unroll
    for (int b = 0; b < kWavePlanes; ++b)
        w[b] = b < kCountPlanes ? cnt[b] : 0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        // counts are below 12 * 2^l before this level: 4 + l planes in use, one more after it
        uint64_t c = 0;
#pragma unroll
        for (int b = 0; b < kCountPlanes + l + 1 && b < kWavePlanes; ++b) {
            const uint64_t o = shfl_xor64(w[b], 1 << l);
            const uint64_t sum = w[b] ^ o ^ c;
            c = (w[b] & o) | (c & (w[b] ^ o));
            w[b] = sum;
        }
    }
    uint64_t tot = 0;
#pragma unroll
    for (int b = 0; b < kWavePlanes; ++b)
        tot |= ((w[b] >> lane) & 1ull) << b;
    return tot;
}

static_assert(kSmallSites % (2 * kSmallThreads) == 0, "whole sites of each colour per thread");

template <int PRNG>
__global__ __launch_bounds__(kSmallThreads) void k_small_sweeps(uint64_t *__restrict__ S,
                                                                const uint64_t *__restrict__ J, int L,
                                                                int nsamples, uint32_t mk, uint64_t pkey, int64_t t0,
                                                                uint32_t a0, int nsweeps, Thresholds T,
                                                                uint64_t *__restrict__ out)
{
    __shared__ uint64_t s[kSmallSites];
    __shared__ uint64_t jw[3][kSmallSites];
    __shared__ uint64_t part[kSmallThreads / 64][64];
    const int LL = L * L;
    const int V = LL * L;
    const int half = V / 2;
    const int hx = L / 2;
    const int64_t Vj = coupling_stride(L);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    for (int i = tid; i < V; i += kSmallThreads) {
        s[i] = S[i];
        jw[0][i] = J[i];
        jw[1][i] = J[Vj + i];
        jw[2][i] = J[2 * Vj + i];
    }
    // this thread's sites: site[c][m] of colour c (-1 past the end), their six
    // neighbours (+x, -x, +y, -y, +z, -z, periodic) and their seeds, all fixed for
    // the call
    int site[2][kPerThread];
    int nb[2][kPerThread][6];
    uint32_t seed[2][kPerThread];
    uint64_t jown[2][kPerThread][3];  // couplings of the site's +x, +y, +z bonds (static)
    uint64_t sown[2][kPerThread];     // the site's spin word (only this thread writes it)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < kPerThread; ++m) {
            const int g = tid + m * kSmallThreads;
            site[c][m] = -1;
            seed[c][m] = 0;
            jown[c][m][0] = jown[c][m][1] = jown[c][m][2] = 0;
            sown[c][m] = 0;
#pragma unroll
            for (int d = 0; d < 6; ++d)
                nb[c][m][d] = 0;
            if (g < half) {
                const int xh = g % hx;
                const int row = g / hx;
                const int y = row % L;
                const int z = row / L;
                const int x = 2 * xh + ((y + z + c) & 1);
                const int i = x + L * y + LL * z;
                site[c][m] = i;
                nb[c][m][0] = (x + 1 == L) ? i - (L - 1) : i + 1;
                nb[c][m][1] = (x == 0) ? i + (L - 1) : i - 1;
                nb[c][m][2] = (y + 1 == L) ? i - (L - 1) * L : i + L;
                nb[c][m][3] = (y == 0) ? i + (L - 1) * L : i - L;
                nb[c][m][4] = (z + 1 == L) ? i - (V - LL) : i + LL;
                nb[c][m][5] = (z == 0) ? i + (V - LL) : i - LL;
                seed[c][m] = minstd_seed((uint32_t)(x + L * y), minstd_plane_key((uint32_t)z, mk));
                sown[c][m] = S[i];
                jown[c][m][0] = J[i];
                jown[c][m][1] = J[Vj + i];
                jown[c][m][2] = J[2 * Vj + i];
            }
        }
    __syncthreads();
    uint32_t a = a0;  // 16807^(t+1) mod (2^31 - 1) of the current sweep t
    for (int k = 0; k < nsweeps; ++k) {
        const int64_t t = t0 + k;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int m = 0; m < kPerThread; ++m) {
                const int i = site[c][m];
                if (i < 0)
                    continue;
                const int ixp = nb[c][m][0], ixm = nb[c][m][1], iyp = nb[c][m][2], iym = nb[c][m][3];
                const int izp = nb[c][m][4], izm = nb[c][m][5];
                const uint64_t si = sown[c][m];
                uint64_t sn;
                if (PRNG == SG_PHILOX)
                    sn = flip_site_ps(si, s[ixp], s[iyp], s[izp], s[ixm], s[iym], s[izm], jown[c][m][0],
                                        jown[c][m][1], jown[c][m][2], jw[0][ixm], jw[1][iym], jw[2][izm], (uint64_t)i,
                                        (uint64_t)t, (uint32_t)pkey, (uint32_t)(pkey >> 32), T);
                else
                    sn = flip_site(si, s[ixp], s[iyp], s[izp], s[ixm], s[iym], s[izm], jown[c][m][0], jown[c][m][1],
                                     jown[c][m][2], jw[0][ixm], jw[1][iym], jw[2][izm], minstd_jump(a, seed[c][m]), T);
                s[i] = sn;
                sown[c][m] = sn;
            }
            __syncthreads();
        }
        if (out && nsamples <= kDirectSamples) {
            // bond (i, i + d) of sample j is unsatisfied when bit j of J[d][i] ^ s_i ^ s_{i+d}
            // is 1 (the bond bit of Sec. 4).  A few samples: an integer count per sample
            // and thread from the low word, summed over the wave by a butterfly; lane j
            // keeps sample j's total.
            uint32_t cj[kDirectSamples] = {};
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int m = 0; m < kPerThread; ++m) {
                    const int i = site[c][m];
                    if (i < 0)
                        continue;
                    const uint32_t si = (uint32_t)sown[c][m];
                    const uint32_t w0 = bop3<bop::kXor3>((uint32_t)jown[c][m][0], si, (uint32_t)s[nb[c][m][0]]);
                    const uint32_t w1 = bop3<bop::kXor3>((uint32_t)jown[c][m][1], si, (uint32_t)s[nb[c][m][2]]);
                    const uint32_t w2 = bop3<bop::kXor3>((uint32_t)jown[c][m][2], si, (uint32_t)s[nb[c][m][4]]);
#pragma unroll
                    for (int j = 0; j < kDirectSamples; ++j) {
                        if (j >= nsamples)
                            break;
                        cj[j] += ((w0 >> j) & 1u) + ((w1 >> j) & 1u) + ((w2 >> j) & 1u);
                    }
                }
            uint64_t mine = 0;
#pragma unroll
            for (int j = 0; j < kDirectSamples; ++j) {
                if (j >= nsamples)
                    break;
                uint32_t v = cj[j];
#pragma unroll
                for (int d = 1; d < 64; d <<= 1)
                    v += (uint32_t)__shfl_xor((int)v, d, 64);
                mine = lane == j ? v : mine;
            }
            part[wave][lane] = mine;
            __syncthreads();
            if (tid < 64) {
                uint64_t sum = 0;
                for (int w = 0; w < kSmallThreads / 64; ++w)
                    sum += part[w][tid];
                out[(size_t)k * 64 + tid] = sum;
            }
            // no barrier here: part is written again only after the next sweep's two
            // colour barriers, which these threads reach once their sums are done
        } else if (out) {
            // the same bond bits, bit-sliced counts: plane b = bit b of 64 counts
            uint64_t cnt[kCountPlanes] = {};
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int m = 0; m < kPerThread; ++m) {
                    const int i = site[c][m];
                    if (i < 0)
                        continue;
                    const uint64_t si = sown[c][m];
                    const uint64_t w[3] = {jown[c][m][0] ^ si ^ s[nb[c][m][0]], jown[c][m][1] ^ si ^ s[nb[c][m][2]],
                                           jown[c][m][2] ^ si ^ s[nb[c][m][4]]};
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        uint64_t v = w[d];
#pragma unroll
                        for (int b = 0; b < kCountPlanes; ++b) {
                            const uint64_t carry = cnt[b] & v;
                            cnt[b] ^= v;
                            v = carry;
                        }
                    }
                }
            // per wave, lane j keeps sample j's total: up to kBallotSamples samples, the
            // sum over planes b of 2^b times the lanes whose plane b has bit j set
            // (samples past nsamples are simulated but not counted); for more, the
            // butterfly
            uint64_t mine = 0;
            if (nsamples <= kBallotSamples) {
                for (int j = 0; j < nsamples; ++j) {
                    uint64_t tot = 0;
#pragma unroll
                    for (int b = 0; b < kCountPlanes; ++b)
                        tot += (uint64_t)__popcll(__ballot((cnt[b] >> j) & 1ull)) << b;
                    mine = lane == j ? tot : mine;
                }
            } else {
                mine = wave_counts(cnt, lane);
            }
            part[wave][lane] = mine;
            __syncthreads();
            if (tid < 64) {
                uint64_t sum = 0;
                for (int w = 0; w < kSmallThreads / 64; ++w)
                    sum += part[w][tid];
                out[(size_t)k * 64 + tid] = sum;
            }
            // no barrier here: part is written again only after the next sweep's two
            // colour barriers, which these threads reach once their sums are done
        }
        a = minstd_jump(a, 16807u);
    }
    for (int i = tid; i < V; i += kSmallThreads)
        S[i] = s[i];
}

}  // namespace

hipError_t launch_small_sweeps(uint64_t *S, const uint64_t *J, int L, int nsamples, int prng, uint32_t mk,
                               uint64_t pkey, int64_t t0, uint32_t a0, int nsweeps, const Thresholds &T, uint64_t *out,
                               hipStream_t s)
{
    if ((int64_t)L * L * L > kSmallSites || L < 2 || (L & 1) || nsweeps < 1 || nsamples < 1 || nsamples > 64 ||
        (prng != SG_MINSTD && prng != SG_PHILOX))
        return hipErrorInvalidValue;
    if (prng == SG_PHILOX)
        hipLaunchKernelGGL(k_small_sweeps<SG_PHILOX>, dim3(1), dim3(kSmallThreads), 0, s, S, J, L, nsamples, mk, pkey,
                           t0, a0, nsweeps, T, out);
    else
        hipLaunchKernelGGL(k_small_sweeps<SG_MINSTD>, dim3(1), dim3(kSmallThreads), 0, s, S, J, L, nsamples, mk, pkey,
                           t0, a0, nsweeps, T, out);
    return hipGetLastError();
}

}  // namespace sg
