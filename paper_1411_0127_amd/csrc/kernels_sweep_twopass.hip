// Two-pass checkerboard sweep (Sec. 1: one kernel per colour, which keeps the
// updates of one colour independent of each other).  One lane per site word of
// the colour being updated; the other colour is only read, so the update is in
// place.  Neighbours and couplings come straight from global memory (L1/L2 catch
// the reuse).  This kernel is the reference schedule for the fused one and the
// fallback for lattice shapes the fused tiling does not cover.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kBlock = 256;

template <int PRNG>
__global__ __launch_bounds__(kBlock) void k_twopass(uint64_t *__restrict__ S, const uint64_t *__restrict__ J,
                                                    const uint32_t *__restrict__ rnd, uint32_t mk, int L,
                                                    int colour, uint32_t a, uint64_t pkey, int64_t t, Thresholds T)
{
    const int64_t LL = (int64_t)L * L;
    const int64_t V = LL * L;
    const int64_t Vj = coupling_stride(L);
    const int64_t half = V / 2;
    const int hx = L >> 1;
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < half; g += (int64_t)gridDim.x * kBlock) {
        const int xh = (int)(g % hx);
        const int64_t row = g / hx;
        const int y = (int)(row % L);
        const int z = (int)(row / L);
        const int x = 2 * xh + ((y + z + colour) & 1);
        const int64_t i = x + (int64_t)L * y + LL * z;
        const int64_t ixp = (x + 1 == L) ? i - (L - 1) : i + 1;
        const int64_t ixm = (x == 0) ? i + (L - 1) : i - 1;
        const int64_t iyp = (y + 1 == L) ? i - (int64_t)(L - 1) * L : i + L;
        const int64_t iym = (y == 0) ? i + (int64_t)(L - 1) * L : i - L;
        const int64_t izp = (z + 1 == L) ? i - (V - LL) : i + LL;
        const int64_t izm = (z == 0) ? i + (V - LL) : i - LL;
        const uint64_t s = S[i];
        if (PRNG == SG_PHILOX) {
            S[i] = flip_site_ps(s, S[ixp], S[iyp], S[izp], S[ixm], S[iym], S[izm], J[i], J[Vj + i], J[2 * Vj + i],
                                J[ixm], J[Vj + iym], J[2 * Vj + izm], (uint64_t)i, (uint64_t)t, (uint32_t)pkey,
                                (uint32_t)(pkey >> 32), T);
        } else {
            const uint32_t R =
                (PRNG == SG_MINSTD)
                    ? minstd_jump(a, minstd_seed((uint32_t)(x + L * y), minstd_plane_key((uint32_t)z, mk)))
                    : rnd[i];
            S[i] = flip_site(s, S[ixp], S[iyp], S[izp], S[ixm], S[iym], S[izm], J[i], J[Vj + i], J[2 * Vj + i],
                             J[ixm], J[Vj + iym], J[2 * Vj + izm], R, T);
        }
    }
}

}  // namespace

hipError_t launch_sweep_twopass(const SweepArgs &a, hipStream_t s)
{
    const int64_t V = (int64_t)a.L * a.L * a.L;
    int64_t g = (V / 2 + kBlock * 4 - 1) / (kBlock * 4);
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    for (int r = 0; r < a.nrep; ++r)
        for (int colour = 0; colour < 2; ++colour) {
            if (a.prng == SG_MINSTD)
                hipLaunchKernelGGL(k_twopass<SG_MINSTD>, dim3((unsigned)g), dim3(kBlock), 0, s, a.src[r], a.J,
                                   a.rnd[r], a.mk[r], a.L, colour, a.minstd_a, a.pkey[r], a.t, a.T);
            else if (a.prng == SG_MT19937)
                hipLaunchKernelGGL(k_twopass<SG_MT19937>, dim3((unsigned)g), dim3(kBlock), 0, s, a.src[r], a.J,
                                   a.rnd[r], a.mk[r], a.L, colour, a.minstd_a, a.pkey[r], a.t, a.T);
            else
                hipLaunchKernelGGL(k_twopass<SG_PHILOX>, dim3((unsigned)g), dim3(kBlock), 0, s, a.src[r], a.J,
                                   a.rnd[r], a.mk[r], a.L, colour, a.minstd_a, a.pkey[r], a.t, a.T);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
    return hipSuccess;
}

}  // namespace sg
