// Colour-separated layout and its two-pass sweep (the "standard" separate-
// allocation scheme of Sec. 2's layout study: red and blue sites in separate
// arrays, so that the threads of one colour read their neighbours of the other
// colour with unit stride; no coordinate transformation).
//
// Layout (this library's form of it): for colour c (0 = red, x+y+z even; 1 = blue)
// the array C_c[z][y][h], h = 0 .. L/2-1, holds the site x = 2h + ((y + z + c) & 1)
// of row (y, z).  A site's own couplings J[d] (bond to +d) go with its colour:
// K_c[d][z][y][h].  For a site of colour c at (z, y, h) with p = (y + z + c) & 1,
// every neighbour has the other colour c' and sits at
//   x+1: h + p (0 past the row end) ... x-1: h + p - 1 (L/2 - 1 before the start),
//   y+-1, z+-1: the same h in the neighbouring row or plane,
// so a wave of one colour reads its six neighbours and six couplings as contiguous
// runs.  Sites of one colour are independent, so each pass updates in place.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n)
{
    int64_t g = (n + kBlock * 4 - 1) / (kBlock * 4);
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// cube word of (colour c, z, y, h)
__device__ __forceinline__ int64_t cube_index(int L, int c, int64_t z, int64_t y, int64_t h)
{
    const int64_t x = 2 * h + ((y + z + c) & 1);
    return x + (int64_t)L * (y + (int64_t)L * z);
}

// nw cube arrays of V words (stride src_stride) -> separated: dst[k][c][V/2] for k < nw
__global__ void k_to_separated(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, int L, int nw,
                            int64_t src_stride)
{
    const int64_t V = (int64_t)L * L * L, half = V / 2, hx = L / 2;
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < V; g += (int64_t)gridDim.x * kBlock) {
        const int c = g >= half;
        const int64_t r = g - c * half;
        const int64_t h = r % hx, row = r / hx, y = row % L, z = row / L;
        const int64_t i = cube_index(L, c, z, y, h);
        for (int k = 0; k < nw; ++k)
            dst[k * V + g] = src[k * src_stride + i];
    }
}

__global__ void k_from_separated(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, int L)
{
    const int64_t V = (int64_t)L * L * L, half = V / 2, hx = L / 2;
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < V; g += (int64_t)gridDim.x * kBlock) {
        const int c = g >= half;
        const int64_t r = g - c * half;
        const int64_t h = r % hx, row = r / hx, y = row % L, z = row / L;
        dst[cube_index(L, c, z, y, h)] = src[g];
    }
}

// One colour pass.  S: separated spins [2][V/2]; K: separated couplings [3][2][V/2].
template <int PRNG>
__global__ __launch_bounds__(kBlock) void k_twopass_separated(uint64_t *__restrict__ S, const uint64_t *__restrict__ K,
                                                           const uint32_t *__restrict__ rnd, uint32_t mk, int L,
                                                           int colour, uint32_t a, uint64_t pkey, int64_t t,
                                                           Thresholds T)
{
    const int64_t V = (int64_t)L * L * L, half = V / 2;
    const int hx = L >> 1;
    const int64_t rowlen = hx, plane = (int64_t)hx * L;
    uint64_t *__restrict__ me = S + colour * half;
    const uint64_t *__restrict__ ot = S + (1 - colour) * half;
    const uint64_t *__restrict__ Km = K + colour * half;        // K[d] of this colour at Km + 2*d*half
    const uint64_t *__restrict__ Ko = K + (1 - colour) * half;  // K[d] of the other colour
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < half; g += (int64_t)gridDim.x * kBlock) {
        const int h = (int)(g % hx);
        const int64_t row = g / hx;
        const int y = (int)(row % L);
        const int z = (int)(row / L);
        const int p = (y + z + colour) & 1;
        const int64_t base = g - h;  // start of the row
        const int hp = (h + p == hx) ? 0 : h + p;
        const int hm = (h + p == 0) ? hx - 1 : h + p - 1;
        const int64_t iyp = (y + 1 == L) ? g - (int64_t)(L - 1) * rowlen : g + rowlen;
        const int64_t iym = (y == 0) ? g + (int64_t)(L - 1) * rowlen : g - rowlen;
        const int64_t izp = (z + 1 == L) ? g - (int64_t)(L - 1) * plane : g + plane;
        const int64_t izm = (z == 0) ? g + (int64_t)(L - 1) * plane : g - plane;
        const uint64_t s = me[g];
        const uint64_t nxp = ot[base + hp], nxm = ot[base + hm];
        const uint64_t jxp = Km[g], jyp = Km[2 * half + g], jzp = Km[4 * half + g];
        const uint64_t jxm = Ko[base + hm], jym = Ko[2 * half + iym], jzm = Ko[4 * half + izm];
        const int x = 2 * h + p;
        const int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
        uint64_t nw;
        if (PRNG == SG_PHILOX) {
            nw = flip_site_ps(s, nxp, ot[iyp], ot[izp], nxm, ot[iym], ot[izm], jxp, jyp, jzp, jxm, jym, jzm,
                              (uint64_t)i, (uint64_t)t, (uint32_t)pkey, (uint32_t)(pkey >> 32), T);
        } else {
            const uint32_t R = (PRNG == SG_MINSTD)
                                   ? minstd_jump(a, minstd_seed((uint32_t)(x + L * y), minstd_plane_key((uint32_t)z, mk)))
                                   : rnd[i];
            nw = flip_site(s, nxp, ot[iyp], ot[izp], nxm, ot[iym], ot[izm], jxp, jyp, jzp, jxm, jym, jzm, R, T);
        }
        me[g] = nw;
    }
}

}  // namespace

hipError_t launch_to_separated(const uint64_t *cube, uint64_t *sliced, int L, int nwords, int64_t src_stride,
                            hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_to_separated, dim3(grid_for(V)), dim3(kBlock), 0, s, cube, sliced, L, nwords, src_stride);
    return hipGetLastError();
}

hipError_t launch_from_separated(const uint64_t *sliced, uint64_t *cube, int L, hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_from_separated, dim3(grid_for(V)), dim3(kBlock), 0, s, sliced, cube, L);
    return hipGetLastError();
}

hipError_t launch_sweep_separated(const SweepArgs &a, uint64_t *S, const uint64_t *K, hipStream_t s)
{
    const int64_t V = (int64_t)a.L * a.L * a.L;
    const int g = grid_for(V / 2);
    for (int colour = 0; colour < 2; ++colour) {
        if (a.prng == SG_MINSTD)
            hipLaunchKernelGGL(k_twopass_separated<SG_MINSTD>, dim3(g), dim3(kBlock), 0, s, S, K, a.rnd[0], a.mk[0], a.L,
                               colour, a.minstd_a, a.pkey[0], a.t, a.T);
        else if (a.prng == SG_PHILOX)
            hipLaunchKernelGGL(k_twopass_separated<SG_PHILOX>, dim3(g), dim3(kBlock), 0, s, S, K, a.rnd[0], a.mk[0], a.L,
                               colour, a.minstd_a, a.pkey[0], a.t, a.T);
        else
            hipLaunchKernelGGL(k_twopass_separated<SG_MT19937>, dim3(g), dim3(kBlock), 0, s, S, K, a.rnd[0], a.mk[0],
                               a.L, colour, a.minstd_a, a.pkey[0], a.t, a.T);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace sg
