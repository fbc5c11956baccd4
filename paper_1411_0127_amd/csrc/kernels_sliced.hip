// Sliced layout and its two-pass sweep (Sec. 2, the cubic-stencil access pattern
// built on a coordinate transformation).
//
// The transformation x' = x, y' = y - x, z' = x - y + z (all mod L) maps the
// periodic cube onto itself, and every z' plane is one colour: z' has the parity
// of x + y + z, so with L even red sites (x+y+z even) fill the even planes and
// blue sites the odd ones.  A site's six neighbours then lie in the two planes
// z' +- 1, at in-plane offsets
//   z' + 1:  +z (0, 0),   -y (0, -1),   +x (+1, -1)     as (dx', dy')
//   z' - 1:  -z (0, 0),   +y (0, +1),   -x (-1, +1)
// (Sec. 2, the transformed nearest-neighbour coordinates), so a plane of one
// colour is updated from the two planes of the other colour around it.
//
// Storage: colour c = z' & 1 goes to its own array, plane m = z' / 2 of it
// (Sec. 2: z' labels run over L/2 planes per colour), row y', word x':
//   S[c][m][y'][x']      spin word of the site
//   K[d][c][m][y'][x']   its own couplings J[d], bond to the +d neighbour
// A red site (z' = 2m) has its "up" blue plane at m and its "down" one at m - 1;
// a blue site (z' = 2m + 1) its up red plane at m + 1 and its down one at m.  The
// three bonds a site does not own are J[x] of its -x neighbour, J[y] of its -y
// neighbour and J[z] of its -z neighbour, read from the other colour's K.
//
// One lane per site word, x' fastest, so a wave reads each of its 12 neighbour
// and coupling operands as a contiguous run (shifted by one word for the x'
// offsets).  Sites of one colour are independent, so each pass updates in place.
// The random streams are keyed by the cube site (x, y, z), recovered with the
// inverse transformation x = x', y = y' + x', z = z' + y'.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n)
{
    int64_t g = (n + kBlock * 4 - 1) / (kBlock * 4);
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// cube index of sliced position g = x' + L*(y' + L*m) of colour c
__device__ __forceinline__ int64_t sliced_to_cube(int L, int c, int64_t g)
{
    const int64_t LL = (int64_t)L * L;
    const int xp = (int)(g % L);
    const int yp = (int)((g / L) % L);
    const int zp = (int)(2 * (g / LL) + c);
    int y = xp + yp;
    y -= y >= L ? L : 0;
    int z = zp + yp;
    z -= z >= L ? L : 0;
    return xp + (int64_t)L * (y + (int64_t)L * z);
}

// nw cube arrays (src_stride words apart) -> sliced: dst[k][c][V/2] for k < nw.
// Reads are gathers (one cube word per lane, stride L + 1 along x'); the sliced
// side is written contiguously.
__global__ void k_to_sliced(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, int L, int nw,
                            int64_t src_stride)
{
    const int64_t V = (int64_t)L * L * L, half = V / 2;
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < V; g += (int64_t)gridDim.x * kBlock) {
        const int c = g >= half;
        const int64_t i = sliced_to_cube(L, c, g - c * half);
        for (int k = 0; k < nw; ++k)
            dst[k * V + g] = src[k * src_stride + i];
    }
}

__global__ void k_from_sliced(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, int L)
{
    const int64_t V = (int64_t)L * L * L, half = V / 2;
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < V; g += (int64_t)gridDim.x * kBlock) {
        const int c = g >= half;
        dst[sliced_to_cube(L, c, g - c * half)] = src[g];
    }
}

// One colour pass over the planes of colour `colour`.
template <int PRNG>
__global__ __launch_bounds__(kBlock) void k_twopass_sliced(uint64_t *__restrict__ S, const uint64_t *__restrict__ K,
                                                           const uint32_t *__restrict__ rnd, uint32_t mk, int L,
                                                           int colour, uint32_t a, uint64_t pkey, int64_t t,
                                                           Thresholds T)
{
    const int64_t LL = (int64_t)L * L, half = LL * L / 2;
    const int M = L >> 1;  // planes per colour
    uint64_t *__restrict__ me = S + colour * half;
    const uint64_t *__restrict__ ot = S + (1 - colour) * half;
    const uint64_t *__restrict__ Km = K + colour * half;        // K[d] of this colour at Km + 2*d*half
    const uint64_t *__restrict__ Ko = K + (1 - colour) * half;  // K[d] of the other colour
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g < half; g += (int64_t)gridDim.x * kBlock) {
        const int xp = (int)(g % L);
        const int yp = (int)((g / L) % L);
        const int m = (int)(g / LL);
        // the other colour's planes above (z' + 1) and below (z' - 1)
        int mu = m + colour, md = m + colour - 1;
        mu -= mu == M ? M : 0;
        md += md < 0 ? M : 0;
        const int xpp = xp + 1 == L ? 0 : xp + 1, xpm = xp == 0 ? L - 1 : xp - 1;
        const int ypp = yp + 1 == L ? 0 : yp + 1, ypm = yp == 0 ? L - 1 : yp - 1;
        const int64_t up = (int64_t)mu * LL, dn = (int64_t)md * LL;
        const int64_t rz = (int64_t)yp * L, rm = (int64_t)ypm * L, rp = (int64_t)ypp * L;
        const uint64_t s = me[g];
        const uint64_t nzp = ot[up + rz + xp];    // +z
        const uint64_t nym = ot[up + rm + xp];    // -y
        const uint64_t nxp = ot[up + rm + xpp];   // +x
        const uint64_t nzm = ot[dn + rz + xp];    // -z
        const uint64_t nyp = ot[dn + rp + xp];    // +y
        const uint64_t nxm = ot[dn + rp + xpm];   // -x
        const uint64_t jxp = Km[g], jyp = Km[2 * half + g], jzp = Km[4 * half + g];
        const uint64_t jxm = Ko[dn + rp + xpm];             // J[x] of the -x neighbour
        const uint64_t jym = Ko[2 * half + up + rm + xp];   // J[y] of the -y neighbour
        const uint64_t jzm = Ko[4 * half + dn + rz + xp];   // J[z] of the -z neighbour
        // cube coordinates of the site (inverse transformation)
        const int zp = 2 * m + colour;
        int y = xp + yp;
        y -= y >= L ? L : 0;
        int z = zp + yp;
        z -= z >= L ? L : 0;
        const int64_t i = xp + (int64_t)L * (y + (int64_t)L * z);
        uint64_t nw;
        if (PRNG == SG_PHILOX) {
            nw = flip_site_ps(s, nxp, nyp, nzp, nxm, nym, nzm, jxp, jyp, jzp, jxm, jym, jzm, (uint64_t)i, (uint64_t)t,
                              (uint32_t)pkey, (uint32_t)(pkey >> 32), T);
        } else {
            const uint32_t R = (PRNG == SG_MINSTD)
                                   ? minstd_jump(a, minstd_seed((uint32_t)(xp + L * y), minstd_plane_key((uint32_t)z, mk)))
                                   : rnd[i];
            nw = flip_site(s, nxp, nyp, nzp, nxm, nym, nzm, jxp, jyp, jzp, jxm, jym, jzm, R, T);
        }
        me[g] = nw;
    }
}

}  // namespace

hipError_t launch_to_sliced(const uint64_t *cube, uint64_t *sl, int L, int nwords, int64_t src_stride,
                            hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_to_sliced, dim3(grid_for(V)), dim3(kBlock), 0, s, cube, sl, L, nwords, src_stride);
    return hipGetLastError();
}

hipError_t launch_from_sliced(const uint64_t *sl, uint64_t *cube, int L, hipStream_t s)
{
    const int64_t V = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_from_sliced, dim3(grid_for(V)), dim3(kBlock), 0, s, sl, cube, L);
    return hipGetLastError();
}

hipError_t launch_sweep_sliced(const SweepArgs &a, uint64_t *S, const uint64_t *K, hipStream_t s)
{
    const int64_t V = (int64_t)a.L * a.L * a.L;
    const int g = grid_for(V / 2);
    for (int colour = 0; colour < 2; ++colour) {
        if (a.prng == SG_MINSTD)
            hipLaunchKernelGGL(k_twopass_sliced<SG_MINSTD>, dim3(g), dim3(kBlock), 0, s, S, K, a.rnd[0], a.mk[0], a.L,
                               colour, a.minstd_a, a.pkey[0], a.t, a.T);
        else if (a.prng == SG_PHILOX)
            hipLaunchKernelGGL(k_twopass_sliced<SG_PHILOX>, dim3(g), dim3(kBlock), 0, s, S, K, a.rnd[0], a.mk[0], a.L,
                               colour, a.minstd_a, a.pkey[0], a.t, a.T);
        else
            hipLaunchKernelGGL(k_twopass_sliced<SG_MT19937>, dim3(g), dim3(kBlock), 0, s, S, K, a.rnd[0], a.mk[0],
                               a.L, colour, a.minstd_a, a.pkey[0], a.t, a.T);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace sg
