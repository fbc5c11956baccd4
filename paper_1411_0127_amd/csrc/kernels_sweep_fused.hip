// Fused single-pass checkerboard sweep for gfx950.
//
// The paper updates red and blue with one kernel each (Sec. 1), so the couplings
// are read twice per sweep.  Here one launch does the whole sweep and reads every
// word once: a workgroup owns a tile of x-y columns and marches z.  At step k it
// updates the red sites of plane k, then the blue sites of plane k-1, whose six
// neighbours are then all new (red at k-2, k-1, k) -- the order of the paper's
// red-then-blue sweep, site by site.
//
// Lanes.  A lane owns a pair of sites (x = 2m, 2m+1) of one row y: one of them is
// red and one blue in every plane, so every lane works at every step.  At step k
// the lane updates half p = (y+k)&1 of its pair: red at plane k, blue at plane
// k-1 (the same x).  Neighbours along z are the lane's own registers; in-plane
// neighbours (x+-1 across pairs, y+-1) come from the other lanes through LDS, one
// barrier per step, two buffer sets so that a step's writes never meet the
// previous step's reads.
//
// Tiles.  Lanes cover the tile's tile_x x tile_y pairs plus a ring: one pair each
// side in x and two rows each side in y.  Old spins are read from one buffer and
// new spins written to the other, so a tile never sees a neighbour tile's writes;
// the red sites one step outside the tile, which its blue sites need, are
// recomputed from old spins -- bit-identical to what the owning tile computes,
// because a site's random number depends only on (stream, site, sweep).  A z-chunk
// likewise recomputes the red plane below and above it.
//
// Launch.  One workgroup per (tile, z-chunk); block ids are spread so that
// consecutive tiles land on the same XCD (blocks are dealt to the 8 XCDs round
// robin), where their shared ring rows meet in the same L2.
#include "sg_internal.h"

namespace sg {
namespace {

struct FusedParams {
    const uint64_t *J;
    const uint64_t *src[2];
    uint64_t *dst[2];
    const uint32_t *rnd[2];
    int L, P;            // side, pairs per row
    int TXp, TY, ZC;     // tile: pairs, rows, planes
    int EX, EY;          // lanes per tile row (TXp + 2), tile rows incl. ring (TY + 4)
    int ntx, nty, nzc;   // tiles along x, y, z
    uint32_t a;          // MINSTD multiplier of this sweep
    Thresholds T;
};

template <int NREP>
struct Plane {
    uint64_t slo[NREP], shi[NREP];
    uint64_t jxlo, jxhi, jylo, jyhi, jzlo, jzhi;
    uint32_t rlo[NREP], rhi[NREP];
};

template <int NREP>
__device__ __forceinline__ void load_plane(const FusedParams &p, int64_t off, int64_t V, bool lane, bool full,
                                           Plane<NREP> &d)
{
#pragma unroll
    for (int r = 0; r < NREP; ++r) {
        d.slo[r] = 0;
        d.shi[r] = 0;
        d.rlo[r] = 0;
        d.rhi[r] = 0;
    }
    d.jxlo = d.jxhi = d.jylo = d.jyhi = d.jzlo = d.jzhi = 0;
    if (lane) {
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(p.src[r] + off);
            d.slo[r] = v.x;
            d.shi[r] = v.y;
        }
        const ulonglong2 jy = *reinterpret_cast<const ulonglong2 *>(p.J + V + off);
        d.jylo = jy.x;
        d.jyhi = jy.y;
    }
    if (full) {
        const ulonglong2 jx = *reinterpret_cast<const ulonglong2 *>(p.J + off);
        const ulonglong2 jz = *reinterpret_cast<const ulonglong2 *>(p.J + 2 * V + off);
        d.jxlo = jx.x;
        d.jxhi = jx.y;
        d.jzlo = jz.x;
        d.jzhi = jz.y;
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            const uint2 rr = *reinterpret_cast<const uint2 *>(p.rnd[r] + off);
            d.rlo[r] = rr.x;
            d.rhi[r] = rr.y;
        }
    }
}

__device__ __forceinline__ uint64_t pick(bool c, uint64_t a, uint64_t b) { return c ? a : b; }

// Largest workgroup per replica count: two replicas hold twice the spin state, so
// they get a 512-lane bound and with it up to 256 registers per lane.
template <int NREP>
struct MaxThreads {
    static constexpr int value = NREP == 1 ? 1024 : 512;
};

template <int PRNG, int NREP>
__global__ __launch_bounds__(MaxThreads<NREP>::value) void k_fused(FusedParams p)
{
    extern __shared__ uint64_t lds[];
    const int nl = p.EX * p.EY;
    // one LDS set: blue_old[NREP][nl], red_new[NREP][nl], jx_hi[nl], jy_lo[nl], jy_hi[nl]
    const int set_words = nl * (2 * NREP + 3);

    // ---- tile of this workgroup ---------------------------------------------
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int tile = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int ty = tile % p.nty;
    const int rest = tile / p.nty;
    const int tx = rest % p.ntx;
    const int zc = rest / p.ntx;
    const int TXe = min(p.TXp, p.P - tx * p.TXp);
    const int TYe = min(p.TY, p.L - ty * p.TY);
    const int z0 = zc * p.ZC;
    const int ZCe = min(p.ZC, p.L - z0);

    // ---- lane roles -----------------------------------------------------------
    const int lid = threadIdx.x;
    const bool lane = lid < nl;
    const int ex = lane ? lid % p.EX : 0;
    const int ey = lane ? lid / p.EX : 0;
    const bool full = lane && ey >= 1 && ey <= TYe + 2;  // rows whose red sites are computed
    const bool inter = lane && ex >= 1 && ex <= TXe && ey >= 2 && ey <= TYe + 1;
    const int m = (tx * p.TXp + ex - 1 + p.P) % p.P;
    const int y = (ty * p.TY + ey - 2 + p.L) % p.L;
    const int me = lane ? lid : 0;
    const int ixm = ey * p.EX + max(ex - 1, 0);
    const int ixp = ey * p.EX + min(ex + 1, p.EX - 1);
    const int iym = max(ey - 1, 0) * p.EX + ex;
    const int iyp = min(ey + 1, p.EY - 1) * p.EX + ex;

    const int L = p.L;
    const int64_t LL = (int64_t)L * L;
    const int64_t V = LL * L;
    const int64_t col = (int64_t)y * L + 2 * m;
    auto plane_off = [&](int q) -> int64_t {
        int qq = q % L;
        qq = qq < 0 ? qq + L : qq;
        return (int64_t)qq * LL + col;
    };

    // ---- prologue: planes z0-2 .. z0+1 ------------------------------------------
    const int kfirst = z0 - 1;
    const int klast = z0 + ZCe;
    Plane<NREP> A, B, C, D;  // planes k-1, k, k+1, k+2
    load_plane<NREP>(p, plane_off(kfirst - 1), V, lane, full, A);
    load_plane<NREP>(p, plane_off(kfirst), V, lane, full, B);
    load_plane<NREP>(p, plane_off(kfirst + 1), V, lane, full, C);
    load_plane<NREP>(p, plane_off(kfirst + 2), V, lane, full, D);

    uint64_t jzm2lo = 0, jzm2hi = 0;         // jz of plane k-2
    uint64_t jxl_prev = 0, jyulo_prev = 0, jyuhi_prev = 0;  // neighbour couplings of plane k-1
    uint64_t rn1[NREP], rn2[NREP];           // new red words of planes k-1, k-2
#pragma unroll
    for (int r = 0; r < NREP; ++r)
        rn1[r] = rn2[r] = 0;

    {
        // publish plane kfirst: its blue words and its couplings
        uint64_t *S = lds + ((kfirst + 2) & 1) * set_words;
        const bool pk = ((y + kfirst + L) & 1) != 0;
        if (lane) {
#pragma unroll
            for (int r = 0; r < NREP; ++r)
                S[r * nl + me] = pick(pk, B.slo[r], B.shi[r]);
            S[2 * NREP * nl + me] = B.jxhi;
            S[(2 * NREP + 1) * nl + me] = B.jylo;
            S[(2 * NREP + 2) * nl + me] = B.jyhi;
        }
    }
    __syncthreads();

    for (int k = kfirst; k <= klast; ++k) {
        const bool pk = ((y + k + L) & 1) != 0;  // half updated at this step
        const uint64_t *S = lds + ((k + 2) & 1) * set_words;
        const int ixn = pk ? ixp : ixm;

        // ---- neighbours from LDS --------------------------------------------------
        uint64_t nbx_b[NREP], nym_b[NREP], nyp_b[NREP];
        uint64_t nbx_r[NREP], nym_r[NREP], nyp_r[NREP];
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            nbx_b[r] = S[r * nl + ixn];
            nym_b[r] = S[r * nl + iym];
            nyp_b[r] = S[r * nl + iyp];
            nbx_r[r] = S[(NREP + r) * nl + ixn];
            nym_r[r] = S[(NREP + r) * nl + iym];
            nyp_r[r] = S[(NREP + r) * nl + iyp];
        }
        const uint64_t jxl = S[2 * NREP * nl + ixm];
        const uint64_t jyulo = S[(2 * NREP + 1) * nl + iym];
        const uint64_t jyuhi = S[(2 * NREP + 2) * nl + iym];

        // ---- red sites of plane k -----------------------------------------------
        uint64_t rn[NREP];
        {
            const uint64_t jxp = pick(pk, B.jxhi, B.jxlo);
            const uint64_t jxm = pick(pk, B.jxlo, jxl);
            const uint64_t jyp = pick(pk, B.jyhi, B.jylo);
            const uint64_t jym = pick(pk, jyuhi, jyulo);
            const uint64_t jzp = pick(pk, B.jzhi, B.jzlo);
            const uint64_t jzm = pick(pk, A.jzhi, A.jzlo);
#pragma unroll
            for (int r = 0; r < NREP; ++r) {
                const uint64_t s = pick(pk, B.shi[r], B.slo[r]);
                const uint64_t other = pick(pk, B.slo[r], B.shi[r]);
                const uint64_t nxp = pick(pk, nbx_b[r], other);
                const uint64_t nxm = pick(pk, other, nbx_b[r]);
                const uint64_t nzp = pick(pk, C.shi[r], C.slo[r]);
                const uint64_t nzm = pick(pk, A.shi[r], A.slo[r]);
                uint32_t R = pk ? B.rhi[r] : B.rlo[r];
                if (PRNG == SG_MINSTD)
                    R = minstd_jump(p.a, R);
                rn[r] = s ^ flip_mask(s, nxp, nyp_b[r], nzp, nxm, nym_b[r], nzm, jxp, jyp, jzp, jxm, jym, jzm,
                                      R, p.T);
            }
        }

        // ---- blue sites of plane k-1 ----------------------------------------------
        if (k >= z0 + 1) {
            const uint64_t jxp = pick(pk, A.jxhi, A.jxlo);
            const uint64_t jxm = pick(pk, A.jxlo, jxl_prev);
            const uint64_t jyp = pick(pk, A.jyhi, A.jylo);
            const uint64_t jym = pick(pk, jyuhi_prev, jyulo_prev);
            const uint64_t jzp = pick(pk, A.jzhi, A.jzlo);
            const uint64_t jzm = pick(pk, jzm2hi, jzm2lo);
            const int64_t off = plane_off(k - 1);
#pragma unroll
            for (int r = 0; r < NREP; ++r) {
                const uint64_t s = pick(pk, A.shi[r], A.slo[r]);
                const uint64_t nxp = pick(pk, nbx_r[r], rn1[r]);
                const uint64_t nxm = pick(pk, rn1[r], nbx_r[r]);
                uint32_t R = pk ? A.rhi[r] : A.rlo[r];
                if (PRNG == SG_MINSTD)
                    R = minstd_jump(p.a, R);
                const uint64_t bn = s ^ flip_mask(s, nxp, nyp_r[r], rn[r], nxm, nym_r[r], rn2[r], jxp, jyp, jzp, jxm,
                                                  jym, jzm, R, p.T);
                if (inter) {
                    ulonglong2 w;
                    w.x = pk ? rn1[r] : bn;
                    w.y = pk ? bn : rn1[r];
                    *reinterpret_cast<ulonglong2 *>(p.dst[r] + off) = w;
                }
            }
        }

        // ---- publish for step k+1: new red of plane k, old blue and couplings of k+1
        if (k < klast) {
            uint64_t *W = lds + ((k + 3) & 1) * set_words;
            if (lane) {
#pragma unroll
                for (int r = 0; r < NREP; ++r) {
                    W[r * nl + me] = pick(pk, C.shi[r], C.slo[r]);
                    W[(NREP + r) * nl + me] = rn[r];
                }
                W[2 * NREP * nl + me] = C.jxhi;
                W[(2 * NREP + 1) * nl + me] = C.jylo;
                W[(2 * NREP + 2) * nl + me] = C.jyhi;
            }
            __syncthreads();
        }

        // ---- rotate the plane pipeline ------------------------------------------------
        jzm2lo = A.jzlo;
        jzm2hi = A.jzhi;
        jxl_prev = jxl;
        jyulo_prev = jyulo;
        jyuhi_prev = jyuhi;
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            rn2[r] = rn1[r];
            rn1[r] = rn[r];
        }
        A = B;
        B = C;
        C = D;
        if (k + 3 <= klast + 1)
            load_plane<NREP>(p, plane_off(k + 3), V, lane, full, D);
    }
}

}  // namespace

static size_t fused_lds_bytes(int nrep, int tile_x, int tile_y)
{
    return (size_t)2 * (tile_x + 2) * (tile_y + 4) * (2 * nrep + 3) * sizeof(uint64_t);
}

static int max_threads(int nrep) { return nrep == 1 ? MaxThreads<1>::value : MaxThreads<2>::value; }

static int max_lds_bytes();

bool fused_shape_ok(int L, int nrep, int tile_x, int tile_y, int z_chunk)
{
    if (L < 2 || (L & 1) || nrep < 1 || nrep > 2)
        return false;
    const int P = L / 2;
    if (tile_x < 1 || tile_x > P || tile_y < 1 || tile_y > L || z_chunk < 1 || z_chunk > L)
        return false;
    const int lanes = (tile_x + 2) * (tile_y + 4);
    if ((lanes + 63) / 64 * 64 > max_threads(nrep))
        return false;
    if (fused_lds_bytes(nrep, tile_x, tile_y) > (size_t)max_lds_bytes())
        return false;
    return true;
}

static int max_lds_bytes()
{
    // dynamic LDS is kept within 64 KB per workgroup
    static int v = -1;
    if (v < 0) {
        int dev = 0, x = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || x <= 0)
            x = 65536;
        v = x < 65536 ? x : 65536;
    }
    return v;
}

void fused_default_shape(int L, int nrep, int &tile_x, int &tile_y, int &z_chunk)
{
    // Pick the tile that needs the fewest lanes (whole waves, ragged tiles
    // included) per pair of the lattice plane.
    const int P = L / 2;
    double best = 1e30;
    tile_x = 1;
    tile_y = 1;
    for (int tx = 1; tx <= P && tx <= 126; ++tx)
        for (int ty = 1; ty <= L && ty <= 252; ++ty) {
            const int lanes = (tx + 2) * (ty + 4);
            const int threads = (lanes + 63) / 64 * 64;
            if (threads > max_threads(nrep) || fused_lds_bytes(nrep, tx, ty) > (size_t)max_lds_bytes())
                continue;
            const int64_t ntx = (P + tx - 1) / tx, nty = (L + ty - 1) / ty;
            const double cost = (double)(ntx * nty * threads) / ((double)P * L);
            if (cost < best - 1e-9 || (cost < best + 1e-9 && lanes > (tile_x + 2) * (tile_y + 4))) {
                best = cost;
                tile_x = tx;
                tile_y = ty;
            }
        }
    // z chunks: enough workgroups to fill 256 CUs a few times over, chunks of at
    // least 16 planes (each chunk recomputes two red planes and loads four extra)
    const int64_t tiles = (int64_t)((P + tile_x - 1) / tile_x) * ((L + tile_y - 1) / tile_y);
    int zc = L;
    while (zc >= 32 && tiles * ((L + zc - 1) / zc) < 1024)
        zc = (zc + 1) / 2;
    z_chunk = zc;
}

hipError_t launch_sweep_fused(const SweepArgs &a, int tile_x, int tile_y, int z_chunk, hipStream_t s)
{
    FusedParams p;
    p.J = a.J;
    for (int r = 0; r < 2; ++r) {
        p.src[r] = a.src[r];
        p.dst[r] = a.dst[r];
        p.rnd[r] = a.rnd[r];
    }
    p.L = a.L;
    p.P = a.L / 2;
    p.TXp = tile_x;
    p.TY = tile_y;
    p.ZC = z_chunk;
    p.EX = tile_x + 2;
    p.EY = tile_y + 4;
    p.ntx = (p.P + tile_x - 1) / tile_x;
    p.nty = (p.L + tile_y - 1) / tile_y;
    p.nzc = (p.L + z_chunk - 1) / z_chunk;
    p.a = a.minstd_a;
    p.T = a.T;
    const int nl = p.EX * p.EY;
    const int threads = (nl + 63) / 64 * 64;
    const size_t lds = fused_lds_bytes(a.nrep, tile_x, tile_y);
    if (threads > max_threads(a.nrep) || lds > (size_t)max_lds_bytes())
        return hipErrorInvalidConfiguration;
    const int64_t blocks = (int64_t)p.ntx * p.nty * p.nzc;
    if (blocks < 1 || blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks), block((unsigned)threads);
    if (a.nrep == 1) {
        if (a.prng == SG_MINSTD)
            hipLaunchKernelGGL((k_fused<SG_MINSTD, 1>), grid, block, lds, s, p);
        else
            hipLaunchKernelGGL((k_fused<SG_MT19937, 1>), grid, block, lds, s, p);
    } else {
        if (a.prng == SG_MINSTD)
            hipLaunchKernelGGL((k_fused<SG_MINSTD, 2>), grid, block, lds, s, p);
        else
            hipLaunchKernelGGL((k_fused<SG_MT19937, 2>), grid, block, lds, s, p);
    }
    return hipGetLastError();
}

}  // namespace sg
