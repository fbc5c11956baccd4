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
// Launch.  One workgroup per (tile, z-chunk); block ids are spread so that as many
// consecutive tiles as an XCD holds workgroups land on the same XCD (blocks are
// dealt to the 8 XCDs round robin), and tiles are numbered in column-major blocks
// a few tiles tall, so the workgroups resident on an XCD together cover a compact
// block of the plane, next to the blocks the other XCDs run at the same time.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>

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
    int WE;              // waves holding the even tile rows
    int WO[2];           // two sweeps per launch: waves of outer ring rows, even and odd class
    int band;            // tile rows per group of the tile order
    int xgroup;          // consecutive work items given to one XCD in turn (its resident workgroups)
    uint32_t a;          // MINSTD multiplier of this sweep
    uint32_t a2;         // two sweeps per launch: multiplier of the second sweep
    int nrep;            // two sweeps per launch: replicas, one per workgroup (interleaved items)
    uint32_t mk[2];      // MINSTD key per replica
    uint64_t pkey[2];    // per-sample numbers (SG_PHILOX): key per replica
    int64_t t;           // sweep index of the (first) sweep of this launch
    Thresholds T;
};

template <int NREP>
struct Plane {
    uint64_t slo[NREP], shi[NREP];
    uint64_t jxlo, jxhi, jylo, jyhi, jzlo, jzhi;
    uint32_t rlo[NREP], rhi[NREP];  // buffered draws of the (first) sweep
    uint32_t r2lo, r2hi;            // two-sweep march: buffered draws of the second sweep
};

// Raw buffer access.  A plane of an array gets its own descriptor (base = the
// plane, size = the plane's bytes), so 32-bit offsets suffice at any L; a lane
// that must not touch memory uses an offset past the end, which the hardware
// turns into a dropped store or a zero load.  Every load and store of the march
// is then issued unconditionally and in a fixed order, which lets the compiler
// wait for exactly the plane a step needs while later planes are in flight.
constexpr uint32_t kOOB = 0x80000000u;
constexpr int kRsrcFlags = 0x00020000;  // raw 32-bit buffer format word of gfx9 descriptors
constexpr int kStoreDevice = 16;         // cache policy sc1: a store coherent at device scope

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, int64_t byte_off, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(static_cast<const char *>(base)) + byte_off,
                                             (short)0, (int)nbytes, kRsrcFlags);
}

__device__ __forceinline__ void ld_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t &lo, uint64_t &hi)
{
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    lo = (uint64_t)v.x | ((uint64_t)v.y << 32);
    hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
}

// AUX is the store's cache policy: 0 for the sweeps of a launch (the kernel's end
// makes them visible), kStoreDevice where other workgroups read the words in the
// same launch (the persistent batch kernel).
template <int AUX>
__device__ __forceinline__ void st_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t lo, uint64_t hi)
{
    u32x4 v;
    v.x = (uint32_t)lo;
    v.y = (uint32_t)(lo >> 32);
    v.z = (uint32_t)hi;
    v.w = (uint32_t)(hi >> 32);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, AUX);
}

// Per-lane byte offsets inside a plane (kOOB where the lane reads nothing).
struct Offsets {
    uint32_t s;   // spins and J[y]: every lane of the tile
    uint32_t f;   // J[x], J[z]: lanes whose red sites are computed
    uint32_t r;   // random-stream words (4 bytes per site)
};

template <int PRNG, int NREP>
__device__ __forceinline__ void load_plane(const FusedParams &p, int q, const Offsets &o, Plane<NREP> &d)
{
    const int64_t LL = (int64_t)p.L * p.L;
    const int64_t V = LL * p.L;
    const uint32_t pb = (uint32_t)(LL * 8);
    const int64_t qo = (int64_t)q * LL * 8;
#pragma unroll
    for (int r = 0; r < NREP; ++r)
        ld_pair(plane_rsrc(p.src[r], qo, pb), o.s, d.slo[r], d.shi[r]);
    const int64_t Vj8 = coupling_stride(p.L) * 8;
    ld_pair(plane_rsrc(p.J, Vj8 + qo, pb), o.s, d.jylo, d.jyhi);
    ld_pair(plane_rsrc(p.J, qo, pb), o.f, d.jxlo, d.jxhi);
    ld_pair(plane_rsrc(p.J, 2 * Vj8 + qo, pb), o.f, d.jzlo, d.jzhi);
#pragma unroll
    for (int r = 0; r < NREP; ++r) {
        if (PRNG == SG_MT19937) {  // MINSTD draws are computed from the site, nothing to load
            const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(p.rnd[r], (int64_t)q * LL * 4, pb / 2),
                                                                o.r, 0, 0);
            d.rlo[r] = v.x;
            d.rhi[r] = v.y;
        } else {
            d.rlo[r] = d.rhi[r] = 0;
        }
    }
}

// New word of one site: with SG_PHILOX every sample draws its own number, keyed
// by the site index (plane z, in-plane index xy) and the sweep; otherwise R is the
// site's number.  Fold picks the counter form of flip_site.
template <int PRNG, bool Fold = false>
__device__ __forceinline__ uint64_t site_update(const FusedParams &p, int r, int64_t sweep, uint32_t z, uint32_t xy,
                                                uint32_t R, uint64_t s, uint64_t nxp, uint64_t nyp, uint64_t nzp,
                                                uint64_t nxm, uint64_t nym, uint64_t nzm, uint64_t jxp, uint64_t jyp,
                                                uint64_t jzp, uint64_t jxm, uint64_t jym, uint64_t jzm)
{
    if (PRNG == SG_PHILOX) {
        const uint64_t site = (uint64_t)z * ((uint64_t)p.L * (uint64_t)p.L) + xy;
        return flip_site_ps(s, nxp, nyp, nzp, nxm, nym, nzm, jxp, jyp, jzp, jxm, jym, jzm, site, (uint64_t)sweep,
                            (uint32_t)p.pkey[r], (uint32_t)(p.pkey[r] >> 32), p.T);
    }
    return flip_site<PRNG == SG_MINSTD, Fold>(s, nxp, nyp, nzp, nxm, nym, nzm, jxp, jyp, jzp, jxm, jym, jzm, R, p.T);
}

// Loads of one plane given its byte offset qo = plane * L*L * 8 (draw-buffered
// generators excluded: their numbers are not read by the two-sweep march).
template <int PRNG>
__device__ __forceinline__ void load_plane_at(const FusedParams &p, int64_t qo, const Offsets &o, Plane<1> &d)
{
    const int64_t LL8 = (int64_t)p.L * p.L * 8;
    const int64_t V8 = LL8 * p.L;
    const uint32_t pb = (uint32_t)LL8;
    ld_pair(plane_rsrc(p.src[0], qo, pb), o.s, d.slo[0], d.shi[0]);
    const int64_t Vj8 = coupling_stride(p.L) * 8;
    ld_pair(plane_rsrc(p.J, Vj8 + qo, pb), o.s, d.jylo, d.jyhi);
    ld_pair(plane_rsrc(p.J, qo, pb), o.f, d.jxlo, d.jxhi);
    ld_pair(plane_rsrc(p.J, 2 * Vj8 + qo, pb), o.f, d.jzlo, d.jzhi);
    if (PRNG == SG_MT19937) {  // buffered draws of both sweeps, 4 bytes per site each
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(p.rnd[0], qo / 2, pb / 2), o.r, 0, 0);
        const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(p.rnd[0], V8 / 2 + qo / 2, pb / 2), o.r, 0, 0);
        d.rlo[0] = v.x;
        d.rhi[0] = v.y;
        d.r2lo = w.x;
        d.r2hi = w.y;
    } else {
        d.rlo[0] = d.rhi[0] = d.r2lo = d.r2hi = 0;
    }
}

// Half H of a pair: 0 = even x, 1 = odd x.
template <int H, int NREP>
__device__ __forceinline__ uint64_t sp(const Plane<NREP> &d, int r) { return H ? d.shi[r] : d.slo[r]; }

// Lane-constant data of the march.
struct Lane {
    int nl, set_words;
    int me, ixm, ixp, iym, iyp;
    bool lane;
    uint32_t col;  // in-plane index of the lane's even site, x + L*y
};

// Values carried from one step to the next.
template <int NREP>
struct Carry {
    uint64_t jzm2lo, jzm2hi;                 // jz of plane k-2
    uint64_t jxl, jyulo, jyuhi;              // neighbour couplings of plane k-1 (read at step k-1)
    uint64_t rn1[NREP], rn2[NREP];           // new red words of planes k-1, k-2
    uint32_t zk1[NREP];                      // MINSTD plane key of plane k-1
};

// Step k of the march with the lane's half H = (y + k) & 1 known at compile time:
// red of plane k (pair half H), then blue of plane k-1 (half H), then publish the
// words the neighbours need at step k+1.  A, B, C hold planes k-1, k, k+1.
template <int PRNG, int NREP, int H>
__device__ __forceinline__ void fused_step(const FusedParams &p, const Lane &c, uint64_t *lds, int k, bool do_blue,
                                           bool do_publish, const Plane<NREP> &A, const Plane<NREP> &B,
                                           const Plane<NREP> &C, Carry<NREP> &cy, const uint32_t (&zk)[NREP],
                                           uint32_t zr, uint32_t zb, uint64_t (&rn)[NREP], uint64_t (&wlo)[NREP],
                                           uint64_t (&whi)[NREP], uint64_t &jxl, uint64_t &jyulo, uint64_t &jyuhi)
{
    const uint64_t *S = lds + ((k + 2) & 1) * c.set_words;
    const int ixn = H ? c.ixp : c.ixm;  // lane holding the x-neighbour outside the pair
    jxl = S[2 * NREP * c.nl + c.ixm];
    jyulo = S[(2 * NREP + 1) * c.nl + c.iym];
    jyuhi = S[(2 * NREP + 2) * c.nl + c.iym];

    // ---- red site of plane k: x = 2m + H -----------------------------------------
    {
        const uint64_t jxp = H ? B.jxhi : B.jxlo;
        const uint64_t jxm = H ? B.jxlo : jxl;
        const uint64_t jyp = H ? B.jyhi : B.jylo;
        const uint64_t jym = H ? jyuhi : jyulo;
        const uint64_t jzp = H ? B.jzhi : B.jzlo;
        const uint64_t jzm = H ? A.jzhi : A.jzlo;
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            const uint64_t nbx = S[r * c.nl + ixn];
            const uint64_t nym = S[r * c.nl + c.iym];
            const uint64_t nyp = S[r * c.nl + c.iyp];
            const uint64_t s = sp<H>(B, r);
            const uint64_t other = sp<1 - H>(B, r);
            const uint64_t nxp = H ? nbx : other;
            const uint64_t nxm = H ? other : nbx;
            const uint32_t R = (PRNG == SG_MINSTD) ? minstd_jump(p.a, minstd_seed(c.col + H, zk[r]))
                                                   : (H ? B.rhi[r] : B.rlo[r]);
            rn[r] = site_update<PRNG>(p, r, p.t, zr, c.col + H, R, s, nxp, nyp, sp<H>(C, r), nxm, nym, sp<H>(A, r),
                                      jxp, jyp, jzp, jxm, jym, jzm);
        }
    }

    // ---- blue site of plane k-1: same x; its neighbours are all new red ------------
    if (do_blue) {
        const uint64_t jxp = H ? A.jxhi : A.jxlo;
        const uint64_t jxm = H ? A.jxlo : cy.jxl;
        const uint64_t jyp = H ? A.jyhi : A.jylo;
        const uint64_t jym = H ? cy.jyuhi : cy.jyulo;
        const uint64_t jzp = H ? A.jzhi : A.jzlo;
        const uint64_t jzm = H ? cy.jzm2hi : cy.jzm2lo;
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            const uint64_t nbx = S[(NREP + r) * c.nl + ixn];
            const uint64_t nym = S[(NREP + r) * c.nl + c.iym];
            const uint64_t nyp = S[(NREP + r) * c.nl + c.iyp];
            const uint64_t s = sp<H>(A, r);
            const uint64_t nxp = H ? nbx : cy.rn1[r];
            const uint64_t nxm = H ? cy.rn1[r] : nbx;
            const uint32_t R = (PRNG == SG_MINSTD) ? minstd_jump(p.a, minstd_seed(c.col + H, cy.zk1[r]))
                                                   : (H ? A.rhi[r] : A.rlo[r]);
            const uint64_t bn = site_update<PRNG>(p, r, p.t, zb, c.col + H, R, s, nxp, nyp, rn[r], nxm, nym,
                                                  cy.rn2[r], jxp, jyp, jzp, jxm, jym, jzm);
            wlo[r] = H ? cy.rn1[r] : bn;
            whi[r] = H ? bn : cy.rn1[r];
        }
    }

    // ---- publish: new red of plane k, old blue (half H) and couplings of k+1 ------
    if (do_publish) {
        uint64_t *W = lds + ((k + 3) & 1) * c.set_words;
#pragma unroll
        for (int r = 0; r < NREP; ++r) {
            W[r * c.nl + c.me] = sp<H>(C, r);
            W[(NREP + r) * c.nl + c.me] = rn[r];
        }
        W[2 * NREP * c.nl + c.me] = C.jxhi;
        W[(2 * NREP + 1) * c.nl + c.me] = C.jylo;
        W[(2 * NREP + 2) * c.nl + c.me] = C.jyhi;
    }
}

// Largest workgroup: 512 lanes, so that two workgroups can share a CU.
constexpr int kMaxThreads = 512;

template <int I>
using IC = std::integral_constant<int, I>;

// Planes in flight: a ring of NS planes holds k-1 .. k+NS-2 at step k, so a plane is
// requested NS-3 steps before the step that first reads it.
// Six planes for one replica; two replicas hold twice the spins, five planes.
template <int NREP>
struct Ring {
    static constexpr int value = NREP == 1 ? 6 : 5;
};

// The march of one tile: tile = tile index within the lattice (z chunk major).
template <int PRNG, int NREP, int SAUX, int... Is>
__device__ __forceinline__ void fused_march(const FusedParams &p, const int tile, uint64_t *lds,
                                            std::integer_sequence<int, Is...>)
{
    constexpr int NS = sizeof...(Is);
    Lane c;
    // one LDS set: blue_old[NREP], red_new[NREP], jx_hi, jy_lo, jy_hi, each with a slot
    // per tile lane plus one that threads outside the tile write, so that every
    // thread publishes without a branch
    c.nl = p.EX * p.EY + 1;
    c.set_words = c.nl * (2 * NREP + 3);

    // ---- tile of this workgroup ---------------------------------------------
    // Tile order within a z chunk: groups of `band` tile rows; inside a group the
    // tiles go down a column of the group, then to the next column.  The workgroups
    // that run together on one XCD then form a block `band` tiles tall, whose
    // inner ring rows are read once into that XCD's L2.
    const int per_chunk = p.ntx * p.nty;
    const int zc = tile / per_chunk;
    const int r0 = tile - zc * per_chunk;
    const int g = r0 / (p.ntx * p.band);
    const int gh = min(p.band, p.nty - g * p.band);  // tile rows in this group
    const int q0 = r0 - g * p.ntx * p.band;
    const int tx = q0 / gh;
    const int ty = g * p.band + (q0 - tx * gh);
    const int TXe = min(p.TXp, p.P - tx * p.TXp);
    const int TYe = min(p.TY, p.L - ty * p.TY);
    const int z0 = zc * p.ZC;
    const int ZCe = min(p.ZC, p.L - z0);

    // ---- lanes: waves hold tile rows of one parity (even rows first) ---------------
    // so the pair half a lane updates, (y + k) & 1, is the same across its wave.
    const int lid = threadIdx.x;
    const int cls = lid < 64 * p.WE ? 0 : 1;
    const int idx = cls ? lid - 64 * p.WE : lid;
    const int rows_cls = cls ? p.EY / 2 : (p.EY + 1) / 2;
    c.lane = idx < p.EX * rows_cls;
    const int ex = c.lane ? idx % p.EX : 0;
    const int ey = c.lane ? 2 * (idx / p.EX) + cls : cls;
    const bool full = c.lane && ey >= 1 && ey <= TYe + 2;  // rows whose red sites are computed
    const bool inter = c.lane && ex >= 1 && ex <= TXe && ey >= 2 && ey <= TYe + 1;
    const int m = (tx * p.TXp + ex - 1 + p.P) % p.P;
    const int y = (ty * p.TY + ey - 2 + p.L) % p.L;
    c.me = c.lane ? ey * p.EX + ex : c.nl - 1;
    c.ixm = ey * p.EX + max(ex - 1, 0);
    c.ixp = ey * p.EX + min(ex + 1, p.EX - 1);
    c.iym = max(ey - 1, 0) * p.EX + ex;
    c.iyp = min(ey + 1, p.EY - 1) * p.EX + ex;
    // parity of the row, the same for the whole wave (L is even, so wrapping keeps it)
    const int ypar = __builtin_amdgcn_readfirstlane((ty * p.TY + ey) & 1);

    const int L = p.L;
    const int64_t LL = (int64_t)L * L;
    const uint32_t col = (uint32_t)y * (uint32_t)L + 2u * (uint32_t)m;  // site index within a plane
    c.col = col;
    Offsets o;
    o.s = c.lane ? col * 8u : kOOB;
    o.f = full ? col * 8u : kOOB;
    o.r = full ? col * 4u : kOOB;
    const uint32_t o_st = inter ? col * 8u : kOOB;
    Offsets o_none;  // past the last plane a chunk needs: loads issued, nothing read
    o_none.s = o_none.f = o_none.r = kOOB;
    auto wrap = [&](int q) -> int {  // q lies in [-2, 2L)
        return q < 0 ? q + L : (q >= L ? q - L : q);
    };

    // ---- prologue: planes z0-2 .. z0+1 --------------------------------------------
    const int kfirst = z0 - 1;
    const int klast = z0 + ZCe;
    Plane<NREP> ring[NS];  // ring[j] starts with plane kfirst - 1 + j
    ((load_plane<PRNG, NREP>(p, wrap(kfirst - 1 + Is), o, ring[Is])), ...);

    Carry<NREP> cy;
    cy.jzm2lo = cy.jzm2hi = cy.jxl = cy.jyulo = cy.jyuhi = 0;
#pragma unroll
    for (int r = 0; r < NREP; ++r) {
        cy.rn1[r] = cy.rn2[r] = 0;
        cy.zk1[r] = 0;
    }

    {
        // publish plane kfirst: its old blue words (half 1-H) and its couplings
        uint64_t *S = lds + ((kfirst + 2) & 1) * c.set_words;
        const bool hred = ((ypar + kfirst + L) & 1) != 0;
#pragma unroll
        for (int r = 0; r < NREP; ++r)
            S[r * c.nl + c.me] = hred ? ring[1].slo[r] : ring[1].shi[r];
        S[2 * NREP * c.nl + c.me] = ring[1].jxhi;
        S[(2 * NREP + 1) * c.nl + c.me] = ring[1].jylo;
        S[(2 * NREP + 2) * c.nl + c.me] = ring[1].jyhi;
    }
    __syncthreads();

    int k = kfirst;
    // One step with planes (A, B, C) = (k-1, k, k+1); the other ring slots hold
    // k+2 .. k+NS-2 in flight, and A's slot receives k+NS-1 at the end.  The steps
    // of one turn of the ring are unrolled, so it turns without register copies.
#define SG_FUSED_STEP(A, B, C)                                                                                   \
    {                                                                                                             \
        uint64_t rn[NREP], wlo[NREP], whi[NREP];                                                                  \
        _Pragma("unroll") for (int r = 0; r < NREP; ++r) wlo[r] = whi[r] = 0;                                    \
        uint64_t jxl, jyulo, jyuhi;                                                                               \
        const bool do_blue = k >= z0 + 1;                                                                         \
        const bool do_pub = k < klast;                                                                            \
        uint32_t zk[NREP];                                                                                        \
        _Pragma("unroll") for (int r = 0; r < NREP; ++r) zk[r] = minstd_plane_key((uint32_t)wrap(k), p.mk[r]);   \
        if ((ypar + k + L) & 1)                                                                                   \
            fused_step<PRNG, NREP, 1>(p, c, lds, k, do_blue, do_pub, A, B, C, cy, zk, (uint32_t)wrap(k),            \
                                      (uint32_t)wrap(k - 1), rn, wlo, whi, jxl, jyulo,                            \
                                      jyuhi);                                                                     \
        else                                                                                                      \
            fused_step<PRNG, NREP, 0>(p, c, lds, k, do_blue, do_pub, A, B, C, cy, zk, (uint32_t)wrap(k),            \
                                      (uint32_t)wrap(k - 1), rn, wlo, whi, jxl, jyulo,                            \
                                      jyuhi);                                                                     \
        {                                                                                                         \
            const int64_t qo = (int64_t)wrap(k - 1) * LL * 8;                                                     \
            const uint32_t ost = do_blue ? o_st : kOOB;                                                           \
            _Pragma("unroll") for (int r = 0; r < NREP; ++r)                                                     \
                st_pair<SAUX>(plane_rsrc(p.dst[r], qo, (uint32_t)(LL * 8)), ost, wlo[r], whi[r]);                       \
        }                                                                                                         \
        if (do_pub)                                                                                               \
            __syncthreads();                                                                                      \
        cy.jzm2lo = A.jzlo;                                                                                       \
        cy.jzm2hi = A.jzhi;                                                                                       \
        cy.jxl = jxl;                                                                                             \
        cy.jyulo = jyulo;                                                                                         \
        cy.jyuhi = jyuhi;                                                                                         \
        _Pragma("unroll") for (int r = 0; r < NREP; ++r)                                                         \
        {                                                                                                         \
            cy.rn2[r] = cy.rn1[r];                                                                                \
            cy.rn1[r] = rn[r];                                                                                    \
            cy.zk1[r] = zk[r];                                                                                    \
        }                                                                                                         \
        load_plane<PRNG, NREP>(p, wrap(k + NS - 1), (k + NS - 1 <= klast + 1) ? o : o_none, A);                 \
    }

    auto step = [&](auto I) -> bool {
        constexpr int i = decltype(I)::value;
        SG_FUSED_STEP(ring[i], ring[(i + 1) % NS], ring[(i + 2) % NS])
        return ++k <= klast;
    };
    while ((step(IC<Is>{}) && ...)) {
    }
#undef SG_FUSED_STEP
}

// Block b -> work item.  Blocks are dealt to the 8 XCDs round robin; here groups of
// G consecutive items go to one XCD in turn, G = the workgroups an XCD holds at
// once, so that those workgroups cover one compact block of tiles (their shared
// ring lines are read once into the XCD's L2) and the blocks of the eight XCDs
// running at the same time are neighbours (lines shared across XCDs are then read
// at about the same time, while the memory-side cache still holds them).  Grids
// below 8 G use groups of nb / 8; blocks past the last whole round keep their
// index.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_item(int b, int nb, int G)
{
    if (nb < 8 * G)
        G = nb / 8;
    if (G < 1)
        return b;
    const int full = nb / (8 * G) * (8 * G);
    if (b >= full)
        return b;
    const int x = b & 7, k = b >> 3;
    return ((k / G) * 8 + x) * G + k % G;
}

// Block b -> work item of a batch, whose items differ in length (lattices of
// different sides): groups of kBatchGroup consecutive items are dealt to the XCDs
// round robin, so every XCD gets a similar share of long and short items while the
// items running together on one XCD stay neighbours.  The grid is a multiple of
// kBatchQueues * kBatchGroup; this is a bijection of [0, grid).
static_assert(kBatchQueues == 8, "blocks are dealt to the 8 XCDs round robin");
__device__ __forceinline__ int xcd_group_item(int b)
{
    const int x = b & 7, k = b >> 3;
    return ((k / kBatchGroup) * 8 + x) * kBatchGroup + k % kBatchGroup;
}

template <int PRNG, int NREP>
__global__ __launch_bounds__(kMaxThreads) void k_fused(FusedParams p)
{
    extern __shared__ uint64_t lds[];
    fused_march<PRNG, NREP, 0>(p, xcd_item(blockIdx.x, gridDim.x, p.xgroup), lds,
                            std::make_integer_sequence<int, Ring<NREP>::value>{});
}

// 16807^(t+1) mod (2^31 - 1), by square and multiply (uniform, scalar unit).
__device__ __forceinline__ uint32_t minstd_power(int64_t t)
{
    uint64_t result = 1, base = 16807;
    uint64_t e = (uint64_t)t + 1;
    while (e) {
        if (e & 1) {
            const uint64_t q = result * base;
            result = (q & 0x7FFFFFFFull) + (q >> 31);
            result = result >= 0x7FFFFFFFull ? result - 0x7FFFFFFFull : result;
        }
        const uint64_t q = base * base;
        base = (q & 0x7FFFFFFFull) + (q >> 31);
        base = base >= 0x7FFFFFFFull ? base - 0x7FFFFFFFull : base;
        e >>= 1;
    }
    return (uint32_t)result;
}

__global__ void k_round_advance(int64_t *round_ctr)
{
    if (threadIdx.x == 0)
        round_ctr[threadIdx.x] += 1;
}

__global__ void k_round_reset(int64_t *round_ctr)
{
    if (threadIdx.x == 0)
        round_ctr[threadIdx.x] = 0;
}

// ===========================================================================
// Two sweeps per launch.
//
// The same z-march carries a second sweep two planes behind the first.  At step k
// a lane does, on its pair half H = (y + k) & 1:
//   first sweep:  red of plane k, blue of plane k-1        (as above)
//   second sweep: red of plane k-2, blue of plane k-3
// The second sweep's red at k-2 needs the first sweep's blue at k-3 .. k-1, done
// by then (blue k-1 a moment earlier in the same step); its blue at k-3 needs its
// own red at k-4 .. k-2.  Every site therefore sees exactly the neighbours of two
// consecutive sweeps, and only the second sweep's words are stored: spins and
// couplings cross HBM once per two sweeps.  The second sweep updates the same
// sites as the first did two steps earlier, so the coupling operands and the
// stream seed of those updates are kept for two steps instead of reloaded.
//
// The ring around the tile doubles: the second sweep's blue on the tile needs its
// red one step out, which needs the first sweep's blue two out, its red three out
// and the old spins four out.  Lanes cover the tile plus two pairs each side in x
// and four rows each side in y; a z chunk recomputes three planes below and above.
// ===========================================================================
constexpr int kF2OldBlue = 0, kF2Red = 1, kF2Jx = 2, kF2JyLo = 3, kF2JyHi = 4, kF2Blue = 5, kF2Red2 = 6;
constexpr int kF2Words = 7;  // LDS words per lane and buffer set

// Coupling operands and stream seed of one site update (MINSTD: the seed;
// SG_PHILOX: the site's plane, the numbers being keyed by the site).
struct SiteOps {
    uint64_t jxp, jyp, jzp, jxm, jym, jzm;
    uint32_t seed;  // MINSTD seed, Philox plane key, or the second sweep's buffered draw
};

struct Carry2 {
    uint64_t jzm2lo, jzm2hi;     // jz of plane k-2
    uint64_t jxl, jyulo, jyuhi;  // neighbour couplings of plane k-1
    uint64_t ar1, ar2;           // first sweep: new red of planes k-1, k-2
    uint64_t ab1, ab2;           // first sweep: new blue of planes k-2, k-3
    uint64_t br1, br2;           // second sweep: new red of planes k-3, k-4
    SiteOps r1, b1, r2, b2;      // first sweep's red / blue operands of steps k-1, k-2
};

template <int PRNG, int H, bool Fold>
__device__ __forceinline__ void fused2_step(const FusedParams &p, const Lane &c, uint64_t *lds, int k, bool do_ab,
                                            bool do_br, bool do_bb, bool do_pub, const Plane<1> &A,
                                            const Plane<1> &B, const Plane<1> &C, const Carry2 &cy, uint32_t zk,
                                            uint32_t zk1, uint32_t zr, uint32_t zb, uint64_t &ar0, uint64_t &ab0,
                                            uint64_t &br0, uint64_t &bb0, SiteOps &r0, SiteOps &b0, uint64_t &jxl,
                                            uint64_t &jyulo, uint64_t &jyuhi)
{
    const uint32_t xy = c.col + H;
    const uint64_t *S = lds + ((k + 2) & 1) * c.set_words;
    const int ixn = H ? c.ixp : c.ixm;  // lane holding the x-neighbour outside the pair
    const int nl = c.nl;
    jxl = S[kF2Jx * nl + c.ixm];
    jyulo = S[kF2JyLo * nl + c.iym];
    jyuhi = S[kF2JyHi * nl + c.iym];
    // In-plane neighbour words of the four updates.  The five-plane form reads all of
    // them before any update (one LDS round trip per step); the six-plane form reads
    // each update's words where they are used (the autotuner times both forms).
    constexpr int kSlot[4] = {kF2OldBlue, kF2Red, kF2Blue, kF2Red2};
    uint64_t nb[4][3];
    if (!Fold) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            nb[w][0] = S[kSlot[w] * nl + ixn];
            nb[w][1] = S[kSlot[w] * nl + c.iym];
            nb[w][2] = S[kSlot[w] * nl + c.iyp];
        }
    }
    auto words = [&](int w, uint64_t &x, uint64_t &ym, uint64_t &yp) {
        if (Fold) {
            x = S[kSlot[w] * nl + ixn];
            ym = S[kSlot[w] * nl + c.iym];
            yp = S[kSlot[w] * nl + c.iyp];
        } else {
            x = nb[w][0];
            ym = nb[w][1];
            yp = nb[w][2];
        }
    };

    // ---- first sweep, red of plane k -----------------------------------------
    r0.jxp = H ? B.jxhi : B.jxlo;
    r0.jxm = H ? B.jxlo : jxl;
    r0.jyp = H ? B.jyhi : B.jylo;
    r0.jym = H ? jyuhi : jyulo;
    r0.jzp = H ? B.jzhi : B.jzlo;
    r0.jzm = H ? A.jzhi : A.jzlo;
    // the number a site draws: MINSTD jumps its seed to the sweep, buffered draws
    // come with the plane (the second sweep's is carried in the seed slot)
    constexpr bool kBuf = PRNG == SG_MT19937;
    r0.seed = PRNG == SG_PHILOX ? zr : kBuf ? (H ? B.r2hi : B.r2lo) : minstd_seed(xy, zk);
    {
        uint64_t nbx, nym, nyp;
        words(0, nbx, nym, nyp);
        const uint64_t s = sp<H>(B, 0), other = sp<1 - H>(B, 0);
        const uint32_t R = kBuf ? (H ? B.rhi[0] : B.rlo[0]) : minstd_jump(p.a, r0.seed);
        ar0 = site_update<PRNG, Fold>(p, 0, p.t, r0.seed, xy, R, s, H ? nbx : other, nyp,
                                      sp<H>(C, 0), H ? other : nbx, nym, sp<H>(A, 0), r0.jxp, r0.jyp, r0.jzp, r0.jxm,
                                      r0.jym, r0.jzm);
    }

    // ---- first sweep, blue of plane k-1: neighbours are new red ----------------
    b0.jxp = H ? A.jxhi : A.jxlo;
    b0.jxm = H ? A.jxlo : cy.jxl;
    b0.jyp = H ? A.jyhi : A.jylo;
    b0.jym = H ? cy.jyuhi : cy.jyulo;
    b0.jzp = H ? A.jzhi : A.jzlo;
    b0.jzm = H ? cy.jzm2hi : cy.jzm2lo;
    b0.seed = PRNG == SG_PHILOX ? zb : kBuf ? (H ? A.r2hi : A.r2lo) : minstd_seed(xy, zk1);
    if (do_ab) {
        uint64_t nbx, nym, nyp;
        words(1, nbx, nym, nyp);
        const uint32_t R = kBuf ? (H ? A.rhi[0] : A.rlo[0]) : minstd_jump(p.a, b0.seed);
        ab0 = site_update<PRNG, Fold>(p, 0, p.t, b0.seed, xy, R, sp<H>(A, 0), H ? nbx : cy.ar1,
                                      nyp, ar0, H ? cy.ar1 : nbx, nym, cy.ar2, b0.jxp, b0.jyp, b0.jzp, b0.jxm, b0.jym,
                                      b0.jzm);
    }

    // ---- second sweep, red of plane k-2: neighbours are the first sweep's blue --
    if (do_br) {
        uint64_t nbx, nym, nyp;
        words(2, nbx, nym, nyp);
        const SiteOps &o = cy.r2;
        const uint32_t R = kBuf ? o.seed : minstd_jump(p.a2, o.seed);
        br0 = site_update<PRNG, Fold>(p, 0, p.t + 1, o.seed, xy, R, cy.ar2, H ? nbx : cy.ab1,
                                      nyp, ab0, H ? cy.ab1 : nbx, nym, cy.ab2, o.jxp, o.jyp, o.jzp, o.jxm, o.jym, o.jzm);
    }

    // ---- second sweep, blue of plane k-3: neighbours are its own new red --------
    if (do_bb) {
        uint64_t nbx, nym, nyp;
        words(3, nbx, nym, nyp);
        const SiteOps &o = cy.b2;
        const uint32_t R = kBuf ? o.seed : minstd_jump(p.a2, o.seed);
        bb0 = site_update<PRNG, Fold>(p, 0, p.t + 1, o.seed, xy, R, cy.ab2, H ? nbx : cy.br1,
                                      nyp, br0, H ? cy.br1 : nbx, nym, cy.br2, o.jxp, o.jyp, o.jzp, o.jxm, o.jym, o.jzm);
    }

    // ---- publish for step k+1 ----------------------------------------------------
    if (do_pub) {
        uint64_t *W = lds + ((k + 3) & 1) * c.set_words;
        W[kF2OldBlue * nl + c.me] = sp<H>(C, 0);
        W[kF2Red * nl + c.me] = ar0;
        W[kF2Jx * nl + c.me] = C.jxhi;
        W[kF2JyLo * nl + c.me] = C.jylo;
        W[kF2JyHi * nl + c.me] = C.jyhi;
        W[kF2Blue * nl + c.me] = ab0;
        W[kF2Red2 * nl + c.me] = br0;
    }
}

// Planes in flight for the two-sweep march (a plane is requested NS-2 steps before
// the step that first reads it): 5 or 6, chosen per lattice; batches use 5.
constexpr int kRing2Batch = 5;
template <int NS>
using Ring2Steps = std::make_integer_sequence<int, NS % 2 ? 2 * NS : NS>;  // unrolled steps per loop turn

// The march of one work item after its lanes are set up.  P0 = (row parity +
// first step) & 1 is the same for a whole wave; with an even ring the pair half
// of ring slot i is then (P0 + i) & 1, known at compile time, so the steps of a
// turn of the ring are straight-line code.
template <int PRNG, int P0, int NS, int SAUX, int... Is>
__device__ __forceinline__ void fused2_run(const FusedParams &p, const Lane &c, uint64_t *lds, const int z0,
                                           const int ZCe, const Offsets &o, const uint32_t o_st,
                                           const bool second, std::integer_sequence<int, Is...>)
{
    // Is enumerates the unrolled steps: one turn of an even ring, two of an odd one,
    // so that each unrolled step has a fixed ring slot and pair half.
    static_assert(sizeof...(Is) == (NS % 2 ? 2 * NS : NS), "one or two turns of the ring");
    const int L = p.L;
    const int64_t LL = (int64_t)L * L;
    Offsets o_none;
    o_none.s = o_none.f = o_none.r = kOOB;
    auto wrap = [&](int q) -> int {  // q lies in [-6, L+6), inside [-L, 2L) as L >= 8
        return q < 0 ? q + L : (q >= L ? q - L : q);
    };

    // first sweep's red runs over planes z0-3 .. z0+ZCe+2, reading old planes one beyond
    const int kfirst = z0 - 3;
    const int klast = z0 + ZCe + 2;
    const int64_t LL8 = LL * 8, V8 = LL8 * L;
    Plane<1> ring[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j)
        load_plane_at<PRNG>(p, (int64_t)wrap(kfirst - 1 + j) * LL8, o, ring[j]);
    // byte offsets of the next plane to load (k + NS - 1) and of the plane stored at
    // step k (k - 3), both advanced by one plane per step
    int64_t q_load = (int64_t)wrap(kfirst + NS - 1) * LL8;
    int64_t q_store = (int64_t)wrap(kfirst - 3) * LL8;

    Carry2 cy;
    cy.jzm2lo = cy.jzm2hi = cy.jxl = cy.jyulo = cy.jyuhi = 0;
    cy.ar1 = cy.ar2 = cy.ab1 = cy.ab2 = cy.br1 = cy.br2 = 0;
    cy.r1 = cy.b1 = cy.r2 = cy.b2 = SiteOps{0, 0, 0, 0, 0, 0, 0};

    {
        // publish plane kfirst: its old blue words (half 1-P0) and its couplings
        uint64_t *S = lds + ((kfirst + 2) & 1) * c.set_words;
        S[kF2OldBlue * c.nl + c.me] = P0 ? ring[1].slo[0] : ring[1].shi[0];
        S[kF2Jx * c.nl + c.me] = ring[1].jxhi;
        S[kF2JyLo * c.nl + c.me] = ring[1].jylo;
        S[kF2JyHi * c.nl + c.me] = ring[1].jyhi;
    }
    __syncthreads();

    int k = kfirst;
    uint32_t zk_prev = minstd_plane_key((uint32_t)wrap(kfirst - 1), p.mk[0]);
    // One step with ring slots (A, B, C) = planes (k-1, k, k+1); A's slot receives
    // plane k+NS-1 at the end.
    auto step = [&](auto I) -> bool {
        constexpr int i = decltype(I)::value;
        constexpr int H = (P0 + i) & 1;
        Plane<1> &A = ring[i % NS];
        const Plane<1> &B = ring[(i + 1) % NS];
        const Plane<1> &C = ring[(i + 2) % NS];
        uint64_t ar0 = 0, ab0 = 0, br0 = 0, bb0 = 0, jxl, jyulo, jyuhi;
        SiteOps r0, b0;
        const bool do_ab = k >= z0 - 1;
        const bool do_br = second && k >= z0 + 1;
        const bool do_bb = second && k >= z0 + 3;
        const bool do_pub = k < klast;
        const uint32_t zk = minstd_plane_key((uint32_t)wrap(k), p.mk[0]);
        const uint32_t zk1 = zk_prev;  // key of plane k-1, from the previous step
        zk_prev = zk;
        // six planes in flight count with the fold form, five with the shorter
        // three-input form; the autotuner times both
        constexpr bool kFold = NS == 6;
        fused2_step<PRNG, H, kFold>(p, c, lds, k, do_ab, do_br, do_bb, do_pub, A, B, C, cy, zk, zk1, (uint32_t)wrap(k),
                                    (uint32_t)wrap(k - 1), ar0, ab0, br0, bb0, r0, b0, jxl, jyulo, jyuhi);
        {
            const uint64_t wlo = H ? cy.br1 : bb0, whi = H ? bb0 : cy.br1;
            st_pair<SAUX>(plane_rsrc(p.dst[0], q_store, (uint32_t)LL8), do_bb ? o_st : kOOB, wlo, whi);
            q_store = q_store + LL8 == V8 ? 0 : q_store + LL8;
        }
        if (do_pub)
            __syncthreads();
        cy.jzm2lo = A.jzlo;
        cy.jzm2hi = A.jzhi;
        cy.jxl = jxl;
        cy.jyulo = jyulo;
        cy.jyuhi = jyuhi;
        cy.ar2 = cy.ar1;
        cy.ar1 = ar0;
        cy.ab2 = cy.ab1;
        cy.ab1 = ab0;
        cy.br2 = cy.br1;
        cy.br1 = br0;
        cy.r2 = cy.r1;
        cy.r1 = r0;
        cy.b2 = cy.b1;
        cy.b1 = b0;
        load_plane_at<PRNG>(p, q_load, (k + NS - 1 <= klast + 1) ? o : o_none, A);
        q_load = q_load + LL8 == V8 ? 0 : q_load + LL8;
        return ++k <= klast;
    };
    while ((step(IC<Is>{}) && ...)) {
    }
}

template <int PRNG, int NS, int SAUX, int... Is>
__device__ __forceinline__ void fused2_march(const FusedParams &pp, const int item, uint64_t *lds,
                                             std::integer_sequence<int, Is...> seq)
{
    // replicas are interleaved: consecutive items are the same tile of each replica
    const int rep = item % pp.nrep;
    const int tile = item / pp.nrep;
    FusedParams p = pp;
    p.src[0] = pp.src[rep];
    p.dst[0] = pp.dst[rep];
    p.rnd[0] = pp.rnd[rep];
    p.mk[0] = pp.mk[rep];
    p.pkey[0] = pp.pkey[rep];

    Lane c;
    c.nl = p.EX * p.EY + 1;
    c.set_words = c.nl * kF2Words;

    const int per_chunk = p.ntx * p.nty;
    const int zc = tile / per_chunk;
    const int r0 = tile - zc * per_chunk;
    const int g = r0 / (p.ntx * p.band);
    const int gh = min(p.band, p.nty - g * p.band);
    const int q0 = r0 - g * p.ntx * p.band;
    const int tx = q0 / gh;
    const int ty = g * p.band + (q0 - tx * gh);
    const int TXe = min(p.TXp, p.P - tx * p.TXp);
    const int TYe = min(p.TY, p.L - ty * p.TY);
    const int z0 = zc * p.ZC;
    const int ZCe = min(p.ZC, p.L - z0);

    // ---- lanes: waves hold tile rows of one parity (the even class first); within a
    // class the outer ring rows (two or more rows from the tile: 0..2 and EY-3..EY-1)
    // come first, in waves of their own, which skip the second sweep: it is needed
    // only up to one row from the tile.
    const int lid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(lid >> 6);
    const int cls = wave < p.WE ? 0 : 1;
    const int w = cls ? wave - p.WE : wave;
    const bool outer = w < p.WO[cls];
    const int idx = (outer ? w : w - p.WO[cls]) * 64 + (lid & 63);
    const int nbot = cls ? 1 : 2;                              // rows 0..2 of this parity
    const int t0 = ((p.EY - 3) & 1) == cls ? p.EY - 3 : p.EY - 2;  // first top outer row of this parity
    const int ntop = ((p.EY - 3) & 1) == cls ? 2 : 1;
    const int ifirst = cls ? 3 : 4;                            // first inner row of this parity
    const int nin = ifirst <= p.EY - 4 ? (p.EY - 4 - ifirst) / 2 + 1 : 0;
    const int rrow = idx / p.EX;
    c.lane = idx < p.EX * (outer ? nbot + ntop : nin);
    const int ex = c.lane ? idx - rrow * p.EX : 0;
    const int ey = !c.lane ? cls : (outer ? (rrow < nbot ? cls + 2 * rrow : t0 + 2 * (rrow - nbot)) : ifirst + 2 * rrow);
    const bool full = c.lane && ey >= 1 && ey <= TYe + 6;  // rows whose red sites are computed
    const bool inter = c.lane && ex >= 2 && ex <= TXe + 1 && ey >= 4 && ey <= TYe + 3;
    const int m = (tx * p.TXp + ex - 2 + 2 * p.P) % p.P;
    const int y = (ty * p.TY + ey - 4 + 4 * p.L) % p.L;
    c.me = c.lane ? ey * p.EX + ex : c.nl - 1;
    c.ixm = ey * p.EX + max(ex - 1, 0);
    c.ixp = ey * p.EX + min(ex + 1, p.EX - 1);
    c.iym = max(ey - 1, 0) * p.EX + ex;
    c.iyp = min(ey + 1, p.EY - 1) * p.EX + ex;
    const int ypar = __builtin_amdgcn_readfirstlane((ty * p.TY + ey) & 1);

    const uint32_t col = (uint32_t)y * (uint32_t)p.L + 2u * (uint32_t)m;
    c.col = col;
    Offsets o;
    o.s = c.lane ? col * 8u : kOOB;
    o.f = full ? col * 8u : kOOB;
    o.r = PRNG == SG_MT19937 && full ? col * 4u : kOOB;  // 4-byte draws
    const uint32_t o_st = inter ? col * 8u : kOOB;
    if ((ypar + z0 - 3 + p.L) & 1)
        fused2_run<PRNG, 1, NS, SAUX>(p, c, lds, z0, ZCe, o, o_st, !outer, seq);
    else
        fused2_run<PRNG, 0, NS, SAUX>(p, c, lds, z0, ZCe, o, o_st, !outer, seq);
}

template <int PRNG, int NS>
__global__ __launch_bounds__(kMaxThreads) void k_fused2(FusedParams p)
{
    extern __shared__ uint64_t lds[];
    fused2_march<PRNG, NS, 0>(p, xcd_item(blockIdx.x, gridDim.x, p.xgroup), lds, Ring2Steps<NS>{});
}

// One work item of a batch round: item `local` (tile and z chunk) of lattice e in
// round r of the current run.  A lattice with two-sweep rounds does sweeps 2r and
// 2r+1 of its run in round r (only 2r when that is its last), otherwise sweep r;
// it takes part while that first sweep is below its sweep count for this run.
// Its current spins are buffer c0 ^ (r & 1).
template <int SAUX>
__device__ __forceinline__ void batch_item(const BatchEntry &e, int64_t r, int local, uint64_t *lds)
{
    const int64_t s0 = e.two ? 2 * r : r;  // first sweep of this round, counted from the run's start
    if (s0 >= e.nsweeps)
        return;
    const bool deep = e.two && s0 + 2 <= e.nsweeps;
    FusedParams p;
    p.J = e.J;
    const int c = e.c0 ^ (int)(r & 1);
    p.src[0] = e.spins[c];
    p.dst[0] = e.spins[c ^ 1];
    p.rnd[0] = nullptr;
    p.mk[0] = e.mk;
    p.src[1] = p.src[0];
    p.dst[1] = p.dst[0];
    p.rnd[1] = nullptr;
    p.mk[1] = e.mk;
    p.L = e.L;
    p.P = e.L / 2;
    p.TXp = e.TXp;
    p.TY = e.TY;
    p.ZC = e.ZC;
    p.ntx = e.ntx;
    p.nty = e.nty;
    p.nzc = e.nzc;
    p.band = e.band;
    p.xgroup = kBatchGroup;  // unused: batch items are placed by the run's own order
    p.nrep = 1;
    p.t = e.t0 + s0;
    p.pkey[0] = p.pkey[1] = 0;
    p.a = minstd_power(e.t0 + s0);
    p.T = Thresholds{e.t4, e.t8, e.t12};
    if (deep) {
        p.EX = e.TXp + 4;
        p.EY = e.TY + 8;
        p.WE = e.WE2;
        p.WO[0] = e.WO0;
        p.WO[1] = e.WO1;
        p.a2 = minstd_power(e.t0 + s0 + 1);
        fused2_march<SG_MINSTD, kRing2Batch, SAUX>(p, local, lds, Ring2Steps<kRing2Batch>{});
    } else {
        p.EX = e.TXp + 2;
        p.EY = e.TY + 4;
        p.WE = e.WE;
        p.WO[0] = p.WO[1] = 0;
        p.a2 = 0;
        fused_march<SG_MINSTD, 1, SAUX>(p, local, lds, std::make_integer_sequence<int, Ring<1>::value>{});
    }
}

// Many lattices per launch ("round").  Work items of all lattices are numbered
// consecutively; item_lat maps an item to its lattice.  The round number is read
// from device memory, so a captured graph of rounds replays without new
// arguments.
__global__ __launch_bounds__(kMaxThreads) void k_fused_batch(const BatchEntry *__restrict__ E,
                                                             const uint32_t *__restrict__ item_lat, int nitems,
                                                             const int64_t *__restrict__ round_ctr)
{
    extern __shared__ uint64_t lds[];
    const int item = xcd_group_item(blockIdx.x);
    if (item >= nitems)
        return;
    const int li = __builtin_amdgcn_readfirstlane((int)item_lat[item]);
    const BatchEntry &e = E[li];
    batch_item<0>(e, *round_ctr, item - e.item0, lds);
}

// All rounds of a run in one launch.  The work of the run is a set of (round,
// item) entries, one queue per XCD: round r holds the items of the lattices still
// active in it, which the host numbers first (lattices sorted by the rounds they
// need), so its items are 0 .. n_r - 1, and they are dealt to the queues in groups
// of kBatchGroup as the per-round launch deals them to the XCDs (group g to queue
// g mod 8).  Each queue lists its entries in round-major order.  Workgroup b
// starts on queue b mod 8, i.e. on the queue of the XCD it runs on, and moves to
// the next queue once that one is empty.  It takes the next entry with an atomic
// counter, waits until the entry's lattice has finished the previous round
// (done[lattice] counts the lattice's finished items in this run, so round r may
// start once it reaches r x items), runs the item, makes its stores visible to the
// device and counts it done.
//
// Progress: an entry waits only for entries of an earlier round.  In its queue
// those come first, so a workgroup holds an entry of round r only once every
// entry of that queue's earlier rounds has been taken; an entry of an earlier
// round is therefore either taken (by a running workgroup) or first in line in its
// queue, which its home workgroups (and any workgroup whose own queue ran empty)
// take next.  The wait is bounded all the same: past spin_cap polls (or once
// another workgroup has given up) the workgroup sets *error and leaves, and every
// waiting workgroup then leaves too, so the grid always drains; the host reports
// the error.
struct PersistentArgs {
    const BatchEntry *E;
    const uint32_t *item_lat;
    const uint64_t *cum;   // [kBatchQueues][nrounds + 1], cum[q][0] = 0
    int nrounds;
    unsigned long long *queue;  // [kBatchQueues]
    uint32_t *done;        // per lattice
    uint32_t *error;
    uint32_t spin_cap;
};

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(kMaxThreads) void k_batch_persistent(PersistentArgs a)
{
    extern __shared__ uint64_t lds[];
    // what wave 0 hands the workgroup for one entry: round, item, lattice, go on
    __shared__ int s_round, s_item, s_lat;
    __shared__ uint32_t s_go;
    // Control flow here is uniform per wave: wave 0 does the hand-off with all its
    // lanes (lane 0 alone is told apart by the amount it adds to a counter, never by
    // a branch), and every decision is taken on readfirstlane values.  A branch on
    // the lane id around this loop's back edge lets the compiler split the loop so
    // that the other lanes reach the next barrier ahead of lane 0's counter updates.
    const bool wave0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) == 0;
    const uint32_t one = (threadIdx.x & 63) == 0 ? 1u : 0u;
    const int stride = a.nrounds + 1;
    int q = (int)(blockIdx.x % kBatchQueues);  // current queue (wave 0's copy is the one used)
    int qleft = kBatchQueues;                  // queues not yet found empty
    int acq_lat = -1, acq_round = -1;          // (lattice, round) of wave 0's last acquire
    for (;;) {
        if (wave0) {
            uint32_t go = 0u;
            int lo = 0, item = 0, li = 0;
            while (qleft > 0) {
                const uint64_t *cq = a.cum + (size_t)q * stride;
                const uint64_t total = uniform64(cq[a.nrounds]);
                const uint64_t k = uniform64(atomicAdd(a.queue + q, (unsigned long long)one));
                if (k < total) {
                    // round of entry k: the largest r with cq[r] <= k
                    int hi = a.nrounds;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (uniform64(cq[mid]) <= k)
                            lo = mid;
                        else
                            hi = mid;
                    }
                    const int j = (int)(k - uniform64(cq[lo]));
                    item = (q + kBatchQueues * (j / kBatchGroup)) * kBatchGroup + j % kBatchGroup;
                    go = 1u;
                    break;
                }
                q = (q + 1) % kBatchQueues;
                --qleft;
            }
            if (go) {
                li = __builtin_amdgcn_readfirstlane((int)a.item_lat[item]);
                const uint32_t need =
                    (uint32_t)lo * (uint32_t)__builtin_amdgcn_readfirstlane((int)a.E[li].nitems);
                uint32_t polls = 0;
                for (;;) {
                    const uint32_t d = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(&a.done[li], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (d >= need)
                        break;
                    const uint32_t err = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (err != 0u || ++polls > a.spin_cap) {
                        __hip_atomic_fetch_or(a.error, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        go = 0u;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(32);
                }
                // the previous round's words, written on any XCD, are visible from here
                // on: the acquire drops this CU's and this XCD's stale lines, which
                // serves every wave of the workgroup, as the others read only after the
                // barrier below (one invalidation per item, not one per wave); the wait
                // makes the invalidation complete before that barrier.  An item of the
                // lattice and round of this workgroup's last acquire needs none: that
                // acquire came after the whole previous round was done, and nothing can
                // bring an older copy of those words into the caches since.
                if (go && (li != acq_lat || lo != acq_round)) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    __builtin_amdgcn_s_waitcnt(0);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    acq_lat = li;
                    acq_round = lo;
                }
            }
            // every lane of the wave writes the same values
            s_round = lo;
            s_item = item;
            s_lat = li;
            s_go = go;
        }
        __syncthreads();
        const uint32_t go = __builtin_amdgcn_readfirstlane(s_go);
        const int lo = __builtin_amdgcn_readfirstlane(s_round);
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        const int li = __builtin_amdgcn_readfirstlane(s_lat);
        if (go == 0u)
            break;
        const BatchEntry &e = a.E[li];
        batch_item<kStoreDevice>(e, lo, item - e.item0, lds);
        // The item's spin words went out as device-coherent stores, so they are
        // visible to every XCD once they have completed: each wave waits for its
        // stores, and the barrier orders all waves' before wave 0 counts the item.
        // (An agent-scope release would instead write back this XCD's whole L2 at
        // every item, which cost the batch a sixth of its speed.)  The barrier also
        // keeps the next entry's LDS writes after every wave's last read.
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        if (wave0)
            __hip_atomic_fetch_add(&a.done[li], one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Clears the queues, the error flag and the per-lattice counters of a run.
__global__ void k_persistent_reset(unsigned long long *queue, uint32_t *error, uint32_t *done, int nlat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kBatchQueues)
        queue[i] = 0ull;
    if (i == 0)
        *error = 0u;
    for (int j = i; j < nlat; j += gridDim.x * blockDim.x)
        done[j] = 0u;
}

}  // namespace

static size_t fused_lds_bytes(int nrep, int tile_x, int tile_y)
{
    return (size_t)2 * ((tile_x + 2) * (tile_y + 4) + 1) * (2 * nrep + 3) * sizeof(uint64_t);
}

// Threads of a workgroup: even tile rows fill whole waves, then the odd rows.
static int fused_waves_even(int tile_x, int tile_y) { return ((tile_x + 2) * ((tile_y + 5) / 2) + 63) / 64; }
static int fused_threads(int tile_x, int tile_y)
{
    return 64 * (fused_waves_even(tile_x, tile_y) + ((tile_x + 2) * ((tile_y + 4) / 2) + 63) / 64);
}
static int max_threads(int) { return kMaxThreads; }

// ---- two sweeps per launch ---------------------------------------------------
static size_t fused2_lds_bytes(int tile_x, int tile_y)
{
    return (size_t)2 * ((tile_x + 4) * (tile_y + 8) + 1) * kF2Words * sizeof(uint64_t);
}
// Waves of the two-sweep workgroup: per row parity class, the outer ring rows
// (0..2 and EY-3..EY-1) and the inner rows (3..EY-4), each in whole waves.
struct F2Waves {
    int outer[2], inner[2];
};
static F2Waves fused2_waves(int tile_x, int tile_y)
{
    const int EX = tile_x + 4, EY = tile_y + 8;
    F2Waves w;
    for (int cls = 0; cls < 2; ++cls) {
        const int nout = (cls ? 1 : 2) + (((EY - 3) & 1) == cls ? 2 : 1);
        const int ifirst = cls ? 3 : 4;
        const int nin = ifirst <= EY - 4 ? (EY - 4 - ifirst) / 2 + 1 : 0;
        w.outer[cls] = (nout * EX + 63) / 64;
        w.inner[cls] = (nin * EX + 63) / 64;
    }
    return w;
}
static int fused2_threads(int tile_x, int tile_y)
{
    const F2Waves w = fused2_waves(tile_x, tile_y);
    return 64 * (w.outer[0] + w.inner[0] + w.outer[1] + w.inner[1]);
}


static int max_lds_bytes();

bool fused_shape_ok(int L, int nrep, int tile_x, int tile_y, int z_chunk)
{
    if (L < 2 || (L & 1) || nrep < 1 || nrep > 2)
        return false;
    const int P = L / 2;
    if (tile_x < 1 || tile_x > P || tile_y < 1 || tile_y > L || z_chunk < 0 || z_chunk > L)
        return false;
    if (fused_threads(tile_x, tile_y) > max_threads(nrep))
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
    // Measured on MI355X: tiles 32 or 16 pairs wide that divide the row, so that
    // the workgroups running together read whole rows; 8 or 16 rows tall.
    const int P = L / 2;
    z_chunk = 0;  // chosen at launch from the occupancy
    const int pref[][2] = {{32, 8}, {16, 16}, {16, 8}, {8, 16}};
    for (const auto &c : pref) {
        if (P % c[0] == 0 && P >= c[0] && L >= c[1] && fused_threads(c[0], c[1]) <= max_threads(nrep) &&
            fused_lds_bytes(nrep, c[0], c[1]) <= (size_t)max_lds_bytes()) {
            tile_x = c[0];
            tile_y = c[1];
            return;
        }
    }
    // small or odd-shaped planes: the tile needing the fewest lanes per pair
    double best = 1e30;
    tile_x = 1;
    tile_y = 1;
    for (int tx = 1; tx <= P && tx <= 126; ++tx)
        for (int ty = 1; ty <= L && ty <= 252; ++ty) {
            const int threads = fused_threads(tx, ty);
            if (threads > max_threads(nrep) || fused_lds_bytes(nrep, tx, ty) > (size_t)max_lds_bytes())
                continue;
            const int64_t ntx = (P + tx - 1) / tx, nty = (L + ty - 1) / ty;
            const double cost = (double)(ntx * nty * threads) / ((double)P * L);
            if (cost < best - 1e-9) {
                best = cost;
                tile_x = tx;
                tile_y = ty;
            }
        }
}

// Workgroups of kernel `fn` resident at once: per XCD (the item group of xcd_item)
// and on the device.
struct Residency {
    int per_xcd;
    int64_t slots;
};
static Residency residency(const void *fn, int threads, size_t lds)
{
    // queried once per (device, kernel, shape): launches of one lattice repeat them
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int, size_t>, Residency> known;
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess)
        dev = -1;
    const auto key = std::make_tuple(dev, fn, threads, lds);
    {
        std::lock_guard<std::mutex> g(mu);
        const auto it = known.find(key);
        if (it != known.end())
            return it->second;
    }
    if (dev >= 0)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const Residency r{std::max(1, cus / 8 * per_cu), (int64_t)cus * per_cu};
    std::lock_guard<std::mutex> g(mu);
    known[key] = r;
    return r;
}

// z chunk length for a grid of `tiles` work items per chunk: workgroups run in
// rounds of `slots`; take the chunk count with the shortest rounds * (ZC + extra)
// (`extra` planes are loaded per chunk beyond its own: 4 for one sweep per launch,
// 8 for two).
static int choose_z_chunk(int L, int64_t tiles, int64_t slots, int extra)
{
    int best_zc = L;
    double best = 1e300;
    for (int nzc = 1; nzc <= L && nzc <= 128; ++nzc) {
        const int zc = (L + nzc - 1) / nzc;
        const int64_t n = (L + zc - 1) / zc;
        const int64_t rounds = (tiles * n + slots - 1) / slots;
        const double cost = (double)rounds * (zc + extra);
        if (cost < best - 1e-9) {
            best = cost;
            best_zc = zc;
        }
    }
    return best_zc;
}

bool fill_batch_entry(BatchEntry &e, int L, int tile_x, int tile_y, int z_chunk, int band, bool two)
{
    if (!fused_shape_ok(L, 1, tile_x, tile_y, z_chunk) || z_chunk < 1)
        return false;
    const int P = L / 2;
    e.L = L;
    e.TXp = tile_x;
    e.TY = tile_y;
    e.ZC = z_chunk;
    e.ntx = (P + tile_x - 1) / tile_x;
    e.nty = (L + tile_y - 1) / tile_y;
    e.nzc = (L + z_chunk - 1) / z_chunk;
    e.WE = fused_waves_even(tile_x, tile_y);
    e.two = (two && fused2_shape_ok(L, tile_x, tile_y, z_chunk)) ? 1 : 0;
    const F2Waves w = fused2_waves(tile_x, tile_y);
    e.WE2 = w.outer[0] + w.inner[0];
    e.WO0 = w.outer[0];
    e.WO1 = w.outer[1];
    e.band = band < 1 ? 1 : (band > e.nty ? e.nty : band);
    e.nitems = e.ntx * e.nty * e.nzc;
    return true;
}

size_t fused_batch_lds_bytes(const BatchEntry &e)
{
    const size_t one = fused_lds_bytes(1, e.TXp, e.TY);
    return e.two ? std::max(one, fused2_lds_bytes(e.TXp, e.TY)) : one;
}

hipError_t launch_fused_batch(const BatchEntry *E, const uint32_t *item_lat, int nitems, const int64_t *round_ctr,
                              size_t lds, hipStream_t s)
{
    if (nitems < 1)
        return hipSuccess;
    if (lds > (size_t)max_lds_bytes())
        return hipErrorInvalidConfiguration;
    const int64_t per = 8 * kBatchGroup;
    const int64_t grid = (nitems + per - 1) / per * per;
    if (grid > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_fused_batch, dim3((unsigned)grid), dim3(kMaxThreads), lds, s, E, item_lat, nitems, round_ctr);
    return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned long long *queues, uint32_t *error, uint32_t *done, int nlat, hipStream_t s)
{
    hipLaunchKernelGGL(k_persistent_reset, dim3(std::max(1, std::min(64, (nlat + 255) / 256))), dim3(256), 0, s,
                       queues, error, done, nlat);
    return hipGetLastError();
}

hipError_t launch_batch_persistent(const BatchEntry *E, const uint32_t *item_lat, const uint64_t *cum, int nrounds,
                                   unsigned long long *queue, uint32_t *done, uint32_t *error, int nlat,
                                   uint32_t spin_cap, size_t lds, int64_t total_items, hipStream_t s)
{
    if (nrounds < 1 || total_items < 1)
        return hipSuccess;
    if (lds > (size_t)max_lds_bytes())
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_persistent_reset, dim3(std::max(1, std::min(64, (nlat + 255) / 256))), dim3(256), 0, s,
                       queue, error, done, nlat);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // as many workgroups as can be resident at once (progress does not depend on
    // it, see k_batch_persistent), at most one per queue entry
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch_persistent, kMaxThreads, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t grid = std::min<int64_t>((int64_t)cus * per_cu, total_items);
    PersistentArgs a{E, item_lat, cum, nrounds, queue, done, error, spin_cap};
    hipLaunchKernelGGL(k_batch_persistent, dim3((unsigned)grid), dim3(kMaxThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_round_advance(int64_t *round_ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_advance, dim3(1), dim3(64), 0, s, round_ctr);
    return hipGetLastError();
}

hipError_t launch_round_reset(int64_t *round_ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_reset, dim3(1), dim3(64), 0, s, round_ctr);
    return hipGetLastError();
}

hipError_t launch_sweep_fused(const SweepArgs &a, int tile_x, int tile_y, int z_chunk, int band, hipStream_t s)
{
    const void *fn = a.nrep == 1 ? (a.prng == SG_MINSTD    ? (const void *)k_fused<SG_MINSTD, 1>
                                     : a.prng == SG_PHILOX ? (const void *)k_fused<SG_PHILOX, 1>
                                                           : (const void *)k_fused<SG_MT19937, 1>)
                                  : (a.prng == SG_MINSTD    ? (const void *)k_fused<SG_MINSTD, 2>
                                     : a.prng == SG_PHILOX ? (const void *)k_fused<SG_PHILOX, 2>
                                                           : (const void *)k_fused<SG_MT19937, 2>);
    const Residency res = residency(fn, fused_threads(tile_x, tile_y), fused_lds_bytes(a.nrep, tile_x, tile_y));
    if (z_chunk == 0) {
        const int P = a.L / 2;
        const int64_t tiles = (int64_t)((P + tile_x - 1) / tile_x) * ((a.L + tile_y - 1) / tile_y);
        z_chunk = choose_z_chunk(a.L, tiles, res.slots, 4);
    }
    FusedParams p;
    p.J = a.J;
    for (int r = 0; r < 2; ++r) {
        p.src[r] = a.src[r];
        p.dst[r] = a.dst[r];
        p.rnd[r] = a.rnd[r];
        p.mk[r] = a.mk[r];
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
    p.a2 = a.minstd_a2;
    p.nrep = a.nrep;
    p.t = a.t;
    p.pkey[0] = a.pkey[0];
    p.pkey[1] = a.pkey[1];
    p.T = a.T;
    p.WE = fused_waves_even(tile_x, tile_y);
    p.WO[0] = p.WO[1] = 0;
    p.band = band < 1 ? 1 : (band > p.nty ? p.nty : band);
    p.xgroup = res.per_xcd;
    const int threads = fused_threads(tile_x, tile_y);
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
        else if (a.prng == SG_PHILOX)
            hipLaunchKernelGGL((k_fused<SG_PHILOX, 1>), grid, block, lds, s, p);
        else
            hipLaunchKernelGGL((k_fused<SG_MT19937, 1>), grid, block, lds, s, p);
    } else {
        if (a.prng == SG_MINSTD)
            hipLaunchKernelGGL((k_fused<SG_MINSTD, 2>), grid, block, lds, s, p);
        else if (a.prng == SG_PHILOX)
            hipLaunchKernelGGL((k_fused<SG_PHILOX, 2>), grid, block, lds, s, p);
        else
            hipLaunchKernelGGL((k_fused<SG_MT19937, 2>), grid, block, lds, s, p);
    }
    return hipGetLastError();
}


bool fused2_shape_ok(int L, int tile_x, int tile_y, int z_chunk)
{
    // the march touches planes z0-6 .. z0+ZC+5, which the one-step wrap maps
    // into [0, L) only for L >= 6
    if (L < 8 || (L & 1))
        return false;
    const int P = L / 2;
    if (tile_x < 1 || tile_x > P || tile_y < 1 || tile_y > L || z_chunk < 0 || z_chunk > L)
        return false;
    return fused2_threads(tile_x, tile_y) <= kMaxThreads && fused2_lds_bytes(tile_x, tile_y) <= (size_t)max_lds_bytes();
}

void fused2_default_shape(int L, int &tile_x, int &tile_y, int &z_chunk)
{
    const int P = L / 2;
    z_chunk = 0;
    const int pref[][2] = {{16, 16}, {16, 12}, {8, 24}, {8, 16}};
    for (const auto &c : pref)
        if (P % c[0] == 0 && L >= c[1] && fused2_shape_ok(L, c[0], c[1], 0)) {
            tile_x = c[0];
            tile_y = c[1];
            return;
        }
    double best = 1e30;
    tile_x = 1;
    tile_y = 1;
    for (int tx = 1; tx <= P && tx <= 124; ++tx)
        for (int ty = 1; ty <= L && ty <= 248; ++ty) {
            if (!fused2_shape_ok(L, tx, ty, 0))
                continue;
            const int64_t ntx = (P + tx - 1) / tx, nty = (L + ty - 1) / ty;
            const double cost = (double)(ntx * nty * fused2_threads(tx, ty)) / ((double)P * L);
            if (cost < best - 1e-9) {
                best = cost;
                tile_x = tx;
                tile_y = ty;
            }
        }
}

int fused2_default_ring(int) { return 5; }  // measured fastest at L = 256 .. 1024

hipError_t launch_sweep_fused2(const SweepArgs &a, int tile_x, int tile_y, int z_chunk, int band, int ring,
                               hipStream_t s)
{
    if (a.nrep < 1 || a.nrep > 2 || !fused2_shape_ok(a.L, tile_x, tile_y, z_chunk))
        return hipErrorInvalidConfiguration;
    const bool buf = a.prng == SG_MT19937;  // buffered draws of two sweeps in a.rnd
    if (ring == 0)
        ring = buf ? 5 : fused2_default_ring(a.L);
    if (ring != 5 && (ring != 6 || buf))
        return hipErrorInvalidValue;
    const bool px = a.prng == SG_PHILOX;
    const void *fn = buf         ? (const void *)k_fused2<SG_MT19937, 5>
                     : ring == 5 ? (px ? (const void *)k_fused2<SG_PHILOX, 5> : (const void *)k_fused2<SG_MINSTD, 5>)
                                 : (px ? (const void *)k_fused2<SG_PHILOX, 6> : (const void *)k_fused2<SG_MINSTD, 6>);
    const int threads = fused2_threads(tile_x, tile_y);
    const size_t lds = fused2_lds_bytes(tile_x, tile_y);
    const int P = a.L / 2;
    const int64_t tiles = (int64_t)((P + tile_x - 1) / tile_x) * ((a.L + tile_y - 1) / tile_y);
    const Residency res = residency(fn, threads, lds);
    if (z_chunk == 0)
        z_chunk = choose_z_chunk(a.L, tiles * a.nrep, res.slots, 8);
    FusedParams p;
    p.J = a.J;
    for (int r = 0; r < 2; ++r) {
        p.src[r] = a.src[r];
        p.dst[r] = a.dst[r];
        p.rnd[r] = a.rnd[r];
        p.mk[r] = a.mk[r];
    }
    p.L = a.L;
    p.P = P;
    p.TXp = tile_x;
    p.TY = tile_y;
    p.ZC = z_chunk;
    p.EX = tile_x + 4;
    p.EY = tile_y + 8;
    p.ntx = (P + tile_x - 1) / tile_x;
    p.nty = (a.L + tile_y - 1) / tile_y;
    p.nzc = (a.L + z_chunk - 1) / z_chunk;
    p.a = a.minstd_a;
    p.a2 = a.minstd_a2;
    p.nrep = a.nrep;
    p.t = a.t;
    p.pkey[0] = a.pkey[0];
    p.pkey[1] = a.pkey[1];
    p.T = a.T;
    const F2Waves fw = fused2_waves(tile_x, tile_y);
    p.WE = fw.outer[0] + fw.inner[0];
    p.WO[0] = fw.outer[0];
    p.WO[1] = fw.outer[1];
    p.band = band < 1 ? 1 : (band > p.nty ? p.nty : band);
    p.xgroup = res.per_xcd;
    const int64_t blocks = (int64_t)p.ntx * p.nty * p.nzc * a.nrep;
    if (blocks < 1 || blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    void *args[] = {&p};
    return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3((unsigned)threads), args, lds, s);
}

}  // namespace sg
