// Host side of the libsg C ABI (include/sg.h): argument checks, the memory carve
// of a lattice inside the caller's device buffer, per-sweep host scalars
// (thresholds, MINSTD multiplier), kernel choice and launches, readbacks.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <array>
#include <atomic>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {
thread_local std::string g_err;
constexpr uint32_t kM31 = 0x7FFFFFFFu;

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

bool valid_L(int L) { return L >= 2 && L <= 2048 && (L % 2) == 0; }
bool valid_prng(int prng)
{
    return prng == SG_MINSTD || prng == SG_MT19937 || prng == SG_PHILOX || prng == SG_PARISI_RAPUANO;
}

// 16807^(t+1) mod (2^31 - 1) by square and multiply.
uint32_t minstd_multiplier(int64_t t)
{
    uint64_t result = 1, base = 16807;
    uint64_t e = (uint64_t)t + 1;
    while (e) {
        if (e & 1)
            result = (result * base) % kM31;
        base = (base * base) % kM31;
        e >>= 1;
    }
    return (uint32_t)result;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return SG_OK;
    return hip_fail(e, what);
}

// numbers handed to caller-provided coupling sets, one per sg_lattice_create
std::atomic<uint64_t> g_coupling_sets{1};
}  // namespace

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return SG_EDEVICE;
}

// Arrays of a lattice's buffer.  Each starts kSkew bytes past the end of the one
// before: at power-of-two sides the arrays' sizes are powers of two, and the same
// plane of every array would otherwise sit at the same low address bits, where the
// planes a step reads and writes contend for the same memory channels.  With this
// skew and the pad between the coupling arrays (coupling_stride), the L = 1024 sweep
// measured 8-10% faster.
constexpr size_t kSkew = 37 * 256;

Carve carve(int L, int prng, bool own_J)
{
    const size_t V = (size_t)L * L * L;
    Carve c{};
    size_t off = 0;
    c.spins0 = off;
    off = align_up(off + 8 * V) + kSkew;
    c.spins1 = off;
    off = align_up(off + 8 * V) + kSkew;
    c.J = off;
    if (own_J)
        off = align_up(off + 24 * (size_t)coupling_stride(L)) + kSkew;
    c.mt_state = off;
    if (prng == SG_MT19937)
        off = align_up(off + (size_t)4 * kMtN * L * L) + kSkew;
    if (prng == SG_PARISI_RAPUANO)
        off = align_up(off + (size_t)4 * 64 * L * L) + kSkew;
    c.rbuf = off;
    if (buffered_draws(prng))  // draws of the two sweeps of a two-sweep launch
        off = align_up(off + 8 * V) + kSkew;
    c.scratch = off;
    off = align_up(off + 8 * ((size_t)kMaxReduceBlocks * 64 + 64));
    c.total = off;
    return c;
}

}  // namespace sg

using namespace sg;

namespace {

// The handle handed out: the lattice plus the identity of its couplings.  Two
// lattices hold the same couplings when both fields agree: kind kFromSeed with
// the same coupling seed, or kind kFromCaller with the same set number.
enum CouplingKind { kFromSeed = 1, kFromCaller = 2 };
struct Handle : sg_lattice {
    int coupling_kind = 0;
    uint64_t coupling_value = 0;
};

Handle *H(sg_lattice *p) { return static_cast<Handle *>(p); }
const Handle *H(const sg_lattice *p) { return static_cast<const Handle *>(p); }

int init_streams(sg_lattice *lat)
{
    hipError_t e = launch_init_spins(lat->spins[0], lat->L, lat->key_spin, lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, "init spins");
    if (lat->prng == SG_MT19937)
        e = launch_init_mt(lat->mt_state, lat->L, lat->key_mt, lat->stream);
    else if (lat->prng == SG_PARISI_RAPUANO)
        e = launch_init_pr(lat->mt_state, lat->L, lat->key_pr, lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, "init streams");
    return SG_OK;
}

int setup(Handle *lat, int L, int nsamples, int prng, uint64_t spin_seed, uint32_t replica, void *dev_buf,
          size_t dev_bytes, void *stream, bool own_J)
{
    const Carve c = carve(L, prng, own_J);
    if (dev_bytes < c.total)
        return fail(SG_EINVAL, "device buffer too small: need " + std::to_string(c.total) + " bytes");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0)
        return fail(SG_EINVAL, "device buffer must be 256-byte aligned");
    lat->L = L;
    lat->nsamples = nsamples;
    lat->prng = prng;
    lat->V = (int64_t)L * L * L;
    lat->spin_seed = spin_seed;
    lat->replica = replica;
    lat->key_spin = derive_key(spin_seed, kTagSpin, replica);
    lat->key_minstd = derive_key(spin_seed, kTagMinstd, replica);
    lat->minstd_k = (uint32_t)lat->key_minstd;
    lat->key_mt = derive_key(spin_seed, kTagMt, replica);
    lat->key_philox = derive_key(spin_seed, kTagPhilox, replica);
    lat->key_pr = derive_key(spin_seed, kTagPr, replica);
    lat->base = static_cast<uint8_t *>(dev_buf);
    lat->bytes = dev_bytes;
    lat->spins[0] = reinterpret_cast<uint64_t *>(lat->base + c.spins0);
    lat->spins[1] = reinterpret_cast<uint64_t *>(lat->base + c.spins1);
    if (own_J)
        lat->J = reinterpret_cast<uint64_t *>(lat->base + c.J);
    lat->mt_state = buffered_draws(prng) ? reinterpret_cast<uint32_t *>(lat->base + c.mt_state) : nullptr;
    lat->rbuf = buffered_draws(prng) ? reinterpret_cast<uint32_t *>(lat->base + c.rbuf) : nullptr;
    lat->scratch = reinterpret_cast<uint64_t *>(lat->base + c.scratch);
    lat->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&lat->device) != hipSuccess)
        return fail(SG_EDEVICE, "no current HIP device");
    lat->cur = 0;
    lat->t = 0;
    return SG_OK;
}

// Kernel for sweeps of nrep lattices: 2 = two sweeps per launch, 1 = fused, 0 =
// two-pass (shape in tx, ty, zc); negative = error (an explicitly chosen tile
// that does not fit).
int pick_kernel(const sg_lattice *lat, int nrep, int &tx, int &ty, int &zc)
{
    if (lat->kernel == SG_KERNEL_TWOPASS)
        return 0;
    if (lat->kernel == SG_KERNEL_FUSED2 || lat->kernel == SG_KERNEL_AUTO) {
        if (lat->kernel == SG_KERNEL_FUSED2 && lat->tile_x > 0) {
            tx = lat->tile_x;
            ty = lat->tile_y;
            zc = lat->z_chunk;
            if (!fused2_shape_ok(lat->L, tx, ty, zc))
                return fail(SG_EINVAL, "the chosen two-sweep tile does not fit this lattice");
            return 2;
        }
        fused2_default_shape(lat->L, tx, ty, zc);
        if (lat->z_chunk > 0)
            zc = lat->z_chunk;
        if (fused2_shape_ok(lat->L, tx, ty, zc))
            return 2;
        if (lat->kernel == SG_KERNEL_FUSED2)
            return fail(SG_EINVAL, "no two-sweep tile fits this lattice");
    }
    if (lat->kernel == SG_KERNEL_FUSED && lat->tile_x > 0) {
        tx = lat->tile_x;
        ty = lat->tile_y;
        zc = lat->z_chunk;
        if (!fused_shape_ok(lat->L, nrep, tx, ty, zc))
            return fail(SG_EINVAL, "the chosen fused tile does not fit " + std::to_string(nrep) + " replica(s)");
        return 1;
    }
    fused_default_shape(lat->L, nrep, tx, ty, zc);
    if (lat->z_chunk > 0)
        zc = lat->z_chunk;
    if (fused_shape_ok(lat->L, nrep, tx, ty, zc))
        return 1;
    if (lat->kernel == SG_KERNEL_FUSED)
        return fail(SG_EINVAL, "no fused tile fits this lattice");
    return 0;
}

// One launch of `kind` (see pick_kernel) for n (1 or 2) lattices that share
// couplings, stream and sweep count: two sweeps for kind 2, one otherwise.
int sweep_launch(sg_lattice *const *lats, int n, const Thresholds &T, int kind, int tx, int ty, int zc)
{
    sg_lattice *l0 = lats[0];
    const int64_t t = l0->t;
    hipError_t e;
    if (buffered_draws(l0->prng)) {
        uint32_t *st[2], *rb[2];
        for (int r = 0; r < n; ++r) {
            st[r] = lats[r]->mt_state;
            rb[r] = lats[r]->rbuf;
        }
        const int nsw = kind == 2 ? 2 : 1;
        e = l0->prng == SG_MT19937 ? launch_mt_fill(st, rb, n, l0->L, t, nsw, l0->stream)
                                   : launch_pr_fill(st, rb, n, l0->L, t, nsw, l0->stream);
        if (e != hipSuccess)
            return hip_fail(e, "stream fill");
        for (int r = 0; r < n; ++r)
            lats[r]->rlast = nsw - 1;
    }
    SweepArgs a{};
    a.J = l0->J;
    a.nrep = n;
    a.L = l0->L;
    // the sweep kernels read buffered numbers the same way for both generators
    a.prng = buffered_draws(l0->prng) ? SG_MT19937 : l0->prng;
    a.minstd_a = minstd_multiplier(t);
    a.minstd_a2 = minstd_multiplier(t + 1);
    a.t = t;
    a.T = T;
    for (int r = 0; r < n; ++r) {
        a.src[r] = lats[r]->spins[lats[r]->cur];
        a.dst[r] = lats[r]->spins[1 - lats[r]->cur];
        a.rnd[r] = lats[r]->rbuf;
        a.mk[r] = lats[r]->minstd_k;
        a.pkey[r] = lats[r]->key_philox;
    }
    const int band = l0->band > 0 ? l0->band : 1;
    int done = 1;
    if (kind == 2) {
        e = launch_sweep_fused2(a, tx, ty, zc, band, l0->ring, l0->stream);
        if (e != hipSuccess)
            return hip_fail(e, "two-sweep launch");
        done = 2;
    } else if (kind == 1) {
        e = launch_sweep_fused(a, tx, ty, zc, band, l0->stream);
        if (e != hipSuccess)
            return hip_fail(e, "fused sweep launch");
    } else {
        e = launch_sweep_twopass(a, l0->stream);
        if (e != hipSuccess)
            return hip_fail(e, "two-pass sweep launch");
    }
    for (int r = 0; r < n; ++r) {
        if (kind != 0)
            lats[r]->cur ^= 1;
        lats[r]->t += done;
    }
    return SG_OK;
}

// nsweeps sweeps of n (1 or 2) lattices as above.  With the two-sweep kernel an
// odd last sweep runs on the one-sweep fused kernel (same tile when it fits).
int sweep_n(sg_lattice *const *lats, int n, int64_t nsweeps, const Thresholds &T)
{
    int tx = 0, ty = 0, zc = 0;
    const int kind = pick_kernel(lats[0], n, tx, ty, zc);
    if (kind < 0)
        return kind;
    while (nsweeps > 0) {
        int k = kind, x = tx, y = ty, z = zc;
        if (k == 2 && nsweeps < 2) {
            k = 1;
            if (!fused_shape_ok(lats[0]->L, n, x, y, z)) {
                fused_default_shape(lats[0]->L, n, x, y, z);
                if (!fused_shape_ok(lats[0]->L, n, x, y, z))
                    k = 0;
            }
        }
        const int rc = sweep_launch(lats, n, T, k, x, y, z);
        if (rc != SG_OK)
            return rc;
        nsweeps -= (k == 2) ? 2 : 1;
    }
    return SG_OK;
}

int check_beta(double beta)
{
    if (std::isnan(beta) || beta < 0)
        return fail(SG_EINVAL, "beta must be >= 0");
    return SG_OK;
}

int count_to_host(sg_lattice *lat, int nblocks, int64_t *out)
{
    uint64_t *out64 = lat->scratch + (size_t)kMaxReduceBlocks * 64;
    hipError_t e = launch_reduce_partials(lat->scratch, nblocks, out64, lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, "reduce launch");
    uint64_t host[64];
    e = hipMemcpyAsync(host, out64, sizeof(host), hipMemcpyDeviceToHost, lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, "readback");
    e = hipStreamSynchronize(lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, "synchronize");
    for (int j = 0; j < 64; ++j)
        out[j] = (int64_t)host[j];
    return SG_OK;
}

// nsweeps two-pass sweeps of lat on a layout of the study of Sec. 2: the
// current spins and the couplings are converted into `work` (32 bytes per site,
// checked by the caller), swept there, and the spins converted back.
struct LayoutOps {
    hipError_t (*to)(const uint64_t *, uint64_t *, int, int, int64_t, hipStream_t);
    hipError_t (*from)(const uint64_t *, uint64_t *, int, hipStream_t);
    hipError_t (*sweep)(const SweepArgs &, uint64_t *, const uint64_t *, hipStream_t);
    const char *name;
};
const LayoutOps kSeparated{launch_to_separated, launch_from_separated, launch_sweep_separated, "separated"};
const LayoutOps kSliced{launch_to_sliced, launch_from_sliced, launch_sweep_sliced, "sliced"};

int layout_sweep(sg_lattice *lat, int64_t nsweeps, double beta, uint64_t *work, const LayoutOps &ops)
{
    uint64_t T[3];
    sg_thresholds(beta, lat->prng, T);
    const int64_t V = lat->V;
    uint64_t *S = work;
    uint64_t *K = S + V;
    const std::string nm(ops.name);
    hipError_t e = ops.to(lat->spins[lat->cur], S, lat->L, 1, lat->V, lat->stream);
    if (e == hipSuccess)
        e = ops.to(lat->J, K, lat->L, 3, coupling_stride(lat->L), lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, ("to " + nm + " layout").c_str());
    for (int64_t k = 0; k < nsweeps; ++k) {
        const int64_t t = lat->t;
        if (buffered_draws(lat->prng)) {
            e = lat->prng == SG_MT19937 ? launch_mt_fill(&lat->mt_state, &lat->rbuf, 1, lat->L, t, 1, lat->stream)
                                        : launch_pr_fill(&lat->mt_state, &lat->rbuf, 1, lat->L, t, 1, lat->stream);
            lat->rlast = 0;
            if (e != hipSuccess)
                return hip_fail(e, "stream fill");
        }
        SweepArgs a{};
        a.J = nullptr;
        a.nrep = 1;
        a.L = lat->L;
        a.prng = buffered_draws(lat->prng) ? SG_MT19937 : lat->prng;
        a.minstd_a = minstd_multiplier(t);
        a.t = t;
        a.T = Thresholds{T[0], T[1], T[2]};
        a.rnd[0] = lat->rbuf;
        a.mk[0] = lat->minstd_k;
        a.pkey[0] = lat->key_philox;
        e = ops.sweep(a, S, K, lat->stream);
        if (e != hipSuccess)
            return hip_fail(e, (nm + " sweep").c_str());
        lat->t += 1;
    }
    e = ops.from(S, lat->spins[lat->cur], lat->L, lat->stream);
    return e == hipSuccess ? SG_OK : hip_fail(e, ("from " + nm + " layout").c_str());
}

int layout_sweep_checked(sg_lattice *lat, int64_t nsweeps, double beta, void *work, size_t work_bytes,
                         const LayoutOps &ops)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    if (nsweeps < 0)
        return fail(SG_EINVAL, "nsweeps < 0");
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    size_t need = 0;
    sg_sliced_footprint(lat->L, &need);
    if (!work || work_bytes < need)
        return fail(SG_EINVAL, "layout work buffer too small: need " + std::to_string(need) + " bytes");
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0)
        return fail(SG_EINVAL, "layout work buffer must be 256-byte aligned");
    return layout_sweep(lat, nsweeps, beta, static_cast<uint64_t *>(work), ops);
}

}  // namespace

// Work area of sg_sweep_sliced_static, for callers that cannot allocate: the
// sliced copy of one lattice (32 bytes per site) of side up to kStaticSide.  Each
// GPU the library runs on holds its own copy until the process ends.  In host code
// this name is a host-side stand-in: the area's device address comes from
// static_area() and nothing else.
constexpr int kStaticSide = 64;
constexpr size_t kStaticBytes = (size_t)32 * kStaticSide * kStaticSide * kStaticSide;  // 8 MiB
static __device__ __align__(256) uint64_t scratch[kStaticBytes / sizeof(uint64_t)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
uint64_t *g_static_ptr[kMaxDevices] = {};

// Device address of the static work area on `device`, looked up once per device
// with that device current (and the caller's current device restored after).
int static_area(int device, uint64_t **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(SG_EDEVICE, "device index out of range for the static work area");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device)
            e = hipSetDevice(device);
        if (e != hipSuccess)
            return hip_fail(e, "select the lattice's device");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t r = prev != device ? hipSetDevice(prev) : hipSuccess;
        if (e != hipSuccess)
            return hip_fail(e, "address of the static work area");
        if (r != hipSuccess)
            return hip_fail(r, "restore the current device");
        if (!p)
            return fail(SG_EDEVICE, "the static work area has no device address");
        g_static_ptr[device] = static_cast<uint64_t *>(p);
    }
    *out = g_static_ptr[device];
    return SG_OK;
}

}  // namespace

extern "C" {

const char *sg_last_error(void) { return g_err.c_str(); }

static int footprint(int L, int nsamples, int prng, bool own_couplings, size_t *dev_bytes)
{
    if (!valid_L(L))
        return fail(SG_EINVAL, "L must be even and in [2, 2048]");
    if (nsamples < 1 || nsamples > 64)
        return fail(SG_EINVAL, "nsamples must be in [1, 64]");
    if (!valid_prng(prng))
        return fail(SG_EINVAL, "unknown prng");
    if (!dev_bytes)
        return fail(SG_EINVAL, "dev_bytes is NULL");
    *dev_bytes = carve(L, prng, own_couplings).total;
    return SG_OK;
}

int sg_footprint(int L, int nsamples, int prng, size_t *dev_bytes)
{
    return footprint(L, nsamples, prng, true, dev_bytes);
}

int sg_replica_footprint(int L, int nsamples, int prng, size_t *dev_bytes)
{
    return footprint(L, nsamples, prng, false, dev_bytes);
}

int sg_thresholds(double beta, int prng, uint64_t T[3])
{
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    if (!valid_prng(prng))
        return fail(SG_EINVAL, "unknown prng");
    if (!T)
        return fail(SG_EINVAL, "T is NULL");
    // Sec. 4: accept dE > 0 iff R < R_range * exp(-beta dE); rounding the product
    // up makes the integer comparison exact.
    const double range = prng == SG_MINSTD ? 2147483647.0 : 4294967296.0;
    for (int k = 1; k <= 3; ++k) {
        const double dE = 4.0 * k;
        const double prob = std::exp(-(beta * dE));
        T[k - 1] = (uint64_t)std::ceil(range * prob);
    }
    return SG_OK;
}

int sg_lattice_create(int L, int nsamples, int prng, const uint64_t *J_host, uint64_t coupling_seed,
                      uint64_t spin_seed, uint32_t replica, void *dev_buf, size_t dev_bytes, void *stream,
                      sg_lattice **out)
{
    if (!out)
        return fail(SG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!valid_L(L))
        return fail(SG_EINVAL, "L must be even and in [2, 2048]");
    if (nsamples < 1 || nsamples > 64)
        return fail(SG_EINVAL, "nsamples must be in [1, 64]");
    if (!valid_prng(prng))
        return fail(SG_EINVAL, "unknown prng");
    if (!dev_buf)
        return fail(SG_EINVAL, "dev_buf is NULL");
    Handle *lat = new (std::nothrow) Handle();
    if (!lat)
        return fail(SG_ENOMEM, "out of host memory");
    int rc = setup(lat, L, nsamples, prng, spin_seed, replica, dev_buf, dev_bytes, stream, true);
    if (rc != SG_OK) {
        delete lat;
        return rc;
    }
    lat->coupling_seed = coupling_seed;
    hipError_t e = hipSuccess;
    if (J_host) {
        for (int d = 0; d < 3 && e == hipSuccess; ++d)
            e = hipMemcpyAsync(lat->J + d * coupling_stride(L), J_host + (size_t)d * lat->V, (size_t)8 * lat->V,
                               hipMemcpyHostToDevice, lat->stream);
        lat->coupling_kind = kFromCaller;
        lat->coupling_value = g_coupling_sets.fetch_add(1);
        if (e == hipSuccess)
            e = hipStreamSynchronize(lat->stream);  // J_host is only borrowed
    } else {
        lat->key_j = derive_key(coupling_seed, kTagJ, 0);
        e = launch_init_couplings(lat->J, L, lat->key_j, lat->stream);
        lat->coupling_kind = kFromSeed;
        lat->coupling_value = coupling_seed;
    }
    if (e != hipSuccess) {
        delete lat;
        return hip_fail(e, "couplings");
    }
    rc = init_streams(lat);
    if (rc == SG_OK) {
        e = hipStreamSynchronize(lat->stream);
        if (e != hipSuccess)
            rc = hip_fail(e, "create");
    }
    if (rc != SG_OK) {
        delete lat;
        return rc;
    }
    *out = lat;
    return SG_OK;
}

int sg_lattice_create_replica(const sg_lattice *base, uint64_t spin_seed, uint32_t replica, void *dev_buf,
                              size_t dev_bytes, void *stream, sg_lattice **out)
{
    if (!out || !base)
        return fail(SG_EINVAL, "NULL argument");
    *out = nullptr;
    if (!dev_buf)
        return fail(SG_EINVAL, "dev_buf is NULL");
    Handle *lat = new (std::nothrow) Handle();
    if (!lat)
        return fail(SG_ENOMEM, "out of host memory");
    int rc = setup(lat, base->L, base->nsamples, base->prng, spin_seed, replica, dev_buf, dev_bytes, stream, false);
    if (rc != SG_OK) {
        delete lat;
        return rc;
    }
    lat->J = base->J;
    lat->J_owner = base->J_owner ? base->J_owner : base;
    lat->coupling_seed = base->coupling_seed;
    lat->coupling_kind = H(base)->coupling_kind;
    lat->coupling_value = H(base)->coupling_value;
    lat->kernel = base->kernel;
    lat->tile_x = base->tile_x;
    lat->tile_y = base->tile_y;
    lat->z_chunk = base->z_chunk;
    lat->band = base->band;
    rc = init_streams(lat);
    if (rc == SG_OK) {
        hipError_t e = hipStreamSynchronize(lat->stream);
        if (e != hipSuccess)
            rc = hip_fail(e, "create replica");
    }
    if (rc != SG_OK) {
        delete lat;
        return rc;
    }
    *out = lat;
    return SG_OK;
}

int sg_sweep(sg_lattice *lat, int64_t nsweeps, double beta)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    if (nsweeps < 0)
        return fail(SG_EINVAL, "nsweeps < 0");
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    uint64_t T[3];
    sg_thresholds(beta, lat->prng, T);
    const Thresholds th{T[0], T[1], T[2]};
    return sweep_n(&lat, 1, nsweeps, th);
}

int sg_sweep_replicas(sg_lattice *const *lats, int n, int64_t nsweeps, double beta)
{
    if (!lats || n < 1)
        return fail(SG_EINVAL, "no lattices");
    if (nsweeps < 0)
        return fail(SG_EINVAL, "nsweeps < 0");
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    for (int r = 0; r < n; ++r) {
        if (!lats[r])
            return fail(SG_EINVAL, "NULL lattice");
        if (lats[r]->L != lats[0]->L || lats[r]->prng != lats[0]->prng || lats[r]->J != lats[0]->J ||
            lats[r]->stream != lats[0]->stream || lats[r]->t != lats[0]->t)
            return fail(SG_EMISMATCH, "replicas must share L, prng, couplings, stream and sweep count");
        for (int q = 0; q < r; ++q)
            if (lats[q] == lats[r])
                return fail(SG_EINVAL, "a lattice appears twice");
    }
    uint64_t T[3];
    sg_thresholds(beta, lats[0]->prng, T);
    const Thresholds th{T[0], T[1], T[2]};
    for (int r = 0; r < n; r += 2) {
        const int m = (n - r) >= 2 ? 2 : 1;
        const int rc = sweep_n(lats + r, m, nsweeps, th);
        if (rc != SG_OK)
            return rc;
    }
    return SG_OK;
}

int sg_sliced_footprint(int L, size_t *dev_bytes)
{
    if (L < 2 || (L & 1) || L > 2048 || !dev_bytes)
        return fail(SG_EINVAL, "L must be even, 2..2048");
    *dev_bytes = (size_t)32 * L * L * L;  // spins and three coupling words per site
    return SG_OK;
}

int sg_sweep_separated(sg_lattice *lat, int64_t nsweeps, double beta, void *work, size_t work_bytes)
{
    return layout_sweep_checked(lat, nsweeps, beta, work, work_bytes, kSeparated);
}

int sg_sweep_sliced(sg_lattice *lat, int64_t nsweeps, double beta, void *work, size_t work_bytes)
{
    return layout_sweep_checked(lat, nsweeps, beta, work, work_bytes, kSliced);
}

int sg_sweep_sliced_static(sg_lattice *lat, int64_t nsweeps, double beta)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    if (nsweeps < 0)
        return fail(SG_EINVAL, "nsweeps < 0");
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    if (lat->L > kStaticSide)
        return fail(SG_EINVAL, "sg_sweep_sliced_static takes sides up to " + std::to_string(kStaticSide) +
                                   " (a static work area of " + std::to_string(kStaticBytes) + " bytes); L = " +
                                   std::to_string(lat->L) + " needs " +
                                   std::to_string((size_t)32 * lat->L * lat->L * lat->L));
    uint64_t *area = nullptr;
    const int rc = static_area(lat->device, &area);
    if (rc != SG_OK)
        return rc;
    // the layout conversion writes every word of the area it then reads, so
    // nothing needs clearing between calls
    return layout_sweep(lat, nsweeps, beta, area, kSliced);
}

int sg_sweep_energies(sg_lattice *lat, int64_t nsweeps, double beta, int64_t *unsat)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    if (nsweeps < 0)
        return fail(SG_EINVAL, "nsweeps < 0");
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    if (!unsat && nsweeps > 0)
        return fail(SG_EINVAL, "unsat is NULL");
    uint64_t T[3];
    sg_thresholds(beta, lat->prng, T);
    const Thresholds th{T[0], T[1], T[2]};
    const size_t words = (size_t)kMaxReduceBlocks * 64 + 64;  // the reduction area
    std::vector<uint64_t> host;
    auto read_back = [&](const uint64_t *rows, int64_t done, int64_t chunk) -> int {
        host.resize((size_t)chunk * 64);
        hipError_t e = hipMemcpyAsync(host.data(), rows, 8 * host.size(), hipMemcpyDeviceToHost, lat->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(lat->stream);
        if (e != hipSuccess)
            return hip_fail(e, "energy readback");
        for (int64_t k = 0; k < chunk; ++k)
            for (int j = 0; j < lat->nsamples; ++j)
                unsat[(done + k) * lat->nsamples + j] = (int64_t)host[(size_t)k * 64 + j];
        return SG_OK;
    };
    if (lat->V <= kSmallSites && (lat->prng == SG_MINSTD || lat->prng == SG_PHILOX)) {
        // one workgroup runs a chunk of sweeps with the lattice in LDS, one row of 64
        // totals per sweep in the reduction area
        const int64_t cap = (int64_t)(words / 64);
        for (int64_t done = 0; done < nsweeps;) {
            const int chunk = (int)std::min<int64_t>(cap, nsweeps - done);
            const hipError_t e = launch_small_sweeps(lat->spins[lat->cur], lat->J, lat->L, lat->nsamples, lat->prng,
                                                     lat->minstd_k,
                                                     lat->key_philox, lat->t, minstd_multiplier(lat->t), chunk, th,
                                                     lat->scratch, lat->stream);
            if (e != hipSuccess)
                return hip_fail(e, "small-lattice sweeps");
            lat->t += chunk;
            const int rc = read_back(lat->scratch, done, chunk);
            if (rc != SG_OK)
                return rc;
            done += chunk;
        }
        return SG_OK;
    }
    // The reduction area holds the per-block rows of one count and, after them, one
    // row of 64 totals per sweep of a chunk; a chunk is read back with one copy.
    int nblocks = 0;
    for (int64_t done = 0; done < nsweeps;) {
        int64_t chunk = 0;
        uint64_t *rows = nullptr;
        hipError_t e = hipSuccess;
        for (; done + chunk < nsweeps; ++chunk) {
            int rc = sweep_n(&lat, 1, 1, th);
            if (rc != SG_OK)
                return rc;
            e = launch_count_unsat(lat->spins[lat->cur], lat->J, lat->L, lat->scratch, nblocks, lat->stream);
            if (e != hipSuccess)
                return hip_fail(e, "energy launch");
            rows = lat->scratch + (size_t)nblocks * 64;
            const int64_t cap = (int64_t)((words - (size_t)nblocks * 64) / 64);  // >= 1
            e = launch_reduce_partials(lat->scratch, nblocks, rows + (size_t)chunk * 64, lat->stream);
            if (e != hipSuccess)
                return hip_fail(e, "reduce launch");
            if (chunk + 1 == cap) {
                ++chunk;
                break;
            }
        }
        const int rc = read_back(rows, done, chunk);
        if (rc != SG_OK)
            return rc;
        done += chunk;
    }
    return SG_OK;
}

int sg_energy(sg_lattice *lat, int64_t *unsat, double *e_per_spin)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    int nblocks = 0;
    hipError_t e = launch_count_unsat(lat->spins[lat->cur], lat->J, lat->L, lat->scratch, nblocks, lat->stream);
    if (e != hipSuccess)
        return hip_fail(e, "energy launch");
    int64_t U[64];
    int rc = count_to_host(lat, nblocks, U);
    if (rc != SG_OK)
        return rc;
    for (int j = 0; j < lat->nsamples; ++j) {
        if (unsat)
            unsat[j] = U[j];
        if (e_per_spin)
            e_per_spin[j] = (2.0 * (double)U[j] - 3.0 * (double)lat->V) / (double)lat->V;
    }
    return SG_OK;
}

int sg_overlap(const sg_lattice *a, const sg_lattice *b, int64_t *ndiff, double *q)
{
    if (!a || !b)
        return fail(SG_EINVAL, "NULL lattice");
    if (a->L != b->L || a->nsamples != b->nsamples || H(a)->coupling_kind != H(b)->coupling_kind ||
        H(a)->coupling_value != H(b)->coupling_value)
        return fail(SG_EMISMATCH, "overlap needs lattices of equal size, samples and couplings");
    sg_lattice *wa = const_cast<sg_lattice *>(a);
    if (b->stream != a->stream) {
        hipError_t e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess)
            return hip_fail(e, "synchronize");
    }
    int nblocks = 0;
    hipError_t e = launch_count_diff(a->spins[a->cur], b->spins[b->cur], a->V, wa->scratch, nblocks, a->stream);
    if (e != hipSuccess)
        return hip_fail(e, "overlap launch");
    int64_t N[64];
    int rc = count_to_host(wa, nblocks, N);
    if (rc != SG_OK)
        return rc;
    for (int j = 0; j < a->nsamples; ++j) {
        if (ndiff)
            ndiff[j] = N[j];
        if (q)
            q[j] = 1.0 - 2.0 * (double)N[j] / (double)a->V;
    }
    return SG_OK;
}

int sg_get_words(const sg_lattice *lat, uint64_t *out, size_t n)
{
    if (!lat || !out)
        return fail(SG_EINVAL, "NULL argument");
    if (n != (size_t)lat->V)
        return fail(SG_EINVAL, "n must be L^3");
    hipError_t e = hipMemcpyAsync(out, lat->spins[lat->cur], 8 * n, hipMemcpyDeviceToHost, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    return check_hip(e, "get words");
}

int sg_set_spins(sg_lattice *lat, const uint64_t *in, size_t n)
{
    if (!lat || !in)
        return fail(SG_EINVAL, "NULL argument");
    if (n != (size_t)lat->V)
        return fail(SG_EINVAL, "n must be L^3");
    hipError_t e = hipMemcpyAsync(lat->spins[lat->cur], in, 8 * n, hipMemcpyHostToDevice, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    return check_hip(e, "set spins");
}

int sg_get_couplings(const sg_lattice *lat, uint64_t *out, size_t n)
{
    if (!lat || !out)
        return fail(SG_EINVAL, "NULL argument");
    if (n != (size_t)(3 * lat->V))
        return fail(SG_EINVAL, "n must be 3 L^3");
    hipError_t e = hipSuccess;
    for (int d = 0; d < 3 && e == hipSuccess; ++d)
        e = hipMemcpyAsync(out + (size_t)d * lat->V, lat->J + d * coupling_stride(lat->L), (size_t)8 * lat->V,
                           hipMemcpyDeviceToHost, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    return check_hip(e, "get couplings");
}

int sg_get_spins(const sg_lattice *lat, int8_t *out, size_t n)
{
    if (!lat || !out)
        return fail(SG_EINVAL, "NULL argument");
    const size_t V = (size_t)lat->V;
    if (n != (size_t)lat->nsamples * V)
        return fail(SG_EINVAL, "n must be nsamples * L^3");
    std::vector<uint64_t> w;
    try {
        w.resize(V);
    } catch (...) {
        return fail(SG_ENOMEM, "out of host memory");
    }
    int rc = sg_get_words(lat, w.data(), V);
    if (rc != SG_OK)
        return rc;
    for (int j = 0; j < lat->nsamples; ++j) {
        int8_t *o = out + (size_t)j * V;
        for (size_t i = 0; i < V; ++i)
            o[i] = ((w[i] >> j) & 1ull) ? 1 : -1;
    }
    return SG_OK;
}

int sg_get_randoms(const sg_lattice *lat, uint32_t *out, size_t n)
{
    if (!lat || !out)
        return fail(SG_EINVAL, "NULL argument");
    if (n != (size_t)lat->V)
        return fail(SG_EINVAL, "n must be L^3");
    if (lat->t == 0)
        return fail(SG_EINVAL, "no sweep done yet");
    if (lat->prng == SG_PHILOX)
        return fail(SG_EINVAL, "per-sample numbers: 64 per site, not one");
    hipError_t e;
    if (buffered_draws(lat->prng)) {
        e = hipMemcpyAsync(out, lat->rbuf + (size_t)lat->rlast * n, 4 * n, hipMemcpyDeviceToHost, lat->stream);
    } else {
        // MINSTD draws are a function of (site, sweep): a kernel evaluates the last
        // sweep's with the sweep kernels' own seed and jump functions, into the spare
        // spin buffer (free between calls: the next fused sweep writes all of it)
        uint32_t *dev = reinterpret_cast<uint32_t *>(lat->spins[1 - lat->cur]);
        e = launch_minstd_draws(dev, lat->L, minstd_multiplier(lat->t - 1), lat->minstd_k, lat->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, dev, 4 * n, hipMemcpyDeviceToHost, lat->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    return check_hip(e, "get randoms");
}

int64_t sg_sweep_count(const sg_lattice *lat) { return lat ? lat->t : -1; }

int sg_set_sweep_count(sg_lattice *lat, int64_t t)
{
    if (!lat || t < 0)
        return fail(SG_EINVAL, "bad argument");
    if (!buffered_draws(lat->prng)) {  // draws are functions of (site, sweep)
        lat->t = t;
        return SG_OK;
    }
    if (t < lat->t || lat->t != 0)
        return fail(SG_EINVAL, "a lattice with stream states can only be moved forward before its first sweep");
    for (int64_t k = 0; k < t; ++k) {
        hipError_t e = lat->prng == SG_MT19937
                           ? launch_mt_fill(&lat->mt_state, &lat->rbuf, 1, lat->L, k, 1, lat->stream)
                           : launch_pr_fill(&lat->mt_state, &lat->rbuf, 1, lat->L, k, 1, lat->stream);
        if (e != hipSuccess)
            return hip_fail(e, "stream fill");
    }
    lat->rlast = 0;
    lat->t = t;
    return check_hip(hipStreamSynchronize(lat->stream), "synchronize");
}

int sg_flip_words(int form, const uint64_t *in, const uint32_t *R, uint64_t n, double beta, int prng, uint64_t *out,
                  void *stream)
{
    if (form < 0 || form > 3)
        return fail(SG_EINVAL, "form must be 0..3");
    if (check_beta(beta) != SG_OK)
        return SG_EINVAL;
    if (!valid_prng(prng))
        return fail(SG_EINVAL, "unknown prng");
    if ((form & 2) == 0 && prng != SG_MINSTD)
        return fail(SG_EINVAL, "the 32-bit comparisons (forms 0, 1) hold only for MINSTD's thresholds");
    if (n > 0 && (!in || !R || !out))
        return fail(SG_EINVAL, "NULL buffer");
    uint64_t T[3];
    sg_thresholds(beta, prng, T);
    return check_hip(launch_flip_words(form, in, R, n, Thresholds{T[0], T[1], T[2]}, out,
                                       static_cast<hipStream_t>(stream)),
                     "flip rule launch");
}

int sg_probe_bandwidth(int kind, void *dst, const void *src, size_t bytes, int blocks, void *stream)
{
    if (kind < 0 || kind > 5)
        return fail(SG_EINVAL, "kind must be 0 (read), 1 (copy), 2 (fill), or 3..5 for their streaming forms");
    if (blocks == 0)
        blocks = 4096;
    if (blocks < 1 || blocks > 65536)
        return fail(SG_EINVAL, "blocks must be in [1, 65536]");
    if (bytes < 16 || (bytes & 15) != 0)
        return fail(SG_EINVAL, "bytes must be a positive multiple of 16");
    if (!dst || (kind != 2 && kind != 5 && !src))
        return fail(SG_EINVAL, "NULL buffer");
    if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) != 0)
        return fail(SG_EINVAL, "buffers must be 16-byte aligned");
    return check_hip(launch_probe(kind, dst, src, bytes, blocks, static_cast<hipStream_t>(stream)), "probe launch");
}

int sg_stream_state_bytes(const sg_lattice *lat, size_t *bytes)
{
    if (!lat || !bytes)
        return fail(SG_EINVAL, "NULL argument");
    const size_t cols = (size_t)lat->L * lat->L;
    *bytes = lat->prng == SG_MT19937 ? 4 * (size_t)kMtN * cols : lat->prng == SG_PARISI_RAPUANO ? 4 * 64 * cols : 0;
    return SG_OK;
}

int sg_get_stream_state(const sg_lattice *lat, void *out, size_t bytes)
{
    size_t need = 0;
    if (sg_stream_state_bytes(lat, &need) != SG_OK)
        return SG_EINVAL;
    if (bytes != need || (need > 0 && !out))
        return fail(SG_EINVAL, "bytes must be sg_stream_state_bytes() (" + std::to_string(need) + ")");
    if (need == 0)
        return SG_OK;
    hipError_t e = hipMemcpyAsync(out, lat->mt_state, need, hipMemcpyDeviceToHost, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    return check_hip(e, "get stream state");
}

int sg_set_stream_state(sg_lattice *lat, const void *in, size_t bytes, int64_t t)
{
    size_t need = 0;
    if (sg_stream_state_bytes(lat, &need) != SG_OK)
        return SG_EINVAL;
    if (t < 0)
        return fail(SG_EINVAL, "t < 0");
    if (bytes != need || (need > 0 && !in))
        return fail(SG_EINVAL, "bytes must be sg_stream_state_bytes() (" + std::to_string(need) + ")");
    if (need > 0) {
        hipError_t e = hipMemcpyAsync(lat->mt_state, in, need, hipMemcpyHostToDevice, lat->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(lat->stream);  // `in` is only borrowed
        if (e != hipSuccess)
            return hip_fail(e, "set stream state");
    }
    lat->t = t;
    lat->rlast = 0;
    return SG_OK;
}

int sg_set_kernel(sg_lattice *lat, int kind, int tile_x, int tile_y, int z_chunk, int band)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    if (kind != SG_KERNEL_AUTO && kind != SG_KERNEL_TWOPASS && kind != SG_KERNEL_FUSED && kind != SG_KERNEL_FUSED2)
        return fail(SG_EINVAL, "unknown kernel");
    if (band < 0)
        return fail(SG_EINVAL, "band must be >= 0");
    if (kind == SG_KERNEL_FUSED && (tile_x != 0 || tile_y != 0)) {
        if (!fused_shape_ok(lat->L, 1, tile_x, tile_y, z_chunk))
            return fail(SG_EINVAL, "invalid fused tile shape");
    } else if (kind == SG_KERNEL_FUSED2 && (tile_x != 0 || tile_y != 0)) {
        if (!fused2_shape_ok(lat->L, tile_x, tile_y, z_chunk))
            return fail(SG_EINVAL, "invalid two-sweep tile shape");
    } else if (z_chunk < 0 || z_chunk > lat->L) {
        return fail(SG_EINVAL, "invalid z_chunk");
    }
    lat->kernel = kind;
    lat->band = band;
    lat->ring = 0;
    if (kind == SG_KERNEL_FUSED || kind == SG_KERNEL_FUSED2) {
        lat->tile_x = tile_x;
        lat->tile_y = tile_y;
        lat->z_chunk = z_chunk;
    } else {
        lat->tile_x = lat->tile_y = 0;
        lat->z_chunk = z_chunk;
    }
    return SG_OK;
}

int sg_set_ring(sg_lattice *lat, int planes)
{
    if (!lat)
        return fail(SG_EINVAL, "NULL lattice");
    if (planes != 0 && planes != 5 && planes != 6)
        return fail(SG_EINVAL, "planes in flight must be 0 (default), 5 or 6");
    if (planes == 6 && buffered_draws(lat->prng))
        return fail(SG_EINVAL, "with buffered draws the two-sweep march keeps 5 planes in flight");
    lat->ring = planes;
    return SG_OK;
}

int sg_get_kernel(const sg_lattice *lat, int out[6])
{
    if (!lat || !out)
        return fail(SG_EINVAL, "NULL argument");
    int tx = 0, ty = 0, zc = 0;
    const int kind = pick_kernel(lat, 1, tx, ty, zc);
    if (kind < 0)
        return kind;
    out[0] = kind == 2 ? SG_KERNEL_FUSED2 : (kind == 1 ? SG_KERNEL_FUSED : SG_KERNEL_TWOPASS);
    out[1] = tx;
    out[2] = ty;
    out[3] = zc;
    out[4] = lat->band > 0 ? lat->band : 1;
    out[5] = kind == 2 ? (lat->ring ? lat->ring : fused2_default_ring(lat->L)) : 0;
    return SG_OK;
}

namespace {
struct TuneKey {
    int dev, L, n, prng;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(dev, L, n, prng) < std::tie(o.dev, o.L, o.n, o.prng);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, 6>> g_tuned;  // kind, tile_x, tile_y, z_chunk, band, ring
}  // namespace

int sg_autotune(sg_lattice *const *lats, int n, int reps, int best[5], double *ms)
{
    if (!lats || n < 1 || n > 2)
        return fail(SG_EINVAL, "autotune takes 1 or 2 lattices");
    for (int r = 0; r < n; ++r)
        if (!lats[r] || lats[r]->L != lats[0]->L || lats[r]->prng != lats[0]->prng || lats[r]->J != lats[0]->J ||
            lats[r]->stream != lats[0]->stream)
            return fail(SG_EMISMATCH, "autotune: lattices must share L, prng, couplings and stream");
    for (int r = 1; r < n; ++r)
        if (lats[r] == lats[0])
            return fail(SG_EINVAL, "a lattice appears twice");
    sg_lattice *l0 = lats[0];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        dev = 0;
    const TuneKey key{dev, l0->L, n, l0->prng};
    std::array<int, 6> pick{0, 0, 0, 0, 1, 0};
    double pick_ms = -1.0;
    bool cached = false;
    if (reps >= 0) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            pick = it->second;
            cached = true;
        }
    }
    if (!cached) {
        const int nrep_launch = reps > 0 ? reps : 5;
        uint64_t T[3];
        sg_thresholds(1.0, l0->prng, T);
        SweepArgs a{};
        a.J = l0->J;
        a.nrep = n;
        a.L = l0->L;
        a.prng = buffered_draws(l0->prng) ? SG_MT19937 : l0->prng;
        a.minstd_a = 16807u;
        a.minstd_a2 = 282475249u;
        a.t = l0->t;
        a.T = Thresholds{T[0], T[1], T[2]};
        for (int r = 0; r < n; ++r) {
            a.src[r] = lats[r]->spins[lats[r]->cur];
            a.dst[r] = lats[r]->spins[1 - lats[r]->cur];
            a.rnd[r] = lats[r]->rbuf;
            a.mk[r] = lats[r]->minstd_k;
            a.pkey[r] = lats[r]->key_philox;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0)
                (void)hipEventDestroy(e0);
            return fail(SG_EDEVICE, "autotune: cannot create events");
        }
        const int P = l0->L / 2;
        const int txs[] = {8, 16, 32, 64};
        const int tys[] = {4, 6, 8, 12, 16, 24};
        const int bands[] = {1, 2, 4};
        double best_ms = 1e300;
        int rc = SG_OK;
        auto time_launches = [&](auto launch, float &t_ms) {
            hipError_t e = launch();  // warm-up
            if (e == hipSuccess)
                e = hipEventRecord(e0, l0->stream);
            for (int k = 0; e == hipSuccess && k < nrep_launch; ++k)
                e = launch();
            if (e == hipSuccess)
                e = hipEventRecord(e1, l0->stream);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&t_ms, e0, e1);
            return e;
        };
        {
            // kind 0: the two-pass kernel updates in place, so it is timed on a copy of
            // the spins in the spare buffer; the lattices' own spins stay as they are
            SweepArgs b = a;
            hipError_t e = hipSuccess;
            for (int r = 0; r < n && e == hipSuccess; ++r) {
                e = hipMemcpyAsync(a.dst[r], a.src[r], 8 * (size_t)l0->V, hipMemcpyDeviceToDevice, l0->stream);
                b.src[r] = a.dst[r];
            }
            float t_ms = 0.f;
            if (e == hipSuccess)
                e = time_launches([&]() { return launch_sweep_twopass(b, l0->stream); }, t_ms);
            if (e != hipSuccess)
                rc = hip_fail(e, "autotune launch");
            else {
                best_ms = (double)t_ms / nrep_launch;
                pick = {SG_KERNEL_TWOPASS, 0, 0, 0, 1, 0};
            }
        }
        // kind 1: one sweep per launch; kind 2: two, with a ring of 5 or 6 planes (5
        // only for buffered draws); compared per sweep
        for (int kind = 1; kind <= 2 && rc == SG_OK; ++kind) {
            for (int ring : {5, 6}) {
                if (ring == 6 && (kind == 1 || buffered_draws(l0->prng)))
                    break;
                for (int tx : txs) {
                    if (tx > P)
                        continue;
                    for (int ty : tys) {
                        if (ty > l0->L)
                            continue;
                        if (kind == 1 ? !fused_shape_ok(l0->L, n, tx, ty, 0) : !fused2_shape_ok(l0->L, tx, ty, 0))
                            continue;
                        for (int band : bands) {
                            auto launch = [&]() {
                                return kind == 1 ? launch_sweep_fused(a, tx, ty, 0, band, l0->stream)
                                                 : launch_sweep_fused2(a, tx, ty, 0, band, ring, l0->stream);
                            };
                            float t_ms = 0.f;
                            const hipError_t e = time_launches(launch, t_ms);
                            if (e != hipSuccess) {
                                rc = hip_fail(e, "autotune launch");
                                break;
                            }
                            const double per_sweep = (double)t_ms / nrep_launch / kind;
                            if (per_sweep < best_ms) {
                                best_ms = per_sweep;
                                pick = {kind == 1 ? SG_KERNEL_FUSED : SG_KERNEL_FUSED2, tx, ty, 0, band,
                                        kind == 1 ? 0 : ring};
                            }
                        }
                        if (rc != SG_OK)
                            break;
                    }
                    if (rc != SG_OK)
                        break;
                }
                if (rc != SG_OK)
                    break;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != SG_OK)
            return rc;
        if (pick[0] == 0)
            return fail(SG_EINVAL, "autotune: no kernel could be timed");
        pick_ms = best_ms;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[key] = pick;
    }
    for (int r = 0; r < n; ++r) {
        lats[r]->kernel = pick[0];
        lats[r]->tile_x = pick[1];
        lats[r]->tile_y = pick[2];
        lats[r]->z_chunk = pick[3];
        lats[r]->band = pick[4];
        lats[r]->ring = pick[5];
    }
    if (best)
        for (int k = 0; k < 5; ++k)
            best[k] = pick[k];
    if (ms)
        *ms = pick_ms;
    return SG_OK;
}

int sg_destroy(sg_lattice *lat)
{
    delete H(lat);
    return SG_OK;
}

}  // extern "C"
