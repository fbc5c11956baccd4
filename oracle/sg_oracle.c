/*
 * CPU oracle for the checkerboard Metropolis dynamics of the 3D Edwards-Anderson
 * spin glass with bimodal couplings (Lulli, Bernaschi, Parisi, "Highly optimized
 * simulations on single- and multi-GPU systems of 3D Ising spin glass",
 * arXiv:1411.0127).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this file.  It shares no code with
 * the GPU library: it is the plain definition of what the GPU path computes, one
 * signed byte per spin, one sample at a time, in the order the paper states it.
 *
 * Conventions (readings of the paper, each justified where it is used):
 *   - extents Lx, Ly, Lz are even (Sec. 1: checkerboard needs L = 2n);
 *   - site index i = x + Lx*(y + Ly*z);
 *   - J[d*V + i] is the coupling of the bond between i and its +d neighbour
 *     (periodic), d = 0,1,2 for x,y,z; every site owns three bonds, 3V in all;
 *   - "red" sites have x+y+z even and are updated first, then the "blue" ones;
 *     one red pass plus one blue pass is one sweep (Sec. 1; psFlip definition
 *     in Sec. 4.1 times red + blue);
 *   - the random number used by site i in a sweep is R[i], an unsigned integer
 *     handed in by the caller; the generators that produce it are below.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* MINSTD (Sec. 3, Lehmer / Park-Miller congruential generator):             */
/*   R_{n+1} = 16807 * R_n  mod  (2^31 - 1).                                  */
/* Written with a plain 64-bit product and the % operator: slow and obvious.  */
/* ------------------------------------------------------------------------- */
uint32_t oc_minstd_next(uint32_t r)
{
    return (uint32_t)(((uint64_t)16807u * (uint64_t)r) % 2147483647ull);
}

/* Advance every per-site MINSTD state once and return the new values.
 * One draw per site per sweep, shared by every sample coded at that site
 * (asynchronous multispin coding, Sec. 4). */
void oc_minstd_draws(int64_t V, uint32_t *state, uint32_t *R)
{
    for (int64_t i = 0; i < V; ++i) {
        state[i] = oc_minstd_next(state[i]);
        R[i] = state[i];
    }
}

/* ------------------------------------------------------------------------- */
/* MT19937 (Sec. 3; M. Matsumoto and T. Nishimura, ACM TOMACS 8 (1998) 3-30). */
/* State of 624 words, initialised by the published init_genrand recurrence;  */
/* a full twist regenerates all 624 words when they are used up; outputs are  */
/* tempered.                                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t mt[624];
    int32_t mti;
} oc_mt;

void oc_mt_init(oc_mt *s, uint32_t seed)
{
    s->mt[0] = seed;
    for (int k = 1; k < 624; ++k) {
        uint32_t prev = s->mt[k - 1];
        s->mt[k] = 1812433253u * (prev ^ (prev >> 30)) + (uint32_t)k;
    }
    s->mti = 624;
}

static void oc_mt_twist(oc_mt *s)
{
    for (int k = 0; k < 624; ++k) {
        uint32_t y = (s->mt[k] & 0x80000000u) | (s->mt[(k + 1) % 624] & 0x7fffffffu);
        uint32_t v = s->mt[(k + 397) % 624] ^ (y >> 1);
        if (y & 1u)
            v ^= 0x9908b0dfu;
        s->mt[k] = v;
    }
    s->mti = 0;
}

uint32_t oc_mt_next(oc_mt *s)
{
    if (s->mti >= 624)
        oc_mt_twist(s);
    uint32_t y = s->mt[s->mti++];
    y ^= y >> 11;
    y ^= (y << 7) & 0x9d2c5680u;
    y ^= (y << 15) & 0xefc60000u;
    y ^= y >> 18;
    return y;
}

int64_t oc_mt_sizeof(void) { return (int64_t)sizeof(oc_mt); }

void oc_mt_init_many(int64_t n, oc_mt *s, const uint32_t *seeds)
{
    for (int64_t c = 0; c < n; ++c)
        oc_mt_init(&s[c], seeds[c]);
}

void oc_mt_outputs(uint32_t seed, int64_t n, uint32_t *out)
{
    oc_mt s;
    oc_mt_init(&s, seed);
    for (int64_t k = 0; k < n; ++k)
        out[k] = oc_mt_next(&s);
}

/* One stream per x-y column c = x + Lx*y; within a sweep the column's site at
 * height z takes the column's next output, z = 0, 1, ..., Lz-1 in order. */
void oc_mt_draws(int Lx, int Ly, int Lz, oc_mt *cols, uint32_t *R)
{
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            oc_mt *s = &cols[x + (int64_t)Lx * y];
            for (int z = 0; z < Lz; ++z)
                R[x + (int64_t)Lx * (y + (int64_t)Ly * z)] = oc_mt_next(s);
        }
}

/* ------------------------------------------------------------------------- */
/* Parisi-Rapuano (Sec. 3; G. Parisi, F. Rapuano, Phys. Lett. B 157 (1985)     */
/* 301): a lagged-Fibonacci generator,                                        */
/*   x_n = x_{n-24} + x_{n-55}  (mod 2^32),   R_n = x_n XOR x_{n-61},          */
/* started from 61 seed words x_{-61} .. x_{-1}.  The state is a circular     */
/* buffer of 64 words, x_n at index n mod 64 (61 live words suffice).         */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t w[64];
    int64_t n; /* index of the next number */
} oc_pr;

int64_t oc_pr_sizeof(void) { return (int64_t)sizeof(oc_pr); }

void oc_pr_init(oc_pr *s, const uint32_t seed[61])
{
    memset(s, 0, sizeof(*s));
    for (int k = 0; k < 61; ++k)
        s->w[(k - 61 + 64) & 63] = seed[k];
    s->n = 0;
}

uint32_t oc_pr_next(oc_pr *s)
{
    const int64_t n = s->n;
    const uint32_t x = s->w[(n - 24) & 63] + s->w[(n - 55) & 63];
    const uint32_t r = x ^ s->w[(n - 61) & 63];
    s->w[n & 63] = x;
    s->n = n + 1;
    return r;
}

void oc_pr_init_many(int64_t n, oc_pr *s, const uint32_t *seeds)
{
    for (int64_t c = 0; c < n; ++c)
        oc_pr_init(&s[c], seeds + 61 * c);
}

void oc_pr_outputs(const uint32_t seed[61], int64_t n, uint32_t *out)
{
    oc_pr s;
    oc_pr_init(&s, seed);
    for (int64_t k = 0; k < n; ++k)
        out[k] = oc_pr_next(&s);
}

/* Column streams as for MT19937: in a sweep the site at height z of column c
 * takes that column's next number, z = 0 .. Lz-1 in order. */
void oc_pr_draws(int Lx, int Ly, int Lz, oc_pr *cols, uint32_t *R)
{
    const int64_t LL = (int64_t)Lx * Ly;
    for (int64_t c = 0; c < LL; ++c)
        for (int z = 0; z < Lz; ++z)
            R[z * LL + c] = oc_pr_next(&cols[c]);
}

/* ------------------------------------------------------------------------- */
/* Per-sample draws (a variant of Sec. 4 with one random number per coded     */
/* sample instead of one per site word): Philox4x32-10 (J. K. Salmon, M. A.  */
/* Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, */
/* 3", SC'11), a counter-based generator: ten rounds of a multiply-and-xor    */
/* bijection of a 128-bit counter, the 64-bit key bumped by two Weyl constants */
/* between rounds.                                                             */
/* ------------------------------------------------------------------------- */
void oc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n[4] = {(uint32_t)(p1 >> 32) ^ c[1] ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c[3] ^ k1,
                               (uint32_t)p0};
        memcpy(c, n, sizeof(c));
    }
    memcpy(out, c, sizeof(c));
}

/* The 32-bit numbers of the 64 samples at site i in sweep t (this project's
 * convention): 32 bit-planes W[0..31] of 64 bits, bit j of W[b] being bit 31-b
 * of sample j's number; planes 2q and 2q+1 are the outputs (o0 | o1 << 32) and
 * (o2 | o3 << 32) of Philox4x32-10 at counter (lo32(i), hi32(i) << 8 | q,
 * lo32(t), hi32(t)) under key (lo32(key), hi32(key)). */
static void sample_draws_n(uint64_t key, int64_t i, int64_t t, int n, uint32_t *R)
{
    uint64_t W[32];
    const uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    for (int q = 0; q < 16; ++q) {
        const uint32_t ctr[4] = {(uint32_t)i, ((uint32_t)((uint64_t)i >> 32) << 8) | (uint32_t)q, (uint32_t)t,
                                 (uint32_t)((uint64_t)t >> 32)};
        uint32_t o[4];
        oc_philox4x32_10(ctr, k, o);
        W[2 * q] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        W[2 * q + 1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    }
    for (int j = 0; j < n; ++j) {
        uint32_t r = 0;
        for (int b = 0; b < 32; ++b)
            r |= (uint32_t)((W[b] >> j) & 1u) << (31 - b);
        R[j] = r;
    }
}

void oc_sample_draws(uint64_t key, int64_t i, int64_t t, uint32_t R[64]) { sample_draws_n(key, i, t, 64, R); }

/* Numbers of every site for samples 0..S-1 in sweep t: R[j*V + i]. */
void oc_sample_draws_all(int64_t V, int S, uint64_t key, int64_t t, uint32_t *R)
{
    uint32_t r[64];
    for (int64_t i = 0; i < V; ++i) {
        sample_draws_n(key, i, t, S, r);
        for (int j = 0; j < S; ++j)
            R[(int64_t)j * V + i] = r[j];
    }
}

/* ------------------------------------------------------------------------- */
/* Integer acceptance thresholds (Sec. 4): a flip with energy change dE > 0 is */
/* accepted when the integer random number R is below R_max * exp(-beta dE),   */
/* called EXP4, EXP8, EXP12.  Reading: R_max is the size of the generator's    */
/* output range (2^31 - 1 for MINSTD, whose outputs lie in [1, 2^31 - 2];      */
/* 2^32 for MT19937, Parisi-Rapuano and the per-sample Philox numbers), the     */
/* product is rounded  */
/* up, and the test is strict, so                                             */
/* R < T holds exactly when R < R_max * p; beta = 0 then accepts every          */
/* proposal and beta = +inf none.  T[k-1] is the threshold for dE = 4k.        */
/* ------------------------------------------------------------------------- */
void oc_thresholds(double beta, uint64_t range, uint64_t T[3])
{
    for (int k = 1; k <= 3; ++k) {
        double dE = 4.0 * k;
        double p = exp(-(beta * dE));
        T[k - 1] = (uint64_t)ceil((double)range * p);
    }
}

/* ------------------------------------------------------------------------- */
/* One Metropolis sweep of one sample (Sec. 1 checkerboard; Sec. 4 P_flip).   */
/* s: V spins in {-1,+1}; J: 3V couplings in {-1,+1}; R: one number per site. */
/* ------------------------------------------------------------------------- */
static inline int64_t idx(int Lx, int Ly, int x, int y, int z)
{
    return x + (int64_t)Lx * (y + (int64_t)Ly * z);
}

/* Update the sites of one colour in planes z0 .. z1-1.  Sites of one colour
 * have no bond between them (checkerboard, Sec. 1), so the planes of a colour
 * pass may be visited in any order, or split among threads, with the same
 * result. */
static void sweep_colour(int Lx, int Ly, int Lz, int8_t *s, const int8_t *J, const uint32_t *R,
                         const uint64_t T[3], int colour, int z0, int z1)
{
    const int64_t V = (int64_t)Lx * Ly * Lz;
    for (int z = z0; z < z1; ++z)
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x) {
                if (((x + y + z) & 1) != colour)
                    continue;
                const int xp = (x + 1) % Lx, xm = (x + Lx - 1) % Lx;
                const int yp = (y + 1) % Ly, ym = (y + Ly - 1) % Ly;
                const int zp = (z + 1) % Lz, zm = (z + Lz - 1) % Lz;
                const int64_t i = idx(Lx, Ly, x, y, z);
                /* local field: the three bonds the site owns and the three
                 * bonds its -d neighbours own towards it */
                int h = J[0 * V + i] * s[idx(Lx, Ly, xp, y, z)]
                      + J[1 * V + i] * s[idx(Lx, Ly, x, yp, z)]
                      + J[2 * V + i] * s[idx(Lx, Ly, x, y, zp)]
                      + J[0 * V + idx(Lx, Ly, xm, y, z)] * s[idx(Lx, Ly, xm, y, z)]
                      + J[1 * V + idx(Lx, Ly, x, ym, z)] * s[idx(Lx, Ly, x, ym, z)]
                      + J[2 * V + idx(Lx, Ly, x, y, zm)] * s[idx(Lx, Ly, x, y, zm)];
                /* H = -sum J s_i s_k, so flipping s_i changes it by 2 s_i h */
                const int dE = 2 * s[i] * h;
                int accept;
                if (dE <= 0)
                    accept = 1;
                else
                    accept = (uint64_t)R[i] < T[dE / 4 - 1];
                if (accept)
                    s[i] = (int8_t)(-s[i]);
            }
}

void oc_sweep(int Lx, int Ly, int Lz, int8_t *s, const int8_t *J, const uint32_t *R,
              const uint64_t T[3])
{
    for (int colour = 0; colour < 2; ++colour)
        sweep_colour(Lx, Ly, Lz, s, J, R, T, colour, 0, Lz);
}

/* Number of unsatisfied bonds U (bonds with -J s_i s_k = +1); the energy of
 * Eq. (1) is E = 2U - 3V. */
int64_t oc_unsatisfied(int Lx, int Ly, int Lz, const int8_t *s, const int8_t *J)
{
    const int64_t V = (int64_t)Lx * Ly * Lz;
    int64_t U = 0;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x) {
                const int64_t i = idx(Lx, Ly, x, y, z);
                const int64_t nb[3] = {idx(Lx, Ly, (x + 1) % Lx, y, z),
                                       idx(Lx, Ly, x, (y + 1) % Ly, z),
                                       idx(Lx, Ly, x, y, (z + 1) % Lz)};
                for (int d = 0; d < 3; ++d)
                    U += (-J[d * V + i] * s[i] * s[nb[d]]) > 0;
            }
    return U;
}

/* Number of sites where two replicas differ; q = 1 - 2 N / V. */
int64_t oc_ndiff(int64_t V, const int8_t *a, const int8_t *b)
{
    int64_t n = 0;
    for (int64_t i = 0; i < V; ++i)
        n += a[i] != b[i];
    return n;
}

/* ------------------------------------------------------------------------- */
/* Exact Gibbs averages (Eq. (3)) by enumeration of all 2^V configurations,   */
/* V <= 24.  Outputs <E>, <E^2> and the probability of each energy level      */
/* E = -3V + 2U, U = 0..3V (hist has 3V+1 entries).                           */
/* ------------------------------------------------------------------------- */
int oc_gibbs(int Lx, int Ly, int Lz, const int8_t *J, double beta, double *meanE,
             double *meanE2, double *hist)
{
    const int64_t V = (int64_t)Lx * Ly * Lz;
    if (V > 24)
        return -1;
    int8_t *s = (int8_t *)malloc((size_t)V);
    double *w = (double *)calloc((size_t)(3 * V + 1), sizeof(double));
    if (!s || !w) {
        free(s);
        free(w);
        return -2;
    }
    /* count states per U first, then weight: exact in double for V <= 24 */
    for (uint64_t c = 0; c < (1ull << V); ++c) {
        for (int64_t i = 0; i < V; ++i)
            s[i] = (c >> i) & 1 ? 1 : -1;
        w[oc_unsatisfied(Lx, Ly, Lz, s, J)] += 1.0;
    }
    int64_t Umin = 0;
    while (w[Umin] == 0.0)
        ++Umin;
    double Z = 0.0, e1 = 0.0, e2 = 0.0;
    for (int64_t U = 0; U <= 3 * V; ++U) {
        double E = 2.0 * U - 3.0 * V;
        double b = w[U] * exp(-beta * 2.0 * (double)(U - Umin));
        hist[U] = b;
        Z += b;
        e1 += b * E;
        e2 += b * E * E;
    }
    for (int64_t U = 0; U <= 3 * V; ++U)
        hist[U] /= Z;
    *meanE = e1 / Z;
    *meanE2 = e2 / Z;
    free(s);
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* n sweeps of S samples sharing one stream set (prng 0: per-site MINSTD       */
/* states, 1: per-column MT19937 states, 2: per-sample Philox numbers with     */
/* state {key, next sweep index}, 3: per-column Parisi-Rapuano states),       */
/* thresholds fixed.  Records the                                              */
/* unsatisfied-bond count of every sample after every sweep when U != NULL     */
/* (U[t*S + j]).  s: S*V bytes; J: S*3V bytes, sample-major.                    */
/* ------------------------------------------------------------------------- */
int oc_run(int Lx, int Ly, int Lz, int S, int8_t *s, const int8_t *J, int prng, void *state,
           int64_t nsweeps, const uint64_t T[3], int64_t *U)
{
    const int64_t V = (int64_t)Lx * Ly * Lz;
    uint32_t *R = (uint32_t *)malloc((size_t)V * (prng == 2 ? S : 1) * sizeof(uint32_t));
    if (!R)
        return -2;
    for (int64_t t = 0; t < nsweeps; ++t) {
        if (prng == 0) {
            oc_minstd_draws(V, (uint32_t *)state, R);
        } else if (prng == 1) {
            oc_mt_draws(Lx, Ly, Lz, (oc_mt *)state, R);
        } else if (prng == 3) {
            oc_pr_draws(Lx, Ly, Lz, (oc_pr *)state, R);
        } else {
            uint64_t *ks = (uint64_t *)state;
            oc_sample_draws_all(V, S, ks[0], (int64_t)ks[1], R);
            ks[1] += 1;
        }
        for (int j = 0; j < S; ++j) {
            oc_sweep(Lx, Ly, Lz, s + (int64_t)j * V, J + (int64_t)j * 3 * V, R + (prng == 2 ? (int64_t)j * V : 0), T);
            if (U)
                U[t * S + j] = oc_unsatisfied(Lx, Ly, Lz, s + (int64_t)j * V, J + (int64_t)j * 3 * V);
        }
    }
    free(R);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The same run spread over host threads, for timing the oracle on all cores. */
/* Nothing is computed differently: the draws of a sweep are per site (MINSTD, */
/* per-sample numbers) or per column (MT19937, Parisi-Rapuano), so ranges of   */
/* sites or columns go to different threads; a colour pass is split by planes, */
/* which is allowed because sites of one colour are independent (Sec. 1); the  */
/* two colour passes and the sweeps stay in order.  The result equals oc_run's. */
/* ------------------------------------------------------------------------- */
typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi);
typedef struct {
    range_fn fn;
    void *ctx;
    int64_t lo, hi;
} range_job;

static void *range_main(void *p)
{
    range_job *j = (range_job *)p;
    j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

/* fn(ctx, lo, hi) over [0, n) in nthreads contiguous pieces; a piece whose
 * thread cannot be started runs on the calling thread. */
static void parallel_for(int nthreads, int64_t n, range_fn fn, void *ctx)
{
    enum { kMaxThreads = 256 };
    if (nthreads > kMaxThreads)
        nthreads = kMaxThreads;
    if (nthreads > n)
        nthreads = (int)n;
    if (nthreads <= 1) {
        fn(ctx, 0, n);
        return;
    }
    pthread_t th[kMaxThreads];
    range_job job[kMaxThreads];
    int started[kMaxThreads];
    for (int k = 0; k < nthreads; ++k) {
        job[k].fn = fn;
        job[k].ctx = ctx;
        job[k].lo = n * k / nthreads;
        job[k].hi = n * (k + 1) / nthreads;
        started[k] = pthread_create(&th[k], NULL, range_main, &job[k]) == 0;
        if (!started[k])
            fn(ctx, job[k].lo, job[k].hi);
    }
    for (int k = 0; k < nthreads; ++k)
        if (started[k])
            pthread_join(th[k], NULL);
}

typedef struct {
    int Lx, Ly, Lz, S, prng, colour;
    int8_t *s;
    const int8_t *J;
    void *state;
    const uint32_t *R;
    uint32_t *Rout;
    const uint64_t *T;
    uint64_t key;
    int64_t t;
} run_ctx;

static void draws_range(void *p, int64_t lo, int64_t hi)
{
    run_ctx *c = (run_ctx *)p;
    const int64_t LL = (int64_t)c->Lx * c->Ly, V = LL * c->Lz;
    if (c->prng == 0) { /* sites lo..hi-1 */
        uint32_t *st = (uint32_t *)c->state;
        for (int64_t i = lo; i < hi; ++i) {
            st[i] = oc_minstd_next(st[i]);
            c->Rout[i] = st[i];
        }
    } else if (c->prng == 1 || c->prng == 3) { /* columns lo..hi-1 */
        for (int64_t col = lo; col < hi; ++col)
            for (int z = 0; z < c->Lz; ++z)
                c->Rout[z * LL + col] = c->prng == 1 ? oc_mt_next(&((oc_mt *)c->state)[col])
                                                     : oc_pr_next(&((oc_pr *)c->state)[col]);
    } else { /* per-sample numbers of sites lo..hi-1 */
        uint32_t r[64];
        for (int64_t i = lo; i < hi; ++i) {
            sample_draws_n(c->key, i, c->t, c->S, r);
            for (int j = 0; j < c->S; ++j)
                c->Rout[(int64_t)j * V + i] = r[j];
        }
    }
}

static void colour_range(void *p, int64_t lo, int64_t hi)
{
    run_ctx *c = (run_ctx *)p;
    sweep_colour(c->Lx, c->Ly, c->Lz, c->s, c->J, c->R, c->T, c->colour, (int)lo, (int)hi);
}

int oc_run_threads(int Lx, int Ly, int Lz, int S, int8_t *s, const int8_t *J, int prng, void *state,
                   int64_t nsweeps, const uint64_t T[3], int64_t *U, int nthreads)
{
    const int64_t LL = (int64_t)Lx * Ly, V = LL * Lz;
    uint32_t *R = (uint32_t *)malloc((size_t)V * (prng == 2 ? S : 1) * sizeof(uint32_t));
    if (!R)
        return -2;
    run_ctx c;
    memset(&c, 0, sizeof(c));
    c.Lx = Lx;
    c.Ly = Ly;
    c.Lz = Lz;
    c.S = S;
    c.prng = prng;
    c.state = state;
    c.Rout = R;
    c.T = T;
    for (int64_t t = 0; t < nsweeps; ++t) {
        if (prng == 2) {
            uint64_t *ks = (uint64_t *)state;
            c.key = ks[0];
            c.t = (int64_t)ks[1];
            parallel_for(nthreads, V, draws_range, &c);
            ks[1] += 1;
        } else {
            parallel_for(nthreads, (prng == 0) ? V : LL, draws_range, &c);
        }
        for (int j = 0; j < S; ++j) {
            c.s = s + (int64_t)j * V;
            c.J = J + (int64_t)j * 3 * V;
            c.R = R + (prng == 2 ? (int64_t)j * V : 0);
            for (int colour = 0; colour < 2; ++colour) {
                c.colour = colour;
                parallel_for(nthreads, Lz, colour_range, &c);
            }
            if (U)
                U[t * S + j] = oc_unsatisfied(Lx, Ly, Lz, c.s, c.J);
        }
    }
    free(R);
    return 0;
}
