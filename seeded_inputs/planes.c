/*
 * Bit planes of the seeded inputs at large sizes (the same definitions as the
 * numpy code of this package, which documents them): the coupling and spin bits
 * of chosen samples, and the per-site MINSTD seeds, for lattices whose full
 * 64-sample words would not fit in host memory.  Input generation only: nothing
 * of the Metropolis method is here.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t out(uint64_t key, uint64_t n) { return mix64(key + n * GAMMA); }

static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

typedef struct {
    int kind; /* 0 couplings, 1 spins, 2 MINSTD seeds */
    int L, np;
    int64_t V, lo, hi;
    uint64_t key;
    const int *planes;
    uint8_t *bits;
    uint32_t *seeds;
} job;

static void *work(void *p)
{
    job *j = (job *)p;
    for (int64_t i = j->lo; i < j->hi; ++i) {
        if (j->kind == 0) {
            for (int d = 0; d < 3; ++d) {
                const uint64_t w = out(j->key, 1ull + 3ull * (uint64_t)i + (uint64_t)d);
                for (int k = 0; k < j->np; ++k)
                    j->bits[((int64_t)k * 3 + d) * j->V + i] = (uint8_t)((w >> j->planes[k]) & 1u);
            }
        } else if (j->kind == 1) {
            const uint64_t w = out(j->key, 1ull + (uint64_t)i);
            for (int k = 0; k < j->np; ++k)
                j->bits[(int64_t)k * j->V + i] = (uint8_t)((w >> j->planes[k]) & 1u);
        } else {
            const int64_t LL = (int64_t)j->L * j->L;
            const uint32_t z = (uint32_t)(i / LL), xy = (uint32_t)(i % LL);
            uint32_t h = fmix32(xy ^ fmix32(z ^ (uint32_t)j->key)) >> 1;
            if (h >= 0x7FFFFFFEu)
                h -= 0x7FFFFFFEu;
            j->seeds[i] = h + 1u;
        }
    }
    return NULL;
}

static void run(job base, int nthreads)
{
    enum { kMax = 256 };
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > kMax)
        nthreads = kMax;
    pthread_t th[kMax];
    job jobs[kMax];
    int started[kMax];
    for (int k = 0; k < nthreads; ++k) {
        jobs[k] = base;
        jobs[k].lo = base.V * k / nthreads;
        jobs[k].hi = base.V * (k + 1) / nthreads;
        started[k] = pthread_create(&th[k], NULL, work, &jobs[k]) == 0;
        if (!started[k])
            work(&jobs[k]);
    }
    for (int k = 0; k < nthreads; ++k)
        if (started[k])
            pthread_join(th[k], NULL);
}

/* bits[k][d][i] = bit planes[k] of the coupling word of bond (i, d). */
void si_coupling_bits(int64_t V, uint64_t key, const int *planes, int np, uint8_t *bits, int nthreads)
{
    job j = {0, 0, np, V, 0, V, key, planes, bits, NULL};
    run(j, nthreads);
}

/* bits[k][i] = bit planes[k] of the initial spin word of site i. */
void si_spin_bits(int64_t V, uint64_t key, const int *planes, int np, uint8_t *bits, int nthreads)
{
    job j = {1, 0, np, V, 0, V, key, planes, bits, NULL};
    run(j, nthreads);
}

/* MINSTD seed of every site, k = low 32 bits of the replica's MINSTD key. */
void si_minstd_seeds(int L, uint32_t k, uint32_t *seeds, int nthreads)
{
    const int64_t V = (int64_t)L * L * L;
    job j = {2, L, 0, V, 0, V, k, NULL, NULL, seeds};
    run(j, nthreads);
}
