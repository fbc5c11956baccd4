/*
 * sg.h -- C ABI of libsg, a gfx950 (MI355X) engine for the checkerboard Metropolis
 * dynamics of the 3D Edwards-Anderson spin glass with bimodal couplings, using
 * asynchronous multispin coding: 64 disorder samples per uint64 word, one bit per
 * spin, one random number per site word shared by its 64 samples.
 *
 * Method: M. Lulli, M. Bernaschi, G. Parisi, "Highly optimized simulations on single-
 * and multi-GPU systems of 3D Ising spin glass", arXiv:1411.0127.
 *   Hamiltonian and couplings ........ Sec. 1, Eqs. (1)-(2)
 *   red/blue checkerboard, balance ... Sec. 1
 *   MINSTD, MT19937 .................. Sec. 3
 *   Metropolis, integer thresholds,
 *   bit encoding, bond bits, bit sum,
 *   flip mask ........................ Sec. 4
 *   psFlip ........................... Sec. 4.1
 *
 * Data layout (one cubic lattice of side L, V = L^3 sites, site index
 * i = x + L*(y + L*z)):
 *   spins     uint64 S[V]     bit j = sample j, 1 <=> sigma = +1 (Sec. 4 bit mapping)
 *   couplings uint64 J[3][V]  J[d][i] = bond (i, i + d^), d = x,y,z; bit j = 1 <=> J = -1
 * Host arrays (sg_lattice_create's J_host, sg_get_couplings) are packed as above.  In
 * the device buffer the three coupling arrays, like the other arrays of a lattice,
 * are placed apart by a small skew beyond their length (so that the same plane of
 * each does not fall on the same memory channels); the buffer's layout is private.
 * One sweep = every red site (x+y+z even) once, then every blue site once.
 *
 * Random streams (this library's convention; all keyed, so results do not depend
 * on the kernel, tile shape or launch split):
 *   SG_MINSTD  one MINSTD stream per site and replica; in sweep t (t = 0, 1, ...)
 *              site i draws 16807^(t+1) * seed_i mod (2^31 - 1), with
 *              seed_i = 1 + ((fmix32((x + L*y) ^ fmix32(z ^ k)) >> 1) mod (2^31 - 2)),
 *              fmix32 the MurmurHash3 finalizer, k the low 32 bits of the
 *              replica's keyed word; no per-site state is stored;
 *   SG_MT19937 one MT19937 stream per x-y column and replica, seeded with
 *              init_genrand; in sweep t the site at height z draws the column's
 *              output number t*L + z;
 *   SG_PARISI_RAPUANO  one Parisi-Rapuano stream per x-y column and replica
 *              (Sec. 3): x_n = x_{n-24} + x_{n-55} mod 2^32, R_n = x_n ^ x_{n-61},
 *              started from 61 seed words x_{-61+k} = lo32(out(key, 1 + 61c + k)),
 *              k = 0..60, the first made odd; the site at height z draws the
 *              column's number t*L + z in sweep t;
 *   SG_PHILOX  one number per coded sample instead of one per site word (a
 *              variant of Sec. 4's asynchronous coding): sample j of site i
 *              draws a 32-bit R_j in sweep t from Philox4x32-10 (Salmon et al.,
 *              SC'11) in bit-sliced form -- plane b (0..31) is a 64-bit word
 *              whose bit j is bit 31-b of R_j, and planes 2q, 2q+1 are the
 *              outputs (o0 | o1 << 32, o2 | o3 << 32) at counter (lo32(i),
 *              hi32(i) << 8 | q, lo32(t), hi32(t)) under the replica's 64-bit
 *              keyed word; the planes are drawn from the most significant down
 *              only until every sample's comparison is decided.
 * The keys, the MT19937 seeds, the initial spins and (unless given) the
 * couplings come from the SplitMix64 keyed generator documented with the
 * seeded-input module (Steele, Lea, Flood 2014), evaluated on the device.
 *
 * Acceptance: a proposal with dE > 0 is accepted iff R < T(dE) with
 * T(dE) = ceil(R_range * exp(-beta * dE)), R_range = 2^31 - 1 (MINSTD) or 2^32
 * (MT19937, PARISI_RAPUANO, PHILOX); dE <= 0 is always accepted (Sec. 4, P_flip and
 * EXP4/EXP8/EXP12).
 *
 * Conventions of every entry point:
 *   - returns SG_OK (0) or a negative SG_E* code; sg_last_error() then holds a
 *     message (per thread);
 *   - device memory belongs to the caller: a lattice lives inside one caller
 *     buffer of at least sg_footprint() bytes, which the library never frees;
 *     it must stay allocated until sg_destroy() of this lattice and of every
 *     replica created from it;
 *   - host pointers are borrowed for the duration of the call;
 *   - work is queued on the hipStream_t given at creation (NULL = default
 *     stream); calls that return data to the host synchronise that stream;
 *   - a handle must not be used from two threads at once.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_lattice sg_lattice;

enum { SG_MINSTD = 0, SG_MT19937 = 1, SG_PHILOX = 2, SG_PARISI_RAPUANO = 3 };

enum {
    SG_OK = 0,
    SG_EINVAL = -1,    /* bad argument: L odd or out of [2, 2048], nsamples not in [1,64],
                          beta < 0 or NaN, unknown prng, NULL where a pointer is needed,
                          buffer too small, wrong element count */
    SG_ENOMEM = -2,    /* host allocation failed */
    SG_EDEVICE = -3,   /* a HIP call or kernel launch failed (message has the HIP error) */
    SG_EMISMATCH = -4  /* lattices that must match (size, samples, couplings) do not */
};

/* Sweep kernels.  Every kernel gives bit-identical spins; they differ in speed.
 * SG_KERNEL_TWOPASS: one launch per colour, in place, one lane per site word.
 * SG_KERNEL_FUSED:   one launch per sweep; each workgroup marches a tile of x-y
 *                    columns along z, red plane k then blue plane k-1, in-plane
 *                    neighbours exchanged through LDS, old/new spins in two
 *                    buffers and tile-edge red sites recomputed by both tiles.
 * SG_KERNEL_FUSED2:  two sweeps per launch: the same march carries sweep t+1 two
 *                    planes behind sweep t, so spins and couplings cross HBM once
 *                    per two sweeps (the buffered generators, SG_MT19937 and
 *                    SG_PARISI_RAPUANO, first write both sweeps' numbers); an odd
 *                    last sweep of a call runs on SG_KERNEL_FUSED.
 * SG_KERNEL_AUTO picks SG_KERNEL_FUSED2 where its tile fits (L >= 8) and
 * SG_KERNEL_FUSED otherwise, with default tiles (sg_autotune picks by timing). */
enum { SG_KERNEL_AUTO = 0, SG_KERNEL_TWOPASS = 1, SG_KERNEL_FUSED = 2, SG_KERNEL_FUSED2 = 3 };

/* Bytes of device memory a lattice needs.  own_couplings = 1 for a lattice that
 * holds its couplings (sg_lattice_create), 0 for a replica that reads another
 * lattice's (sg_lattice_create_replica). */
int sg_footprint(int L, int prng, int own_couplings, size_t *dev_bytes);

/* Create a lattice of side L (even, 2..2048) holding nsamples (1..64) samples.
 * J_host: 3*L^3 coupling words in the layout above, or NULL to generate them
 *         from coupling_seed (Sec. 1: J = +-1 with probability 1/2 each);
 * spin_seed, replica: key the initial spins and the random streams;
 * dev_buf, dev_bytes: caller's device buffer (>= sg_footprint(L, prng, 1));
 * stream: hipStream_t for all work on this lattice, or NULL.
 * Bits j >= nsamples are simulated like the others and ignored by observables. */
int sg_lattice_create(int L, int nsamples, int prng, const uint64_t *J_host,
                      uint64_t coupling_seed, uint64_t spin_seed, uint32_t replica,
                      void *dev_buf, size_t dev_bytes, void *stream, sg_lattice **out);

/* A replica (Sec. 2: same couplings, its own initial spins and evolution):
 * shares base's coupling buffer, draws its spins and streams from
 * (spin_seed, replica).  dev_buf >= sg_footprint(L, prng, 0). */
int sg_lattice_create_replica(const sg_lattice *base, uint64_t spin_seed, uint32_t replica,
                              void *dev_buf, size_t dev_bytes, void *stream,
                              sg_lattice **out);

/* Queue nsweeps >= 0 sweeps at inverse temperature beta >= 0 (beta = +inf allowed:
 * only dE <= 0 is accepted). */
int sg_sweep(sg_lattice *lat, int64_t nsweeps, double beta);

/* The same for n lattices that share one coupling buffer (replicas), moving the
 * couplings once per sweep for all of them when the kernel allows; all must have
 * the same L, prng and stream. */
int sg_sweep_replicas(sg_lattice *const *lats, int n, int64_t nsweeps, double beta);

/* ---- Colour-separated layout (the layout study of Sec. 2) ----------------------
 * Bytes of the work buffer sg_sweep_sliced needs: 32 per site. */
int sg_sliced_footprint(int L, size_t *dev_bytes);

/* nsweeps sweeps with the two-pass kernel on the colour-separated layout: the
 * current spins and the couplings are copied into `work` (caller's device buffer,
 * >= sg_sliced_footprint bytes, 256-byte aligned) with red and blue sites of each
 * row in separate arrays indexed by (z, y, x/2) and each site's three couplings with
 * its colour, swept there, and the spins copied back.  The spins are bit-identical
 * to sg_sweep's; `work` is scratch, free again when the queued work is done. */
int sg_sweep_sliced(sg_lattice *lat, int64_t nsweeps, double beta, void *work, size_t work_bytes);

/* Observables of Sec. 1, Eq. (1), per sample j < nsamples:
 * unsat[j] = number of unsatisfied bonds (-J s_i s_k = +1) among the 3V bonds,
 * e_per_spin[j] = (2*unsat[j] - 3V) / V.  Either output may be NULL. */
int sg_energy(sg_lattice *lat, int64_t *unsat, double *e_per_spin);

/* Two-replica overlap per sample: ndiff[j] = number of sites where the replicas
 * differ, q[j] = 1 - 2*ndiff[j]/V.  a, b: same L and nsamples. */
int sg_overlap(const sg_lattice *a, const sg_lattice *b, int64_t *ndiff, double *q);

/* Spins as +-1 bytes, sample-major: out[j*V + i], j < nsamples; n = nsamples*V. */
int sg_get_spins(const sg_lattice *lat, int8_t *out, size_t n);

/* Raw spin words (n = V) and coupling words (n = 3V). */
int sg_get_words(const sg_lattice *lat, uint64_t *out, size_t n);
int sg_set_words(sg_lattice *lat, const uint64_t *in, size_t n);
int sg_get_couplings(const sg_lattice *lat, uint64_t *out, size_t n);

/* The random number each site used in the last sweep (n = V), for checks;
 * SG_EINVAL for SG_PHILOX lattices, whose samples draw 64 numbers per site. */
int sg_get_randoms(const sg_lattice *lat, uint32_t *out, size_t n);

/* Integer thresholds T[k-1] for dE = 4k, k = 1,2,3 (Sec. 4, EXP4/EXP8/EXP12). */
int sg_thresholds(double beta, int prng, uint64_t T[3]);

/* Sweeps done so far; setting it (resume from a checkpoint) also moves the
 * MINSTD streams; for MT19937 only a lattice that has not swept may be moved
 * forward, by regenerating its streams up to that point. */
int64_t sg_sweep_count(const sg_lattice *lat);
int sg_set_sweep_count(sg_lattice *lat, int64_t t);

/* Choose the sweep kernel and, for SG_KERNEL_FUSED(2), its tile: tile_x pairs of
 * sites per row (x extent 2*tile_x), tile_y rows, z_chunk planes per workgroup,
 * band = tile rows per group of the tile order (the workgroups running together
 * cover a block about band tiles tall); 0 = default for any of the four.  Invalid
 * shapes return SG_EINVAL and change nothing. */
int sg_set_kernel(sg_lattice *lat, int kind, int tile_x, int tile_y, int z_chunk, int band);

/* Planes the two-sweep march keeps in flight (requested planes-2 steps ahead): 5 or
 * 6, or 0 for the default (5; the buffered generators reject 6).  Reset by
 * sg_set_kernel. */
int sg_set_ring(sg_lattice *lat, int planes);

/* The kernel the next sweeps of this lattice use: out[6] = kind (SG_KERNEL_TWOPASS,
 * _FUSED or _FUSED2), tile_x, tile_y, z_chunk (0 = chosen at launch), band, and the
 * planes in flight of the two-sweep march (0 for the others). */
int sg_get_kernel(const sg_lattice *lat, int out[6]);

/* Autotune the sweep kernel for n (1 or 2) lattices swept together (n = 2:
 * replicas sharing couplings, as in sg_sweep_replicas).  Candidate kernels
 * (SG_KERNEL_TWOPASS; SG_KERNEL_FUSED, and SG_KERNEL_FUSED2 with 5 or, but for
 * the buffered generators, 6 planes in flight, over their tiles) are timed with
 * `reps` launches each on the lattices' own data without changing their state
 * (the launches read the current spins and write only the spare buffer, the
 * in-place two-pass kernel a copy of the spins there; sweep count and streams do
 * not move), and compared by time per sweep.  The fastest
 * is set on every lattice (as sg_set_kernel and sg_set_ring) and remembered for this device, L,
 * n and prng; a later call with the same key reuses it without timing unless
 * reps < 0 forces a new search.  best[5] (may be NULL) receives kind, tile_x,
 * tile_y, z_chunk, band; ms (may be NULL) the best time per sweep, or -1 when the
 * choice came from the cache. */
int sg_autotune(sg_lattice *const *lats, int n, int reps, int best[5], double *ms);

/* ---- Batches: many lattices advanced together --------------------------------
 * A batch holds lattices of any sizes (one replica each, SG_MINSTD, all on the
 * batch's stream, which must not be the legacy default stream when graphs are
 * used), each with its own inverse temperature and sweep count.  A run queues
 * rounds; a round advances every lattice that has sweeps left, all of them in one
 * launch (one work item per fused tile and z chunk of every lattice): by two
 * sweeps for a lattice on SG_KERNEL_AUTO or SG_KERNEL_FUSED2 whose tile allows
 * the two-sweep march (one for its odd last sweep), else by one.  The spins of
 * each lattice after n sweeps are bit-identical to n calls of sg_sweep on it
 * alone.  Lattices join with sg_batch_add and leave when their sweeps are done
 * (sg_batch_take_finished); both take effect at run boundaries.  A lattice must
 * not be swept or destroyed while it is in a batch. */
typedef struct sg_batch sg_batch;

/* Device workspace for a batch of up to max_lattices lattices and max_items work
 * items (tiles x z chunks, summed over the lattices it holds at once). */
int sg_batch_footprint(int max_lattices, int max_items, size_t *dev_bytes);
int sg_batch_create(int max_lattices, int max_items, void *dev_buf, size_t dev_bytes, void *stream,
                    sg_batch **out);

/* Queue nsweeps >= 1 sweeps at beta for lat. */
int sg_batch_add(sg_batch *b, sg_lattice *lat, int64_t nsweeps, double beta);

/* Queue up to max_rounds rounds (fewer if every lattice finishes first).  With
 * rounds_per_graph > 0 the rounds are captured once into a hipGraph of that many
 * rounds (re-captured when the set of work items changes) and replayed.  Returns
 * as soon as the work is queued; lattices whose sweeps are all queued move to the
 * finished list.  *rounds_done (may be NULL) = rounds queued. */
int sg_batch_run(sg_batch *b, int64_t max_rounds, int rounds_per_graph, int64_t *rounds_done);

/* Move up to max finished lattices to out[]; *n = how many. */
int sg_batch_take_finished(sg_batch *b, sg_lattice **out, int max, int *n);

/* Lattices with sweeps left, finished lattices not yet taken, and the work items
 * the active lattices need (any output may be NULL). */
int sg_batch_size(const sg_batch *b, int *active, int *finished, int *items);

/* Rounds until the first and until the last active lattice finishes (0 and 0
 * when none is active); either output may be NULL. */
int sg_batch_rounds_left(const sg_batch *b, int64_t *first, int64_t *last);

int sg_batch_destroy(sg_batch *b);

/* Release the handle (never the caller's device buffer). */
int sg_destroy(sg_lattice *lat);

/* Message of the last failed call on this thread ("" if none). */
const char *sg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
