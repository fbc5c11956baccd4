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

/* Bytes of device memory a lattice of side L needs (Sec. 1: a cubic lattice of
 * V = L^3 spins with 3V bonds; Sec. 4: one bit per spin and coupling per coded
 * sample, so the size does not depend on nsamples, which is only checked):
 * sg_footprint for a lattice that holds its couplings (sg_lattice_create),
 * sg_replica_footprint for a replica that reads another lattice's
 * (sg_lattice_create_replica).  SG_EINVAL for L odd or outside [2, 2048],
 * nsamples outside [1, 64], an unknown prng or dev_bytes NULL. */
int sg_footprint(int L, int nsamples, int prng, size_t *dev_bytes);
int sg_replica_footprint(int L, int nsamples, int prng, size_t *dev_bytes);

/* Create a lattice of side L (even, 2..2048) holding nsamples (1..64) samples
 * (Sec. 1, Eqs. (1)-(2): the +-J model on a periodic cube, random start; Sec. 4:
 * the samples coded one per bit of a word).
 * J_host: 3*L^3 coupling words in the layout above, or NULL to generate them
 *         from coupling_seed (Sec. 1: J = +-1 with probability 1/2 each);
 * spin_seed, replica: key the initial spins and the random streams;
 * dev_buf, dev_bytes: caller's device buffer, >= sg_footprint(L, nsamples, prng)
 *         bytes, 256-byte aligned (the size is checked: SG_EINVAL when short);
 * stream: hipStream_t for all work on this lattice, or NULL.
 * Bits j >= nsamples are simulated like the others and ignored by observables. */
int sg_lattice_create(int L, int nsamples, int prng, const uint64_t *J_host,
                      uint64_t coupling_seed, uint64_t spin_seed, uint32_t replica,
                      void *dev_buf, size_t dev_bytes, void *stream, sg_lattice **out);

/* A replica (Sec. 2: same couplings, its own initial spins and evolution):
 * shares base's coupling buffer, draws its spins and streams from
 * (spin_seed, replica).  dev_buf >= sg_replica_footprint(L, nsamples, prng);
 * base must outlive the replica. */
int sg_lattice_create_replica(const sg_lattice *base, uint64_t spin_seed, uint32_t replica,
                              void *dev_buf, size_t dev_bytes, void *stream,
                              sg_lattice **out);

/* Queue nsweeps >= 0 Metropolis sweeps at inverse temperature beta >= 0 (Sec. 1:
 * one sweep updates every red site, then every blue site; Sec. 4: acceptance by
 * integer thresholds on the coded words).  beta = +inf is allowed: only dE <= 0
 * is accepted.  Asynchronous on the lattice's stream; SG_EINVAL for nsweeps < 0
 * or beta < 0 / NaN, SG_EDEVICE when a launch fails. */
int sg_sweep(sg_lattice *lat, int64_t nsweeps, double beta);

/* The same for n lattices that share one coupling buffer (replicas, Sec. 2: the
 * paper sweeps its replicas in one kernel), moving the couplings once per sweep
 * for pairs of them when the kernel allows; all must have the same L, prng,
 * couplings, stream and sweep count (else SG_EMISMATCH). */
int sg_sweep_replicas(sg_lattice *const *lats, int n, int64_t nsweeps, double beta);

/* ---- Layout study (Sec. 2, memory allocation strategies) ------------------------
 * Bytes of the work buffer sg_sweep_separated and sg_sweep_sliced need: 32 per
 * site (the spin word and three coupling words). */
int sg_sliced_footprint(int L, size_t *dev_bytes);

/* nsweeps sweeps with the two-pass kernel on the colour-separated ("standard")
 * layout of Sec. 2: the current spins and the couplings are copied into `work`
 * (caller's device buffer, >= sg_sliced_footprint bytes, 256-byte aligned) with
 * red and blue sites of each row in separate arrays indexed by (z, y, x/2) and
 * each site's three couplings with its colour, swept there, and the spins copied
 * back.  The spins are bit-identical to sg_sweep's; `work` is scratch, free again
 * when the queued work is done.  MINSTD, MT19937, Parisi-Rapuano and per-sample
 * lattices. */
int sg_sweep_separated(sg_lattice *lat, int64_t nsweeps, double beta, void *work, size_t work_bytes);

/* The same on the paper's sliced layout (Sec. 2, cubic stencil: the coordinate
 * transformation x' = x, y' = y - x, z' = x - y + z mod L makes every z' plane one
 * colour, red for z' even).  In `work` colour c = z' & 1 is stored at
 * [c][z'/2][y'][x'], spins first, then each site's own three couplings J[d][c][...];
 * a site's neighbours are the words (x', y'), (x', y'-1), (x'+1, y'-1) of the
 * plane above and (x', y'), (x', y'+1), (x'-1, y'+1) of the plane below (the
 * transformed neighbour coordinates of Sec. 2).  One two-pass sweep per sweep;
 * bit-identical to sg_sweep.  Arguments, checks and ownership as above. */
int sg_sweep_sliced(sg_lattice *lat, int64_t nsweeps, double beta, void *work, size_t work_bytes);

/* sg_sweep_sliced without a work buffer, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, hosts that forbid
 * allocation): the sliced copy lives in a static device array of the library of
 * 8 MiB, so L <= 64 (32 bytes per site); a larger lattice returns SG_EINVAL with
 * the limit in sg_last_error.  Allocates nothing, on the host or the device.
 * Every call on one GPU shares that GPU's array (each call overwrites the part it
 * uses before reading it): calls that overlap on one GPU, e.g. on two streams,
 * race and give undefined spins; serialise them.  Results are bit-identical to
 * sg_sweep_sliced and sg_sweep. */
int sg_sweep_sliced_static(sg_lattice *lat, int64_t nsweeps, double beta);

/* Energy of Sec. 1, Eq. (1), per sample j < nsamples: unsat[j] = number of
 * unsatisfied bonds (-J s_i s_k = +1) among the 3V bonds, e_per_spin[j] =
 * (2*unsat[j] - 3V) / V, i.e. H/V.  Either output may be NULL.  Synchronises the
 * lattice's stream. */
int sg_energy(sg_lattice *lat, int64_t *unsat, double *e_per_spin);

/* nsweeps sweeps at beta with the energy of Sec. 1, Eq. (1) after every one:
 * unsat[k * nsamples + j] = unsatisfied bonds of sample j after sweep k+1 of this
 * call (host array of nsweeps * nsamples).  Same spins as sg_sweep.  Up to L = 16
 * with MINSTD or per-sample numbers, one workgroup runs up to 2049 sweeps per
 * launch with the lattice in LDS; otherwise each sweep is a launch of its own.
 * The counts stay on the device and are copied back in chunks (of up to ~2000
 * sweeps at small L, one at L >= 1024), so the stream is not synchronised after
 * every sweep.  Synchronises the lattice's stream before returning. */
int sg_sweep_energies(sg_lattice *lat, int64_t nsweeps, double beta, int64_t *unsat);

/* Two-replica overlap per sample.  The paper simulates replicas (Sec. 2) but
 * does not define the overlap; this is the textbook q_j = (1/V) sum_i
 * s^a_i s^b_i, returned as ndiff[j] = number of sites where the replicas differ
 * and q[j] = 1 - 2*ndiff[j]/V.  a, b: same L, nsamples and couplings (else
 * SG_EMISMATCH).  Synchronises a's stream (and b's, if different). */
int sg_overlap(const sg_lattice *a, const sg_lattice *b, int64_t *ndiff, double *q);

/* Spins as +-1 bytes, sample-major: out[j*V + i], j < nsamples, i = x + L*(y +
 * L*z); n = nsamples*V (else SG_EINVAL).  Decodes the bit mapping of Sec. 4
 * (bit j of site i's word is 1 for s = +1).  Synchronises the stream. */
int sg_get_spins(const sg_lattice *lat, int8_t *out, size_t n);

/* Raw spin words, n = V (Sec. 4 bit mapping): sg_get_words reads the current
 * configuration, sg_set_spins replaces it (resume from a checkpoint, gauge
 * tests); host arrays are borrowed, both synchronise the stream. */
int sg_get_words(const sg_lattice *lat, uint64_t *out, size_t n);
int sg_set_spins(sg_lattice *lat, const uint64_t *words_host, size_t n);

/* Coupling words, n = 3V, packed J[3][V] (Sec. 1, Eq. (2); bit 1 = J = -1). */
int sg_get_couplings(const sg_lattice *lat, uint64_t *out, size_t n);

/* The random number each site used in the last sweep (n = V; Sec. 3 generators,
 * Sec. 4 one number per site word), read from the device: the buffered numbers
 * of MT19937 / Parisi-Rapuano, or MINSTD's evaluated by a kernel with the sweep
 * kernels' functions.  SG_EINVAL before the first sweep and for SG_PHILOX
 * lattices, whose samples draw 64 numbers per site. */
int sg_get_randoms(const sg_lattice *lat, uint32_t *out, size_t n);

/* Integer thresholds T[k-1] = ceil(R_range * exp(-4k beta)) for dE = 4k, k = 1,2,3
 * (Sec. 4, EXP4/EXP8/EXP12; R_range as above).  Host only; the CPU checker uses
 * the same definition. */
int sg_thresholds(double beta, int prng, uint64_t T[3]);

/* Sweeps done so far (the sweep index t of the Sec. 3 streams; Sec. 4.1 times
 * t_sw per sweep), -1 for NULL.  Setting it (resume from a checkpoint) also moves
 * the MINSTD and per-sample streams, which are functions of (site, sweep); a
 * MT19937 or Parisi-Rapuano lattice that has not swept may be moved forward by
 * regenerating its streams up to that point -- for one that has, restore its
 * stream state with sg_set_stream_state. */
int64_t sg_sweep_count(const sg_lattice *lat);
int sg_set_sweep_count(sg_lattice *lat, int64_t t);

/* Checkpoint of the per-column stream states of Sec. 3 (MT19937: 624 words per
 * column, Parisi-Rapuano: 64; word k of column c at k*L*L + c, the paper's
 * strided per-stream layout).  sg_stream_state_bytes gives their size (0 for
 * MINSTD and SG_PHILOX, which keep none); sg_get_stream_state copies them out,
 * sg_set_stream_state copies them in and sets the sweep count to t, the count
 * at which they were taken.  Together with sg_get_words / sg_set_spins this
 * resumes any lattice mid-run bit-exactly.  bytes must equal the size. */
int sg_stream_state_bytes(const sg_lattice *lat, size_t *bytes);
int sg_get_stream_state(const sg_lattice *lat, void *out, size_t bytes);
int sg_set_stream_state(sg_lattice *lat, const void *in, size_t bytes, int64_t t);

/* Library runtime (verification of Sec. 4): the bit-sliced flip rule applied to
 * n given local configurations, so that a test can drive every pattern of a
 * site's spin, six neighbours and six couplings (64 samples per word) through
 * each acceptance region of R.  in: n * 13 device words per configuration (s,
 * n0..n5, j0..j5; bond k joins n_k with coupling j_k, bit 1 <=> J = -1 and
 * sigma = +1); R: n device numbers; out: n device words, the new spin words.
 * Thresholds from sg_thresholds(beta, prng).  form: bit 0 the count of the
 * six-plane march (else the five-plane one), bit 1 the 64-bit comparisons of the
 * buffered and per-sample generators (else MINSTD's 32-bit ones, which only
 * MINSTD's thresholds allow: SG_EINVAL otherwise).  Asynchronous on `stream`. */
int sg_flip_words(int form, const uint64_t *in, const uint32_t *R, uint64_t n, double beta, int prng, uint64_t *out,
                  void *stream);

/* Library runtime (measurement): bandwidth probes, the measured peaks the sweep
 * is set against (the paper's analog: the peak bandwidth of a device copy, Sec.
 * 4.1).  kind 0: read `bytes` from src, writing blocks*16 bytes of folded words to
 * dst (dst must hold them); 1: copy `bytes` from src to dst; 2: fill `bytes` of
 * dst; 3, 4, 5: the same with non-temporal (streaming) loads and stores.  bytes a
 * positive multiple of 16, buffers 16-byte aligned, blocks = 0 for 4096
 * workgroups of 256 lanes (else 1..65536).  Asynchronous on `stream`; the caller
 * times it. */
int sg_probe_bandwidth(int kind, void *dst, const void *src, size_t bytes, int blocks, void *stream);

/* Library runtime (kernel choice; no counterpart in the paper, whose launch
 * configurations are studied in Sec. 4.1).
 * Choose the sweep kernel and, for SG_KERNEL_FUSED(2), its tile: tile_x pairs of
 * sites per row (x extent 2*tile_x), tile_y rows, z_chunk planes per workgroup,
 * band = tile rows per group of the tile order (the workgroups running together
 * cover a block about band tiles tall); 0 = default for any of the four.  Invalid
 * shapes return SG_EINVAL and change nothing. */
int sg_set_kernel(sg_lattice *lat, int kind, int tile_x, int tile_y, int z_chunk, int band);

/* Library runtime.  Planes the two-sweep march keeps in flight (requested planes-2 steps ahead): 5 or
 * 6, or 0 for the default (5; the buffered generators reject 6).  Reset by
 * sg_set_kernel. */
int sg_set_ring(sg_lattice *lat, int planes);

/* Library runtime.  The kernel the next sweeps of this lattice use: out[6] = kind (SG_KERNEL_TWOPASS,
 * _FUSED or _FUSED2), tile_x, tile_y, z_chunk (0 = chosen at launch), band, and the
 * planes in flight of the two-sweep march (0 for the others). */
int sg_get_kernel(const sg_lattice *lat, int out[6]);

/* Library runtime (the paper scans launch configurations by hand, Sec. 4.1).
 * Autotune the sweep kernel for n (1 or 2) lattices swept together (n = 2:
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
 * rounds; a round advances every lattice that has sweeps left (one work item per
 * fused tile and z chunk of every lattice): by two sweeps for a lattice on
 * SG_KERNEL_AUTO or SG_KERNEL_FUSED2 whose tile allows the two-sweep march (one
 * for its odd last sweep), else by one.  By default a run is one persistent launch
 * that takes (round, item) entries from a queue and starts a lattice's round as
 * soon as that lattice's previous round is done (sg_batch_set_persistent); the
 * other form launches once per round.  The spins of each lattice after n sweeps
 * are bit-identical to n calls of sg_sweep on it alone.  Lattices join with
 * sg_batch_add and leave when their sweeps are done (sg_batch_take_finished);
 * both take effect at run boundaries.  A lattice must not be swept or destroyed
 * while it is in a batch. */
typedef struct sg_batch sg_batch;

/* Library runtime (the paper's nearest analog: k coded sample sets per launch,
 * Sec. 2 and Sec. 4.1).  Device workspace for a batch of up to max_lattices
 * lattices and max_items work items (tiles x z chunks, summed over the lattices it
 * holds at once). */
int sg_batch_footprint(int max_lattices, int max_items, size_t *dev_bytes);
int sg_batch_create(int max_lattices, int max_items, void *dev_buf, size_t dev_bytes, void *stream,
                    sg_batch **out);

/* Library runtime.  Queue nsweeps >= 1 sweeps (Sec. 1) at beta for lat. */
int sg_batch_add(sg_batch *b, sg_lattice *lat, int64_t nsweeps, double beta);

/* Library runtime.  Queue up to max_rounds rounds (fewer if every lattice
 * finishes first).  With
 * rounds_per_graph > 0 the rounds are captured once into a hipGraph of that many
 * rounds (re-captured when the set of work items changes) and replayed.  Returns
 * as soon as the work is queued; lattices whose sweeps are all queued move to the
 * finished list.  *rounds_done (may be NULL) = rounds queued. */
int sg_batch_run(sg_batch *b, int64_t max_rounds, int rounds_per_graph, int64_t *rounds_done);

/* Library runtime.  on = 1: each run is one persistent launch (the default);
 * on = 0: one launch per round.  spin_cap bounds the polls (about 1 us each) a
 * workgroup of a persistent run makes while it waits for a lattice's previous
 * round; past it the run gives up, every workgroup leaves, and sg_batch_check
 * reports SG_EDEVICE (0 = the default, 2^22).  Takes effect at the next run. */
int sg_batch_set_persistent(sg_batch *b, int on, uint32_t spin_cap);

/* Library runtime.  Persistent runs launch the active lattices in groups taken in
 * order (one launch per group, one after another on the batch's stream), each
 * group holding lattices whose spins and couplings (40 B per site) add up to at
 * most `bytes` (a lattice larger than that alone); bytes = 0 puts every lattice in
 * one launch, and so does a run of fewer than 4 rounds.  Results do not depend on
 * it.  Default 12 GiB; takes effect at the next run. */
int sg_batch_set_group_bytes(sg_batch *b, size_t bytes);

/* Library runtime.  Synchronise the batch's stream and report whether every
 * persistent run queued so far completed (SG_OK) or gave up waiting
 * (SG_EDEVICE: the lattices of that run hold no valid state). */
int sg_batch_check(sg_batch *b);

/* Library runtime.  Move up to max finished lattices to out[]; *n = how many. */
int sg_batch_take_finished(sg_batch *b, sg_lattice **out, int max, int *n);

/* Library runtime.  Lattices with sweeps left, finished lattices not yet taken,
 * and the work items the active lattices need (any output may be NULL). */
int sg_batch_size(const sg_batch *b, int *active, int *finished, int *items);

/* Library runtime.  Rounds until the first and until the last active lattice
 * finishes (0 and 0 when none is active); either output may be NULL. */
int sg_batch_rounds_left(const sg_batch *b, int64_t *first, int64_t *last);

/* Library runtime.  Release the batch handle (never the caller's workspace). */
int sg_batch_destroy(sg_batch *b);

/* Library runtime (no counterpart in the paper).  Release the handle, never the
 * caller's device buffer; NULL is allowed. */
int sg_destroy(sg_lattice *lat);

/* Library runtime.  Message of the last failed call on this thread ("" if none). */
const char *sg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
