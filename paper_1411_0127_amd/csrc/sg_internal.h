// Internal declarations of libsg: lattice handle, device arithmetic shared by the
// sweep kernels, launch helpers.  Not part of the public ABI (include/sg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "sg.h"

namespace sg {

// ---------------------------------------------------------------------------
// Keyed input generator: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  The n-th
// output of a generator whose state starts at k is mix64(k + n * GAMMA).  Key
// derivation, tags and word indices follow the seeded-input convention stated in
// include/sg.h.
// ---------------------------------------------------------------------------
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kTagJ = 1, kTagSpin = 2, kTagMinstd = 3, kTagMt = 4, kTagPhilox = 5, kTagPr = 6;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t sm_out(uint64_t key, uint64_t n)
{
    return mix64(key + n * kGamma);
}

inline uint64_t derive_key(uint64_t seed, uint32_t tag, uint32_t replica)
{
    return sm_out(sm_out(seed, 1ull + tag), 1ull + replica);
}

// MurmurHash3's 32-bit finalizer (A. Appleby): a bijection of 32-bit words.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// MINSTD seed of site (x, y, z): 1 + ((fmix32((x + L*y) ^ zkey) >> 1) mod (2^31 - 2)),
// zkey = fmix32(z ^ k), k = low 32 bits of key(spin_seed, TAG_MINSTD, replica).
// The per-plane part zkey is the same for a whole plane.
__host__ __device__ __forceinline__ uint32_t minstd_plane_key(uint32_t z, uint32_t k) { return fmix32(z ^ k); }

__host__ __device__ __forceinline__ uint32_t minstd_seed(uint32_t xy, uint32_t zkey)
{
    uint32_t v = fmix32(xy ^ zkey) >> 1;           // < 2^31
    v = (v >= 0x7FFFFFFEu) ? v - 0x7FFFFFFEu : v;  // mod 2^31 - 2
    return v + 1u;
}

// ---------------------------------------------------------------------------
// MINSTD jump: a * s mod (2^31 - 1) for a, s in [1, 2^31 - 2].  The product is
// < 2^62; folding the bits above bit 30 back in uses 2^31 = 1 (mod 2^31 - 1).
// The per-sweep multiplier a = 16807^(t+1) mod (2^31 - 1) comes from the host.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t minstd_jump(uint32_t a, uint32_t s)
{
    const uint64_t p = (uint64_t)a * (uint64_t)s;
    uint32_t r = (uint32_t)(p & 0x7FFFFFFFull) + (uint32_t)(p >> 31);
    return (r >= 0x7FFFFFFFu) ? r - 0x7FFFFFFFu : r;
}

// ---------------------------------------------------------------------------
// Bit-sliced local update (Sec. 4).  For each of the 64 samples coded in a word:
// bond bit b_k = J_k ^ ~s ^ n_k is 1 when bond k is satisfied before the flip
// (the paper's e_ik taken with the flipped spin), the six bits are added by
// full adders into a 3-bit count v = 0..6 per sample, dE = 4v - 12, and the flip
// mask keeps every sample with v <= 3, those with v = 4 if R < T4, v = 5 if
// R < T8 and v = 6 if R < T12.  One R per word (asynchronous multispin coding).
// ---------------------------------------------------------------------------
struct Thresholds {
    uint64_t t4, t8, t12;
};

// Words from one coupling array to the next (J[x], J[y], J[z] of a lattice): L^3
// and a pad.  At power-of-two sides L^3 words are a power of two, and the same
// plane of the three arrays, which a sweep reads together, would otherwise sit at
// the same low address bits and contend for the same memory channels.  The pad,
// 64 KB + 256 bytes, measured best among the pads tried at L = 1024.
constexpr int64_t kJPadWords = 8224;
__host__ __device__ inline int64_t coupling_stride(int L) { return (int64_t)L * L * L + kJPadWords; }

// v_bitop3_b32 (gfx950): any bitwise function of three words in one instruction.
// Its 8-bit table is the function evaluated on the bit patterns 0xF0, 0xCC, 0xAA
// standing for the first, second and third operand.
namespace bop {
constexpr uint32_t A = 0xF0, B = 0xCC, C = 0xAA;
constexpr int table(uint32_t v) { return (int)(v & 0xFFu); }
constexpr int kXor3 = table(A ^ B ^ C);                          // a ^ b ^ c
constexpr int kXnor3 = table(~(A ^ B ^ C));                      // ~(a ^ b ^ c)
constexpr int kMaj = table((A & B) | (A & C) | (B & C));         // majority
constexpr int kBothEq = table(~(A ^ C) & ~(B ^ C));              // bitwise a == c and b == c
constexpr int kOrAnd = table(A | (B & C));                       // a | (b & c)
constexpr int kSel = table((A & B) | (~A & C));                  // a ? b : c
constexpr int kXorOrNot = table(A ^ (~B | C));                   // a ^ (b ? c : 1)
}  // namespace bop

template <int T>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, T);
}

// Bits of the satisfied-bond count v = c2 c1 c0 of 32 samples.  Bond k is
// satisfied when J_k s n_k = +1; with bit 1 for J = -1 and for a spin +1 that is
// w_k = ~(j_k ^ s ^ n_k), one three-input operation per bond.  v = w0 + ... + w5
// = (B1 + B2) + 2 (K1 + K2), B and K the sums and carries of the two triples.
struct VBits {
    uint32_t c0, c1, c2;
};
__device__ __forceinline__ VBits vcount_half(uint32_t s, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3,
                                             uint32_t n4, uint32_t n5, uint32_t j0, uint32_t j1, uint32_t j2,
                                             uint32_t j3, uint32_t j4, uint32_t j5)
{
    const uint32_t w0 = bop3<bop::kXnor3>(j0, n0, s), w1 = bop3<bop::kXnor3>(j1, n1, s),
                   w2 = bop3<bop::kXnor3>(j2, n2, s), w3 = bop3<bop::kXnor3>(j3, n3, s),
                   w4 = bop3<bop::kXnor3>(j4, n4, s), w5 = bop3<bop::kXnor3>(j5, n5, s);
    const uint32_t b1 = bop3<bop::kXor3>(w0, w1, w2), k1 = bop3<bop::kMaj>(w0, w1, w2);
    const uint32_t b2 = bop3<bop::kXor3>(w3, w4, w5), k2 = bop3<bop::kMaj>(w3, w4, w5);
    const uint32_t k3 = b1 & b2;  // carry of B1 + B2
    VBits v;
    v.c0 = b1 ^ b2;
    v.c1 = bop3<bop::kXor3>(k1, k2, k3);
    v.c2 = bop3<bop::kMaj>(k1, k2, k3);
    return v;
}

// The same three bits from x_k = j_k ^ n_k, the spin folded in afterwards: w_k =
// x_k ^ ~s, and since a three-input sum or majority of (x ^ c) is sum(x) ^ c or
// maj(x) ^ c, the complement of s is carried through the adder and cancels in the
// XOR of two such terms.  Two more operations than vcount_half, but the six x_k
// do not wait for s.
__device__ __forceinline__ VBits vcount_half_fold(uint32_t s, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3,
                                                  uint32_t n4, uint32_t n5, uint32_t j0, uint32_t j1, uint32_t j2,
                                                  uint32_t j3, uint32_t j4, uint32_t j5)
{
    const uint32_t x0 = j0 ^ n0, x1 = j1 ^ n1, x2 = j2 ^ n2, x3 = j3 ^ n3, x4 = j4 ^ n4, x5 = j5 ^ n5;
    const uint32_t s1 = bop3<bop::kXor3>(x0, x1, x2);    // B1 = s1 ^ ~s
    const uint32_t k1 = bop3<bop::kMaj>(x0, x1, x2);     // K1 = k1 ^ ~s
    const uint32_t s2 = bop3<bop::kXor3>(x3, x4, x5);
    const uint32_t k2 = bop3<bop::kMaj>(x3, x4, x5);
    VBits v;
    v.c0 = s1 ^ s2;
    const uint32_t k3 = bop3<bop::kBothEq>(s1, s2, s);   // B1 & B2, B = (s1 == s)
    const uint32_t t = k1 ^ k2;
    v.c1 = t ^ k3;
    const uint32_t kk = bop3<bop::kBothEq>(k1, k2, s);   // K1 & K2, K = (k == s)
    v.c2 = bop3<bop::kOrAnd>(kk, k3, t);                 // majority of K1, K2, k3
    return v;
}

// 32 samples of the update with one number for the word; returns the new spin
// word.  a4, a8, a12 are all-ones when R < T4, T8, T12; since T12 <= T8 <= T4
// they are nested, and the accepted set is v <= 3, or v = 4 with a4, v = 5 with
// a8, v = 6 with a12.  Fold selects vcount_half_fold.
template <bool Fold>
__device__ __forceinline__ uint32_t flip_half(uint32_t s, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3,
                                              uint32_t n4, uint32_t n5, uint32_t j0, uint32_t j1, uint32_t j2,
                                              uint32_t j3, uint32_t j4, uint32_t j5, uint32_t a4, uint32_t a8,
                                              uint32_t a12)
{
    const VBits v = Fold ? vcount_half_fold(s, n0, n1, n2, n3, n4, n5, j0, j1, j2, j3, j4, j5)
                         : vcount_half(s, n0, n1, n2, n3, n4, n5, j0, j1, j2, j3, j4, j5);
    const uint32_t mid = bop3<bop::kSel>(v.c0, a8, a4);  // v = 4 or 5: accepted
    const uint32_t hi = bop3<bop::kSel>(v.c1, a12, mid); // v >= 4: accepted (a12 lies in mid)
    return bop3<bop::kXorOrNot>(s, v.c2, hi);            // s ^ (v <= 3 or accepted)
}

#define SG_LO(v) ((uint32_t)(v))          // low and high 32 samples of a word
#define SG_HI(v) ((uint32_t)((v) >> 32))

// New spin word of a 64-sample site: s the spin word, n0..n5 the neighbour words
// and j0..j5 the coupling words of the same six bonds, one R for the word.
// Narrow: every threshold lies below 2^32 (MINSTD's range is 2^31 - 1), so the
// comparisons take 32 bits.  Fold: count with vcount_half_fold.
template <bool Narrow = false, bool Fold = false>
__device__ __forceinline__ uint64_t flip_site(uint64_t s, uint64_t n0, uint64_t n1, uint64_t n2, uint64_t n3,
                                              uint64_t n4, uint64_t n5, uint64_t j0, uint64_t j1, uint64_t j2,
                                              uint64_t j3, uint64_t j4, uint64_t j5, uint32_t R,
                                              const Thresholds &T)
{
    uint32_t a4, a8, a12;
    if (Narrow) {
        a4 = R < (uint32_t)T.t4 ? ~0u : 0u;
        a8 = R < (uint32_t)T.t8 ? ~0u : 0u;
        a12 = R < (uint32_t)T.t12 ? ~0u : 0u;
    } else {
        const uint64_t r = (uint64_t)R;
        a4 = r < T.t4 ? ~0u : 0u;
        a8 = r < T.t8 ? ~0u : 0u;
        a12 = r < T.t12 ? ~0u : 0u;
    }
    const uint32_t lo = flip_half<Fold>(SG_LO(s), SG_LO(n0), SG_LO(n1), SG_LO(n2), SG_LO(n3), SG_LO(n4), SG_LO(n5),
                                  SG_LO(j0), SG_LO(j1), SG_LO(j2), SG_LO(j3), SG_LO(j4), SG_LO(j5), a4, a8, a12);
    const uint32_t hi = flip_half<Fold>(SG_HI(s), SG_HI(n0), SG_HI(n1), SG_HI(n2), SG_HI(n3), SG_HI(n4), SG_HI(n5),
                                  SG_HI(j0), SG_HI(j1), SG_HI(j2), SG_HI(j3), SG_HI(j4), SG_HI(j5), a4, a8, a12);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// ---------------------------------------------------------------------------
// One number per sample (a variant of the acceptance step of Sec. 4: every coded
// sample draws its own 32-bit number R_j, per site and sweep).  The numbers come
// from Philox4x32-10 (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) in bit-sliced form: plane
// b (b = 0..31) is a 64-bit word whose bit j is bit 31-b of R_j; planes 2q and
// 2q+1 are the four outputs (o0 | o1 << 32, o2 | o3 << 32) of Philox at counter
// (lo32(i), hi32(i) << 8 | q, lo32(t), hi32(t)) under the lattice's 64-bit key,
// i the site and t the sweep.  R_j < T is then decided from the most significant
// plane down: a sample is decided at the first plane where its bit differs from
// T's, so the loop stops as soon as every sample of the word is decided -- the
// result is the same as comparing the full 32-bit numbers.
// ---------------------------------------------------------------------------
struct PhiloxOut {
    uint32_t o0, o1, o2, o3;
};
__device__ __forceinline__ PhiloxOut philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                   uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = bop3<bop::kXor3>((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = bop3<bop::kXor3>((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return PhiloxOut{c0, c1, c2, c3};
}

// New spin word of a 64-sample site whose samples draw their own numbers:
// site index i, sweep t, Philox key (k0, k1); T as for MT19937 (range 2^32).
__device__ __forceinline__ uint64_t flip_site_ps(uint64_t s, uint64_t n0, uint64_t n1, uint64_t n2, uint64_t n3,
                                                 uint64_t n4, uint64_t n5, uint64_t j0, uint64_t j1, uint64_t j2,
                                                 uint64_t j3, uint64_t j4, uint64_t j5, uint64_t i, uint64_t t,
                                                 uint32_t k0, uint32_t k1, const Thresholds &T)
{
    const VBits lo = vcount_half(SG_LO(s), SG_LO(n0), SG_LO(n1), SG_LO(n2), SG_LO(n3), SG_LO(n4), SG_LO(n5),
                                 SG_LO(j0), SG_LO(j1), SG_LO(j2), SG_LO(j3), SG_LO(j4), SG_LO(j5));
    const VBits hi = vcount_half(SG_HI(s), SG_HI(n0), SG_HI(n1), SG_HI(n2), SG_HI(n3), SG_HI(n4), SG_HI(n5),
                                 SG_HI(j0), SG_HI(j1), SG_HI(j2), SG_HI(j3), SG_HI(j4), SG_HI(j5));
#undef SG_LO
#undef SG_HI
    const uint64_t c0 = lo.c0 | ((uint64_t)hi.c0 << 32);
    const uint64_t c1 = lo.c1 | ((uint64_t)hi.c1 << 32);
    const uint64_t c2 = lo.c2 | ((uint64_t)hi.c2 << 32);
    // samples with v = 4, 5, 6 (v = 7 cannot occur)
    const uint64_t m4 = c2 & ~(c1 | c0), m5 = c2 & c0, m6 = c2 & c1;
    // thresholds of 2^32 accept at once, of 0 reject at once; the others compare
    const uint64_t all4 = T.t4 > 0xFFFFFFFFull ? ~0ull : 0, all8 = T.t8 > 0xFFFFFFFFull ? ~0ull : 0,
                   all12 = T.t12 > 0xFFFFFFFFull ? ~0ull : 0;
    const uint64_t cmp4 = (T.t4 - 1) < 0xFFFFFFFFull ? ~0ull : 0, cmp8 = (T.t8 - 1) < 0xFFFFFFFFull ? ~0ull : 0,
                   cmp12 = (T.t12 - 1) < 0xFFFFFFFFull ? ~0ull : 0;
    uint64_t acc = (m4 & all4) | (m5 & all8) | (m6 & all12);
    uint64_t und = (m4 & cmp4) | (m5 & cmp8) | (m6 & cmp12);
    const uint32_t T4 = (uint32_t)T.t4, T8 = (uint32_t)T.t8, T12 = (uint32_t)T.t12;
    const uint32_t ilo = (uint32_t)i, ihi = (uint32_t)(i >> 32) << 8, tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
    PhiloxOut o{0, 0, 0, 0};
    for (int b = 0; b < 32 && und != 0; ++b) {
        if ((b & 1) == 0)
            o = philox4x32_10(ilo, ihi | (uint32_t)(b >> 1), tlo, thi, k0, k1);
        const uint64_t w = (b & 1) ? (o.o2 | ((uint64_t)o.o3 << 32)) : (o.o0 | ((uint64_t)o.o1 << 32));
        const int sh = 31 - b;
        const uint64_t tb4 = ((T4 >> sh) & 1u) ? ~0ull : 0, tb8 = ((T8 >> sh) & 1u) ? ~0ull : 0,
                       tb12 = ((T12 >> sh) & 1u) ? ~0ull : 0;
        // each undecided sample's threshold bit: T12 for v = 6, T8 for v = 5, T4 for v = 4
        const uint64_t tb = (c1 & tb12) | (~c1 & ((c0 & tb8) | (~c0 & tb4)));
        acc |= und & ~w & tb;   // its bit is 0 where T's is 1: R_j < T
        und &= ~(w ^ tb);       // still equal to T so far
    }
    return s ^ (~c2 | acc);
}

// ---------------------------------------------------------------------------
// Lattice handle
// ---------------------------------------------------------------------------
constexpr int kMtN = 624;
constexpr int kMaxReduceBlocks = 2048;

}  // namespace sg

struct sg_lattice {
    int L = 0;
    int nsamples = 0;
    int prng = 0;
    int64_t V = 0;
    uint64_t coupling_seed = 0, spin_seed = 0;
    uint32_t replica = 0;
    uint64_t key_spin = 0, key_minstd = 0, key_mt = 0, key_j = 0, key_philox = 0, key_pr = 0;
    uint32_t minstd_k = 0;  // low 32 bits of key_minstd
    uint8_t *base = nullptr;
    size_t bytes = 0;
    uint64_t *spins[2] = {nullptr, nullptr};
    int cur = 0;  // spins[cur] holds the current configuration
    uint64_t *J = nullptr;
    const sg_lattice *J_owner = nullptr;  // nullptr: this lattice owns J
    uint32_t *mt_state = nullptr;         // MT19937 (624 words) or Parisi-Rapuano (64) state, word k of column c at k*L*L + c
    uint32_t *rbuf = nullptr;             // MT19937 / Parisi-Rapuano draws of the sweeps being done [2V]
    int rlast = 0;                        // half of rbuf that holds the last sweep's draws
    uint64_t *scratch = nullptr;          // reduction partials
    hipStream_t stream = nullptr;
    int device = 0;  // HIP device that was current at creation
    int64_t t = 0;  // sweeps done
    int kernel = SG_KERNEL_AUTO;
    int tile_x = 0, tile_y = 0, z_chunk = 0, band = 0;
    int ring = 0;  // planes in flight of the two-sweep march (0 = default)
};

namespace sg {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Memory carve of one lattice buffer.
struct Carve {
    size_t spins0, spins1, J, mt_state, rbuf, scratch, total;
};
Carve carve(int L, int prng, bool own_J);

// Kernels (launchers return hipError_t of the launch).
hipError_t launch_init_couplings(uint64_t *J, int L, uint64_t key, hipStream_t s);
hipError_t launch_init_spins(uint64_t *S, int L, uint64_t key, hipStream_t s);
hipError_t launch_init_mt(uint32_t *state, int L, uint64_t key, hipStream_t s);
// Draws of sweep t for n (1 or 2) stream sets of side L.
// Buffered draws of sweeps t .. t+nsw-1 (nsw = 1 or 2) of n stream sets: sweep
// t+s's draw of site i goes to rbuf[r][s*L^3 + i].
hipError_t launch_mt_fill(uint32_t *const *state, uint32_t *const *rbuf, int n, int L, int64_t t, int nsw,
                          hipStream_t s);
hipError_t launch_init_pr(uint32_t *state, int L, uint64_t key, hipStream_t s);
// MINSTD numbers of sweep t (a = 16807^(t+1) mod (2^31 - 1)) of every site, out[V].
hipError_t launch_minstd_draws(uint32_t *out, int L, uint32_t a, uint32_t mk, hipStream_t s);
hipError_t launch_pr_fill(uint32_t *const *state, uint32_t *const *rbuf, int n, int L, int64_t t, int nsw,
                          hipStream_t s);
// Generators whose numbers are read from a per-sweep buffer filled beforehand.
inline bool buffered_draws(int prng) { return prng == SG_MT19937 || prng == SG_PARISI_RAPUANO; }

struct SweepArgs {
    const uint64_t *J;
    uint64_t *src[2];      // per replica: current spins
    uint64_t *dst[2];      // per replica: next spins (fused) -- unused by two-pass
    const uint32_t *rnd[2];  // per replica: MT19937 draws (unused for MINSTD)
    uint32_t mk[2];          // per replica: MINSTD key (low 32 bits of its keyed word)
    int nrep;
    int L;
    int prng;
    uint32_t minstd_a;     // 16807^(t+1) mod (2^31 - 1)
    uint32_t minstd_a2;    // 16807^(t+2) mod (2^31 - 1): second sweep of a two-sweep launch
    uint64_t pkey[2];      // per replica: key of the per-sample numbers (SG_PHILOX)
    int64_t t;             // sweep index of the (first) sweep of this launch
    Thresholds T;
};
hipError_t launch_sweep_twopass(const SweepArgs &a, hipStream_t s);
// Colour-separated layout: conversion of nwords cube arrays (src_stride words
// apart), and a sweep of one lattice (a.src[0] unused) on separated spins S
// [2][V/2] and couplings K [3][2][V/2].
hipError_t launch_to_separated(const uint64_t *cube, uint64_t *sep, int L, int nwords, int64_t src_stride,
                               hipStream_t s);
hipError_t launch_from_separated(const uint64_t *sep, uint64_t *cube, int L, hipStream_t s);
hipError_t launch_sweep_separated(const SweepArgs &a, uint64_t *S, const uint64_t *K, hipStream_t s);
// Sliced layout (Sec. 2 coordinate transformation): site (x, y, z) at (x', y', z')
// = (x, y - x, x - y + z) mod L, colour c = z' & 1, stored at [c][z'/2][y'][x'];
// spins S [2][V/2] and each site's own couplings K [3][2][V/2].
hipError_t launch_to_sliced(const uint64_t *cube, uint64_t *sl, int L, int nwords, int64_t src_stride,
                            hipStream_t s);
hipError_t launch_from_sliced(const uint64_t *sl, uint64_t *cube, int L, hipStream_t s);
hipError_t launch_sweep_sliced(const SweepArgs &a, uint64_t *S, const uint64_t *K, hipStream_t s);
bool fused_shape_ok(int L, int nrep, int tile_x, int tile_y, int z_chunk);
void fused_default_shape(int L, int nrep, int &tile_x, int &tile_y, int &z_chunk);
hipError_t launch_sweep_fused(const SweepArgs &a, int tile_x, int tile_y, int z_chunk, int band, hipStream_t s);
// Two sweeps (t and t+1) per launch, every generator (buffered draws: a.rnd holds
// both sweeps' numbers); replicas share one launch.
bool fused2_shape_ok(int L, int tile_x, int tile_y, int z_chunk);
void fused2_default_shape(int L, int &tile_x, int &tile_y, int &z_chunk);
// ring: planes in flight, 5 or 6 (0 = the default, fused2_default_ring).
hipError_t launch_sweep_fused2(const SweepArgs &a, int tile_x, int tile_y, int z_chunk, int band, int ring,
                               hipStream_t s);
int fused2_default_ring(int L);

// One lattice of a batched launch (device copy; see k_fused_batch).
struct BatchEntry {
    const uint64_t *J;
    uint64_t *spins[2];
    uint32_t mk;     // MINSTD key
    int L, TXp, TY, ZC, ntx, nty, nzc, WE, band;
    int two;         // 1: rounds of two sweeps (two-sweep march), 0: one sweep per round
    int WE2, WO0, WO1;  // wave layout of the two-sweep march
    int c0;          // current spin buffer when the run starts
    int item0;       // first work item
    int nitems;      // work items: tiles x z chunks
    int64_t t0;      // sweeps done when the run starts
    int64_t nsweeps; // sweeps to do in this run
    uint64_t t4, t8, t12;
};
// two: ask for two-sweep rounds; it is cleared when the tile does not fit them.
bool fill_batch_entry(BatchEntry &e, int L, int tile_x, int tile_y, int z_chunk, int band, bool two);
size_t fused_batch_lds_bytes(const BatchEntry &e);
hipError_t launch_fused_batch(const BatchEntry *E, const uint32_t *item_lat, int nitems, const int64_t *round_ctr,
                              size_t lds, hipStream_t s);
// Work items of a batch round are dealt to the XCDs in groups of kBatchGroup
// consecutive items, group g to XCD g mod kBatchQueues (neighbouring tiles run
// together on one XCD and share its L2).
constexpr int kBatchGroup = 32;
constexpr int kBatchQueues = 8;
// All rounds of a run in one launch (see k_batch_persistent), one queue per XCD:
// cum[q * (nrounds + 1) + r] = entries of queue q before round r; a round's
// active items are the first ones of item_lat (lattices sorted by rounds left).
hipError_t launch_batch_persistent(const BatchEntry *E, const uint32_t *item_lat, const uint64_t *cum, int nrounds,
                                   unsigned long long *queues, uint32_t *done, uint32_t *error, int nlat,
                                   uint32_t spin_cap, size_t lds, int64_t total_items, hipStream_t s);
// Clears the queue counters, the error flag and nlat per-lattice counters.
hipError_t launch_batch_reset(unsigned long long *queues, uint32_t *error, uint32_t *done, int nlat, hipStream_t s);
hipError_t launch_round_advance(int64_t *round_ctr, hipStream_t s);
hipError_t launch_round_reset(int64_t *round_ctr, hipStream_t s);

// Lattices of at most kSmallSites sites (L <= 16): nsweeps sweeps in one launch
// of one workgroup, spins and couplings resident in LDS (spins in place in S), and
// when out is not NULL the unsatisfied-bond counts of samples 0 .. nsamples-1
// after every sweep in out[nsweeps][64].  MINSTD (a0 = 16807^(t0+1) mod (2^31 - 1)) and per-sample
// Philox numbers.
constexpr int kSmallSites = 4096;
hipError_t launch_small_sweeps(uint64_t *S, const uint64_t *J, int L, int nsamples, int prng, uint32_t mk,
                               uint64_t pkey, int64_t t0, uint32_t a0, int nsweeps, const Thresholds &T, uint64_t *out,
                               hipStream_t s);

// The flip rule applied to n sets of 13 words (s, n0..n5, j0..j5) with one R each:
// out[q] = flip_site<Narrow = !(form & 2), Fold = form & 1>.  Verification only.
hipError_t launch_flip_words(int form, const uint64_t *in, const uint32_t *R, uint64_t n, const Thresholds &T,
                             uint64_t *out, hipStream_t s);

// Bandwidth probes (kind 0 read-only into dst[blocks*4] words, 1 copy, 2 fill;
// 3..5 the same with non-temporal loads and stores).
hipError_t launch_probe(int kind, void *dst, const void *src, size_t bytes, int blocks, hipStream_t s);

hipError_t launch_count_unsat(const uint64_t *S, const uint64_t *J, int L, uint64_t *partials, int &nblocks,
                              hipStream_t s);
hipError_t launch_count_diff(const uint64_t *A, const uint64_t *B, int64_t V, uint64_t *partials, int &nblocks,
                             hipStream_t s);
hipError_t launch_reduce_partials(const uint64_t *partials, int nblocks, uint64_t *out64, hipStream_t s);

}  // namespace sg
