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
constexpr uint32_t kTagJ = 1, kTagSpin = 2, kTagMinstd = 3, kTagMt = 4;

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

// MINSTD seed of a site from its keyed word: 1 + ((h >> 33) mod (2^31 - 2)).
__host__ __device__ __forceinline__ uint32_t minstd_seed_from(uint64_t h)
{
    uint32_t v = (uint32_t)(h >> 33);              // < 2^31
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

__device__ __forceinline__ void full_add(uint64_t a, uint64_t b, uint64_t c, uint64_t &sum, uint64_t &carry)
{
    const uint64_t t = a ^ b;
    sum = t ^ c;
    carry = (t & c) | (~t & a);
}

__device__ __forceinline__ uint64_t flip_mask(uint64_t s, uint64_t n0, uint64_t n1, uint64_t n2, uint64_t n3,
                                              uint64_t n4, uint64_t n5, uint64_t j0, uint64_t j1, uint64_t j2,
                                              uint64_t j3, uint64_t j4, uint64_t j5, uint32_t R,
                                              const Thresholds &T)
{
    const uint64_t ns = ~s;
    uint64_t a0, a1, b0, b1, c1, c2;
    full_add(j0 ^ ns ^ n0, j1 ^ ns ^ n1, j2 ^ ns ^ n2, a0, a1);
    full_add(j3 ^ ns ^ n3, j4 ^ ns ^ n4, j5 ^ ns ^ n5, b0, b1);
    const uint64_t c0 = a0 ^ b0;
    full_add(a1, b1, a0 & b0, c1, c2);
    const uint64_t r = (uint64_t)R;
    const uint64_t all8 = (r < T.t8) ? ~0ull : 0ull;
    const uint64_t all4 = (r < T.t4) ? ~0ull : 0ull;
    const uint64_t all12 = (r < T.t12) ? ~0ull : 0ull;
    // v in {4, 5}: c2 & ~c1; v = 4 needs R < T4, v = 5 needs R < T8
    const uint64_t mid = all8 | (all4 & ~c0);
    return all12 | ~c2 | (~c1 & mid);
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
    uint64_t key_spin = 0, key_minstd = 0, key_mt = 0, key_j = 0;
    uint8_t *base = nullptr;
    size_t bytes = 0;
    uint64_t *spins[2] = {nullptr, nullptr};
    int cur = 0;  // spins[cur] holds the current configuration
    uint64_t *J = nullptr;
    const sg_lattice *J_owner = nullptr;  // nullptr: this lattice owns J
    uint32_t *seeds = nullptr;            // MINSTD per-site seeds [V]
    uint32_t *mt_state = nullptr;         // MT19937 state, word k of column c at k*L*L + c
    uint32_t *rbuf = nullptr;             // MT19937 draws of the sweep being done [V]
    uint64_t *scratch = nullptr;          // reduction partials
    hipStream_t stream = nullptr;
    int64_t t = 0;  // sweeps done
    int kernel = SG_KERNEL_AUTO;
    int tile_x = 0, tile_y = 0, z_chunk = 0;
};

namespace sg {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Memory carve of one lattice buffer.
struct Carve {
    size_t spins0, spins1, J, seeds, mt_state, rbuf, scratch, total;
};
Carve carve(int L, int prng, bool own_J);

// Kernels (launchers return hipError_t of the launch).
hipError_t launch_init_couplings(uint64_t *J, int L, uint64_t key, hipStream_t s);
hipError_t launch_init_spins(uint64_t *S, int L, uint64_t key, hipStream_t s);
hipError_t launch_init_minstd(uint32_t *seeds, int L, uint64_t key, hipStream_t s);
hipError_t launch_init_mt(uint32_t *state, int L, uint64_t key, hipStream_t s);
hipError_t launch_mt_fill(uint32_t *state, uint32_t *rbuf, int L, int64_t t, hipStream_t s);
hipError_t launch_minstd_draws(const uint32_t *seeds, uint32_t *R, int L, uint32_t a, hipStream_t s);

struct SweepArgs {
    const uint64_t *J;
    uint64_t *src[2];      // per replica: current spins
    uint64_t *dst[2];      // per replica: next spins (fused) -- unused by two-pass
    const uint32_t *rnd[2];  // per replica: MINSTD seeds or MT19937 draws
    int nrep;
    int L;
    int prng;
    uint32_t minstd_a;     // 16807^(t+1) mod (2^31 - 1)
    Thresholds T;
};
hipError_t launch_sweep_twopass(const SweepArgs &a, hipStream_t s);
bool fused_shape_ok(int L, int nrep, int tile_x, int tile_y, int z_chunk);
void fused_default_shape(int L, int nrep, int &tile_x, int &tile_y, int &z_chunk);
hipError_t launch_sweep_fused(const SweepArgs &a, int tile_x, int tile_y, int z_chunk, hipStream_t s);

hipError_t launch_count_unsat(const uint64_t *S, const uint64_t *J, int L, uint64_t *partials, int &nblocks,
                              hipStream_t s);
hipError_t launch_count_diff(const uint64_t *A, const uint64_t *B, int64_t V, uint64_t *partials, int &nblocks,
                             hipStream_t s);
hipError_t launch_reduce_partials(const uint64_t *partials, int nblocks, uint64_t *out64, hipStream_t s);

}  // namespace sg
