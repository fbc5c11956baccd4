// Verification kernel: the bit-sliced flip rule of Sec. 4 applied to given
// words, so that a test can drive it through every local configuration of a
// site (its spin, six neighbours and six couplings: 2^13 patterns, 64 per word)
// and every acceptance region of R, in each compiled form the sweep kernels use.
// Not part of a sweep.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kBlock = 256;

// form: bit 0 = Fold (the six-plane march's count), bit 1 = wide comparisons
// (thresholds up to 2^32: MT19937, Parisi-Rapuano, per-sample numbers) instead of
// the 32-bit ones MINSTD's range allows.
template <bool Narrow, bool Fold>
__global__ __launch_bounds__(kBlock) void k_flip_words(const uint64_t *__restrict__ in, const uint32_t *__restrict__ R,
                                                        uint64_t n, Thresholds T, uint64_t *__restrict__ out)
{
    for (uint64_t q = blockIdx.x * (uint64_t)kBlock + threadIdx.x; q < n; q += (uint64_t)gridDim.x * kBlock) {
        const uint64_t *w = in + 13 * q;  // s, n0..n5, j0..j5
        out[q] = flip_site<Narrow, Fold>(w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7], w[8], w[9], w[10], w[11],
                                         w[12], R[q], T);
    }
}

}  // namespace

hipError_t launch_flip_words(int form, const uint64_t *in, const uint32_t *R, uint64_t n, const Thresholds &T,
                             uint64_t *out, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const unsigned grid = (unsigned)std::min<uint64_t>((n + kBlock - 1) / kBlock, 4096);
    switch (form) {
    case 0:
        hipLaunchKernelGGL((k_flip_words<true, false>), dim3(grid), dim3(kBlock), 0, s, in, R, n, T, out);
        break;
    case 1:
        hipLaunchKernelGGL((k_flip_words<true, true>), dim3(grid), dim3(kBlock), 0, s, in, R, n, T, out);
        break;
    case 2:
        hipLaunchKernelGGL((k_flip_words<false, false>), dim3(grid), dim3(kBlock), 0, s, in, R, n, T, out);
        break;
    case 3:
        hipLaunchKernelGGL((k_flip_words<false, true>), dim3(grid), dim3(kBlock), 0, s, in, R, n, T, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sg
