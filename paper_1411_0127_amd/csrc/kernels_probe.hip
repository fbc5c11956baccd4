// Bandwidth probes: a read-only stream, a device copy and a write-only fill
// over large device buffers.  They give the measured peaks that the sweep's
// bandwidth is set against, as the paper sets its kernels against the peak
// bandwidth a device copy reaches (Sec. 4.1, bandwidth figure).  Not part of
// the sweep.
//
// 16-byte accesses, four independent ones per lane and iteration, a grid of
// many workgroups per CU striding over the buffer.  The read probe folds what
// it reads with XOR and writes one word per wave, so its loads cannot be
// dropped; those writes are 1/1024 of the bytes read at most.  Each probe has a
// streaming form (NT: non-temporal loads and stores, which do not keep the lines
// in the caches); the caller takes the faster of the two.
#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 4;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ uint4 ld16(const uint4 *p)
{
    if (NT) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    return *p;
}

template <bool NT>
__device__ __forceinline__ void st16(uint4 *p, const uint4 v)
{
    if (NT) {
        u32x4 w;
        w.x = v.x;
        w.y = v.y;
        w.z = v.z;
        w.w = v.w;
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(p));
    } else {
        *p = v;
    }
}

template <bool NT>
__global__ __launch_bounds__(kBlock) void k_probe_read(const uint4 *__restrict__ src, size_t n,
                                                       uint32_t *__restrict__ sink)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            v[u] = ld16<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) {
        const uint4 v = ld16<NT>(src + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    for (int off = 32; off > 0; off >>= 1)
        acc ^= __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0)
        sink[((size_t)blockIdx.x * kBlock + threadIdx.x) >> 6] = acc;
}

template <bool NT>
__global__ __launch_bounds__(kBlock) void k_probe_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                       size_t n)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            v[u] = ld16<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            st16<NT>(dst + i + u * stride, v[u]);
    }
    for (; i < n; i += stride)
        st16<NT>(dst + i, ld16<NT>(src + i));
}

template <bool NT>
__global__ __launch_bounds__(kBlock) void k_probe_fill(uint4 *__restrict__ dst, size_t n, uint32_t pattern)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    const uint4 v = make_uint4(pattern, pattern ^ 1u, pattern ^ 2u, pattern ^ 3u);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        st16<NT>(dst + i, v);
}

}  // namespace

hipError_t launch_probe(int kind, void *dst, const void *src, size_t bytes, int blocks, hipStream_t s)
{
    const size_t n = bytes / 16;
    const uint4 *in = static_cast<const uint4 *>(src);
    uint4 *out = static_cast<uint4 *>(dst);
    switch (kind) {
    case 0:
        hipLaunchKernelGGL(k_probe_read<false>, dim3(blocks), dim3(kBlock), 0, s, in, n, static_cast<uint32_t *>(dst));
        break;
    case 1:
        hipLaunchKernelGGL(k_probe_copy<false>, dim3(blocks), dim3(kBlock), 0, s, in, out, n);
        break;
    case 2:
        hipLaunchKernelGGL(k_probe_fill<false>, dim3(blocks), dim3(kBlock), 0, s, out, n, 0x5A5A5A5Au);
        break;
    case 3:
        hipLaunchKernelGGL(k_probe_read<true>, dim3(blocks), dim3(kBlock), 0, s, in, n, static_cast<uint32_t *>(dst));
        break;
    case 4:
        hipLaunchKernelGGL(k_probe_copy<true>, dim3(blocks), dim3(kBlock), 0, s, in, out, n);
        break;
    default:
        hipLaunchKernelGGL(k_probe_fill<true>, dim3(blocks), dim3(kBlock), 0, s, out, n, 0x5A5A5A5Au);
        break;
    }
    return hipGetLastError();
}

}  // namespace sg
