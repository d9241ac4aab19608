// ceiling.hip -- streaming kernels that measure the HBM rate this device
// reaches with plain, fully coalesced traffic: the practical ceiling against
// which the advection kernels' roofline fractions are read.
//
// Every lane moves 16 bytes per access (one dwordx4), four accesses in flight
// per lane per loop trip, over a grid-stride loop; stores are non-temporal
// (streamed past the caches).  Three forms: read only (the words are folded
// into one value per wave, so nothing is dropped), write only (a constant),
// and a 1:1 copy.
#include "monc_internal.hpp"

namespace monc {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int CEIL_UNROLL = 4;

__global__ void __launch_bounds__(256) ceil_read(const u32x4* __restrict__ src, long n16,
                                                 u32x4* __restrict__ sink) {
    const long stride = (long)gridDim.x * blockDim.x;
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (; t + (CEIL_UNROLL - 1) * stride < n16; t += CEIL_UNROLL * stride) {
        u32x4 x[CEIL_UNROLL];
#pragma unroll
        for (int r = 0; r < CEIL_UNROLL; r++) x[r] = __builtin_nontemporal_load(src + t + r * stride);
#pragma unroll
        for (int r = 0; r < CEIL_UNROLL; r++) acc ^= x[r];
    }
    for (; t < n16; t += stride) acc ^= __builtin_nontemporal_load(src + t);
    unsigned int v = acc.x ^ acc.y ^ acc.z ^ acc.w;
    for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) {
        const u32x4 r = {v, 0u, 0u, 0u};
        sink[((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6] = r;
    }
}

__global__ void __launch_bounds__(256) ceil_write(u32x4* __restrict__ dst, long n16) {
    const long stride = (long)gridDim.x * blockDim.x;
    const u32x4 c = {0x3ff00000u, 0u, 0x3ff00000u, 0u};
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n16; t += stride)
        __builtin_nontemporal_store(c, dst + t);
}

__global__ void __launch_bounds__(256) ceil_copy(const u32x4* __restrict__ src,
                                                 u32x4* __restrict__ dst, long n16) {
    const long stride = (long)gridDim.x * blockDim.x;
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; t + (CEIL_UNROLL - 1) * stride < n16; t += CEIL_UNROLL * stride) {
        u32x4 x[CEIL_UNROLL];
#pragma unroll
        for (int r = 0; r < CEIL_UNROLL; r++) x[r] = __builtin_nontemporal_load(src + t + r * stride);
#pragma unroll
        for (int r = 0; r < CEIL_UNROLL; r++) __builtin_nontemporal_store(x[r], dst + t + r * stride);
    }
    for (; t < n16; t += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + t), dst + t);
}

}  // namespace

size_t ceiling_sink_bytes(int blocks) { return (size_t)blocks * 4 * 16; }

hipError_t launch_ceiling(int mode, const void* src, void* dst, size_t nbytes, int blocks,
                          hipStream_t s) {
    const long n16 = (long)(nbytes / 16);
    if (mode == MONC_CEIL_READ)
        ceil_read<<<blocks, 256, 0, s>>>((const u32x4*)src, n16, (u32x4*)dst);
    else if (mode == MONC_CEIL_WRITE)
        ceil_write<<<blocks, 256, 0, s>>>((u32x4*)dst, n16);
    else
        ceil_copy<<<blocks, 256, 0, s>>>((const u32x4*)src, (u32x4*)dst, n16);
    return hipGetLastError();
}

}  // namespace monc
