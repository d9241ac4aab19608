// support.hip -- halo fill, marshalling casts and the final budget reduction.
#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

// ---------------------------------------------------------------------------
// Periodic 2-deep lateral halo (the halo swap of Sec. 2.1 on one periodic
// domain).  One thread per (halo column, level); the halo columns of all
// fields are enumerated in one launch: first the 2+2 full rows i in {-2,-1,
// nx, nx+1} (ny+4 columns each), then the 2+2 partial rows j in {-2,-1,ny,ny+1}
// for i in [0,nx).  The copy moves raw bits.
// ---------------------------------------------------------------------------
struct HaloArgs {
    void* f[3 + MAXS];
    int nfields, nx, ny, nz;
};

template <typename E>
__global__ void __launch_bounds__(256) halo_kernel(HaloArgs a) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long ncol = 4L * (ny + 4) + 4L * nx;
    const long per_field = ncol * nz;
    const long total = per_field * a.nfields;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long)gridDim.x * blockDim.x) {
        const int f = (int)(t / per_field);
        const long r = t - (long)f * per_field;
        const long h = r / nz;
        const int k = (int)(r - h * nz);
        int i, j;
        if (h < 4L * (ny + 4)) {
            const int row = (int)(h / (ny + 4));
            j = (int)(h % (ny + 4)) - 2;
            i = row < 2 ? row - 2 : nx + (row - 2);
        } else {
            const long h2 = h - 4L * (ny + 4);
            const int row = (int)(h2 / nx);
            i = (int)(h2 % nx);
            j = row < 2 ? row - 2 : ny + (row - 2);
        }
        int si = i % nx;
        if (si < 0) si += nx;
        int sj = j % ny;
        if (sj < 0) sj += ny;
        E* p = (E*)a.f[f];
        const long dst = ((long)(i + 2) * (ny + 4) + (j + 2)) * nz + k;
        const long src = ((long)(si + 2) * (ny + 4) + (sj + 2)) * nz + k;
        p[dst] = p[src];
    }
}

// ---------------------------------------------------------------------------
// Marshalling (Sec. 4.1): FP64 field minus a constant, rounded to FP32 or
// BF16 (round to nearest even), over the whole padded array.  A streaming
// copy: blockIdx.y picks the field, every lane converts four consecutive
// values per trip (two 16-byte loads, one 16- or 8-byte store, all
// non-temporal), and the last n % 4 values of a field go to the first lanes.
// ---------------------------------------------------------------------------
struct CastArgs {
    const double* src[3 + MAXS];
    void* dst[3 + MAXS];
    double off[3 + MAXS];
    int nfields;
    long n;
};

typedef double cast_d2 __attribute__((ext_vector_type(2)));
typedef float cast_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int cast_u2 __attribute__((ext_vector_type(2)));

template <int DT>
__global__ void __launch_bounds__(256) cast_kernel(CastArgs a) {
    const int f = blockIdx.y;
    const double* __restrict__ src = a.src[f];
    const double off = a.off[f];
    const long n4 = a.n >> 2;
    const long stride = (long)gridDim.x * blockDim.x;
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long t = t0; t < n4; t += stride) {
        const cast_d2 x0 = __builtin_nontemporal_load((const cast_d2*)src + 2 * t);
        const cast_d2 x1 = __builtin_nontemporal_load((const cast_d2*)src + 2 * t + 1);
        const float y0 = (float)(x0.x - off), y1 = (float)(x0.y - off);
        const float y2 = (float)(x1.x - off), y3 = (float)(x1.y - off);
        if constexpr (DT == MONC_F32) {
            const cast_f4 y = {y0, y1, y2, y3};
            __builtin_nontemporal_store(y, (cast_f4*)a.dst[f] + t);
        } else {
            const cast_u2 y = {(unsigned)f32_to_bf16_rne(y0) | ((unsigned)f32_to_bf16_rne(y1) << 16),
                               (unsigned)f32_to_bf16_rne(y2) | ((unsigned)f32_to_bf16_rne(y3) << 16)};
            __builtin_nontemporal_store(y, (cast_u2*)a.dst[f] + t);
        }
    }
    const long e = 4 * n4 + t0;  // the tail (fewer than four values)
    if (e < a.n) {
        const float y = (float)(src[e] - off);
        if constexpr (DT == MONC_F32)
            ((float*)a.dst[f])[e] = y;
        else
            ((uint16_t*)a.dst[f])[e] = f32_to_bf16_rne(y);
    }
}

// ---------------------------------------------------------------------------
// Final budget reduction: one workgroup combines the per-workgroup partials
// in a fixed order (strided per thread, then a fixed butterfly per wave, then
// the waves in order), so the result is bitwise repeatable.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bop(int q) {
    if (q == MONC_B_COURANT) return 1;
    if (q >= MONC_B_SCALAR0 && (q - MONC_B_SCALAR0) % 3 == 2) return 2;
    return 0;
}

__device__ __forceinline__ double bcomb(double a, double b, int op) {
    return op == 0 ? a + b : (op == 1 ? fmax(a, b) : fmin(a, b));
}

__global__ void __launch_bounds__(256) budget_final(const double* __restrict__ partials,
                                                    int nblocks, double* __restrict__ out) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = blockIdx.x;  // one workgroup per budget entry
    const int op = bop(q);
    double v = op == 2 ? __builtin_huge_val() : 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) v = bcomb(v, partials[(long)b * NB + q], op);
    for (int o = 32; o > 0; o >>= 1) v = bcomb(v, __shfl_xor(v, o, 64), op);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < 4; w++) r = bcomb(r, red[w], op);
        out[q] = r;
    }
}

int grid_for(long total) {
    long b = (total + 255) / 256;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_halo(int elem_bytes, int nfields, void* const* fields, int nx,
                       int ny, int nz, hipStream_t s) {
    HaloArgs a;
    for (int f = 0; f < nfields; f++) a.f[f] = fields[f];
    a.nfields = nfields;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    const long total = (4L * (ny + 4) + 4L * nx) * nz * nfields;
    const int g = grid_for(total);
    if (elem_bytes == 8)
        halo_kernel<uint64_t><<<g, 256, 0, s>>>(a);
    else if (elem_bytes == 4)
        halo_kernel<uint32_t><<<g, 256, 0, s>>>(a);
    else
        halo_kernel<uint16_t><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_cast(int dtype, int nfields, const double* const* src,
                       void* const* dst, const double* offset, long n, hipStream_t s) {
    CastArgs a;
    for (int f = 0; f < nfields; f++) {
        a.src[f] = src[f];
        a.dst[f] = dst[f];
        a.off[f] = offset ? offset[f] : 0.0;
    }
    a.nfields = nfields;
    a.n = n;
    // about 2048 workgroups in all, each lane a few trips of four values
    long gx = ((n >> 2) + 255) / 256;
    const long cap = (2048 + nfields - 1) / nfields;
    if (gx > cap) gx = cap;
    if (gx < 1) gx = 1;
    const dim3 grid((unsigned)gx, (unsigned)nfields);
    if (dtype == MONC_F32)
        cast_kernel<MONC_F32><<<grid, 256, 0, s>>>(a);
    else
        cast_kernel<MONC_BF16><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_budget_final(const double* partials, int nblocks, double* budgets,
                               hipStream_t s) {
    budget_final<<<NB, 256, 0, s>>>(partials, nblocks, budgets);
    return hipGetLastError();
}

}  // namespace monc
