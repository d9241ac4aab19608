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
// BF16 (round to nearest even), over the whole padded array.
// ---------------------------------------------------------------------------
struct CastArgs {
    const double* src[3 + MAXS];
    void* dst[3 + MAXS];
    double off[3 + MAXS];
    int nfields;
    long n;
};

template <int DT>
__global__ void __launch_bounds__(256) cast_kernel(CastArgs a) {
    const long total = a.n * a.nfields;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long)gridDim.x * blockDim.x) {
        const int f = (int)(t / a.n);
        const long e = t - (long)f * a.n;
        const double x = a.src[f][e] - a.off[f];
        if constexpr (DT == MONC_F32) {
            ((float*)a.dst[f])[e] = (float)x;
        } else {
            ((uint16_t*)a.dst[f])[e] = f32_to_bf16_rne((float)x);
        }
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
    const int g = grid_for(n * nfields);
    if (dtype == MONC_F32)
        cast_kernel<MONC_F32><<<g, 256, 0, s>>>(a);
    else
        cast_kernel<MONC_BF16><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_budget_final(const double* partials, int nblocks, double* budgets,
                               hipStream_t s) {
    budget_final<<<NB, 256, 0, s>>>(partials, nblocks, budgets);
    return hipGetLastError();
}

}  // namespace monc
