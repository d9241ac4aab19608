// learned.hip -- the learned coarse-grid flux correction on gfx950.
//
// Restriction of fine states to a 4x coarser grid, the feature gather, a
// 300 -> 64 -> 64 -> 4 GELU MLP evaluated and trained with BF16 MFMA
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation, FP32 master weights + Adam),
// the flux-divergence loss, and the corrected coarse step with its fallback to
// the plain PW/TVD step.
#include <math.h>

#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

constexpr int NIN = MONC_MLP_NIN, KP = MONC_MLP_K, HID = MONC_MLP_H, NO = MONC_MLP_NOUT;
constexpr int OFF_W1 = 0, OFF_B1 = HID * KP, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + NO * HID;
constexpr int NPARAM = OFF_B3 + NO;
static_assert(NPARAM == MONC_MLP_NPARAM, "parameter layout");
// bf16 weight pack: W1 [64][320] | W2 [64][64] | W3 padded to [32][64]
constexpr int PK_W1 = 0, PK_W2 = HID * KP, PK_W3 = PK_W2 + HID * HID;
constexpr int PK_SIZE = PK_W3 + 32 * HID;
static_assert(PK_SIZE == MONC_MLP_WPACK, "pack layout");

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
struct u16x8 {
    uint16_t v[8];
};

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// FP32 -> BF16, round to nearest even: the native conversion of gfx950
// (v_cvt_pk_bf16_f32), the same rounding as f32_to_bf16_rne in fewer
// instructions (the activations of every layer pass through it)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ bf16x8_t ld8(const uint16_t* p) {  // 16-byte aligned
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8_t, v);
}
__device__ __forceinline__ bf16x8_t gather8(const uint16_t* p, int stride) {
    u16x8 t;
#pragma unroll
    for (int v = 0; v < 8; v++) t.v[v] = p[v * stride];
    return __builtin_bit_cast(bf16x8_t, t);
}
__device__ __forceinline__ bf16x8_t zero8() {
    u16x8 t;
#pragma unroll
    for (int v = 0; v < 8; v++) t.v[v] = 0;
    return __builtin_bit_cast(bf16x8_t, t);
}
__device__ __forceinline__ f32x16_t mfma(bf16x8_t a, bf16x8_t b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// Accumulator element r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32
// of the 32x32 tile.  Operand fragments: lane l supplies row (A) / column (B)
// l%32 and the 8 k-values 8(l/32) .. 8(l/32)+7 of each 16-wide k block (the
// same k assignment for A and B, which is all the product needs).
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// GELU(z) = z Phi(z) with Phi(z) = erfc(-z/sqrt 2)/2, which keeps its relative
// accuracy for negative z (1 + erf(z/sqrt 2) cancels there).  erfc is the
// Chebyshev fit of Numerical Recipes (Press et al., 2nd ed., Sec. 6.2,
// fractional error below 1.2e-7 for all x): branch-free, one exponential and
// one reciprocal, far below the BF16 rounding that follows.
__device__ __forceinline__ float erfc_cheb(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.5f * ax);  // v_rcp_f32, about 1 ulp
    float p = 0.17087277f;
    p = fmaf(p, t, -0.82215223f);
    p = fmaf(p, t, 1.48851587f);
    p = fmaf(p, t, -1.13520398f);
    p = fmaf(p, t, 0.27886807f);
    p = fmaf(p, t, -0.18628806f);
    p = fmaf(p, t, 0.09678418f);
    p = fmaf(p, t, 0.37409196f);
    p = fmaf(p, t, 1.00002368f);
    p = fmaf(p, t, -1.26551223f);
    const float r = t * __expf(p - ax * ax);
    return x >= 0.0f ? r : 2.0f - r;
}
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * erfc_cheb(-z * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * erfc_cheb(-z * 0.70710678118654752f) +
           z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// MFMA k-assignment of the first layer: in 16-wide block kk, lanes 0-31 take
// 8 consecutive slots of one field and lanes 32-63 the same 8 slots of the
// next field (fields u, v for kk < 10, w, theta after), so both halves of a
// row share their neighbourhood offsets.  With 80 slots per field the 8
// values are one aligned 16-byte chunk of a feature row or weight row.
__device__ __forceinline__ int kslot(int kk, int h) { return (2 * (kk / 10) + h) * 80 + 8 * (kk % 10); }

// ---------------------------------------------------------------------------
// 4x restriction: mass-weighted scalars, mass-flux-weighted face means for u,
// v, plain means for w on the coarse top faces; coarse profiles.
// ---------------------------------------------------------------------------
struct RestrictArgs {
    const double* fine[3 + MAXS];
    double* coarse[3 + MAXS];
    int nscal, nx, ny, nz;
    const double *rdz, *rho, *rhon;
    double *rdz_c, *rho_c, *rhon_c;
};

__global__ void __launch_bounds__(256) restrict_profiles(RestrictArgs a) {
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= a.nz / 4) return;
    double dZ = 0.0, mZ = 0.0;
    for (int k = 4 * K; k < 4 * K + 4; k++) {
        const double dz = 1.0 / a.rdz[k];
        dZ += dz;
        mZ += a.rhon[k] * dz;
    }
    a.rdz_c[K] = 1.0 / dZ;
    a.rhon_c[K] = mZ / dZ;
    a.rho_c[K] = a.rho[4 * K + 3];
}

__global__ void __launch_bounds__(256) restrict_fields(RestrictArgs a) {
    const int NX = a.nx / 4, NY = a.ny / 4, NZ = a.nz / 4;
    const long n = (long)NX * NY * NZ;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int K = (int)(t % NZ), J = (int)((t / NZ) % NY), I = (int)(t / ((long)NZ * NY));
    const long fsx = (long)(a.ny + 4) * a.nz;
    auto F = [&](int f, int i, int j, int k) -> double {
        return a.fine[f][(long)(i + 2) * fsx + (long)(j + 2) * a.nz + k];
    };
    double mZ = 0.0;
    for (int k = 4 * K; k < 4 * K + 4; k++) mZ += a.rhon[k] / a.rdz[k];
    double su = 0.0, sv = 0.0, sw = 0.0;
    for (int j = 4 * J; j < 4 * J + 4; j++)
        for (int k = 4 * K; k < 4 * K + 4; k++) su += a.rhon[k] / a.rdz[k] * F(0, 4 * I + 3, j, k);
    for (int i = 4 * I; i < 4 * I + 4; i++)
        for (int k = 4 * K; k < 4 * K + 4; k++) sv += a.rhon[k] / a.rdz[k] * F(1, i, 4 * J + 3, k);
    for (int i = 4 * I; i < 4 * I + 4; i++)
        for (int j = 4 * J; j < 4 * J + 4; j++) sw += F(2, i, j, 4 * K + 3);
    const long c = (long)(I + 2) * (NY + 4) * NZ + (long)(J + 2) * NZ + K;
    a.coarse[0][c] = su / (4.0 * mZ);
    a.coarse[1][c] = sv / (4.0 * mZ);
    a.coarse[2][c] = K == NZ - 1 ? 0.0 : sw / 16.0;
    for (int s = 0; s < a.nscal; s++) {
        double sp = 0.0;
        for (int i = 4 * I; i < 4 * I + 4; i++)
            for (int j = 4 * J; j < 4 * J + 4; j++)
                for (int k = 4 * K; k < 4 * K + 4; k++) sp += a.rhon[k] / a.rdz[k] * F(3 + s, i, j, k);
        a.coarse[3 + s][c] = sp / (16.0 * mZ);
    }
}

// ---------------------------------------------------------------------------
// Feature gather: row c of X = the 5x5x3 neighbourhood of (u, v, w, theta)
// around cell cells[c] (or c), standardised, in BF16; orient 1 exchanges x and
// y (and u, v).  One thread per (row, feature).
// ---------------------------------------------------------------------------
struct FeatArgs {
    const double* f[4];
    double mean[4], inv_std[4];
    int nx, ny, nz, orient;
    const int* cells;
    long ncells;
    uint16_t* X;
};

__global__ void __launch_bounds__(256) features_kernel(FeatArgs a) {
    // one thread per (row, 8-slot chunk): 40 chunks of a 320-slot row, one
    // 16-byte store; the cell is decoded once for its 8 values
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.ncells * (KP / 8)) return;
    const long row = t / (KP / 8);
    const int chunk = (int)(t - row * (KP / 8));
    const int f = chunk / 10, p0 = 8 * (chunk % 10);
    const int cell = a.cells ? a.cells[row] : (int)row;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const bool inside = (unsigned)cell < (unsigned)(nx * ny * nz);
    const int c = inside ? cell : 0;
    const int k = c % nz, ij = c / nz;
    const int j = ij % ny, i = ij / ny;
    const int src = a.orient ? (f == 0 ? 1 : (f == 1 ? 0 : f)) : f;
    const double* fld = a.f[src];
    const double mean = a.mean[src], inv = a.inv_std[src];
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int pos = p0 + e;
        uint16_t out = 0;
        if (pos < 75 && inside) {
            const int a5 = pos / 15, b5 = (pos / 3) % 5, c3 = pos % 3;
            const int di = a.orient ? b5 - 2 : a5 - 2;
            const int dj = a.orient ? a5 - 2 : b5 - 2;
            int ii = i + di, jj = j + dj;  // offsets of at most 2 cells: wrap by adds
            ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
            ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
            jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
            jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
            int kk = k + c3 - 1;
            kk = kk < 0 ? 0 : (kk > nz - 1 ? nz - 1 : kk);
            const double x = fld[((long)(ii + 2) * (ny + 4) + (jj + 2)) * nz + kk];
            out = f2bf((float)((x - mean) * inv));
        }
        v.v[e] = out;
    }
    reinterpret_cast<uint4*>(a.X)[t] = __builtin_bit_cast(uint4, v);
}

// ---------------------------------------------------------------------------
// Weight pack (FP32 master -> BF16 MFMA operands)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pack_kernel(const float* __restrict__ p, uint16_t* __restrict__ w) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= PK_SIZE) return;
    float v = 0.0f;
    if (t < PK_W2) {
        v = p[OFF_W1 + t];
    } else if (t < PK_W3) {
        v = p[OFF_W2 + (t - PK_W2)];
    } else {
        const int r = (t - PK_W3) / HID, c = (t - PK_W3) % HID;
        v = r < NO ? p[OFF_W3 + r * HID + c] : 0.0f;
    }
    w[t] = f2bf(v);
}

// ---------------------------------------------------------------------------
// Forward: 4 waves x 32 rows.  H = GELU(X W1^T + b1), H2 = GELU(H W2^T + b2),
// Y = H2 W3^T + b3, with BF16 operands (X, W, H, H2) and FP32 accumulation.
// ---------------------------------------------------------------------------
constexpr int FWD_ROWS = 128;
// LDS copies of the weights and the hidden activations use row strides padded
// by 8 elements (16 bytes): with the unpadded strides (640 and 128 bytes) all
// 32 rows that a 16-byte fragment load touches fall on the same LDS banks.
constexpr int LW1 = KP + 8, LWH = HID + 8;
constexpr int S_W1 = 0, S_W2 = HID * LW1, S_W3 = S_W2 + HID * LWH, S_WEND = S_W3 + 32 * LWH;
constexpr size_t FWD_LDS = (size_t)S_WEND * 2 + 4 * 32 * LWH * 2 + (2 * HID + NO) * 4;

// Global weight pack -> padded LDS copy, 16 bytes per thread and step.
__device__ __forceinline__ void load_pack_padded(const uint16_t* __restrict__ wpack, uint16_t* sw) {
    for (int t = threadIdx.x; t < PK_SIZE / 8; t += blockDim.x) {
        const int g = 8 * t;
        int d;
        if (g < PK_W2) {
            d = S_W1 + (g / KP) * LW1 + g % KP;
        } else if (g < PK_W3) {
            d = S_W2 + ((g - PK_W2) / HID) * LWH + (g - PK_W2) % HID;
        } else {
            d = S_W3 + ((g - PK_W3) / HID) * LWH + (g - PK_W3) % HID;
        }
        *reinterpret_cast<uint4*>(sw + d) = reinterpret_cast<const uint4*>(wpack)[t];
    }
}

__global__ void __launch_bounds__(256) mlp_forward(const uint16_t* __restrict__ X, int m,
                                                   const float* __restrict__ params,
                                                   const uint16_t* __restrict__ wpack,
                                                   float* __restrict__ Y, uint16_t* H1o,
                                                   uint16_t* H2o, float* Z1o, float* Z2o) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* sw = reinterpret_cast<uint16_t*>(smem);  // pack
    uint16_t* sH = sw + S_WEND;                           // [4][32][LWH]
    float* sb = reinterpret_cast<float*>(sH + 4 * 32 * LWH);
    load_pack_padded(wpack, sw);
    for (int t = threadIdx.x; t < 2 * HID + NO; t += 256)
        sb[t] = t < HID ? params[OFF_B1 + t] : (t < 2 * HID ? params[OFF_B2 + t - HID] : params[OFF_B3 + t - 2 * HID]);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = blockIdx.x * FWD_ROWS + 32 * w;
    const int ar = row0 + (lane & 31);  // A-operand row of this lane
    const int kh = 8 * (lane >> 5);
    uint16_t* H = sH + w * 32 * LWH;

    // layer 1
    const int h = lane >> 5;
    f32x16_t acc1[2] = {{}, {}};
    for (int kk = 0; kk < KP / 16; kk++) {
        const int ks = kslot(kk, h);
        const bf16x8_t av = ar < m ? ld8(X + (size_t)ar * KP + ks) : zero8();
#pragma unroll
        for (int nt = 0; nt < 2; nt++)
            acc1[nt] = mfma(av, ld8(sw + S_W1 + (32 * nt + (lane & 31)) * LW1 + ks), acc1[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
        const f32x16_t acc = acc1[nt];
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int lr = acc_row(r, lane), col = 32 * nt + (lane & 31);
            const int row = row0 + lr;
            const float z = acc[r] + sb[col];
            const uint16_t h = f2bf(gelu(z));
            H[lr * LWH + col] = h;
            if (row < m) {
                if (Z1o) Z1o[(size_t)row * HID + col] = z;
                if (H1o) H1o[(size_t)row * HID + col] = h;
            }
        }
    }
    __syncthreads();
    // layer 2
    f32x16_t acc2[2];
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
        f32x16_t acc = {};
#pragma unroll
        for (int kk = 0; kk < HID / 16; kk++) {
            const bf16x8_t av = ld8(H + (lane & 31) * LWH + 16 * kk + kh);
            const bf16x8_t bv = ld8(sw + S_W2 + (32 * nt + (lane & 31)) * LWH + 16 * kk + kh);
            acc = mfma(av, bv, acc);
        }
        acc2[nt] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int lr = acc_row(r, lane), col = 32 * nt + (lane & 31);
            const int row = row0 + lr;
            const float z = acc2[nt][r] + sb[HID + col];
            const uint16_t h = f2bf(gelu(z));
            H[lr * LWH + col] = h;
            if (row < m) {
                if (Z2o) Z2o[(size_t)row * HID + col] = z;
                if (H2o) H2o[(size_t)row * HID + col] = h;
            }
        }
    }
    __syncthreads();
    // layer 3 (4 outputs, padded to a 32-wide tile)
    f32x16_t acc = {};
#pragma unroll
    for (int kk = 0; kk < HID / 16; kk++) {
        const bf16x8_t av = ld8(H + (lane & 31) * LWH + 16 * kk + kh);
        const bf16x8_t bv = ld8(sw + S_W3 + (lane & 31) * LWH + 16 * kk + kh);
        acc = mfma(av, bv, acc);
    }
    const int col = lane & 31;
    if (col < NO) {
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int row = row0 + acc_row(r, lane);
            if (row < m) Y[(size_t)row * NO + col] = acc[r] + sb[2 * HID + col];
        }
    }
}

// ---------------------------------------------------------------------------
// Inference over every cell with the feature gather fused in: each lane builds
// its MFMA operand fragments straight from the fields (no feature matrix in
// memory), then the three layers run as in mlp_forward.  Workgroups are
// persistent, so the weight pack is loaded into LDS once per workgroup.  The
// features, products and sums are the same operations in the same order as
// mlp_features followed by mlp_forward, so the outputs are bitwise the same.
// ---------------------------------------------------------------------------
struct InferArgs {
    const double* f[4];
    double mean[4], inv_std[4];
    int nx, ny, nz;
    long m;  // nx * ny * nz rows
    const float* params;
    const uint16_t* wpack;
    float* Y;
};

// Per-row gather state: wrapped plane offsets xo, column offsets yo, clamped
// levels ko of the row's cell, and this lane's field of each pair (lanes 0-31:
// u then w; lanes 32-63: v then theta, exchanged with u/v for y-faces).
struct RowGather {
    long xo[5], yo[5];
    int ko[3];
    const double* f[2];
    double mean[2], inv[2];
};

template <int ORIENT>
__device__ __forceinline__ void row_setup(const InferArgs& a, long row, int h, RowGather& g) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int k = (int)(row % nz);
    const long col = row / nz;
    const int j = (int)(col % ny), i = (int)(col / ny);
#pragma unroll
    for (int d = 0; d < 5; d++) {
        const int ii = ((i + d - 2) % nx + nx) % nx, jj = ((j + d - 2) % ny + ny) % ny;
        // y-faces exchange the roles of x and y
        const long xoff = (long)(ii + 2) * (ny + 4) * nz, yoff = (long)(jj + 2) * nz;
        g.xo[d] = ORIENT ? yoff : xoff;
        g.yo[d] = ORIENT ? xoff : yoff;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int kk = k + c - 1;
        g.ko[c] = kk < 0 ? 0 : (kk > nz - 1 ? nz - 1 : kk);
    }
#pragma unroll
    for (int pr = 0; pr < 2; pr++) {
        const int fi = 2 * pr + h;                                  // feature field
        const int src = ORIENT ? (fi == 0 ? 1 : (fi == 1 ? 0 : fi)) : fi;  // stored field
        g.f[pr] = a.f[src];
        g.mean[pr] = a.mean[src];
        g.inv[pr] = a.inv_std[src];
    }
}

// Operand fragment of block kk: slots 8(kk%10) .. +7 of this lane's field of
// pair kk/10; slot p < 75 is neighbour (a, b, c) = (p/15, (p/3)%5, p%3).
__device__ __forceinline__ bf16x8_t row_fragment(const RowGather& g, int kk) {
    const int pr = kk / 10, p0 = 8 * (kk % 10);
    u16x8 t;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int pos = p0 + e;
        if (pos < 75) {
            const int a5 = pos / 15, b5 = (pos / 3) % 5, c3 = pos % 3;
            const double v = g.f[pr][g.xo[a5] + g.yo[b5] + g.ko[c3]];
            t.v[e] = f2bf((float)((v - g.mean[pr]) * g.inv[pr]));
        } else {
            t.v[e] = 0;
        }
    }
    return __builtin_bit_cast(bf16x8_t, t);
}

// Staged gather (STAGED): on grids of 32 levels whose columns come in groups of
// four along y (ny % 4 == 0), a tile's 128 rows are four whole columns of one
// x-plane.  The tile's whole neighbourhood -- 5 x-planes, the 4 columns plus 2
// on each side, 32 levels, 4 fields: 160 columns of 32 values -- is read once,
// every load issued before any is used, standardised and rounded to BF16 into
// the LDS that later holds the hidden activations; the operand fragments are
// then gathered from LDS.  The values are the same operations on the same
// numbers, so the outputs are bitwise those of the direct gather.
constexpr int SNZ = 32;                        // levels of a staged grid
constexpr int SCOLS = FWD_ROWS / SNZ + 4;      // staged columns per x-plane (8)
constexpr int SPT = 4 * 5 * SCOLS * SNZ / 256; // staged values per thread (20)
constexpr int STAGE_BYTES_MAX = 4 * 32 * (HID + 8) * 2;  // the activation area
static_assert(4 * 5 * SCOLS * SNZ * 2 <= STAGE_BYTES_MAX, "staged tile fits");
static_assert(4 * 5 * SCOLS * SNZ == SPT * 256, "whole passes");

__host__ __device__ constexpr bool infer_staged_ok(int ny, int nz) {
    return nz == SNZ && ny % (FWD_ROWS / SNZ) == 0;
}

template <int ORIENT>
__device__ __forceinline__ void stage_tile(const InferArgs& a, long tile, uint16_t* st) {
    const int nx = a.nx, ny = a.ny;
    const long col0 = tile * (FWD_ROWS / SNZ);  // first column (i * ny + j) of the tile
    const int i = (int)(col0 / ny), j0 = (int)(col0 % ny);
    const int kk = threadIdx.x % SNZ;
    double v[SPT];
    // all loads first: SPT independent requests in flight per thread
#pragma unroll
    for (int q = 0; q < SPT; q++) {
        const int col = q * (256 / SNZ) + (int)threadIdx.x / SNZ;  // (f, xi, c) column
        const int c = col % SCOLS, xi = (col / SCOLS) % 5, f = col / (5 * SCOLS);
        int ii = i + xi - 2, jj = j0 + c - 2;
        ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
        ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
        jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
        jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
        v[q] = a.f[f][((long)(ii + 2) * (ny + 4) + (jj + 2)) * SNZ + kk];
    }
#pragma unroll
    for (int q = 0; q < SPT; q++) {
        const int col = q * (256 / SNZ) + (int)threadIdx.x / SNZ;
        const int f = col / (5 * SCOLS);
        st[q * 256 + threadIdx.x] = f2bf((float)((v[q] - a.mean[f]) * a.inv_std[f]));
    }
}

// Fragment of block kk from the staged tile: lane's local column lc, level k.
template <int ORIENT>
__device__ __forceinline__ bf16x8_t row_fragment_staged(const uint16_t* st, int lc, int k,
                                                        int h, int kk) {
    const int pr = kk / 10, p0 = 8 * (kk % 10);
    const int fi = 2 * pr + h;
    const int src = ORIENT ? (fi == 0 ? 1 : (fi == 1 ? 0 : fi)) : fi;
    const uint16_t* base = st + src * 5 * SCOLS * SNZ + lc * SNZ;
    int kc[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int q = k + c - 1;
        kc[c] = q < 0 ? 0 : (q > SNZ - 1 ? SNZ - 1 : q);
    }
    u16x8 t;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int pos = p0 + e;
        if (pos < 75) {
            const int a5 = pos / 15, b5 = (pos / 3) % 5, c3 = pos % 3;
            const int xi = ORIENT ? b5 : a5, yj = ORIENT ? a5 : b5;
            t.v[e] = base[(xi * SCOLS + yj) * SNZ + kc[c3]];
        } else {
            t.v[e] = 0;
        }
    }
    return __builtin_bit_cast(bf16x8_t, t);
}

// ORIENT 0: x-faces, 1: y-faces (the exchanged frame), 2: both from one
// staged tile (staged grids only): Y receives the x-face rows, then the
// y-face rows at Y + m * NO.
template <int ORIENT, bool STAGED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    mlp_infer(InferArgs a) {
    static_assert(ORIENT < 2 || STAGED, "both orientations only from a staged tile");
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* sw = reinterpret_cast<uint16_t*>(smem);  // pack
    uint16_t* sH = sw + S_WEND;                           // [4][32][LWH]
    float* sb = reinterpret_cast<float*>(sH + 4 * 32 * LWH);
    load_pack_padded(a.wpack, sw);
    for (int t = threadIdx.x; t < 2 * HID + NO; t += 256)
        sb[t] = t < HID ? a.params[OFF_B1 + t]
                        : (t < 2 * HID ? a.params[OFF_B2 + t - HID] : a.params[OFF_B3 + t - 2 * HID]);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kh = 8 * (lane >> 5);
    const int h = lane >> 5;
    uint16_t* H = sH + w * 32 * LWH;
    const long ntiles = (a.m + FWD_ROWS - 1) / FWD_ROWS;
    constexpr int NOR = ORIENT == 2 ? 2 : 1;
    // layer 1 of orientation O from the staged tile
    auto layer1_staged = [&](auto O, const uint16_t* st, f32x16_t* acc1) {
        const int lc = w, k = lane & 31;  // 32 rows per wave = one column
#pragma unroll
        for (int kk = 0; kk < KP / 16; kk++) {
            const int ks = kslot(kk, h);
            const bf16x8_t av = row_fragment_staged<decltype(O)::value>(st, lc, k, h, kk);
#pragma unroll
            for (int nt = 0; nt < 2; nt++)
                acc1[nt] = mfma(av, ld8(sw + S_W1 + (32 * nt + (lane & 31)) * LW1 + ks), acc1[nt]);
        }
    };
    // the first hidden layer's activations of this lane, BF16, two per word
    auto activate1 = [&](const f32x16_t* acc1, uint32_t* hv) {
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
            const float b = sb[32 * nt + (lane & 31)];
#pragma unroll
            for (int r = 0; r < 16; r += 2)
                hv[8 * nt + r / 2] = (uint32_t)f2bf(gelu(acc1[nt][r] + b)) |
                                     ((uint32_t)f2bf(gelu(acc1[nt][r + 1] + b)) << 16);
        }
    };
    // layers 2 and 3 of one orientation from its first activations; rows to Yo
    auto finish_rows = [&](const uint32_t* hv, long row0, float* Yo) {
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int lr = acc_row(r, lane), col = 32 * nt + (lane & 31);
                H[lr * LWH + col] = (uint16_t)(hv[8 * nt + r / 2] >> (16 * (r & 1)));
            }
        }
        __syncthreads();
        // layer 2
        f32x16_t acc2[2];
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < HID / 16; kk++) {
                const bf16x8_t av = ld8(H + (lane & 31) * LWH + 16 * kk + kh);
                const bf16x8_t bv = ld8(sw + S_W2 + (32 * nt + (lane & 31)) * LWH + 16 * kk + kh);
                acc = mfma(av, bv, acc);
            }
            acc2[nt] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int lr = acc_row(r, lane), col = 32 * nt + (lane & 31);
                H[lr * LWH + col] = f2bf(gelu(acc2[nt][r] + sb[HID + col]));
            }
        }
        __syncthreads();
        // layer 3
        f32x16_t acc = {};
#pragma unroll
        for (int kk = 0; kk < HID / 16; kk++) {
            const bf16x8_t av = ld8(H + (lane & 31) * LWH + 16 * kk + kh);
            const bf16x8_t bv = ld8(sw + S_W3 + (lane & 31) * LWH + 16 * kk + kh);
            acc = mfma(av, bv, acc);
        }
        const int col = lane & 31;
        if (col < NO) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const long row = row0 + acc_row(r, lane);
                if (row < a.m) Yo[(size_t)row * NO + col] = acc[r] + sb[2 * HID + col];
            }
        }
        __syncthreads();  // H is rewritten next
    };
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long row0 = tile * FWD_ROWS + 32 * w;
        const long ar = row0 + (lane & 31);
        const bool live = ar < a.m;
        f32x16_t acc1[2] = {{}, {}};
        uint32_t hv[NOR][16];  // first activations, per orientation
        if constexpr (STAGED) {
            uint16_t* st = sH;  // the activation area, free until layer 1 ends
            stage_tile<ORIENT == 1 ? 1 : 0>(a, tile, st);
            __syncthreads();
            if constexpr (ORIENT == 2) {
                // x-faces, activated before the y-faces' layer 1 (fewer live sums)
                layer1_staged(std::integral_constant<int, 0>(), st, acc1);
                activate1(acc1, hv[0]);
                acc1[0] = acc1[1] = f32x16_t{};
                // keep the scheduler from interleaving the two gathers (their
                // loads in flight together would not fit the registers)
                __builtin_amdgcn_sched_barrier(0);
                layer1_staged(std::integral_constant<int, 1>(), st, acc1);
                activate1(acc1, hv[1]);
            } else {
                layer1_staged(std::integral_constant<int, ORIENT>(), st, acc1);
                activate1(acc1, hv[0]);
            }
            __syncthreads();  // every wave is done with the staged tile
        } else {
            RowGather g;
            row_setup<ORIENT>(a, live ? ar : 0, h, g);
            // layer 1: fragments built block by block straight from the
            // fields; fully unrolled, so every slot index is a constant and the
            // gather state stays in registers
#pragma unroll
            for (int kk = 0; kk < KP / 16; kk++) {
                const int ks = kslot(kk, h);
                const bf16x8_t av = live ? row_fragment(g, kk) : zero8();
#pragma unroll
                for (int nt = 0; nt < 2; nt++)
                    acc1[nt] = mfma(av, ld8(sw + S_W1 + (32 * nt + (lane & 31)) * LW1 + ks),
                                    acc1[nt]);
            }
            activate1(acc1, hv[0]);
        }
#pragma unroll
        for (int o = 0; o < NOR; o++) {
            finish_rows(hv[o], row0, a.Y + (size_t)o * a.m * NO);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ---------------------------------------------------------------------------
// Backward: a persistent grid of at most BWD_GRID workgroups (4 waves); each
// takes 64-row chunks c = blockIdx.x, blockIdx.x + gridDim.x, ... and keeps
// its gradient sums in registers across them (the MFMA tiles of dW1 and dW2
// in their accumulators), then writes one partial row.  The grid depends only
// on m, so the rows and their fixed-order sum (reduce_partials: one column
// per lane, rows in order) are repeatable bit for bit.
// ---------------------------------------------------------------------------
constexpr int BWD_ROWS = 64;
constexpr int BWD_GRID = 256;
constexpr size_t BWD_LDS = (size_t)BWD_ROWS * KP * 2 + 4 * (size_t)BWD_ROWS * HID * 2 +
                           (size_t)HID * HID * 2 + (size_t)BWD_ROWS * NO * 4 + NO * HID * 4 +
                           2 * 256 * 4;

int bwd_grid(int m) {
    const int chunks = (m + BWD_ROWS - 1) / BWD_ROWS;
    return chunks < BWD_GRID ? chunks : BWD_GRID;
}

__global__ void __launch_bounds__(256) mlp_backward(const uint16_t* __restrict__ X,
                                                    const uint16_t* __restrict__ H1,
                                                    const uint16_t* __restrict__ H2,
                                                    const float* __restrict__ Z1,
                                                    const float* __restrict__ Z2,
                                                    const float* __restrict__ dY, int m,
                                                    const uint16_t* __restrict__ wpack,
                                                    float* __restrict__ partials) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* sX = reinterpret_cast<uint16_t*>(smem);  // [64][320]
    uint16_t* sH1 = sX + BWD_ROWS * KP;                   // [64][64]
    uint16_t* sH2 = sH1 + BWD_ROWS * HID;
    uint16_t* sdZ2 = sH2 + BWD_ROWS * HID;
    uint16_t* sdZ1 = sdZ2 + BWD_ROWS * HID;
    uint16_t* sW2 = sdZ1 + BWD_ROWS * HID;               // W2[j2][j1]
    float* sdY = reinterpret_cast<float*>(sW2 + HID * HID);  // [64][4]
    float* sW3 = sdY + BWD_ROWS * NO;                    // [4][64] (bf16 values)
    float* red = sW3 + NO * HID;                          // [2][256]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    float* part = partials + (size_t)blockIdx.x * NPARAM;
    const int nchunks = (m + BWD_ROWS - 1) / BWD_ROWS;
    const int kh = 8 * (lane >> 5);

    for (int t = tid; t < HID * HID; t += 256) sW2[t] = wpack[PK_W2 + t];
    for (int t = tid; t < NO * HID; t += 256) sW3[t] = bf2f(wpack[PK_W3 + t]);

    // sums kept across the chunks
    float db2 = 0.0f;     // column tid % 64, rows tid/64 + 4q
    float colsum1 = 0.0f; // b1: column 32 ct + lane % 32 of this wave's dZ1 tile
    f32x16_t accW2 = {};  // dW2 tile (w >> 1, w & 1)
    f32x16_t accW1[5];    // dW1 tiles w, w + 4, .., w + 16 of the 2 x 10
#pragma unroll
    for (int q = 0; q < 5; q++) accW1[q] = f32x16_t{};
    float sW3acc = 0.0f, sB3acc = 0.0f;

    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int row0 = c * BWD_ROWS;
        __syncthreads();  // the previous chunk is done with the LDS
        for (int t = tid; t < BWD_ROWS * KP / 8; t += 256) {
            const int r = t / (KP / 8);
            uint4 v = make_uint4(0, 0, 0, 0);
            if (row0 + r < m)
                v = reinterpret_cast<const uint4*>(X + (size_t)(row0 + r) * KP)[t % (KP / 8)];
            reinterpret_cast<uint4*>(sX)[t] = v;
        }
        for (int t = tid; t < BWD_ROWS * HID; t += 256) {
            const int r = t / HID;
            const bool ok = row0 + r < m;
            sH1[t] = ok ? H1[(size_t)row0 * HID + t] : (uint16_t)0;
            sH2[t] = ok ? H2[(size_t)row0 * HID + t] : (uint16_t)0;
        }
        for (int t = tid; t < BWD_ROWS * NO; t += 256)
            sdY[t] = (row0 + t / NO < m) ? dY[(size_t)row0 * NO + t] : 0.0f;
        __syncthreads();

        // dZ2 = (dY W3) * gelu'(Z2); bias gradient b2
        {
            const int col = tid & 63;
            for (int r = tid >> 6; r < BWD_ROWS; r += 4) {
                float dz = 0.0f;
                if (row0 + r < m) {
                    float dh = 0.0f;
#pragma unroll
                    for (int q = 0; q < NO; q++) dh += sdY[r * NO + q] * sW3[q * HID + col];
                    dz = dh * gelu_grad(Z2[(size_t)(row0 + r) * HID + col]);
                }
                db2 += dz;
                sdZ2[r * HID + col] = f2bf(dz);
            }
        }
        __syncthreads();

        // dH1 = dZ2 W2 (MFMA), dZ1 = dH1 * gelu'(Z1): one 32x32 tile per wave;
        // b1 sums the FP32 dZ1 values (each lane its 16 rows of the tile)
        {
            const int rt = w >> 1, ct = w & 1;
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < HID / 16; kk++) {
                const bf16x8_t av = ld8(sdZ2 + (32 * rt + (lane & 31)) * HID + 16 * kk + kh);
                const bf16x8_t bv = gather8(sW2 + (16 * kk + kh) * HID + 32 * ct + (lane & 31), HID);
                acc = mfma(av, bv, acc);
            }
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int lr = 32 * rt + acc_row(r, lane), col = 32 * ct + (lane & 31);
                float dz = 0.0f;
                if (row0 + lr < m) dz = acc[r] * gelu_grad(Z1[(size_t)(row0 + lr) * HID + col]);
                sdZ1[lr * HID + col] = f2bf(dz);
                colsum1 += dz;
            }
        }
        __syncthreads();
        // dW2[j2][j1] += sum_rows dZ2[row][j2] H1[row][j1]
        {
            const int it = w >> 1, jt = w & 1;
#pragma unroll
            for (int kk = 0; kk < BWD_ROWS / 16; kk++) {
                const bf16x8_t av = gather8(sdZ2 + (16 * kk + kh) * HID + 32 * it + (lane & 31), HID);
                const bf16x8_t bv = gather8(sH1 + (16 * kk + kh) * HID + 32 * jt + (lane & 31), HID);
                accW2 = mfma(av, bv, accW2);
            }
        }
        // dW1[j][k] += sum_rows dZ1[row][j] X[row][k]: tiles tt = w + 4 q
#pragma unroll
        for (int q = 0; q < 5; q++) {
            const int tt = w + 4 * q, it = tt / 10, kt = tt % 10;
#pragma unroll
            for (int kk = 0; kk < BWD_ROWS / 16; kk++) {
                const bf16x8_t av = gather8(sdZ1 + (16 * kk + kh) * HID + 32 * it + (lane & 31), HID);
                const bf16x8_t bv = gather8(sX + (16 * kk + kh) * KP + 32 * kt + (lane & 31), KP);
                accW1[q] = mfma(av, bv, accW1[q]);
            }
        }
        // dW3[q][j2] += sum_rows dY[row][q] H2[row][j2]; db3
        {
            const int q = tid / HID, j2 = tid % HID;  // 256 = 4 x 64
            for (int r = 0; r < BWD_ROWS; r++) sW3acc += sdY[r * NO + q] * bf2f(sH2[r * HID + j2]);
            if (tid < NO)
                for (int r = 0; r < BWD_ROWS; r++) sB3acc += sdY[r * NO + tid];
        }
    }

    // the workgroup's partial row
    __syncthreads();
    red[tid] = db2;
    {
        const int rt = w >> 1, ct = w & 1;
        red[256 + (2 * rt + (lane >> 5)) * HID + 32 * ct + (lane & 31)] = colsum1;
    }
    __syncthreads();
    if (tid < HID) {
        part[OFF_B2 + tid] = red[tid] + red[tid + 64] + red[tid + 128] + red[tid + 192];
        part[OFF_B1 + tid] = red[256 + tid] + red[256 + HID + tid] + red[256 + 2 * HID + tid] +
                             red[256 + 3 * HID + tid];
    }
    {
        const int it = w >> 1, jt = w & 1;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int j2 = 32 * it + acc_row(r, lane), j1 = 32 * jt + (lane & 31);
            part[OFF_W2 + j2 * HID + j1] = accW2[r];
        }
    }
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const int tt = w + 4 * q, it = tt / 10, kt = tt % 10;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int j = 32 * it + acc_row(r, lane), k = 32 * kt + (lane & 31);
            part[OFF_W1 + j * KP + k] = accW1[q][r];
        }
    }
    {
        const int q = tid / HID, j2 = tid % HID;
        part[OFF_W3 + q * HID + j2] = sW3acc;
        if (tid < NO) part[OFF_B3 + tid] = sB3acc;
    }
}

// Sum of the partial rows: a workgroup takes 64 parameters (one per lane),
// its four waves sum consecutive quarters of the rows in order, and the four
// quarter sums are added in order (a fixed association for a given row count).
__global__ void __launch_bounds__(256) reduce_partials(const float* __restrict__ partials, int nb,
                                                       int n, float* __restrict__ out) {
    __shared__ float q[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    const int per = (nb + 3) / 4;
    const int b0 = w * per, b1 = min(nb, b0 + per);
    float s = 0.0f;
    if (p < n)
        for (int b = b0; b < b1; b++) s += partials[(size_t)b * n + p];
    q[w][lane] = s;
    __syncthreads();
    if (w == 0 && p < n) out[p] = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
}

// ---------------------------------------------------------------------------
// Flux-divergence loss over B sampled cells; Y4 rows: x(i) | x(i-1) | y(j) |
// y(j-1), B each; the y outputs are in the exchanged frame (u, v swapped).
// The target of field q at a cell is the coarse residual
//   r_q = (c1_q - c0_q)/dt - tend_q   (restricted fine evolution minus the
// plain coarse source term), divided by scale_q; w on the lid is masked out.
// ---------------------------------------------------------------------------
struct LossArgs {
    const float* Y4;
    int B;
    const int* cells;
    const double* c0[4];
    const double* c1[4];
    const double* tend[4];
    int nx, ny, nz;
    double inv_dt;
    double inv_scale[4];
    const double *rho, *rhon;
    double inv_n;
    float* dY4;
    double* partial;
};

__global__ void __launch_bounds__(256) loss_kernel(LossArgs a) {
    __shared__ double red[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int B = a.B;
    double l = 0.0;
    if (b < B) {
        const int sw[4] = {1, 0, 2, 3};
        int cell = a.cells[b];
        // a cell outside the grid contributes nothing (its terms are masked)
        const bool valid = (unsigned)cell < (unsigned)(a.nx * a.ny * a.nz);
        if (!valid) cell = 0;
        const int k = cell % a.nz, j = (cell / a.nz) % a.ny, i = cell / (a.nz * a.ny);
        const long g = ((long)(i + 2) * (a.ny + 4) + (j + 2)) * a.nz + k;
        for (int q = 0; q < 4; q++) {
            const float yxp = a.Y4[(size_t)b * 4 + q], yxm = a.Y4[(size_t)(B + b) * 4 + q];
            const float yyp = a.Y4[(size_t)(2 * B + b) * 4 + sw[q]],
                        yym = a.Y4[(size_t)(3 * B + b) * 4 + sw[q]];
            const float rh = (float)(q == 2 ? a.rho[k] / a.rho[0] : a.rhon[k] / a.rhon[0]);
            const float tgt = (float)(((a.c1[q][g] - a.c0[q][g]) * a.inv_dt - a.tend[q][g]) *
                                      a.inv_scale[q]);
            const float msk = (!valid || (q == 2 && k == a.nz - 1)) ? 0.0f : 1.0f;
            const float c = -(yxp - yxm + yyp - yym) / rh;
            const float err = (c - tgt) * msk;
            l += (double)err * (double)err;
            const float gr = (float)(2.0 * (double)err * a.inv_n) / rh;
            a.dY4[(size_t)b * 4 + q] = -gr;
            a.dY4[(size_t)(B + b) * 4 + q] = gr;
            a.dY4[(size_t)(2 * B + b) * 4 + sw[q]] = -gr;
            a.dY4[(size_t)(3 * B + b) * 4 + sw[q]] = gr;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0] * a.inv_n;
}

__global__ void __launch_bounds__(256) loss_final(const double* __restrict__ partial, int nb,
                                                  float* __restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)red[0];
}

// ---------------------------------------------------------------------------
// Adam on the FP32 master weights, then the BF16 pack
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, float* __restrict__ m1,
                                                   float* __restrict__ m2,
                                                   const float* __restrict__ g, float lr,
                                                   float b1, float omb1, float b2, float omb2,
                                                   float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPARAM) return;
    const float gt = g[t];
    const float a = b1 * m1[t] + omb1 * gt;
    const float v = b2 * m2[t] + omb2 * gt * gt;
    m1[t] = a;
    m2[t] = v;
    p[t] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// ---------------------------------------------------------------------------
// Fused training step.  A workgroup (4 waves) takes chunks of TR_CELLS sampled
// cells; the chunk's 64 rows are the four face rows of its cells (row 16 f + c
// is face f = x(i), x(i-1), y(j), y(j-1) of cell c), so the loss of a cell sees
// all of its rows inside the workgroup.  Per chunk: the features are gathered
// from the fields into LDS, the three layers run with their activations and
// GELU derivatives kept in LDS, the loss terms and dY follow, then the
// backward pass, whose parameter-gradient sums stay in registers across the
// chunks (the dW1/dW2 MFMA tiles in their accumulators).  Every per-row value
// is the same operation on the same numbers as in features_kernel,
// mlp_forward, loss_kernel and mlp_backward; only the order in which rows are
// summed into the gradient differs.  One partial gradient row and one loss
// partial per workgroup; the grid depends only on the batch size, so the
// result is repeatable bit for bit.
// ---------------------------------------------------------------------------
constexpr int TR_CELLS = 16, TR_ROWS = 4 * TR_CELLS;
constexpr int TR_GRID = 256;
constexpr int LX = KP + 8;  // padded feature row in LDS (see LW1)
constexpr size_t TR_SX = (size_t)S_WEND * 2;                     // X [64][LX] bf16
constexpr size_t TR_SH1 = TR_SX + (size_t)TR_ROWS * LX * 2;      // H1 [64][LWH] bf16
constexpr size_t TR_SH2 = TR_SH1 + (size_t)TR_ROWS * LWH * 2;    // H2, then dZ2 [64][LWH] bf16
constexpr size_t TR_SG1 = TR_SH2 + (size_t)TR_ROWS * LWH * 2;    // gelu'(Z1) [64][64] f32
constexpr size_t TR_SG2 = TR_SG1 + (size_t)TR_ROWS * HID * 4;    // gelu'(Z2) [64][64] f32
constexpr size_t TR_SDZ1 = TR_SG2 + (size_t)TR_ROWS * HID * 4;   // dZ1 [64][64] bf16
constexpr size_t TR_SY = TR_SDZ1 + (size_t)TR_ROWS * HID * 2;    // Y [64][4] f32
constexpr size_t TR_SDY = TR_SY + (size_t)TR_ROWS * NO * 4;      // dY [64][4] f32
constexpr size_t TR_SW3 = TR_SDY + (size_t)TR_ROWS * NO * 4;     // W3 (bf16 values) [4][64] f32
constexpr size_t TR_SB = TR_SW3 + (size_t)NO * HID * 4;          // b1 | b2 | b3 f32
constexpr size_t TR_LDS = TR_SB + (size_t)(2 * HID + NO) * 4;
static_assert(TR_LDS <= 160 * 1024, "fused training step fits the LDS");
static_assert(TR_ROWS * LX * 2 >= 2 * 256 * 4, "end-of-kernel sums fit the feature area");

int train_grid(int b) {
    const int chunks = (b + TR_CELLS - 1) / TR_CELLS;
    return chunks < TR_GRID ? chunks : TR_GRID;
}

struct TrainArgs {
    const double* c0[4];
    const double* c1[4];
    const double* tend[4];
    double mean[4], inv_std[4];
    int nx, ny, nz;
    const int* cells;
    int B;
    double inv_dt;
    double inv_scale[4];
    const double *rho, *rhon;
    double inv_n;
    const float* params;
    const uint16_t* wpack;
    float* partials;      // [grid][NPARAM]
    double* loss_part;    // [grid]
};

template <typename P>
__device__ __forceinline__ P pick4(int q, P a0, P a1, P a2, P a3) {
    return q == 0 ? a0 : (q == 1 ? a1 : (q == 2 ? a2 : a3));
}

__global__ void __launch_bounds__(256) mlp_train(TrainArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* sw = reinterpret_cast<uint16_t*>(smem);
    uint16_t* sX = reinterpret_cast<uint16_t*>(smem + TR_SX);
    uint16_t* sH1 = reinterpret_cast<uint16_t*>(smem + TR_SH1);
    uint16_t* sH2 = reinterpret_cast<uint16_t*>(smem + TR_SH2);  // later dZ2
    float* sG1 = reinterpret_cast<float*>(smem + TR_SG1);
    float* sG2 = reinterpret_cast<float*>(smem + TR_SG2);
    uint16_t* sdZ1 = reinterpret_cast<uint16_t*>(smem + TR_SDZ1);
    float* sY = reinterpret_cast<float*>(smem + TR_SY);
    float* sdY = reinterpret_cast<float*>(smem + TR_SDY);
    float* sW3 = reinterpret_cast<float*>(smem + TR_SW3);
    float* sb = reinterpret_cast<float*>(smem + TR_SB);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int h = lane >> 5, kh = 8 * h;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned ncell = (unsigned)nx * ny * nz;
    const int nchunks = (a.B + TR_CELLS - 1) / TR_CELLS;

    load_pack_padded(a.wpack, sw);
    for (int t = tid; t < 2 * HID + NO; t += 256)
        sb[t] = t < HID ? a.params[OFF_B1 + t]
                        : (t < 2 * HID ? a.params[OFF_B2 + t - HID] : a.params[OFF_B3 + t - 2 * HID]);
    for (int t = tid; t < NO * HID; t += 256) sW3[t] = bf2f(a.wpack[PK_W3 + t]);

    // sums kept across the chunks
    float db2 = 0.0f;      // column tid % 64, rows tid/64 + 4q
    float colsum1 = 0.0f;  // b1: column 32 ct + lane % 32 of this wave's dZ1 tile
    f32x16_t accW2 = {};   // dW2 tile (w >> 1, w & 1)
    f32x16_t accW1[5];     // dW1 tiles w, w + 4, .., w + 16 of the 2 x 10
#pragma unroll
    for (int q = 0; q < 5; q++) accW1[q] = f32x16_t{};
    float sW3acc = 0.0f, sB3acc = 0.0f;
    double lsum = 0.0;     // squared errors (wave 0)
    const int rt = w >> 1, ct = w & 1;  // this wave's 32 x 32 output tile

    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        __syncthreads();  // the previous chunk is done with the LDS (and the weights are in)

        // ---- features: lane = row, wave = feature field ----
        {
            const int r = lane, face = r >> 4, b = c * TR_CELLS + (r & 15);
            int cell = b < a.B ? a.cells[b] : -1;
            const bool valid = (unsigned)cell < ncell;
            if (!valid) cell = 0;  // gathers in bounds, values masked
            const int k = cell % nz, ij = cell / nz;
            int j = ij % ny, i = ij / ny;
            if (face == 1) i = i == 0 ? nx - 1 : i - 1;
            if (face == 3) j = j == 0 ? ny - 1 : j - 1;
            const bool orient = face >= 2;
            // the stored field of feature field w (y-face rows exchange u, v)
            const int src = orient && w < 2 ? 1 - w : w;
            const double* fld = pick4(src, a.c0[0], a.c0[1], a.c0[2], a.c0[3]);
            const double mean = pick4(src, a.mean[0], a.mean[1], a.mean[2], a.mean[3]);
            const double inv = pick4(src, a.inv_std[0], a.inv_std[1], a.inv_std[2], a.inv_std[3]);
            long ao[5], bo[5];
            int ko[3];
#pragma unroll
            for (int d = 0; d < 5; d++) {
                int ii = i + d - 2, jj = j + d - 2;  // offsets of at most 2 cells: wrap by adds
                ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
                ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
                jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
                jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
                const long xoff = (long)(ii + 2) * (ny + 4) * nz, yoff = (long)(jj + 2) * nz;
                ao[d] = orient ? yoff : xoff;  // first neighbourhood axis
                bo[d] = orient ? xoff : yoff;  // second
            }
#pragma unroll
            for (int e = 0; e < 3; e++) {
                const int kk = k + e - 1;
                ko[e] = kk < 0 ? 0 : (kk > nz - 1 ? nz - 1 : kk);
            }
            uint16_t* dst = sX + r * LX + w * 80;
#pragma unroll
            for (int g8 = 0; g8 < 10; g8++) {
                u16x8 v;
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int pos = 8 * g8 + e;
                    uint16_t out = 0;
                    if (pos < 75) {
                        const int a5 = pos / 15, b5 = (pos / 3) % 5, c3 = pos % 3;
                        const double x = fld[ao[a5] + bo[b5] + ko[c3]];
                        out = valid ? f2bf((float)((x - mean) * inv)) : (uint16_t)0;
                    }
                    v.v[e] = out;
                }
                *reinterpret_cast<uint4*>(dst + 8 * g8) = __builtin_bit_cast(uint4, v);
            }
        }
        __syncthreads();

        // ---- layer 1: Z1 = X W1^T + b1 ----
        {
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < KP / 16; kk++) {
                const int ks = kslot(kk, h);
                acc = mfma(ld8(sX + (32 * rt + (lane & 31)) * LX + ks),
                           ld8(sw + S_W1 + (32 * ct + (lane & 31)) * LW1 + ks), acc);
            }
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int lr = 32 * rt + acc_row(r, lane), col = 32 * ct + (lane & 31);
                const float z = acc[r] + sb[col];
                sH1[lr * LWH + col] = f2bf(gelu(z));
                sG1[lr * HID + col] = gelu_grad(z);
            }
        }
        __syncthreads();
        // ---- layer 2 ----
        {
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < HID / 16; kk++)
                acc = mfma(ld8(sH1 + (32 * rt + (lane & 31)) * LWH + 16 * kk + kh),
                           ld8(sw + S_W2 + (32 * ct + (lane & 31)) * LWH + 16 * kk + kh), acc);
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int lr = 32 * rt + acc_row(r, lane), col = 32 * ct + (lane & 31);
                const float z = acc[r] + sb[HID + col];
                sH2[lr * LWH + col] = f2bf(gelu(z));
                sG2[lr * HID + col] = gelu_grad(z);
            }
        }
        __syncthreads();
        // ---- layer 3 (4 outputs, padded to a 32-wide tile): waves 0, 1 ----
        if (w < 2) {
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < HID / 16; kk++)
                acc = mfma(ld8(sH2 + (32 * w + (lane & 31)) * LWH + 16 * kk + kh),
                           ld8(sw + S_W3 + (lane & 31) * LWH + 16 * kk + kh), acc);
            const int col = lane & 31;
            if (col < NO) {
#pragma unroll
                for (int r = 0; r < 16; r++)
                    sY[(32 * w + acc_row(r, lane)) * NO + col] = acc[r] + sb[2 * HID + col];
            }
        }
        __syncthreads();
        // ---- loss terms and dY: wave 0, lane = (cell, field) ----
        if (w == 0) {
            const int cl = lane >> 2, q = lane & 3, sq = q < 2 ? 1 - q : q;
            const int b = c * TR_CELLS + cl;
            int cell = b < a.B ? a.cells[b] : -1;
            const bool valid = (unsigned)cell < ncell;
            if (!valid) cell = 0;
            const int k = cell % nz, j = (cell / nz) % ny, i = cell / (nz * ny);
            const long g = ((long)(i + 2) * (ny + 4) + (j + 2)) * nz + k;
            const float yxp = sY[cl * NO + q], yxm = sY[(TR_CELLS + cl) * NO + q];
            const float yyp = sY[(2 * TR_CELLS + cl) * NO + sq],
                        yym = sY[(3 * TR_CELLS + cl) * NO + sq];
            const float rh = (float)(q == 2 ? a.rho[k] / a.rho[0] : a.rhon[k] / a.rhon[0]);
            const double* f0 = pick4(q, a.c0[0], a.c0[1], a.c0[2], a.c0[3]);
            const double* f1 = pick4(q, a.c1[0], a.c1[1], a.c1[2], a.c1[3]);
            const double* ft = pick4(q, a.tend[0], a.tend[1], a.tend[2], a.tend[3]);
            const double isc = pick4(q, a.inv_scale[0], a.inv_scale[1], a.inv_scale[2],
                                     a.inv_scale[3]);
            const float tgt = (float)(((f1[g] - f0[g]) * a.inv_dt - ft[g]) * isc);
            const float msk = (!valid || (q == 2 && k == nz - 1)) ? 0.0f : 1.0f;
            const float cc = -(yxp - yxm + yyp - yym) / rh;
            const float err = (cc - tgt) * msk;
            lsum += (double)err * (double)err;
            const float gr = (float)(2.0 * (double)err * a.inv_n) / rh;
            sdY[cl * NO + q] = -gr;
            sdY[(TR_CELLS + cl) * NO + q] = gr;
            sdY[(2 * TR_CELLS + cl) * NO + sq] = -gr;
            sdY[(3 * TR_CELLS + cl) * NO + sq] = gr;
        }
        __syncthreads();

        // ---- backward ----
        // dW3[q][j2] += sum_rows dY[row][q] H2[row][j2]; db3
        {
            const int q = tid / HID, j2 = tid % HID;  // 256 = 4 x 64
            for (int r = 0; r < TR_ROWS; r++) sW3acc += sdY[r * NO + q] * bf2f(sH2[r * LWH + j2]);
            if (tid < NO)
                for (int r = 0; r < TR_ROWS; r++) sB3acc += sdY[r * NO + tid];
        }
        // dZ2 = (dY W3) * gelu'(Z2), kept in registers until H2 is no longer read
        float dz2[TR_ROWS / 4];
        {
            const int col = tid & 63;
#pragma unroll
            for (int q4 = 0; q4 < TR_ROWS / 4; q4++) {
                const int r = (tid >> 6) + 4 * q4;
                float dh = 0.0f;
#pragma unroll
                for (int q = 0; q < NO; q++) dh += sdY[r * NO + q] * sW3[q * HID + col];
                const float dz = dh * sG2[r * HID + col];
                db2 += dz;
                dz2[q4] = dz;
            }
        }
        __syncthreads();
        uint16_t* sdZ2 = sH2;
        {
            const int col = tid & 63;
#pragma unroll
            for (int q4 = 0; q4 < TR_ROWS / 4; q4++)
                sdZ2[((tid >> 6) + 4 * q4) * LWH + col] = f2bf(dz2[q4]);
        }
        __syncthreads();
        // dH1 = dZ2 W2 (MFMA), dZ1 = dH1 * gelu'(Z1); b1 sums the FP32 dZ1
        {
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < HID / 16; kk++)
                acc = mfma(ld8(sdZ2 + (32 * rt + (lane & 31)) * LWH + 16 * kk + kh),
                           gather8(sw + S_W2 + (16 * kk + kh) * LWH + 32 * ct + (lane & 31), LWH),
                           acc);
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int lr = 32 * rt + acc_row(r, lane), col = 32 * ct + (lane & 31);
                const float dz = acc[r] * sG1[lr * HID + col];
                sdZ1[lr * HID + col] = f2bf(dz);
                colsum1 += dz;
            }
        }
        __syncthreads();
        // dW2[j2][j1] += sum_rows dZ2[row][j2] H1[row][j1]
#pragma unroll
        for (int kk = 0; kk < TR_ROWS / 16; kk++)
            accW2 = mfma(gather8(sdZ2 + (16 * kk + kh) * LWH + 32 * rt + (lane & 31), LWH),
                         gather8(sH1 + (16 * kk + kh) * LWH + 32 * ct + (lane & 31), LWH), accW2);
        // dW1[j][k] += sum_rows dZ1[row][j] X[row][k]: tiles tt = w + 4 q
#pragma unroll
        for (int q = 0; q < 5; q++) {
            const int tt = w + 4 * q, it = tt / 10, kt = tt % 10;
#pragma unroll
            for (int kk = 0; kk < TR_ROWS / 16; kk++)
                accW1[q] = mfma(gather8(sdZ1 + (16 * kk + kh) * HID + 32 * it + (lane & 31), HID),
                                gather8(sX + (16 * kk + kh) * LX + 32 * kt + (lane & 31), LX),
                                accW1[q]);
        }
    }

    // ---- the workgroup's partial row and loss ----
    float* part = a.partials + (size_t)blockIdx.x * NPARAM;
    __syncthreads();
    float* red = reinterpret_cast<float*>(smem + TR_SX);  // [2][256]
    red[tid] = db2;
    red[256 + (2 * rt + (lane >> 5)) * HID + 32 * ct + (lane & 31)] = colsum1;
    __syncthreads();
    if (tid < HID) {
        part[OFF_B2 + tid] = red[tid] + red[tid + 64] + red[tid + 128] + red[tid + 192];
        part[OFF_B1 + tid] = red[256 + tid] + red[256 + HID + tid] + red[256 + 2 * HID + tid] +
                             red[256 + 3 * HID + tid];
    }
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int j2 = 32 * rt + acc_row(r, lane), j1 = 32 * ct + (lane & 31);
        part[OFF_W2 + j2 * HID + j1] = accW2[r];
    }
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const int tt = w + 4 * q, it = tt / 10, kt = tt % 10;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int j = 32 * it + acc_row(r, lane), k = 32 * kt + (lane & 31);
            part[OFF_W1 + j * KP + k] = accW1[q][r];
        }
    }
    {
        const int q = tid / HID, j2 = tid % HID;
        part[OFF_W3 + q * HID + j2] = sW3acc;
        if (tid < NO) part[OFF_B3 + tid] = sB3acc;
    }
    if (w == 0) {
        double v = lsum;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) a.loss_part[blockIdx.x] = v * a.inv_n;
    }
}

// The update after mlp_train: a workgroup of 16 waves takes 64 parameters;
// wave g sums rows g*per .. g*per + per - 1 of their partial rows in order (all
// its loads in flight at once: the sum is bound by latency, not bytes), then
// wave 0 adds the 16 group sums in order, writes the gradient, takes the Adam
// step and writes the BF16 pack entries of the weights; workgroup 0 also sums
// the loss partials.
constexpr int UPD_GROUPS = 16;
constexpr int UPD_PER_MAX = TR_GRID / UPD_GROUPS;
static_assert(TR_GRID % UPD_GROUPS == 0 && TR_GRID <= 256, "row groups");

struct UpdateArgs {
    const float* partials;
    int nb;
    const double* loss_part;
    float* grad;
    float* p;
    float* m1;
    float* m2;
    uint16_t* wpack;
    float* loss;
    float lr, b1, omb1, b2, omb2, eps, c1, c2;
};

__global__ void __launch_bounds__(64 * UPD_GROUPS) mlp_update(UpdateArgs a) {
    __shared__ float qs[UPD_GROUPS][64];
    __shared__ double red[256];
    const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    const int p = blockIdx.x * 64 + lane;
    const int per = (a.nb + UPD_GROUPS - 1) / UPD_GROUPS;
    const int r0 = grp * per;
    float v[UPD_PER_MAX];
#pragma unroll
    for (int e = 0; e < UPD_PER_MAX; e++) {
        const int r = r0 + e;
        v[e] = (e < per && r < a.nb && p < NPARAM) ? a.partials[(size_t)r * NPARAM + p] : 0.0f;
    }
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < UPD_PER_MAX; e++) s += v[e];  // rows in order; absent rows add 0
    qs[grp][lane] = s;
    if (blockIdx.x == 0 && tid < 256) {
        double l = 0.0;
        for (int r = tid; r < a.nb; r += 256) l += a.loss_part[r];
        red[tid] = l;
    }
    __syncthreads();
    if (grp == 0 && p < NPARAM) {
        float gt = qs[0][lane];
#pragma unroll
        for (int g = 1; g < UPD_GROUPS; g++) gt += qs[g][lane];
        a.grad[p] = gt;
        const float m = a.b1 * a.m1[p] + a.omb1 * gt;
        const float v2 = a.b2 * a.m2[p] + a.omb2 * gt * gt;
        a.m1[p] = m;
        a.m2[p] = v2;
        const float np = a.p[p] - a.lr * (m / a.c1) / (sqrtf(v2 / a.c2) + a.eps);
        a.p[p] = np;
        int pk = -1;  // the pack entry of a weight (biases are not packed)
        if (p < OFF_B1) pk = PK_W1 + p;
        else if (p >= OFF_W2 && p < OFF_B2) pk = PK_W2 + (p - OFF_W2);
        else if (p >= OFF_W3 && p < OFF_B3) pk = PK_W3 + (p - OFF_W3);
        if (pk >= 0) a.wpack[pk] = f2bf(np);
    }
    if (blockIdx.x == 0) {
        for (int q = 128; q > 0; q >>= 1) {
            if (tid < q) red[tid] += red[tid + q];
            __syncthreads();
        }
        if (tid == 0) a.loss[0] = (float)red[0];
    }
}

// ---------------------------------------------------------------------------
// Corrected coarse step: state_out = state_in + dt (tend + c), with c the flux
// divergence of the network's face fluxes (times the per-field scale).
// Guards, in order:
//  * any non-finite face flux: the whole step is the plain one (flags bit 1);
//  * theta: each lateral face's corrected flux is clamped so that the corrected
//    face value stays in the ULTIMATE admissible interval of that face (the
//    interval between the upwind value and the monotone bound, Sec. 3.1's
//    positivity-preserving scheme), which keeps the 1-D update bounded;
//  * growth: if the corrected state's kinetic energy or theta variance exceeds
//    `growth` times the plain step's, the whole step is the plain one (bit 2).
// ---------------------------------------------------------------------------
// The corrected step is computed unconditionally; the thread of a cell also
// checks that cell's face outputs and sets bit 1 of flags[0] if one is not
// finite, and corr_decide then makes the whole step the plain one.
// partial sums: KE corrected, KE plain, m th^2 and m th corrected, the same
// plain, the mass m, and the clamped theta faces (added to flags[3] unless
// the step falls back for non-finite outputs)
constexpr int CORR_NSUM = 8;

struct CorrArgs {
    const double* in[4];
    const double* tend[4];
    double* out[4];
    const float* gx;
    const float* gy;
    int nx, ny, nz;
    double dx, dy, dt;
    double rdx, rdy, dt_dx, dt_dy;  // 1/dx, 1/dy, dt/dx, dt/dy
    double scale[4];
    const double *rdz, *rho, *rhon;
    int* flags;
    double* partial;  // [nblocks][CORR_NSUM]
    double growth;
};

__global__ void __launch_bounds__(256) corr_clear(int* flags) {
    if (threadIdx.x == 0) flags[0] = 0;
}

// ULTIMATE-limited QUICKEST value of a face and its admissible interval
// [lo, hi], from the far-upwind, upwind and downwind values and the Courant
// number c in [0, 1].  At a local extremum only the upwind value is admissible.
__device__ __forceinline__ void ult_interval(double pU, double pC, double pD, double c,
                                             double& f, double& lo, double& hi) {
    const double del = pD - pU, kap = pD - 2.0 * pC + pU;
    if (fabs(kap) >= fabs(del)) {
        f = lo = hi = pC;
        return;
    }
    const double quick = 0.5 * (pC + pD) - 0.5 * c * (pD - pC) - (1.0 - c * c) / 6.0 * kap;
    const double bnd = c > 0.0 ? pU + (pC - pU) / c : pD;
    if (del > 0.0) {
        lo = pC;
        hi = fmin(pD, bnd);
    } else {
        lo = fmax(pD, bnd);
        hi = pC;
    }
    f = fmin(fmax(quick, lo), hi);
}

// The theta correction flux through one lateral face after the clamp.  a: the
// normal velocity on the face; p[0..3]: theta at the cells -1, 0, +1, +2
// relative to the face's left cell; G: the unclamped correction flux (physical
// flux units, rhon * velocity * theta).  Returns the admissible part of G.
__device__ __forceinline__ double clamp_face(double a, const double* p, double dt_over_h,
                                             double mass, double G, bool& clamped) {
    double f, lo, hi;
    const double c = fabs(a) * dt_over_h;
    if (a >= 0.0)
        ult_interval(p[0], p[1], p[2], c, f, lo, hi);
    else
        ult_interval(p[3], p[2], p[1], c, f, lo, hi);
    const double F = mass * a * f;
    const double F1 = mass * a * lo, F2 = mass * a * hi;
    const double Fmin = fmin(F1, F2), Fmax = fmax(F1, F2);
    const double Fc = fmin(fmax(F + G, Fmin), Fmax);
    clamped = Fc != F + G;
    return Fc - F;
}

// Per-level factors of the corrected step: mass rhon dz, w mass rho dz (0 on
// the lid), the inverse density ratios of the correction, 1/rhon.
enum { CL_M, CL_MW, CL_RHN, CL_RHW, CL_RMK, CL_N };

__global__ void __launch_bounds__(256) corr_step(CorrArgs a) {
    __shared__ double lev[CL_N][MONC_MAX_NZ];
    __shared__ double red[4][CORR_NSUM];
    const long n = (long)a.nx * a.ny * a.nz;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        lev[CL_M][k] = a.rhon[k] / a.rdz[k];
        lev[CL_MW][k] = k < nz - 1 ? a.rho[k] / a.rdz[k] : 0.0;
        lev[CL_RHN][k] = a.rhon[0] / a.rhon[k];
        lev[CL_RHW][k] = a.rho[0] / a.rho[k];
        lev[CL_RMK][k] = 1.0 / a.rhon[k];
    }
    __syncthreads();
    double sum[CORR_NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (t < n) {
        const int k = (int)(t % nz), j = (int)((t / nz) % ny), i = (int)(t / ((long)nz * ny));
        const int im = i == 0 ? nx - 1 : i - 1, jm = j == 0 ? ny - 1 : j - 1;
        const long cm_x = ((long)im * ny + j) * nz + k, cm_y = ((long)i * ny + jm) * nz + k;
        const long sx = (long)(ny + 4) * nz;
        const long g = (long)(i + 2) * sx + (long)(j + 2) * nz + k;
        const double m = lev[CL_M][k], mw = lev[CL_MW][k];
        // this cell's face outputs, each checked once (by its cell's thread)
        const float4 gxc = reinterpret_cast<const float4*>(a.gx)[t];
        const float4 gyc = reinterpret_cast<const float4*>(a.gy)[t];
        const float4 gxm = reinterpret_cast<const float4*>(a.gx)[cm_x];
        const float4 gym = reinterpret_cast<const float4*>(a.gy)[cm_y];
        const bool bad = !(isfinite(gxc.x) && isfinite(gxc.y) && isfinite(gxc.z) &&
                           isfinite(gxc.w) && isfinite(gyc.x) && isfinite(gyc.y) &&
                           isfinite(gyc.z) && isfinite(gyc.w));
        if (bad) atomicOr(a.flags, 1);
        double cq[4];
        {
            // y outputs are in the exchanged frame: u and v swapped
            const double gxq[3] = {gxc.x, gxc.y, gxc.z}, gxmq[3] = {gxm.x, gxm.y, gxm.z};
            const double gyq[3] = {gyc.y, gyc.x, gyc.z}, gymq[3] = {gym.y, gym.x, gym.z};
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const double rhi = q == 2 ? lev[CL_RHW][k] : lev[CL_RHN][k];
                const double div = gxq[q] - gxmq[q] + gyq[q] - gymq[q];
                cq[q] = -a.scale[q] * div * rhi;
            }
        }
        {
            // theta: clamped face fluxes; G = h rhon(0) S g for a face of width h
            const double* th = a.in[3];
            const double* u = a.in[0];
            const double* v = a.in[1];
            const double mk = a.rhon[k];
            const double cx = a.dx * a.rhon[0] * a.scale[3], cy = a.dy * a.rhon[0] * a.scale[3];
            auto wx = [&](int ii) { ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii); return ii; };
            auto wy = [&](int jj) { jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj); return jj; };
            auto at = [&](const double* f, int ii, int jj) {
                return f[(long)(ii + 2) * sx + (long)(jj + 2) * nz + k];
            };
            // theta at offsets -2 .. +2 along x and y; a face's four cells
            // (-1, 0, +1, +2 from its left cell) start at index 1 for the face
            // i+1/2 (left cell i) and at index 0 for i-1/2 (left cell i-1)
            double px[5], py[5];
#pragma unroll
            for (int o = 0; o < 5; o++) {
                px[o] = at(th, wx(i - 2 + o), j);
                py[o] = at(th, i, wy(j - 2 + o));
            }
            bool c1, c2, c3, c4;
            const double Gxp = clamp_face(at(u, i, j), px + 1, a.dt_dx, mk, cx * (double)gxc.w, c1);
            const double Gxm = clamp_face(at(u, im, j), px, a.dt_dx, mk, cx * (double)gxm.w, c2);
            const double Gyp = clamp_face(at(v, i, j), py + 1, a.dt_dy, mk, cy * (double)gyc.w, c3);
            const double Gym = clamp_face(at(v, i, jm), py, a.dt_dy, mk, cy * (double)gym.w, c4);
            cq[3] = -((Gxp - Gxm) * a.rdx + (Gyp - Gym) * a.rdy) * lev[CL_RMK][k];
            sum[7] = (double)((int)c1 + (int)c3);  // faces i+1/2 and j+1/2 belong to this cell
        }
        double o[4], pl[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const double in = a.in[q][g], td = a.tend[q][g];
            pl[q] = in + a.dt * td;
            o[q] = in + a.dt * (td + cq[q]);
            if (q == 2 && k == nz - 1) o[q] = pl[q] = 0.0;
            a.out[q][g] = o[q];
        }
        sum[0] = m * (o[0] * o[0] + o[1] * o[1]) + mw * o[2] * o[2];
        sum[1] = m * (pl[0] * pl[0] + pl[1] * pl[1]) + mw * pl[2] * pl[2];
        sum[2] = m * o[3] * o[3];
        sum[3] = m * o[3];
        sum[4] = m * pl[3] * pl[3];
        sum[5] = m * pl[3];
        sum[6] = m;
    }
    // fixed-order workgroup sums: each wave by shuffles, then the four waves
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < CORR_NSUM; q++) {
        double v = sum[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[w][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < CORR_NSUM) {
        const int q = threadIdx.x;
        a.partial[(long)blockIdx.x * CORR_NSUM + q] =
            ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    }
}

// Sums the block partials in a fixed order and takes the step's decision:
// flags[1] counts non-finite fallbacks, flags[2] growth fallbacks, flags[3]
// the clamped theta faces of the steps that keep their correction; bit 2 of
// flags[0] tells corr_revert to write the plain step.
__global__ void __launch_bounds__(256) corr_decide(const double* __restrict__ partial, int nb,
                                                   double growth, int* flags) {
    __shared__ double red[CORR_NSUM][256];
    double s[CORR_NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int q = 0; q < CORR_NSUM; q++) s[q] += partial[(long)b * CORR_NSUM + q];
    for (int q = 0; q < CORR_NSUM; q++) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int q = 0; q < CORR_NSUM; q++) red[q][threadIdx.x] += red[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (flags[0] & 1) {
            flags[0] |= 2;
            flags[1] += 1;
            return;
        }
        flags[3] += (int)red[7][0];
        const double ke_c = red[0][0], ke_p = red[1][0], mass = red[6][0];
        const double var_c = red[2][0] / mass - (red[3][0] / mass) * (red[3][0] / mass);
        const double var_p = red[4][0] / mass - (red[5][0] / mass) * (red[5][0] / mass);
        if (!(ke_c <= growth * ke_p) || !(var_c <= growth * var_p)) {
            flags[0] |= 2;
            flags[2] += 1;
        }
    }
}

__global__ void __launch_bounds__(256) corr_revert(CorrArgs a) {
    if ((a.flags[0] & 2) == 0) return;
    const long n = (long)a.nx * a.ny * a.nz;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int k = (int)(t % a.nz), j = (int)((t / a.nz) % a.ny), i = (int)(t / ((long)a.nz * a.ny));
    const long g = ((long)(i + 2) * (a.ny + 4) + (j + 2)) * a.nz + k;
    for (int q = 0; q < 4; q++) {
        double v = a.in[q][g] + a.dt * a.tend[q][g];
        if (q == 2 && k == a.nz - 1) v = 0.0;
        a.out[q][g] = v;
    }
}

int blocks_for(long n) { return (int)((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_restrict4(int nscal, const double* const* fine, double* const* coarse, int nx,
                            int ny, int nz, const double* rdz, const double* rho,
                            const double* rhon, double* rdz_c, double* rho_c, double* rhon_c,
                            hipStream_t s) {
    RestrictArgs a;
    for (int f = 0; f < 3 + nscal; f++) {
        a.fine[f] = fine[f];
        a.coarse[f] = coarse[f];
    }
    a.nscal = nscal;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.rdz = rdz;
    a.rho = rho;
    a.rhon = rhon;
    a.rdz_c = rdz_c;
    a.rho_c = rho_c;
    a.rhon_c = rhon_c;
    restrict_profiles<<<1, 256, 0, s>>>(a);
    restrict_fields<<<blocks_for((long)(nx / 4) * (ny / 4) * (nz / 4)), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_features(const double* const* state, int nx, int ny, int nz, const double* norm,
                           int orient, const int* cells, long ncells, uint16_t* X, hipStream_t s) {
    FeatArgs a;
    for (int f = 0; f < 4; f++) {
        a.f[f] = state[f];
        a.mean[f] = norm[2 * f];
        a.inv_std[f] = 1.0 / norm[2 * f + 1];
    }
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.orient = orient;
    a.cells = cells;
    a.ncells = ncells;
    a.X = X;
    features_kernel<<<blocks_for(ncells * (KP / 8)), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float* params, uint16_t* wpack, hipStream_t s) {
    pack_kernel<<<blocks_for(PK_SIZE), 256, 0, s>>>(params, wpack);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t* X, int m, const float* params,
                              const uint16_t* wpack, float* Y, uint16_t* H1, uint16_t* H2,
                              float* Z1, float* Z2, hipStream_t s) {
    static std::atomic<unsigned long long> attr{0};
    hipError_t e = set_lds_limit_once((const void*)mlp_forward, FWD_LDS, &attr);
    if (e != hipSuccess) return e;
    mlp_forward<<<(m + FWD_ROWS - 1) / FWD_ROWS, 256, FWD_LDS, s>>>(X, m, params, wpack, Y, H1, H2,
                                                                    Z1, Z2);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const double* const* state, int nx, int ny, int nz,
                           const double* norm, int orient, const float* params,
                           const uint16_t* wpack, float* Y, hipStream_t s) {
    const bool staged = infer_staged_ok(ny, nz);
    if (orient == 2 && !staged) {
        // no staged tile to share: one launch per orientation
        hipError_t e = launch_mlp_infer(state, nx, ny, nz, norm, 0, params, wpack, Y, s);
        if (e != hipSuccess) return e;
        return launch_mlp_infer(state, nx, ny, nz, norm, 1, params, wpack,
                                Y + (size_t)nx * ny * nz * NO, s);
    }
    static std::atomic<unsigned long long> attr[2][3] = {{{0}, {0}, {0}}, {{0}, {0}, {0}}};
    const void* kern = staged ? (orient == 2 ? (const void*)mlp_infer<2, true>
                                 : orient ? (const void*)mlp_infer<1, true>
                                          : (const void*)mlp_infer<0, true>)
                              : (orient ? (const void*)mlp_infer<1, false>
                                        : (const void*)mlp_infer<0, false>);
    hipError_t e = set_lds_limit_once(kern, FWD_LDS, &attr[staged ? 1 : 0][orient]);
    if (e != hipSuccess) return e;
    // the current device's compute units (devices may differ)
    int dev = 0, ncu = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    InferArgs a;
    for (int f = 0; f < 4; f++) {
        a.f[f] = state[f];
        a.mean[f] = norm[2 * f];
        a.inv_std[f] = 1.0 / norm[2 * f + 1];
    }
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.m = (long)nx * ny * nz;
    a.params = params;
    a.wpack = wpack;
    a.Y = Y;
    const long ntiles = (a.m + FWD_ROWS - 1) / FWD_ROWS;
    const int grid = (int)(ntiles < 2L * ncu ? ntiles : 2L * ncu);
    if (staged) {
        if (orient == 2)
            mlp_infer<2, true><<<grid, 256, FWD_LDS, s>>>(a);
        else if (orient)
            mlp_infer<1, true><<<grid, 256, FWD_LDS, s>>>(a);
        else
            mlp_infer<0, true><<<grid, 256, FWD_LDS, s>>>(a);
    } else {
        if (orient)
            mlp_infer<1, false><<<grid, 256, FWD_LDS, s>>>(a);
        else
            mlp_infer<0, false><<<grid, 256, FWD_LDS, s>>>(a);
    }
    return hipGetLastError();
}

size_t mlp_backward_workspace(int m) { return (size_t)bwd_grid(m) * NPARAM * sizeof(float); }

hipError_t launch_mlp_backward(const uint16_t* X, const uint16_t* H1, const uint16_t* H2,
                               const float* Z1, const float* Z2, const float* dY, int m,
                               const uint16_t* wpack, float* grad, void* ws, hipStream_t s) {
    static std::atomic<unsigned long long> attr{0};
    hipError_t e = set_lds_limit_once((const void*)mlp_backward, BWD_LDS, &attr);
    if (e != hipSuccess) return e;
    const int nb = bwd_grid(m);
    mlp_backward<<<nb, 256, BWD_LDS, s>>>(X, H1, H2, Z1, Z2, dY, m, wpack, (float*)ws);
    reduce_partials<<<(NPARAM + 63) / 64, 256, 0, s>>>((const float*)ws, nb, NPARAM, grad);
    return hipGetLastError();
}

size_t mlp_loss_workspace(int b) { return (size_t)((b + 255) / 256) * sizeof(double); }

hipError_t launch_mlp_loss(const float* Y4, int b, const int* cells, const double* const* c0,
                           const double* const* c1, const double* const* tend, int nx, int ny,
                           int nz, double dt, const double* scale, const double* rho,
                           const double* rhon, double inv_n, float* dY4, float* loss, void* ws,
                           hipStream_t s) {
    LossArgs a;
    a.Y4 = Y4;
    a.B = b;
    a.cells = cells;
    for (int q = 0; q < 4; q++) {
        a.c0[q] = c0[q];
        a.c1[q] = c1[q];
        a.tend[q] = tend[q];
        a.inv_scale[q] = 1.0 / scale[q];
    }
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.inv_dt = 1.0 / dt;
    a.rho = rho;
    a.rhon = rhon;
    a.inv_n = inv_n;
    a.dY4 = dY4;
    a.partial = (double*)ws;
    const int nb = (b + 255) / 256;
    loss_kernel<<<nb, 256, 0, s>>>(a);
    loss_final<<<1, 256, 0, s>>>((const double*)ws, nb, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m1, float* m2, const float* grad, int t,
                           double lr, double b1, double b2, double eps, uint16_t* wpack,
                           hipStream_t s) {
    const float c1 = (float)(1.0 - pow(b1, t)), c2 = (float)(1.0 - pow(b2, t));
    // 1 - beta in FP64 before rounding: 1.0f - 0.999f is 1.3e-5 away from 0.001 in
    // relative terms, far more than the FP32 rounding of 0.001 itself.
    adam_kernel<<<blocks_for(NPARAM), 256, 0, s>>>(params, m1, m2, grad, (float)lr, (float)b1,
                                                  (float)(1.0 - b1), (float)b2, (float)(1.0 - b2),
                                                  (float)eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_mlp_pack(params, wpack, s);
}

size_t mlp_train_workspace(int b) {
    const size_t g = (size_t)train_grid(b);
    return g * NPARAM * sizeof(float) + g * sizeof(double);
}

hipError_t launch_mlp_train(const double* const* c0, const double* const* c1,
                            const double* const* tend, int nx, int ny, int nz, const double* norm,
                            const int* cells, int b, double dt, const double* scale,
                            const double* rho, const double* rhon, double inv_n, float* params,
                            float* m1, float* m2, int t, double lr, double b1, double b2,
                            double eps, uint16_t* wpack, float* grad, float* loss, void* ws,
                            hipStream_t s) {
    static std::atomic<unsigned long long> attr{0};
    hipError_t e = set_lds_limit_once((const void*)mlp_train, TR_LDS, &attr);
    if (e != hipSuccess) return e;
    const int grid = train_grid(b);
    TrainArgs a;
    for (int q = 0; q < 4; q++) {
        a.c0[q] = c0[q];
        a.c1[q] = c1[q];
        a.tend[q] = tend[q];
        a.mean[q] = norm[2 * q];
        a.inv_std[q] = 1.0 / norm[2 * q + 1];
        a.inv_scale[q] = 1.0 / scale[q];
    }
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.cells = cells;
    a.B = b;
    a.inv_dt = 1.0 / dt;
    a.rho = rho;
    a.rhon = rhon;
    a.inv_n = inv_n;
    a.params = params;
    a.wpack = wpack;
    a.partials = (float*)ws;
    a.loss_part = (double*)((float*)ws + (size_t)grid * NPARAM);
    mlp_train<<<grid, 256, TR_LDS, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    UpdateArgs u;
    u.partials = a.partials;
    u.nb = grid;
    u.loss_part = a.loss_part;
    u.grad = grad;
    u.p = params;
    u.m1 = m1;
    u.m2 = m2;
    u.wpack = wpack;
    u.loss = loss;
    // as in launch_mlp_adam
    u.lr = (float)lr;
    u.b1 = (float)b1;
    u.omb1 = (float)(1.0 - b1);
    u.b2 = (float)b2;
    u.omb2 = (float)(1.0 - b2);
    u.eps = (float)eps;
    u.c1 = (float)(1.0 - pow(b1, t));
    u.c2 = (float)(1.0 - pow(b2, t));
    mlp_update<<<(NPARAM + 63) / 64, 64 * UPD_GROUPS, 0, s>>>(u);
    return hipGetLastError();
}

size_t correct_step_workspace_bytes(int nx, int ny, int nz) {
    return (size_t)blocks_for((long)nx * ny * nz) * CORR_NSUM * sizeof(double);
}

hipError_t launch_correct_step(double* const* in, double* const* tend, const float* gx,
                               const float* gy, double* const* out, int nx, int ny, int nz,
                               double dx, double dy, const double* scale, const double* rdz,
                               const double* rho, const double* rhon, double dt, double growth,
                               int* flags, void* workspace, hipStream_t s) {
    CorrArgs a;
    for (int q = 0; q < 4; q++) {
        a.in[q] = in[q];
        a.tend[q] = tend[q];
        a.out[q] = out[q];
        a.scale[q] = scale[q];
    }
    a.gx = gx;
    a.gy = gy;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.dx = dx;
    a.dy = dy;
    a.dt = dt;
    a.rdx = 1.0 / dx;
    a.rdy = 1.0 / dy;
    a.dt_dx = dt / dx;
    a.dt_dy = dt / dy;
    a.rdz = rdz;
    a.rho = rho;
    a.rhon = rhon;
    a.flags = flags;
    a.partial = static_cast<double*>(workspace);
    a.growth = growth;
    const long n = (long)nx * ny * nz;
    const int nb = blocks_for(n);
    corr_clear<<<1, 64, 0, s>>>(flags);
    corr_step<<<nb, 256, 0, s>>>(a);
    corr_decide<<<1, 256, 0, s>>>(a.partial, nb, growth, flags);
    corr_revert<<<nb, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace monc
