// march.hpp -- the fused MONC advection kernel for gfx950 ("column march").
//
// Evaluates the Piacsek-Williams momentum source terms and the ULTIMATE /
// QUICKEST scalar source terms (Brown et al., Sec. 3.1) for every interior
// point, optionally integrates them ("step fields", Sec. 3) and accumulates
// FP64 budget partials, in one pass over the fields.
//
// Work decomposition.  A workgroup of 8 waves owns TJ = 8/NCH consecutive
// columns j0..j0+TJ-1; a column of nz <= 64*NCH levels is split into NCH
// chunks of 64 levels, one wave per (column, chunk), lane l <-> level
// k = 64*chunk + l.  The workgroup marches along x through a segment of
// planes i0..i1-1.
//   * x-neighbours: a register window per column (planes i-1..i+1 for the
//     velocities, i-1..i+2 for scalars), each plane read from HBM once and
//     prefetched one plane ahead;
//   * y-neighbours: LDS slices of the current planes, 1 halo column each
//     side for velocities (two planes per velocity, double-buffered by plane
//     parity) and 2 for scalars; the halo columns are loaded round-robin by
//     the waves, one plane ahead;
//   * z-neighbours of values: the same LDS slices at k +- 1, +- 2;
//   * every face flux is computed once: the x-face i-1/2 is carried in
//     registers from the previous plane, the y-face j-1/2 is read from the
//     neighbouring wave through LDS, the z-face k-1/2 from the neighbouring
//     lane through a cross-lane shuffle (across a chunk boundary, through a
//     small LDS array).
// Per plane: store slices, barrier, finish the scalars of the previous plane
// (their y- and chunk faces come from other waves), compute values and faces.
// One barrier per plane: the velocity slices rotate over three planes and the
// scalar slices and face arrays over two, so a wave that runs ahead into the
// next plane's stores never overwrites what a slower wave still reads.
#pragma once

#include <type_traits>

#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

struct MarchArgs {
    AdvArgs a;
    int s0;          // first scalar of this launch's group
    int ns;          // number of scalars in the group
    int ti;          // planes per x-segment
    int njt;         // tiles along y
    int nseg;        // segments along x
    int first_pass;  // this launch writes every budget slot it does not own
};

// Per-level coefficient table kept in LDS.
enum {
    LV_ZTERM = 0, LV_RHOKM, LV_RHO, LV_RHOKP, LV_ALPHA, LV_BETA, LV_RHOINV, LV_RDZN,
    LV_RHON, LV_RHONINV, LV_RDZ, LV_RFZ, LV_MASS, LV_WMASS, LV_DZ, NLEV
};

template <typename Ts>
__device__ __forceinline__ Ts zero_of() {
    return Ts(0);
}
template <>
__device__ __forceinline__ bf16 zero_of<bf16>() {
    bf16 z;
    z.bits = 0;
    return z;
}

// Raw buffer access.  A buffer resource covers one x-plane of one field; an
// offset at or beyond its size reads as 0 and drops a store, so a lane that
// must not load (beyond the column, beyond the tile, the lid level of w) or
// must not store gets the offset MARCH_OOB instead of a branch around the
// access: the loads issue without waiting on one another and need no
// zero-initialised destination.
typedef int march_v2i __attribute__((ext_vector_type(2)));
constexpr uint32_t MARCH_OOB = 0xFFFFFFF0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, uint32_t bytes) {
    // descriptor word 3: 32-bit data format, raw (unswizzled) addressing
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename Ts>
__device__ __forceinline__ Ts bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ bf16 bload<bf16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    bf16 x;
    x.bits = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    return x;
}
// Cache policy of the stores: 2 = non-temporal.  The outputs are not read
// again by the launch; streamed past L2 they leave it to the input planes, and
// the neighbouring tiles' halo columns then hit there more often (measured on
// the FP64 step at 1024 x 1024 x 128: fetched bytes 1.30 -> 1.13 x the
// algorithmic reads).
#ifndef MONC_STORE_AUX
#define MONC_STORE_AUX 2
#endif
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(march_v2i, v), r, off, 0,
                                          MONC_STORE_AUX);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, off, 0, MONC_STORE_AUX);
}

// storage -> compute, subtracting `off` first when the storage is FP64
template <typename T, typename Ts>
__device__ __forceinline__ T cvt(Ts x, double off) {
    if constexpr (std::is_same<Ts, double>::value) {
        return (T)(x - off);
    } else if constexpr (std::is_same<Ts, float>::value) {
        return (T)x;
    } else {
        return __uint_as_float(((uint32_t)x.bits) << 16);
    }
}
template <typename T, typename Ts>
__device__ __forceinline__ T cvt0(Ts x) {
    if constexpr (std::is_same<Ts, bf16>::value) {
        return __uint_as_float(((uint32_t)x.bits) << 16);
    } else {
        return (T)x;
    }
}

// A copy the register allocator cannot fold into a renaming: the prefetch
// registers then keep one physical register each through the march, instead
// of rotating with the windows (a rotation that the unrolled loop does not
// close costs copies at its back-edge, and those wait for the newest loads).
template <typename Ts>
__device__ __forceinline__ Ts pinned_copy(Ts x) {
    if constexpr (sizeof(Ts) == 8) {
        double r;
        asm("v_mov_b64 %0, %1" : "=&v"(r) : "v"(x));
        return r;
    } else if constexpr (std::is_same<Ts, float>::value) {
        float r;
        asm("v_mov_b32 %0, %1" : "=&v"(r) : "v"(x));
        return r;
    } else {
        uint32_t r;
        asm("v_mov_b32 %0, %1" : "=&v"(r) : "v"((uint32_t)x.bits));
        return Ts{(uint16_t)r};
    }
}

// A value that is the same in every lane, moved to scalar registers.  The
// read that produces it then runs in every lane (the compiler would otherwise
// fold a read used by one lane into a branch on that lane).
__device__ __forceinline__ double wave_uniform(double x) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                            __builtin_amdgcn_readfirstlane(__double2loint(x)));
}
__device__ __forceinline__ float wave_uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Waves per workgroup: 8 when FP64 values are held (a wave needs up to 256
// registers, so two waves share a SIMD), 16 when storage and compute are both
// 32-bit or narrower.  MONC_MARCH_WAVES64 sets the FP64 count at build time
// (4 gives two workgroups per CU, whose barriers then overlap).
#ifndef MONC_MARCH_WAVES64
#define MONC_MARCH_WAVES64 8
#endif
template <typename Ts, typename T>
__host__ __device__ constexpr int march_waves() {
    return (sizeof(T) == 8 || sizeof(Ts) == 8) ? MONC_MARCH_WAVES64 : 16;
}

__host__ __device__ constexpr int march_nq(int ns, int nch, int wv) {
    return ((6 + 4 * ns) * nch + wv - 1) / wv;
}

// LDS columns hold levels -2 .. 64*NCH+1; the two levels below and above are
// zero, so neighbour reads at k-1, k+1, k+2 need no bounds checks.
template <int NCH>
__host__ __device__ constexpr int march_csz() { return 64 * NCH + 4; }

template <typename Ts, typename T, int NS, int NCH>
__host__ __device__ constexpr size_t march_lds_bytes() {
    constexpr int MARCH_WAVES = march_waves<Ts, T>();
    constexpr int TJ = MARCH_WAVES / NCH;
    return (size_t)(9 * (TJ + 2) + 2 * NS * (TJ + 4)) * march_csz<NCH>() * sizeof(T) +
           (size_t)(2 * NS * (TJ + 1) + NLEV) * (64 * NCH) * sizeof(T) +
           (size_t)2 * (NS > 0 ? NS : 1) * MARCH_WAVES * sizeof(T) + 64 * sizeof(T);
}

__device__ __forceinline__ int bud_op(int q) {
    if (q == MONC_B_COURANT) return 1;
    if (q >= MONC_B_SCALAR0 && (q - MONC_B_SCALAR0) % 3 == 2) return 2;
    return 0;
}
__device__ __forceinline__ double bud_comb(double a, double b, int op) {
    return op == 0 ? a + b : (op == 1 ? fmax(a, b) : fmin(a, b));
}
__device__ __forceinline__ double bud_ident(int op) {
    return op == 2 ? __builtin_huge_val() : 0.0;
}

// One tile of the march: columns jt*TJ .. jt*TJ+TJ-1, planes seg*ti .. .
struct TileJob {
    int s0;               // first scalar of this group
    int ti;               // planes per x-segment
    int jt, seg;          // the tile
    double* partial_row;  // budget partials of this tile (BUD only)
    int first_pass;       // write the budget slots this group does not own
};

// Options of the fused step (FP64 STEP only): OPT_DYN adds the other dynamics
// source terms (Coriolis, buoyancy of scalar 0) to the momentum; OPT_SPW
// advects the scalars with the centred (PW) flux form instead of TVD.
// OPT_WORK (momentum source terms only, TEND) evaluates the PW arithmetic
// a.work times on the same values (the work-scaled experiment).
enum { OPT_DYN = 1, OPT_SPW = 2, OPT_WORK = 4 };

// Makes x opaque to the optimiser and orders it after `dep` (an empty asm).
template <typename T>
__device__ __forceinline__ void chain(T& x, T dep) {
    asm volatile("" : "+v"(x) : "v"(dep));
}

template <typename Ts, typename T, int MODE, bool PW, int NS, bool BUD, int NCH, int OPT>
__device__ __forceinline__ void march_tile(const AdvArgs& a, const TileJob& tj,
                                           unsigned char* smem_raw) {
    using To = typename std::conditional<std::is_same<T, double>::value, double, float>::type;
    constexpr bool STEP64 = MODE == STEP && std::is_same<T, double>::value;
    constexpr bool DYN = (OPT & OPT_DYN) != 0;
    constexpr bool SPW = (OPT & OPT_SPW) != 0;
    constexpr bool WORK = (OPT & OPT_WORK) != 0;
    static_assert((OPT & ~OPT_WORK) == 0 || STEP64, "options of the FP64 step only");
    static_assert(!WORK || (MODE == TEND && PW && NS == 0), "work repetitions: PW source terms");
    // scalar face flux: TVD, or the centred flux form when SPW
    auto sflux = [&](T a_, T pm, T p0, T p1, T p2, T cfac, T rfac, T mass) -> T {
        if constexpr (SPW) {
            (void)pm, (void)p2, (void)cfac, (void)rfac;
            return centred_flux<T>(a_, p0, p1, mass);
        } else {
            return tvd_flux<T>(a_, pm, p0, p1, p2, cfac, rfac, mass);
        }
    };
    constexpr int MARCH_WAVES = march_waves<Ts, T>();
    constexpr int TJ = MARCH_WAVES / NCH;
    constexpr int NZP = 64 * NCH;
    constexpr int CSZ = march_csz<NCH>();  // LDS column stride (padded)
    constexpr int VC = TJ + 2;             // velocity slice columns: j0-1 .. j0+TJ
    constexpr int SC = TJ + 4;             // scalar slice columns:   j0-2 .. j0+TJ+1
    constexpr int FC = TJ + 1;             // y-faces j0-1/2 .. j0+TJ-1/2
    constexpr int NSA = NS > 0 ? NS : 1;
    constexpr int NQ = march_nq(NS, NCH, MARCH_WAVES);
    constexpr int NJ = (6 + 4 * NS) * NCH;
    constexpr int NACC = MONC_B_SCALAR0 + 3 * NS;

    constexpr int VSL = VC * CSZ;       // one velocity slice (one field, one plane)
    constexpr int SSL = NS * SC * CSZ;  // the scalar slices of one plane
    constexpr int FSL = NS * FC * NZP;  // the y-faces of one plane
    T* const vel = reinterpret_cast<T*>(smem_raw);  // [3][plane % 3][VC][CSZ]
    T* const sph0 = vel + 9 * VSL;                  // [plane % 2][NS][SC][CSZ]
    T* const sfy0 = sph0 + 2 * SSL;                 // [plane % 2][NS][FC][NZP]
    T* const lev = sfy0 + 2 * FSL;                  // [NLEV][NZP]
    T* const fzc0 = lev + NLEV * NZP;               // [plane % 2][NS][TJ][NCH] chunk-top faces
    T* const sink = fzc0 + 2 * NSA * MARCH_WAVES;   // [64] stores of unused halo jobs

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t sx = (size_t)(ny + 4) * nz;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cc = wv / NCH;  // column within the tile
    const int ch = wv % NCH;  // chunk within the column
    const int k = 64 * ch + lane;

    const int j0 = tj.jt * TJ;
    const int i0 = tj.seg * tj.ti;
    const int i1 = min(i0 + tj.ti, nx);
    const int j = j0 + cc;
    const bool own_ok = j <= ny + 1;  // a column the tile reads (interior or its neighbours)
    const bool active = j < ny;       // interior column: compute and store
    const bool kin = k < nz;
    const bool store = active && kin;

    const double dt = a.dt;
    const double cdx = dt / a.dx, cdy = dt / a.dy;  // Courant number per unit speed
    // ---- level table (vertical geometry from rdz, rho, rhon) ----
    for (int kk = threadIdx.x; kk < NZP; kk += MARCH_WAVES * 64) {
        double v[NLEV];
#pragma unroll
        for (int q = 0; q < NLEV; q++) v[q] = 0.0;
        if (kk < nz) {
            const double rdzk = a.rdz[kk], rhonk = a.rhon[kk], rhok = a.rho[kk];
            const double dzk = 1.0 / rdzk;
            v[LV_ZTERM] = rdzk / (4.0 * rhonk);
            v[LV_RHOKM] = kk > 0 ? a.rho[kk - 1] : 0.0;
            v[LV_RHO] = rhok;
            v[LV_RHOKP] = kk < nz - 1 ? a.rho[kk + 1] : 0.0;
            v[LV_RHOINV] = 1.0 / rhok;
            v[LV_RHON] = rhonk;
            v[LV_RHONINV] = 1.0 / rhonk;
            v[LV_RDZ] = rdzk;
            v[LV_MASS] = rhonk * dzk;
            v[LV_DZ] = dzk;
            if (kk < nz - 1) {
                const double dzk1 = 1.0 / a.rdz[kk + 1];
                const double dzn = 0.5 * (dzk + dzk1);
                v[LV_RDZN] = 1.0 / dzn;
                v[LV_ALPHA] = dzk * rhonk / (2.0 * dzn);
                v[LV_BETA] = dzk1 * a.rhon[kk + 1] / (2.0 * dzn);
                v[LV_RFZ] = dzn / dt;
                v[LV_WMASS] = rhok * dzn;
            }
        }
#pragma unroll
        for (int q = 0; q < NLEV; q++) lev[q * NZP + kk] = (T)v[q];
    }
    // zero the padding levels of every slice column
    for (int t = threadIdx.x; t < (9 * VC + 2 * NS * SC) * 4; t += MARCH_WAVES * 64) {
        const int col = t >> 2, w4 = t & 3;
        vel[(size_t)col * CSZ + (w4 < 2 ? w4 : NZP + w4)] = (T)0;
    }

    const T r4dx = (T)(0.25 / a.dx), r4dy = (T)(0.25 / a.dy);
    const T r2dx = (T)(0.5 / a.dx), r2dy = (T)(0.5 / a.dy);
    const T rdx = (T)(1.0 / a.dx), rdy = (T)(1.0 / a.dy);
    const T cfx = (T)(dt / a.dx), cfy = (T)(dt / a.dy);
    const T rfx = (T)(a.dx / dt), rfy = (T)(a.dy / dt);
    const T dtc = (T)dt;

    // field pointers: 0..2 velocities, 3.. the scalars of this group
    const Ts* fptr[3 + NSA];
    fptr[0] = (const Ts*)a.in[0];
    fptr[1] = (const Ts*)a.in[1];
    fptr[2] = (const Ts*)a.in[2];
    double off[NSA];
    T phi0c[NSA];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        fptr[3 + s] = (const Ts*)a.in[3 + tj.s0 + s];
        // the FP64 step keeps the state as it is (no anomaly offset): a
        // compile-time zero, so the subtractions and the constant's term fold
        // away
        off[s] = STEP64 ? 0.0 : (MODE == STEP ? a.phi0[tj.s0 + s] : 0.0);
        phi0c[s] = STEP64 ? (T)0 : (T)a.phi0[tj.s0 + s];
    }
    // Periodic neighbours are read at wrapped indices: the arrays' halos are
    // never read.  plane ii of field pointer p (uniform) ...
    // indices reach at most two periods outside [0, n): wrap by adds, not
    // by an integer division
    auto wrapx = [&](int ii) -> int {
        if (ii < 0) ii += nx;
        if (ii < 0) ii += nx;
        if (ii >= nx) ii -= nx;
        if (ii >= nx) ii -= nx;
        return ii;
    };
    auto wrapy = [&](int jj) -> int {
        if (jj < 0) jj += ny;
        if (jj < 0) jj += ny;
        if (jj >= ny) jj -= ny;
        if (jj >= ny) jj -= ny;
        return jj;
    };
    const uint32_t pbytes = (uint32_t)(sx * sizeof(Ts));  // one x-plane of a field
    // element offset of plane ii (wrapped) within a field
    auto poff = [&](int ii) -> size_t { return (size_t)(wrapx(ii) + 2) * sx; };
    // load from the plane at element offset po of field pointer p, at byte
    // offset boff within the plane
    auto ldo = [&](const Ts* p, size_t po, uint32_t boff) -> Ts {
        return bload<Ts>(plane_rsrc(p + po, pbytes), boff);
    };
    auto ld = [&](const Ts* p, int ii, uint32_t boff) -> Ts { return ldo(p, poff(ii), boff); };
    // own column: byte offsets within a plane; lanes that do not load (or
    // store) get MARCH_OOB (the lid level of w reads as 0)
    const bool ok_s = own_ok && kin;
    const bool ok_w = own_ok && k < nz - 1;
    const uint32_t col_off = (uint32_t)(((wrapy(j) + 2) * nz + k) * (int)sizeof(Ts));
    const uint32_t roff_s = ok_s ? col_off : MARCH_OOB;  // loads of u, v, scalars
    const uint32_t roff_w = ok_w ? col_off : MARCH_OOB;  // loads of w
    const uint32_t woff = store ? (uint32_t)(((j + 2) * nz + k) * (int)sizeof(To)) : MARCH_OOB;
    const uint32_t wbytes = (uint32_t)(sx * sizeof(To));
    const uint32_t wbytes64 = (uint32_t)(sx * sizeof(double));
    const uint32_t woff64 = store ? (uint32_t)(((j + 2) * nz + k) * (int)sizeof(double)) : MARCH_OOB;

    // Halo jobs of one plane step, for each chunk: velocities u(i), v(i+1),
    // w(i+1) at columns j0-1 and j0+TJ; scalar s at plane i, columns j0-2,
    // j0-1, j0+TJ, j0+TJ+1.  Job id = wv + 8 q; decoded once here.
    int hj_f[NQ], hj_dpl[NQ], hj_lds[NQ], hj_par[NQ];
    double hj_o[NQ];
    const Ts* hj_ptr[NQ];
    uint32_t hj_boff[NQ];
    bool hj_ok[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int id = wv + MARCH_WAVES * q;
        const int chunk = id % NCH, h = id / NCH;
        int f, dpl, jj, c;
        if (h < 6) {
            f = h >> 1;
            dpl = f == 0 ? 0 : 1;
            const bool right = h & 1;
            jj = right ? j0 + TJ : j0 - 1;
            c = right ? TJ + 1 : 0;
        } else {
            const int s = (h - 6) >> 2, qq = (h - 6) & 3;
            f = 3 + s;
            dpl = 0;
            jj = qq == 0 ? j0 - 2 : (qq == 1 ? j0 - 1 : (qq == 2 ? j0 + TJ : j0 + TJ + 1));
            c = qq == 0 ? 0 : (qq == 1 ? 1 : (qq == 2 ? TJ + 2 : TJ + 3));
        }
        const int kk = 64 * chunk + lane;
        const bool valid = id < NJ && jj <= ny + 1;
        hj_f[q] = valid ? f : 0;
        const Ts* fp = fptr[0];
#pragma unroll
        for (int f2 = 1; f2 < 3 + NS; f2++)
            if (hj_f[q] == f2) fp = fptr[f2];
        hj_ptr[q] = fp;
        hj_dpl[q] = dpl;
        hj_ok[q] = valid && kk < nz && !(f == 2 && kk >= nz - 1);
        hj_boff[q] = hj_ok[q] ? (uint32_t)(((wrapy(jj) + 2) * nz + kk) * (int)sizeof(Ts))
                              : MARCH_OOB;
        // LDS element offset (velocity slots: the parity term hj_par is added
        // on odd planes); a job without a column stores into the sink
        hj_lds[q] = !valid ? (int)(sink - vel) + lane
                    : f < 3 ? ((f * 3) * VC + c) * CSZ + 2 + kk
                            : (int)(sph0 - vel) + ((f - 3) * SC + c) * CSZ + 2 + kk;
        // slot stride: velocity slices rotate over three planes, scalar
        // slices over two (sink stores take no offset)
        hj_par[q] = !valid ? 0 : (f < 3 ? VSL : SSL);
        double o = 0.0;
#pragma unroll
        for (int s = 0; s < NS; s++)
            if (valid && f == 3 + s) o = off[s];
        hj_o[q] = o;
    }
    // halo loads of plane step i + 1 (o1, o2: offsets of planes i + 1 and i + 2)
    auto job_load = [&](int q, size_t o1, size_t o2) -> Ts {
        return ldo(hj_ptr[q], hj_dpl[q] ? o2 : o1, hj_boff[q]);
    };
    // planes i >= -1 to their slots
    auto slot3 = [](int plane_i) -> int { return (plane_i + 3) % 3; };
    // no branch: every job stores, unused ones into the sink
    auto job_store = [&](int q, int i, Ts x) {
        const int slot = hj_f[q] < 3 ? slot3(i + hj_dpl[q]) : (i & 1);
        vel[hj_lds[q] + slot * hj_par[q]] = cvt<T, Ts>(x, hj_o[q]);
    };
    // own column slot addresses
    auto vslot = [&](int f, int plane_i) -> T* { return vel + (f * 3 + slot3(plane_i)) * VSL; };
    auto sphs = [&](int plane_i) -> T* { return sph0 + (plane_i & 1) * SSL; };
    auto sfys = [&](int plane_i) -> T* { return sfy0 + (plane_i & 1) * FSL; };
    auto fzcs = [&](int plane_i) -> T* { return fzc0 + (plane_i & 1) * (NSA * MARCH_WAVES); };
    const int ownv = (cc + 1) * CSZ + 2 + k;  // own column in a velocity slot
    const int owns = (cc + 2) * CSZ + 2 + k;  // own column in a scalar slice

    // ---- register windows ----
    Ts U[3], V[3], W[3];  // planes i-1, i, i+1 of the own column
    Ts P[NSA][4];         // planes i-1 .. i+2
    T FXm[NSA];           // flux through the x-face i-1/2 (rhon factored out)
    // Data of a later step t, loaded DEPTH steps ahead into one of DEPTH sets
    // used in turn (the march is unrolled by DEPTH): velocities of plane t+1,
    // scalars of plane t+2, halo columns of step t.  Step t shifts its set
    // into the windows before the set is reloaded, so a load has DEPTH steps
    // to arrive before anything waits for it.  (Three sets measured no
    // faster than two for FP64 on 1024 x 1024 x 128.)
    struct Ahead {
        Ts u, v, w;
        Ts p[NSA];
        Ts h[NQ];
    };
    constexpr int DEPTH = 2;
    Ahead S[DEPTH];
    double acc[BUD ? NACC : 1];
    int nonfinite = 0;  // non-finite values written by this lane
    double amax[3] = {0.0, 0.0, 0.0};  // largest |u|, |v|, |w| over the march
    if constexpr (BUD) {
#pragma unroll
        for (int q = 0; q < NACC; q++) acc[q] = bud_ident(bud_op(q));
    }

    // ---- prologue: windows one plane behind i0 (step i0 shifts in its own
    // data), the carried x-face, the first slices ----
    __syncthreads();  // level table visible
#pragma unroll
    for (int p = 0; p < 3; p++) {
        U[p] = ld(fptr[0], i0 - 2 + p, roff_s);
        V[p] = ld(fptr[1], i0 - 2 + p, roff_s);
        W[p] = ld(fptr[2], i0 - 2 + p, roff_w);
    }
#pragma unroll
    for (int s = 0; s < NS; s++) {
#pragma unroll
        for (int p = 0; p < 4; p++) P[s][p] = ld(fptr[3 + s], i0 - 2 + p, roff_s);
        // x-face i0-1/2: u of plane i0-1, scalars of planes i0-2 .. i0+1
        FXm[s] = sflux(cvt0<T, Ts>(U[1]), cvt<T, Ts>(P[s][0], off[s]),
                             cvt<T, Ts>(P[s][1], off[s]), cvt<T, Ts>(P[s][2], off[s]),
                             cvt<T, Ts>(P[s][3], off[s]), cfx, rfx, (T)1);
    }
    // own slots of u(i0-1), v(i0), w(i0) (a column past ny+1 stores zeros
    // that nothing reads)
    vslot(0, i0 - 1)[ownv] = cvt0<T, Ts>(U[1]);
    vslot(1, i0)[ownv] = cvt0<T, Ts>(V[2]);
    vslot(2, i0)[ownv] = cvt0<T, Ts>(W[2]);
    // halo columns of u(i0-1), v(i0), w(i0)
    for (int id = wv; id < 6 * NCH; id += MARCH_WAVES) {
        const int chunk = id % NCH, h = id / NCH;
        const int f = h >> 1;
        const bool right = h & 1;
        const int jj = right ? j0 + TJ : j0 - 1;
        const int c = right ? TJ + 1 : 0;
        const int pl = f == 0 ? i0 - 1 : i0;
        if (jj > ny + 1) continue;
        const int kk = 64 * chunk + lane;
        const bool ok = kk < nz && !(f == 2 && kk >= nz - 1);
        const Ts* fp = f == 0 ? fptr[0] : (f == 1 ? fptr[1] : fptr[2]);
        const Ts x =
            ld(fp, pl, ok ? (uint32_t)(((wrapy(jj) + 2) * nz + kk) * (int)sizeof(Ts)) : MARCH_OOB);
        vslot(f, pl)[c * CSZ + 2 + kk] = cvt0<T, Ts>(x);
    }
    // the data of steps i0 .. i0+DEPTH-1, set by set in this order (the
    // scheduler may not interleave them: the loop's waits count on it)
#pragma unroll
    for (int d = 0; d < DEPTH; d++) {
        const size_t p0 = poff(i0 + d), p1 = poff(i0 + d + 1), p2 = poff(i0 + d + 2);
        S[d].u = ldo(fptr[0], p1, roff_s);
        S[d].v = ldo(fptr[1], p1, roff_s);
        S[d].w = ldo(fptr[2], p1, roff_w);
#pragma unroll
        for (int s = 0; s < NS; s++) S[d].p[s] = ldo(fptr[3 + s], p2, roff_s);
#pragma unroll
        for (int q = 0; q < NQ; q++) S[d].h[q] = job_load(q, p0, p1);
        __builtin_amdgcn_sched_barrier(0);
    }
    // plane offsets carried through the march: at step i, planes i+DEPTH
    // (halo columns), i+DEPTH+1 (velocities), i+DEPTH+2 (scalars) of the data
    // it prefetches; each step shifts them and wraps the newest with one
    // compare
    size_t o_h = poff(i0 + DEPTH), o_v = poff(i0 + DEPTH + 1), o_s = poff(i0 + DEPTH + 2);
    const size_t o_end = (size_t)(nx + 2) * sx, o_span = (size_t)nx * sx;

    // per-level constants of this lane
    const bool bottom = k == 0;           // the ground face is below
    const bool top2 = k + 2 >= nz;        // no far-upwind cell above the top face

    // ---- finishing a plane's scalars: the y-face below from LDS, the z-face
    // below from the neighbouring lane (or the chunk below); pv: 0 or 1, the
    // window slot that holds the plane's own values at the call ----
    T part_c[NSA], up_c[NSA];
    auto finish = [&](int ip, int pv) __attribute__((always_inline)) {
        const T rdz = lev[LV_RDZ * NZP + k];
        const T rhon_inv = lev[LV_RHONINV * NZP + k];
        const size_t gplane = (size_t)(ip + 2) * sx;
#pragma unroll
        for (int s = 0; s < NS; s++) {
            T fzm = up_c[s];
            if constexpr (NCH > 1) {
                // read unconditionally (one address: a broadcast), then select
                const T below =
                    wave_uniform(fzcs(ip)[(s * TJ + cc) * NCH + (ch > 0 ? ch - 1 : 0)]);
                fzm = lane == 0 ? (ch == 0 ? (T)0 : below) : fzm;
            } else {
                fzm = lane == 0 ? (T)0 : fzm;
            }
            const T fym = sfys(ip)[(s * FC + cc) * NZP + k];
            const T val = part_c[s] + fym * rdy + rhon_inv * rdz * fzm;
            const Ts pown = P[s][pv];
            if constexpr (MODE == TEND) {
                (void)pown;
                bstore(plane_rsrc((To*)a.out[3 + tj.s0 + s] + gplane, wbytes), woff, (To)val);
            } else {
                // the state is FP64 whatever the compute type
                const double nsv = (double)pown + dt * (double)val;
                bstore(plane_rsrc((double*)a.out[3 + tj.s0 + s] + gplane, wbytes64), woff64, nsv);
                if constexpr (BUD) {
                    // every lane sums and counts; a lane that stores nothing
                    // drops its sums and count after the march
                    const double phd = (double)pown;
                    acc[MONC_B_SCALAR0 + 3 * s] += (double)val;
                    acc[MONC_B_SCALAR0 + 3 * s + 1] += phd;
                    acc[MONC_B_SCALAR0 + 3 * s + 2] = fmin(acc[MONC_B_SCALAR0 + 3 * s + 2], phd);
                    nonfinite += !isfinite(nsv);
                }
            }
        }
    };

    // ---- the march: one step; Xs holds step i's data and receives step
    // i+DEPTH's ----
    auto march_step = [&](int i, Ahead& Xs) __attribute__((always_inline)) {
        // shift step i's planes into the windows
        U[0] = U[1];
        U[1] = U[2];
        U[2] = pinned_copy(Xs.u);
        V[0] = V[1];
        V[1] = V[2];
        V[2] = pinned_copy(Xs.v);
        W[0] = W[1];
        W[1] = W[2];
        W[2] = pinned_copy(Xs.w);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            P[s][0] = P[s][1];
            P[s][1] = P[s][2];
            P[s][2] = P[s][3];
            P[s][3] = pinned_copy(Xs.p[s]);
        }
        // slices of step i (a column past ny+1 stores zeros that nothing reads)
        vslot(0, i)[ownv] = cvt0<T, Ts>(U[1]);
        vslot(1, i + 1)[ownv] = cvt0<T, Ts>(V[2]);
        vslot(2, i + 1)[ownv] = cvt0<T, Ts>(W[2]);
#pragma unroll
        for (int s = 0; s < NS; s++) sphs(i)[s * SC * CSZ + owns] = cvt<T, Ts>(P[s][1], off[s]);
#pragma unroll
        for (int q = 0; q < NQ; q++) job_store(q, i, Xs.h[q]);
        // prefetch of step i+DEPTH (planes stay in bounds past the segment end:
        // they wrap, and the extra data is not used)
        Xs.u = ldo(fptr[0], o_v, roff_s);
        Xs.v = ldo(fptr[1], o_v, roff_s);
        Xs.w = ldo(fptr[2], o_v, roff_w);
#pragma unroll
        for (int s = 0; s < NS; s++) Xs.p[s] = ldo(fptr[3 + s], o_s, roff_s);
#pragma unroll
        for (int q = 0; q < NQ; q++) Xs.h[q] = job_load(q, o_h, o_v);
        __syncthreads();
        // the previous plane's scalars: their y-faces and chunk faces are
        // visible now (after this step's shift its values are P[s][0])
        if (i > i0) finish(i - 1, 0);

        const T* u_i = vslot(0, i);
        const T* u_im = vslot(0, i - 1);
        const T* v_i = vslot(1, i);
        const T* v_ip = vslot(1, i + 1);
        const T* w_i = vslot(2, i);
        const T* w_ip = vslot(2, i + 1);
        const size_t gplane = (size_t)(i + 2) * sx;

        // Scalars keep until the next plane's barrier only a partial sum and
        // the top face of the level below (part_c, up_c); momentum is finished
        // (and stored) now.
        T fxp[NSA];
        const T uc = cvt0<T, Ts>(U[1]), um = cvt0<T, Ts>(U[0]);
        // x-faces first: they need registers only, and overlap the LDS reads
#pragma unroll
        for (int s = 0; s < NS; s++) {
            fxp[s] = sflux(uc, cvt<T, Ts>(P[s][0], off[s]), cvt<T, Ts>(P[s][1], off[s]),
                                 cvt<T, Ts>(P[s][2], off[s]), cvt<T, Ts>(P[s][3], off[s]), cfx,
                                 rfx, (T)1);
        }
        const T vc = cvt0<T, Ts>(V[1]);
        const T wc = cvt0<T, Ts>(W[1]);
        const T vs = v_i[ownv - CSZ];
        const T wb = w_i[ownv - 1];
        const T rhon = lev[LV_RHON * NZP + k];
        const T rho = lev[LV_RHO * NZP + k];
        const T rho_km = lev[LV_RHOKM * NZP + k];
        const T rdz = lev[LV_RDZ * NZP + k];
        const T rhon_inv = lev[LV_RHONINV * NZP + k];
        // anelastic mass divergence of this cell
        const T D = rhon * ((uc - um) * rdx + (vc - vs) * rdy) + rdz * (rho * wc - rho_km * wb);
        if constexpr (PW) {
            const T up = cvt0<T, Ts>(U[2]);
            const T vw = cvt0<T, Ts>(V[0]), ve = cvt0<T, Ts>(V[2]);
            const T ww = cvt0<T, Ts>(W[0]), we = cvt0<T, Ts>(W[2]);
            Level<T> L;
            L.zterm = lev[LV_ZTERM * NZP + k];
            L.rho_km = rho_km;
            L.rho = rho;
            L.rho_kp = lev[LV_RHOKP * NZP + k];
            L.alpha = lev[LV_ALPHA * NZP + k];
            L.beta = lev[LV_BETA * NZP + k];
            L.rho_inv = lev[LV_RHOINV * NZP + k];
            L.rdzn = lev[LV_RDZN * NZP + k];
            const T us = u_i[ownv - CSZ], un = u_i[ownv + CSZ];
            const T ub = u_i[ownv - 1], ut = u_i[ownv + 1];
            const T u_nw = u_im[ownv + CSZ], u_wt = u_im[ownv + 1];
            const T vn = v_i[ownv + CSZ];
            const T vb = v_i[ownv - 1], vt = v_i[ownv + 1];
            const T v_st = v_i[ownv - CSZ + 1], v_es = v_ip[ownv - CSZ];
            const T ws = w_i[ownv - CSZ], wn = w_i[ownv + CSZ];
            const T wt = w_i[ownv + 1], w_nb = w_i[ownv + CSZ - 1];
            const T w_eb = w_ip[ownv - 1];
            T su = pw_su<T>(um, uc, up, us, un, ub, ut, vs, v_es, vc, ve, wb, w_eb, wc, we, L,
                            r4dx, r4dy);
            T sv = pw_sv<T>(vw, vc, ve, vs, vn, vb, vt, um, u_nw, uc, un, wb, w_nb, wc, wn, L,
                            r4dx, r4dy);
            T swc = pw_sw<T>(uc, ut, um, u_wt, vc, vt, vs, v_st, wc, ww, we, ws, wn, wb, wt, L,
                             r2dx, r2dy);
            if constexpr (WORK) {
                // the same arithmetic again on the same values, every input of a
                // repetition made to depend on the previous result, so nothing
                // is merged or dropped and the result is that of one evaluation
                T x[27] = {um, uc, up, us, un, ub, ut, vs, v_es, vc, ve, wb, w_eb, wc,
                           we, vw, vn, vb, vt, u_nw, w_nb, wn, u_wt, v_st, ww, ws, wt};
                for (int r = 1; r < a.work; r++) {
                    const T dep = su + sv + swc;
#pragma unroll
                    for (int q = 0; q < 27; q++) chain(x[q], dep);
                    su = pw_su<T>(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], x[8], x[9],
                                  x[10], x[11], x[12], x[13], x[14], L, r4dx, r4dy);
                    sv = pw_sv<T>(x[15], x[9], x[10], x[7], x[16], x[17], x[18], x[0], x[19],
                                  x[1], x[4], x[11], x[20], x[13], x[21], L, r4dx, r4dy);
                    swc = pw_sw<T>(x[1], x[6], x[0], x[22], x[9], x[18], x[7], x[23], x[13],
                                   x[24], x[14], x[25], x[21], x[11], x[26], L, r2dx, r2dy);
                }
            }
            const T sw = k < nz - 1 ? swc : (T)0;
            if constexpr (MODE == TEND) {
                bstore(plane_rsrc((To*)a.out[0] + gplane, wbytes), woff, (To)su);
                bstore(plane_rsrc((To*)a.out[1] + gplane, wbytes), woff, (To)sv);
                bstore(plane_rsrc((To*)a.out[2] + gplane, wbytes), woff, (To)sw);
            } else {
                double nu, nv, nw;
                if constexpr (DYN) {
                    // the other dynamics source terms, added to the advection
                    // source terms before the step (scalar 0 is theta; FP64
                    // state, no anomaly offset)
                    static_assert(NS >= 1 && std::is_same<T, double>::value, "DYN needs theta");
                    const double du = coriolis_u(a.fcor, a.vg, (double)vc, (double)ve,
                                                 (double)vs, (double)v_es);
                    const double dv = coriolis_v(a.fcor, a.ug, (double)uc, (double)um,
                                                 (double)un, (double)u_nw);
                    const double th_k = (double)P[0][1];
                    const double th_kp = (double)sphs(i)[owns + 1] + off[0];
                    const double dw = buoyancy_w(a.gth, a.th0, th_k, th_kp);
                    nu = (double)U[1] + dt * ((double)su + du);
                    nv = (double)V[1] + dt * ((double)sv + dv);
                    nw = k < nz - 1 ? (double)W[1] + dt * ((double)sw + dw) : 0.0;
                } else {
                    nu = (double)U[1] + dt * (double)su;
                    nv = (double)V[1] + dt * (double)sv;
                    nw = k < nz - 1 ? (double)W[1] + dt * (double)sw : 0.0;
                }
                bstore(plane_rsrc((double*)a.out[0] + gplane, wbytes64), woff64, nu);
                bstore(plane_rsrc((double*)a.out[1] + gplane, wbytes64), woff64, nv);
                bstore(plane_rsrc((double*)a.out[2] + gplane, wbytes64), woff64, nw);
                if constexpr (BUD) {
                    // Per-lane sums and non-finite counts over the march (one
                    // level k per lane): the level's weights (rhon dz, rho
                    // dzn, -dz/4) multiply once at the end.  Every lane sums
                    // and counts (whether a lane stores is fixed for the
                    // march); one that stores nothing drops them at the end.
                    // The Courant number keeps the largest |u|, |v|, |w| and
                    // scales them at the end: scaling by a positive factor is
                    // monotone, so the maximum is the same.
                    const double ucd = (double)U[1], umd = (double)U[0];
                    const double vcd = (double)V[1], vsd = (double)vs;
                    const double wcd = (double)W[1], wbd = (double)wb;
                    const double Dd = (double)D;
                    acc[MONC_B_CU] += (double)su;
                    acc[MONC_B_CV] += (double)sv;
                    acc[MONC_B_PU] = fma(ucd, (double)su, acc[MONC_B_PU]);
                    acc[MONC_B_PV] = fma(vcd, (double)sv, acc[MONC_B_PV]);
                    acc[MONC_B_QU] = fma(Dd, fma(ucd, ucd, umd * umd), acc[MONC_B_QU]);
                    acc[MONC_B_QV] = fma(Dd, fma(vcd, vcd, vsd * vsd), acc[MONC_B_QV]);
                    acc[MONC_B_QW] = fma(Dd, fma(wcd, wcd, wbd * wbd), acc[MONC_B_QW]);
                    acc[MONC_B_CW] += (double)sw;
                    acc[MONC_B_PW] = fma(wcd, (double)sw, acc[MONC_B_PW]);
                    amax[0] = fmax(amax[0], fabs(ucd));
                    amax[1] = fmax(amax[1], fabs(vcd));
                    amax[2] = fmax(amax[2], fabs(wcd));
                    nonfinite += !isfinite(nu) + !isfinite(nv) + !isfinite(nw);
                }
            }
        }
        const T rfz = lev[LV_RFZ * NZP + k];
        const T cfz = dtc * lev[LV_RDZN * NZP + k];
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const T* ph = sphs(i) + s * SC * CSZ;
            const T pc = cvt<T, Ts>(P[s][1], off[s]);
            // lateral fluxes are computed without the common rhon factor
            const T ps = ph[owns - CSZ], pn = ph[owns + CSZ], pnn = ph[owns + 2 * CSZ];
            const T fyp = sflux(vc, ps, pc, pn, pnn, cfy, rfy, (T)1);
            sfys(i)[(s * FC + cc + 1) * NZP + k] = fyp;
            // top face k+1/2.  Where the far-upwind cell is outside the column
            // it is replaced by the upwind cell, which makes the limiter return
            // the upwind value (first-order upwind); on the lid w is zero.
            const T pb = ph[owns - 1], pt = ph[owns + 1], ptt = ph[owns + 2];
            const T fz = sflux(wc, bottom ? pc : pb, pc, pt, top2 ? pt : ptt, cfz, rfz, rho);
            up_c[s] = __shfl_up(fz, 1, 64);  // the face below, from the lane below
            // the chunk's top face, for the chunk above: lane 63 stores it, the
            // other lanes store into the sink (no branch; 64 lanes writing one
            // address would serialise in the LDS)
            if constexpr (NCH > 1) {
                T* const dst = lane == 63 ? fzcs(i) + (s * TJ + cc) * NCH + ch : sink + lane;
                *dst = fz;
            }
            // everything but the faces shared with the neighbours (j-1/2,
            // k-1/2); stored values are anomalies from phi0: add the term of
            // the constant
            part_c[s] = -((fxp[s] - FXm[s]) * rdx + fyp * rdy) - rhon_inv * rdz * fz;
            if constexpr (!STEP64) part_c[s] -= phi0c[s] * D * rhon_inv;
            FXm[s] = fxp[s];
        }
        // the tile's first column also computes the y-face j0-1/2 (one
        // wave-uniform block for all scalars; spreading these faces over
        // waves on different SIMDs measured no faster)
        if (cc == 0) {
#pragma unroll
            for (int s = 0; s < NS; s++) {
                const T* ph = sphs(i) + s * SC * CSZ;
                sfys(i)[(s * FC) * NZP + k] =
                    sflux(vs, ph[owns - 2 * CSZ], ph[owns - CSZ], ph[owns], ph[owns + CSZ],
                                cfy, rfy, (T)1);
            }
        }
        // advance the plane offsets
        o_h = o_v;
        o_v = o_s;
        o_s += sx;
        if (o_s >= o_end) o_s -= o_span;
    };
    for (int i = i0; i < i1; i += DEPTH) {
        march_step(i, S[0]);
#pragma unroll
        for (int d = 1; d < DEPTH; d++)
            if (i + d < i1) march_step(i + d, S[d]);
    }
    // the last plane's scalars (no shift followed: its values are P[s][1])
    __syncthreads();
    if (i1 > i0) finish(i1 - 1, 1);

    if constexpr (BUD) {
        // the level's weights in FP64 from the profiles (the level table may
        // be FP32), the lane's count
        {
            if (!store) {
#pragma unroll
                for (int q = 0; q < NACC; q++) acc[q] = bud_ident(bud_op(q));
            }
            double mass = 0.0, wmass = 0.0, qf = 0.0, rdzn = 0.0;
            if (k < nz) {
                const double dzk = 1.0 / a.rdz[k];
                mass = a.rhon[k] * dzk;
                qf = -0.25 * dzk;
                if (k < nz - 1) {
                    const double dzn = 0.5 * (dzk + 1.0 / a.rdz[k + 1]);
                    wmass = a.rho[k] * dzn;
                    rdzn = 1.0 / dzn;
                }
            }
            acc[MONC_B_CU] *= mass;
            acc[MONC_B_CV] *= mass;
            acc[MONC_B_PU] *= mass;
            acc[MONC_B_PV] *= mass;
            acc[MONC_B_QU] *= qf;
            acc[MONC_B_QV] *= qf;
            acc[MONC_B_QW] *= qf;
            acc[MONC_B_CW] *= wmass;
            acc[MONC_B_PW] *= wmass;
#pragma unroll
            for (int s = 0; s < NS; s++) {
                acc[MONC_B_SCALAR0 + 3 * s] *= mass;
                acc[MONC_B_SCALAR0 + 3 * s + 1] *= mass;
            }
            if constexpr (PW) {
                // FP64 compute scales by the level table's 1/dzn, which is
                // what the faces use
                const double rz =
                    std::is_same<T, double>::value ? (double)lev[LV_RDZN * NZP + k] : rdzn;
                if (store)
                    acc[MONC_B_COURANT] =
                        fmax(fmax(amax[0] * cdx, amax[1] * cdy), amax[2] * dt * rz);
            }
            (void)rdzn;
            acc[MONC_B_NONFINITE] = store ? (double)nonfinite : 0.0;
        }
        // block reduction in a fixed order, reusing the LDS
        __syncthreads();
        double* red = reinterpret_cast<double*>(smem_raw);  // [waves][NACC]
#pragma unroll
        for (int q = 0; q < NACC; q++) {
            const int op = bud_op(q);
            double v = acc[q];
            for (int o = 32; o > 0; o >>= 1) v = bud_comb(v, __shfl_xor(v, o, 64), op);
            if (lane == 0) red[wv * NACC + q] = v;
        }
        __syncthreads();
        if (threadIdx.x < NB) {
            const int q = threadIdx.x;
            const int op = bud_op(q);
            double* row = tj.partial_row;
            const bool scalar_slot = q >= MONC_B_SCALAR0;
            const int s = scalar_slot ? (q - MONC_B_SCALAR0) / 3 : -1;
            const bool mine_scalar = scalar_slot && s >= tj.s0 && s < tj.s0 + NS;
            const bool mine_mom = !scalar_slot && PW;
            if (mine_scalar || mine_mom || q == MONC_B_NONFINITE) {
                const int lq = scalar_slot ? q - 3 * tj.s0 : q;
                double v = red[lq];
                for (int w2 = 1; w2 < MARCH_WAVES; w2++) v = bud_comb(v, red[w2 * NACC + lq], op);
                if (q == MONC_B_NONFINITE && !tj.first_pass) v += row[q];
                row[q] = v;
            } else if (tj.first_pass) {
                row[q] = bud_ident(op);
            }
        }
    }
}

// One workgroup per tile.
template <typename Ts, typename T, int MODE, bool PW, int NS, bool BUD, int NCH,
          int OPT = 0>
__global__ void __launch_bounds__((march_waves<Ts, T>() * 64))
    __attribute__((amdgpu_waves_per_eu(2))) advect_march(MarchArgs m) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // Consecutive tiles along y go to the same XCD (workgroups are dealt to
    // the 8 XCDs round-robin), so neighbouring tiles share halo columns
    // through that XCD's L2.
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    TileJob t;
    t.s0 = m.s0;
    t.ti = m.ti;
    t.jt = b % m.njt;
    t.seg = b / m.njt;
    t.partial_row = BUD ? m.a.partials + (size_t)blockIdx.x * NB : nullptr;
    t.first_pass = m.first_pass;
    march_tile<Ts, T, MODE, PW, NS, BUD, NCH, OPT>(m.a, t, smem_raw);
}

}  // namespace monc
