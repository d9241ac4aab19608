// scaled.hip -- the work-scaled Piacsek-Williams experiment.
//
// Brown et al. (Sec. 4) scale the arithmetic of the PW scheme up to that of
// the ULTIMATE scheme (about sixteen times as much) to see how a GPU behaves
// once the same data carries more computation.  Here the same question is put
// to one MI355X in roofline terms: the PW source terms are evaluated `work`
// times per grid point on the same loaded values, each repetition chained to
// the previous one through an empty asm statement so that the compiler can
// neither merge nor drop repetitions.  The result is bitwise the result of
// one evaluation; bytes per point stay the same while arithmetic grows
// `work`-fold, so a sweep shows where FP64 and FP32 turn from HBM-bound to
// ALU-bound.
//
// One thread per grid point: a wave covers 64 levels of one column, a
// workgroup 4 columns; neighbours are read from global memory (the L1/L2
// caches serve the re-reads) at wrapped periodic indices, and the per-level
// coefficients come from an LDS table built once per workgroup.
#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

constexpr int SC_COLS = 4;

struct ScaledArgs {
    const void* u;
    const void* v;
    const void* w;
    void* su;
    void* sv;
    void* sw;
    int nx, ny, nz;
    double dx, dy;
    const double *rdz, *rho, *rhon;
    int work;
};

// Makes x opaque to the optimiser and orders it after `dep`.
template <typename T>
__device__ __forceinline__ void chain(T& x, T dep) {
    asm volatile("" : "+v"(x) : "v"(dep));
}

template <typename T>
__global__ void __launch_bounds__(64 * SC_COLS) pw_scaled(ScaledArgs a) {
    __shared__ Level<T> lev[64];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nchunk = (nz + 63) / 64;
    const int chunk = blockIdx.x % nchunk;
    const int jb = blockIdx.x / nchunk;
    const int i = blockIdx.y;
    const int k = 64 * chunk + (int)threadIdx.x;
    const int j = jb * SC_COLS + (int)threadIdx.y;
    if (threadIdx.y == 0 && k < nz) lev[threadIdx.x] = make_level<T>(a.rdz, a.rho, a.rhon, k, nz);
    __syncthreads();
    if (k >= nz || j >= ny) return;
    const Level<T> L = lev[threadIdx.x];

    const T* U = static_cast<const T*>(a.u);
    const T* V = static_cast<const T*>(a.v);
    const T* W = static_cast<const T*>(a.w);
    const long sx = (long)(ny + 4) * nz;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
    const int km = k > 0 ? k - 1 : 0, kp = k < nz - 1 ? k + 1 : k;
    auto at = [&](const T* f, int ii, int jj, int kk) {
        return f[(long)(ii + 2) * sx + (long)(jj + 2) * nz + kk];
    };
    // values outside the column are zero; w on the lid is zero
    const bool hb = k > 0, ht = k < nz - 1;
    auto wv = [&](int ii, int jj, int kk) { return kk < nz - 1 ? at(W, ii, jj, kk) : (T)0; };

    T uc = at(U, i, j, k), um = at(U, im, j, k), up = at(U, ip, j, k);
    T us = at(U, i, jm, k), un = at(U, i, jp, k);
    T ub = hb ? at(U, i, j, km) : (T)0, ut = ht ? at(U, i, j, kp) : (T)0;
    T u_nw = at(U, im, jp, k), u_wt = ht ? at(U, im, j, kp) : (T)0;
    T vc = at(V, i, j, k), vw = at(V, im, j, k), ve = at(V, ip, j, k);
    T vs = at(V, i, jm, k), vn = at(V, i, jp, k);
    T vb = hb ? at(V, i, j, km) : (T)0, vt = ht ? at(V, i, j, kp) : (T)0;
    T v_es = at(V, ip, jm, k), v_st = ht ? at(V, i, jm, kp) : (T)0;
    T wc = wv(i, j, k), we = wv(ip, j, k), ww = wv(im, j, k);
    T ws = wv(i, jm, k), wn = wv(i, jp, k);
    T wb = hb ? wv(i, j, km) : (T)0, wt = ht ? wv(i, j, kp) : (T)0;
    T w_eb = hb ? wv(ip, j, km) : (T)0, w_nb = hb ? wv(i, jp, km) : (T)0;

    const T r4dx = (T)(0.25 / a.dx), r4dy = (T)(0.25 / a.dy);
    const T r2dx = (T)(0.5 / a.dx), r2dy = (T)(0.5 / a.dy);
    T su = (T)0, sv = (T)0, sw = (T)0;
    for (int r = 0; r < a.work; r++) {
        // every input of this repetition depends on the previous result
        const T dep = su + sv + sw;
        chain(uc, dep); chain(um, dep); chain(up, dep); chain(us, dep); chain(un, dep);
        chain(ub, dep); chain(ut, dep); chain(u_nw, dep); chain(u_wt, dep);
        chain(vc, dep); chain(vw, dep); chain(ve, dep); chain(vs, dep); chain(vn, dep);
        chain(vb, dep); chain(vt, dep); chain(v_es, dep); chain(v_st, dep);
        chain(wc, dep); chain(we, dep); chain(ww, dep); chain(ws, dep); chain(wn, dep);
        chain(wb, dep); chain(wt, dep); chain(w_eb, dep); chain(w_nb, dep);
        su = pw_su<T>(um, uc, up, us, un, ub, ut, vs, v_es, vc, ve, wb, w_eb, wc, we, L, r4dx,
                      r4dy);
        sv = pw_sv<T>(vw, vc, ve, vs, vn, vb, vt, um, u_nw, uc, un, wb, w_nb, wc, wn, L, r4dx,
                      r4dy);
        sw = k < nz - 1 ? pw_sw<T>(uc, ut, um, u_wt, vc, vt, vs, v_st, wc, ww, we, ws, wn, wb, wt,
                                   L, r2dx, r2dy)
                        : (T)0;
    }
    const long g = (long)(i + 2) * sx + (long)(j + 2) * nz + k;
    static_cast<T*>(a.su)[g] = su;
    static_cast<T*>(a.sv)[g] = sv;
    static_cast<T*>(a.sw)[g] = sw;
}

}  // namespace

hipError_t launch_pw_scaled(int dtype, const void* u, const void* v, const void* w, void* su,
                            void* sv, void* sw, int nx, int ny, int nz, double dx, double dy,
                            const double* rdz, const double* rho, const double* rhon, int work,
                            hipStream_t s) {
    ScaledArgs a{u, v, w, su, sv, sw, nx, ny, nz, dx, dy, rdz, rho, rhon, work};
    const dim3 grid(((nz + 63) / 64) * ((ny + SC_COLS - 1) / SC_COLS), nx);
    const dim3 block(64, SC_COLS);
    if (dtype == MONC_F64)
        pw_scaled<double><<<grid, block, 0, s>>>(a);
    else
        pw_scaled<float><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace monc
