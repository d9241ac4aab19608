// monc_scheme.hpp -- device arithmetic of the MONC advection schemes.
//
// Piacsek-Williams momentum source terms and ULTIMATE-limited QUICKEST scalar
// fluxes (the two advection schemes of Brown et al., Sec. 3.1), written for
// the GPU: reciprocals are precomputed per level, and the ULTIMATE bound is
// evaluated in flux space so that no division remains in the inner loop.
// Every function is templated on the compute type T (double or float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace monc {

// Per-level vertical coefficients.  Built once per level
// from rdz, rho, rhon (float64) and rounded to T.
template <typename T>
struct Level {
    T rdz;        // 1/dz_k
    T rhon;       // density at the centre of cell k
    T rho;        // density at the top face of cell k
    T rho_km;     // density at the top face of cell k-1 (0 for k = 0)
    T rho_kp;     // density at the top face of cell k+1 (0 for k = nz-1)
    T zterm;      // rdz_k / (4 rhon_k)
    T rhon_inv;   // 1/rhon_k
    T rho_inv;    // 1/rho_k
    T rdzn;       // 1/dzn_k, dzn_k = (dz_k + dz_{k+1})/2 (0 on the lid)
    T alpha;      // dz_k rhon_k / (2 dzn_k)
    T beta;       // dz_{k+1} rhon_{k+1} / (2 dzn_k)
    T mass;       // rhon_k dz_k   (budget weight, p-cells)
    T wmass;      // rho_k dzn_k   (budget weight, w-cells)
    T dz;         // dz_k
};

template <typename T>
__device__ __forceinline__ Level<T> make_level(const double* __restrict__ rdz,
                                               const double* __restrict__ rho,
                                               const double* __restrict__ rhon,
                                               int k, int nz) {
    Level<T> L;
    double rdzk = rdz[k];
    double dzk = 1.0 / rdzk;
    double rhonk = rhon[k];
    double rhok = rho[k];
    L.rdz = (T)rdzk;
    L.rhon = (T)rhonk;
    L.rho = (T)rhok;
    L.rho_km = (T)(k > 0 ? rho[k - 1] : 0.0);
    L.rho_kp = (T)(k < nz - 1 ? rho[k + 1] : 0.0);
    L.zterm = (T)(rdzk / (4.0 * rhonk));
    L.rhon_inv = (T)(1.0 / rhonk);
    L.rho_inv = (T)(1.0 / rhok);
    L.dz = (T)dzk;
    L.mass = (T)(rhonk * dzk);
    if (k < nz - 1) {
        double dzk1 = 1.0 / rdz[k + 1];
        double dzn = 0.5 * (dzk + dzk1);
        L.rdzn = (T)(1.0 / dzn);
        L.alpha = (T)(dzk * rhonk / (2.0 * dzn));
        L.beta = (T)(dzk1 * rhon[k + 1] / (2.0 * dzn));
        L.wmass = (T)(rhok * dzn);
    } else {
        L.rdzn = (T)0;
        L.alpha = (T)0;
        L.beta = (T)0;
        L.wmass = (T)0;
    }
    return L;
}

// ---------------------------------------------------------------------------
// PW, u-component at (i+1/2, j, k).  Names: u_m/u_p = u at i-1/i+1, u_s/u_n =
// j-1/j+1, u_b/u_t = k-1/k+1; v_c/v_e = v at (i,j)/(i+1,j), v_cs/v_es at j-1;
// w_c/w_e = w at (i,k)/(i+1,k), w_cb/w_eb at k-1 (already zero through the
// ground / lid where applicable).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T pw_su(T u_m, T u_c, T u_p, T u_s, T u_n, T u_b, T u_t,
                                   T v_cs, T v_es, T v_c, T v_e, T w_cb, T w_eb,
                                   T w_c, T w_e, const Level<T>& L, T r4dx, T r4dy) {
    T a = u_m + u_c, b = u_c + u_p;
    T xt = (a * a - b * b) * r4dx;
    T yt = ((v_cs + v_es) * (u_s + u_c) - (v_c + v_e) * (u_c + u_n)) * r4dy;
    T fb = L.rho_km * (w_cb + w_eb) * (u_b + u_c);
    T ft = L.rho * (w_c + w_e) * (u_c + u_t);
    return xt + yt + L.zterm * (fb - ft);
}

// PW, v-component at (i, j+1/2, k): the mirror of pw_su with x and y swapped.
// u_cw/u_nw = u at (i-1, j)/(i-1, j+1), u_c/u_n = u at (i,j)/(i,j+1);
// v_w/v_e = v at i-1/i+1, v_s/v_n = j-1/j+1; w_c/w_n = w at (j,k)/(j+1,k).
template <typename T>
__device__ __forceinline__ T pw_sv(T v_w, T v_c, T v_e, T v_s, T v_n, T v_b, T v_t,
                                   T u_cw, T u_nw, T u_c, T u_n, T w_cb, T w_nb,
                                   T w_c, T w_n, const Level<T>& L, T r4dx, T r4dy) {
    T a = v_s + v_c, b = v_c + v_n;
    T yt = (a * a - b * b) * r4dy;
    T xt = ((u_cw + u_nw) * (v_w + v_c) - (u_c + u_n) * (v_c + v_e)) * r4dx;
    T fb = L.rho_km * (w_cb + w_nb) * (v_b + v_c);
    T ft = L.rho * (w_c + w_n) * (v_c + v_t);
    return xt + yt + L.zterm * (fb - ft);
}

// PW, w-component at (i, j, k+1/2), k < nz-1.  u_c/u_ct = u at (i,k)/(i,k+1),
// u_w/u_wt at i-1; v_c/v_ct, v_s/v_st likewise in y; w_w/w_e/w_s/w_n lateral
// neighbours, w_b/w_t = w at k-1/k+1 (zero at ground / lid).
template <typename T>
__device__ __forceinline__ T pw_sw(T u_c, T u_ct, T u_w, T u_wt, T v_c, T v_ct, T v_s,
                                   T v_st, T w_c, T w_w, T w_e, T w_s, T w_n, T w_b,
                                   T w_t, const Level<T>& L, T r2dx, T r2dy) {
    T fxe = (L.alpha * u_c + L.beta * u_ct) * (w_c + w_e);
    T fxw = (L.alpha * u_w + L.beta * u_wt) * (w_w + w_c);
    T fyn = (L.alpha * v_c + L.beta * v_ct) * (w_c + w_n);
    T fys = (L.alpha * v_s + L.beta * v_st) * (w_s + w_c);
    T fzt = (L.rho * w_c + L.rho_kp * w_t) * (w_c + w_t);
    T fzb = (L.rho_km * w_b + L.rho * w_c) * (w_b + w_c);
    return -L.rho_inv * ((fxe - fxw) * r2dx + (fyn - fys) * r2dy +
                         L.rdzn * (T)0.25 * (fzt - fzb));
}

// ---------------------------------------------------------------------------
// ULTIMATE-limited QUICKEST flux through one face.
//   a      normal velocity on the face
//   pm,p0  scalar in the two cells on the minus side (far, near)
//   p1,p2  scalar in the two cells on the plus side (near, far)
//   cfac   dt / spacing (Courant number per unit speed)
//   rfac   spacing / dt
//   mass   density factor of the face (rhon_k for lateral faces, rho_k for
//          vertical ones)
// For a >= 0 the upwind triple is (U,C,D) = (pm,p0,p1), else (p2,p1,p0).
//
// The limited face value is written as C plus an offset, and everything is
// multiplied by a, so that no division and no choice of the upwind triple
// beyond C and one difference remains.  With s = sign(a), d1 = p1 - p0 and
// e = C - U times s (p0 - pm for a >= 0, p2 - p1 otherwise):
//   a (D - C)        = |a| d1
//   a (phi* - C)     = |a| [ (1-c)/2 d1 - (1-c^2)/6 (d1 - e) ]     (QUICKEST)
//   a (bound - C)    = e (spacing/dt - |a|)      bound = U + (C-U)/c
// The profile is monotone exactly where d1 and e have the same sign.  Taking
// all three offsets into the frame where d1 >= 0 (multiplying by sign(d1)),
// the ULTIMATE clamp of phi* between C and the nearer of D and the bound is
// max(0, min of the three), and where the profile is not monotone the third
// offset is <= 0, so the same expression returns C.  This needs Courant
// numbers c = |a| dt / spacing <= 1 (the stability limit of the scheme).
// ---------------------------------------------------------------------------
// x with its sign flipped where s has its sign bit set
__device__ __forceinline__ double flip_sign_by(double x, double s) {
    return __hiloint2double(__double2hiint(x) ^ (__double2hiint(s) & (int)0x80000000),
                            __double2loint(x));
}
__device__ __forceinline__ float flip_sign_by(float x, float s) {
    return __uint_as_float(__float_as_uint(x) ^ (__float_as_uint(s) & 0x80000000u));
}

template <typename T>
__device__ __forceinline__ T tvd_flux(T a, T pm, T p0, T p1, T p2, T cfac, T rfac,
                                      T mass) {
    const bool pos = a >= (T)0;
    const T d1 = p1 - p0;
    const T e = pos ? p0 - pm : p2 - p1;
    const T C = pos ? p0 : p1;
    const T A = fabs(a);
    const T c = A * cfac;
    const T se = flip_sign_by(e, d1);  // e in the frame d1 >= 0
    const T ad1 = fabs(d1);
    const T x_down = A * ad1;           // toward D
    const T x_bound = se * (rfac - A);  // toward the ULTIMATE bound
    const T h = fma((T)-0.5, c, (T)0.5);
    const T q6 = fma(-c, c * (T)(1.0 / 6.0), (T)(1.0 / 6.0));
    const T x_star = A * fma(h, ad1, -(q6 * (ad1 - se)));  // toward phi*
    const T lim = fmax(fmin(fmin(x_star, x_down), x_bound), (T)0);
    return mass * fma(a, C, copysign(lim, d1));
}

// ---------------------------------------------------------------------------
// Other source terms of the dynamics group, combined with the advection
// source terms before the fields are stepped (the paper's hybrid structure,
// Sec. 3: the non-advection components run beside the advection).  The paper
// defines no such component; the two here are the f-plane Coriolis force
// toward a geostrophic wind and the buoyancy of theta.
//   coriolis_u: at the u point (i+1/2, j); v_c, v_e = v at (i, j), (i+1, j),
//               v_s, v_es = v at (i, j-1), (i+1, j-1) (the four v points
//               around it)
//   coriolis_v: at the v point (i, j+1/2); u_c, u_w = u at (i, j), (i-1, j),
//               u_n, u_nw = u at (i, j+1), (i-1, j+1)
//   buoyancy_w: at the top face of cell k (k < nz-1): theta of cells k, k+1,
//               gth = grav / th0
// ---------------------------------------------------------------------------
__device__ __forceinline__ double coriolis_u(double fcor, double vg, double v_c, double v_e,
                                             double v_s, double v_es) {
    return fcor * ((((v_c + v_e) + v_s) + v_es) * 0.25 - vg);
}
__device__ __forceinline__ double coriolis_v(double fcor, double ug, double u_c, double u_w,
                                             double u_n, double u_nw) {
    return -fcor * ((((u_c + u_w) + u_n) + u_nw) * 0.25 - ug);
}
__device__ __forceinline__ double buoyancy_w(double gth, double th0, double th_k,
                                             double th_kp) {
    return gth * ((th_k + th_kp) * 0.5 - th0);
}

// Centred flux (the PW flux form applied to a scalar, MONC's alternative
// scalar scheme): the face value is the mean of the two cells beside the face.
template <typename T>
__device__ __forceinline__ T centred_flux(T a, T p0, T p1, T mass) {
    return mass * a * ((p0 + p1) * (T)0.5);
}

// First-order upwind flux (used where the far-upwind cell lies outside the
// column, next to the ground and the lid).
template <typename T>
__device__ __forceinline__ T upwind_flux(T a, T p0, T p1, T mass) {
    return mass * a * (a >= (T)0 ? p0 : p1);
}

// ---------------------------------------------------------------------------
// Storage conversions
// ---------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};

template <typename Ts, typename T>
__device__ __forceinline__ T to_compute(Ts x) {
    return (T)x;
}
template <>
__device__ __forceinline__ float to_compute<bf16, float>(bf16 x) {
    return __uint_as_float(((uint32_t)x.bits) << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    const uint32_t b = __float_as_uint(f);
    const uint32_t rounded = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
    // inf and nan keep their class (a nan stays a quiet nan); a select, not a branch
    const uint32_t special = (b >> 16) | ((b & 0xffffu) ? 0x40u : 0u);
    return (uint16_t)(((b & 0x7f800000u) == 0x7f800000u) ? special : rounded);
}

}  // namespace monc
