// advect.hip -- fused MONC advection kernels for gfx950.
//
// One launch evaluates the Piacsek-Williams momentum source terms and the
// ULTIMATE/QUICKEST scalar source terms (Brown et al., Sec. 3.1) for every
// interior point, and in the step variant also integrates them ("step
// fields", Sec. 3) and accumulates the FP64 budget partials.
#include <type_traits>

#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

constexpr int BLOCK = 256;

template <typename Ts, typename T>
__device__ __forceinline__ T ldf(const Ts* __restrict__ p, long idx, double off) {
    if constexpr (std::is_same<Ts, double>::value) {
        return (T)(p[idx] - off);
    } else if constexpr (std::is_same<Ts, float>::value) {
        return (T)p[idx];
    } else {
        return to_compute<bf16, float>(p[idx]);
    }
}

__device__ __forceinline__ double wave_reduce(double v, int op) {
    // op: 0 sum, 1 max, 2 min.  Fixed butterfly; lane 0's result is used.
    for (int o = 32; o > 0; o >>= 1) {
        double w = __shfl_xor(v, o, 64);
        v = op == 0 ? v + w : (op == 1 ? fmax(v, w) : fmin(v, w));
    }
    return v;
}

__host__ __device__ __forceinline__ int budget_op(int q) {
    if (q == MONC_B_COURANT) return 1;
    if (q >= MONC_B_SCALAR0 && (q - MONC_B_SCALAR0) % 3 == 2) return 2;
    return 0;
}

__device__ __forceinline__ double budget_identity(int q) {
    int op = budget_op(q);
    return op == 2 ? __builtin_huge_val() : 0.0;
}

// Block-level deterministic reduction of NB per-thread values into
// partials[blockIdx.x][q].
__device__ void block_budget(double* acc, double* partials) {
    __shared__ double red[BLOCK / 64][NB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < NB; q++) {
        double v = wave_reduce(acc[q], budget_op(q));
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        int q = threadIdx.x, op = budget_op(q);
        double v = red[0][q];
        for (int w = 1; w < BLOCK / 64; w++) {
            double x = red[w][q];
            v = op == 0 ? v + x : (op == 1 ? fmax(v, x) : fmin(v, x));
        }
        partials[(long)blockIdx.x * NB + q] = v;
    }
}

// ---------------------------------------------------------------------------
// Point-per-thread fused kernel.  Grid-stride over interior points, z fastest.
// Ts = storage type of the inputs, To = output type, T = compute type.
// ---------------------------------------------------------------------------
template <typename Ts, typename To, typename T, int MODE, bool PW, bool TVD, bool BUD>
__global__ void __launch_bounds__(BLOCK) advect_point(AdvArgs a) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long sy = nz, sx = (long)(ny + 4) * nz;
    const long npts = (long)nx * ny * nz;
    const T r4dx = (T)(0.25 / a.dx), r4dy = (T)(0.25 / a.dy);
    const T r2dx = (T)(0.5 / a.dx), r2dy = (T)(0.5 / a.dy);
    const T rdx = (T)(1.0 / a.dx), rdy = (T)(1.0 / a.dy);
    const T cfx = (T)(a.dt / a.dx), cfy = (T)(a.dt / a.dy);
    const T rfx = (T)(a.dx / a.dt), rfy = (T)(a.dy / a.dt);
    const Ts* __restrict__ U = (const Ts*)a.in[0];
    const Ts* __restrict__ V = (const Ts*)a.in[1];
    const Ts* __restrict__ W = (const Ts*)a.in[2];

    double acc[BUD ? NB : 1];
    if constexpr (BUD) {
        for (int q = 0; q < NB; q++) acc[q] = budget_identity(q);
    }

    for (long p = (long)blockIdx.x * BLOCK + threadIdx.x; p < npts;
         p += (long)gridDim.x * BLOCK) {
        const int k = (int)(p % nz);
        const long col = p / nz;
        const int j = (int)(col % ny);
        const int i = (int)(col / ny);
        const long c = (long)(i + 2) * sx + (long)(j + 2) * sy + k;
        const Level<T> L = make_level<T>(a.rdz, a.rho, a.rhon, k, nz);
        const bool hb = k > 0, ht = k < nz - 1;

        auto u = [&](int di, int dj, int dk) -> T {
            return ldf<Ts, T>(U, c + di * sx + dj * sy + dk, 0.0);
        };
        auto v = [&](int di, int dj, int dk) -> T {
            return ldf<Ts, T>(V, c + di * sx + dj * sy + dk, 0.0);
        };
        auto w = [&](int di, int dj, int dk) -> T {
            const int kk = k + dk;
            if (kk < 0 || kk >= nz - 1) return (T)0;
            return ldf<Ts, T>(W, c + di * sx + dj * sy + dk, 0.0);
        };

        const T u_c = u(0, 0, 0), v_c = v(0, 0, 0), w_c = w(0, 0, 0);
        const T u_m = u(-1, 0, 0), v_s = v(0, -1, 0), w_b = w(0, 0, -1);
        // anelastic mass divergence of this p-cell
        const T D = L.rhon * ((u_c - u_m) * rdx + (v_c - v_s) * rdy) +
                    L.rdz * (L.rho * w_c - L.rho_km * w_b);

        T s_u = 0, s_v = 0, s_w = 0;
        if constexpr (PW) {
            const T u_b = hb ? u(0, 0, -1) : (T)0, u_t = ht ? u(0, 0, 1) : (T)0;
            const T v_b = hb ? v(0, 0, -1) : (T)0, v_t = ht ? v(0, 0, 1) : (T)0;
            s_u = pw_su<T>(u_m, u_c, u(1, 0, 0), u(0, -1, 0), u(0, 1, 0), u_b, u_t,
                           v_s, v(1, -1, 0), v_c, v(1, 0, 0), w_b, w(1, 0, -1), w_c,
                           w(1, 0, 0), L, r4dx, r4dy);
            s_v = pw_sv<T>(v(-1, 0, 0), v_c, v(1, 0, 0), v_s, v(0, 1, 0), v_b, v_t,
                           u_m, u(-1, 1, 0), u_c, u(0, 1, 0), w_b, w(0, 1, -1), w_c,
                           w(0, 1, 0), L, r4dx, r4dy);
            if (ht)
                s_w = pw_sw<T>(u_c, u_t, u_m, u(-1, 0, 1), v_c, v_t, v_s, v(0, -1, 1),
                               w_c, w(-1, 0, 0), w(1, 0, 0), w(0, -1, 0), w(0, 1, 0),
                               w_b, w(0, 0, 1), L, r2dx, r2dy);
            else
                s_w = (T)0;
            if constexpr (MODE == TEND) {
                ((To*)a.out[0])[c] = (To)s_u;
                ((To*)a.out[1])[c] = (To)s_v;
                ((To*)a.out[2])[c] = (To)s_w;
            }
        }

        // vertical coefficients of the face below (k-1/2)
        T rdzn_b = 0;
        if (hb) rdzn_b = (T)(2.0 / (1.0 / a.rdz[k - 1] + 1.0 / a.rdz[k]));

        double s_sc[MAXS];
        if constexpr (TVD) {
            for (int s = 0; s < a.nscal; s++) {
                const Ts* __restrict__ Q = (const Ts*)a.in[3 + s];
                const double off = (MODE == STEP) ? a.phi0[s] : 0.0;
                auto f = [&](int di, int dj, int dk) -> T {
                    return ldf<Ts, T>(Q, c + di * sx + dj * sy + dk, off);
                };
                const T p_c = f(0, 0, 0);
                const T p_w = f(-1, 0, 0), p_ww = f(-2, 0, 0), p_e = f(1, 0, 0),
                        p_ee = f(2, 0, 0);
                const T p_s = f(0, -1, 0), p_ss = f(0, -2, 0), p_n = f(0, 1, 0),
                        p_nn = f(0, 2, 0);
                const T fxp = tvd_flux<T>(u_c, p_w, p_c, p_e, p_ee, cfx, rfx, L.rhon);
                const T fxm = tvd_flux<T>(u_m, p_ww, p_w, p_c, p_e, cfx, rfx, L.rhon);
                const T fyp = tvd_flux<T>(v_c, p_s, p_c, p_n, p_nn, cfy, rfy, L.rhon);
                const T fym = tvd_flux<T>(v_s, p_ss, p_s, p_c, p_n, cfy, rfy, L.rhon);
                // top face k+1/2
                T fzp = 0;
                if (ht) {
                    const T p_t = f(0, 0, 1);
                    const bool pos = w_c >= (T)0;
                    if ((pos && k == 0) || (!pos && k + 2 > nz - 1)) {
                        fzp = upwind_flux<T>(w_c, p_c, p_t, L.rho);
                    } else {
                        const T p_b = hb ? f(0, 0, -1) : p_c;
                        const T p_tt = (k + 2 <= nz - 1) ? f(0, 0, 2) : p_t;
                        const T cfz = (T)a.dt * L.rdzn;
                        const T rfz = (T)(1.0 / (a.dt * (double)L.rdzn));
                        fzp = tvd_flux<T>(w_c, p_b, p_c, p_t, p_tt, cfz, rfz, L.rho);
                    }
                }
                // bottom face k-1/2 (= top face of cell k-1)
                T fzm = 0;
                if (hb) {
                    const T p_b = f(0, 0, -1);
                    const int kb = k - 1;
                    const bool pos = w_b >= (T)0;
                    if ((pos && kb == 0) || (!pos && kb + 2 > nz - 1)) {
                        fzm = upwind_flux<T>(w_b, p_b, p_c, L.rho_km);
                    } else {
                        const T p_bb = (kb >= 1) ? f(0, 0, -2) : p_b;
                        const T p_t = (kb + 2 <= nz - 1) ? f(0, 0, 1) : p_c;
                        const T cfz = (T)a.dt * rdzn_b;
                        const T rfz = (T)(1.0 / (a.dt * (double)rdzn_b));
                        fzm = tvd_flux<T>(w_b, p_bb, p_b, p_c, p_t, cfz, rfz, L.rho_km);
                    }
                }
                T ss = -L.rhon_inv *
                       ((fxp - fxm) * rdx + (fyp - fym) * rdy + L.rdz * (fzp - fzm));
                // stored values are anomalies from phi0: add the term of the constant
                ss -= (T)a.phi0[s] * D * L.rhon_inv;
                s_sc[s] = (double)ss;
                if constexpr (MODE == TEND) ((To*)a.out[3 + s])[c] = (To)ss;
            }
        }

        if constexpr (MODE == STEP) {
            const double dt = a.dt;
            const double* __restrict__ Ud = (const double*)a.in[0];
            const double* __restrict__ Vd = (const double*)a.in[1];
            const double* __restrict__ Wd = (const double*)a.in[2];
            const double nu = Ud[c] + dt * (double)s_u;
            const double nv = Vd[c] + dt * (double)s_v;
            const double nw = ht ? Wd[c] + dt * (double)s_w : 0.0;
            ((double*)a.out[0])[c] = nu;
            ((double*)a.out[1])[c] = nv;
            ((double*)a.out[2])[c] = nw;
            double nsc[MAXS];
            for (int s = 0; s < a.nscal; s++) {
                const double* __restrict__ Qd = (const double*)a.in[3 + s];
                nsc[s] = Qd[c] + dt * s_sc[s];
                ((double*)a.out[3 + s])[c] = nsc[s];
            }
            if constexpr (BUD) {
                const double rdzk = a.rdz[k];
                const double mass = a.rhon[k] / rdzk;
                const double dzk = 1.0 / rdzk;
                const double uc = Ud[c], vc = Vd[c];
                const double wc = ht ? Wd[c] : 0.0;
                const double um = Ud[c - sx], vs = Vd[c - sy];
                const double wb = hb ? Wd[c - 1] : 0.0;
                const double Dd = (double)D;
                acc[MONC_B_CU] += mass * (double)s_u;
                acc[MONC_B_CV] += mass * (double)s_v;
                acc[MONC_B_PU] += mass * uc * (double)s_u;
                acc[MONC_B_PV] += mass * vc * (double)s_v;
                acc[MONC_B_QU] += -0.25 * dzk * Dd * (uc * uc + um * um);
                acc[MONC_B_QV] += -0.25 * dzk * Dd * (vc * vc + vs * vs);
                acc[MONC_B_QW] += -0.25 * dzk * Dd * (wc * wc + wb * wb);
                double cr = fmax(fabs(uc) * dt / a.dx, fabs(vc) * dt / a.dy);
                if (ht) {
                    const double dzn = 0.5 * (dzk + 1.0 / a.rdz[k + 1]);
                    const double wmass = a.rho[k] * dzn;
                    acc[MONC_B_CW] += wmass * (double)s_w;
                    acc[MONC_B_PW] += wmass * wc * (double)s_w;
                    cr = fmax(cr, fabs(wc) * dt / dzn);
                }
                acc[MONC_B_COURANT] = fmax(acc[MONC_B_COURANT], cr);
                double nf = (!isfinite(nu)) + (!isfinite(nv)) + (!isfinite(nw));
                for (int s = 0; s < a.nscal; s++) {
                    const double* __restrict__ Qd = (const double*)a.in[3 + s];
                    const double ph = Qd[c];
                    acc[MONC_B_SCALAR0 + 3 * s] += mass * s_sc[s];
                    acc[MONC_B_SCALAR0 + 3 * s + 1] += mass * ph;
                    acc[MONC_B_SCALAR0 + 3 * s + 2] = fmin(acc[MONC_B_SCALAR0 + 3 * s + 2], ph);
                    nf += !isfinite(nsc[s]);
                }
                acc[MONC_B_NONFINITE] += nf;
            }
        }
    }
    if constexpr (BUD) block_budget(acc, a.partials);
}

template <typename Ts, typename To, typename T, int MODE>
hipError_t launch_variant(bool pw, bool tvd, bool bud, const AdvArgs& a, hipStream_t s) {
    const long npts = (long)a.nx * a.ny * a.nz;
    int blocks = (MODE == STEP) ? step_blocks(a.nx, a.ny, a.nz)
                                : (int)((npts + BLOCK - 1) / BLOCK);
    if (blocks < 1) blocks = 1;
    if (pw && tvd) {
        if (bud)
            advect_point<Ts, To, T, MODE, true, true, true><<<blocks, BLOCK, 0, s>>>(a);
        else
            advect_point<Ts, To, T, MODE, true, true, false><<<blocks, BLOCK, 0, s>>>(a);
    } else if (pw) {
        advect_point<Ts, To, T, MODE, true, false, false><<<blocks, BLOCK, 0, s>>>(a);
    } else {
        advect_point<Ts, To, T, MODE, false, true, false><<<blocks, BLOCK, 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

int step_blocks(int nx, int ny, int nz) {
    const long npts = (long)nx * ny * nz;
    long b = (npts + BLOCK - 1) / BLOCK;
    if (b > 2048) b = 2048;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_advect(int dtype, int mode, bool pw, bool tvd, bool mixed,
                         const AdvArgs& a, hipStream_t s) {
    const bool bud = a.partials != nullptr;
    if (mode == STEP) {
        if (mixed) return launch_variant<double, double, float, STEP>(true, true, bud, a, s);
        return launch_variant<double, double, double, STEP>(true, true, bud, a, s);
    }
    switch (dtype) {
        case MONC_F64:
            return launch_variant<double, double, double, TEND>(pw, tvd, false, a, s);
        case MONC_F32:
            return launch_variant<float, float, float, TEND>(pw, tvd, false, a, s);
        case MONC_BF16:
            return launch_variant<bf16, float, float, TEND>(pw, tvd, false, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace monc
