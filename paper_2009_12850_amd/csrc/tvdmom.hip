// tvdmom.hip -- TVD (ULTIMATE-limited QUICKEST) advection of momentum.
//
// The ULTIMATE scheme that Brown et al. (Sec. 3.1) use for the scalars,
// applied to the three velocity components, each on its own C-grid control
// volume.  The mass flux through a face of that volume is the one the PW
// scheme uses; the value carried through the face is the limited QUICKEST
// value of the velocity component along the flux direction, upwind by the
// sign of the mass flux (with the mean of the two values beside the face in
// its place the scheme is PW).
//   u at (i+1/2,j,k): x-faces at cell centres carry rhon_k (u_i+u_{i+1})/2,
//                     y-faces at (i+1/2,j+1/2) rhon_k (v_ij+v_{i+1,j})/2,
//                     z-faces at (i+1/2,j,k+1/2) rho_k (w_ik+w_{i+1,k})/2;
//                     nothing passes the ground or the lid
//   v                 the same with x and y exchanged
//   w at (i,j,k+1/2): lateral faces carry alpha_k u_k + beta_k u_{k+1} (the
//                     mass weights of the PW w-equation), the z-face at the
//                     centre of cell q carries (rho_{q-1} w_{q-1} + rho_q w_q)/2
//                     with the ground and the lid as w = 0
// The Courant number of a face is |mass flux| over the density where the
// face sits, times dt over the distance between the two values beside it;
// where the far-upwind value of a z-stencil does not exist the face takes the
// upwind value.  tvd_flux takes any flux-like advecting quantity a with its
// own dt/spacing factor, so the w faces pass the mass flux itself.
//
// One thread per grid point: a wave covers 64 levels of one column, a
// workgroup 4 columns along y, and neighbours come through the caches.  Each
// interior face is evaluated by both points that share it.  Periodic
// neighbours are read at wrapped indices; halos are neither read nor written.
#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

constexpr int TM_COLS = 4;

// Flux through a z-face whose far-upwind value may not exist (next to the
// ground or the lid): first-order upwind there.
__device__ __forceinline__ double zface(double a, double pm, double p0, double p1, double p2,
                                        bool has_pm, bool has_p2, double cfac, double rfac,
                                        double mass) {
    const double t = tvd_flux(a, pm, p0, p1, p2, cfac, rfac, mass);
    const bool first = a >= 0.0 ? !has_pm : !has_p2;
    return first ? upwind_flux(a, p0, p1, mass) : t;
}

__device__ __forceinline__ int wrap(int x, int n) {
    x %= n;
    return x < 0 ? x + n : x;
}

__global__ void tvdmom_clear(double* cmax) {
    if (threadIdx.x == 0) cmax[0] = 0.0;
}

template <bool STEPF>
__global__ void __launch_bounds__(64 * TM_COLS) tvdmom_kernel(TvdMomArgs A) {
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    // Consecutive workgroups go to the same XCD (they are dealt to the 8 XCDs
    // round-robin), so neighbouring columns share that XCD's L2.
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int nchunk = (nz + 63) / 64;
    const int njg = (ny + TM_COLS - 1) / TM_COLS;
    const int chunk = b % nchunk;
    const int jg = (b / nchunk) % njg;
    const int i = b / (nchunk * njg);
    const int k = 64 * chunk + (int)threadIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(jg * TM_COLS + (int)threadIdx.y);
    const bool live = k < nz && j < ny;
    const int kc = k < nz ? k : nz - 1;  // dead lanes load in bounds, store nothing
    const int jc = j < ny ? j : ny - 1;

    auto col = [&](int ii, int jj) -> long {
        return ((long)(wrap(ii, nx) + 2) * (ny + 4) + (wrap(jj, ny) + 2)) * nz;
    };
    const long c00 = col(i, jc);
    const long cxm2 = col(i - 2, jc), cxm1 = col(i - 1, jc), cxp1 = col(i + 1, jc),
               cxp2 = col(i + 2, jc);
    const long cym2 = col(i, jc - 2), cym1 = col(i, jc - 1), cyp1 = col(i, jc + 1),
               cyp2 = col(i, jc + 2);
    const long cxp1ym1 = col(i + 1, jc - 1), cxm1yp1 = col(i - 1, jc + 1);

    const double* __restrict__ U = A.u;
    const double* __restrict__ V = A.v;
    const double* __restrict__ W = A.w;
    const bool zm1 = kc >= 1, zm2 = kc >= 2, zp1 = kc + 1 <= nz - 1, zp2 = kc + 2 <= nz - 1;
    const bool wlev = kc <= nz - 2;  // w at level k is not the lid

    // u and v: lateral stencils at level k, z stencils in the column
    const double u0 = U[c00 + kc];
    const double uxm2 = U[cxm2 + kc], uxm1 = U[cxm1 + kc], uxp1 = U[cxp1 + kc],
                 uxp2 = U[cxp2 + kc];
    const double uym2 = U[cym2 + kc], uym1 = U[cym1 + kc], uyp1 = U[cyp1 + kc],
                 uyp2 = U[cyp2 + kc];
    const double u_xm1yp1 = U[cxm1yp1 + kc];
    const double uzm2 = zm2 ? U[c00 + kc - 2] : 0.0, uzm1 = zm1 ? U[c00 + kc - 1] : 0.0;
    const double uzp1 = zp1 ? U[c00 + kc + 1] : 0.0, uzp2 = zp2 ? U[c00 + kc + 2] : 0.0;
    const double u_xm1zp1 = zp1 ? U[cxm1 + kc + 1] : 0.0;

    const double v0 = V[c00 + kc];
    const double vxm2 = V[cxm2 + kc], vxm1 = V[cxm1 + kc], vxp1 = V[cxp1 + kc],
                 vxp2 = V[cxp2 + kc];
    const double vym2 = V[cym2 + kc], vym1 = V[cym1 + kc], vyp1 = V[cyp1 + kc],
                 vyp2 = V[cyp2 + kc];
    const double v_xp1ym1 = V[cxp1ym1 + kc];
    const double vzm2 = zm2 ? V[c00 + kc - 2] : 0.0, vzm1 = zm1 ? V[c00 + kc - 1] : 0.0;
    const double vzp1 = zp1 ? V[c00 + kc + 1] : 0.0, vzp2 = zp2 ? V[c00 + kc + 2] : 0.0;
    const double v_ym1zp1 = zp1 ? V[cym1 + kc + 1] : 0.0;

    // w: zero on the ground (level -1) and the lid (level nz-1)
    const double w0 = wlev ? W[c00 + kc] : 0.0;
    const double wxm2 = wlev ? W[cxm2 + kc] : 0.0, wxm1 = wlev ? W[cxm1 + kc] : 0.0;
    const double wxp1 = wlev ? W[cxp1 + kc] : 0.0, wxp2 = wlev ? W[cxp2 + kc] : 0.0;
    const double wym2 = wlev ? W[cym2 + kc] : 0.0, wym1 = wlev ? W[cym1 + kc] : 0.0;
    const double wyp1 = wlev ? W[cyp1 + kc] : 0.0, wyp2 = wlev ? W[cyp2 + kc] : 0.0;
    const double wzm1 = zm1 ? W[c00 + kc - 1] : 0.0, wzm2 = zm2 ? W[c00 + kc - 2] : 0.0;
    const double wzp1 = kc + 1 <= nz - 2 ? W[c00 + kc + 1] : 0.0;
    const double wzp2 = kc + 2 <= nz - 2 ? W[c00 + kc + 2] : 0.0;
    const double w_xp1zm1 = zm1 ? W[cxp1 + kc - 1] : 0.0;
    const double w_yp1zm1 = zm1 ? W[cyp1 + kc - 1] : 0.0;

    // per-level geometry (as in the PW w-equation)
    const double rdz_k = A.rdz[kc], rhon_k = A.rhon[kc], rho_k = A.rho[kc];
    const double dz_k = 1.0 / rdz_k;
    const double rhon_inv = 1.0 / rhon_k, rho_inv = 1.0 / rho_k;
    double rdzn_k = 0.0, dzn_k = 0.0, alpha = 0.0, beta = 0.0, cz_t = 0.0, rz_t = 0.0;
    if (wlev) {
        const double rdz_kp = A.rdz[kc + 1], rhon_kp = A.rhon[kc + 1];
        const double dz_kp = 1.0 / rdz_kp;
        dzn_k = 0.5 * (dz_k + dz_kp);
        rdzn_k = 1.0 / dzn_k;
        alpha = dz_k * rhon_k / (2.0 * dzn_k);
        beta = dz_kp * rhon_kp / (2.0 * dzn_k);
        cz_t = A.dt * rdz_kp / rhon_kp;  // w z-face at the centre of cell k+1
        rz_t = dz_kp * rhon_kp * A.rdt;
    }
    double rho_km = 0.0, rdzn_km = 0.0, dzn_km = 0.0;
    if (zm1) {
        rho_km = A.rho[kc - 1];
        dzn_km = 0.5 * (1.0 / A.rdz[kc - 1] + dz_k);
        rdzn_km = 1.0 / dzn_km;
    }
    const double cz_b = A.dt * rdz_k * rhon_inv;  // w z-face at the centre of cell k
    const double rz_b = dz_k * rhon_k * A.rdt;

    const double cdx = A.cdx, cdy = A.cdy, rfx = A.rfx, rfy = A.rfy;

    // ---- u ----
    const double a_ue = 0.5 * (u0 + uxp1), a_uw = 0.5 * (uxm1 + u0);
    const double a_un = 0.5 * (v0 + vxp1), a_us = 0.5 * (vym1 + v_xp1ym1);
    const double a_ut = 0.5 * (w0 + wxp1), a_ub = 0.5 * (wzm1 + w_xp1zm1);
    double fe = tvd_flux(a_ue, uxm1, u0, uxp1, uxp2, cdx, rfx, rhon_k);
    double fw = tvd_flux(a_uw, uxm2, uxm1, u0, uxp1, cdx, rfx, rhon_k);
    double fn = tvd_flux(a_un, uym1, u0, uyp1, uyp2, cdy, rfy, rhon_k);
    double fs = tvd_flux(a_us, uym2, uym1, u0, uyp1, cdy, rfy, rhon_k);
    double ft = wlev ? zface(a_ut, uzm1, u0, uzp1, uzp2, zm1, zp2, A.dt * rdzn_k,
                             dzn_k * A.rdt, rho_k)
                     : 0.0;
    double fb = zm1 ? zface(a_ub, uzm2, uzm1, u0, uzp1, zm2, zp1, A.dt * rdzn_km,
                            dzn_km * A.rdt, rho_km)
                    : 0.0;
    const double su = -rhon_inv * ((fe - fw) * A.rdx + (fn - fs) * A.rdy + rdz_k * (ft - fb));

    // ---- v ----
    const double a_ve = 0.5 * (u0 + uyp1), a_vw = 0.5 * (uxm1 + u_xm1yp1);
    const double a_vn = 0.5 * (v0 + vyp1), a_vs = 0.5 * (vym1 + v0);
    const double a_vt = 0.5 * (w0 + wyp1), a_vb = 0.5 * (wzm1 + w_yp1zm1);
    fe = tvd_flux(a_ve, vxm1, v0, vxp1, vxp2, cdx, rfx, rhon_k);
    fw = tvd_flux(a_vw, vxm2, vxm1, v0, vxp1, cdx, rfx, rhon_k);
    fn = tvd_flux(a_vn, vym1, v0, vyp1, vyp2, cdy, rfy, rhon_k);
    fs = tvd_flux(a_vs, vym2, vym1, v0, vyp1, cdy, rfy, rhon_k);
    ft = wlev ? zface(a_vt, vzm1, v0, vzp1, vzp2, zm1, zp2, A.dt * rdzn_k, dzn_k * A.rdt,
                      rho_k)
              : 0.0;
    fb = zm1 ? zface(a_vb, vzm2, vzm1, v0, vzp1, zm2, zp1, A.dt * rdzn_km, dzn_km * A.rdt,
                     rho_km)
             : 0.0;
    const double sv = -rhon_inv * ((fe - fw) * A.rdx + (fn - fs) * A.rdy + rdz_k * (ft - fb));

    // ---- w (levels below the lid) ----
    const double m_we = alpha * u0 + beta * uzp1, m_ww = alpha * uxm1 + beta * u_xm1zp1;
    const double m_wn = alpha * v0 + beta * vzp1, m_ws = alpha * vym1 + beta * v_ym1zp1;
    const double m_wt = 0.5 * (rho_k * w0 + (wlev ? A.rho[kc + 1] : 0.0) * wzp1);
    const double m_wb = 0.5 * (rho_km * wzm1 + rho_k * w0);
    const double cwx = cdx * rho_inv, cwy = cdy * rho_inv;
    const double rwx = rfx * rho_k, rwy = rfy * rho_k;
    fe = tvd_flux(m_we, wxm1, w0, wxp1, wxp2, cwx, rwx, 1.0);
    fw = tvd_flux(m_ww, wxm2, wxm1, w0, wxp1, cwx, rwx, 1.0);
    fn = tvd_flux(m_wn, wym1, w0, wyp1, wyp2, cwy, rwy, 1.0);
    fs = tvd_flux(m_ws, wym2, wym1, w0, wyp1, cwy, rwy, 1.0);
    // top: between w_k and w_{k+1}, far values w_{k-1} (always there: the
    // ground at k = 0) and w_{k+2} (there up to the lid)
    ft = zface(m_wt, wzm1, w0, wzp1, wzp2, true, kc + 2 <= nz - 1, cz_t, rz_t, 1.0);
    // bottom: between w_{k-1} and w_k, far values w_{k-2} (there from k = 1)
    // and w_{k+1}
    fb = zface(m_wb, wzm2, wzm1, w0, wzp1, zm1, true, cz_b, rz_b, 1.0);
    const double sw =
        wlev ? -rho_inv * ((fe - fw) * A.rdx + (fn - fs) * A.rdy + rdzn_k * (ft - fb)) : 0.0;

    if (live) {
        const long c = c00 + k;
        if constexpr (STEPF) {
            A.out_u[c] = u0 + A.dt * su;
            A.out_v[c] = v0 + A.dt * sv;
            A.out_w[c] = wlev ? w0 + A.dt * sw : 0.0;
        } else {
            A.out_u[c] = su;
            A.out_v[c] = sv;
            A.out_w[c] = sw;
        }
    }

    if (A.cmax) {
        // largest Courant number of every face this point evaluated
        double cm = fmax(fmax(fmax(fabs(a_ue), fabs(a_uw)), fmax(fabs(a_ve), fabs(a_vw))) * cdx,
                         fmax(fmax(fabs(a_un), fabs(a_us)), fmax(fabs(a_vn), fabs(a_vs))) * cdy);
        if (wlev) {
            cm = fmax(cm, fmax(fabs(a_ut), fabs(a_vt)) * (A.dt * rdzn_k));
            cm = fmax(cm, fmax(fmax(fabs(m_we), fabs(m_ww)) * cwx,
                               fmax(fabs(m_wn), fabs(m_ws)) * cwy));
            cm = fmax(cm, fmax(fabs(m_wt) * cz_t, fabs(m_wb) * cz_b));
        }
        if (zm1) cm = fmax(cm, fmax(fabs(a_ub), fabs(a_vb)) * (A.dt * rdzn_km));
        if (!live) cm = 0.0;
        for (int o = 32; o > 0; o >>= 1) cm = fmax(cm, __shfl_xor(cm, o, 64));
        if (threadIdx.x == 0)
            atomicMax((unsigned long long*)A.cmax, (unsigned long long)__double_as_longlong(cm));
    }
}

}  // namespace

hipError_t launch_tvd_momentum(const TvdMomArgs& a, bool step, hipStream_t s) {
    if (a.cmax) {
        tvdmom_clear<<<1, 64, 0, s>>>(a.cmax);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const long nb = (long)((a.nz + 63) / 64) * ((a.ny + TM_COLS - 1) / TM_COLS) * a.nx;
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    if (step)
        tvdmom_kernel<true><<<(unsigned)nb, dim3(64, TM_COLS), 0, s>>>(a);
    else
        tvdmom_kernel<false><<<(unsigned)nb, dim3(64, TM_COLS), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace monc
