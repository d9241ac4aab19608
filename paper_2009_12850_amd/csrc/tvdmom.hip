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
// One thread per grid point of a column's 64-level chunk.  A workgroup is one
// column, one wave per chunk, marching through a segment of x-planes: the
// x-stencil stays in a four-plane register window and the east face of a
// plane is the next plane's west face, so an x-face is evaluated once (twice
// on segment edges); a wave evaluates both y-faces of its column.  A level
// evaluates its top z-faces; its bottom faces are the top faces of the level
// below, from the lane below, or across a chunk boundary from the chunk
// below's last lane through LDS; only the lowest level evaluates the w face at
// the centre of the lowest cell (nothing passes the ground for u and v).  The
// per-level geometry is built once per workgroup in LDS.  Periodic neighbours
// are read at wrapped indices; halos are neither read nor written.
#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

constexpr int TM_TI = 64;  // x-planes per segment
constexpr int TM_NCH = 2;  // 64-level chunks per column at most
// Level table: levels -1 .. nz (entry q + 1 for level q).
constexpr int TM_LEV = MONC_MAX_NZ + 2;
static_assert(MONC_MAX_NZ <= 64 * TM_NCH, "columns fit the chunks of a workgroup");
enum { L_RDZ, L_RHON, L_RHO, L_RHONI, L_RHOI, L_RDZN, L_DZN, L_ALPHA, L_BETA, L_CZ, L_RZ, L_N };

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

// Two waves per SIMD: the march holds about 230 registers without spilling.
// Columns that share their y-faces through LDS (two or four per workgroup,
// one barrier per plane) ran 5 and 22 % slower: the exchange and the waves
// left waiting at the barrier cost more than the faces it saves.
template <bool STEPF>
__global__ void __launch_bounds__(64 * TM_NCH) tvdmom_kernel(TvdMomArgs A) {
    __shared__ double tab[L_N][TM_LEV];
    __shared__ double zlast[2][TM_NCH][3];  // top faces of a chunk's last level, by plane parity
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    // Consecutive workgroups go to the same XCD (they are dealt to the 8 XCDs
    // round-robin); neighbouring columns of one segment are consecutive, so
    // the columns they share are still in that XCD's L2.
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int j = b % ny;
    const int seg = b / ny;
    const int chunk = (int)threadIdx.y;
    const int lane = (int)threadIdx.x;
    const int k0 = 64 * chunk;
    const int k = k0 + lane;
    const int i0 = TM_TI * seg;
    const int i1 = min(i0 + TM_TI, nx);
    const bool live = k < nz;
    const int kc = k < nz ? k : nz - 1;  // dead lanes load in bounds, store nothing

    // level table (one division set per level per workgroup)
    {
        for (int t = (int)threadIdx.y * 64 + lane; t < nz + 2; t += 64 * (int)blockDim.y) {
            const int q = t - 1;
            double row[L_N];
            for (int e = 0; e < L_N; e++) row[e] = 0.0;
            if (q >= 0 && q < nz) {
                const double rdz = A.rdz[q], rhon = A.rhon[q], rho = A.rho[q];
                const double dz = 1.0 / rdz;
                row[L_RDZ] = rdz;
                row[L_RHON] = rhon;
                row[L_RHO] = rho;
                row[L_RHONI] = 1.0 / rhon;
                row[L_RHOI] = 1.0 / rho;
                row[L_CZ] = A.dt * rdz * row[L_RHONI];  // w z-face at the centre of cell q
                row[L_RZ] = dz * rhon * A.rdt;
                if (q <= nz - 2) {
                    const double dz1 = 1.0 / A.rdz[q + 1];
                    const double dzn = 0.5 * (dz + dz1);
                    const double rdzn = 1.0 / dzn;
                    row[L_DZN] = dzn;
                    row[L_RDZN] = rdzn;
                    row[L_ALPHA] = dz * rhon * (0.5 * rdzn);
                    row[L_BETA] = dz1 * A.rhon[q + 1] * (0.5 * rdzn);
                }
            }
            for (int e = 0; e < L_N; e++) tab[e][t] = row[e];
        }
    }

    const double* __restrict__ U = A.u;
    const double* __restrict__ V = A.v;
    const double* __restrict__ W = A.w;
    const bool zm1 = kc >= 1, zm2 = kc >= 2, zp1 = kc + 1 <= nz - 1, zp2 = kc + 2 <= nz - 1;
    const bool wlev = kc <= nz - 2;  // w at level k is not the lid
    const long sx = (long)(ny + 4) * nz;
    auto px = [&](int ii) -> long { return (long)(wrap(ii, nx) + 2) * sx; };
    auto oy = [&](int jj) -> long { return (long)(wrap(jj, ny) + 2) * nz; };
    const long oj = oy(j), ojm1 = oy(j - 1), ojm2 = oy(j - 2), ojp1 = oy(j + 1),
               ojp2 = oy(j + 2);

    // A value of this column (or of a neighbouring one) at level k - d or
    // k + d of the same plane: the lane d below or above holds it; the lanes
    // at the chunk's edge load it.  Where the level does not exist (has =
    // false) the value is 0, as the direct loads gave.
    auto below = [&](double x, const double* F, long col, int d, bool has) -> double {
        double y = __shfl_up(x, d, 64);
        if (lane < d && has) y = F[col + kc - d];
        return has ? y : 0.0;
    };
    auto above = [&](double x, const double* F, long col, int d, bool has) -> double {
        double y = __shfl_down(x, d, 64);
        if (lane >= 64 - d && has) y = F[col + kc + d];
        return has ? y : 0.0;
    };

    // x-window of the own column: planes i-1, i, i+1, i+2; the plane after
    // is prefetched one step ahead
    double xu[4], xv[4], xw[4];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const long p = px(i0 - 1 + d) + oj + kc;
        xu[d] = U[p];
        xv[d] = V[p];
        xw[d] = wlev ? W[p] : 0.0;
    }
    double nu, nv, nw;
    {
        const long p = px(i0 + 2) + oj + kc;
        nu = U[p];
        nv = V[p];
        nw = wlev ? W[p] : 0.0;
    }

    __syncthreads();  // level table ready
    const int r = kc + 1;  // row of level k; k-1 and k+1 are its neighbours
    const double rdz_k = tab[L_RDZ][r], rhon_k = tab[L_RHON][r], rho_k = tab[L_RHO][r];
    const double rhon_inv = tab[L_RHONI][r], rho_inv = tab[L_RHOI][r];
    const double rdzn_k = tab[L_RDZN][r], dzn_k = tab[L_DZN][r];
    const double alpha = tab[L_ALPHA][r], beta = tab[L_BETA][r];
    const double cz_b = tab[L_CZ][r], rz_b = tab[L_RZ][r];
    const double cz_t = tab[L_CZ][r + 1], rz_t = tab[L_RZ][r + 1], rho_kp = tab[L_RHO][r + 1];
    const double rho_km = tab[L_RHO][r - 1];

    const double cdx = A.cdx, cdy = A.cdy, rfx = A.rfx, rfy = A.rfy;
    const double cwx = cdx * rho_inv, cwy = cdy * rho_inv;
    const double rwx = rfx * rho_k, rwy = rfy * rho_k;
    const double czu_t = A.dt * rdzn_k, rzu_t = dzn_k * A.rdt;

    // west faces of the first plane: the east faces of the plane before it,
    // evaluated the same way
    double fw_u, fw_v, fw_w, cm;
    {
        const long pm1 = px(i0 - 1), pm2 = px(i0 - 2);
        const double um2 = U[pm2 + oj + kc], vm2 = V[pm2 + oj + kc];
        const double wm2 = wlev ? W[pm2 + oj + kc] : 0.0;
        const double u_xm1yp1 = U[pm1 + ojp1 + kc];
        const double u_xm1zp1 = zp1 ? U[pm1 + oj + kc + 1] : 0.0;
        const double a_u = 0.5 * (xu[0] + xu[1]), a_v = 0.5 * (xu[0] + u_xm1yp1);
        const double m_w = alpha * xu[0] + beta * u_xm1zp1;
        fw_u = tvd_flux(a_u, um2, xu[0], xu[1], xu[2], cdx, rfx, rhon_k);
        fw_v = tvd_flux(a_v, vm2, xv[0], xv[1], xv[2], cdx, rfx, rhon_k);
        fw_w = tvd_flux(m_w, wm2, xw[0], xw[1], xw[2], cwx, rwx, 1.0);
        cm = fmax(fmax(fabs(a_u), fabs(a_v)) * cdx, wlev ? fabs(m_w) * cwx : 0.0);
    }

    for (int i = i0; i < i1; i++) {
        xu[3] = nu;
        xv[3] = nv;
        xw[3] = nw;
        if (i + 1 < i1) {  // prefetch plane i+3
            const long p = px(i + 3) + oj + kc;
            nu = U[p];
            nv = V[p];
            nw = wlev ? W[p] : 0.0;
        }
        const long p0 = px(i), pp1 = px(i + 1);
        const long c00 = p0 + oj;
        const double u0 = xu[1], v0 = xv[1], w0 = xw[1];

        // y-stencils at plane i
        const double uym1 = U[p0 + ojm1 + kc], uyp1 = U[p0 + ojp1 + kc], uyp2 = U[p0 + ojp2 + kc];
        const double vym1 = V[p0 + ojm1 + kc], vyp1 = V[p0 + ojp1 + kc], vyp2 = V[p0 + ojp2 + kc];
        const double wym1 = wlev ? W[p0 + ojm1 + kc] : 0.0;
        const double wyp1 = wlev ? W[p0 + ojp1 + kc] : 0.0;
        const double wyp2 = wlev ? W[p0 + ojp2 + kc] : 0.0;
        // z-stencils of the own column at plane i, from the neighbouring lanes
        const double uzm1 = below(u0, U, c00, 1, zm1);
        const double uzp1 = above(u0, U, c00, 1, zp1), uzp2 = above(u0, U, c00, 2, zp2);
        const double vzm1 = below(v0, V, c00, 1, zm1);
        const double vzp1 = above(v0, V, c00, 1, zp1), vzp2 = above(v0, V, c00, 2, zp2);
        const double wzm1 = below(w0, W, c00, 1, zm1), wzm2 = below(w0, W, c00, 2, zm2);
        const double wzp1 = above(w0, W, c00, 1, kc + 1 <= nz - 2);
        const double wzp2 = above(w0, W, c00, 2, kc + 2 <= nz - 2);

        // ---- east faces (the next plane's west faces) ----
        const double a_ue = 0.5 * (u0 + xu[2]), a_ve = 0.5 * (u0 + uyp1);
        const double m_we = alpha * u0 + beta * uzp1;
        const double fe_u = tvd_flux(a_ue, xu[0], u0, xu[2], xu[3], cdx, rfx, rhon_k);
        const double fe_v = tvd_flux(a_ve, xv[0], v0, xv[2], xv[3], cdx, rfx, rhon_k);
        const double fe_w = tvd_flux(m_we, xw[0], w0, xw[2], xw[3], cwx, rwx, 1.0);
        // ---- north faces ----
        const double a_un = 0.5 * (v0 + xv[2]), a_vn = 0.5 * (v0 + vyp1);
        const double m_wn = alpha * v0 + beta * vzp1;
        const double fn_u = tvd_flux(a_un, uym1, u0, uyp1, uyp2, cdy, rfy, rhon_k);
        const double fn_v = tvd_flux(a_vn, vym1, v0, vyp1, vyp2, cdy, rfy, rhon_k);
        const double fn_w = tvd_flux(m_wn, wym1, w0, wyp1, wyp2, cwy, rwy, 1.0);
        // ---- south faces (the previous column's north faces, evaluated the
        // same way) ----
        const double uym2 = U[p0 + ojm2 + kc], vym2 = V[p0 + ojm2 + kc];
        const double wym2 = wlev ? W[p0 + ojm2 + kc] : 0.0;
        const double v_xp1ym1 = V[pp1 + ojm1 + kc];
        const double v_ym1zp1 = above(vym1, V, p0 + ojm1, 1, zp1);
        const double a_us = 0.5 * (vym1 + v_xp1ym1), a_vs = 0.5 * (vym1 + v0);
        const double m_ws = alpha * vym1 + beta * v_ym1zp1;
        const double fs_u = tvd_flux(a_us, uym2, uym1, u0, uyp1, cdy, rfy, rhon_k);
        const double fs_v = tvd_flux(a_vs, vym2, vym1, v0, vyp1, cdy, rfy, rhon_k);
        const double fs_w = tvd_flux(m_ws, wym2, wym1, w0, wyp1, cwy, rwy, 1.0);
        // ---- z faces: top k+1/2 of u, v and the centre k+1 of w; the bottom
        // faces are the top faces of the level below ----
        const double a_ut = 0.5 * (w0 + xw[2]), a_vt = 0.5 * (w0 + wyp1);
        const double ft_u = wlev ? zface(a_ut, uzm1, u0, uzp1, uzp2, zm1, zp2, czu_t, rzu_t, rho_k)
                                 : 0.0;
        const double ft_v = wlev ? zface(a_vt, vzm1, v0, vzp1, vzp2, zm1, zp2, czu_t, rzu_t, rho_k)
                                 : 0.0;
        const double m_wt = 0.5 * (rho_k * w0 + rho_kp * wzp1);
        const double m_wb = 0.5 * (rho_km * wzm1 + rho_k * w0);
        // top: between w_k and w_{k+1}, far values w_{k-1} (always there: the
        // ground at k = 0) and w_{k+2} (there up to the lid)
        const double ft_w = zface(m_wt, wzm1, w0, wzp1, wzp2, true, kc + 2 <= nz - 1, cz_t, rz_t,
                                  1.0);
        double fb_u = __shfl_up(ft_u, 1, 64), fb_v = __shfl_up(ft_v, 1, 64),
               fb_w = __shfl_up(ft_w, 1, 64);
        if (chunk == 0) {
            // the lowest level: nothing passes the ground for u and v; the w
            // face at the centre of the lowest cell, between the ground and w_0
            const double fw0 = zface(m_wb, wzm2, wzm1, w0, wzp1, zm1, true, cz_b, rz_b, 1.0);
            if (lane == 0) {
                fb_u = 0.0;
                fb_v = 0.0;
                fb_w = fw0;
            }
        }
        // a chunk's last level hands its top faces to the next chunk's first
        const int par = i & 1;
        if (lane == 63) {
            zlast[par][chunk][0] = ft_u;
            zlast[par][chunk][1] = ft_v;
            zlast[par][chunk][2] = ft_w;
        }

        // The handed faces are double-buffered by plane parity: a wave writes
        // the other buffer next, and cannot reach the plane after that before
        // every wave has passed this barrier.
        __syncthreads();
        if (chunk > 0 && lane == 0) {
            fb_u = zlast[par][chunk - 1][0];
            fb_v = zlast[par][chunk - 1][1];
            fb_w = zlast[par][chunk - 1][2];
        }

        const double su =
            -rhon_inv * ((fe_u - fw_u) * A.rdx + (fn_u - fs_u) * A.rdy + rdz_k * (ft_u - fb_u));
        const double sv =
            -rhon_inv * ((fe_v - fw_v) * A.rdx + (fn_v - fs_v) * A.rdy + rdz_k * (ft_v - fb_v));
        const double sw = wlev ? -rho_inv * ((fe_w - fw_w) * A.rdx + (fn_w - fs_w) * A.rdy +
                                             rdzn_k * (ft_w - fb_w))
                               : 0.0;
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
            // a south face is the previous column's north face, counted there
            cm = fmax(cm, fmax(fmax(fabs(a_ue), fabs(a_ve)) * cdx,
                               fmax(fabs(a_un), fabs(a_vn)) * cdy));
            // a bottom face is the top face of the level below, counted there;
            // the lowest level also counts the w face at the lowest centre
            if (wlev) {
                cm = fmax(cm, fmax(fabs(a_ut), fabs(a_vt)) * czu_t);
                cm = fmax(cm, fmax(fabs(m_we) * cwx, fabs(m_wn) * cwy));
                cm = fmax(cm, fmax(fabs(m_wt) * cz_t, fabs(m_wb) * cz_b));
            }
        }

        fw_u = fe_u;
        fw_v = fe_v;
        fw_w = fe_w;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            xu[d] = xu[d + 1];
            xv[d] = xv[d + 1];
            xw[d] = xw[d + 1];
        }
    }

    if (A.cmax) {
        // largest Courant number of the faces this wave counted; every face
        // of a live point is counted by some wave (a south face as the
        // previous column's north face, a bottom face as the top face of the
        // level below)
        if (!live) cm = 0.0;
        for (int o = 32; o > 0; o >>= 1) cm = fmax(cm, __shfl_xor(cm, o, 64));
        // Non-negative doubles order like their bit patterns.  The atomic is
        // issued only where it raises the maximum read back from L2 (a stale
        // read costs an extra atomic, never a wrong result), so the waves do
        // not queue on one address.
        unsigned long long* slot = (unsigned long long*)A.cmax;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(cm);
        if (lane == 0 &&
            bits > __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(slot, bits);
    }
}

}  // namespace

hipError_t launch_tvd_momentum(const TvdMomArgs& a, bool step, hipStream_t s) {
    if (a.cmax) {
        tvdmom_clear<<<1, 64, 0, s>>>(a.cmax);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int nch = (a.nz + 63) / 64;
    if (nch > TM_NCH) return hipErrorInvalidValue;
    const long nb = (long)a.ny * ((a.nx + TM_TI - 1) / TM_TI);
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    if (step)
        tvdmom_kernel<true><<<(unsigned)nb, dim3(64, nch), 0, s>>>(a);
    else
        tvdmom_kernel<false><<<(unsigned)nb, dim3(64, nch), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace monc
