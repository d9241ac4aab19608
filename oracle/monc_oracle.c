/*
 * monc_oracle.c -- plain, slow, FP64 CPU oracle for the MONC advection hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * What it computes (Brown et al., "A directive based hybrid Met Office NERC
 * Cloud model", Sec. 2.1 and Sec. 3.1): the advection source terms of the
 * prognostic fields u, v, w and the scalars (theta and the q fields).  The paper
 * names the two schemes -- the energy-conserving Piacsek-Williams (PW) scheme
 * for momentum and Leonard's positivity-preserving ULTIMATE (TVD) scheme for
 * scalars -- but prints no formulas, so the discretisation below is the
 * project's stated reading of those published methods:
 *
 *   Grid     Arakawa C-grid, periodic in x and y with a 2-deep halo, nz cells in
 *            z.  u[i] sits on the +x face of cell i, v[j] on the +y face, w[k]
 *            on the TOP face of cell k; the ground face (w = 0) is implicit and
 *            w[nz-1] is the rigid lid (treated as identically 0).
 *   Profiles rdz[k] = 1/dz_k (cell thickness), rho[k] = reference density at
 *            the top face of cell k, rhon[k] = at the cell centre.  zn_k is the
 *            midpoint of cell k, so dzn_k = (dz_k + dz_{k+1})/2.
 *   PW       centred flux form with mass fluxes interpolated so that the
 *            discrete kinetic energy budget closes exactly (sum by parts).
 *   TVD      QUICKEST face value (Leonard 1979) limited by the ULTIMATE
 *            universal limiter (Leonard 1991), one 1-D flux per face, unsplit.
 *   Step     forward update f <- f + dt*s (the "step fields" component, Sec. 3).
 *
 * Storage: every field is a [(nx+4)][(ny+4)][nz] array, z fastest; element
 * (i,j,k) with i in [-2,nx+2), j in [-2,ny+2) is at ((i+2)*(ny+4)+(j+2))*nz+k.
 *
 * Built with -O2 -ffp-contract=off -fno-fast-math so every product and sum is
 * rounded as written.  Loops are plain; OpenMP only splits the outer i loop.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ECFL (-3)

/* Number of OpenMP threads of the parallel loops below (the CPU baseline times
 * one thread and all of them); returns the count in effect, 1 without OpenMP. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

typedef struct {
    int nx, ny, nz;
} grid_t;

static inline long at(const grid_t *g, int i, int j, int k) {
    return ((long)(i + 2) * (g->ny + 4) + (j + 2)) * g->nz + k;
}

static int posmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* ---------------------------------------------------------------------------
 * Periodic lateral halo fill, depth 2 (the model's halo swap, Sec. 2.1, on one
 * domain with periodic neighbours).  Every halo element, corners included,
 * becomes a copy of the interior element at the wrapped index.
 * ------------------------------------------------------------------------- */
int oracle_halo_fill(double *f, int nx, int ny, int nz) {
    if (!f || nx < 1 || ny < 1 || nz < 1) return OR_EINVAL;
    grid_t g = {nx, ny, nz};
    for (int i = -2; i < nx + 2; i++)
        for (int j = -2; j < ny + 2; j++) {
            if (i >= 0 && i < nx && j >= 0 && j < ny) continue;
            int si = posmod(i, nx), sj = posmod(j, ny);
            for (int k = 0; k < nz; k++) f[at(&g, i, j, k)] = f[at(&g, si, sj, k)];
        }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Vertical geometry derived from the profiles (the constants the paper copies
 * to the device once, Sec. 3).  dz_k = 1/rdz_k; dzn_k = (dz_k + dz_{k+1})/2
 * for k < nz-1 (distance between the centres of cells k and k+1).
 * ------------------------------------------------------------------------- */
typedef struct {
    double *dz, *dzn, *rdzn;
} vgeom_t;

static void vgeom_make(vgeom_t *vg, const double *rdz, int nz) {
    vg->dz = (double *)malloc(sizeof(double) * nz);
    vg->dzn = (double *)malloc(sizeof(double) * nz);
    vg->rdzn = (double *)malloc(sizeof(double) * nz);
    for (int k = 0; k < nz; k++) vg->dz[k] = 1.0 / rdz[k];
    for (int k = 0; k < nz; k++) {
        if (k < nz - 1) {
            vg->dzn[k] = 0.5 * (vg->dz[k] + vg->dz[k + 1]);
            vg->rdzn[k] = 1.0 / vg->dzn[k];
        } else {
            vg->dzn[k] = 0.0; /* no w-cell above the lid */
            vg->rdzn[k] = 0.0;
        }
    }
}

static void vgeom_free(vgeom_t *vg) {
    free(vg->dz);
    free(vg->dzn);
    free(vg->rdzn);
}

/* w with the boundary conditions applied: the ground face (k = -1) and the
 * lid (k = nz-1) carry no flow whatever the array holds there. */
static inline double W(const grid_t *g, const double *w, int i, int j, int k) {
    if (k < 0 || k >= g->nz - 1) return 0.0;
    return w[at(g, i, j, k)];
}

/* ---------------------------------------------------------------------------
 * Piacsek-Williams momentum source terms (Sec. 3.1: the energy-conserving
 * scheme).  Flux form, centred:
 *
 * su = [ (u_{i-1}+u_i)^2 - (u_i+u_{i+1})^2 ] / (4 dx)
 *    + [ (v_{i,j-1}+v_{i+1,j-1})(u_{j-1}+u_j) - (v_{ij}+v_{i+1,j})(u_j+u_{j+1}) ] / (4 dy)
 *    + rdz_k/(4 rhon_k) [ rho_{k-1}(w_{i,k-1}+w_{i+1,k-1})(u_{k-1}+u_k)
 *                         - rho_k (w_{ik}+w_{i+1,k})(u_k+u_{k+1}) ]
 * sv is the same with the roles of x and y exchanged.
 * For k = 0..nz-2, with a_k = dz_k rhon_k/(2 dzn_k), b_k = dz_{k+1} rhon_{k+1}/(2 dzn_k):
 * sw = -(1/rho_k) { [ (a u_{ik}+b u_{i,k+1})(w_i+w_{i+1}) - (a u_{i-1,k}+b u_{i-1,k+1})(w_{i-1}+w_i) ]/(2dx)
 *                 + [ same in y with v ]/(2dy)
 *                 + rdzn_k/4 [ (rho_k w_k + rho_{k+1} w_{k+1})(w_k+w_{k+1})
 *                              - (rho_{k-1} w_{k-1} + rho_k w_k)(w_{k-1}+w_k) ] }
 * sw[nz-1] = 0.  Terms that would reach through the ground or the lid vanish
 * because w is zero there.
 *
 * Computes the interior points i in [i0,i1), j in [j0,j1), all k.  Halos of
 * u, v, w must be valid.  Output halos are not touched.
 * ------------------------------------------------------------------------- */
int oracle_pw(const double *u, const double *v, const double *w, double *su,
              double *sv, double *sw, int nx, int ny, int nz, double dx,
              double dy, const double *rdz, const double *rho,
              const double *rhon, int i0, int i1, int j0, int j1) {
    if (!u || !v || !w || !su || !sv || !sw || !rdz || !rho || !rhon)
        return OR_EINVAL;
    if (nx < 1 || ny < 1 || nz < 2 || !(dx > 0) || !(dy > 0)) return OR_EINVAL;
    if (i0 < 0 || i1 > nx || j0 < 0 || j1 > ny || i0 > i1 || j0 > j1)
        return OR_EINVAL;
    grid_t g = {nx, ny, nz};
    vgeom_t vg;
    vgeom_make(&vg, rdz, nz);

#pragma omp parallel for schedule(static)
    for (int i = i0; i < i1; i++)
        for (int j = j0; j < j1; j++)
            for (int k = 0; k < nz; k++) {
                long c = at(&g, i, j, k);
                /* ---- su ---- */
                double um = u[at(&g, i - 1, j, k)], u0 = u[c],
                       up = u[at(&g, i + 1, j, k)];
                double x_term = ((um + u0) * (um + u0) - (u0 + up) * (u0 + up)) /
                                (4.0 * dx);
                double y_term =
                    ((v[at(&g, i, j - 1, k)] + v[at(&g, i + 1, j - 1, k)]) *
                         (u[at(&g, i, j - 1, k)] + u0) -
                     (v[c] + v[at(&g, i + 1, j, k)]) *
                         (u0 + u[at(&g, i, j + 1, k)])) /
                    (4.0 * dy);
                double flux_bot = 0.0, flux_top = 0.0;
                if (k > 0)
                    flux_bot = rho[k - 1] *
                               (W(&g, w, i, j, k - 1) + W(&g, w, i + 1, j, k - 1)) *
                               (u[at(&g, i, j, k - 1)] + u0);
                if (k < nz - 1)
                    flux_top = rho[k] * (W(&g, w, i, j, k) + W(&g, w, i + 1, j, k)) *
                               (u0 + u[at(&g, i, j, k + 1)]);
                double z_term = rdz[k] / (4.0 * rhon[k]) * (flux_bot - flux_top);
                su[c] = x_term + y_term + z_term;

                /* ---- sv ---- */
                double vm = v[at(&g, i, j - 1, k)], v0 = v[c],
                       vp = v[at(&g, i, j + 1, k)];
                double x_term_v =
                    ((u[at(&g, i - 1, j, k)] + u[at(&g, i - 1, j + 1, k)]) *
                         (v[at(&g, i - 1, j, k)] + v0) -
                     (u[c] + u[at(&g, i, j + 1, k)]) *
                         (v0 + v[at(&g, i + 1, j, k)])) /
                    (4.0 * dx);
                double y_term_v =
                    ((vm + v0) * (vm + v0) - (v0 + vp) * (v0 + vp)) / (4.0 * dy);
                double fb = 0.0, ft = 0.0;
                if (k > 0)
                    fb = rho[k - 1] *
                         (W(&g, w, i, j, k - 1) + W(&g, w, i, j + 1, k - 1)) *
                         (v[at(&g, i, j, k - 1)] + v0);
                if (k < nz - 1)
                    ft = rho[k] * (W(&g, w, i, j, k) + W(&g, w, i, j + 1, k)) *
                         (v0 + v[at(&g, i, j, k + 1)]);
                double z_term_v = rdz[k] / (4.0 * rhon[k]) * (fb - ft);
                sv[c] = x_term_v + y_term_v + z_term_v;

                /* ---- sw ---- */
                if (k == nz - 1) {
                    sw[c] = 0.0;
                    continue;
                }
                double a = vg.dz[k] * rhon[k] / (2.0 * vg.dzn[k]);
                double b = vg.dz[k + 1] * rhon[k + 1] / (2.0 * vg.dzn[k]);
                double wc = W(&g, w, i, j, k);
                double fxe = (a * u[at(&g, i, j, k)] + b * u[at(&g, i, j, k + 1)]) *
                             (wc + W(&g, w, i + 1, j, k));
                double fxw =
                    (a * u[at(&g, i - 1, j, k)] + b * u[at(&g, i - 1, j, k + 1)]) *
                    (W(&g, w, i - 1, j, k) + wc);
                double fyn = (a * v[at(&g, i, j, k)] + b * v[at(&g, i, j, k + 1)]) *
                             (wc + W(&g, w, i, j + 1, k));
                double fys =
                    (a * v[at(&g, i, j - 1, k)] + b * v[at(&g, i, j - 1, k + 1)]) *
                    (W(&g, w, i, j - 1, k) + wc);
                double wkp = W(&g, w, i, j, k + 1), wkm = W(&g, w, i, j, k - 1);
                double rho_kp = rho[k + 1];
                double rho_km = (k > 0) ? rho[k - 1] : 0.0; /* multiplies w_{-1} = 0 */
                double fzt = (rho[k] * wc + rho_kp * wkp) * (wc + wkp);
                double fzb = (rho_km * wkm + rho[k] * wc) * (wkm + wc);
                sw[c] = -(1.0 / rho[k]) *
                        ((fxe - fxw) / (2.0 * dx) + (fyn - fys) / (2.0 * dy) +
                         vg.rdzn[k] / 4.0 * (fzt - fzb));
            }
    vgeom_free(&vg);
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * ULTIMATE-limited QUICKEST face value (Sec. 3.1: Leonard's positivity-
 * preserving scheme).  phiU = far-upwind, phiC = upwind, phiD = downwind cell,
 * c = Courant number |a| dt / spacing.
 *   delta = phiD - phiU, kappa = phiD - 2 phiC + phiU.
 *   |kappa| >= |delta|  -> phiC (local extremum or flat: first-order upwind).
 *   QUICKEST: phi* = (phiC+phiD)/2 - c (phiD-phiC)/2 - (1-c^2)/6 kappa.
 *   ULTIMATE bounds: phi_f between phiC and min/max(phiD, phiU + (phiC-phiU)/c).
 * ------------------------------------------------------------------------- */
double oracle_ultimate_face(double phiU, double phiC, double phiD, double c) {
    double delta = phiD - phiU;
    double kappa = phiD - 2.0 * phiC + phiU;
    if (fabs(kappa) >= fabs(delta)) return phiC;
    double phistar = 0.5 * (phiC + phiD) - 0.5 * c * (phiD - phiC) -
                     (1.0 - c * c) / 6.0 * kappa;
    double bound = (c > 0.0) ? phiU + (phiC - phiU) / c : phiD;
    if (delta > 0.0)
        return fmin(fmax(phistar, phiC), fmin(phiD, bound));
    return fmax(fmin(phistar, phiC), fmax(phiD, bound));
}

/* Flux through the +x face of cell (i,j,k): rhon_k * u * phi_face. */
static double flux_x(const grid_t *g, const double *u, const double *phi, int i,
                     int j, int k, double dx, double dt, const double *rhon,
                     double *cmax) {
    double a = u[at(g, i, j, k)];
    double c = fabs(a) * dt / dx;
    if (c > *cmax) *cmax = c;
    double pf;
    if (a >= 0.0)
        pf = oracle_ultimate_face(phi[at(g, i - 1, j, k)], phi[at(g, i, j, k)],
                                  phi[at(g, i + 1, j, k)], c);
    else
        pf = oracle_ultimate_face(phi[at(g, i + 2, j, k)], phi[at(g, i + 1, j, k)],
                                  phi[at(g, i, j, k)], c);
    return rhon[k] * a * pf;
}

/* Flux through the +y face of cell (i,j,k): rhon_k * v * phi_face. */
static double flux_y(const grid_t *g, const double *v, const double *phi, int i,
                     int j, int k, double dy, double dt, const double *rhon,
                     double *cmax) {
    double a = v[at(g, i, j, k)];
    double c = fabs(a) * dt / dy;
    if (c > *cmax) *cmax = c;
    double pf;
    if (a >= 0.0)
        pf = oracle_ultimate_face(phi[at(g, i, j - 1, k)], phi[at(g, i, j, k)],
                                  phi[at(g, i, j + 1, k)], c);
    else
        pf = oracle_ultimate_face(phi[at(g, i, j + 2, k)], phi[at(g, i, j + 1, k)],
                                  phi[at(g, i, j, k)], c);
    return rhon[k] * a * pf;
}

/* Flux through the top face of cell (i,j,k): rho_k * w_k * phi_face, zero at
 * the ground (k = -1) and at the lid (k = nz-1).  Where the far-upwind cell
 * lies outside the column the face takes the upwind value. */
static double flux_z(const grid_t *g, const double *w, const double *phi, int i,
                     int j, int k, double dt, const double *rho,
                     const vgeom_t *vg, double *cmax) {
    if (k < 0 || k >= g->nz - 1) return 0.0;
    double a = w[at(g, i, j, k)];
    double c = fabs(a) * dt * vg->rdzn[k];
    if (c > *cmax) *cmax = c;
    double pf;
    if (a >= 0.0) {
        if (k - 1 < 0)
            pf = phi[at(g, i, j, k)];
        else
            pf = oracle_ultimate_face(phi[at(g, i, j, k - 1)], phi[at(g, i, j, k)],
                                      phi[at(g, i, j, k + 1)], c);
    } else {
        if (k + 2 > g->nz - 1)
            pf = phi[at(g, i, j, k + 1)];
        else
            pf = oracle_ultimate_face(phi[at(g, i, j, k + 2)], phi[at(g, i, j, k + 1)],
                                      phi[at(g, i, j, k)], c);
    }
    return rho[k] * a * pf;
}

/* ---------------------------------------------------------------------------
 * TVD scalar source term:
 *   s = -(1/rhon_k) [ (Fx_{i+1/2}-Fx_{i-1/2})/dx + (Fy_{j+1/2}-Fy_{j-1/2})/dy
 *                     + rdz_k (Fz_{k+1/2}-Fz_{k-1/2}) ]
 * Halos (depth 2) of u, v, w, phi must be valid.  Returns OR_ECFL (after
 * filling the output) when any Courant number used exceeds 1; *cmax_out, if
 * given, receives the largest Courant number met.
 * ------------------------------------------------------------------------- */
int oracle_tvd(const double *u, const double *v, const double *w,
               const double *phi, double *sphi, int nx, int ny, int nz,
               double dx, double dy, const double *rdz, const double *rho,
               const double *rhon, double dt, int i0, int i1, int j0, int j1,
               double *cmax_out) {
    if (!u || !v || !w || !phi || !sphi || !rdz || !rho || !rhon) return OR_EINVAL;
    if (nx < 1 || ny < 1 || nz < 2 || !(dx > 0) || !(dy > 0) || !(dt >= 0))
        return OR_EINVAL;
    if (i0 < 0 || i1 > nx || j0 < 0 || j1 > ny || i0 > i1 || j0 > j1)
        return OR_EINVAL;
    grid_t g = {nx, ny, nz};
    vgeom_t vg;
    vgeom_make(&vg, rdz, nz);
    double cmax = 0.0;

#pragma omp parallel for schedule(static) reduction(max : cmax)
    for (int i = i0; i < i1; i++)
        for (int j = j0; j < j1; j++)
            for (int k = 0; k < nz; k++) {
                double fe = flux_x(&g, u, phi, i, j, k, dx, dt, rhon, &cmax);
                double fw = flux_x(&g, u, phi, i - 1, j, k, dx, dt, rhon, &cmax);
                double fn = flux_y(&g, v, phi, i, j, k, dy, dt, rhon, &cmax);
                double fs = flux_y(&g, v, phi, i, j - 1, k, dy, dt, rhon, &cmax);
                double ft = flux_z(&g, w, phi, i, j, k, dt, rho, &vg, &cmax);
                double fb = flux_z(&g, w, phi, i, j, k - 1, dt, rho, &vg, &cmax);
                sphi[at(&g, i, j, k)] =
                    -(1.0 / rhon[k]) *
                    ((fe - fw) / dx + (fn - fs) / dy + rdz[k] * (ft - fb));
            }
    vgeom_free(&vg);
    if (cmax_out) *cmax_out = cmax;
    return cmax > 1.0 ? OR_ECFL : OR_OK;
}

/* ---------------------------------------------------------------------------
 * Anelastic mass divergence of p-cell (i,j,k):
 *   D = rhon_k [ (u_i-u_{i-1})/dx + (v_j-v_{j-1})/dy ] + rdz_k (rho_k w_k - rho_{k-1} w_{k-1})
 * with w zero at the ground and the lid.
 * ------------------------------------------------------------------------- */
static double divergence(const grid_t *g, const double *u, const double *v,
                         const double *w, int i, int j, int k, double dx,
                         double dy, const double *rdz, const double *rho,
                         const double *rhon) {
    double horiz = (u[at(g, i, j, k)] - u[at(g, i - 1, j, k)]) / dx +
                   (v[at(g, i, j, k)] - v[at(g, i, j - 1, k)]) / dy;
    double wt = rho[k] * W(g, w, i, j, k);
    double wb = (k > 0) ? rho[k - 1] * W(g, w, i, j, k - 1) : 0.0;
    return rhon[k] * horiz + rdz[k] * (wt - wb);
}

int oracle_divergence(const double *u, const double *v, const double *w,
                      double *d, int nx, int ny, int nz, double dx, double dy,
                      const double *rdz, const double *rho, const double *rhon) {
    if (!u || !v || !w || !d || nx < 1 || ny < 1 || nz < 2) return OR_EINVAL;
    grid_t g = {nx, ny, nz};
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; i++)
        for (int j = 0; j < ny; j++)
            for (int k = 0; k < nz; k++)
                d[at(&g, i, j, k)] =
                    divergence(&g, u, v, w, i, j, k, dx, dy, rdz, rho, rhon);
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * One forward step of the whole path ("step fields", Sec. 3): halo fill of the
 * input state, PW for u,v,w, TVD for every scalar, then f_out = f_in + dt*s,
 * with w at the lid set to 0.  state_in[0..2] = u,v,w, state_in[3..] = scalars.
 * The input's halo is rewritten; the output's halo is left as it was.
 * Returns OR_ECFL (with the output still written) if a Courant number > 1.
 * ------------------------------------------------------------------------- */
int oracle_step(double *const *state_in, double *const *state_out, int nscal,
                int nx, int ny, int nz, double dx, double dy, const double *rdz,
                const double *rho, const double *rhon, double dt) {
    if (!state_in || !state_out || nscal < 0) return OR_EINVAL;
    int nf = 3 + nscal;
    for (int f = 0; f < nf; f++) {
        if (!state_in[f] || !state_out[f]) return OR_EINVAL;
        int rc = oracle_halo_fill(state_in[f], nx, ny, nz);
        if (rc) return rc;
    }
    long n = (long)(nx + 4) * (ny + 4) * nz;
    double *tend = (double *)calloc((size_t)n, sizeof(double));
    if (!tend) return OR_EINVAL;
    grid_t g = {nx, ny, nz};
    int status = OR_OK;
    double *su = (double *)calloc((size_t)n, sizeof(double));
    double *sv = (double *)calloc((size_t)n, sizeof(double));
    double *sw = (double *)calloc((size_t)n, sizeof(double));
    int rc = oracle_pw(state_in[0], state_in[1], state_in[2], su, sv, sw, nx, ny,
                       nz, dx, dy, rdz, rho, rhon, 0, nx, 0, ny);
    if (rc) status = rc;
    double *tends[3] = {su, sv, sw};
    for (int f = 0; f < 3; f++)
        for (int i = 0; i < nx; i++)
            for (int j = 0; j < ny; j++)
                for (int k = 0; k < nz; k++) {
                    long c = at(&g, i, j, k);
                    double val = state_in[f][c] + dt * tends[f][c];
                    if (f == 2 && k == nz - 1) val = 0.0;
                    state_out[f][c] = val;
                }
    for (int s = 0; s < nscal && status != OR_EINVAL; s++) {
        rc = oracle_tvd(state_in[0], state_in[1], state_in[2], state_in[3 + s], tend,
                        nx, ny, nz, dx, dy, rdz, rho, rhon, dt, 0, nx, 0, ny, NULL);
        if (rc == OR_EINVAL) status = rc;
        if (rc == OR_ECFL && status == OR_OK) status = rc;
        for (int i = 0; i < nx; i++)
            for (int j = 0; j < ny; j++)
                for (int k = 0; k < nz; k++) {
                    long c = at(&g, i, j, k);
                    state_out[3 + s][c] = state_in[3 + s][c] + dt * tend[c];
                }
    }
    free(su);
    free(sv);
    free(sw);
    free(tend);
    return status;
}

/* ---------------------------------------------------------------------------
 * FP64 budgets of one tendency evaluation (conservation and the kinetic
 * energy identity that makes PW "energy conserving", Sec. 3.1).
 * Inputs: the state (halos valid) and its tendencies (interior valid).
 * out[] layout (this file's own; callers map it by name):
 *   0 C_u = sum rhon dz su        1 C_v = sum rhon dz sv
 *   2 C_w = sum_{k<nz-1} rho dzn sw
 *   3 P_u = sum rhon dz u su      4 Q_u = -sum dz (u^2/2) (D_i + D_{i+1})/2
 *   5 P_v = sum rhon dz v sv      6 Q_v = -sum dz (v^2/2) (D_j + D_{j+1})/2
 *   7 P_w = sum rho dzn w sw      8 Q_w = -sum (w^2/2) (dz_k D_k + dz_{k+1} D_{k+1})/2
 *   9 C_w closed form = sum_ij (rho_0 w_0^2 - rho_{nz-2} w_{nz-2}^2)/4
 *  10 + 3s + 0: C_s = sum rhon dz s_s
 *  10 + 3s + 1: M_s = sum rhon dz phi_s
 *  10 + 3s + 2: min phi_s
 * plus absolute-value companions of 0..8 at abs_out[0..8] (for tolerances).
 * Sums run over i in order, then j, then k, each i-slab summed separately and
 * the slabs added in i order.
 * ------------------------------------------------------------------------- */
int oracle_budgets(const double *u, const double *v, const double *w,
                   const double *su, const double *sv, const double *sw,
                   int nscal, const double *const *phi,
                   const double *const *sphi, int nx, int ny, int nz, double dx,
                   double dy, const double *rdz, const double *rho,
                   const double *rhon, double *out, double *abs_out) {
    if (!u || !v || !w || !su || !sv || !sw || !out) return OR_EINVAL;
    grid_t g = {nx, ny, nz};
    vgeom_t vg;
    vgeom_make(&vg, rdz, nz);
    int nout = 10 + 3 * nscal;
    double *slab = (double *)calloc((size_t)nx * nout, sizeof(double));
    double *slab_abs = (double *)calloc((size_t)nx * 9, sizeof(double));

#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; i++) {
        double *o = slab + (long)i * nout;
        double *oa = slab_abs + (long)i * 9;
        for (int s = 0; s < nscal; s++) o[10 + 3 * s + 2] = INFINITY;
        for (int j = 0; j < ny; j++)
            for (int k = 0; k < nz; k++) {
                long c = at(&g, i, j, k);
                double dz = vg.dz[k];
                double t;
                t = rhon[k] * dz * su[c];
                o[0] += t;
                oa[0] += fabs(t);
                t = rhon[k] * dz * sv[c];
                o[1] += t;
                oa[1] += fabs(t);
                t = rhon[k] * dz * u[c] * su[c];
                o[3] += t;
                oa[3] += fabs(t);
                t = rhon[k] * dz * v[c] * sv[c];
                o[5] += t;
                oa[5] += fabs(t);
                double D0 = divergence(&g, u, v, w, i, j, k, dx, dy, rdz, rho, rhon);
                double Dx = divergence(&g, u, v, w, i + 1, j, k, dx, dy, rdz, rho, rhon);
                double Dy = divergence(&g, u, v, w, i, j + 1, k, dx, dy, rdz, rho, rhon);
                t = -dz * (u[c] * u[c] / 2.0) * (D0 + Dx) / 2.0;
                o[4] += t;
                oa[4] += fabs(t);
                t = -dz * (v[c] * v[c] / 2.0) * (D0 + Dy) / 2.0;
                o[6] += t;
                oa[6] += fabs(t);
                if (k < nz - 1) {
                    double wc = W(&g, w, i, j, k);
                    t = rho[k] * vg.dzn[k] * sw[c];
                    o[2] += t;
                    oa[2] += fabs(t);
                    t = rho[k] * vg.dzn[k] * wc * sw[c];
                    o[7] += t;
                    oa[7] += fabs(t);
                    double Dz = divergence(&g, u, v, w, i, j, k + 1, dx, dy, rdz, rho, rhon);
                    t = -(wc * wc / 2.0) * (dz * D0 + vg.dz[k + 1] * Dz) / 2.0;
                    o[8] += t;
                    oa[8] += fabs(t);
                }
                for (int s = 0; s < nscal; s++) {
                    if (sphi && sphi[s]) o[10 + 3 * s] += rhon[k] * dz * sphi[s][c];
                    if (phi && phi[s]) {
                        double p = phi[s][c];
                        o[10 + 3 * s + 1] += rhon[k] * dz * p;
                        if (p < o[10 + 3 * s + 2]) o[10 + 3 * s + 2] = p;
                    }
                }
            }
        {
            double cw = 0.0;
            for (int j = 0; j < ny; j++) {
                double w0 = W(&g, w, i, j, 0);
                double wt = W(&g, w, i, j, nz - 2);
                cw += (rho[0] * w0 * w0 - rho[nz - 2] * wt * wt) / 4.0;
            }
            o[9] = cw;
        }
    }
    for (int q = 0; q < nout; q++) out[q] = 0.0;
    for (int s = 0; s < nscal; s++) out[10 + 3 * s + 2] = INFINITY;
    if (abs_out)
        for (int q = 0; q < 9; q++) abs_out[q] = 0.0;
    for (int i = 0; i < nx; i++) {
        for (int q = 0; q < nout; q++) {
            if (q >= 10 && (q - 10) % 3 == 2) {
                if (slab[(long)i * nout + q] < out[q]) out[q] = slab[(long)i * nout + q];
            } else {
                out[q] += slab[(long)i * nout + q];
            }
        }
        if (abs_out)
            for (int q = 0; q < 9; q++) abs_out[q] += slab_abs[(long)i * 9 + q];
    }
    free(slab);
    free(slab_abs);
    vgeom_free(&vg);
    return OR_OK;
}

/* Largest Courant number over every face of the domain: |u| dt/dx on all
 * x-faces, |v| dt/dy on all y-faces, |w_k| dt/dzn_k on the interior z-faces. */
double oracle_max_courant(const double *u, const double *v, const double *w,
                          int nx, int ny, int nz, double dx, double dy,
                          const double *rdz, double dt) {
    grid_t g = {nx, ny, nz};
    vgeom_t vg;
    vgeom_make(&vg, rdz, nz);
    double cmax = 0.0;
    for (int i = 0; i < nx; i++)
        for (int j = 0; j < ny; j++)
            for (int k = 0; k < nz; k++) {
                long c = at(&g, i, j, k);
                double cx = fabs(u[c]) * dt / dx, cy = fabs(v[c]) * dt / dy;
                if (cx > cmax) cmax = cx;
                if (cy > cmax) cmax = cy;
                if (k < nz - 1) {
                    double cz = fabs(w[c]) * dt * vg.rdzn[k];
                    if (cz > cmax) cmax = cz;
                }
            }
    vgeom_free(&vg);
    return cmax;
}

/* ---------------------------------------------------------------------------
 * 4x restriction of a fine state to a coarse grid (the coarse-graining used to
 * build training targets for the learned flux correction).  nx, ny, nz must be
 * multiples of 4.  Coarse cell (I,J,K) covers fine cells 4I..4I+3 etc.
 *   dZ_K   = sum of dz over the 4 fine cells
 *   RHON_K = sum rhon dz / dZ_K          (mass-weighted centre density)
 *   RHO_K  = rho of the fine top face 4K+3
 *   scalar = sum rhon dz phi / (16 sum rhon dz)       (mass-weighted mean)
 *   U      = sum_{j,k} rhon dz u(4I+3) / (4 RHON_K dZ_K) (mass-flux mean on the face)
 *   V      likewise on the fine face 4J+3
 *   W      = mean of w over the 16 fine faces at level 4K+3
 * With these, the coarse mass flux through a coarse face is the sum of the fine
 * mass fluxes through it, so the coarse mass divergence is the volume-weighted
 * mean of the fine ones.  Outputs: coarse fields (interior), rdz_c, rho_c,
 * rhon_c [nz/4].
 * ------------------------------------------------------------------------- */
int oracle_restrict4(double *const *fine, double *const *coarse, int nscal, int nx,
                     int ny, int nz, const double *rdz, const double *rho,
                     const double *rhon, double *rdz_c, double *rho_c,
                     double *rhon_c) {
    if (nx % 4 || ny % 4 || nz % 4 || nx < 4 || ny < 4 || nz < 4) return OR_EINVAL;
    grid_t gf = {nx, ny, nz};
    grid_t gc = {nx / 4, ny / 4, nz / 4};
    int NX = nx / 4, NY = ny / 4, NZ = nz / 4;
    double *dZ = (double *)malloc(sizeof(double) * NZ);
    double *mZ = (double *)malloc(sizeof(double) * NZ); /* sum rhon dz */
    for (int K = 0; K < NZ; K++) {
        dZ[K] = 0.0;
        mZ[K] = 0.0;
        for (int k = 4 * K; k < 4 * K + 4; k++) {
            double dz = 1.0 / rdz[k];
            dZ[K] += dz;
            mZ[K] += rhon[k] * dz;
        }
        rdz_c[K] = 1.0 / dZ[K];
        rhon_c[K] = mZ[K] / dZ[K];
        rho_c[K] = rho[4 * K + 3];
    }
    for (int I = 0; I < NX; I++)
        for (int J = 0; J < NY; J++)
            for (int K = 0; K < NZ; K++) {
                long c = at(&gc, I, J, K);
                double su = 0.0, sv = 0.0, sw = 0.0;
                for (int j = 4 * J; j < 4 * J + 4; j++)
                    for (int k = 4 * K; k < 4 * K + 4; k++)
                        su += rhon[k] / rdz[k] * fine[0][at(&gf, 4 * I + 3, j, k)];
                for (int i = 4 * I; i < 4 * I + 4; i++)
                    for (int k = 4 * K; k < 4 * K + 4; k++)
                        sv += rhon[k] / rdz[k] * fine[1][at(&gf, i, 4 * J + 3, k)];
                for (int i = 4 * I; i < 4 * I + 4; i++)
                    for (int j = 4 * J; j < 4 * J + 4; j++)
                        sw += fine[2][at(&gf, i, j, 4 * K + 3)];
                coarse[0][c] = su / (4.0 * mZ[K]);
                coarse[1][c] = sv / (4.0 * mZ[K]);
                coarse[2][c] = (K == NZ - 1) ? 0.0 : sw / 16.0;
                for (int s = 0; s < nscal; s++) {
                    double sp = 0.0;
                    for (int i = 4 * I; i < 4 * I + 4; i++)
                        for (int j = 4 * J; j < 4 * J + 4; j++)
                            for (int k = 4 * K; k < 4 * K + 4; k++)
                                sp += rhon[k] / rdz[k] * fine[3 + s][at(&gf, i, j, k)];
                    coarse[3 + s][c] = sp / (16.0 * mZ[K]);
                }
            }
    free(dZ);
    free(mZ);
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Other source terms of the dynamics group (Sec. 3 and its hybrid-structure
 * figure: the CPU computes the non-advection components of the group while
 * the GPU computes advection, then the source terms are combined before the
 * fields are stepped).  The paper does not name or define these components;
 * the two taken here are standard members of an LES dynamics group:
 *
 *   Coriolis on an f-plane, relaxing toward a geostrophic wind (ug, vg):
 *     su(i,j,k) =  fcor * (vbar - vg),  vbar = mean of v at (i,j), (i+1,j),
 *                                              (i,j-1), (i+1,j-1)
 *     sv(i,j,k) = -fcor * (ubar - ug),  ubar = mean of u at (i,j), (i-1,j),
 *                                              (i,j+1), (i-1,j+1)
 *   (the four C-grid neighbours around the u point and the v point)
 *
 *   Buoyancy of theta on the w faces (Boussinesq, constant reference th0):
 *     sw(i,j,k) = grav * ((th(k) + th(k+1))/2 - th0) / th0   for k < nz-1,
 *     sw(i,j,nz-1) = 0 (the lid)
 *
 * Neighbours are read at wrapped periodic indices (halos are not used).
 * ------------------------------------------------------------------------- */
int oracle_dyn(const double *u, const double *v, const double *th, double *su,
               double *sv, double *sw, int nx, int ny, int nz, double fcor,
               double ug, double vg, double grav, double th0) {
    if (!u || !v || !th || !su || !sv || !sw || nx < 1 || ny < 1 || nz < 1) return OR_EINVAL;
    if (!(th0 > 0.0)) return OR_EINVAL;
    grid_t g = {nx, ny, nz};
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; i++) {
        int im = posmod(i - 1, nx), ip = posmod(i + 1, nx);
        for (int j = 0; j < ny; j++) {
            int jm = posmod(j - 1, ny), jp = posmod(j + 1, ny);
            for (int k = 0; k < nz; k++) {
                long c = at(&g, i, j, k);
                double vbar = (v[at(&g, i, j, k)] + v[at(&g, ip, j, k)] +
                               v[at(&g, i, jm, k)] + v[at(&g, ip, jm, k)]) / 4.0;
                double ubar = (u[at(&g, i, j, k)] + u[at(&g, im, j, k)] +
                               u[at(&g, i, jp, k)] + u[at(&g, im, jp, k)]) / 4.0;
                su[c] = fcor * (vbar - vg);
                sv[c] = -fcor * (ubar - ug);
                if (k < nz - 1) {
                    double thf = (th[c] + th[at(&g, i, j, k + 1)]) / 2.0;
                    sw[c] = grav * (thf - th0) / th0;
                } else {
                    sw[c] = 0.0;
                }
            }
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * MONC's other scalar scheme: the scalar advected with the centred flux form
 * (the Piacsek-Williams scheme of Sec. 3.1 applied to a cell-centred field).
 * Face value = mean of the two cells beside the face:
 *   Fx(i+1/2) = rhon_k u_i (phi_i + phi_{i+1})/2,   Fy alike,
 *   Fz(k+1/2) = rho_k w_k (phi_k + phi_{k+1})/2 for k < nz-1, zero through
 *   the ground and the lid,
 *   s = -(1/rhon_k)[(Fx(i+1/2)-Fx(i-1/2))/dx + (Fy(j+1/2)-Fy(j-1/2))/dy
 *                   + rdz_k (Fz(k+1/2)-Fz(k-1/2))].
 * Neighbours at wrapped periodic indices.
 * ------------------------------------------------------------------------- */
static double cflux_x(const grid_t *g, const double *u, const double *phi, int i, int j,
                      int k, const double *rhon) {
    int ip = posmod(i + 1, g->nx);
    int ii = posmod(i, g->nx);
    return rhon[k] * u[at(g, ii, j, k)] * (phi[at(g, ii, j, k)] + phi[at(g, ip, j, k)]) / 2.0;
}
static double cflux_y(const grid_t *g, const double *v, const double *phi, int i, int j,
                      int k, const double *rhon) {
    int jp = posmod(j + 1, g->ny);
    int jj = posmod(j, g->ny);
    return rhon[k] * v[at(g, i, jj, k)] * (phi[at(g, i, jj, k)] + phi[at(g, i, jp, k)]) / 2.0;
}
static double cflux_z(const grid_t *g, const double *w, const double *phi, int i, int j,
                      int k, const double *rho) {
    if (k < 0 || k >= g->nz - 1) return 0.0;
    return rho[k] * w[at(g, i, j, k)] * (phi[at(g, i, j, k)] + phi[at(g, i, j, k + 1)]) / 2.0;
}

int oracle_pw_scalar(const double *u, const double *v, const double *w, const double *phi,
                     double *s, int nx, int ny, int nz, double dx, double dy,
                     const double *rdz, const double *rho, const double *rhon) {
    if (!u || !v || !w || !phi || !s || nx < 1 || ny < 1 || nz < 1) return OR_EINVAL;
    grid_t g = {nx, ny, nz};
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; i++)
        for (int j = 0; j < ny; j++)
            for (int k = 0; k < nz; k++) {
                double fx = (cflux_x(&g, u, phi, i, j, k, rhon) -
                             cflux_x(&g, u, phi, i - 1, j, k, rhon)) / dx;
                double fy = (cflux_y(&g, v, phi, i, j, k, rhon) -
                             cflux_y(&g, v, phi, i, j - 1, k, rhon)) / dy;
                double fz = rdz[k] * (cflux_z(&g, w, phi, i, j, k, rho) -
                                      cflux_z(&g, w, phi, i, j, k - 1, rho));
                s[at(&g, i, j, k)] = -(fx + fy + fz) / rhon[k];
            }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * TVD advection of momentum: the ULTIMATE scheme of Sec. 3.1 applied to the
 * velocity components themselves (MONC offers it as the alternative to PW for
 * momentum; the paper gives no formulas).  Each velocity component has its
 * own control volume on the C-grid.  The mass flux through each face of that
 * volume is the one the PW scheme above uses, and the value carried through
 * the face is the ULTIMATE-limited QUICKEST value of the advected component
 * along the flux direction, upwind by the sign of the mass flux.  With the
 * mean of the two values beside each face in place of the limited value the
 * scheme is exactly PW (the `centred` switch; used only to check that).
 *
 *   u at (i+1/2, j, k):
 *     x-face at the centre of cell i+1:  m = rhon_k (u_i + u_{i+1})/2
 *     y-face at (i+1/2, j+1/2):          m = rhon_k (v_{i,j} + v_{i+1,j})/2
 *     z-face at (i+1/2, j, k+1/2):       m = rho_k (w_{i,k} + w_{i+1,k})/2 for
 *                                        k < nz-1; none through ground or lid
 *     su = -(1/rhon_k)[(Fx_{i+1}-Fx_i)/dx + (Fy_{j+1/2}-Fy_{j-1/2})/dy
 *                      + rdz_k (Fz_{k+1/2}-Fz_{k-1/2})]
 *   v alike with the roles of x and y exchanged.
 *   w at (i, j, k+1/2), k < nz-1, with a_k, b_k of the PW w-equation:
 *     x-face at (i+1/2, j, k+1/2):       m = a_k u_{i,k} + b_k u_{i,k+1}
 *     y-face alike with v
 *     z-face at the centre of cell q, between w_{q-1} and w_q (q = 0..nz-1):
 *                                        m = (rho_{q-1} w_{q-1} + rho_q w_q)/2
 *     sw = -(1/rho_k)[(Fx_{i+1/2}-Fx_{i-1/2})/dx + (Fy_{j+1/2}-Fy_{j-1/2})/dy
 *                     + rdzn_k (Fz_{k+1}-Fz_k)],   sw_{nz-1} = 0.
 *   The ground face w_{-1} and the lid w_{nz-1} are values of w (both 0).
 *
 * Courant number of a face: |m| divided by the reference density where the
 * face sits, times dt over the distance between the two values beside it --
 * rhon_k with dx or dy for the lateral faces of u and v, rho_k with dzn_k for
 * their z-faces, rho_k with dx or dy for the lateral faces of w, rhon_q with
 * dz_q for the z-faces of w.  A z-stencil whose far-upwind value does not
 * exist (u, v: levels 0..nz-1; w: faces -1..nz-1) takes the upwind value.
 * Computes the points i in [i0,i1), j in [j0,j1), all k.  Neighbours at
 * wrapped periodic indices; halos are not read.  Returns OR_ECFL (after
 * filling the outputs) when a Courant number exceeds 1; *cmax_out, if given,
 * receives the largest one met.
 * ------------------------------------------------------------------------- */
typedef struct {
    grid_t g;
    double dx, dy, dt;
    const double *rdz, *rho, *rhon;
    const vgeom_t *vg;
    int centred;
} momctx_t;

/* value at wrapped lateral indices */
static inline double fv(const momctx_t *M, const double *f, int i, int j, int k) {
    return f[at(&M->g, posmod(i, M->g.nx), posmod(j, M->g.ny), k)];
}

/* w at wrapped lateral indices with the ground and lid set to zero */
static inline double wv(const momctx_t *M, const double *w, int i, int j, int k) {
    if (k < 0 || k >= M->g.nz - 1) return 0.0;
    return fv(M, w, i, j, k);
}

/* Value carried through a face with mass flux m: p0, p1 the values beside the
 * face (p0 on the lower-index side), pm and p2 the next ones out, has_pm and
 * has_p2 whether those exist. */
static double mom_face(const momctx_t *M, double m, double c, double pm, double p0,
                       double p1, double p2, int has_pm, int has_p2) {
    if (M->centred) return 0.5 * (p0 + p1);
    if (m >= 0.0) return has_pm ? oracle_ultimate_face(pm, p0, p1, c) : p0;
    return has_p2 ? oracle_ultimate_face(p2, p1, p0, c) : p1;
}

static inline void note_c(double c, double *cmax) {
    if (c > *cmax) *cmax = c;
}

/* u-equation fluxes.  ux: face between u_{i} and u_{i+1}. */
static double fu_x(const momctx_t *M, const double *u, int i, int j, int k, double *cm) {
    double a = (fv(M, u, i, j, k) + fv(M, u, i + 1, j, k)) / 2.0;
    double c = fabs(a) * M->dt / M->dx;
    note_c(c, cm);
    double pf = mom_face(M, a, c, fv(M, u, i - 1, j, k), fv(M, u, i, j, k),
                         fv(M, u, i + 1, j, k), fv(M, u, i + 2, j, k), 1, 1);
    return M->rhon[k] * a * pf;
}
/* face between u_{i,j} and u_{i,j+1} */
static double fu_y(const momctx_t *M, const double *u, const double *v, int i, int j, int k,
                   double *cm) {
    double a = (fv(M, v, i, j, k) + fv(M, v, i + 1, j, k)) / 2.0;
    double c = fabs(a) * M->dt / M->dy;
    note_c(c, cm);
    double pf = mom_face(M, a, c, fv(M, u, i, j - 1, k), fv(M, u, i, j, k),
                         fv(M, u, i, j + 1, k), fv(M, u, i, j + 2, k), 1, 1);
    return M->rhon[k] * a * pf;
}
/* face between u_{i,j,k} and u_{i,j,k+1}; zero through ground and lid */
static double fu_z(const momctx_t *M, const double *u, const double *w, int i, int j, int k,
                   double *cm) {
    int nz = M->g.nz;
    if (k < 0 || k >= nz - 1) return 0.0;
    double a = (wv(M, w, i, j, k) + wv(M, w, i + 1, j, k)) / 2.0;
    double c = fabs(a) * M->dt * M->vg->rdzn[k];
    note_c(c, cm);
    double pm = k - 1 >= 0 ? fv(M, u, i, j, k - 1) : 0.0;
    double p2 = k + 2 <= nz - 1 ? fv(M, u, i, j, k + 2) : 0.0;
    double pf = mom_face(M, a, c, pm, fv(M, u, i, j, k), fv(M, u, i, j, k + 1), p2,
                         k - 1 >= 0, k + 2 <= nz - 1);
    return M->rho[k] * a * pf;
}

/* v-equation fluxes (x and y exchanged). */
static double fv_x(const momctx_t *M, const double *u, const double *v, int i, int j, int k,
                   double *cm) {
    double a = (fv(M, u, i, j, k) + fv(M, u, i, j + 1, k)) / 2.0;
    double c = fabs(a) * M->dt / M->dx;
    note_c(c, cm);
    double pf = mom_face(M, a, c, fv(M, v, i - 1, j, k), fv(M, v, i, j, k),
                         fv(M, v, i + 1, j, k), fv(M, v, i + 2, j, k), 1, 1);
    return M->rhon[k] * a * pf;
}
static double fv_y(const momctx_t *M, const double *v, int i, int j, int k, double *cm) {
    double a = (fv(M, v, i, j, k) + fv(M, v, i, j + 1, k)) / 2.0;
    double c = fabs(a) * M->dt / M->dy;
    note_c(c, cm);
    double pf = mom_face(M, a, c, fv(M, v, i, j - 1, k), fv(M, v, i, j, k),
                         fv(M, v, i, j + 1, k), fv(M, v, i, j + 2, k), 1, 1);
    return M->rhon[k] * a * pf;
}
static double fv_z(const momctx_t *M, const double *v, const double *w, int i, int j, int k,
                   double *cm) {
    int nz = M->g.nz;
    if (k < 0 || k >= nz - 1) return 0.0;
    double a = (wv(M, w, i, j, k) + wv(M, w, i, j + 1, k)) / 2.0;
    double c = fabs(a) * M->dt * M->vg->rdzn[k];
    note_c(c, cm);
    double pm = k - 1 >= 0 ? fv(M, v, i, j, k - 1) : 0.0;
    double p2 = k + 2 <= nz - 1 ? fv(M, v, i, j, k + 2) : 0.0;
    double pf = mom_face(M, a, c, pm, fv(M, v, i, j, k), fv(M, v, i, j, k + 1), p2,
                         k - 1 >= 0, k + 2 <= nz - 1);
    return M->rho[k] * a * pf;
}

/* w-equation fluxes at level k (k < nz-1).  wx: face between w_i and w_{i+1}. */
static double fw_x(const momctx_t *M, const double *u, const double *w, int i, int j, int k,
                   double *cm) {
    const vgeom_t *vg = M->vg;
    double a = vg->dz[k] * M->rhon[k] / (2.0 * vg->dzn[k]);
    double b = vg->dz[k + 1] * M->rhon[k + 1] / (2.0 * vg->dzn[k]);
    double m = a * fv(M, u, i, j, k) + b * fv(M, u, i, j, k + 1);
    double c = fabs(m) / M->rho[k] * M->dt / M->dx;
    note_c(c, cm);
    double pf = mom_face(M, m, c, wv(M, w, i - 1, j, k), wv(M, w, i, j, k),
                         wv(M, w, i + 1, j, k), wv(M, w, i + 2, j, k), 1, 1);
    return m * pf;
}
static double fw_y(const momctx_t *M, const double *v, const double *w, int i, int j, int k,
                   double *cm) {
    const vgeom_t *vg = M->vg;
    double a = vg->dz[k] * M->rhon[k] / (2.0 * vg->dzn[k]);
    double b = vg->dz[k + 1] * M->rhon[k + 1] / (2.0 * vg->dzn[k]);
    double m = a * fv(M, v, i, j, k) + b * fv(M, v, i, j, k + 1);
    double c = fabs(m) / M->rho[k] * M->dt / M->dy;
    note_c(c, cm);
    double pf = mom_face(M, m, c, wv(M, w, i, j - 1, k), wv(M, w, i, j, k),
                         wv(M, w, i, j + 1, k), wv(M, w, i, j + 2, k), 1, 1);
    return m * pf;
}
/* face at the centre of cell q, between w_{q-1} and w_q (q = 0..nz-1) */
static double fw_z(const momctx_t *M, const double *w, int i, int j, int q, double *cm) {
    int nz = M->g.nz;
    double lo = q - 1 >= 0 ? M->rho[q - 1] * wv(M, w, i, j, q - 1) : 0.0; /* ground: w = 0 */
    double m = (lo + M->rho[q] * wv(M, w, i, j, q)) / 2.0;
    double c = fabs(m) / M->rhon[q] * M->dt * M->rdz[q];
    note_c(c, cm);
    double pf = mom_face(M, m, c, wv(M, w, i, j, q - 2), wv(M, w, i, j, q - 1),
                         wv(M, w, i, j, q), wv(M, w, i, j, q + 1), q - 2 >= -1,
                         q + 1 <= nz - 1);
    return m * pf;
}

int oracle_tvd_momentum(const double *u, const double *v, const double *w, double *su,
                        double *sv, double *sw, int nx, int ny, int nz, double dx,
                        double dy, const double *rdz, const double *rho,
                        const double *rhon, double dt, int centred, int i0, int i1,
                        int j0, int j1, double *cmax_out) {
    if (!u || !v || !w || !su || !sv || !sw || !rdz || !rho || !rhon) return OR_EINVAL;
    if (nx < 1 || ny < 1 || nz < 2 || !(dx > 0) || !(dy > 0) || !(dt >= 0))
        return OR_EINVAL;
    if (i0 < 0 || i1 > nx || j0 < 0 || j1 > ny || i0 > i1 || j0 > j1) return OR_EINVAL;
    vgeom_t vg;
    vgeom_make(&vg, rdz, nz);
    momctx_t M = {{nx, ny, nz}, dx, dy, dt, rdz, rho, rhon, &vg, centred};
    double cmax = 0.0;

#pragma omp parallel for schedule(static) reduction(max : cmax)
    for (int i = i0; i < i1; i++)
        for (int j = j0; j < j1; j++)
            for (int k = 0; k < nz; k++) {
                long c = at(&M.g, i, j, k);
                double ex = fu_x(&M, u, i, j, k, &cmax) - fu_x(&M, u, i - 1, j, k, &cmax);
                double ey = fu_y(&M, u, v, i, j, k, &cmax) - fu_y(&M, u, v, i, j - 1, k, &cmax);
                double ez = fu_z(&M, u, w, i, j, k, &cmax) - fu_z(&M, u, w, i, j, k - 1, &cmax);
                su[c] = -(1.0 / rhon[k]) * (ex / dx + ey / dy + rdz[k] * ez);

                ex = fv_x(&M, u, v, i, j, k, &cmax) - fv_x(&M, u, v, i - 1, j, k, &cmax);
                ey = fv_y(&M, v, i, j, k, &cmax) - fv_y(&M, v, i, j - 1, k, &cmax);
                ez = fv_z(&M, v, w, i, j, k, &cmax) - fv_z(&M, v, w, i, j, k - 1, &cmax);
                sv[c] = -(1.0 / rhon[k]) * (ex / dx + ey / dy + rdz[k] * ez);

                if (k == nz - 1) {
                    sw[c] = 0.0;
                    continue;
                }
                ex = fw_x(&M, u, w, i, j, k, &cmax) - fw_x(&M, u, w, i - 1, j, k, &cmax);
                ey = fw_y(&M, v, w, i, j, k, &cmax) - fw_y(&M, v, w, i, j - 1, k, &cmax);
                ez = fw_z(&M, w, i, j, k + 1, &cmax) - fw_z(&M, w, i, j, k, &cmax);
                sw[c] = -(1.0 / rho[k]) * (ex / dx + ey / dy + vg.rdzn[k] * ez);
            }
    vgeom_free(&vg);
    if (cmax_out) *cmax_out = cmax;
    return cmax > 1.0 ? OR_ECFL : OR_OK;
}
