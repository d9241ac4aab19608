/*
 * monc_adv.h -- C ABI of the MI355X advection library (libmoncadv.so).
 *
 * The operation is the advection component of the MONC LES dynamical core
 * (Brown et al., arXiv 2009.12850).  Sec. 2.1: advection is the longest
 * running component; the prognostic fields are u, v, w, theta and any number
 * of further scalars.  Sec. 3: each dynamics component adds a source term and
 * the field update integrates them last.  Sec. 3.1: momentum uses the
 * energy-conserving Piacsek-Williams scheme, scalars Leonard's ULTIMATE
 * (positivity-preserving, TVD) scheme.  Sec. 4.1: the single-precision
 * variant.  The discretisation itself (flux form on the Arakawa C grid,
 * QUICKEST face values with the ULTIMATE limiter, first-order upwind where
 * the far upwind cell lies outside the column, no flux through ground or lid)
 * is stated with each entry point below.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.   Every field is a dense [(nx+4)][(ny+4)][nz] array, z fastest, with
 *           a 2-deep periodic halo in x and y and none in z.  The advection
 *           calls read periodic neighbours at wrapped interior indices, so
 *           halo contents are never read by them (monc_halo_fill fills the
 *           halos for callers that need them).  Interior element
 *           (i,j,k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz, lives at
 *           ((i+2)*(ny+4) + (j+2))*nz + k.  Profiles rdz, rho, rhon are [nz]
 *           float64 arrays: rdz[k] = 1/dz_k (thickness of cell k), rho[k] =
 *           reference density on the top face of cell k, rhon[k] = at its
 *           centre.  w[k] is the vertical velocity on the top face of cell k;
 *           w[nz-1] is the lid and is treated as 0 whatever it holds.
 * Memory.   All array pointers are DEVICE pointers owned by the caller; the
 *           library keeps no pointer after a call returns and allocates no
 *           device memory outside an ensemble plan.  Scratch space is passed
 *           in as `workspace`, sized by the matching *_workspace_bytes call.
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *           enqueue work and never synchronise; results are ready when the
 *           stream is.
 * Errors.   Calls return MONC_OK or a negative code.  Arguments are validated
 *           before any HIP call (MONC_EINVAL, detail in monc_last_error(),
 *           which is thread-local).  A launch failure returns MONC_EHIP.
 *           Conditions found on the device (Courant number > 1, non-finite
 *           values) are written into the budgets array and turned into codes
 *           by monc_budgets_check() after the caller has synchronised.
 * Aliasing. Outputs must not alias inputs.
 * Limits.   nx, ny >= 1; 2 <= nz <= MONC_MAX_NZ; nscal <= MONC_MAX_SCALARS;
 *           dx, dy > 0; dt > 0 wherever TVD is involved.
 */
#ifndef MONC_ADV_H
#define MONC_ADV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *monc_stream_t;

enum {
    MONC_OK = 0,
    MONC_EINVAL = -1,
    MONC_EHIP = -2,
    MONC_ECFL = -3,
    MONC_ENONFINITE = -4,
    MONC_EUNSUPPORTED = -5
};

#define MONC_MAX_SCALARS 8
#define MONC_MAX_NZ 128

/* Storage types of the precision form (Sec. 4.1 marshals the fields into a
 * narrower type before advection and widens the source terms afterwards). */
enum { MONC_F64 = 0, MONC_F32 = 1, MONC_BF16 = 2 };

/* Budgets written by monc_step* when `budgets` is non-NULL (float64 array of
 * MONC_NBUDGET entries, device memory).  They describe the INPUT state of the
 * step and the tendencies computed from it:
 *   C_*  conservation sums: C_u = sum rhon dz su, C_v likewise,
 *        C_w = sum_{k<nz-1} rho dzn sw, C_s = sum rhon dz s_phi (all ~0 except
 *        C_w, which equals sum_ij (rho_0 w_0^2 - rho_{nz-2} w_{nz-2}^2)/4);
 *   P_*, Q_*  the two sides of the kinetic-energy identity of the PW scheme:
 *        P_u = sum rhon dz u su, Q_u = -sum dz (u^2/2)(D_i + D_{i+1})/2,
 *        P_w = sum rho dzn w sw, Q_w = -sum (w^2/2)(dz_k D_k + dz_{k+1} D_{k+1})/2,
 *        where D is the anelastic mass divergence of a cell;
 *   COURANT  the largest |u|dt/dx, |v|dt/dy, |w_k| dt/dzn_k over all faces;
 *   NONFINITE number of non-finite values written (output state or tendencies);
 *   M_s = sum rhon dz phi_s and MIN_s = min phi_s of the input scalars.
 * Sums run in a fixed order for a given grid, so they are bitwise repeatable. */
enum {
    MONC_B_CU = 0, MONC_B_CV, MONC_B_CW, MONC_B_PU, MONC_B_QU, MONC_B_PV,
    MONC_B_QV, MONC_B_PW, MONC_B_QW, MONC_B_COURANT, MONC_B_NONFINITE,
    MONC_B_SCALAR0 /* scalar s: C_s at 11+3s, M_s at 12+3s, MIN_s at 13+3s */
};
#define MONC_NBUDGET (MONC_B_SCALAR0 + 3 * MONC_MAX_SCALARS)

/* ---------------------------------------------------------------------------
 * Periodic halo fill (the halo swap that opens every timestep, Sec. 2.1,
 * on a single periodic domain).  fields: host array of nfields device
 * pointers; each field's 2-deep x-y halo, corners included, becomes a copy of
 * the interior at the wrapped index.  Bitwise copy.
 * ------------------------------------------------------------------------- */
int monc_halo_fill(int nfields, double *const *fields, int nx, int ny, int nz,
                   monc_stream_t stream);
int monc_halo_fill_f32(int nfields, float *const *fields, int nx, int ny, int nz,
                       monc_stream_t stream);
int monc_halo_fill_bf16(int nfields, uint16_t *const *fields, int nx, int ny,
                        int nz, monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Piacsek-Williams momentum source terms (Sec. 3.1, energy-conserving
 * scheme) in FP64.  Flux form on the C grid: each velocity component is
 * carried by the mass flux through the faces of its own staggered cell, the
 * face values being two-point means, with the anelastic densities rho/rhon
 * weighting the vertical fluxes, so that the kinetic-energy source summed over
 * a periodic domain is the energy flux through its boundary (zero here).
 * Outputs su, sv, sw (interior written, halo untouched; sw[...][nz-1] = 0).
 * ------------------------------------------------------------------------- */
int monc_advect_pw(const double *u, const double *v, const double *w,
                   double *su, double *sv, double *sw, int nx, int ny, int nz,
                   double dx, double dy, const double *rdz, const double *rho,
                   const double *rhon, monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Work-scaled PW (the experiment of Sec. 4 that raises the PW arithmetic to
 * that of the ULTIMATE scheme, about sixteen-fold): the PW source terms of
 * monc_advect_pw evaluated `work` times per grid point (1 <= work <=
 * MONC_MAX_WORK) on the same loaded values, each repetition chained to the
 * previous one so that none is merged or dropped; the result does not depend
 * on `work`.  dtype MONC_F64 (double in and out) or MONC_F32 (float in and
 * out).  Bytes per point are fixed (one read of u, v, w, one write of su, sv,
 * sw); arithmetic is 92 floating-point operations per point per repetition.
 * Halos are not read.  A measurement kernel: one thread per grid point.
 * ------------------------------------------------------------------------- */
#define MONC_MAX_WORK 64
int monc_advect_pw_scaled(int dtype, const void *u, const void *v, const void *w, void *su,
                          void *sv, void *sw, int nx, int ny, int nz, double dx, double dy,
                          const double *rdz, const double *rho, const double *rhon, int work,
                          monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * ULTIMATE-limited QUICKEST (TVD) scalar source terms (Sec. 3.1,
 * positivity-preserving scheme) in FP64, for nscal scalars at once.  q and sq
 * are host arrays of nscal device pointers.  Face values are third-order
 * QUICKEST values clipped by the ULTIMATE limiter between the upwind cell and
 * the monotone bound set by the Courant number; dt enters through the Courant
 * numbers, and a face with Courant number above 1 is reported in the budgets
 * of the fused calls (here the result is then undefined).
 * ------------------------------------------------------------------------- */
int monc_advect_tvd(const double *u, const double *v, const double *w,
                    int nscal, const double *const *q, double *const *sq,
                    int nx, int ny, int nz, double dx, double dy,
                    const double *rdz, const double *rho, const double *rhon,
                    double dt, monc_stream_t stream);

/* The PW part and the TVD part of monc_advect for one narrow storage type
 * (Sec. 4.1's single-precision advection as separate calls): FP32 copies
 * (_f32) or bfloat16 bits (_bf16) in, FP32 arithmetic, FP32 source terms out;
 * the layout, validation and aliasing rules of monc_advect_pw and
 * monc_advect_tvd, and phi0 (host [nscal], or NULL for zeros) as for
 * monc_advect.  The results are those of monc_advect with the same dtype. */
int monc_advect_pw_f32(const float *u, const float *v, const float *w, float *su, float *sv,
                       float *sw, int nx, int ny, int nz, double dx, double dy,
                       const double *rdz, const double *rho, const double *rhon,
                       monc_stream_t stream);
int monc_advect_pw_bf16(const uint16_t *u, const uint16_t *v, const uint16_t *w, float *su,
                        float *sv, float *sw, int nx, int ny, int nz, double dx, double dy,
                        const double *rdz, const double *rho, const double *rhon,
                        monc_stream_t stream);
int monc_advect_tvd_f32(const float *u, const float *v, const float *w, int nscal,
                        const float *const *q, float *const *sq, const double *phi0, int nx,
                        int ny, int nz, double dx, double dy, const double *rdz,
                        const double *rho, const double *rhon, double dt,
                        monc_stream_t stream);
int monc_advect_tvd_bf16(const uint16_t *u, const uint16_t *v, const uint16_t *w, int nscal,
                         const uint16_t *const *q, float *const *sq, const double *phi0,
                         int nx, int ny, int nz, double dx, double dy, const double *rdz,
                         const double *rho, const double *rhon, double dt,
                         monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Fused source terms: PW for u, v, w and TVD for nscal scalars in one pass, in the
 * storage type `dtype` (MONC_F64: double in, double out; MONC_F32: float in,
 * float out; MONC_BF16: bfloat16 bits in, float out).  in = host array of
 * 3+nscal device pointers (u, v, w, scalars), out likewise.  phi0 (host array
 * of nscal doubles, may be NULL = zeros) gives the constant each stored scalar
 * is an anomaly from: the source term returned is that of phi0 + stored value,
 * i.e. the stored anomaly's term minus phi0*D/rhon (exact by the affine
 * equivariance of the flux form).  Halos are not read.
 * ------------------------------------------------------------------------- */
int monc_advect(int dtype, const void *const *in, void *const *out, int nscal,
                const double *phi0, int nx, int ny, int nz, double dx,
                double dy, const double *rdz, const double *rho,
                const double *rhon, double dt, monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * One forward step of advection and field update (the update integrates
 * the source terms last, Sec. 3): PW + TVD from state_in (periodic neighbours read
 * at wrapped indices), state_out = state_in + dt * s, w lid = 0, and
 * optionally the FP64 budgets.  state_in/state_out: host arrays of 3+nscal
 * device pointers, FP64, state_out must not alias state_in (halos are neither
 * read nor written).  budgets: device float64
 * [MONC_NBUDGET] or NULL.  workspace: device memory of at least
 * monc_step_workspace_bytes(nx, ny, nz, nscal) bytes when budgets != NULL.
 * ------------------------------------------------------------------------- */
size_t monc_step_workspace_bytes(int nx, int ny, int nz, int nscal);
int monc_step(double *const *state_in, double *const *state_out, int nscal,
              int nx, int ny, int nz, double dx, double dy, const double *rdz,
              const double *rho, const double *rhon, double dt,
              double *budgets, void *workspace, monc_stream_t stream);

/* monc_step with budgets, allocation-free: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments as monc_step without the
 * workspace; budgets (device float64 [MONC_NBUDGET]) is required.  The
 * budget partial rows (one per workgroup of the launch, MONC_NBUDGET doubles
 * each) go to a static device array of MONC_STATIC_MAX_ROWS rows (2.3 MB)
 * that the library holds on every device it runs on until the process ends;
 * grids that need more rows (monc_step_workspace_bytes / (8 * MONC_NBUDGET))
 * return MONC_EINVAL.  No allocation happens on any call; the first call on a
 * device looks the array's address up once.  Every call on one device shares
 * the array: calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller.  Nothing in the array needs to
 * start at zero (every row is written before it is read).  Results and budgets
 * are bitwise those of monc_step with a workspace. */
#define MONC_STATIC_MAX_ROWS 8192
#define MONC_STATIC_MAX_DEVICES 64
int monc_step_static(double *const *state_in, double *const *state_out, int nscal,
                     int nx, int ny, int nz, double dx, double dy, const double *rdz,
                     const double *rho, const double *rhon, double dt, double *budgets,
                     monc_stream_t stream);

/* The same step with the tendencies computed in FP32 from the FP64 state
 * (scalars first reduced by phi0 in FP64, then rounded) and accumulated in
 * FP64: the single-precision advection of Sec. 4.1 without a separate
 * marshalling pass.  Budgets stay FP64. */
int monc_step_mixed(double *const *state_in, double *const *state_out,
                    int nscal, const double *phi0, int nx, int ny, int nz,
                    double dx, double dy, const double *rdz, const double *rho,
                    const double *rhon, double dt, double *budgets,
                    void *workspace, monc_stream_t stream);

/* Marshalling (Sec. 4.1): write a narrower working copy of FP64 fields.
 * dtype MONC_F32 or MONC_BF16 (round to nearest even); work[f] receives
 * src[f] - offset[f] (offset may be NULL = zeros) over the whole padded array,
 * halo included.  src[f] and work[f] must be 16-byte aligned (MONC_EINVAL
 * otherwise); a streaming pass of 12 (FP32) or 10 (BF16) bytes per value. */
int monc_cast_working(int dtype, int nfields, const double *const *src,
                      void *const *work, const double *offset, int nx, int ny,
                      int nz, monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Batched ensemble.  Many independent LES members of uneven size advance
 * together, each with the monc_step_mixed step (FP32 source terms, FP64
 * state): one persistent launch per column-height class (nz <= 64, nz <= 128)
 * walks a cost-sorted list of (member, tile) work items, and monc_ensemble_run
 * replays N steps captured once into a hipGraph.  The segment length and grid
 * size of each class are picked by timing candidates on the members (tune !=
 * 0), cached in the JSON file `tune_cache` (may be NULL: no cache).  Results
 * are bitwise those of monc_step_mixed on each member alone.
 * members: host array; state[p][f] are device FP64 arrays in the usual layout
 * (f = u, v, w, scalars), state[0] the initial state; the plan keeps the
 * pointers until destroyed and owns only its own small device tables.
 * nscal <= 3 (MONC_EUNSUPPORTED otherwise).  monc_ensemble_parity() tells
 * which buffer (0/1) holds the current state.  Calls on one plan must not
 * overlap.
 * ------------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dt;
    const double *rdz, *rho, *rhon;
    double *state[2][3 + MONC_MAX_SCALARS];
    double phi0[MONC_MAX_SCALARS];
} monc_member;

typedef struct monc_ensemble monc_ensemble;

int monc_ensemble_create(const monc_member *members, int nmembers, int nscal,
                         const char *tune_cache, int tune, monc_ensemble **plan);
int monc_ensemble_run(monc_ensemble *plan, int nsteps, monc_stream_t stream);

/* Budgets of every member and every step (the FP64 checks of Sec. 3.1 kept
 * on the device for the batched form).  budgets: device float64 array of
 * nslots x nmembers x MONC_NBUDGET, owned by the caller and kept by the plan
 * until detached (budgets = NULL) or the plan is destroyed.  Once attached,
 * step t (t = 0 .. N-1) of a monc_ensemble_run of N steps writes, in slot t,
 * member m's budgets at [(t * nmembers + m) * MONC_NBUDGET], with the
 * meaning of monc_step_mixed's budgets (of the state the step reads);
 * monc_ensemble_step writes slot 0.  A run of more than nslots steps returns
 * MONC_EINVAL.  The plan allocates one row of partials per work item (its
 * own memory, freed on detach or destroy); attaching or detaching waits for
 * the device and drops the captured graphs.  Each member's sums run in a
 * fixed order, so repeated runs give the same bits. */
int monc_ensemble_set_budgets(monc_ensemble *plan, double *budgets, int nslots);
int monc_ensemble_step(monc_ensemble *plan, monc_stream_t stream);
int monc_ensemble_parity(const monc_ensemble *plan);
int monc_ensemble_info(const monc_ensemble *plan, int *ti, int *grid, int *nitems);
int monc_ensemble_destroy(monc_ensemble *plan);

/* ---------------------------------------------------------------------------
 * Learned coarse-grid flux correction.  A fine run is restricted to a
 * grid 4x coarser in x, y and z; a small MLP (300 inputs = the 5x5x3
 * neighbourhood of u, v, w, theta around a cell, standardised; two 64-unit
 * GELU layers; 4 outputs = correction fluxes of u, v, w, theta through one face)
 * is trained on the difference between the restricted fine evolution and the
 * plain coarse PW/TVD step, and its flux divergence corrects the coarse step.
 * Evaluation and training use BF16 MFMA with FP32 accumulation; FP32 master
 * weights; Adam.  The plain step is the fallback.
 *
 * Feature order: index f*80 + (a*5 + b)*3 + c for field f in (u, v, w,
 * theta), a = offset along the face normal + 2, b = tangential offset + 2, c =
 * vertical offset + 1; periodic in x and y, edge-replicated in z; orient 1
 * (y-faces) exchanges x and y and swaps u and v; slots f*80 + 75..79 are 0
 * (300 values in 320 slots; W1 columns follow the same order).
 * Parameter vector (FP32, MONC_MLP_NPARAM): W1[64][320] | b1[64] |
 * W2[64][64] (W2[out][in]) | b2[64] | W3[4][64] | b3[4].
 * BF16 weight pack (MONC_MLP_WPACK uint16): W1 | W2 | W3 padded to [32][64].
 * ------------------------------------------------------------------------- */
#define MONC_MLP_NIN 300
#define MONC_MLP_K 320
#define MONC_MLP_H 64
#define MONC_MLP_NOUT 4
#define MONC_MLP_NPARAM (MONC_MLP_H * MONC_MLP_K + MONC_MLP_H + MONC_MLP_H * MONC_MLP_H + \
                         MONC_MLP_H + MONC_MLP_NOUT * MONC_MLP_H + MONC_MLP_NOUT)
#define MONC_MLP_WPACK (MONC_MLP_H * MONC_MLP_K + MONC_MLP_H * MONC_MLP_H + 32 * MONC_MLP_H)

/* Fine -> coarse restriction (nx, ny, nz multiples of 4): scalars are
 * mass-weighted means over 4x4x4 blocks, u and v mass-flux-weighted means over
 * the coarse face, w the mean over the coarse top face; coarse profiles
 * rdz_c, rho_c, rhon_c [nz/4] (thickness sum, top-face density, mass-weighted
 * centre density).  The coarse mass divergence is the volume-weighted mean of
 * the fine one.  fine/coarse: host arrays of 3+nscal device pointers. */
int monc_restrict4(int nscal, const double *const *fine, double *const *coarse, int nx,
                   int ny, int nz, const double *rdz, const double *rho,
                   const double *rhon, double *rdz_c, double *rho_c, double *rhon_c,
                   monc_stream_t stream);
/* Gather BF16 features (rows [ncells][320]) of cells (device linear indices
 * (i*ny + j)*nz + k, or NULL for all cells in that order; a listed cell outside
 * the grid gives a zero row).  state: host array of 4 device pointers (u, v, w,
 * theta); norm: host [8] = mean, std per field; X 16-byte aligned. */
int monc_mlp_features(const double *const *state, int nx, int ny, int nz,
                      const double *norm, int orient, const int *cells, int ncells,
                      uint16_t *X, monc_stream_t stream);
/* BF16 weight pack from the FP32 parameters. */
int monc_mlp_pack(const float *params, uint16_t *wpack, monc_stream_t stream);
/* Y[m][4] = MLP(X[m][320]).  H1, H2 (BF16 [m][64]) and Z1, Z2 (FP32 [m][64],
 * pre-activations) are saved for training when non-NULL. */
int monc_mlp_forward(const uint16_t *X, int m, const float *params, const uint16_t *wpack,
                     float *Y, uint16_t *H1, uint16_t *H2, float *Z1, float *Z2,
                     monc_stream_t stream);
/* Inference over every cell, cell order (i*ny + j)*nz + k: Y[nx*ny*nz][4] is
 * bitwise what monc_mlp_features (cells = NULL, same orient) followed by
 * monc_mlp_forward gives, but the features are gathered from the fields into
 * the matrix operands directly and never stored.  state: host array of 4
 * device pointers (u, v, w, theta); norm: host [8]; wpack 16-byte aligned.
 * orient 2 evaluates both face orientations (Y[2][nx*ny*nz][4]: x-faces,
 * then y-faces), on 32-level grids with ny % 4 == 0 from one staged
 * neighbourhood per tile (the y-face rows use the same 5 x 5 x 3 cells with x
 * and y exchanged), elsewhere as two launches; each half is bitwise the
 * single-orientation result. */
int monc_mlp_infer(const double *const *state, int nx, int ny, int nz, const double *norm,
                   int orient, const float *params, const uint16_t *wpack, float *Y,
                   monc_stream_t stream);
/* Parameter gradient grad[MONC_MLP_NPARAM] from dY[m][4] and the saved forward
 * activations; deterministic.  workspace >= monc_mlp_backward_workspace_bytes(m). */
size_t monc_mlp_backward_workspace_bytes(int m);
int monc_mlp_backward(const uint16_t *X, const uint16_t *H1, const uint16_t *H2,
                      const float *Z1, const float *Z2, const float *dY, int m,
                      const uint16_t *wpack, float *grad, void *workspace,
                      monc_stream_t stream);
/* Loss of the flux-divergence correction on b sampled cells (device linear
 * indices `cells`).  Y4 = MLP outputs of the rows x(i), x(i-1), y(j), y(j-1)
 * of those cells (b rows each, y outputs in the exchanged frame).  Correction
 * c_q = -(gx(i) - gx(i-1) + gy(j) - gy(j-1)) / rhohat_q(k); target r_q / scale_q
 * with the residual r_q = (c1_q - c0_q)/dt - tend_q of the coarse fields
 * (c0, c1: the restricted state at t and t+dt; tend: the plain coarse source
 * terms at c0; host arrays of 4 device pointers, u v w theta); w on the lid
 * is masked, and so are all terms of a listed cell outside the grid.
 * loss[0] = inv_count * sum (c - target)^2; dY4 = its gradient.
 * workspace >= monc_mlp_loss_workspace_bytes(b). */
size_t monc_mlp_loss_workspace_bytes(int b);
int monc_mlp_loss(const float *Y4, int b, const int *cells, const double *const *c0,
                  const double *const *c1, const double *const *tend, int nx, int ny, int nz,
                  double dt, const double *scale, const double *rho, const double *rhon,
                  double inv_count, float *dY4, float *loss, void *workspace,
                  monc_stream_t stream);
/* One Adam step (t >= 1) on the FP32 parameters, then the BF16 pack. */
int monc_mlp_adam(float *params, float *m1, float *m2, const float *grad, int t, double lr,
                  double beta1, double beta2, double eps, uint16_t *wpack,
                  monc_stream_t stream);
/* One training step of the correction, fused.  For b sampled cells (device
 * linear indices `cells`, as for monc_mlp_loss), one launch computes the
 * features of the four face rows of every cell -- x(i), x(i-1), y(j), y(j-1),
 * the i-1 and j-1 neighbours taken with the periodic wrap -- the forward pass,
 * the loss and dY, and the parameter gradient, keeping every activation on
 * chip; a second launch sums the gradient in a fixed order into
 * grad[MONC_MLP_NPARAM], takes one Adam step (t >= 1) on the FP32 parameters,
 * writes their BF16 pack and loss[0] (the loss before the update).  Each row's
 * features, activations, loss terms and dY are the operations of
 * monc_mlp_features, monc_mlp_forward and monc_mlp_loss on the same numbers;
 * the gradient is monc_mlp_backward's up to the order of the sum over rows.  A
 * listed cell outside the grid contributes nothing.  c0, c1, tend: host arrays
 * of 4 device pointers (u v w theta, padded coarse fields); norm: host [8]
 * (mean, std per field); scale: host [4]; rho, rhon: device [nz]; wpack
 * 16-byte aligned; workspace >= monc_mlp_train_workspace_bytes(b) bytes of
 * device memory.  Deterministic for a given b. */
size_t monc_mlp_train_workspace_bytes(int b);
int monc_mlp_train_step(const double *const *c0, const double *const *c1,
                        const double *const *tend, int nx, int ny, int nz, const double *norm,
                        const int *cells, int b, double dt, const double *scale,
                        const double *rho, const double *rhon, double inv_count, float *params,
                        float *m1, float *m2, int t, double lr, double beta1, double beta2,
                        double eps, uint16_t *wpack, float *grad, float *loss, void *workspace,
                        monc_stream_t stream);
/* Corrected coarse step for u, v, w, theta: out = in + dt (tend + c_q), with
 *   c_q = -scale_q (gx_q(i) - gx_q(i-1) + gy_q(j) - gy_q(j-1)) / rhohat_q(k)
 * for u, v, w, where gx, gy are [nx*ny*nz][4] face outputs of the network (gy
 * in the exchanged frame, u and v swapped) and rhohat = rho(k)/rho(0) for w,
 * rhon(k)/rhon(0) otherwise.  tend: the plain source terms (monc_advect of
 * state_in).  Guards:
 *  - theta: the correction flux through each lateral face, G = h rhon(0)
 *    scale_3 g (h = dx or dy), is clamped so that the corrected face value
 *    (plain flux + G) / (rhon(k) * normal velocity) stays within the ULTIMATE
 *    admissible interval of that face (between the upwind value and the
 *    monotone bound; only the upwind value at a local extremum);
 *  - if any face output is not finite, the step is the plain one;
 *  - if the corrected state's kinetic energy (sum of m u^2 + m v^2 + m_w w^2,
 *    m = rhon dz, m_w = rho dz) or theta variance (mass-weighted) exceeds
 *    `growth` times that of the plain step from the same state, the step is
 *    the plain one.
 * flags: device int[4]; flags[0] is scratch, flags[1] and flags[2] count the
 * steps that fell back (non-finite, growth), flags[3] counts the clamped theta
 * faces of the steps that did not fall back for non-finite outputs; the
 * caller zeroes flags[1..3] once.  gx, gy 16-byte aligned.  workspace: device
 * memory of at least monc_correct_step_workspace_bytes(nx, ny, nz) bytes;
 * deterministic. */
size_t monc_correct_step_workspace_bytes(int nx, int ny, int nz);
int monc_correct_step(double *const *state_in, double *const *tend, const float *gx,
                      const float *gy, double *const *state_out, int nx, int ny, int nz,
                      double dx, double dy, const double *scale, const double *rdz,
                      const double *rho, const double *rhon, double dt, double growth,
                      int *flags, void *workspace, monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Other source terms of the dynamics group and the combined step (the hybrid
 * structure of Sec. 3 and its hybrid-dynamics figure: the other components of
 * the dynamics group run beside the advection, then every source term is
 * combined before the fields are stepped).  The paper names no such
 * component; the two provided are the f-plane Coriolis force toward a
 * geostrophic wind and the buoyancy of theta:
 *   su = fcor (vbar - vg), vbar = mean of v at (i,j), (i+1,j), (i,j-1), (i+1,j-1)
 *   sv = -fcor (ubar - ug), ubar = mean of u at (i,j), (i-1,j), (i,j+1), (i-1,j+1)
 *   sw = grav ((th_k + th_{k+1})/2 - th0) / th0 for k < nz-1, 0 on the lid.
 * Periodic neighbours are read at wrapped indices; halos are neither read nor
 * written.  All fields are device FP64 arrays in the usual padded layout.
 * Errors: MONC_EINVAL for NULL pointers, bad sizes, non-finite parameters,
 * th0 <= 0, or aliasing outputs.
 * ------------------------------------------------------------------------- */
typedef struct {
    double fcor;     /* Coriolis parameter (1/s) */
    double ug, vg;   /* geostrophic wind (m/s) */
    double grav;     /* gravitational acceleration (m/s^2) */
    double th0;      /* reference potential temperature (K), > 0 */
} monc_dyn_params;

/* The other dynamics source terms alone: su, sv, sw from u, v and theta. */
int monc_dyn_tend(const double *u, const double *v, const double *theta, double *su,
                  double *sv, double *sw, int nx, int ny, int nz,
                  const monc_dyn_params *p, monc_stream_t stream);

/* Combine source terms and step: out[f] = in[f] + dt (ta[f] + tb[f]) for f
 * in 0..nfields-1 (fields ordered u, v, w, scalars; w = 0 on the lid).  tb may
 * be NULL, and so may any tb[f]: that field then steps with ta alone.  in, ta,
 * tb, out: host arrays of device pointers; out must not alias an input. */
int monc_combine_step(int nfields, const double *const *in, const double *const *ta,
                      const double *const *tb, double *const *out, int nx, int ny,
                      int nz, double dt, monc_stream_t stream);

/* The hybrid step on two streams: the other dynamics source terms on
 * side_stream (into dyn_tend[0..2], device buffers of the caller) while the
 * advection source terms of all 3+nscal fields run on `stream` (into
 * tend[0..2+nscal]); `stream` then waits for the side stream and the combine
 * pass steps the fields: state_out = state_in + dt (s_adv + s_dyn), s_dyn = 0
 * for the scalars.  theta is scalar 0 (nscal >= 1); halos are neither read
 * nor written.  tend and dyn_tend must not alias the states or each other.
 * side_stream may equal stream (then the passes run one after another).  On
 * return every pass is enqueued; the side stream also waits for `stream` at
 * entry, so both streams see state_in as it is when the call is made.
 * Results are bitwise those of monc_step_dyn. */
int monc_hybrid_step(double *const *state_in, double *const *state_out,
                     double *const *tend, double *const *dyn_tend, int nscal, int nx,
                     int ny, int nz, double dx, double dy, const double *rdz,
                     const double *rho, const double *rhon, double dt,
                     const monc_dyn_params *p, monc_stream_t stream,
                     monc_stream_t side_stream);

/* The same step in one pass: the Coriolis and buoyancy terms are added to the
 * PW source terms inside the advection march, so no source term goes through
 * HBM (the paper's further-work idea of combining source terms on the device
 * before they leave it, Sec. 5).  Arguments as monc_step without budgets;
 * nscal >= 1 (theta = scalar 0). */
int monc_step_dyn(double *const *state_in, double *const *state_out, int nscal, int nx,
                  int ny, int nz, double dx, double dy, const double *rdz,
                  const double *rho, const double *rhon, double dt,
                  const monc_dyn_params *p, monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * The FP64 step with MONC's other scalar scheme: every scalar advected with
 * the centred flux form (the PW scheme of Sec. 3.1 applied to a cell-centred
 * field) instead of the TVD scheme; momentum as in monc_step.  The face value
 * is the mean of the two cells beside the face; the flux through a z-face is
 * rho_k w_k times that mean, zero through the ground and the lid.  Centred
 * fluxes are not bounded: this is the cheap, non-monotone choice.  Arguments
 * as monc_step without budgets.
 * ------------------------------------------------------------------------- */
int monc_step_pw_scalars(double *const *state_in, double *const *state_out, int nscal,
                         int nx, int ny, int nz, double dx, double dy, const double *rdz,
                         const double *rho, const double *rhon, double dt,
                         monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * TVD advection of momentum: the ULTIMATE scheme of Sec. 3.1 (there used for
 * the scalars) applied to u, v and w, the alternative to PW for momentum.  The
 * mass flux through each face of a velocity's control volume is the PW one,
 * and the value carried through the face is the ULTIMATE-limited QUICKEST
 * value of that velocity component along the flux direction, upwind by the
 * sign of the mass flux (with the mean of the two values beside the face it
 * is PW):
 *   u at (i+1/2,j,k): x-faces at cell centres carry rhon_k (u_i + u_{i+1})/2,
 *     y-faces at (i+1/2,j+1/2) rhon_k (v_{ij} + v_{i+1,j})/2, z-faces at
 *     (i+1/2,j,k+1/2) rho_k (w_{ik} + w_{i+1,k})/2, none through ground or lid;
 *     su = -(1/rhon_k)[dFx/dx + dFy/dy + rdz_k dFz];  v likewise in y;
 *   w at (i,j,k+1/2), k < nz-1: lateral faces carry a_k u_k + b_k u_{k+1} with
 *     a_k = dz_k rhon_k/(2 dzn_k), b_k = dz_{k+1} rhon_{k+1}/(2 dzn_k); the
 *     z-face at the centre of cell q carries (rho_{q-1} w_{q-1} + rho_q w_q)/2
 *     with w = 0 on the ground and the lid; sw = -(1/rho_k)[dFx/dx + dFy/dy
 *     + dFz/dzn_k], sw = 0 on the lid.
 * Courant number of a face: |mass flux| / (reference density where the face
 * sits) * dt / (distance between the two values beside it).  A z-stencil
 * whose far-upwind value does not exist takes the upwind value.
 *
 * u, v, w: FP64 device fields; su, sv, sw: FP64 device outputs (interior
 * written, halos untouched).  cmax: device double or NULL; when given it is
 * overwritten with the largest Courant number of the momentum faces (the
 * scheme needs <= 1; beyond that the values are unspecified).  Halos are not
 * read.  Outputs must not alias inputs or each other.
 * ------------------------------------------------------------------------- */
int monc_advect_tvd_momentum(const double *u, const double *v, const double *w, double *su,
                             double *sv, double *sw, int nx, int ny, int nz, double dx,
                             double dy, const double *rdz, const double *rho,
                             const double *rhon, double dt, double *cmax,
                             monc_stream_t stream);

/* One forward step with TVD for every field: the momentum as in
 * monc_advect_tvd_momentum, the scalars as in monc_step; state_out = state_in
 * + dt * s, w lid = 0.  Two passes on `stream`: the momentum pass writes
 * u, v, w of state_out, the scalar march the scalars.  Arguments as monc_step
 * without budgets; cmax as above (momentum faces only; the scalar faces use
 * the face velocities, whose largest Courant number monc_step's budgets
 * report). */
int monc_step_tvd_momentum(double *const *state_in, double *const *state_out, int nscal,
                           int nx, int ny, int nz, double dx, double dy, const double *rdz,
                           const double *rho, const double *rhon, double dt, double *cmax,
                           monc_stream_t stream);

/* ---------------------------------------------------------------------------
 * Streaming ceiling (measurement).  The HBM rate this device reaches with
 * plain coalesced traffic, the yardstick for the roofline fractions of the
 * advection kernels (which are bandwidth-bound, Sec. 3.1 and 4: advection
 * moves every field through memory once per step).  mode:
 *   MONC_CEIL_READ   read nbytes of src; dst receives
 *                    monc_ceiling_sink_bytes(blocks) bytes of folded words;
 *   MONC_CEIL_WRITE  write nbytes of a constant to dst (src unused);
 *   MONC_CEIL_COPY   copy nbytes from src to dst (must not overlap).
 * src, dst: device pointers, 16-byte aligned; nbytes a multiple of 16.
 * blocks: workgroups of 256 lanes (1 .. 65536); every lane moves 16 bytes
 * per access, stores are non-temporal.  Returns MONC_EINVAL on bad
 * arguments, MONC_EHIP if the launch fails.
 * ------------------------------------------------------------------------- */
enum { MONC_CEIL_READ = 0, MONC_CEIL_WRITE = 1, MONC_CEIL_COPY = 2 };
size_t monc_ceiling_sink_bytes(int blocks);
int monc_stream_ceiling(int mode, const void *src, void *dst, size_t nbytes, int blocks,
                        monc_stream_t stream);

/* Map a budgets array (HOST copy, after synchronising) to a status:
 * MONC_ENONFINITE if any non-finite value was written, MONC_ECFL if the
 * largest Courant number exceeds 1, else MONC_OK. */
int monc_budgets_check(const double *host_budgets);

const char *monc_strerror(int code);
const char *monc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MONC_ADV_H */
