// monc_internal.hpp -- launch interfaces shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <string>

#include "../../include/monc_adv.h"

namespace monc {

constexpr int MAXS = MONC_MAX_SCALARS;
constexpr int NB = MONC_NBUDGET;

enum Mode { TEND = 0, STEP = 1 };

// Everything one advection launch needs.  Pointers are device pointers; the
// storage type of in/out depends on the instantiation.
struct AdvArgs {
    const void* in[3 + MAXS];   // u, v, w, scalars
    void* out[3 + MAXS];        // tendencies (TEND) or new state (STEP)
    double phi0[MAXS];          // anomaly offsets of the scalars
    int nscal;
    int nx, ny, nz;
    double dx, dy, dt;
    const double* rdz;
    const double* rho;
    const double* rhon;
    double* partials;           // [nblocks][NB] budget partials, or null
    // other dynamics source terms fused into the step (monc_step_dyn):
    // Coriolis toward (ug, vg) and buoyancy of scalar 0 (theta)
    int dyn;
    double fcor, ug, vg, gth, th0;
    // scalars advected with the centred flux form (monc_step_pw_scalars)
    int spw;
    // repetitions of the PW arithmetic (the work-scaled experiment); 1 otherwise
    int work;
};

// Raise a kernel's dynamic-LDS limit once per device: `done` holds one bit
// per device index (a function-local static at the call site).  Threads that
// race here both set the same attribute, which is harmless.
inline hipError_t set_lds_limit_once(const void* kern, size_t lds,
                                     std::atomic<unsigned long long>* done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const unsigned long long bit = dev >= 0 && dev < 64 ? 1ull << dev : 0ull;
    if (bit && (done->load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && bit) done->fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

// Number of workgroups of the fused step launch (fixed for a grid so budget
// sums are repeatable), and the budget workspace it needs.
int step_blocks(int nx, int ny, int nz);
// exact number of workgroups (= budget partial rows) of a step launch
int step_grid(int nx, int ny, int nz, bool mixed);

// Launchers (return hipError_t of the launch).
hipError_t launch_halo(int elem_bytes, int nfields, void* const* fields, int nx,
                       int ny, int nz, hipStream_t s);
hipError_t launch_advect(int dtype, int mode, bool pw, bool tvd, bool mixed,
                         const AdvArgs& a, hipStream_t s);
hipError_t launch_budget_final(const double* partials, int nblocks,
                               double* budgets, hipStream_t s);
hipError_t launch_cast(int dtype, int nfields, const double* const* src,
                       void* const* dst, const double* offset, long n,
                       hipStream_t s);

// Streaming ceiling kernels (ceiling.hip).
size_t ceiling_sink_bytes(int blocks);
hipError_t launch_ceiling(int mode, const void* src, void* dst, size_t nbytes, int blocks,
                          hipStream_t s);

// Other dynamics source terms and the combined step (dynamics.hip).
struct DynArgs {
    const double *u, *v, *th;
    double *su, *sv, *sw;
    int nx, ny, nz;
    double fcor, ug, vg, gth, th0;
};
hipError_t launch_dyn_tend(const DynArgs& d, hipStream_t s);
hipError_t launch_combine(int nfields, const double* const* in, const double* const* ta,
                          const double* const* tb, double* const* out, int nx, int ny,
                          int nz, double dt, hipStream_t s);

// TVD advection of momentum (tvdmom.hip).  out_* receive the source terms,
// or the stepped velocities when `step` is set; cmax (device, may be null)
// receives the largest Courant number of the momentum faces.
struct TvdMomArgs {
    const double *u, *v, *w;
    double *out_u, *out_v, *out_w;
    int nx, ny, nz;
    double dt, rdt, rdx, rdy, cdx, cdy, rfx, rfy;
    const double *rdz, *rho, *rhon;
    double* cmax;
};
hipError_t launch_tvd_momentum(const TvdMomArgs& a, bool step, hipStream_t s);

// Learned correction (learned.hip).
hipError_t launch_restrict4(int nscal, const double* const* fine, double* const* coarse, int nx,
                            int ny, int nz, const double* rdz, const double* rho,
                            const double* rhon, double* rdz_c, double* rho_c, double* rhon_c,
                            hipStream_t s);
hipError_t launch_features(const double* const* state, int nx, int ny, int nz, const double* norm,
                           int orient, const int* cells, long ncells, uint16_t* X, hipStream_t s);
hipError_t launch_mlp_pack(const float* params, uint16_t* wpack, hipStream_t s);
hipError_t launch_mlp_infer(const double* const* state, int nx, int ny, int nz,
                           const double* norm, int orient, const float* params,
                           const uint16_t* wpack, float* Y, hipStream_t s);
hipError_t launch_mlp_forward(const uint16_t* X, int m, const float* params,
                              const uint16_t* wpack, float* Y, uint16_t* H1, uint16_t* H2,
                              float* Z1, float* Z2, hipStream_t s);
size_t mlp_backward_workspace(int m);
hipError_t launch_mlp_backward(const uint16_t* X, const uint16_t* H1, const uint16_t* H2,
                               const float* Z1, const float* Z2, const float* dY, int m,
                               const uint16_t* wpack, float* grad, void* ws, hipStream_t s);
size_t mlp_loss_workspace(int b);
hipError_t launch_mlp_loss(const float* Y4, int b, const int* cells, const double* const* c0,
                           const double* const* c1, const double* const* tend, int nx, int ny,
                           int nz, double dt, const double* scale, const double* rho,
                           const double* rhon, double inv_n, float* dY4, float* loss, void* ws,
                           hipStream_t s);
hipError_t launch_mlp_adam(float* params, float* m1, float* m2, const float* grad, int t,
                           double lr, double b1, double b2, double eps, uint16_t* wpack,
                           hipStream_t s);
size_t mlp_train_workspace(int b);
hipError_t launch_mlp_train(const double* const* c0, const double* const* c1,
                            const double* const* tend, int nx, int ny, int nz, const double* norm,
                            const int* cells, int b, double dt, const double* scale,
                            const double* rho, const double* rhon, double inv_n, float* params,
                            float* m1, float* m2, int t, double lr, double b1, double b2,
                            double eps, uint16_t* wpack, float* grad, float* loss, void* ws,
                            hipStream_t s);
hipError_t launch_pw_scaled(int dtype, const AdvArgs& a, hipStream_t s);
size_t correct_step_workspace_bytes(int nx, int ny, int nz);
hipError_t launch_correct_step(double* const* in, double* const* tend, const float* gx,
                               const float* gy, double* const* out, int nx, int ny, int nz,
                               double dx, double dy, const double* scale, const double* rdz,
                               const double* rho, const double* rhon, double dt, double growth,
                               int* flags, void* workspace, hipStream_t s);

// Ensemble plans (ensemble.hip).
struct EnsemblePlan;
int ensemble_create(const monc_member* members, int n, int nscal, const char* tune_cache,
                    int tune, EnsemblePlan** out, std::string* err);
int ensemble_step_eager(EnsemblePlan* P, hipStream_t s, std::string* err);
int ensemble_set_budgets(EnsemblePlan* P, double* budgets, int nslots, std::string* err);
int ensemble_budget_slots(const EnsemblePlan* P);  // -1: no budgets attached
int ensemble_run(EnsemblePlan* P, int nsteps, hipStream_t s, std::string* err);
void ensemble_info(const EnsemblePlan* P, int* ti, int* grid, int* nitems);
int ensemble_parity(const EnsemblePlan* P);
void ensemble_destroy(EnsemblePlan* P);

}  // namespace monc
