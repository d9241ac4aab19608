// abi.hip -- the extern "C" entry points of libmoncadv.so: argument checks
// (before any HIP call), launch sequencing on the caller's stream, and error
// reporting.  See include/monc_adv.h for the contract of every call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>

#include "monc_internal.hpp"

using namespace monc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return MONC_OK;
    return fail(MONC_EHIP, "%s: %s", where, hipGetErrorString(e));
}

int check_grid(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1) return fail(MONC_EINVAL, "nx, ny must be >= 1 (got %d, %d)", nx, ny);
    if (nz < 2 || nz > MONC_MAX_NZ)
        return fail(MONC_EINVAL, "nz must be in [2, %d] (got %d)", MONC_MAX_NZ, nz);
    const double n = (double)(nx + 4) * (ny + 4) * nz;
    if (n > 4.0e12) return fail(MONC_EINVAL, "grid too large");
    // the kernels address one x-plane of a field with 32-bit byte offsets
    if ((double)(ny + 4) * nz * sizeof(double) > 2147483647.0)
        return fail(MONC_EINVAL, "one x-plane of a field ((ny+4)*nz*8 = %.0f bytes) must stay "
                                 "below 2 GiB", (double)(ny + 4) * nz * sizeof(double));
    return MONC_OK;
}

int check_spacing(double dx, double dy) {
    if (!(dx > 0) || !(dy > 0) || !isfinite(dx) || !isfinite(dy))
        return fail(MONC_EINVAL, "dx, dy must be finite and > 0 (got %g, %g)", dx, dy);
    return MONC_OK;
}

int check_dt(double dt) {
    if (!(dt > 0) || !isfinite(dt)) return fail(MONC_EINVAL, "dt must be finite and > 0 (got %g)", dt);
    return MONC_OK;
}

int check_prof(const double* rdz, const double* rho, const double* rhon) {
    if (!rdz || !rho || !rhon) return fail(MONC_EINVAL, "profile pointer is NULL");
    return MONC_OK;
}

int check_nscal(int nscal) {
    if (nscal < 0 || nscal > MONC_MAX_SCALARS)
        return fail(MONC_EINVAL, "nscal must be in [0, %d] (got %d)", MONC_MAX_SCALARS, nscal);
    return MONC_OK;
}

template <typename P>
int check_ptrs(int n, P const* arr, const char* what) {
    if (!arr) return fail(MONC_EINVAL, "%s: pointer array is NULL", what);
    for (int f = 0; f < n; f++)
        if (!arr[f]) return fail(MONC_EINVAL, "%s[%d] is NULL", what, f);
    return MONC_OK;
}

// No output may alias an input.
int check_alias(int nin, const void* const* in, int nout, const void* const* out) {
    for (int a = 0; a < nout; a++) {
        for (int b = 0; b < nin; b++)
            if (out[a] == in[b]) return fail(MONC_EINVAL, "output %d aliases input %d", a, b);
        for (int b = 0; b < a; b++)
            if (out[a] == out[b]) return fail(MONC_EINVAL, "outputs %d and %d alias", a, b);
    }
    return MONC_OK;
}

#define TRY(x)                      \
    do {                            \
        int _rc = (x);              \
        if (_rc != MONC_OK) return _rc; \
    } while (0)

void fill_args(AdvArgs& a, int nx, int ny, int nz, double dx, double dy, double dt,
               const double* rdz, const double* rho, const double* rhon, int nscal) {
    for (int f = 0; f < 3 + MAXS; f++) {
        a.in[f] = nullptr;
        a.out[f] = nullptr;
    }
    for (int s = 0; s < MAXS; s++) a.phi0[s] = 0.0;
    a.nscal = nscal;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.dx = dx;
    a.dy = dy;
    a.dt = dt;
    a.rdz = rdz;
    a.rho = rho;
    a.rhon = rhon;
    a.partials = nullptr;
    a.dyn = 0;
    a.fcor = a.ug = a.vg = a.gth = a.th0 = 0.0;
    a.spw = 0;
    a.work = 1;
}

int do_halo(int bytes, int nfields, void* const* fields, int nx, int ny, int nz,
            monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    if (nfields < 1 || nfields > 3 + MONC_MAX_SCALARS)
        return fail(MONC_EINVAL, "nfields must be in [1, %d]", 3 + MONC_MAX_SCALARS);
    TRY(check_ptrs(nfields, fields, "fields"));
    return hip_status(launch_halo(bytes, nfields, fields, nx, ny, nz, (hipStream_t)stream),
                      "halo_fill");
}

int do_step(double* const* state_in, double* const* state_out, int nscal,
            const double* phi0, int nx, int ny, int nz, double dx, double dy,
            const double* rdz, const double* rho, const double* rhon, double dt,
            double* budgets, void* workspace, monc_stream_t stream, bool mixed) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, state_in, "state_in"));
    TRY(check_ptrs(nf, state_out, "state_out"));
    TRY(check_alias(nf, (const void* const*)state_in, nf, (const void* const*)state_out));
    if (budgets && !workspace)
        return fail(MONC_EINVAL, "budgets requested but workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
    for (int f = 0; f < nf; f++) {
        a.in[f] = state_in[f];
        a.out[f] = state_out[f];
    }
    if (phi0)
        for (int q = 0; q < nscal; q++) a.phi0[q] = phi0[q];
    a.partials = budgets ? (double*)workspace : nullptr;
    TRY(hip_status(launch_advect(MONC_F64, STEP, true, true, mixed, a, s), "step/advect"));
    if (budgets)
        TRY(hip_status(launch_budget_final((const double*)workspace,
                                           step_grid(nx, ny, nz, mixed), budgets, s),
                       "step/budgets"));
    return MONC_OK;
}

int check_dyn(const monc_dyn_params* p) {
    if (!p) return fail(MONC_EINVAL, "dynamics parameters are NULL");
    if (!isfinite(p->fcor) || !isfinite(p->ug) || !isfinite(p->vg) ||
        !isfinite(p->grav) || !isfinite(p->th0))
        return fail(MONC_EINVAL, "dynamics parameters must be finite");
    if (!(p->th0 > 0.0)) return fail(MONC_EINVAL, "th0 must be > 0 (got %g)", p->th0);
    return MONC_OK;
}

void set_dyn(AdvArgs& a, const monc_dyn_params* p) {
    a.dyn = 1;
    a.fcor = p->fcor;
    a.ug = p->ug;
    a.vg = p->vg;
    a.gth = p->grav / p->th0;
    a.th0 = p->th0;
}

DynArgs dyn_args(const double* u, const double* v, const double* th, double* su, double* sv,
                 double* sw, int nx, int ny, int nz, const monc_dyn_params* p) {
    DynArgs d;
    d.u = u;
    d.v = v;
    d.th = th;
    d.su = su;
    d.sv = sv;
    d.sw = sw;
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.fcor = p->fcor;
    d.ug = p->ug;
    d.vg = p->vg;
    d.gth = p->grav / p->th0;
    d.th0 = p->th0;
    return d;
}

}  // namespace

extern "C" {

int monc_halo_fill(int nfields, double* const* fields, int nx, int ny, int nz,
                   monc_stream_t stream) {
    return do_halo(8, nfields, (void* const*)fields, nx, ny, nz, stream);
}

int monc_halo_fill_f32(int nfields, float* const* fields, int nx, int ny, int nz,
                       monc_stream_t stream) {
    return do_halo(4, nfields, (void* const*)fields, nx, ny, nz, stream);
}

int monc_halo_fill_bf16(int nfields, uint16_t* const* fields, int nx, int ny, int nz,
                        monc_stream_t stream) {
    return do_halo(2, nfields, (void* const*)fields, nx, ny, nz, stream);
}

int monc_advect_pw(const double* u, const double* v, const double* w, double* su,
                   double* sv, double* sw, int nx, int ny, int nz, double dx, double dy,
                   const double* rdz, const double* rho, const double* rhon,
                   monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_prof(rdz, rho, rhon));
    const void* in[3] = {u, v, w};
    const void* out[3] = {su, sv, sw};
    TRY(check_ptrs(3, in, "velocity"));
    TRY(check_ptrs(3, out, "tendency"));
    TRY(check_alias(3, in, 3, out));
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, 1.0, rdz, rho, rhon, 0);
    for (int f = 0; f < 3; f++) {
        a.in[f] = in[f];
        a.out[f] = (void*)out[f];
    }
    return hip_status(launch_advect(MONC_F64, TEND, true, false, false, a, (hipStream_t)stream),
                      "advect_pw");
}

int monc_advect_pw_scaled(int dtype, const void* u, const void* v, const void* w, void* su,
                          void* sv, void* sw, int nx, int ny, int nz, double dx, double dy,
                          const double* rdz, const double* rho, const double* rhon, int work,
                          monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_prof(rdz, rho, rhon));
    if (dtype != MONC_F64 && dtype != MONC_F32)
        return fail(MONC_EINVAL, "dtype must be MONC_F64 or MONC_F32 (got %d)", dtype);
    if (work < 1 || work > MONC_MAX_WORK)
        return fail(MONC_EINVAL, "work must be in [1, %d] (got %d)", MONC_MAX_WORK, work);
    const void* in[3] = {u, v, w};
    const void* out[3] = {su, sv, sw};
    TRY(check_ptrs(3, in, "velocity"));
    TRY(check_ptrs(3, out, "tendency"));
    TRY(check_alias(3, in, 3, out));
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, 1.0, rdz, rho, rhon, 0);
    for (int f = 0; f < 3; f++) {
        a.in[f] = in[f];
        a.out[f] = const_cast<void*>(out[f]);
    }
    a.work = work;
    return hip_status(launch_pw_scaled(dtype, a, (hipStream_t)stream), "advect_pw_scaled");
}

int monc_advect_tvd(const double* u, const double* v, const double* w, int nscal,
                    const double* const* q, double* const* sq, int nx, int ny, int nz,
                    double dx, double dy, const double* rdz, const double* rho,
                    const double* rhon, double dt, monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    if (nscal < 1) return fail(MONC_EINVAL, "monc_advect_tvd needs nscal >= 1");
    const void* vel[3] = {u, v, w};
    TRY(check_ptrs(3, vel, "velocity"));
    TRY(check_ptrs(nscal, q, "q"));
    TRY(check_ptrs(nscal, sq, "sq"));
    const void* in[3 + MONC_MAX_SCALARS];
    for (int f = 0; f < 3; f++) in[f] = vel[f];
    for (int s = 0; s < nscal; s++) in[3 + s] = q[s];
    TRY(check_alias(3 + nscal, in, nscal, (const void* const*)sq));
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
    for (int f = 0; f < 3 + nscal; f++) a.in[f] = in[f];
    for (int s = 0; s < nscal; s++) a.out[3 + s] = sq[s];
    return hip_status(launch_advect(MONC_F64, TEND, false, true, false, a, (hipStream_t)stream),
                      "advect_tvd");
}

int monc_advect(int dtype, const void* const* in, void* const* out, int nscal,
                const double* phi0, int nx, int ny, int nz, double dx, double dy,
                const double* rdz, const double* rho, const double* rhon, double dt,
                monc_stream_t stream) {
    if (dtype != MONC_F64 && dtype != MONC_F32 && dtype != MONC_BF16)
        return fail(MONC_EINVAL, "unknown dtype %d", dtype);
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    if (nscal > 0) TRY(check_dt(dt));
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, in, "in"));
    TRY(check_ptrs(nf, out, "out"));
    TRY(check_alias(nf, in, nf, (const void* const*)out));
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, nscal > 0 ? dt : 1.0, rdz, rho, rhon, nscal);
    for (int f = 0; f < nf; f++) {
        a.in[f] = in[f];
        a.out[f] = out[f];
    }
    if (phi0)
        for (int s = 0; s < nscal; s++) a.phi0[s] = phi0[s];
    return hip_status(
        launch_advect(dtype, TEND, true, nscal > 0, false, a, (hipStream_t)stream), "advect");
}

// The PW or TVD part of monc_advect for one storage type (the precision
// form's separate entry points).
static int advect_part(int dtype, bool pw, const void* u, const void* v, const void* w,
                       int nscal, const void* const* q, void* const* sq, void* su, void* sv,
                       void* sw, const double* phi0, int nx, int ny, int nz, double dx,
                       double dy, const double* rdz, const double* rho, const double* rhon,
                       double dt, hipStream_t stream, const char* what) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_prof(rdz, rho, rhon));
    const void* vel[3] = {u, v, w};
    TRY(check_ptrs(3, vel, "velocity"));
    AdvArgs a;
    if (pw) {
        const void* out[3] = {su, sv, sw};
        TRY(check_ptrs(3, out, "tendency"));
        TRY(check_alias(3, vel, 3, out));
        fill_args(a, nx, ny, nz, dx, dy, 1.0, rdz, rho, rhon, 0);
        for (int f = 0; f < 3; f++) {
            a.in[f] = vel[f];
            a.out[f] = const_cast<void*>(out[f]);
        }
    } else {
        TRY(check_dt(dt));
        TRY(check_nscal(nscal));
        if (nscal < 1) return fail(MONC_EINVAL, "%s needs nscal >= 1", what);
        TRY(check_ptrs(nscal, q, "q"));
        TRY(check_ptrs(nscal, (const void* const*)sq, "sq"));
        const void* in[3 + MONC_MAX_SCALARS];
        for (int f = 0; f < 3; f++) in[f] = vel[f];
        for (int s = 0; s < nscal; s++) in[3 + s] = q[s];
        TRY(check_alias(3 + nscal, in, nscal, (const void* const*)sq));
        fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
        for (int f = 0; f < 3 + nscal; f++) a.in[f] = in[f];
        for (int s = 0; s < nscal; s++) a.out[3 + s] = sq[s];
        if (phi0)
            for (int s = 0; s < nscal; s++) a.phi0[s] = phi0[s];
    }
    return hip_status(launch_advect(dtype, TEND, pw, !pw, false, a, stream), what);
}

int monc_advect_pw_f32(const float* u, const float* v, const float* w, float* su, float* sv,
                       float* sw, int nx, int ny, int nz, double dx, double dy,
                       const double* rdz, const double* rho, const double* rhon,
                       monc_stream_t stream) {
    return advect_part(MONC_F32, true, u, v, w, 0, nullptr, nullptr, su, sv, sw, nullptr, nx,
                       ny, nz, dx, dy, rdz, rho, rhon, 0.0, (hipStream_t)stream,
                       "advect_pw_f32");
}

int monc_advect_pw_bf16(const uint16_t* u, const uint16_t* v, const uint16_t* w, float* su,
                        float* sv, float* sw, int nx, int ny, int nz, double dx, double dy,
                        const double* rdz, const double* rho, const double* rhon,
                        monc_stream_t stream) {
    return advect_part(MONC_BF16, true, u, v, w, 0, nullptr, nullptr, su, sv, sw, nullptr, nx,
                       ny, nz, dx, dy, rdz, rho, rhon, 0.0, (hipStream_t)stream,
                       "advect_pw_bf16");
}

int monc_advect_tvd_f32(const float* u, const float* v, const float* w, int nscal,
                        const float* const* q, float* const* sq, const double* phi0, int nx,
                        int ny, int nz, double dx, double dy, const double* rdz,
                        const double* rho, const double* rhon, double dt,
                        monc_stream_t stream) {
    return advect_part(MONC_F32, false, u, v, w, nscal, (const void* const*)q,
                       (void* const*)sq, nullptr, nullptr, nullptr, phi0, nx, ny, nz, dx, dy,
                       rdz, rho, rhon, dt, (hipStream_t)stream, "advect_tvd_f32");
}

int monc_advect_tvd_bf16(const uint16_t* u, const uint16_t* v, const uint16_t* w, int nscal,
                         const uint16_t* const* q, float* const* sq, const double* phi0,
                         int nx, int ny, int nz, double dx, double dy, const double* rdz,
                         const double* rho, const double* rhon, double dt,
                         monc_stream_t stream) {
    return advect_part(MONC_BF16, false, u, v, w, nscal, (const void* const*)q,
                       (void* const*)sq, nullptr, nullptr, nullptr, phi0, nx, ny, nz, dx, dy,
                       rdz, rho, rhon, dt, (hipStream_t)stream, "advect_tvd_bf16");
}

size_t monc_step_workspace_bytes(int nx, int ny, int nz, int nscal) {
    (void)nscal;
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    return (size_t)step_blocks(nx, ny, nz) * NB * sizeof(double);
}

int monc_step(double* const* state_in, double* const* state_out, int nscal, int nx,
              int ny, int nz, double dx, double dy, const double* rdz, const double* rho,
              const double* rhon, double dt, double* budgets, void* workspace,
              monc_stream_t stream) {
    return do_step(state_in, state_out, nscal, nullptr, nx, ny, nz, dx, dy, rdz, rho, rhon,
                   dt, budgets, workspace, stream, false);
}

// ---------------------------------------------------------------------------
// The step with budgets for callers that cannot allocate: the budget partial
// rows live in a file-scope device array.  Its host-side name is only a
// stand-in; the device address is looked up once per device (with that
// device current) and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[(size_t)MONC_STATIC_MAX_ROWS * NB];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[MONC_STATIC_MAX_DEVICES] = {};

int scratch_on_current_device(double** out) {
    int dev = -1;
    TRY(hip_status(hipGetDevice(&dev), "step_static/hipGetDevice"));
    if (dev < 0 || dev >= MONC_STATIC_MAX_DEVICES)
        return fail(MONC_EUNSUPPORTED, "device %d: the static scratch serves devices 0..%d", dev,
                    MONC_STATIC_MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                       "step_static/hipGetSymbolAddress"));
        if (!p) return fail(MONC_EHIP, "step_static: no device address for the scratch array");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return MONC_OK;
}

}  // namespace

int monc_step_static(double* const* state_in, double* const* state_out, int nscal, int nx,
                     int ny, int nz, double dx, double dy, const double* rdz, const double* rho,
                     const double* rhon, double dt, double* budgets, monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, state_in, "state_in"));
    TRY(check_ptrs(nf, state_out, "state_out"));
    TRY(check_alias(nf, (const void* const*)state_in, nf, (const void* const*)state_out));
    if (!budgets) return fail(MONC_EINVAL, "budgets is NULL (monc_step_static computes them)");
    const int rows = step_grid(nx, ny, nz, false);
    if (rows > MONC_STATIC_MAX_ROWS)
        return fail(MONC_EINVAL,
                    "grid %d x %d x %d needs %d budget rows; the static scratch holds %d "
                    "(use monc_step with a workspace)", nx, ny, nz, rows, MONC_STATIC_MAX_ROWS);
    double* ws = nullptr;
    TRY(scratch_on_current_device(&ws));
    return do_step(state_in, state_out, nscal, nullptr, nx, ny, nz, dx, dy, rdz, rho, rhon, dt,
                   budgets, ws, stream, false);
}

int monc_step_mixed(double* const* state_in, double* const* state_out, int nscal,
                    const double* phi0, int nx, int ny, int nz, double dx, double dy,
                    const double* rdz, const double* rho, const double* rhon, double dt,
                    double* budgets, void* workspace, monc_stream_t stream) {
    return do_step(state_in, state_out, nscal, phi0, nx, ny, nz, dx, dy, rdz, rho, rhon,
                   dt, budgets, workspace, stream, true);
}

int monc_dyn_tend(const double* u, const double* v, const double* theta, double* su,
                  double* sv, double* sw, int nx, int ny, int nz, const monc_dyn_params* p,
                  monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_dyn(p));
    const void* in[3] = {u, v, theta};
    const void* out[3] = {su, sv, sw};
    TRY(check_ptrs(3, in, "inputs"));
    TRY(check_ptrs(3, out, "outputs"));
    TRY(check_alias(3, in, 3, out));
    return hip_status(
        launch_dyn_tend(dyn_args(u, v, theta, su, sv, sw, nx, ny, nz, p), (hipStream_t)stream),
        "dyn_tend");
}

int monc_combine_step(int nfields, const double* const* in, const double* const* ta,
                      const double* const* tb, double* const* out, int nx, int ny, int nz,
                      double dt, monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_dt(dt));
    if (nfields < 1 || nfields > 3 + MONC_MAX_SCALARS)
        return fail(MONC_EINVAL, "nfields must be in [1, %d]", 3 + MONC_MAX_SCALARS);
    TRY(check_ptrs(nfields, in, "in"));
    TRY(check_ptrs(nfields, ta, "ta"));
    TRY(check_ptrs(nfields, out, "out"));
    TRY(check_alias(nfields, (const void* const*)in, nfields, (const void* const*)out));
    TRY(check_alias(nfields, (const void* const*)ta, nfields, (const void* const*)out));
    if (tb) {
        for (int f = 0; f < nfields; f++)
            for (int g = 0; g < nfields; g++)
                if (tb[f] && tb[f] == out[g])
                    return fail(MONC_EINVAL, "output %d aliases tb[%d]", g, f);
    }
    return hip_status(launch_combine(nfields, in, ta, tb, out, nx, ny, nz, dt,
                                     (hipStream_t)stream),
                      "combine_step");
}

int monc_hybrid_step(double* const* state_in, double* const* state_out, double* const* tend,
                     double* const* dyn_tend, int nscal, int nx, int ny, int nz, double dx,
                     double dy, const double* rdz, const double* rho, const double* rhon,
                     double dt, const monc_dyn_params* p, monc_stream_t stream,
                     monc_stream_t side_stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    TRY(check_dyn(p));
    if (nscal < 1) return fail(MONC_EINVAL, "the hybrid step needs theta (nscal >= 1)");
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, state_in, "state_in"));
    TRY(check_ptrs(nf, state_out, "state_out"));
    TRY(check_ptrs(nf, tend, "tend"));
    TRY(check_ptrs(3, dyn_tend, "dyn_tend"));
    {
        // no buffer written here may alias any other buffer of the call
        const void* all[4 * (3 + MAXS)];
        int n = 0;
        for (int f = 0; f < nf; f++) all[n++] = state_in[f];
        const int nin = n;
        for (int f = 0; f < nf; f++) all[n++] = state_out[f];
        for (int f = 0; f < nf; f++) all[n++] = tend[f];
        for (int f = 0; f < 3; f++) all[n++] = dyn_tend[f];
        TRY(check_alias(nin, all, n - nin, all + nin));
    }
    hipStream_t s = (hipStream_t)stream, side = (hipStream_t)side_stream;
    const bool two = side != s;
    hipEvent_t start = nullptr, done = nullptr;
    if (two) {
        TRY(hip_status(hipEventCreateWithFlags(&start, hipEventDisableTiming), "event"));
        TRY(hip_status(hipEventCreateWithFlags(&done, hipEventDisableTiming), "event"));
        TRY(hip_status(hipEventRecord(start, s), "event record"));
        TRY(hip_status(hipStreamWaitEvent(side, start, 0), "stream wait"));
    }
    // the other components on the side stream
    TRY(hip_status(launch_dyn_tend(dyn_args(state_in[0], state_in[1], state_in[3], dyn_tend[0],
                                            dyn_tend[1], dyn_tend[2], nx, ny, nz, p),
                                   two ? side : s),
                   "hybrid/dyn_tend"));
    if (two) TRY(hip_status(hipEventRecord(done, side), "event record"));
    // the advection source terms on the main stream
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
    for (int f = 0; f < nf; f++) {
        a.in[f] = state_in[f];
        a.out[f] = tend[f];
    }
    TRY(hip_status(launch_advect(MONC_F64, TEND, true, true, false, a, s), "hybrid/advect"));
    if (two) {
        TRY(hip_status(hipStreamWaitEvent(s, done, 0), "stream wait"));
        // released by the runtime once the recorded work has completed
        (void)hipEventDestroy(start);
        (void)hipEventDestroy(done);
    }
    const double* tb[3 + MAXS];
    for (int f = 0; f < nf; f++) tb[f] = f < 3 ? dyn_tend[f] : nullptr;
    return hip_status(launch_combine(nf, (const double* const*)state_in,
                                     (const double* const*)tend, tb, state_out, nx, ny, nz,
                                     dt, s),
                      "hybrid/combine");
}

int monc_step_dyn(double* const* state_in, double* const* state_out, int nscal, int nx,
                  int ny, int nz, double dx, double dy, const double* rdz, const double* rho,
                  const double* rhon, double dt, const monc_dyn_params* p,
                  monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    TRY(check_dyn(p));
    if (nscal < 1) return fail(MONC_EINVAL, "the fused dynamics step needs theta (nscal >= 1)");
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, state_in, "state_in"));
    TRY(check_ptrs(nf, state_out, "state_out"));
    TRY(check_alias(nf, (const void* const*)state_in, nf, (const void* const*)state_out));
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
    for (int f = 0; f < nf; f++) {
        a.in[f] = state_in[f];
        a.out[f] = state_out[f];
    }
    set_dyn(a, p);
    return hip_status(launch_advect(MONC_F64, STEP, true, true, false, a, (hipStream_t)stream),
                      "step_dyn");
}

int monc_step_pw_scalars(double* const* state_in, double* const* state_out, int nscal,
                         int nx, int ny, int nz, double dx, double dy, const double* rdz,
                         const double* rho, const double* rhon, double dt,
                         monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, state_in, "state_in"));
    TRY(check_ptrs(nf, state_out, "state_out"));
    TRY(check_alias(nf, (const void* const*)state_in, nf, (const void* const*)state_out));
    AdvArgs a;
    fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
    for (int f = 0; f < nf; f++) {
        a.in[f] = state_in[f];
        a.out[f] = state_out[f];
    }
    a.spw = 1;
    return hip_status(launch_advect(MONC_F64, STEP, true, nscal > 0, false, a,
                                    (hipStream_t)stream),
                      "step_pw_scalars");
}

static TvdMomArgs tvdmom_args(const double* u, const double* v, const double* w, double* ou,
                       double* ov, double* ow, int nx, int ny, int nz, double dx, double dy,
                       const double* rdz, const double* rho, const double* rhon, double dt,
                       double* cmax) {
    TvdMomArgs t;
    t.u = u;
    t.v = v;
    t.w = w;
    t.out_u = ou;
    t.out_v = ov;
    t.out_w = ow;
    t.nx = nx;
    t.ny = ny;
    t.nz = nz;
    t.dt = dt;
    t.rdt = 1.0 / dt;
    t.rdx = 1.0 / dx;
    t.rdy = 1.0 / dy;
    t.cdx = dt / dx;
    t.cdy = dt / dy;
    t.rfx = dx / dt;
    t.rfy = dy / dt;
    t.rdz = rdz;
    t.rho = rho;
    t.rhon = rhon;
    t.cmax = cmax;
    return t;
}

int monc_advect_tvd_momentum(const double* u, const double* v, const double* w, double* su,
                             double* sv, double* sw, int nx, int ny, int nz, double dx,
                             double dy, const double* rdz, const double* rho,
                             const double* rhon, double dt, double* cmax,
                             monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    const void* in[3] = {u, v, w};
    const void* out[4] = {su, sv, sw, cmax};
    TRY(check_ptrs(3, in, "velocity"));
    TRY(check_ptrs(3, out, "source term"));
    TRY(check_alias(3, in, cmax ? 4 : 3, out));
    const TvdMomArgs t = tvdmom_args(u, v, w, su, sv, sw, nx, ny, nz, dx, dy, rdz, rho, rhon,
                                     dt, cmax);
    return hip_status(launch_tvd_momentum(t, false, (hipStream_t)stream), "advect_tvd_momentum");
}

int monc_step_tvd_momentum(double* const* state_in, double* const* state_out, int nscal,
                           int nx, int ny, int nz, double dx, double dy, const double* rdz,
                           const double* rho, const double* rhon, double dt, double* cmax,
                           monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_prof(rdz, rho, rhon));
    TRY(check_nscal(nscal));
    const int nf = 3 + nscal;
    TRY(check_ptrs(nf, state_in, "state_in"));
    TRY(check_ptrs(nf, state_out, "state_out"));
    const void* outs[3 + MONC_MAX_SCALARS + 1];
    for (int f = 0; f < nf; f++) outs[f] = state_out[f];
    outs[nf] = cmax;
    TRY(check_alias(nf, (const void* const*)state_in, cmax ? nf + 1 : nf, outs));
    const TvdMomArgs t = tvdmom_args(state_in[0], state_in[1], state_in[2], state_out[0],
                                     state_out[1], state_out[2], nx, ny, nz, dx, dy, rdz, rho,
                                     rhon, dt, cmax);
    hipError_t e = launch_tvd_momentum(t, true, (hipStream_t)stream);
    if (e == hipSuccess && nscal > 0) {
        AdvArgs a;
        fill_args(a, nx, ny, nz, dx, dy, dt, rdz, rho, rhon, nscal);
        for (int f = 0; f < nf; f++) {
            a.in[f] = state_in[f];
            a.out[f] = state_out[f];
        }
        e = launch_advect(MONC_F64, STEP, false, true, false, a, (hipStream_t)stream);
    }
    return hip_status(e, "step_tvd_momentum");
}

int monc_cast_working(int dtype, int nfields, const double* const* src, void* const* work,
                      const double* offset, int nx, int ny, int nz, monc_stream_t stream) {
    if (dtype != MONC_F32 && dtype != MONC_BF16)
        return fail(MONC_EINVAL, "cast dtype must be MONC_F32 or MONC_BF16");
    TRY(check_grid(nx, ny, nz));
    if (nfields < 1 || nfields > 3 + MONC_MAX_SCALARS)
        return fail(MONC_EINVAL, "nfields must be in [1, %d]", 3 + MONC_MAX_SCALARS);
    TRY(check_ptrs(nfields, src, "src"));
    TRY(check_ptrs(nfields, work, "work"));
    for (int f = 0; f < nfields; f++)
        if ((uintptr_t)src[f] % 16 != 0 || (uintptr_t)work[f] % 16 != 0)
            return fail(MONC_EINVAL, "field %d: src and work must be 16-byte aligned", f);
    const long n = (long)(nx + 4) * (ny + 4) * nz;
    return hip_status(launch_cast(dtype, nfields, src, work, offset, n, (hipStream_t)stream),
                      "cast_working");
}

int monc_ensemble_create(const monc_member* members, int nmembers, int nscal,
                         const char* tune_cache, int tune, monc_ensemble** plan) {
    if (!plan) return fail(MONC_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!members || nmembers < 1) return fail(MONC_EINVAL, "need at least one member");
    TRY(check_nscal(nscal));
    if (nscal > 3)
        return fail(MONC_EUNSUPPORTED, "ensembles advect at most 3 scalars (got %d)", nscal);
    for (int m = 0; m < nmembers; m++) {
        const monc_member& M = members[m];
        int rc = check_grid(M.nx, M.ny, M.nz);
        if (rc == MONC_OK) rc = check_spacing(M.dx, M.dy);
        if (rc == MONC_OK) rc = check_dt(M.dt);
        if (rc == MONC_OK) rc = check_prof(M.rdz, M.rho, M.rhon);
        for (int p = 0; p < 2 && rc == MONC_OK; p++)
            for (int f = 0; f < 3 + nscal && rc == MONC_OK; f++)
                if (!M.state[p][f]) rc = fail(MONC_EINVAL, "member %d: state[%d][%d] is NULL", m, p, f);
        if (rc == MONC_OK)
            rc = check_alias(3 + nscal, (const void* const*)M.state[0], 3 + nscal,
                             (const void* const*)M.state[1]);
        if (rc != MONC_OK) {
            std::string d = g_last_error;
            return fail(rc, "member %d: %s", m, d.c_str());
        }
    }
    std::string err;
    EnsemblePlan* P = nullptr;
    const int rc = ensemble_create(members, nmembers, nscal, tune_cache, tune, &P, &err);
    if (rc != MONC_OK) return fail(rc, "ensemble_create: %s", err.c_str());
    *plan = reinterpret_cast<monc_ensemble*>(P);
    return MONC_OK;
}

int monc_ensemble_set_budgets(monc_ensemble* plan, double* budgets, int nslots) {
    if (!plan) return fail(MONC_EINVAL, "plan is NULL");
    if (budgets && nslots < 1) return fail(MONC_EINVAL, "nslots must be >= 1 (got %d)", nslots);
    std::string err;
    const int rc = ensemble_set_budgets(reinterpret_cast<EnsemblePlan*>(plan), budgets,
                                        budgets ? nslots : 0, &err);
    if (rc != MONC_OK) return fail(rc, "ensemble_set_budgets: %s", err.c_str());
    return MONC_OK;
}

int monc_ensemble_run(monc_ensemble* plan, int nsteps, monc_stream_t stream) {
    if (!plan) return fail(MONC_EINVAL, "plan is NULL");
    if (nsteps < 1) return fail(MONC_EINVAL, "nsteps must be >= 1");
    const int slots = ensemble_budget_slots(reinterpret_cast<EnsemblePlan*>(plan));
    if (slots >= 0 && nsteps > slots)
        return fail(MONC_EINVAL, "nsteps %d exceeds the %d attached budget slots", nsteps, slots);
    std::string err;
    const int rc = ensemble_run(reinterpret_cast<EnsemblePlan*>(plan), nsteps,
                                (hipStream_t)stream, &err);
    if (rc != MONC_OK) return fail(rc, "ensemble_run: %s", err.c_str());
    return MONC_OK;
}

int monc_ensemble_step(monc_ensemble* plan, monc_stream_t stream) {
    if (!plan) return fail(MONC_EINVAL, "plan is NULL");
    std::string err;
    const int rc =
        ensemble_step_eager(reinterpret_cast<EnsemblePlan*>(plan), (hipStream_t)stream, &err);
    if (rc != MONC_OK) return fail(rc, "ensemble_step: %s", err.c_str());
    return MONC_OK;
}

int monc_ensemble_parity(const monc_ensemble* plan) {
    if (!plan) return fail(MONC_EINVAL, "plan is NULL");
    return ensemble_parity(reinterpret_cast<const EnsemblePlan*>(plan));
}

int monc_ensemble_info(const monc_ensemble* plan, int* ti, int* grid, int* nitems) {
    if (!plan) return fail(MONC_EINVAL, "plan is NULL");
    ensemble_info(reinterpret_cast<const EnsemblePlan*>(plan), ti, grid, nitems);
    return MONC_OK;
}

int monc_ensemble_destroy(monc_ensemble* plan) {
    if (!plan) return MONC_OK;
    ensemble_destroy(reinterpret_cast<EnsemblePlan*>(plan));
    return MONC_OK;
}

int monc_restrict4(int nscal, const double* const* fine, double* const* coarse, int nx, int ny,
                   int nz, const double* rdz, const double* rho, const double* rhon,
                   double* rdz_c, double* rho_c, double* rhon_c, monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_nscal(nscal));
    if (nx % 4 || ny % 4 || nz % 4 || nz < 8)
        return fail(MONC_EINVAL, "restriction needs nx, ny, nz multiples of 4 (nz >= 8)");
    TRY(check_prof(rdz, rho, rhon));
    if (!rdz_c || !rho_c || !rhon_c) return fail(MONC_EINVAL, "coarse profile pointer is NULL");
    TRY(check_ptrs(3 + nscal, fine, "fine"));
    TRY(check_ptrs(3 + nscal, coarse, "coarse"));
    TRY(check_alias(3 + nscal, (const void* const*)fine, 3 + nscal, (const void* const*)coarse));
    return hip_status(launch_restrict4(nscal, fine, coarse, nx, ny, nz, rdz, rho, rhon, rdz_c,
                                       rho_c, rhon_c, (hipStream_t)stream),
                      "restrict4");
}

int monc_mlp_features(const double* const* state, int nx, int ny, int nz, const double* norm,
                      int orient, const int* cells, int ncells, uint16_t* X,
                      monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_ptrs(4, state, "state"));
    if (!norm || !X) return fail(MONC_EINVAL, "norm or X is NULL");
    if (orient != 0 && orient != 1) return fail(MONC_EINVAL, "orient must be 0 or 1");
    if (ncells < 1) return fail(MONC_EINVAL, "ncells must be >= 1");
    if (!cells && (long)ncells != (long)nx * ny * nz)
        return fail(MONC_EINVAL, "without a cell list ncells must be nx*ny*nz");
    for (int f = 0; f < 4; f++)
        if (!(norm[2 * f + 1] > 0)) return fail(MONC_EINVAL, "norm std %d must be > 0", f);
    if ((uintptr_t)X & 15) return fail(MONC_EINVAL, "X must be 16-byte aligned");
    return hip_status(launch_features(state, nx, ny, nz, norm, orient, cells, ncells, X,
                                      (hipStream_t)stream),
                      "mlp_features");
}

int monc_mlp_pack(const float* params, uint16_t* wpack, monc_stream_t stream) {
    if (!params || !wpack) return fail(MONC_EINVAL, "NULL pointer");
    return hip_status(launch_mlp_pack(params, wpack, (hipStream_t)stream), "mlp_pack");
}

int monc_mlp_infer(const double* const* state, int nx, int ny, int nz, const double* norm,
                   int orient, const float* params, const uint16_t* wpack, float* Y,
                   monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_ptrs(4, state, "state"));
    if (!norm || !params || !wpack || !Y) return fail(MONC_EINVAL, "NULL pointer");
    if (orient < 0 || orient > 2) return fail(MONC_EINVAL, "orient must be 0, 1 or 2");
    for (int f = 0; f < 4; f++)
        if (!(norm[2 * f + 1] > 0)) return fail(MONC_EINVAL, "norm std %d must be > 0", f);
    if ((uintptr_t)wpack & 15) return fail(MONC_EINVAL, "wpack must be 16-byte aligned");
    return hip_status(launch_mlp_infer(state, nx, ny, nz, norm, orient, params, wpack, Y,
                                       (hipStream_t)stream),
                      "mlp_infer");
}

int monc_mlp_forward(const uint16_t* X, int m, const float* params, const uint16_t* wpack,
                     float* Y, uint16_t* H1, uint16_t* H2, float* Z1, float* Z2,
                     monc_stream_t stream) {
    if (!X || !params || !wpack || !Y) return fail(MONC_EINVAL, "NULL pointer");
    if (m < 1) return fail(MONC_EINVAL, "m must be >= 1");
    if (((uintptr_t)X | (uintptr_t)wpack) & 15) return fail(MONC_EINVAL, "X, wpack must be 16-byte aligned");
    return hip_status(launch_mlp_forward(X, m, params, wpack, Y, H1, H2, Z1, Z2,
                                         (hipStream_t)stream),
                      "mlp_forward");
}

size_t monc_mlp_backward_workspace_bytes(int m) { return m < 1 ? 0 : mlp_backward_workspace(m); }

int monc_mlp_backward(const uint16_t* X, const uint16_t* H1, const uint16_t* H2, const float* Z1,
                      const float* Z2, const float* dY, int m, const uint16_t* wpack,
                      float* grad, void* workspace, monc_stream_t stream) {
    if (!X || !H1 || !H2 || !Z1 || !Z2 || !dY || !wpack || !grad || !workspace)
        return fail(MONC_EINVAL, "NULL pointer");
    if (m < 1) return fail(MONC_EINVAL, "m must be >= 1");
    if (((uintptr_t)X | (uintptr_t)wpack) & 15) return fail(MONC_EINVAL, "X, wpack must be 16-byte aligned");
    return hip_status(launch_mlp_backward(X, H1, H2, Z1, Z2, dY, m, wpack, grad, workspace,
                                          (hipStream_t)stream),
                      "mlp_backward");
}

size_t monc_mlp_loss_workspace_bytes(int b) { return b < 1 ? 0 : mlp_loss_workspace(b); }

int monc_mlp_loss(const float* Y4, int b, const int* cells, const double* const* c0,
                  const double* const* c1, const double* const* tend, int nx, int ny, int nz,
                  double dt, const double* scale, const double* rho, const double* rhon,
                  double inv_count, float* dY4, float* loss, void* workspace,
                  monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_dt(dt));
    if (!Y4 || !cells || !dY4 || !loss || !workspace || !scale || !rho || !rhon)
        return fail(MONC_EINVAL, "NULL pointer");
    TRY(check_ptrs(4, c0, "c0"));
    TRY(check_ptrs(4, c1, "c1"));
    TRY(check_ptrs(4, tend, "tend"));
    if (b < 1) return fail(MONC_EINVAL, "b must be >= 1");
    for (int q = 0; q < 4; q++)
        if (!(scale[q] > 0)) return fail(MONC_EINVAL, "scale %d must be > 0", q);
    return hip_status(launch_mlp_loss(Y4, b, cells, c0, c1, tend, nx, ny, nz, dt, scale, rho,
                                      rhon, inv_count, dY4, loss, workspace, (hipStream_t)stream),
                      "mlp_loss");
}

int monc_mlp_adam(float* params, float* m1, float* m2, const float* grad, int t, double lr,
                  double beta1, double beta2, double eps, uint16_t* wpack, monc_stream_t stream) {
    if (!params || !m1 || !m2 || !grad || !wpack) return fail(MONC_EINVAL, "NULL pointer");
    if (t < 1) return fail(MONC_EINVAL, "t must be >= 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(MONC_EINVAL, "bad Adam hyper-parameters");
    return hip_status(launch_mlp_adam(params, m1, m2, grad, t, lr, beta1, beta2, eps, wpack,
                                      (hipStream_t)stream),
                      "mlp_adam");
}

size_t monc_mlp_train_workspace_bytes(int b) { return b < 1 ? 0 : mlp_train_workspace(b); }

int monc_mlp_train_step(const double* const* c0, const double* const* c1,
                        const double* const* tend, int nx, int ny, int nz, const double* norm,
                        const int* cells, int b, double dt, const double* scale, const double* rho,
                        const double* rhon, double inv_count, float* params, float* m1, float* m2,
                        int t, double lr, double beta1, double beta2, double eps, uint16_t* wpack,
                        float* grad, float* loss, void* workspace, monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_dt(dt));
    TRY(check_ptrs(4, c0, "c0"));
    TRY(check_ptrs(4, c1, "c1"));
    TRY(check_ptrs(4, tend, "tend"));
    if (!norm || !cells || !scale || !rho || !rhon || !params || !m1 || !m2 || !wpack || !grad ||
        !loss || !workspace)
        return fail(MONC_EINVAL, "NULL pointer");
    if (b < 1) return fail(MONC_EINVAL, "b must be >= 1");
    if (t < 1) return fail(MONC_EINVAL, "t must be >= 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(MONC_EINVAL, "bad Adam hyper-parameters");
    for (int q = 0; q < 4; q++) {
        if (!(scale[q] > 0)) return fail(MONC_EINVAL, "scale %d must be > 0", q);
        if (!(norm[2 * q + 1] > 0)) return fail(MONC_EINVAL, "norm std %d must be > 0", q);
    }
    if ((uintptr_t)wpack & 15) return fail(MONC_EINVAL, "wpack must be 16-byte aligned");
    return hip_status(launch_mlp_train(c0, c1, tend, nx, ny, nz, norm, cells, b, dt, scale, rho,
                                       rhon, inv_count, params, m1, m2, t, lr, beta1, beta2, eps,
                                       wpack, grad, loss, workspace, (hipStream_t)stream),
                      "mlp_train_step");
}

size_t monc_correct_step_workspace_bytes(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    return correct_step_workspace_bytes(nx, ny, nz);
}

int monc_correct_step(double* const* state_in, double* const* tend, const float* gx,
                      const float* gy, double* const* state_out, int nx, int ny, int nz,
                      double dx, double dy, const double* scale, const double* rdz,
                      const double* rho, const double* rhon, double dt, double growth,
                      int* flags, void* workspace, monc_stream_t stream) {
    TRY(check_grid(nx, ny, nz));
    TRY(check_spacing(dx, dy));
    TRY(check_dt(dt));
    TRY(check_ptrs(4, state_in, "state_in"));
    TRY(check_ptrs(4, tend, "tend"));
    TRY(check_ptrs(4, state_out, "state_out"));
    TRY(check_alias(4, (const void* const*)state_in, 4, (const void* const*)state_out));
    if (!gx || !gy || !scale || !rdz || !rho || !rhon || !flags || !workspace)
        return fail(MONC_EINVAL, "NULL pointer");
    if (!(growth > 0.0)) return fail(MONC_EINVAL, "growth must be > 0 (got %g)", growth);
    for (int q = 0; q < 4; q++)
        if (!isfinite(scale[q])) return fail(MONC_EINVAL, "scale[%d] is not finite", q);
    if (((uintptr_t)gx | (uintptr_t)gy) & 15)
        return fail(MONC_EINVAL, "gx, gy must be 16-byte aligned (one row of 4 floats per load)");
    return hip_status(launch_correct_step(state_in, tend, gx, gy, state_out, nx, ny, nz, dx, dy,
                                          scale, rdz, rho, rhon, dt, growth, flags, workspace,
                                          (hipStream_t)stream),
                      "correct_step");
}

size_t monc_ceiling_sink_bytes(int blocks) {
    return blocks < 1 ? 0 : ceiling_sink_bytes(blocks);
}

int monc_stream_ceiling(int mode, const void* src, void* dst, size_t nbytes, int blocks,
                        monc_stream_t stream) {
    if (mode != MONC_CEIL_READ && mode != MONC_CEIL_WRITE && mode != MONC_CEIL_COPY)
        return fail(MONC_EINVAL, "mode must be MONC_CEIL_READ, _WRITE or _COPY (got %d)", mode);
    if (blocks < 1 || blocks > 65536)
        return fail(MONC_EINVAL, "blocks must be in [1, 65536] (got %d)", blocks);
    if (nbytes == 0 || nbytes % 16 != 0)
        return fail(MONC_EINVAL, "nbytes must be a positive multiple of 16");
    if (!dst || (mode != MONC_CEIL_WRITE && !src))
        return fail(MONC_EINVAL, "NULL buffer");
    if (((uintptr_t)dst | (mode == MONC_CEIL_WRITE ? 0 : (uintptr_t)src)) % 16 != 0)
        return fail(MONC_EINVAL, "buffers must be 16-byte aligned");
    if (mode == MONC_CEIL_COPY) {
        const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
        if (a < b + nbytes && b < a + nbytes) return fail(MONC_EINVAL, "src and dst overlap");
    }
    return hip_status(launch_ceiling(mode, src, dst, nbytes, blocks, (hipStream_t)stream),
                      "stream_ceiling");
}

int monc_budgets_check(const double* b) {
    if (!b) return fail(MONC_EINVAL, "budgets is NULL");
    if (b[MONC_B_NONFINITE] > 0)
        return fail(MONC_ENONFINITE, "%.0f non-finite values written", b[MONC_B_NONFINITE]);
    if (!(b[MONC_B_COURANT] <= 1.0))
        return fail(MONC_ECFL, "largest Courant number %g exceeds 1", b[MONC_B_COURANT]);
    return MONC_OK;
}

const char* monc_strerror(int code) {
    switch (code) {
        case MONC_OK: return "ok";
        case MONC_EINVAL: return "invalid argument";
        case MONC_EHIP: return "HIP runtime error";
        case MONC_ECFL: return "Courant number above 1";
        case MONC_ENONFINITE: return "non-finite value produced";
        case MONC_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown error";
}

const char* monc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
