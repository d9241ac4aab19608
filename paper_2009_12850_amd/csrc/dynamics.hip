// dynamics.hip -- the other source terms of the dynamics group and the
// combined step.
//
// Brown et al. (Sec. 3 and the hybrid-dynamics figure) run advection on the
// GPU while the CPU computes the other components of the dynamics group; the
// CPU then waits for the advection source terms, adds them to its own and
// steps the fields.  On one MI355X the same structure is two streams: the
// other components (here Coriolis toward a geostrophic wind and the buoyancy
// of theta) run on a side stream while the advection source terms are
// computed on the main stream, and one combine pass adds all source terms and
// steps the fields.  The fused alternative (the same terms added inside the
// advection march, monc_step_dyn) is in march.hpp.
//
// Both kernels take one thread per grid point: a wave covers 64 levels of one
// column, a workgroup 4 columns of one x-plane; periodic neighbours are read
// at wrapped indices (halos are not read) and nothing is written outside the
// interior.
#include "monc_internal.hpp"
#include "monc_scheme.hpp"

namespace monc {

namespace {

constexpr int DY_COLS = 4;

__global__ void __launch_bounds__(64 * DY_COLS) dyn_tend_kernel(DynArgs d) {
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int nchunk = (nz + 63) / 64;
    const int k = 64 * (int)(blockIdx.x % nchunk) + (int)threadIdx.x;
    const int j = (int)(blockIdx.x / nchunk) * DY_COLS + (int)threadIdx.y;
    const int i = blockIdx.y;
    if (k >= nz || j >= ny) return;
    const long sx = (long)(ny + 4) * nz;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
    auto at = [&](int ii, int jj, int kk) -> long {
        return (long)(ii + 2) * sx + (long)(jj + 2) * nz + kk;
    };
    const long c = at(i, j, k);
    d.su[c] = coriolis_u(d.fcor, d.vg, d.v[c], d.v[at(ip, j, k)], d.v[at(i, jm, k)],
                         d.v[at(ip, jm, k)]);
    d.sv[c] = coriolis_v(d.fcor, d.ug, d.u[c], d.u[at(im, j, k)], d.u[at(i, jp, k)],
                         d.u[at(im, jp, k)]);
    d.sw[c] = k < nz - 1 ? buoyancy_w(d.gth, d.th0, d.th[c], d.th[c + 1]) : 0.0;
}

struct CombineArgs {
    const double* in[3 + MAXS];
    const double* ta[3 + MAXS];
    const double* tb[3 + MAXS];  // null: no second source term for that field
    double* out[3 + MAXS];
    int nfields, nx, ny, nz;
    double dt;
};

// out = in + dt (ta + tb); w (field 2) is 0 on the lid
__global__ void __launch_bounds__(64 * DY_COLS) combine_kernel(CombineArgs a) {
    const int ny = a.ny, nz = a.nz;
    const int nchunk = (nz + 63) / 64;
    const int k = 64 * (int)(blockIdx.x % nchunk) + (int)threadIdx.x;
    const int j = (int)(blockIdx.x / nchunk) * DY_COLS + (int)threadIdx.y;
    const int i = blockIdx.y;
    if (k >= nz || j >= ny) return;
    const long c = ((long)(i + 2) * (ny + 4) + (j + 2)) * nz + k;
    for (int f = 0; f < a.nfields; f++) {
        double v;
        if (a.tb[f])
            v = a.in[f][c] + a.dt * (a.ta[f][c] + a.tb[f][c]);
        else
            v = a.in[f][c] + a.dt * a.ta[f][c];
        if (f == 2 && k == nz - 1) v = 0.0;
        a.out[f][c] = v;
    }
}

dim3 point_grid(int nx, int ny, int nz) {
    return dim3(((nz + 63) / 64) * ((ny + DY_COLS - 1) / DY_COLS), nx);
}

}  // namespace

hipError_t launch_dyn_tend(const DynArgs& d, hipStream_t s) {
    dyn_tend_kernel<<<point_grid(d.nx, d.ny, d.nz), dim3(64, DY_COLS), 0, s>>>(d);
    return hipGetLastError();
}

hipError_t launch_combine(int nfields, const double* const* in, const double* const* ta,
                          const double* const* tb, double* const* out, int nx, int ny,
                          int nz, double dt, hipStream_t s) {
    CombineArgs a;
    for (int f = 0; f < 3 + MAXS; f++) {
        a.in[f] = f < nfields ? in[f] : nullptr;
        a.ta[f] = f < nfields ? ta[f] : nullptr;
        a.tb[f] = f < nfields && tb ? tb[f] : nullptr;
        a.out[f] = f < nfields ? out[f] : nullptr;
    }
    a.nfields = nfields;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.dt = dt;
    combine_kernel<<<point_grid(nx, ny, nz), dim3(64, DY_COLS), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace monc
