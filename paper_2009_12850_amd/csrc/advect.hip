// advect.hip -- dispatch of the fused advection launches and the x-y tiling.
#include "march_launch.hpp"

namespace monc {

hipError_t launch_march_f64(bool pw, bool tvd, const AdvArgs& a, hipStream_t s);
hipError_t launch_march_f32(bool pw, bool tvd, const AdvArgs& a, hipStream_t s);
hipError_t launch_march_bf16(bool pw, bool tvd, const AdvArgs& a, hipStream_t s);
hipError_t launch_march_step64(bool pw, bool tvd, const AdvArgs& a, hipStream_t s);
hipError_t launch_march_stepmix(bool pw, bool tvd, const AdvArgs& a, hipStream_t s);

// Tiles of `waves` columns along y (half as many when a column needs two
// 64-level chunks); the x range is cut into segments so that the grid holds
// about MONC_TILE_TARGET workgroups, each marching >= 8 planes.  The FP64
// kernels hold one workgroup per CU, so 256 workgroups (one per CU of the
// device) march whole rows of tiles at once, without later rounds whose tiles
// start away from their neighbours (and fewer segment prologues); measured
// 2-4 % faster than 512 or 1024 on 1024 x 1024 x 128.  The tiling
// depends on the grid alone, so the number of budget partial rows, and with
// it the budgets' summation order, is fixed for a grid.
#ifndef MONC_TILE_TARGET
#define MONC_TILE_TARGET 256
#endif
Tiling march_tiling(int nx, int ny, int nz, int waves) {
    Tiling t;
    t.tj = nz <= 64 ? waves : waves / 2;
    t.njt = (ny + t.tj - 1) / t.tj;
    int nseg = MONC_TILE_TARGET / t.njt;
    const int max_seg = nx / 8 > 0 ? nx / 8 : 1;
    if (nseg > max_seg) nseg = max_seg;
    if (nseg < 1) nseg = 1;
    t.ti = (nx + nseg - 1) / nseg;
    if (t.ti > nx) t.ti = nx;
    t.nseg = (nx + t.ti - 1) / t.ti;
    t.nblocks = t.njt * t.nseg;
    return t;
}

// Both step variants hold FP64 state, so they run the FP64 workgroup size.
int step_grid(int nx, int ny, int nz, bool mixed) {
    (void)mixed;
    return march_tiling(nx, ny, nz, march_waves<double, double>()).nblocks;
}

int step_blocks(int nx, int ny, int nz) { return step_grid(nx, ny, nz, false); }

hipError_t launch_advect(int dtype, int mode, bool pw, bool tvd, bool mixed,
                         const AdvArgs& a, hipStream_t s) {
    if (mode == STEP) {
        if (mixed) return launch_march_stepmix(pw, tvd, a, s);
        return launch_march_step64(pw, tvd, a, s);
    }
    switch (dtype) {
        case MONC_F64: return launch_march_f64(pw, tvd, a, s);
        case MONC_F32: return launch_march_f32(pw, tvd, a, s);
        case MONC_BF16: return launch_march_bf16(pw, tvd, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace monc
