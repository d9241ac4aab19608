// scaled.hip -- the work-scaled Piacsek-Williams experiment on the production
// column march.
//
// Brown et al. (Sec. 4) scale the arithmetic of the PW scheme up to that of
// the ULTIMATE scheme (about sixteen times as much) to see how a GPU behaves
// once the same data carries more computation.  Here the same question is put
// to the march kernel that computes the source terms: its momentum-only
// instantiation evaluates the PW arithmetic `work` times per grid point on
// the values it has loaded (each repetition chained to the previous result,
// so the compiler can neither merge nor drop one; the result is bitwise that
// of one evaluation).  Bytes per point stay those of the PW source terms (u,
// v, w read, su, sv, sw written) while the arithmetic grows `work`-fold, so a
// sweep shows where FP64 and FP32 turn from HBM-bound to ALU-bound in the
// kernel the step actually runs.
#include "march_launch.hpp"

namespace monc {

namespace {

template <typename T>
hipError_t launch_work(const AdvArgs& a, hipStream_t s) {
    const Tiling t = march_tiling(a.nx, a.ny, a.nz, march_waves<T, T>());
    MarchArgs m;
    m.a = a;
    m.s0 = 0;
    m.ns = 0;
    m.ti = t.ti;
    m.njt = t.njt;
    m.nseg = t.nseg;
    m.first_pass = 1;
    if (a.nz <= 64) return launch_one<T, T, TEND, true, 0, false, 1, OPT_WORK>(m, t, s);
    return launch_one<T, T, TEND, true, 0, false, 2, OPT_WORK>(m, t, s);
}

}  // namespace

hipError_t launch_pw_scaled(int dtype, const AdvArgs& a, hipStream_t s) {
    if (dtype == MONC_F64) return launch_work<double>(a, s);
    return launch_work<float>(a, s);
}

}  // namespace monc
