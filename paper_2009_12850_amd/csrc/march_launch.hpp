// march_launch.hpp -- host-side launch of the column-march kernel for one
// storage type / compute type / mode.  Included by one source file per
// combination so the instantiations compile in parallel.
#pragma once

#include "march.hpp"

namespace monc {

struct Tiling {
    int tj, ti, njt, nseg, nblocks;
};
Tiling march_tiling(int nx, int ny, int nz, int waves);

template <typename Ts, typename T, int MODE, bool PW, int NS, bool BUD, int R, int OPT>
hipError_t launch_one(const MarchArgs& m, const Tiling& t, hipStream_t s) {
    auto kern = advect_march<Ts, T, MODE, PW, NS, BUD, R, OPT>;
    constexpr size_t lds = march_lds_bytes<Ts, T, NS, R>();
    static std::atomic<unsigned long long> attr_done{0};
    hipError_t e = set_lds_limit_once((const void*)kern, lds, &attr_done);
    if (e != hipSuccess) return e;
    kern<<<t.nblocks, march_waves<Ts, T>() * 64, lds, s>>>(m);
    return hipGetLastError();
}

template <typename Ts, typename T, int MODE, bool PW, bool BUD, int R, int OPT>
hipError_t launch_ns(const MarchArgs& m, const Tiling& t, hipStream_t s) {
    switch (m.ns) {
        case 0:  // momentum only (the fused dynamics terms need theta)
            if constexpr (PW && !(OPT & OPT_DYN))
                return launch_one<Ts, T, MODE, PW, 0, BUD, R, OPT>(m, t, s);
            break;
        case 1: return launch_one<Ts, T, MODE, PW, 1, BUD, R, OPT>(m, t, s);
        case 2: return launch_one<Ts, T, MODE, PW, 2, BUD, R, OPT>(m, t, s);
        case 3:  // with budgets, groups of three only on one-chunk columns
            if constexpr (!BUD || R == 1)
                return launch_one<Ts, T, MODE, PW, 3, BUD, R, OPT>(m, t, s);
            break;
    }
    return hipErrorInvalidValue;
}

template <typename Ts, typename T, int MODE, bool PW, bool BUD, int OPT = 0>
hipError_t launch_r(const MarchArgs& m, const Tiling& t, hipStream_t s) {
    if (m.a.nz <= 64) return launch_ns<Ts, T, MODE, PW, BUD, 1, OPT>(m, t, s);
    return launch_ns<Ts, T, MODE, PW, BUD, 2, OPT>(m, t, s);
}

// Launch the whole evaluation: scalars in groups of at most 3 per pass (2
// when budgets are accumulated on columns of more than 64 levels) so that a wave's state fits its 256
// registers without spilling; the first pass also does the momentum (if
// requested).
template <typename Ts, typename T, int MODE>
hipError_t launch_march_t(bool pw, bool tvd, const AdvArgs& a, hipStream_t s) {
    const Tiling t = march_tiling(a.nx, a.ny, a.nz, march_waves<Ts, T>());
    const bool bud = a.partials != nullptr;
    const int nscal = tvd ? a.nscal : 0;
    // columns of two chunks hold fewer accumulators in registers
    const int group = bud && a.nz > 64 ? 2 : 3;
    int s0 = 0;
    bool first = true;
    do {
        MarchArgs m;
        m.a = a;
        m.s0 = s0;
        m.ns = nscal - s0 < group ? nscal - s0 : group;
        m.ti = t.ti;
        m.njt = t.njt;
        m.nseg = t.nseg;
        m.first_pass = first ? 1 : 0;
        const bool with_pw = pw && first;
        hipError_t e;
        if ((a.dyn && with_pw) || a.spw) {
            // options of the FP64 step, no budgets: the other dynamics
            // source terms ride on the momentum pass (theta, scalar 0, in the
            // first group; later groups are plain); the centred scalar
            // scheme replaces TVD in every group
            if constexpr (MODE == STEP && std::is_same<Ts, double>::value &&
                          std::is_same<T, double>::value) {
                if (bud || (a.dyn && a.spw)) return hipErrorInvalidValue;
                if (a.dyn) {
                    if (m.ns < 1) return hipErrorInvalidValue;
                    e = launch_r<Ts, T, MODE, true, false, OPT_DYN>(m, t, s);
                } else if (with_pw) {
                    e = launch_r<Ts, T, MODE, true, false, OPT_SPW>(m, t, s);
                } else {
                    if (m.ns == 0) break;
                    e = launch_r<Ts, T, MODE, false, false, OPT_SPW>(m, t, s);
                }
            } else {
                return hipErrorInvalidValue;
            }
        } else if (with_pw) {
            e = bud ? launch_r<Ts, T, MODE, true, true>(m, t, s)
                    : launch_r<Ts, T, MODE, true, false>(m, t, s);
        } else {
            if (m.ns == 0) break;
            e = bud ? launch_r<Ts, T, MODE, false, true>(m, t, s)
                    : launch_r<Ts, T, MODE, false, false>(m, t, s);
        }
        if (e != hipSuccess) return e;
        s0 += m.ns;
        first = false;
    } while (s0 < nscal);
    return hipSuccess;
}

}  // namespace monc
