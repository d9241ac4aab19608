// march_step64.hip -- instantiation of the column-march launch for
// storage double, compute double, mode STEP.
#include "march_launch.hpp"

namespace monc {
hipError_t launch_march_step64(bool pw, bool tvd, const AdvArgs& a, hipStream_t s) {
    return launch_march_t<double, double, STEP>(pw, tvd, a, s);
}
}  // namespace monc
