// march_stepmix.hip -- instantiation of the column-march launch for
// storage double, compute float, mode STEP.
#include "march_launch.hpp"

namespace monc {
hipError_t launch_march_stepmix(bool pw, bool tvd, const AdvArgs& a, hipStream_t s) {
    return launch_march_t<double, float, STEP>(pw, tvd, a, s);
}
}  // namespace monc
