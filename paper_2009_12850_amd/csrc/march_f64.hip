// march_f64.hip -- instantiation of the column-march launch for
// storage double, compute double, mode TEND.
#include "march_launch.hpp"

namespace monc {
hipError_t launch_march_f64(bool pw, bool tvd, const AdvArgs& a, hipStream_t s) {
    return launch_march_t<double, double, TEND>(pw, tvd, a, s);
}
}  // namespace monc
