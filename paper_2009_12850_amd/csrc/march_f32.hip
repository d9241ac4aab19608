// march_f32.hip -- instantiation of the column-march launch for
// storage float, compute float, mode TEND.
#include "march_launch.hpp"

namespace monc {
hipError_t launch_march_f32(bool pw, bool tvd, const AdvArgs& a, hipStream_t s) {
    return launch_march_t<float, float, TEND>(pw, tvd, a, s);
}
}  // namespace monc
