// march_bf16.hip -- instantiation of the column-march launch for
// storage bf16, compute float, mode TEND.
#include "march_launch.hpp"

namespace monc {
hipError_t launch_march_bf16(bool pw, bool tvd, const AdvArgs& a, hipStream_t s) {
    return launch_march_t<bf16, float, TEND>(pw, tvd, a, s);
}
}  // namespace monc
