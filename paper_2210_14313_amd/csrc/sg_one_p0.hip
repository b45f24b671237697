// One integrand of the dimension sweep on several workgroups (sg_one.hpp),
// precision mode 0 (FP64).
#include "sg_one.hpp"

namespace sg {
template int launch_one_inst<0>(int, int, int, int, int, const double*, double*, double*, double*, void*);
}  // namespace sg
