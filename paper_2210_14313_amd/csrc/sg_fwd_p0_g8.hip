// Forward-sweep kernel, precision mode 0 (FP64), excess budgets K <= 8, built with the gaussian family
#include "sg_fwd_inst.hpp"

namespace sg {
SG_FORWARD_INSTANCE(0, 8, true)
}  // namespace sg
