// Forward-sweep kernel, precision mode 0 (FP64), excess budgets K <= 6
#include "sg_fwd_inst.hpp"

namespace sg {
SG_FORWARD_INSTANCE(0, 6, false)
}  // namespace sg
