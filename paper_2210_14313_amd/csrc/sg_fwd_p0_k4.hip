// Forward-sweep kernel, precision mode 0 (FP64), excess budgets K <= 4
#include "sg_fwd_inst.hpp"

namespace sg {
SG_FORWARD_INSTANCE(0, 4, false)
}  // namespace sg
