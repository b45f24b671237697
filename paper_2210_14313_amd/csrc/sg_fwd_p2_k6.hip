// Forward-sweep kernel, precision mode 2 (FP32 values, FP64 sums), excess budgets K <= 6
#include "sg_fwd_inst.hpp"

namespace sg {
SG_FORWARD_INSTANCE(2, 6, false)
}  // namespace sg
