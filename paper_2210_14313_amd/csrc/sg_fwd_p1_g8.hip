// Forward-sweep kernel, precision mode 1 (FP32 values, two-sum compensated FP32 sums), excess budgets K <= 8, built with the gaussian family
#include "sg_fwd_inst.hpp"

namespace sg {
SG_FORWARD_INSTANCE(1, 8, true)
}  // namespace sg
