// Oscillatory-quadratic forward sweep with FP32 node values and
// FP64 within-rule sums: the launchers of this precision mode.
#include "sg_oscq_dev.hpp"

namespace sg {

template int launch_oscq_prec<SG_PREC_FP32_FP64_SUM>(int, int, int, int, int, const double*, const float*,
                                      const double*, double*, double*, double*, void*);
template int launch_oscq_batch_prec<SG_PREC_FP32_FP64_SUM>(int, const OscqDesc*, const double*, const float*,
                                            const double*, double*, double*, void*);

}  // namespace sg
