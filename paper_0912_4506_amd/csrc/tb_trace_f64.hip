// Instances of the temporally blocked pass: double, trace mode.
#include "tblock.h"

namespace jac {

KernInfo tb_info_trace_f64(int cfg, int depth)
{
    return tb_info_mode<double, MODE_TRACE>(cfg, depth);
}

}  // namespace jac
