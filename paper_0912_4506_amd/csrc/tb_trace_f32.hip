// Instances of the temporally blocked pass: float, trace mode.
#include "tblock.h"

namespace jac {

KernInfo tb_info_trace_f32(int cfg, int depth)
{
    return tb_info_mode<float, MODE_TRACE>(cfg, depth);
}

}  // namespace jac
