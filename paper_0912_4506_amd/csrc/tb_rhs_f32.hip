// Instances of the temporally blocked pass: float, rhs mode.
#include "tblock.h"

namespace jac {

KernInfo tb_info_rhs_f32(int cfg, int depth)
{
    return tb_info_mode<float, MODE_RHS>(cfg, depth);
}

}  // namespace jac
