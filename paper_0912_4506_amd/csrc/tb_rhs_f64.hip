// Instances of the temporally blocked pass: double, rhs mode.
#include "tblock.h"

namespace jac {

KernInfo tb_info_rhs_f64(int cfg, int depth)
{
    return tb_info_mode<double, MODE_RHS>(cfg, depth);
}

}  // namespace jac
