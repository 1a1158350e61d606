// Instances of the temporally blocked pass: double, plain mode.
#include "tblock.h"

namespace jac {

KernInfo tb_info_plain_f64(int cfg, int depth)
{
    return tb_info_mode<double, MODE_PLAIN>(cfg, depth);
}

}  // namespace jac
