// Instances of the temporally blocked pass: float, plain mode.
#include "tblock.h"

namespace jac {

KernInfo tb_info_plain_f32(int cfg, int depth)
{
    return tb_info_mode<float, MODE_PLAIN>(cfg, depth);
}

}  // namespace jac
