// Instances of the temporally blocked pass: float, compressed single grid.
#include "tblock.h"

namespace jac {

KernInfo tb_info_comp_f32(int cfg, int depth)
{
    return comp_info<float>(cfg, depth);
}

}  // namespace jac
