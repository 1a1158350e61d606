// Instances of the temporally blocked pass: double, compressed single grid.
#include "tblock.h"

namespace jac {

KernInfo tb_info_comp_f64(int cfg, int depth)
{
    return comp_info<double>(cfg, depth);
}

}  // namespace jac
