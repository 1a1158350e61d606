// Instances of the batched (persistent or lockstep) pass: double.
#include "tblock.h"

namespace jac {

KernInfo batch_info_f64(int cfg, int depth, int fixed)
{
    return batch_info<double>(cfg, depth, fixed);
}

}  // namespace jac
