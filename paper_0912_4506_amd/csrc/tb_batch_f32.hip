// Instances of the batched (persistent or lockstep) pass: float.
#include "tblock.h"

namespace jac {

KernInfo batch_info_f32(int cfg, int depth, int fixed)
{
    return batch_info<float>(cfg, depth, fixed);
}

}  // namespace jac
