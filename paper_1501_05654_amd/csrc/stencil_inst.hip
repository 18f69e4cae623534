// Stencil kernels with stage outputs stored with the default cache policy.
#include "stencil_kernels.h"

namespace rsg {
RSG_STENCIL_INST(, false)
}  // namespace rsg
