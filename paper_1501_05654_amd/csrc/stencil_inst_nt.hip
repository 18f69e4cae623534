// Stencil kernels with stage outputs streamed past L2 (non-temporal stores).
#include "stencil_kernels.h"

namespace rsg {
RSG_STENCIL_INST(, true)
}  // namespace rsg
