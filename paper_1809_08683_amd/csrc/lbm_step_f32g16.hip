// Step and initialisation kernels of the F32G16 storage format (all tuning variants).
#include "lbm_step.hpp"

namespace lbm {
LBM_DEFINE_FORMAT(f32g16, FmtF32G16)
}  // namespace lbm
