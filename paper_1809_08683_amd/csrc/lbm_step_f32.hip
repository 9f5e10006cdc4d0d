// Step and initialisation kernels of the F32 storage format (all tuning variants).
#include "lbm_step.hpp"

namespace lbm {
LBM_DEFINE_FORMAT(f32, FmtF32)
}  // namespace lbm
