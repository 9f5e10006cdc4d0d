// Step and initialisation kernels of the F16 storage format (all tuning variants).
#include "lbm_step.hpp"

namespace lbm {
LBM_DEFINE_FORMAT(f16, FmtF16)
}  // namespace lbm
