// Step and initialisation kernels of the F64 storage format (all tuning variants).
#include "lbm_step.hpp"

namespace lbm {
LBM_DEFINE_FORMAT(f64, FmtF64)
}  // namespace lbm
