// Host-side entry points of the step, initialisation and reduction kernels
// (lbm_kernels.hip and the per-format lbm_step_<format>.hip units).
#pragma once
#include <hip/hip_runtime.h>

#include "lbm_params.hpp"

namespace lbm {

// Tuning variants compiled per storage format (see lbm_step.hpp).
constexpr int NUM_STEP_VARIANTS = 5;

// What the work list of a step kernel variant must follow.
struct StepShape {
    int lockstep;        // interior waves of a block march row by row together
    int xw_strips;       // strips next to an x-wall collide its nodes
    int block_waves;     // wavefronts per block
    int blocks_per_cu;   // resident blocks per CU
    double xw_cost;      // time of an edge-strip row relative to a plain row
};

// Device words of a persistent launch (lbm_step.hpp, persistent_kernel).
struct PersistentSync {
    unsigned* counter;      // per case, step arrivals (reset to 0 before the launch)
    int* abort;             // nonzero: a wait timed out, all wavefronts leave
    const int* case_arrivals;  // per case, arrivals per step: the blocks with an item of the case
    unsigned spin_limit;    // polls before a wait gives up
};

int launch_step(int prec, int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity,
                int export_macros, hipStream_t stream);
int step_shape(int prec, int variant, StepShape* out);
// t0: the context's step count, the start of the case's stochastic-rounding step counter
int launch_init(int prec, const CaseParams* d_cases, int case_id, long long nodes, const double* d_fields,
                int parity, unsigned t0, hipStream_t stream);
int launch_totals(const CaseParams* d_cases, int case_id, double* d_partial, int nblocks, double* d_out,
                  hipStream_t stream);
int launch_nusselt(const CaseParams* d_cases, int case_id, int side, double* d_out, hipStream_t stream);
int launch_copy(const void* src, void* dst, long long bytes, hipStream_t stream);
int launch_round_half(const float* v, const unsigned* r, float* out, long long n, hipStream_t stream);
// n steps in one launch of the persistent kernel (the counters and the
// abort word must be cleared first: launch_persistent_reset)
int launch_persistent(int prec, int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity,
                      int nsteps, const PersistentSync& sync, hipStream_t stream);
int launch_persistent_reset(unsigned* counter, int ncases, int* abort, hipStream_t stream);
int persistent_blocks(int prec, int variant, int* blocks_per_cu);

#define LBM_DECLARE_FORMAT(NAME)                                                                             \
    int launch_step_##NAME(int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork,        \
                           int parity, int export_macros, hipStream_t stream);                               \
    int step_shape_##NAME(int variant, StepShape* out);                                                      \
    int launch_persistent_##NAME(int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork,  \
                                 int parity, int nsteps, const PersistentSync& sync, hipStream_t stream);    \
    int persistent_blocks_##NAME(int variant, int* blocks_per_cu);                                           \
    int launch_init_##NAME(const CaseParams* d_cases, int case_id, long long nodes, const double* d_fields,  \
                           int parity, unsigned t0, hipStream_t stream);
LBM_DECLARE_FORMAT(f64)
LBM_DECLARE_FORMAT(f32)
LBM_DECLARE_FORMAT(f16)
LBM_DECLARE_FORMAT(f32g16)
#undef LBM_DECLARE_FORMAT

}  // namespace lbm
