// FP64 reductions, the copy kernel and the dispatch of the step and
// initialisation launches to the translation unit of each storage format.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_launch.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// FP64 reductions (deterministic: fixed per-thread order, fixed tree)
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Partial sums of rho, rho ux, rho uy, rho E over rows of the exported
// macros; out[block * 4 + k].
__global__ __launch_bounds__(RED_THREADS) void totals_partial(const CaseParams* __restrict__ cases, int case_id,
                                                              double* __restrict__ out)
{
    __shared__ double sh[RED_THREADS];
    const CaseParams& P = cases[case_id];
    const long long nn = (long long)P.nx * P.ny;
    const long long per = (nn + gridDim.x - 1) / gridDim.x;
    const long long lo = blockIdx.x * per, hi = min(nn, lo + per);
    double a[4] = {0, 0, 0, 0};
    for (long long i = lo + threadIdx.x; i < hi; i += RED_THREADS) {
        const double rho = P.macro[i], ux = P.macro[nn + i], uy = P.macro[2 * nn + i], T = P.macro[3 * nn + i];
        a[0] += rho;
        a[1] += rho * ux;
        a[2] += rho * uy;
        a[3] += rho * (P.cd.cv_d * T + 0.5 * (ux * ux + uy * uy));
    }
    for (int k = 0; k < 4; ++k) {
        const double s = block_sum(a[k], sh);
        if (threadIdx.x == 0) out[blockIdx.x * 4 + k] = s;
    }
}

__global__ __launch_bounds__(RED_THREADS) void sum_partials(const double* __restrict__ in, int nblocks,
                                                            double* __restrict__ out)
{
    __shared__ double sh[RED_THREADS];
    for (int k = 0; k < 4; ++k) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) a += in[b * 4 + k];
        const double s = block_sum(a, sh);
        if (threadIdx.x == 0) out[k] = s;
    }
}

// Mean Nusselt number through a Dirichlet side: trapezoid rule along the
// side of J_n = -lambda(T) dT/dn with a second-order one-sided dT/dn,
// divided by lambda0 (T_lo - T_hi) of that axis.  mu(T)/mu0 is evaluated in
// FP64; lambda = C_p mu / Pr cancels C_p / Pr against lambda0.
__global__ __launch_bounds__(RED_THREADS) void nusselt_kernel(const CaseParams* __restrict__ cases, int case_id,
                                                              int side, double* __restrict__ out)
{
    __shared__ double sh[RED_THREADS];
    const CaseParams& P = cases[case_id];
    const int nx = P.nx, ny = P.ny;
    const long long nn = (long long)nx * ny;
    const double* T = P.macro + 3 * nn;
    const int len = side < 2 ? ny : nx;
    const int lo = side < 2 ? 0 : 2;
    const double dT = P.cd.side_T[lo] - P.cd.side_T[lo + 1];
    const double S = P.cd.suth_S, T0 = P.cd.T0;
    double acc = 0.0;
    for (int j = threadIdx.x; j < len; j += RED_THREADS) {
        double t0, t1, t2, d;
        if (side < 2) {
            const int x0 = side == 0 ? 0 : nx - 1;
            d = side == 0 ? 1.0 : -1.0;
            const int s1 = side == 0 ? 1 : -1;
            t0 = T[(long long)j * nx + x0];
            t1 = T[(long long)j * nx + x0 + s1];
            t2 = T[(long long)j * nx + x0 + 2 * s1];
        } else {
            const int y0 = side == 2 ? 0 : ny - 1;
            d = side == 2 ? 1.0 : -1.0;
            const int s1 = side == 2 ? 1 : -1;
            t0 = T[(long long)y0 * nx + j];
            t1 = T[(long long)(y0 + s1) * nx + j];
            t2 = T[(long long)(y0 + 2 * s1) * nx + j];
        }
        const double dTdn = d * (-3.0 * t0 + 4.0 * t1 - t2) * 0.5;
        double mu_rel;
        const double th = t0 / T0;
        if (P.visc_law == VISC_CONST) mu_rel = 1.0;
        else if (P.visc_law == VISC_LINEAR) mu_rel = th;
        else mu_rel = th * sqrt(th) * (1.0 + S) / (th + S);
        const double wgt = (j == 0 || j == len - 1) ? 0.5 : 1.0;
        acc += wgt * (-mu_rel * dTdn);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = s / dT;
}

// ---------------------------------------------------------------------------
// plain copy (measured-bandwidth probe and byte-counter calibration)
// ---------------------------------------------------------------------------
// One 16-byte element per thread, one 4 KiB chunk per block, a block per
// chunk (no grid-stride loop): of the patterns measured on MI355X (grid-stride
// loops of 2048-16384 blocks, 2-8 elements per thread, non-temporal loads or
// stores, hipMemcpy device to device) this one moves the most bytes,
// 6.2 TB/s on a 1 GiB copy.
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// FP16 stochastic rounding of n values with the store codec's own code
// (diagnostics): out[i] = the stored FP16 value of v[i] with operand r[i].
__global__ __launch_bounds__(256) void round_half_kernel(const float* __restrict__ v, const unsigned* __restrict__ r,
                                                         float* __restrict__ out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = __half2float(__ushort_as_half(Store<__half>::sr_bits(v[i], r[i])));
}

// clears the step counters and the abort word of a persistent launch
__global__ __launch_bounds__(256) void persistent_reset_kernel(unsigned* counter, int ncases, int* abort)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncases) counter[i] = 0u;
    if (i == 0) *abort = 0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
int launch_persistent_reset(unsigned* counter, int ncases, int* abort, hipStream_t stream)
{
    hipLaunchKernelGGL(persistent_reset_kernel, dim3(unsigned((std::max(ncases, 1) + 255) / 256)), dim3(256), 0,
                       stream, counter, ncases, abort);
    return int(hipGetLastError());
}

int launch_persistent(int prec, int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity,
                      int nsteps, const PersistentSync& sync, hipStream_t stream)
{
    switch (prec) {
    case PREC_F64: return launch_persistent_f64(variant, d_cases, d_work, nwork, parity, nsteps, sync, stream);
    case PREC_F32: return launch_persistent_f32(variant, d_cases, d_work, nwork, parity, nsteps, sync, stream);
    case PREC_F32G16: return launch_persistent_f32g16(variant, d_cases, d_work, nwork, parity, nsteps, sync, stream);
    default: return launch_persistent_f16(variant, d_cases, d_work, nwork, parity, nsteps, sync, stream);
    }
}

int persistent_blocks(int prec, int variant, int* blocks_per_cu)
{
    switch (prec) {
    case PREC_F64: return persistent_blocks_f64(variant, blocks_per_cu);
    case PREC_F32: return persistent_blocks_f32(variant, blocks_per_cu);
    case PREC_F32G16: return persistent_blocks_f32g16(variant, blocks_per_cu);
    default: return persistent_blocks_f16(variant, blocks_per_cu);
    }
}

int launch_round_half(const float* v, const unsigned* r, float* out, long long n, hipStream_t stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(round_half_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, v, r, out, n);
    return int(hipGetLastError());
}

int launch_copy(const void* src, void* dst, long long bytes, hipStream_t stream)
{
    const long long n = bytes / 16;
    const long long blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) return int(hipErrorInvalidValue);
    hipLaunchKernelGGL(copy_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, static_cast<const float4*>(src),
                       static_cast<float4*>(dst), n);
    return int(hipGetLastError());
}

int launch_step(int prec, int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity,
                int export_macros, hipStream_t stream)
{
    switch (prec) {
    case PREC_F64: return launch_step_f64(variant, d_cases, d_work, nwork, parity, export_macros, stream);
    case PREC_F32: return launch_step_f32(variant, d_cases, d_work, nwork, parity, export_macros, stream);
    case PREC_F32G16: return launch_step_f32g16(variant, d_cases, d_work, nwork, parity, export_macros, stream);
    default: return launch_step_f16(variant, d_cases, d_work, nwork, parity, export_macros, stream);
    }
}

// Lockstep rule, x-wall handling, block size and resident blocks per CU of a
// variant of the step kernel (the work list is built for these).
int step_shape(int prec, int variant, StepShape* out)
{
    switch (prec) {
    case PREC_F64: return step_shape_f64(variant, out);
    case PREC_F32: return step_shape_f32(variant, out);
    case PREC_F32G16: return step_shape_f32g16(variant, out);
    default: return step_shape_f16(variant, out);
    }
}

int launch_init(int prec, const CaseParams* d_cases, int case_id, long long nodes, const double* d_fields,
                int parity, unsigned t0, hipStream_t stream)
{
    switch (prec) {
    case PREC_F64: return launch_init_f64(d_cases, case_id, nodes, d_fields, parity, t0, stream);
    case PREC_F32: return launch_init_f32(d_cases, case_id, nodes, d_fields, parity, t0, stream);
    case PREC_F32G16: return launch_init_f32g16(d_cases, case_id, nodes, d_fields, parity, t0, stream);
    default: return launch_init_f16(d_cases, case_id, nodes, d_fields, parity, t0, stream);
    }
}

int launch_totals(const CaseParams* d_cases, int case_id, double* d_partial, int nblocks, double* d_out,
                  hipStream_t stream)
{
    hipLaunchKernelGGL(totals_partial, dim3(nblocks), dim3(RED_THREADS), 0, stream, d_cases, case_id, d_partial);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(RED_THREADS), 0, stream, d_partial, nblocks, d_out);
    return int(hipGetLastError());
}

int launch_nusselt(const CaseParams* d_cases, int case_id, int side, double* d_out, hipStream_t stream)
{
    hipLaunchKernelGGL(nusselt_kernel, dim3(1), dim3(RED_THREADS), 0, stream, d_cases, case_id, side, d_out);
    return int(hipGetLastError());
}

}  // namespace lbm
