// Parameter blocks shared by the host runtime and the kernels.
#pragma once

#include <stdint.h>

namespace lbm {

enum { EOS_DECOUPLED = 0, EOS_IDEAL = 1, EOS_VDW = 2, EOS_CS = 3 };
enum { VISC_CONST = 0, VISC_LINEAR = 1, VISC_SUTHERLAND = 2 };
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_F16S = 2, PREC_F32G16 = 3 };

// Constants of one case in one compute type.
template <typename C>
struct Coef {
    C rho0, T0, inv_T0, R, a_vdw, b_vdw, b_cs;
    C rho0_cp;                 // rho0 C_p (n^eq)
    C mu0, suth_S, suth_1pS;   // viscosity law
    C bulk_over_varpi;         // (bulk / kinematic viscosity ratio) / varpi
    C varpi_over_bulk;
    C inv_kappa_rho0_Pr, kappa_rho0_Pr;
    C fx, fy;
    C side_ux[4], side_uy[4];
    double cv_d, inv_cv_d;     // C_v, used in the FP64 temperature recovery
    double side_T[4];
    // rest state (rho0, u = 0, T0) the stored DFs are measured from
    double rho0_d, T0_d, p0_d, rhoE0_d;   // p_EOS(rho0, T0), rho0 C_v T0
    // Reference of 16-bit g rows (FP32 f + FP16 g and FP16S): the stored g of
    // column x is measured from the rest equilibrium of the conduction state
    // between two Dirichlet x-walls, which differs from the rest state above
    // by g_ref - g_rest = v_q s(x) with s(x) = gs0 + gsk x = rho0 C_p (T_ref(x) - T0).
    // Zero when the case has no such reference.
    C gs0, gsk;
    double R_d, a_d, b_d, bcs_d;           // EOS constants for FP64 evaluation
};

// Columns are stored strip by strip: strip s owns the off-wall columns
// [xlo + 62 s, xlo + 62 s + 62) and keeps them in a region of 64 slots:
// slot j holds column xlo + 62 s - 1 + j, so slots 1..62 are its own columns
// and slots 0 and 63 (the neighbouring strips' edge columns) are not
// written.  On a walled x axis the left wall column sits in slot 0 of strip
// 0, the right wall and ghost columns after the last strip's columns, and
// the left ghost column in the last slot of the row.
constexpr int STRIP_COLS = 62;
constexpr int REGION_SLOTS = 64;

struct CaseParams {
    int nx, ny, pitch;         // pitch: elements per stored row of one DF = REGION_SLOTS * strips (or more)
    int xlo, nstrips;          // first off-wall column, number of strips
    int wall_x, wall_y;        // 1: both sides of that axis are walls
    long long rowblk;          // elements per stored row block = 18 * pitch
    int eos, visc_law, per_mass, cubic, extrap_order;
    int side_adiabatic[4];
    void* buf[2];              // ping-pong DF buffers: (ny + 2) row blocks of 18 DF rows (f then g)
    double* macro;             // [5][ny][nx]: rho, ux, uy, T, p (written on export steps)
    int* flag;                 // divergence flag of this case
    unsigned* tick;            // step counters of the stochastic rounding: a step reads [parity], writes [parity ^ 1]
    Coef<double> cd;
    Coef<float> cf;
};

// One wavefront's share of a step.
//   kind 0: interior strip, output columns [x0, x0 + 62) clipped to the off-wall
//           range, rows [y0, y0 + len), marched upwards (dir 0) or downwards (dir 1)
//   kind 1: wall nodes [x0, x0 + len) of the case's wall-node enumeration
struct WorkItem {
    int case_id, kind, x0, y0, len, dir;
};

}  // namespace lbm
