// Device-side building blocks of the coupled D2Q9 MRT step of Huang, Wu &
// Adams (arXiv:1809.08683), written for gfx950.  Everything here works on one
// lattice node held in registers; the kernels that march over the lattice
// live in lbm_kernels.hip.
//
// Lattice units throughout: dx = dt = c = 1, c_s^2 = 1/3.  Velocities are
// numbered as in Sec. 2: e0 = 0, e1..e4 along +x, +y, -x, -y, e5..e8 along
// (1,1), (-1,1), (-1,-1), (1,-1).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "lbm_params.hpp"
#include "lbm_rounding.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Model constants fixed by the paper: alpha1 = -1, beta1 = 1 (Sec. 2.1),
// varpi = 1/6, gamma1 = -2, gamma2 = 2 (Sec. 4).  alpha2, beta2, k, h, b
// follow from eq. LBE.u.coefficients; the coefficients of R, T and X are the
// entries printed in Sec. 2.1 with the rate-independent factors folded.
// ---------------------------------------------------------------------------
namespace mc {
constexpr double varpi = 1.0 / 6.0;
constexpr double gamma1 = -2.0, gamma2 = 2.0;
constexpr double alpha1 = -1.0, beta1 = 1.0;
constexpr double alpha2 = -(2.0 * alpha1 + varpi + 1.0) / (1.0 - varpi);
constexpr double beta2 = -2.0 * beta1 / (1.0 - varpi);
constexpr double k = 1.0 - varpi;
constexpr double h = 6.0 * varpi * (1.0 - varpi) / (1.0 - 3.0 * varpi);
constexpr double b = (1.0 - varpi) / (1.0 - 3.0 * varpi);
// R entries (rows/cols 1, 7, 8)
constexpr double cR11 = -(9.0 - 15.0 * k - 2.0 * h) / (4.0 * varpi);  // * s_e |u|^2
constexpr double cR17 = -3.0 * (9.0 - 3.0 * k + 2.0 * h) / 4.0;       // * s_p (2-s_e)/(2-s_p) (ux^2-uy^2)
constexpr double cR18 = 12.0 * (3.0 * k + h);                          // * s_p (2-s_e)/(2-s_p) ux uy
constexpr double cR71 = -(3.0 - 4.0 * b) / (4.0 * varpi);              // * s_e (2-s_p)/(2-s_e) (ux^2-uy^2)
constexpr double cR77 = -3.0 * (3.0 + 4.0 * b) / 4.0;                  // * s_p |u|^2
constexpr double cR81 = b / varpi;                                      // * s_e (2-s_p)/(2-s_e) ux uy
constexpr double cR88 = 6.0 * b;                                        // * s_p |u|^2
}  // namespace mc

// ---------------------------------------------------------------------------
// small numeric helpers, specialised per compute type
// ---------------------------------------------------------------------------
// FP64 reciprocal: hardware estimate refined by two Newton steps (relative
// error at the level of the last bit, without the IEEE division sequence)
__device__ __forceinline__ double rcp_d(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return r;
}

template <typename C> __device__ __forceinline__ C rcp(C x);
template <> __device__ __forceinline__ double rcp<double>(double x) { return rcp_d(x); }
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// pointers into global memory (lets the compiler use global, not flat, loads)
template <typename T> using gconst = const __attribute__((address_space(1))) T;
template <typename T> using gmut = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ gconst<T>* as_global(const void* p) { return (gconst<T>*)p; }
template <typename T> __device__ __forceinline__ gmut<T>* as_global_mut(void* p) { return (gmut<T>*)p; }

template <typename C> __device__ __forceinline__ C sqrt_(C x);
template <> __device__ __forceinline__ double sqrt_<double>(double x) { return __builtin_sqrt(x); }
template <> __device__ __forceinline__ float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename C> __device__ __forceinline__ bool finite_pos(C x) { return x > C(0) && x < C(1e300); }

// Constants of one case in the compute type.
template <typename C>
__device__ __forceinline__ const Coef<C>& coef(const CaseParams& P);
template <> __device__ __forceinline__ const Coef<double>& coef<double>(const CaseParams& P) { return P.cd; }
template <> __device__ __forceinline__ const Coef<float>& coef<float>(const CaseParams& P) { return P.cf; }

// ---------------------------------------------------------------------------
// moment transform m = M f (eq. M) and its inverse M^-1 = M^T diag(1/9, 1/36,
// 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4), unrolled with shared partial sums
// ---------------------------------------------------------------------------
template <typename C>
__device__ __forceinline__ void to_moments(const C f[9], C m[9])
{
    const C ax = f[1] + f[3], ay = f[2] + f[4];
    const C a = ax + ay;                     // axis sum
    const C d = f[5] + f[6] + f[7] + f[8];   // diagonal sum
    const C dx = f[5] - f[6] - f[7] + f[8];  // sum over diagonals of e_x
    const C dy = f[5] + f[6] - f[7] - f[8];
    const C sx = f[1] - f[3], sy = f[2] - f[4];
    m[0] = f[0] + a + d;
    m[1] = C(-4) * f[0] - a + C(2) * d;
    m[2] = C(4) * f[0] - C(2) * a + d;
    m[3] = sx + dx;
    m[4] = C(-2) * sx + dx;
    m[5] = sy + dy;
    m[6] = C(-2) * sy + dy;
    m[7] = ax - ay;
    m[8] = f[5] - f[6] + f[7] - f[8];
}

template <typename C>
__device__ __forceinline__ void from_moments(const C m[9], C f[9])
{
    const C a0 = m[0] * C(1.0 / 9.0), a1 = m[1] * C(1.0 / 36.0), a2 = m[2] * C(1.0 / 36.0);
    const C a3 = m[3] * C(1.0 / 6.0), a4 = m[4] * C(1.0 / 12.0);
    const C a5 = m[5] * C(1.0 / 6.0), a6 = m[6] * C(1.0 / 12.0);
    const C a7 = m[7] * C(0.25), a8 = m[8] * C(0.25);
    const C c = a0 - a1 - C(2) * a2;   // common part of the axis directions
    const C d = a0 + C(2) * a1 + a2;   // common part of the diagonals
    const C X = a3 - C(2) * a4, Y = a5 - C(2) * a6;
    const C Pp = a3 + a4, Q = a5 + a6;
    f[0] = a0 - C(4) * a1 + C(4) * a2;
    f[1] = c + X + a7;
    f[3] = c - X + a7;
    f[2] = c + Y - a7;
    f[4] = c - Y - a7;
    f[5] = d + Pp + Q + a8;
    f[6] = d - Pp + Q - a8;
    f[7] = d - Pp - Q + a8;
    f[8] = d + Pp - Q - a8;
}

// ---------------------------------------------------------------------------
// Node state.  The DFs are stored and processed as deviations from the rest
// state (rho0, u = 0, T0): f - f_rest with f_rest = M^-1 m^eq(rho0, 0, eta0)
// and g - g_rest with g_rest = M^-1 n^eq(rho0 C_v T0, 0, T0).  Every moment
// below is the deviation of the paper's moment from its rest value, so the
// small departures that carry the physics keep the full relative precision
// of the storage format; the collision operator is linear in the DFs, so
// the update is the paper's update written for deviations.
// ---------------------------------------------------------------------------
template <typename C>
struct NodeState {
    C drho;               // rho - rho0
    C ux, uy;             // velocity
    C jx, jy;             // rho u = sum e f + F/2, kept as computed (no rho * (j / rho) round trip)
    C dT;                 // T - T0 (T recovered in FP64)
    C drhoE;              // rho E - rho0 C_v T0
    C dp, deta;           // p - p0, eta - eta0
    C H;                  // E + p / rho
    C inv_rho;            // 1 / rho
};

template <typename C> __device__ __forceinline__ C rho_of(const Coef<C>& K, const NodeState<C>& s) { return K.rho0 + s.drho; }
template <typename C> __device__ __forceinline__ C T_of(const Coef<C>& K, const NodeState<C>& s) { return K.T0 + s.dT; }

// external force F (per unit volume, or rho * g per unit mass) and q_e = u.F
template <typename C>
struct Forcing {
    C Fx, Fy, qe;
};
template <typename C>
__device__ __forceinline__ Forcing<C> forcing(const Coef<C>& K, int per_mass, const NodeState<C>& s)
{
    Forcing<C> F;
    const C rho = rho_of(K, s);
    F.Fx = per_mass ? rho * K.fx : K.fx;
    F.Fy = per_mass ? rho * K.fy : K.fy;
    F.qe = s.ux * F.Fx + s.uy * F.Fy;
    return F;
}

template <typename C>
struct Rates {
    C se, sq, sp, we, wp;       // s_eps = s_e, s_0 = s_j = 1
    C sige, sigj;               // sigma_eps = sigma_p = sigma_e, sigma_q = sigma_j, sigma_0 = 1
    C r_ep;                     // (2 - s_e)/(2 - s_p)
    C r_pe;                     // (2 - s_p)/(2 - s_e)
};

// p_EOS(rho, T) in FP64 for the four equations of state (Sec. 4, eqs. EOSs,
// plus van der Waals)
template <typename C>
__device__ __forceinline__ double eos_pressure_d(const Coef<C>& K, int eos, double rho, double T)
{
    switch (eos) {
    case EOS_DECOUPLED: return rho * K.R_d * K.T0_d;
    case EOS_IDEAL: return rho * K.R_d * T;
    case EOS_VDW: return rho * K.R_d * T / (1.0 - K.b_d * rho) - K.a_d * rho * rho;
    default: {  // Carnahan-Starling
        const double be = K.bcs_d * rho * 0.25, omb = 1.0 - be;
        return (1.0 + be + be * be - be * be * be) / (omb * omb * omb) * rho * K.R_d * T;
    }
    }
}

// p - p0: exact deviation forms for the linear-in-rho EOSs, FP64 otherwise
template <typename C>
__device__ __forceinline__ C eos_dp(const Coef<C>& K, int eos, C drho, C dT, double rho_d, double T_d)
{
    if (eos == EOS_DECOUPLED) return K.R * K.T0 * drho;
    if (eos == EOS_IDEAL) return K.R * (drho * (K.T0 + dT) + K.rho0 * dT);   // R (rho T - rho0 T0)
    return C(eos_pressure_d<C>(K, eos, rho_d, T_d) - K.p0_d);
}

// Completes a state from rho, u, T, E (force, p, eta, H).
// eta = [p / c_s^2 - (2 + alpha1) rho] / beta1 (end of Sec. 2.2).
template <typename C>
__device__ __forceinline__ void complete_state(const Coef<C>& K, int eos, NodeState<C>& s, double rho_d,
                                               double T_d, double E_d)
{
    s.dp = eos_dp<C>(K, eos, s.drho, s.dT, rho_d, T_d);
    s.deta = (C(3) * s.dp - C(2.0 + mc::alpha1) * s.drho) * C(1.0 / mc::beta1);
    s.H = C(E_d) + (C(K.p0_d) + s.dp) * s.inv_rho;   // H = E + p/rho
}

// Interior node: rho = sum f, rho u = sum e f + F/2 (eq. rho.u),
// rho E = sum g + q_e/2 (eq. E), T = (E - |u|^2/2)/C_v with E and the
// subtraction carried out in FP64.  dm = M (f - f_rest), dn0 = sum (g - g_rest).
// Returns T in FP64.
template <typename C>
__device__ __forceinline__ double state_from_moments(const Coef<C>& K, int eos, int per_mass,
                                                     const C dm[9], C dn0, NodeState<C>& s)
{
    s.drho = dm[0];
    const C rho = K.rho0 + s.drho;
    s.inv_rho = rcp<C>(rho);
    const C Fx = per_mass ? rho * K.fx : K.fx;
    const C Fy = per_mass ? rho * K.fy : K.fy;
    s.jx = dm[3] + C(0.5) * Fx;
    s.jy = dm[5] + C(0.5) * Fy;
    s.ux = s.jx * s.inv_rho;
    s.uy = s.jy * s.inv_rho;
    s.drhoE = dn0 + C(0.5) * (s.ux * Fx + s.uy * Fy);
    const double rho_d = K.rho0_d + double(s.drho);
    const double uxd = double(s.ux), uyd = double(s.uy);
    const double E_d = (K.rhoE0_d + double(s.drhoE)) * rcp_d(rho_d);
    const double T_d = (E_d - 0.5 * (uxd * uxd + uyd * uyd)) * K.inv_cv_d;
    s.dT = C(T_d - K.T0_d);
    complete_state<C>(K, eos, s, rho_d, T_d, E_d);
    return T_d;
}

// Node of an interior strip whose lane may sit on an x-wall (wl): the
// off-wall formulas of state_from_moments with, on a wall lane, the wall
// velocity and (Dirichlet wall, dir) the wall temperature selected in, which
// gives state_wall's result for the wall lane without a divergent branch.
template <typename C>
__device__ __forceinline__ double state_select(const Coef<C>& K, int eos, int per_mass, const C dm[9], C dn0,
                                               bool wl, C ubx, C uby, bool dir, double Tw, NodeState<C>& s)
{
    s.drho = dm[0];
    const C rho = K.rho0 + s.drho;
    s.inv_rho = rcp<C>(rho);
    const C Fx = per_mass ? rho * K.fx : K.fx;
    const C Fy = per_mass ? rho * K.fy : K.fy;
    const C jx = dm[3] + C(0.5) * Fx, jy = dm[5] + C(0.5) * Fy;
    s.jx = wl ? rho * ubx : jx;
    s.jy = wl ? rho * uby : jy;
    s.ux = wl ? ubx : jx * s.inv_rho;
    s.uy = wl ? uby : jy * s.inv_rho;
    const C drhoE = dn0 + C(0.5) * (s.ux * Fx + s.uy * Fy);
    const double rho_d = K.rho0_d + double(s.drho);
    const double uxd = double(s.ux), uyd = double(s.uy);
    const double u2 = uxd * uxd + uyd * uyd;
    const double E_a = (K.rhoE0_d + double(drhoE)) * rcp_d(rho_d);
    const double T_d = dir ? Tw : (E_a - 0.5 * u2) * K.inv_cv_d;
    const double E_d = dir ? K.cv_d * Tw + 0.5 * u2 : E_a;
    s.drhoE = dir ? C(rho_d * E_d - K.rhoE0_d) : drhoE;
    s.dT = C(T_d - K.T0_d);
    complete_state<C>(K, eos, s, rho_d, T_d, E_d);
    return T_d;
}

// Wall node (Sec. 3.1): rho from the bounce-back-completed DFs, u prescribed,
// T prescribed (Dirichlet) or from rho E = sum g + q_e/2 (adiabatic).
template <typename C>
__device__ __forceinline__ double state_wall(const Coef<C>& K, int eos, int per_mass,
                                             C drho, C dn0, C ubx, C uby, int adiabatic, double Tw,
                                             NodeState<C>& s)
{
    s.drho = drho;
    const C rho = K.rho0 + drho;
    s.inv_rho = rcp<C>(rho);
    s.ux = ubx;
    s.uy = uby;
    s.jx = rho * ubx;
    s.jy = rho * uby;
    const C Fx = per_mass ? rho * K.fx : K.fx;
    const C Fy = per_mass ? rho * K.fy : K.fy;
    const double rho_d = K.rho0_d + double(drho);
    const double u2 = double(ubx) * double(ubx) + double(uby) * double(uby);
    double E_d, T_d;
    if (adiabatic) {
        s.drhoE = dn0 + C(0.5) * (ubx * Fx + uby * Fy);
        E_d = (K.rhoE0_d + double(s.drhoE)) * rcp_d(rho_d);
        T_d = (E_d - 0.5 * u2) * K.inv_cv_d;
    } else {
        T_d = Tw;
        E_d = K.cv_d * Tw + 0.5 * u2;
        s.drhoE = C(rho_d * E_d - K.rhoE0_d);
    }
    s.dT = C(T_d - K.T0_d);
    complete_state<C>(K, eos, s, rho_d, T_d, E_d);
    return T_d;
}

// Prescribed state (initial fields): E = C_v T + |u|^2/2.
template <typename C>
__device__ __forceinline__ double state_prescribed(const Coef<C>& K, int eos, double rho_d, double ux, double uy,
                                                   double T_d, NodeState<C>& s)
{
    s.drho = C(rho_d - K.rho0_d);
    s.inv_rho = rcp<C>(C(rho_d));
    s.ux = C(ux);
    s.uy = C(uy);
    s.jx = C(rho_d * ux);
    s.jy = C(rho_d * uy);
    s.dT = C(T_d - K.T0_d);
    const double E_d = K.cv_d * T_d + 0.5 * (ux * ux + uy * uy);
    s.drhoE = C(rho_d * E_d - K.rhoE0_d);
    complete_state<C>(K, eos, s, rho_d, T_d, E_d);
    return T_d;
}

// Local relaxation rates (Sec. 4): nu = mu(T)/rho = c_s^2 (1/s_p - 1/2);
// (1/s_p - 1/2)(1/s_q - 1/2) = 1/12; bulk = varpi c_s^2 (1/s_e - 1/2) =
// ratio * nu; lambda = C_p mu / Pr = kappa rho0 C_p (1/sigma_j - 1/2);
// (1/sigma_j - 1/2)(1/sigma_e - 1/2) = 1/4.
template <typename C>
__device__ __forceinline__ void local_rates(const Coef<C>& K, int visc_law, const NodeState<C>& s, Rates<C>& r)
{
    const C rho = rho_of(K, s), rho_inv = s.inv_rho, T = T_of(K, s);
    C mu;
    if (visc_law == VISC_CONST) {
        mu = K.mu0;
    } else if (visc_law == VISC_LINEAR) {
        mu = K.mu0 * T * K.inv_T0;
    } else {  // Sutherland, referred to (T0, mu0)
        const C th = T * K.inv_T0;
        mu = K.mu0 * th * sqrt_<C>(th) * K.suth_1pS * rcp<C>(th + K.suth_S);
    }
    const C inv_mu = rcp<C>(mu);
    const C three_nu = C(3) * mu * rho_inv;                 // nu / c_s^2
    const C tp = three_nu + C(0.5);
    const C tq = C(0.5) + C(1.0 / 36.0) * rho * inv_mu;      // 1/2 + (1/12) / (3 nu)
    const C te = C(0.5) + K.bulk_over_varpi * three_nu;     // ratio * nu / (varpi c_s^2)
    const C tj = C(0.5) + mu * K.inv_kappa_rho0_Pr;
    const C tse = C(0.5) + C(0.25) * K.kappa_rho0_Pr * inv_mu;
    r.sp = rcp<C>(tp);
    r.sq = rcp<C>(tq);
    r.se = rcp<C>(te);
    r.sigj = rcp<C>(tj);
    r.sige = rcp<C>(tse);
    r.we = C(0.5) * r.se - C(1);
    r.wp = C(0.5) * r.sp - C(1);
    // (2 - s) = (2 tau - 1) s and (tau_e - 1/2) / (tau_p - 1/2) = ratio / varpi
    r.r_ep = K.bulk_over_varpi * tp * r.se;
    r.r_pe = K.varpi_over_bulk * te * r.sp;
}

// ---------------------------------------------------------------------------
// collision pieces
// ---------------------------------------------------------------------------
// m^eq of Sec. 2.1 (with c = 1) minus its rest value
template <typename C>
__device__ __forceinline__ void meq_f(const NodeState<C>& s, C q[9])
{
    const C ux = s.ux, uy = s.uy;
    const C jx = s.jx, jy = s.jy;                  // rho u
    const C jux = jx * ux, juy = jy * uy;          // rho ux^2, rho uy^2
    const C ru2 = jux + juy;
    q[0] = s.drho;
    q[1] = C(2.0 * mc::alpha1) * s.drho + C(2.0 * mc::beta1) * s.deta + C(3) * ru2;
    q[2] = C(mc::alpha2) * s.drho + C(mc::beta2) * s.deta - C(3) * ru2 + C(9) * jux * uy * uy;
    q[3] = jx;
    q[4] = -jx + C(3) * jx * uy * uy;
    q[5] = jy;
    q[6] = -jy + C(3) * jy * ux * ux;
    q[7] = jux - juy;
    q[8] = jx * uy;
}

// F_m of Sec. 2.1; rows 0, 3, 5 are 0, F_x, F_y
template <typename C>
__device__ __forceinline__ void force_moments(const NodeState<C>& s, const Forcing<C>& F, C q[9])
{
    const C ux = s.ux, uy = s.uy, Fx = F.Fx, Fy = F.Fy;
    const C Fu = Fx * ux + Fy * uy;
    q[0] = C(0);
    q[1] = C(6) * Fu;
    q[2] = C(-6) * Fu + C(18) * ux * uy * (Fx * uy + Fy * ux);
    q[3] = Fx;
    q[4] = -Fx + C(3) * (Fx * uy * uy + C(2) * Fy * ux * uy);
    q[5] = Fy;
    q[6] = -Fy + C(3) * (C(2) * Fx * ux * uy + Fy * ux * ux);
    q[7] = C(2) * (Fx * ux - Fy * uy);
    q[8] = Fx * uy + Fy * ux;
}

// n^eq of Sec. 2.2 minus its rest value
template <typename C>
__device__ __forceinline__ void neq_g(const Coef<C>& K, const NodeState<C>& s, C q[9])
{
    const C rcdT = K.rho0_cp * s.dT;
    const C d = s.drhoE - rcdT;
    q[0] = s.drhoE;
    q[1] = C(-4) * d + C(mc::gamma1) * rcdT;
    q[2] = C(4) * d + C(mc::gamma2) * rcdT;
    q[3] = s.H * s.jx;                             // rho H u
    q[4] = -q[3];
    q[5] = s.H * s.jy;
    q[6] = -q[5];
    q[7] = C(0);
    q[8] = C(0);
}

// Q_m of Sec. 2.2
template <typename C>
__device__ __forceinline__ void source_moments(const NodeState<C>& s, const Forcing<C>& F, C q[9])
{
    const C qe = F.qe;
    q[0] = qe;
    q[1] = C(mc::gamma1) * qe;
    q[2] = C(mc::gamma2) * qe;
    q[3] = qe * s.ux;
    q[4] = -q[3];
    q[5] = qe * s.uy;
    q[6] = -q[5];
    q[7] = C(0);
    q[8] = C(0);
}

// Ntil = (I - S/2) N with the sparse S of Sec. 2.1 (rows 0, 3, 5 of N vanish)
template <typename C>
__device__ __forceinline__ void tilde_f(const NodeState<C>& s, const Rates<C>& r, const C N[9], C Nt[9])
{
    const C sq_we = r.sq * r.we, sq_wp = r.sq * r.wp;
    Nt[0] = C(0);
    Nt[3] = C(0);
    Nt[5] = C(0);
    Nt[1] = -r.we * N[1] - C(0.5 * mc::k) * r.se * r.we * N[2]
            - C(0.5 * mc::h) * sq_we * (s.ux * N[4] + s.uy * N[6]);
    Nt[2] = -r.we * N[2];
    Nt[4] = (C(1) - C(0.5) * r.sq) * N[4];
    Nt[6] = (C(1) - C(0.5) * r.sq) * N[6];
    Nt[7] = -r.wp * N[7] - C(mc::b) * sq_wp * (s.ux * N[4] - s.uy * N[6]);
    Nt[8] = -r.wp * N[8] - C(0.5 * mc::b) * sq_wp * (s.uy * N[4] + s.ux * N[6]);
}

// N = (I - S/2)^-1 Ntil by the closed form of App. B
template <typename C>
__device__ __forceinline__ void untilde_f(const NodeState<C>& s, const Rates<C>& r, const C Nt[9], C N[9])
{
    // [I - diag(S)/2]^-1 first
    const C d1 = rcp<C>(-r.we), dq = rcp<C>(C(1) - C(0.5) * r.sq), dp = rcp<C>(-r.wp);
    const C z2 = Nt[2] * d1, z4 = Nt[4] * dq, z6 = Nt[6] * dq;
    N[0] = C(0);
    N[3] = C(0);
    N[5] = C(0);
    N[2] = z2;
    N[4] = z4;
    N[6] = z6;
    N[1] = Nt[1] * d1 - C(0.5 * mc::k) * r.se * z2 - C(0.5 * mc::h) * r.sq * (s.ux * z4 + s.uy * z6);
    N[7] = Nt[7] * dp - C(mc::b) * r.sq * (s.ux * z4 - s.uy * z6);
    N[8] = Nt[8] * dp - C(0.5 * mc::b) * r.sq * (s.uy * z4 + s.ux * z6);
}

// Htil = (I - L/2) H with the modified L of Sec. 2.2 (App. C steps 2-3);
// H0 = 0 (conserved moment)
template <typename C>
__device__ __forceinline__ void tilde_g(const Rates<C>& r, const C Hm[9], C Ht[9])
{
    const C ce = C(1) - C(0.5) * r.sige, cj = C(1) - C(0.5) * r.sigj;
    Ht[0] = C(0);
    Ht[1] = ce * Hm[1];
    Ht[2] = ce * Hm[2];
    Ht[3] = cj * (Hm[3] + C(0.5) * r.sigj * Hm[4]);
    Ht[4] = cj * Hm[4];
    Ht[5] = cj * (Hm[5] + C(0.5) * r.sigj * Hm[6]);
    Ht[6] = cj * Hm[6];
    Ht[7] = ce * Hm[7];
    Ht[8] = ce * Hm[8];
}

// H = (I - L/2)^-1 Htil by the closed form of App. B
template <typename C>
__device__ __forceinline__ void untilde_g(const Rates<C>& r, const C Ht[9], C Hm[9])
{
    const C ie = rcp<C>(C(1) - C(0.5) * r.sige), ij = rcp<C>(C(1) - C(0.5) * r.sigj);
    Hm[0] = C(0);
    Hm[1] = Ht[1] * ie;
    Hm[2] = Ht[2] * ie;
    Hm[4] = Ht[4] * ij;
    Hm[6] = Ht[6] * ij;
    Hm[3] = Ht[3] * ij - C(0.5) * r.sigj * Hm[4];
    Hm[5] = Ht[5] * ij - C(0.5) * r.sigj * Hm[6];
    Hm[7] = Ht[7] * ie;
    Hm[8] = Ht[8] * ie;
}

// The three correction rows (1, 7, 8) of R Ntil + T.grad(rho) + X.grad(p)
template <typename C>
__device__ __forceinline__ void corrections(const NodeState<C>& s, const Rates<C>& r, int cubic,
                                            const C Nt[9], C gr_x, C gr_y, C gp_x, C gp_y,
                                            C& c1, C& c7, C& c8)
{
    c1 = C(0);
    c7 = C(0);
    c8 = C(0);
    if (cubic <= 0) return;
    const C ux = s.ux, uy = s.uy;
    const C ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2, dd = ux2 - uy2, xy = ux * uy;
    const C sp_ep = r.sp * r.r_ep, se_pe = r.se * r.r_pe;
    c1 = C(mc::cR11) * r.se * u2 * Nt[1] + C(mc::cR17) * sp_ep * dd * Nt[7] + C(mc::cR18) * sp_ep * xy * Nt[8];
    c7 = C(mc::cR71) * se_pe * dd * Nt[1] + C(mc::cR77) * r.sp * u2 * Nt[7];
    c8 = C(mc::cR81) * se_pe * xy * Nt[1] + C(mc::cR88) * r.sp * u2 * Nt[8];
    if (cubic <= 1) return;
    const C tse = C(2) - r.se, tsp = C(2) - r.sp;
    // T and X of Sec. 2.1
    const C t1 = C(1.5) * tse;
    const C T1x = t1 * (C(1.0 - mc::k) * ux2 * ux - C(2.0 * mc::k + mc::h) * ux * uy2);
    const C T1y = t1 * (C(1.0 - mc::k) * uy2 * uy - C(2.0 * mc::k + mc::h) * ux2 * uy);
    const C t7 = C(0.5) * tsp;
    const C T7x = t7 * (ux2 * ux + C(2.0 * mc::b) * ux * uy2);
    const C T7y = -t7 * (uy2 * uy + C(2.0 * mc::b) * ux2 * uy);
    const C v8x = uy2 * uy + C(2) * ux2 * uy, v8y = ux2 * ux + C(2) * ux * uy2;
    const C x1 = C(4.5 * (2.0 * mc::k + mc::h)) * tse;
    const C x7 = C(-3.0 * mc::b) * tsp;
    // row 8: T8 = -(b/2)(2 - s_p) v8, X8 = (3b/2)(2 - s_p) v8
    const C c8s = C(0.5 * mc::b) * tsp;
    c1 += T1x * gr_x + T1y * gr_y + x1 * (ux * uy2 * gp_x + ux2 * uy * gp_y);
    c7 += T7x * gr_x + T7y * gr_y + x7 * (ux * uy2 * gp_x - ux2 * uy * gp_y);
    c8 += c8s * (v8x * (C(3) * gp_x - gr_x) + v8y * (C(3) * gp_y - gr_y));
}

// Post-collision moments from the equilibrium/force parts and the
// non-equilibrium pair (N, Ntil), (H, Htil):
//   mbar = m^eq + F_m/2 - N + 2 Ntil - [R Ntil + T.grad rho + X.grad p]
//   nbar = n^eq + Q_m/2 - H + 2 Htil + Y [(m + mbar)/2 - m^eq]
// (eqs. LBE.u.c and LBE.T.c rearranged with m = m^eq - F_m/2 + N,
//  n = n^eq - Q_m/2 + H, App. C)
template <typename C>
__device__ __forceinline__ void post_collision(const NodeState<C>& s, const Rates<C>& r, int cubic,
                                               const C meq[9], const C Fm[9], const C N[9], const C Nt[9],
                                               const C neq[9], const C Qm[9], const C Hm[9], const C Ht[9],
                                               C gr_x, C gr_y, C gp_x, C gp_y, C mb[9], C nb[9])
{
    C c1, c7, c8;
    corrections<C>(s, r, cubic, Nt, gr_x, gr_y, gp_x, gp_y, c1, c7, c8);
#pragma unroll
    for (int i = 0; i < 9; ++i) mb[i] = meq[i] + C(0.5) * Fm[i] - N[i] + C(2) * Nt[i];
    mb[1] -= c1;
    mb[7] -= c7;
    mb[8] -= c8;
    // (m + mbar)/2 - m^eq on rows 1, 7, 8 equals Ntil - c/2
    const C G1 = Nt[1] - C(0.5) * c1, G7 = Nt[7] - C(0.5) * c7, G8 = Nt[8] - C(0.5) * c8;
    // Y of eq. Y.nonzero, rows 4 and 6 the negatives of rows 3 and 5
    const C y3 = s.ux * (C(1.0 / 3.0) * G1 + G7) + C(2) * s.uy * G8;
    const C y5 = s.uy * (C(1.0 / 3.0) * G1 - G7) + C(2) * s.ux * G8;
#pragma unroll
    for (int i = 0; i < 9; ++i) nb[i] = neq[i] + C(0.5) * Qm[i] - Hm[i] + C(2) * Ht[i];
    nb[3] += y3;
    nb[4] -= y3;
    nb[5] += y5;
    nb[6] -= y5;
}

// Non-equilibrium parts of an off-wall node from its moments:
//   N = m - m^eq + F_m/2, H = n - n^eq + Q_m/2 (rows 0, 3, 5 of N and row 0
//   of H vanish identically) and their tilde forms (eq. neq.redefinition
//   without the Y part).
template <typename C>
__device__ __forceinline__ void nonequilibrium(const NodeState<C>& s, const Rates<C>& r,
                                               const C m[9], const C n[9],
                                               const C meq[9], const C Fm[9], const C neq[9], const C Qm[9],
                                               C N[9], C Nt[9], C Hm[9], C Ht[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        N[i] = m[i] - meq[i] + C(0.5) * Fm[i];
        Hm[i] = n[i] - neq[i] + C(0.5) * Qm[i];
    }
    N[0] = C(0);
    N[3] = C(0);
    N[5] = C(0);
    Hm[0] = C(0);
    tilde_f<C>(s, r, N, Nt);
    tilde_g<C>(r, Hm, Ht);
}

// ---------------------------------------------------------------------------
// storage codecs of the DF deviations: FP64, FP32, FP16 (FP32 arithmetic)
// ---------------------------------------------------------------------------
template <typename S> struct Store;

// Buffer resources for the streaming rows: a raw (stride 0) resource over
// one stored row block.  Accesses whose offset lies beyond the record count
// return zero (loads) or are dropped (stores) by the hardware range check,
// which the interior march uses to switch off the stores of its halo lanes
// without a branch.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit data format, gfx9 CDNA
constexpr int kDropOffset = int(0x80000000u);
// Cache policy of the DF stores: non-temporal.  A post-collision row is read
// again only in the next step, after the whole lattice has streamed through
// the L2, so its lines are marked for early eviction and leave the L2 to the
// source lines that neighbouring strips and segments read shortly after.
constexpr int kStorePolicy = 2;

// A pointer known to be the same in every lane, moved to scalar registers.
template <typename T> __device__ __forceinline__ T* uniform_ptr(T* p)
{
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(v));
    const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(v >> 32));
    return reinterpret_cast<T*>((static_cast<unsigned long long>(hi) << 32) | lo);
}

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(bytes), kRsrcWord3);
}

template <> struct Store<double> {
    using C = double;
    static __device__ __forceinline__ void store_sr(double* p, double v, unsigned) { store(p, v); }
    static __device__ __forceinline__ void bstore_sr(rsrc_t r, int vo, int so, double v, unsigned) { bstore(r, vo, so, v); }
    static __device__ __forceinline__ double load(const double* p) { return *p; }
    static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
    static __device__ __forceinline__ double bload(rsrc_t r, int vo, int so)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    static __device__ __forceinline__ void bstore(rsrc_t r, int vo, int so, double v)
    {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, vo, so, kStorePolicy);
    }
};
template <> struct Store<float> {
    using C = float;
    static __device__ __forceinline__ void store_sr(float* p, float v, unsigned) { store(p, v); }
    static __device__ __forceinline__ void bstore_sr(rsrc_t r, int vo, int so, float v, unsigned) { bstore(r, vo, so, v); }
    static __device__ __forceinline__ float load(const float* p) { return *p; }
    static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
    static __device__ __forceinline__ float bload(rsrc_t r, int vo, int so)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ void bstore(rsrc_t r, int vo, int so, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, kStorePolicy);
    }
};
template <> struct Store<__half> {
    using C = float;
    // stochastic rounding with the random operand rnd (v_cvt_sr_f16_f32; lbm_rounding.hpp)
    static __device__ __forceinline__ unsigned short sr_bits(float v, unsigned rnd)
    {
        typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
        // the instruction writes the low half of its destination and keeps
        // the high half, which nothing reads: passing v's own bits as the kept
        // half lets the result take v's register without clearing one first
        const half2_t old = __builtin_bit_cast(half2_t, v);
        const half2_t h = __builtin_amdgcn_cvt_sr_f16_f32(old, v, rnd, false);
        return __builtin_bit_cast(unsigned short, h[0]);
    }
    static __device__ __forceinline__ void store_sr(__half* p, float v, unsigned rnd)
    {
        *reinterpret_cast<unsigned short*>(p) = sr_bits(v, rnd);
    }
    static __device__ __forceinline__ void bstore_sr(rsrc_t r, int vo, int so, float v, unsigned rnd)
    {
        __builtin_amdgcn_raw_buffer_store_b16(sr_bits(v, rnd), r, vo, so, kStorePolicy);
    }
    static __device__ __forceinline__ float load(const __half* p)
    {
        const unsigned short b = *reinterpret_cast<const unsigned short*>(p);
        return __half2float(__ushort_as_half(b));
    }
    static __device__ __forceinline__ void store(__half* p, float v)
    {
        *reinterpret_cast<unsigned short*>(p) = __half_as_ushort(__float2half_rn(v));
    }
    static __device__ __forceinline__ float bload(rsrc_t r, int vo, int so)
    {
        const unsigned short b = __builtin_bit_cast(unsigned short, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
        return __half2float(__ushort_as_half(b));
    }
    static __device__ __forceinline__ void bstore(rsrc_t r, int vo, int so, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, vo, so, kStorePolicy);
    }
};

}  // namespace lbm
