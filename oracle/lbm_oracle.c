/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).
 *
 * Plain FP64 reference of the coupled D2Q9 MRT scheme of Huang, Wu & Adams
 * (arXiv:1809.08683).  Written for checkability, not speed:
 *   - every matrix of Sec. 2 (M, S, R, T, X, L, Y) is built as a dense array
 *     from its printed definition and applied by dense products;
 *   - the collisions are the matrix forms eq. LBE.u.c and eq. LBE.T.c;
 *   - M^-1, (I - S/2)^-1 and (I - L/2)^-1 come from Gaussian elimination,
 *     not from the closed forms of App. B;
 *   - the wall treatment of Sec. 3 runs in the paper's order: bounce-back
 *     temporaries -> wall macros -> tilde non-equilibrium parts at x_f, x_ff
 *     -> extrapolation -> inversion -> rebuild of all 18 DFs.
 *
 * Readings where the paper is silent (the same readings the HIP library
 * uses):
 *   - gradients in T.grad(rho) and X.grad(p): isotropic 9-point central
 *     difference at nodes off the walls; at wall nodes a second-order
 *     one-sided difference along a walled axis and a two-point central
 *     difference along an open axis; same time level as the collision
 *     (no printed value fixes the stencil; the tests pin its exactness on
 *     quadratics at every kind of node);
 *   - p inside X.grad(p) is p_EOS(rho, T);
 *   - corner nodes: bounce-back temporaries for every unknown DF, velocity
 *     and Dirichlet temperature of the x-wall (else of the y-wall),
 *     extrapolation along the inward diagonal (the paper is silent; the
 *     tests pin exact steady conduction and conservation at corners);
 *   - the start state (t = 0) is m = m^eq - F_m/2, n = n^eq - Q_m/2 at every
 *     node, walls included; wall velocity/temperature apply from t = 1;
 *   - T = (E - |u|^2/2) / C_v for every equation of state (Sec. 2.2);
 *   - local rates: 1/s_p = mu(T)/(rho c_s^2) + 1/2 with the local rho, and
 *     1/sigma_j = 1/2 + lambda(T)/(kappa rho0 C_p) with lambda = C_p mu/Pr;
 *   - mean Nusselt number: trapezoid rule along the wall of
 *     lambda(T_b) (-dT/dn) / (lambda0 (T_lo - T_hi)), with the second-order
 *     one-sided difference (-3 T0 + 4 T1 - T2) / 2 (the tests pin Nu = 1
 *     for pure conduction and second-order convergence to the Kirchhoff
 *     value with a temperature-dependent conductivity).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so
 * results do not depend on the compiler's fusion choices).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* The node loops of a step are independent per node (every node reads the
 * previous arrays and writes only its own entries), so running them on
 * several OpenMP threads gives bitwise the serial result. */
#define ORC_PARALLEL_ROWS _Pragma("omp parallel for schedule(static) num_threads(o->threads) if(o->threads > 1)")

struct orc {
    orc_params P;
    orc_derived D;
    int ex[9], ey[9], opp[9];
    double w[9];
    double M[81], Minv[81];
    double *f, *g;             /* pre-collision DFs at t, [node][9] */
    double *fs, *gs;           /* post-collision scratch */
    double *rho, *ux, *uy, *T, *rhoE, *p;  /* macros at t */
    long long t;
    int ready;
    int threads;               /* OpenMP threads of the node loops (1: serial) */
    char err[256];
};

/* ------------------------------------------------------------------ */
/* small dense linear algebra                                          */
/* ------------------------------------------------------------------ */

static void matvec9(const double* A, const double* x, double* y)
{
    for (int i = 0; i < 9; ++i) {
        double s = 0.0;
        for (int j = 0; j < 9; ++j) s += A[i * 9 + j] * x[j];
        y[i] = s;
    }
}

/* y = A x for a 9x2 matrix A (row-major) and a 2-vector x */
static void matvec92(const double* A, const double* x, double* y)
{
    for (int i = 0; i < 9; ++i) y[i] = A[i * 2 + 0] * x[0] + A[i * 2 + 1] * x[1];
}

/* Solve A x = b (9x9) by Gaussian elimination with partial pivoting. */
static int solve9(const double* A_in, const double* b_in, double* x)
{
    double A[81], b[9];
    memcpy(A, A_in, sizeof A);
    memcpy(b, b_in, sizeof b);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(A[r * 9 + c]) > fabs(A[piv * 9 + c])) piv = r;
        if (A[piv * 9 + c] == 0.0) return -1;
        if (piv != c) {
            for (int j = 0; j < 9; ++j) {
                double tmp = A[c * 9 + j]; A[c * 9 + j] = A[piv * 9 + j]; A[piv * 9 + j] = tmp;
            }
            double tmp = b[c]; b[c] = b[piv]; b[piv] = tmp;
        }
        for (int r = c + 1; r < 9; ++r) {
            double fct = A[r * 9 + c] / A[c * 9 + c];
            if (fct == 0.0) continue;
            for (int j = c; j < 9; ++j) A[r * 9 + j] -= fct * A[c * 9 + j];
            b[r] -= fct * b[c];
        }
    }
    for (int r = 8; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < 9; ++j) s -= A[r * 9 + j] * x[j];
        x[r] = s / A[r * 9 + r];
    }
    return 0;
}

/* Inverse by solving A X = I column by column. */
static int invert9(const double* A, double* Ainv)
{
    for (int c = 0; c < 9; ++c) {
        double e[9] = {0}, col[9];
        e[c] = 1.0;
        if (solve9(A, e, col)) return -1;
        for (int r = 0; r < 9; ++r) Ainv[r * 9 + c] = col[r];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* lattice (Sec. 2, the D2Q9 velocity set) and moment matrix (eq. M)   */
/* ------------------------------------------------------------------ */

void orc_lattice(int ex[9], int ey[9], double w[9])
{
    const double pi = acos(-1.0);
    ex[0] = 0; ey[0] = 0;
    for (int i = 1; i <= 4; ++i) {        /* c (cos, sin)[(i-1) pi/2] */
        ex[i] = (int)lround(cos((i - 1) * pi / 2.0));
        ey[i] = (int)lround(sin((i - 1) * pi / 2.0));
    }
    for (int i = 5; i <= 8; ++i) {        /* sqrt(2) c (cos, sin)[(2i-1) pi/4] */
        ex[i] = (int)lround(sqrt(2.0) * cos((2 * i - 1) * pi / 4.0));
        ey[i] = (int)lround(sqrt(2.0) * sin((2 * i - 1) * pi / 4.0));
    }
    /* standard D2Q9 weights, used only by the isotropic gradient stencil */
    for (int i = 0; i < 9; ++i) {
        int e2 = ex[i] * ex[i] + ey[i] * ey[i];
        w[i] = (e2 == 0) ? 4.0 / 9.0 : (e2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
}

/* The transformation matrix as printed in Sec. 2.1 (eq. M). */
static const double M_PAPER[81] = {
     1,  1,  1,  1,  1,  1,  1,  1,  1,
    -4, -1, -1, -1, -1,  2,  2,  2,  2,
     4, -2, -2, -2, -2,  1,  1,  1,  1,
     0,  1,  0, -1,  0,  1, -1, -1,  1,
     0, -2,  0,  2,  0,  1, -1, -1,  1,
     0,  0,  1,  0, -1,  1,  1, -1, -1,
     0,  0, -2,  0,  2,  1,  1, -1, -1,
     0,  1, -1,  1, -1,  0,  0,  0,  0,
     0,  0,  0,  0,  0,  1, -1,  1, -1,
};

void orc_moment_matrix(double M[81], double Minv[81])
{
    if (M) memcpy(M, M_PAPER, sizeof M_PAPER);
    if (Minv) invert9(M_PAPER, Minv);
}

/* ------------------------------------------------------------------ */
/* closures (Sec. 4)                                                   */
/* ------------------------------------------------------------------ */

static double cs_b(const orc* o)
{
    /* Carnahan-Starling b = sqrt(2) pi / (3 rho0) unless given */
    return o->P.b > 0 ? o->P.b : sqrt(2.0) * acos(-1.0) / (3.0 * o->P.rho0);
}

/* compressibility factor Z of eq. EOSs.3 */
static double cs_Z(double beta)
{
    return (1.0 + beta + beta * beta - beta * beta * beta) / pow(1.0 - beta, 3.0);
}

static double eos_p(const orc* o, double R, double rho, double T)
{
    switch (o->P.eos) {
    case ORC_EOS_DECOUPLED: return rho * R * o->P.T0;
    case ORC_EOS_IDEAL:     return rho * R * T;
    case ORC_EOS_VDW:       return rho * R * T / (1.0 - o->P.b * rho) - o->P.a * rho * rho;
    case ORC_EOS_CS:        return cs_Z(cs_b(o) * rho / 4.0) * rho * R * T;
    }
    return NAN;
}

double orc_pressure(const orc* o, double rho, double T) { return eos_p(o, o->D.R, rho, T); }

/* R such that dp/drho at (rho0, T0) equals c_s^2 (eq. cs) */
static double derive_R(const orc* o, double cs2)
{
    const double rho0 = o->P.rho0, T0 = o->P.T0;
    switch (o->P.eos) {
    case ORC_EOS_DECOUPLED:
    case ORC_EOS_IDEAL:
        return cs2 / T0;
    case ORC_EOS_VDW: {
        /* dp/drho = R T / (1 - b rho)^2 - 2 a rho */
        double omb = 1.0 - o->P.b * rho0;
        return (cs2 + 2.0 * o->P.a * rho0) * omb * omb / T0;
    }
    case ORC_EOS_CS: {
        /* d(Z rho)/drho = Z + beta dZ/dbeta, dZ/dbeta = (4 + 4 beta - 2 beta^2)/(1 - beta)^4 */
        double beta = cs_b(o) * rho0 / 4.0;
        double dZ = (4.0 + 4.0 * beta - 2.0 * beta * beta) / pow(1.0 - beta, 4.0);
        return cs2 / (T0 * (cs_Z(beta) + beta * dZ));
    }
    }
    return NAN;
}

static double viscosity(const orc* o, double T)
{
    double th = T / o->P.T0;
    switch (o->P.visc_law) {
    case ORC_VISC_CONST:  return o->D.mu0;
    case ORC_VISC_LINEAR: return o->D.mu0 * th;
    case ORC_VISC_SUTHERLAND:
        /* Sec. 4.3 Sutherland law referred to (T0, mu0) */
        return o->D.mu0 * pow(th, 1.5) * (1.0 + o->P.suth_S) / (th + o->P.suth_S);
    }
    return NAN;
}

void orc_rates(const orc* o, double rho, double T, double r[10])
{
    const orc_derived* D = &o->D;
    double mu = viscosity(o, T);
    double nu = mu / rho;
    /* nu = c_s^2 (1/s_p - 1/2)  (eq. NSE) */
    double tp = nu / D->cs2 + 0.5;
    /* (1/s_p - 1/2)(1/s_q - 1/2) = 1/12 (Sec. 4) */
    double tq = 0.5 + (1.0 / 12.0) / (tp - 0.5);
    /* bulk viscosity = varpi c_s^2 (1/s_e - 1/2) (eq. NSE) */
    double te = 0.5 + o->P.bulk_ratio * nu / (D->varpi * D->cs2);
    /* lambda = kappa rho0 C_p c^2 (1/sigma_j - 1/2), lambda = C_p mu / Pr */
    double lambda = D->cp * mu / o->P.Pr;
    double tj = 0.5 + lambda / (D->kappa * o->P.rho0 * D->cp);
    /* (1/sigma_j - 1/2)(1/sigma_e - 1/2) = 1/4 (Sec. 4) */
    double tse = 0.5 + 0.25 / (tj - 0.5);
    r[0] = 1.0;            /* s0 */
    r[1] = 1.0 / te;       /* s_e */
    r[2] = 1.0 / te;       /* s_eps = s_e */
    r[3] = 1.0;            /* s_j */
    r[4] = 1.0 / tq;       /* s_q */
    r[5] = 1.0 / tp;       /* s_p */
    r[6] = 1.0;            /* sigma_0 */
    r[7] = 1.0 / tse;      /* sigma_e (= sigma_eps = sigma_p) */
    r[8] = 1.0 / tj;       /* sigma_j */
    r[9] = 1.0 / tj;       /* sigma_q = sigma_j */
}

/* ------------------------------------------------------------------ */
/* equilibria and source moments (Sec. 2.1, Sec. 2.2)                  */
/* ------------------------------------------------------------------ */

void orc_meq(const orc* o, double rho, double ux, double uy, double eta, double m[9])
{
    const orc_derived* D = &o->D;
    double u2 = ux * ux + uy * uy;
    m[0] = rho;
    m[1] = 2.0 * D->alpha1 * rho + 2.0 * D->beta1 * eta + 3.0 * rho * u2;
    m[2] = D->alpha2 * rho + D->beta2 * eta - 3.0 * rho * u2 + 9.0 * rho * ux * ux * uy * uy;
    m[3] = rho * ux;
    m[4] = -rho * ux + 3.0 * rho * ux * uy * uy;
    m[5] = rho * uy;
    m[6] = -rho * uy + 3.0 * rho * uy * ux * ux;
    m[7] = rho * (ux * ux - uy * uy);
    m[8] = rho * ux * uy;
}

void orc_fm(const orc* o, double Fx, double Fy, double ux, double uy, double m[9])
{
    (void)o;
    double Fu = Fx * ux + Fy * uy;
    /* bracket terms: the force takes each tensor slot in turn */
    double Fuuu_xxyy = 2.0 * Fx * ux * uy * uy + 2.0 * Fy * uy * ux * ux;
    double Fuu_xyy = Fx * uy * uy + 2.0 * Fy * ux * uy;
    double Fuu_xxy = 2.0 * Fx * ux * uy + Fy * ux * ux;
    m[0] = 0.0;
    m[1] = 6.0 * Fu;
    m[2] = -6.0 * Fu + 9.0 * Fuuu_xxyy;
    m[3] = Fx;
    m[4] = -Fx + 3.0 * Fuu_xyy;
    m[5] = Fy;
    m[6] = -Fy + 3.0 * Fuu_xxy;
    m[7] = 2.0 * (Fx * ux - Fy * uy);
    m[8] = Fx * uy + Fy * ux;
}

void orc_neq(const orc* o, double rho, double rhoE, double ux, double uy,
             double H, double T, double n[9])
{
    const orc_derived* D = &o->D;
    double rcT = o->P.rho0 * D->cp * T;
    n[0] = rhoE;
    n[1] = -4.0 * (rhoE - rcT) + D->gamma1 * rcT;
    n[2] = 4.0 * (rhoE - rcT) + D->gamma2 * rcT;
    n[3] = rho * H * ux;
    n[4] = -rho * H * ux;
    n[5] = rho * H * uy;
    n[6] = -rho * H * uy;
    n[7] = 0.0;
    n[8] = 0.0;
}

void orc_qm(const orc* o, double qe, double ux, double uy, double q[9])
{
    const orc_derived* D = &o->D;
    q[0] = qe;
    q[1] = D->gamma1 * qe;
    q[2] = D->gamma2 * qe;
    q[3] = qe * ux;
    q[4] = -qe * ux;
    q[5] = qe * uy;
    q[6] = -qe * uy;
    q[7] = 0.0;
    q[8] = 0.0;
}

/* ------------------------------------------------------------------ */
/* collision matrices (Sec. 2.1: S, R, T, X; Sec. 2.2: L, Y)           */
/* ------------------------------------------------------------------ */

void orc_matrices(const orc* o, double rho, double ux, double uy, double Tt,
                  double S[81], double R[81], double Tm[18], double X[18],
                  double L[81], double Y[81])
{
    const orc_derived* D = &o->D;
    double r[10];
    orc_rates(o, rho, Tt, r);
    const double s0 = r[0], se = r[1], seps = r[2], sj = r[3], sq = r[4], sp = r[5];
    const double sig0 = r[6], sige = r[7], sigj = r[8], sigq = r[9];
    const double sigeps = sige, sigp = sige;
    const double k = D->k, h = D->h, b = D->b, vp = D->varpi;
    const double we = se / 2.0 - 1.0, wp = sp / 2.0 - 1.0, wj = sigj / 2.0 - 1.0;

    if (S) {
        memset(S, 0, 81 * sizeof(double));
        S[0 * 9 + 0] = s0;
        S[1 * 9 + 1] = se;
        S[1 * 9 + 2] = k * seps * we;
        S[1 * 9 + 4] = h * ux * sq * we;
        S[1 * 9 + 6] = h * uy * sq * we;
        S[2 * 9 + 2] = seps;
        S[3 * 9 + 3] = sj;
        S[4 * 9 + 4] = sq;
        S[5 * 9 + 5] = sj;
        S[6 * 9 + 6] = sq;
        S[7 * 9 + 4] = 2.0 * b * ux * sq * wp;
        S[7 * 9 + 6] = -2.0 * b * uy * sq * wp;
        S[7 * 9 + 7] = sp;
        S[8 * 9 + 4] = b * uy * sq * wp;
        S[8 * 9 + 6] = b * ux * sq * wp;
        S[8 * 9 + 8] = sp;
    }
    if (R) {
        memset(R, 0, 81 * sizeof(double));
        if (o->P.cubic >= 1) {
            double ss = ux * ux + uy * uy, dd = ux * ux - uy * uy, xy = ux * uy;
            R[1 * 9 + 1] = -(9.0 - 15.0 * k - 2.0 * h) * se / (4.0 * vp) * ss;
            R[1 * 9 + 7] = -3.0 * (9.0 - 3.0 * k + 2.0 * h) * sp * (2.0 - se) / (4.0 * (2.0 - sp)) * dd;
            R[1 * 9 + 8] = 12.0 * (3.0 * k + h) * sp * (2.0 - se) / (2.0 - sp) * xy;
            R[7 * 9 + 1] = -(3.0 - 4.0 * b) * se * (2.0 - sp) / (4.0 * vp * (2.0 - se)) * dd;
            R[7 * 9 + 7] = -3.0 * (3.0 + 4.0 * b) * sp / 4.0 * ss;
            R[7 * 9 + 8] = 0.0;
            R[8 * 9 + 1] = b * se * (2.0 - sp) / (vp * (2.0 - se)) * xy;
            R[8 * 9 + 7] = 0.0;
            R[8 * 9 + 8] = 6.0 * b * sp * ss;
        }
    }
    if (Tm) {
        memset(Tm, 0, 18 * sizeof(double));
        if (o->P.cubic >= 2) {
            double c1 = 3.0 * (2.0 - se) / 2.0, c7 = (2.0 - sp) / 2.0, c8 = -b * (2.0 - sp) / 2.0;
            Tm[1 * 2 + 0] = c1 * ((1.0 - k) * ux * ux * ux - (2.0 * k + h) * ux * uy * uy);
            Tm[1 * 2 + 1] = c1 * ((1.0 - k) * uy * uy * uy - (2.0 * k + h) * ux * ux * uy);
            Tm[7 * 2 + 0] = c7 * (ux * ux * ux + 2.0 * b * ux * uy * uy);
            Tm[7 * 2 + 1] = c7 * (-uy * uy * uy - 2.0 * b * ux * ux * uy);
            Tm[8 * 2 + 0] = c8 * (uy * uy * uy + 2.0 * ux * ux * uy);
            Tm[8 * 2 + 1] = c8 * (ux * ux * ux + 2.0 * ux * uy * uy);
        }
    }
    if (X) {
        memset(X, 0, 18 * sizeof(double));
        if (o->P.cubic >= 2) {
            double c1 = 9.0 * (2.0 * k + h) * (2.0 - se) / 2.0;
            double c7 = -3.0 * b * (2.0 - sp), c8 = 3.0 * b * (2.0 - sp) / 2.0;
            X[1 * 2 + 0] = c1 * ux * uy * uy;
            X[1 * 2 + 1] = c1 * ux * ux * uy;
            X[7 * 2 + 0] = c7 * ux * uy * uy;
            X[7 * 2 + 1] = c7 * (-ux * ux * uy);
            X[8 * 2 + 0] = c8 * (uy * uy * uy + 2.0 * ux * ux * uy);
            X[8 * 2 + 1] = c8 * (ux * ux * ux + 2.0 * ux * uy * uy);
        }
    }
    if (L) {
        memset(L, 0, 81 * sizeof(double));
        L[0 * 9 + 0] = sig0;
        L[1 * 9 + 1] = sige;
        L[2 * 9 + 2] = sigeps;
        L[3 * 9 + 3] = sigj;
        L[3 * 9 + 4] = sigq * wj;
        L[4 * 9 + 4] = sigq;
        L[5 * 9 + 5] = sigj;
        L[5 * 9 + 6] = sigq * wj;
        L[6 * 9 + 6] = sigq;
        L[7 * 9 + 7] = sigp;
        L[8 * 9 + 8] = sigp;
    }
    if (Y) {
        memset(Y, 0, 81 * sizeof(double));
        /* eq. Y.nonzero, with Y_4a = -Y_3a and Y_6a = -Y_5a */
        Y[3 * 9 + 1] = ux / 3.0;
        Y[3 * 9 + 7] = ux;
        Y[3 * 9 + 8] = 2.0 * uy;
        Y[5 * 9 + 1] = uy / 3.0;
        Y[5 * 9 + 7] = -uy;
        Y[5 * 9 + 8] = 2.0 * ux;
        for (int a = 0; a < 9; ++a) {
            Y[4 * 9 + a] = -Y[3 * 9 + a];
            Y[6 * 9 + a] = -Y[5 * 9 + a];
        }
    }
}

/* ------------------------------------------------------------------ */
/* node state                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    double rho, ux, uy, T, rhoE;   /* primary */
    double Fx, Fy, qe, p, eta, E, H;
} nstate;

static void force_at(const orc* o, double rho, double* Fx, double* Fy)
{
    if (o->P.per_mass) { *Fx = rho * o->P.fx; *Fy = rho * o->P.fy; }
    else { *Fx = o->P.fx; *Fy = o->P.fy; }
}

/* complete a node state from rho, u, T and rho*E */
static void complete_state(const orc* o, nstate* s)
{
    const orc_derived* D = &o->D;
    force_at(o, s->rho, &s->Fx, &s->Fy);
    s->qe = s->ux * s->Fx + s->uy * s->Fy;
    s->p = eos_p(o, D->R, s->rho, s->T);
    /* eta from p_LBE = p_EOS: eta = [p/c_s^2 - (2 + alpha1) rho] / beta1 */
    s->eta = (s->p / D->cs2 - (2.0 + D->alpha1) * s->rho) / D->beta1;
    s->E = s->rhoE / s->rho;
    s->H = s->E + s->p / s->rho;
}

/* macros of a node from its DFs (eqs. rho.u and E) */
static void state_from_df(const orc* o, const double* f, const double* g, nstate* s)
{
    double rho = 0, jx = 0, jy = 0, sg = 0;
    for (int q = 0; q < 9; ++q) {
        rho += f[q];
        jx += o->ex[q] * f[q];
        jy += o->ey[q] * f[q];
        sg += g[q];
    }
    double Fx, Fy;
    force_at(o, rho, &Fx, &Fy);
    s->rho = rho;
    s->ux = (jx + 0.5 * Fx) / rho;
    s->uy = (jy + 0.5 * Fy) / rho;
    double qe = s->ux * Fx + s->uy * Fy;
    s->rhoE = sg + 0.5 * qe;
    double E = s->rhoE / rho;
    double eps = E - 0.5 * (s->ux * s->ux + s->uy * s->uy);
    s->T = eps / o->D.cv;
    complete_state(o, s);
}

/* node state from prescribed rho, u, T (E = C_v T + |u|^2/2) */
static void state_from_macros(const orc* o, double rho, double ux, double uy, double T, nstate* s)
{
    s->rho = rho; s->ux = ux; s->uy = uy; s->T = T;
    s->rhoE = rho * (o->D.cv * T + 0.5 * (ux * ux + uy * uy));
    complete_state(o, s);
}

static void state_stored(const orc* o, int i, nstate* s)
{
    s->rho = o->rho[i]; s->ux = o->ux[i]; s->uy = o->uy[i];
    s->T = o->T[i]; s->rhoE = o->rhoE[i];
    complete_state(o, s);
}

static void store_state(orc* o, int i, const nstate* s)
{
    o->rho[i] = s->rho; o->ux[i] = s->ux; o->uy[i] = s->uy;
    o->T[i] = s->T; o->rhoE[i] = s->rhoE; o->p[i] = s->p;
}

/* ------------------------------------------------------------------ */
/* collision (eq. LBE.u.c and eq. LBE.T.c, matrix form)                */
/* ------------------------------------------------------------------ */

static void collide(const orc* o, const double* f, const double* g, const nstate* s,
                    const double grad[4], double* fbar, double* gbar,
                    double* m_out, double* mb_out, double* n_out, double* nb_out)
{
    double S[81], R[81], Tm[18], X[18], L[81], Y[81];
    orc_matrices(o, s->rho, s->ux, s->uy, s->T, S, R, Tm, X, L, Y);

    double m[9], meq[9], Fm[9], N[9], SN[9], IS[81], ISN[9], RISN[9], Tg[9], Xg[9], mb[9];
    matvec9(o->M, f, m);
    orc_meq(o, s->rho, s->ux, s->uy, s->eta, meq);
    orc_fm(o, s->Fx, s->Fy, s->ux, s->uy, Fm);
    for (int i = 0; i < 9; ++i) N[i] = m[i] - meq[i] + 0.5 * Fm[i];
    matvec9(S, N, SN);
    for (int i = 0; i < 81; ++i) IS[i] = ((i % 10) == 0 ? 1.0 : 0.0) - 0.5 * S[i];
    matvec9(IS, N, ISN);
    matvec9(R, ISN, RISN);
    matvec92(Tm, grad + 0, Tg);
    matvec92(X, grad + 2, Xg);
    for (int i = 0; i < 9; ++i)
        mb[i] = m[i] + Fm[i] - SN[i] - RISN[i] - Tg[i] - Xg[i];

    double n[9], neq[9], Qm[9], Hn[9], LH[9], G[9], YG[9], nb[9];
    matvec9(o->M, g, n);
    orc_neq(o, s->rho, s->rhoE, s->ux, s->uy, s->H, s->T, neq);
    orc_qm(o, s->qe, s->ux, s->uy, Qm);
    for (int i = 0; i < 9; ++i) Hn[i] = n[i] - neq[i] + 0.5 * Qm[i];
    matvec9(L, Hn, LH);
    for (int i = 0; i < 9; ++i) G[i] = 0.5 * (m[i] + mb[i]) - meq[i];
    matvec9(Y, G, YG);
    for (int i = 0; i < 9; ++i) nb[i] = n[i] + Qm[i] - LH[i] + YG[i];

    matvec9(o->Minv, mb, fbar);
    matvec9(o->Minv, nb, gbar);
    if (m_out) memcpy(m_out, m, sizeof m);
    if (mb_out) memcpy(mb_out, mb, sizeof mb);
    if (n_out) memcpy(n_out, n, sizeof n);
    if (nb_out) memcpy(nb_out, nb, sizeof nb);
}

void orc_collide_node(const orc* o, const double f[9], const double g[9],
                      const double grad[4], double fbar[9], double gbar[9],
                      double m[9], double mbar[9], double n[9], double nbar[9])
{
    nstate s;
    state_from_df(o, f, g, &s);
    collide(o, f, g, &s, grad, fbar, gbar, m, mbar, n, nbar);
}

/* ------------------------------------------------------------------ */
/* geometry helpers                                                    */
/* ------------------------------------------------------------------ */

static int on_side(const orc* o, int x, int y, int side)
{
    if (!o->P.side_wall[side]) return 0;
    switch (side) {
    case 0: return x == 0;
    case 1: return x == o->P.nx - 1;
    case 2: return y == 0;
    case 3: return y == o->P.ny - 1;
    }
    return 0;
}

static int is_wall(const orc* o, int x, int y)
{
    return on_side(o, x, y, 0) || on_side(o, x, y, 1) || on_side(o, x, y, 2) || on_side(o, x, y, 3);
}

/* wrap a coordinate on a periodic axis; returns -1 if outside a walled axis */
static int wrap_x(const orc* o, int x)
{
    int nx = o->P.nx;
    if (x >= 0 && x < nx) return x;
    if (o->P.side_wall[0]) return -1;
    return ((x % nx) + nx) % nx;
}

static int wrap_y(const orc* o, int y)
{
    int ny = o->P.ny;
    if (y >= 0 && y < ny) return y;
    if (o->P.side_wall[2]) return -1;
    return ((y % ny) + ny) % ny;
}

/* wall velocity and thermal condition at a wall node (x-wall owns corners,
 * except that a Dirichlet y-wall sets T where the x-wall is adiabatic) */
static void wall_spec(const orc* o, int x, int y, double* ux, double* uy, int* adiabatic, double* Tw)
{
    int sx = on_side(o, x, y, 0) ? 0 : (on_side(o, x, y, 1) ? 1 : -1);
    int sy = on_side(o, x, y, 2) ? 2 : (on_side(o, x, y, 3) ? 3 : -1);
    int sv = (sx >= 0) ? sx : sy;
    *ux = o->P.side_ux[sv];
    *uy = o->P.side_uy[sv];
    if (sx >= 0 && !o->P.side_adiabatic[sx]) { *adiabatic = 0; *Tw = o->P.side_T[sx]; return; }
    if (sy >= 0 && !o->P.side_adiabatic[sy]) { *adiabatic = 0; *Tw = o->P.side_T[sy]; return; }
    *adiabatic = 1;
    *Tw = 0.0;
}

/* ------------------------------------------------------------------ */
/* gradients of rho and p at time t                                    */
/* ------------------------------------------------------------------ */

static double field_at(const orc* o, const double* phi, int x, int y)
{
    int xx = wrap_x(o, x), yy = wrap_y(o, y);
    return phi[yy * o->P.nx + xx];
}

/* derivative along one axis (ax = 0: x, 1: y) at a wall node */
static double wall_axis_derivative(const orc* o, const double* phi, int x, int y, int ax)
{
    int lo_side = ax == 0 ? 0 : 2, hi_side = ax == 0 ? 1 : 3;
    int dx = ax == 0 ? 1 : 0, dy = ax == 0 ? 0 : 1;
    if (on_side(o, x, y, lo_side)) {   /* inward direction +axis */
        return (-3.0 * field_at(o, phi, x, y) + 4.0 * field_at(o, phi, x + dx, y + dy)
                - field_at(o, phi, x + 2 * dx, y + 2 * dy)) / 2.0;
    }
    if (on_side(o, x, y, hi_side)) {   /* inward direction -axis */
        return (3.0 * field_at(o, phi, x, y) - 4.0 * field_at(o, phi, x - dx, y - dy)
                + field_at(o, phi, x - 2 * dx, y - 2 * dy)) / 2.0;
    }
    return (field_at(o, phi, x + dx, y + dy) - field_at(o, phi, x - dx, y - dy)) / 2.0;
}

static void gradient(const orc* o, const double* phi, int x, int y, double* gx, double* gy)
{
    if (!is_wall(o, x, y)) {
        /* isotropic: d_a phi = (1/c_s^2) sum_q w_q e_qa phi(x + e_q) */
        double sx = 0, sy = 0;
        for (int q = 1; q < 9; ++q) {
            double v = field_at(o, phi, x + o->ex[q], y + o->ey[q]);
            sx += o->w[q] * o->ex[q] * v;
            sy += o->w[q] * o->ey[q] * v;
        }
        *gx = sx / o->D.cs2;
        *gy = sy / o->D.cs2;
        return;
    }
    *gx = wall_axis_derivative(o, phi, x, y, 0);
    *gy = wall_axis_derivative(o, phi, x, y, 1);
}

void orc_gradient(const orc* o, const double* phi, int x, int y, double* gx, double* gy)
{
    gradient(o, phi, x, y, gx, gy);
}

/* ------------------------------------------------------------------ */
/* lifecycle                                                           */
/* ------------------------------------------------------------------ */

static int fail(orc* o, int code, const char* msg)
{
    if (o) snprintf(o->err, sizeof o->err, "%s", msg);
    return code;
}

const char* orc_error(const orc* o) { return o ? o->err : "null context"; }

void orc_get_derived(const orc* o, orc_derived* d) { *d = o->D; }

int orc_create(const orc_params* p, orc** out)
{
    *out = NULL;
    orc* o = (orc*)calloc(1, sizeof *o);
    if (!o) return -2;
    o->P = *p;
    const orc_params* P = &o->P;
    if (P->nx < 1 || P->ny < 1) { *out = o; return fail(o, -1, "bad grid size"); }
    if (P->side_wall[0] != P->side_wall[1] || P->side_wall[2] != P->side_wall[3]) {
        *out = o; return fail(o, -1, "opposite sides must both be walls or both periodic");
    }
    if ((P->side_wall[0] && P->nx < 5) || (P->side_wall[2] && P->ny < 5)) {
        *out = o; return fail(o, -1, "a walled axis needs at least 5 nodes");
    }
    if (!(P->rho0 > 0) || !(P->T0 > 0) || !(P->Pr > 0) || !(P->gamma > 0) || !(P->nu0 > 0)
        || P->bulk_ratio < 0 || P->extrap_order < 1 || P->extrap_order > 2
        || P->cubic < 0 || P->cubic > 2 || P->eos < 0 || P->eos > 3
        || P->visc_law < 0 || P->visc_law > 2) {
        *out = o; return fail(o, -1, "invalid parameter");
    }

    o->threads = 1;
    orc_lattice(o->ex, o->ey, o->w);
    for (int q = 0; q < 9; ++q)
        for (int r = 0; r < 9; ++r)
            if (o->ex[r] == -o->ex[q] && o->ey[r] == -o->ey[q]) o->opp[q] = r;
    memcpy(o->M, M_PAPER, sizeof M_PAPER);
    if (invert9(o->M, o->Minv)) { *out = o; return fail(o, -1, "singular M"); }

    orc_derived* D = &o->D;
    D->cs2 = 1.0 / 3.0;
    /* Sec. 4: varpi = 1/6, gamma1 = -2, gamma2 = 2; Sec. 2.1: alpha1 = -1, beta1 = 1 */
    D->varpi = 1.0 / 6.0;
    D->gamma1 = -2.0;
    D->gamma2 = 2.0;
    D->alpha1 = -1.0;
    D->beta1 = 1.0;
    /* eq. LBE.u.coefficients */
    D->alpha2 = -(2.0 * D->alpha1 + D->varpi + 1.0) / (1.0 - D->varpi);
    D->beta2 = -2.0 * D->beta1 / (1.0 - D->varpi);
    D->k = 1.0 - D->varpi;
    D->h = 6.0 * D->varpi * (1.0 - D->varpi) / (1.0 - 3.0 * D->varpi);
    D->b = (1.0 - D->varpi) / (1.0 - 3.0 * D->varpi);
    /* eq. ECE.LBE: lambda = (2/3 + gamma1/2 + gamma2/3) rho0 C_p c^2 dt (1/sigma_j - 1/2) */
    D->kappa = 2.0 / 3.0 + D->gamma1 / 2.0 + D->gamma2 / 3.0;
    D->R = P->R > 0 ? P->R : derive_R(o, D->cs2);
    D->cp = P->cp > 0 ? P->cp : 3.5 * D->cs2 / P->T0;
    if (P->cv_rule == 1)
        D->cv = D->cp - eos_p(o, D->R, P->rho0, P->T0) / (P->rho0 * P->T0);
    else
        D->cv = D->cp / P->gamma;
    D->mu0 = P->rho0 * P->nu0;
    if (!(D->cv > 0) || !isfinite(D->R)) { *out = o; return fail(o, -1, "invalid thermodynamics"); }
    {
        double r[10];
        orc_rates(o, P->rho0, P->T0, r);
        if (!(r[5] > 0 && r[5] < 2) || !(r[8] > 0 && r[8] < 2)) {
            *out = o; return fail(o, -1, "relaxation rates out of (0, 2)");
        }
    }

    size_t nn = (size_t)P->nx * P->ny;
    o->f = calloc(nn * 9, sizeof(double));
    o->g = calloc(nn * 9, sizeof(double));
    o->fs = calloc(nn * 9, sizeof(double));
    o->gs = calloc(nn * 9, sizeof(double));
    o->rho = calloc(nn, sizeof(double));
    o->ux = calloc(nn, sizeof(double));
    o->uy = calloc(nn, sizeof(double));
    o->T = calloc(nn, sizeof(double));
    o->rhoE = calloc(nn, sizeof(double));
    o->p = calloc(nn, sizeof(double));
    if (!o->f || !o->g || !o->fs || !o->gs || !o->rho || !o->ux || !o->uy || !o->T || !o->rhoE || !o->p) {
        *out = o; return fail(o, -2, "out of memory");
    }
    *out = o;
    return 0;
}

void orc_destroy(orc* o)
{
    if (!o) return;
    free(o->f); free(o->g); free(o->fs); free(o->gs);
    free(o->rho); free(o->ux); free(o->uy); free(o->T); free(o->rhoE); free(o->p);
    free(o);
}

long long orc_time(const orc* o) { return o->t; }

void orc_set_threads(orc* o, int n) { o->threads = n > 0 ? n : 1; }

static int check_state(orc* o)
{
    size_t nn = (size_t)o->P.nx * o->P.ny;
    for (size_t i = 0; i < nn; ++i) {
        if (!isfinite(o->rho[i]) || !isfinite(o->ux[i]) || !isfinite(o->uy[i])
            || !isfinite(o->T[i]) || !(o->rho[i] > 0) || !(o->T[i] > 0))
            return fail(o, -4, "diverged: non-finite or non-positive rho/T");
    }
    return 0;
}

int orc_init(orc* o, const double* rho, const double* ux, const double* uy, const double* T)
{
    const int nx = o->P.nx, ny = o->P.ny;
    ORC_PARALLEL_ROWS
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int i = y * nx + x;
            nstate s;
            state_from_macros(o, rho ? rho[i] : o->P.rho0, ux ? ux[i] : 0.0, uy ? uy[i] : 0.0,
                              T ? T[i] : o->P.T0, &s);
            store_state(o, i, &s);
            /* m = m^eq - F_m/2, n = n^eq - Q_m/2 (zero non-equilibrium part) */
            double meq[9], Fm[9], neq[9], Qm[9], m[9], n[9];
            orc_meq(o, s.rho, s.ux, s.uy, s.eta, meq);
            orc_fm(o, s.Fx, s.Fy, s.ux, s.uy, Fm);
            orc_neq(o, s.rho, s.rhoE, s.ux, s.uy, s.H, s.T, neq);
            orc_qm(o, s.qe, s.ux, s.uy, Qm);
            for (int q = 0; q < 9; ++q) { m[q] = meq[q] - 0.5 * Fm[q]; n[q] = neq[q] - 0.5 * Qm[q]; }
            matvec9(o->Minv, m, o->f + (size_t)i * 9);
            matvec9(o->Minv, n, o->g + (size_t)i * 9);
        }
    o->t = 0;
    o->ready = 1;
    return check_state(o);
}

/* tilde non-equilibrium moments (eq. neq.redefinition) at an off-wall node */
static void tilde_neq(const orc* o, int i, double Zm[9], double Zn[9])
{
    const double* f = o->f + (size_t)i * 9;
    const double* g = o->g + (size_t)i * 9;
    nstate s;
    state_stored(o, i, &s);
    double S[81], L[81], Y[81];
    orc_matrices(o, s.rho, s.ux, s.uy, s.T, S, NULL, NULL, NULL, L, Y);
    double m[9], meq[9], Fm[9], mneq[9], n[9], neq[9], Qm[9], nneq[9];
    matvec9(o->M, f, m);
    orc_meq(o, s.rho, s.ux, s.uy, s.eta, meq);
    orc_fm(o, s.Fx, s.Fy, s.ux, s.uy, Fm);
    for (int q = 0; q < 9; ++q) mneq[q] = m[q] - meq[q] + 0.5 * Fm[q];
    matvec9(o->M, g, n);
    orc_neq(o, s.rho, s.rhoE, s.ux, s.uy, s.H, s.T, neq);
    orc_qm(o, s.qe, s.ux, s.uy, Qm);
    for (int q = 0; q < 9; ++q) nneq[q] = n[q] - neq[q] + 0.5 * Qm[q];
    double IS[81], IL[81], YZ[9], LZ[9];
    for (int k = 0; k < 81; ++k) {
        double id = (k % 10) == 0 ? 1.0 : 0.0;
        IS[k] = id - 0.5 * S[k];
        IL[k] = id - 0.5 * L[k];
    }
    matvec9(IS, mneq, Zm);
    matvec9(IL, nneq, LZ);
    matvec9(Y, Zm, YZ);
    for (int q = 0; q < 9; ++q) Zn[q] = LZ[q] + 0.5 * YZ[q];
}

static int one_step(orc* o)
{
    const int nx = o->P.nx, ny = o->P.ny;
    const size_t nn = (size_t)nx * ny;

    /* 1. collision at time t of every node, with gradients at time t */
    ORC_PARALLEL_ROWS
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int i = y * nx + x;
            nstate s;
            state_stored(o, i, &s);
            double grad[4];
            gradient(o, o->rho, x, y, &grad[0], &grad[1]);
            gradient(o, o->p, x, y, &grad[2], &grad[3]);
            collide(o, o->f + (size_t)i * 9, o->g + (size_t)i * 9, &s, grad,
                    o->fs + (size_t)i * 9, o->gs + (size_t)i * 9, NULL, NULL, NULL, NULL);
        }

    /* 2. streaming (eqs. LBE.u.s, LBE.T.s); DFs whose source lies outside a
     *    wall take the bounce-back temporaries (eqs. BB.f, BB.g) */
    ORC_PARALLEL_ROWS
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int i = y * nx + x;
            for (int q = 0; q < 9; ++q) {
                int sx = wrap_x(o, x - o->ex[q]), sy = wrap_y(o, y - o->ey[q]);
                if (sx >= 0 && sy >= 0) {
                    int j = sy * nx + sx;
                    o->f[(size_t)i * 9 + q] = o->fs[(size_t)j * 9 + q];
                    o->g[(size_t)i * 9 + q] = o->gs[(size_t)j * 9 + q];
                } else {
                    o->f[(size_t)i * 9 + q] = o->fs[(size_t)i * 9 + o->opp[q]];
                    o->g[(size_t)i * 9 + q] = o->gs[(size_t)i * 9 + o->opp[q]];
                }
            }
        }
    o->t += 1;

    /* 3. macros at t+1: off-wall nodes from their DFs; wall nodes from the
     *    temporaries (rho; rho*E when adiabatic) and the prescribed values */
    ORC_PARALLEL_ROWS
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int i = y * nx + x;
            const double* f = o->f + (size_t)i * 9;
            const double* g = o->g + (size_t)i * 9;
            nstate s;
            if (!is_wall(o, x, y)) {
                state_from_df(o, f, g, &s);
            } else {
                double ubx, uby, Tw;
                int adiabatic;
                wall_spec(o, x, y, &ubx, &uby, &adiabatic, &Tw);
                double rho = 0.0, sg = 0.0;
                for (int q = 0; q < 9; ++q) { rho += f[q]; sg += g[q]; }
                if (adiabatic) {
                    double Fx, Fy;
                    force_at(o, rho, &Fx, &Fy);
                    double qe = ubx * Fx + uby * Fy;
                    double rhoE = sg + 0.5 * qe;
                    double eps = rhoE / rho - 0.5 * (ubx * ubx + uby * uby);
                    s.rho = rho; s.ux = ubx; s.uy = uby; s.T = eps / o->D.cv; s.rhoE = rhoE;
                    complete_state(o, &s);
                } else {
                    state_from_macros(o, rho, ubx, uby, Tw, &s);
                }
            }
            store_state(o, i, &s);
        }

    /* 4. wall nodes: rebuild all DFs from equilibrium, force and the
     *    extrapolated non-equilibrium parts (eqs. decompose, neq.redefinition,
     *    neq.extrapolation).  Results go to the scratch arrays first so that
     *    every extrapolation reads streamed values. */
    int any_wall = o->P.side_wall[0] || o->P.side_wall[2];
    if (any_wall) {
        int singular = 0;
        ORC_PARALLEL_ROWS
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!is_wall(o, x, y)) continue;
                int i = y * nx + x;
                int nxd = on_side(o, x, y, 0) ? 1 : (on_side(o, x, y, 1) ? -1 : 0);
                int nyd = on_side(o, x, y, 2) ? 1 : (on_side(o, x, y, 3) ? -1 : 0);
                int i_f = (y + nyd) * nx + (x + nxd);
                int i_ff = (y + 2 * nyd) * nx + (x + 2 * nxd);
                double Zm[9], Zn[9], Zm_f[9], Zn_f[9];
                tilde_neq(o, i_f, Zm_f, Zn_f);
                if (o->P.extrap_order == 2) {
                    double Zm_ff[9], Zn_ff[9];
                    tilde_neq(o, i_ff, Zm_ff, Zn_ff);
                    for (int q = 0; q < 9; ++q) {
                        Zm[q] = 2.0 * Zm_f[q] - Zm_ff[q];
                        Zn[q] = 2.0 * Zn_f[q] - Zn_ff[q];
                    }
                } else {
                    memcpy(Zm, Zm_f, sizeof Zm);
                    memcpy(Zn, Zn_f, sizeof Zn);
                }
                nstate s;
                state_stored(o, i, &s);
                double S[81], L[81], Y[81], IS[81], IL[81];
                orc_matrices(o, s.rho, s.ux, s.uy, s.T, S, NULL, NULL, NULL, L, Y);
                for (int k = 0; k < 81; ++k) {
                    double id = (k % 10) == 0 ? 1.0 : 0.0;
                    IS[k] = id - 0.5 * S[k];
                    IL[k] = id - 0.5 * L[k];
                }
                double mneq[9], YZ[9], rhs[9], nneq[9];
                if (solve9(IS, Zm, mneq)) {
#pragma omp atomic write
                    singular = 1;
                    continue;
                }
                matvec9(Y, Zm, YZ);
                for (int q = 0; q < 9; ++q) rhs[q] = Zn[q] - 0.5 * YZ[q];
                if (solve9(IL, rhs, nneq)) {
#pragma omp atomic write
                    singular = 2;
                    continue;
                }
                double meq[9], Fm[9], neq[9], Qm[9], m[9], n[9];
                orc_meq(o, s.rho, s.ux, s.uy, s.eta, meq);
                orc_fm(o, s.Fx, s.Fy, s.ux, s.uy, Fm);
                orc_neq(o, s.rho, s.rhoE, s.ux, s.uy, s.H, s.T, neq);
                orc_qm(o, s.qe, s.ux, s.uy, Qm);
                for (int q = 0; q < 9; ++q) {
                    m[q] = meq[q] - 0.5 * Fm[q] + mneq[q];
                    n[q] = neq[q] - 0.5 * Qm[q] + nneq[q];
                }
                matvec9(o->Minv, m, o->fs + (size_t)i * 9);
                matvec9(o->Minv, n, o->gs + (size_t)i * 9);
            }
        if (singular) return fail(o, -4, singular == 1 ? "singular I - S/2" : "singular I - L/2");
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!is_wall(o, x, y)) continue;
                size_t i = (size_t)y * nx + x;
                memcpy(o->f + i * 9, o->fs + i * 9, 9 * sizeof(double));
                memcpy(o->g + i * 9, o->gs + i * 9, 9 * sizeof(double));
            }
    }
    (void)nn;
    return check_state(o);
}

int orc_step(orc* o, long long n)
{
    if (!o->ready) return fail(o, -5, "not initialised");
    for (long long k = 0; k < n; ++k) {
        int rc = one_step(o);
        if (rc) return rc;
    }
    return 0;
}

int orc_macros(const orc* o, double* rho, double* ux, double* uy, double* T, double* p)
{
    size_t nn = (size_t)o->P.nx * o->P.ny;
    if (rho) memcpy(rho, o->rho, nn * sizeof(double));
    if (ux) memcpy(ux, o->ux, nn * sizeof(double));
    if (uy) memcpy(uy, o->uy, nn * sizeof(double));
    if (T) memcpy(T, o->T, nn * sizeof(double));
    if (p) memcpy(p, o->p, nn * sizeof(double));
    return 0;
}

int orc_get_df(const orc* o, double* f, double* g)
{
    size_t nn = (size_t)o->P.nx * o->P.ny;
    if (f) memcpy(f, o->f, nn * 9 * sizeof(double));
    if (g) memcpy(g, o->g, nn * 9 * sizeof(double));
    return 0;
}

/* Mean Nusselt number (Sec. 4.3):
 *   Nu = 1/(lambda0 (T_lo - T_hi)) * integral over the side of J_n,
 * with J_n = -lambda(T) dT/dn, n the side's axis (+x for sides 0 and 1,
 * +y for sides 2 and 3), T_lo/T_hi the Dirichlet values of the low/high
 * side of that axis, a second-order one-sided dT/dn and trapezoid weights. */
int orc_nusselt(const orc* o, int side, double* nu)
{
    const int nx = o->P.nx, ny = o->P.ny;
    if (side < 0 || side > 3 || !o->P.side_wall[side] || o->P.side_adiabatic[side])
        return -1;
    int lo = side < 2 ? 0 : 2, hi = lo + 1;
    if (o->P.side_adiabatic[lo] || o->P.side_adiabatic[hi]) return -1;
    double dT = o->P.side_T[lo] - o->P.side_T[hi];
    if (dT == 0.0) return -1;
    double lambda0 = o->D.cp * o->D.mu0 / o->P.Pr;
    int len = side < 2 ? ny : nx;
    double sum = 0.0;
    for (int j = 0; j < len; ++j) {
        double t0, t1, t2, dTdn;
        if (side < 2) {
            int x0 = side == 0 ? 0 : nx - 1, d = side == 0 ? 1 : -1;
            t0 = o->T[j * nx + x0]; t1 = o->T[j * nx + x0 + d]; t2 = o->T[j * nx + x0 + 2 * d];
            dTdn = d * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
        } else {
            int y0 = side == 2 ? 0 : ny - 1, d = side == 2 ? 1 : -1;
            t0 = o->T[y0 * nx + j]; t1 = o->T[(y0 + d) * nx + j]; t2 = o->T[(y0 + 2 * d) * nx + j];
            dTdn = d * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
        }
        double lam = o->D.cp * viscosity(o, t0) / o->P.Pr;
        double wgt = (j == 0 || j == len - 1) ? 0.5 : 1.0;
        sum += wgt * (-lam * dTdn);
    }
    *nu = sum / (lambda0 * dT);
    return 0;
}

int orc_totals(const orc* o, double* mass, double* momx, double* momy, double* energy)
{
    size_t nn = (size_t)o->P.nx * o->P.ny;
    double m = 0, mx = 0, my = 0, e = 0;
    for (size_t i = 0; i < nn; ++i) {
        m += o->rho[i];
        mx += o->rho[i] * o->ux[i];
        my += o->rho[i] * o->uy[i];
        e += o->rhoE[i];
    }
    if (mass) *mass = m;
    if (momx) *momx = mx;
    if (momy) *momy = my;
    if (energy) *energy = e;
    return 0;
}
