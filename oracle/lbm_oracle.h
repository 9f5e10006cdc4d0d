/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU reference of the coupled density /
 * total-energy D2Q9 MRT lattice Boltzmann step of Huang, Wu & Adams,
 * "Lattice Boltzmann model with self-tuning equation of state for coupled
 * thermo-hydrodynamic flows" (arXiv:1809.08683).
 *
 * It exists so that tests can check the HIP library against the paper.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load it.  It shares no code with the HIP path: every matrix of the paper
 * (M, S, R, T, X, L, Y) is built here as a dense array and applied by plain
 * matrix-vector products, and (I - S/2)^-1, (I - L/2)^-1 and M^-1 are
 * obtained by Gaussian elimination rather than from closed forms.
 *
 * Lattice units: dx = dt = c = 1, c_s^2 = 1/3.
 * Node (x, y) is stored at index y*nx + x (x fastest).
 * Sides: 0 = {x = 0}, 1 = {x = nx-1}, 2 = {y = 0}, 3 = {y = ny-1}.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EOS_DECOUPLED = 0, ORC_EOS_IDEAL = 1, ORC_EOS_VDW = 2, ORC_EOS_CS = 3 };
enum { ORC_VISC_CONST = 0, ORC_VISC_LINEAR = 1, ORC_VISC_SUTHERLAND = 2 };

typedef struct {
    int nx, ny;
    /* equation of state (Sec. 4, eqs. EOSs; van der Waals as an extra kind) */
    int eos;
    double R;           /* <= 0: chosen so that dp/drho(rho0, T0) = c_s^2 (eq. cs) */
    double rho0, T0;
    double a, b;        /* van der Waals a, b; Carnahan-Starling b (<= 0: sqrt(2) pi / (3 rho0)) */
    double Pr, gamma;
    /* transport */
    double nu0;         /* mu0 / rho0 at T0 */
    double bulk_ratio;  /* bulk / kinematic viscosity */
    int visc_law;       /* ORC_VISC_* */
    double suth_S;      /* Sutherland constant in units of T0 */
    /* force: F = (fx, fy) per unit volume, or rho*(fx, fy) when per_mass */
    double fx, fy;
    int per_mass;
    int cubic;          /* 0: no R, T, X; 1: R only; 2: R, T and X (the paper) */
    double cp;          /* <= 0: 3.5 c_s^2 / T0 (eq. Cp) */
    int cv_rule;        /* 0: cv = cp / gamma; 1: cv = cp - p(rho0,T0)/(rho0 T0) (eq. Cp) */
    /* boundaries */
    int side_wall[4];       /* 0 periodic, 1 wall */
    double side_ux[4], side_uy[4];
    int side_adiabatic[4];  /* 1: zero heat flux, 0: Dirichlet */
    double side_T[4];
    int extrap_order;       /* 1 or 2 (eq. neq.extrapolation) */
} orc_params;

typedef struct orc orc;

/* Derived constants (for tests). */
typedef struct {
    double cs2, R, cp, cv, kappa, mu0;
    double alpha1, beta1, alpha2, beta2, varpi, k, h, b, gamma1, gamma2;
} orc_derived;

/* Lifecycle.  Return 0 on success, negative on error. */
int  orc_create(const orc_params* p, orc** out);
void orc_destroy(orc* o);
const char* orc_error(const orc* o);
void orc_get_derived(const orc* o, orc_derived* d);

/* Initial state (t = 0) from macroscopic fields; NULL means uniform
 * rho0, 0, 0, T0.  Arrays are [ny*nx]. */
int  orc_init(orc* o, const double* rho, const double* ux, const double* uy, const double* T);
/* n steps; returns -4 on divergence (non-finite, rho <= 0 or T <= 0). */
int  orc_step(orc* o, long long n);
long long orc_time(const orc* o);
/* OpenMP threads for the node loops of init and step (default 1).  The
 * result is bitwise the same for any count. */
void orc_set_threads(orc* o, int n);
/* Macroscopic fields at the current time (wall nodes report their
 * prescribed / derived values).  Any pointer may be NULL. */
int  orc_macros(const orc* o, double* rho, double* ux, double* uy, double* T, double* p);
/* Pre-collision distributions at the current time, [ny*nx*9], q fastest. */
int  orc_get_df(const orc* o, double* f, double* g);
/* Mean Nusselt number through a Dirichlet side (0..3). */
int  orc_nusselt(const orc* o, int side, double* nu);
/* Sums over all nodes of rho, rho*ux, rho*uy and rho*E. */
int  orc_totals(const orc* o, double* mass, double* momx, double* momy, double* energy);

/* ---- node-level building blocks, exposed for the pin tests ---- */
void orc_lattice(int ex[9], int ey[9], double w[9]);
void orc_moment_matrix(double M[81], double Minv[81]);
double orc_pressure(const orc* o, double rho, double T);
void orc_meq(const orc* o, double rho, double ux, double uy, double eta, double out[9]);
void orc_fm(const orc* o, double fx, double fy, double ux, double uy, double out[9]);
void orc_neq(const orc* o, double rho, double rhoE, double ux, double uy,
             double H, double T, double out[9]);
void orc_qm(const orc* o, double qe, double ux, double uy, double out[9]);
/* rates[10] = s0, se, seps, sj, sq, sp, sig0, sige, sigj, sigq (sigeps = sigp = sige) */
void orc_rates(const orc* o, double rho, double T, double rates[10]);
/* Dense matrices at a node state. */
void orc_matrices(const orc* o, double rho, double ux, double uy, double T,
                  double S[81], double R[81], double Tm[18], double X[18],
                  double L[81], double Y[81]);
/* Gradient (d/dx, d/dy) at node (x, y) of a field phi[ny*nx] with the
 * stencil the collision uses for grad(rho) and grad(p). */
void orc_gradient(const orc* o, const double* phi, int x, int y, double* gx, double* gy);
/* One collision of a node whose pre-collision DFs are f, g, with macros
 * computed from f, g as at an interior node, and the given gradients
 * grad = (drho/dx, drho/dy, dp/dx, dp/dy).  Also returns m, mbar, n, nbar. */
void orc_collide_node(const orc* o, const double f[9], const double g[9],
                      const double grad[4], double fbar[9], double gbar[9],
                      double m[9], double mbar[9], double n[9], double nbar[9]);

#ifdef __cplusplus
}
#endif
#endif
