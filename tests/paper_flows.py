"""The paper's channel validations (Secs. 4.1 and 4.2) as input presets and
closed-form solutions, for the oracle pins and the GPU validation tests.

Lattice units: delta_x = delta_t = 1, c_s^2 = 1/3, rho0 = T0 = 1.  The paper
sets R_g = T0 = rho0 = 1 with c_s defined by the EOS; the analytic profiles
depend only on the groups (Pr, Ec) or (Pr, Ma_e) and on the EOS, so the
lattice cases below reproduce them with R chosen from c_s^2 = 1/3 (eq. cs).
Walls sit on the first and last node rows, W = ny - 1.

Only closed forms and the EOS live here; nothing of the lattice Boltzmann
arithmetic.
"""
import numpy as np

from paper_1809_08683_amd import inputs

P = inputs._periodic
W = inputs._side

CS2 = 1.0 / 3.0
CP = 3.5 * CS2          # eq. Cp with T0 = 1
TAU = 0.8               # Secs. 4.1-4.2: tau = 1/s_p for mu/rho0 (mu0/rho0)
NU = (TAU - 0.5) / 3.0
CS_B = np.sqrt(2.0) * np.pi / 3.0   # b = sqrt(2) pi / (3 rho0) of the Carnahan-Starling EOS


def _eos_kw(eos):
    # C_v = C_p - p(rho0, T0)/(rho0 T0) (eq. Cp); the ideal and decoupling
    # EOSs give gamma = 1.4 with it, Carnahan-Starling 1.101465
    return dict(eos=eos, cv_rule=1, cp=CP)


def poiseuille_case(eos, Pr, Ec, ny=65, nx=64, Ma_lattice=0.2, prec="f64"):
    """Sec. 4.1: force-driven channel, walls at rest, T_c below (= T0) and
    T_h above; U0 = Ma_lattice c_s, F_x = 8 mu U0 / W^2,
    T_h - T_c = U0^2 / (C_p Ec); second-order extrapolation."""
    Wd = ny - 1
    U0 = Ma_lattice * np.sqrt(CS2)
    fx = 8.0 * NU * U0 / Wd ** 2
    dT = U0 ** 2 / (CP * Ec)
    c = inputs.base_case(nx=nx, ny=ny, Pr=Pr, nu0=NU, force=(fx, 0.0), per_mass=False,
                         sides=[P(), P(), W(T=1.0), W(T=1.0 + dT)], extrap_order=2, prec=prec,
                         **_eos_kw(eos))
    c["paper"] = dict(U0=U0, Tc=1.0, Th=1.0 + dT, Pr=Pr, Ec=Ec)
    return c


def couette_case(eos, Pr, Ma_e, ny=65, nx=64, prec="f64"):
    """Sec. 4.2: lower wall at rest and adiabatic, upper wall moving at U0
    and held at T0; mu / mu0 = T / T0 with Pr and C_p constant;
    Ma_e = U0 / sqrt(C_p T0); second-order extrapolation."""
    U0 = Ma_e * np.sqrt(CP)
    c = inputs.base_case(nx=nx, ny=ny, Pr=Pr, nu0=NU, visc_law="linear",
                         sides=[P(), P(), W(thermal="adiabatic", T=1.0), W(u=(U0, 0.0), T=1.0)],
                         extrap_order=2, prec=prec, **_eos_kw(eos))
    c["paper"] = dict(U0=U0, Pr=Pr, Ma_e=Ma_e)
    return c


def poiseuille_profiles(yy, Pr, Ec):
    """eq. Poiseuille.u.T: u_x/U0 and (T - T_c)/(T_h - T_c) at y/W = yy."""
    u = 4.0 * yy * (1.0 - yy)
    theta = Pr * Ec / 3.0 * (1.0 - (1.0 - 2.0 * yy) ** 4) + yy
    return u, theta


def couette_profiles(yy, Pr, Ma_e):
    """eq. Couette.u.T (Liepmann): the cubic for u_x/U0 solved by Newton's
    method at each y/W = yy, then T/T0."""
    k = Pr * Ma_e ** 2
    rhs = (1.0 + k / 3.0) * yy
    u = np.array(yy, dtype=float)
    for _ in range(50):
        g = u + 0.5 * k * (u - u ** 3 / 3.0) - rhs
        dg = 1.0 + 0.5 * k * (1.0 - u ** 2)
        u = u - g / dg
    T = 1.0 + 0.5 * k * (1.0 - u ** 2)
    return u, T


def cs_Z(rho):
    y = CS_B * rho / 4.0
    return (1.0 + y + y * y - y ** 3) / (1.0 - y) ** 3


def cs_R():
    """R from c_s^2 = dp/drho at (rho0, T0) = 1/3 for p = Z rho R T (eq. cs)."""
    h = 1e-6
    dp = ((1 + h) * cs_Z(1 + h) - (1 - h) * cs_Z(1 - h)) / (2 * h)
    return CS2 / dp


def density_profile(eos, T, mass):
    """eq. rho.analytical: rho/rho0 across the channel from the steady T
    profile, with the lattice's node sum of rho equal to `mass` (the initial
    mass; the paper's integral of rho over the width).
      decoupling: rho = rho0;  ideal gas: rho = A T0 / T;
      Carnahan-Starling: Z(rho) rho R T = p uniform, p fixed by the mass."""
    T = np.asarray(T, dtype=float)
    n = T.size
    if eos == "decoupled":
        return np.full(n, mass / n)
    if eos == "ideal":
        inv = 1.0 / T
        return mass / inv.sum() * inv
    R = cs_R()

    def rho_of(p):
        r = np.ones(n)
        for _ in range(60):
            f = cs_Z(r) * r * R * T - p
            h = 1e-7
            df = (cs_Z(r + h) * (r + h) - cs_Z(r - h) * (r - h)) / (2 * h) * R * T
            r = r - f / df
        return r

    lo, hi = 0.1, 10.0
    for _ in range(200):
        p = 0.5 * (lo + hi)
        if rho_of(p).sum() > mass:
            hi = p
        else:
            lo = p
    return rho_of(0.5 * (lo + hi))


# ---------------------------------------------------------------------------
# Constant-property channel flows on the benchmark grids (heated Couette
# 3 x 64, van der Waals Poiseuille 3 x 128): incompressible start-up series
# from rest and the steady closed forms.  eta = y / W, s = nu t / W^2.
# ---------------------------------------------------------------------------
def couette_startup(eta, s, terms=4000):
    """u_x / U of a channel whose upper wall starts moving at U at t = 0
    (lower wall at rest, fluid at rest): the steady eta minus the sine series
    of eta, each mode decaying as exp(-(n pi)^2 s)."""
    n = np.arange(1, terms + 1)[:, None]
    modes = 2.0 * (-1.0) ** (n + 1) / (n * np.pi) * np.sin(n * np.pi * eta)
    return eta - np.sum(modes * np.exp(-(n * np.pi) ** 2 * s), axis=0)


def poiseuille_startup(eta, s, terms=4001):
    """u_x / U0 of a force-driven channel started from rest, F = 8 mu U0 / W^2
    (U0 the steady centre-line velocity): 4 eta (1 - eta) minus its sine
    series (odd modes, coefficients 32 / (n pi)^3)."""
    n = np.arange(1, terms + 1, 2)[:, None]
    modes = 32.0 / (n * np.pi) ** 3 * np.sin(n * np.pi * eta)
    return 4.0 * eta * (1.0 - eta) - np.sum(modes * np.exp(-(n * np.pi) ** 2 * s), axis=0)


def heated_couette_steady(eta, U, T_bottom, T_top, Pr, cp=CP):
    """Steady heated Couette flow with constant mu and lambda = C_p mu / Pr:
    u = U eta and lambda T'' + mu (U / W)^2 = 0, so
    T = T_b + (T_t - T_b) eta + (Pr U^2 / (2 C_p)) eta (1 - eta)."""
    return U * eta, T_bottom + (T_top - T_bottom) * eta + Pr * U * U / (2.0 * cp) * eta * (1.0 - eta)


def poiseuille_steady(eta, U0, T_wall, Pr, cp=CP):
    """Steady force-driven channel with constant mu and lambda and both walls
    at T_w: u = 4 U0 eta (1 - eta) and lambda T'' + mu u'^2 = 0, so
    T = T_w + (Pr U0^2 / (3 C_p)) (1 - (1 - 2 eta)^4)."""
    return 4.0 * U0 * eta * (1.0 - eta), T_wall + Pr * U0 * U0 / (3.0 * cp) * (1.0 - (1.0 - 2.0 * eta) ** 4)
