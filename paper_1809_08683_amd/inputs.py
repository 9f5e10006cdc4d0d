"""Seeded synthetic inputs and problem presets.

This module holds no lattice Boltzmann arithmetic: it only states problems
(grid, closures, boundary values, forces, initial fields) in lattice units,
so that the HIP library, the CPU oracle used by the tests and the benchmark
are all driven by identical inputs.

A case is a plain dict:
    nx, ny                      grid (nodes on the walls, Sec. 3)
    eos                         "decoupled" | "ideal" | "vdw" | "cs"
    R, rho0, T0, a, b           EOS parameters (R <= 0: from c_s^2 = dp/drho)
    Pr, gamma                   Prandtl number, C_p / C_v
    nu0, bulk_ratio             mu0/rho0 at T0, bulk/kinematic viscosity ratio
    visc_law, suth_S            "const" | "linear" | "sutherland", S/T0
    force, per_mass             (fx, fy); per unit mass (gravity) or volume
    cubic                       0 none, 1 R only, 2 R, T and X corrections
    cp, cv_rule                 C_p (<= 0: 3.5 c_s^2/T0); 0: C_v = C_p/gamma
    sides                       4 dicts: kind ("wall" | "periodic"), u, thermal, T
                                order: x = 0, x = nx-1, y = 0, y = ny-1
    extrap_order                1 or 2
    prec                        "f64" | "f32" | "f16s" (library only)

Lattice units throughout: dx = dt = c = 1, c_s^2 = 1/3.
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0
_MASK = (1 << 64) - 1


# ---------------------------------------------------------------------------
# splitmix64 (Steele, Lea & Flood 2014): state += 0x9E3779B97F4A7C15, then the
# published xor-shift-multiply finaliser.  Counter-based, so element i of a
# stream is a pure function of (seed, i).
# ---------------------------------------------------------------------------
def splitmix64(seed: int, n: int) -> np.ndarray:
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def noise(seed: int, n: int) -> np.ndarray:
    """Doubles in [-1, 1)."""
    return 2.0 * uniform01(seed, n) - 1.0


# ---------------------------------------------------------------------------
# presets
# ---------------------------------------------------------------------------
def _side(kind="wall", u=(0.0, 0.0), thermal="dirichlet", T=1.0):
    return {"kind": kind, "u": (float(u[0]), float(u[1])), "thermal": thermal, "T": float(T)}


def _periodic():
    return _side(kind="periodic")


def base_case(**kw) -> dict:
    c = dict(nx=16, ny=16, eos="ideal", R=0.0, rho0=1.0, T0=1.0, a=0.0, b=0.0,
             Pr=0.71, gamma=1.4, nu0=0.05, bulk_ratio=1.0, visc_law="const", suth_S=0.0,
             force=(0.0, 0.0), per_mass=False, cubic=2, cp=0.0, cv_rule=0,
             sides=[_periodic(), _periodic(), _periodic(), _periodic()],
             extrap_order=2, prec="f64")
    c.update(kw)
    return c


def couette(nx=3, ny=64, U=0.05, T_bottom=1.0, T_top=1.02, nu=0.05, prec="f64", **kw) -> dict:
    """Heated Couette channel: periodic x, bottom wall at rest, top wall moving."""
    return base_case(nx=nx, ny=ny, eos="ideal", Pr=0.71, gamma=1.4, nu0=nu,
                     sides=[_periodic(), _periodic(),
                            _side(u=(0, 0), T=T_bottom), _side(u=(U, 0), T=T_top)],
                     extrap_order=2, prec=prec, **kw)


def poiseuille(nx=3, ny=128, U0=0.05, nu=0.1, T_wall=1.0, eos="vdw", a=0.05, b=0.2,
               prec="f64", **kw) -> dict:
    """Force-driven channel: F_x = 8 mu U0 / W^2 with W = ny - 1 (eq. Poiseuille.u.T)."""
    W = ny - 1
    fx = 8.0 * nu * 1.0 * U0 / W ** 2
    return base_case(nx=nx, ny=ny, eos=eos, a=a, b=b, Pr=0.71, gamma=1.4, nu0=nu,
                     force=(fx, 0.0), per_mass=False,
                     sides=[_periodic(), _periodic(), _side(T=T_wall), _side(T=T_wall)],
                     extrap_order=2, prec=prec, **kw)


def bulk_ratio_for_ra(Ra: float) -> float:
    """Bulk/kinematic viscosity ratio of Table 1, rounded up to the next tabulated Ra."""
    if Ra <= 1e6 * (1 + 1e-12):
        return 1.0
    if Ra <= 1e7 * (1 + 1e-12):
        return 2.0
    return 4.0


def cavity(N=512, Ra=1e6, eps=0.6, Pr=0.71, nu0=0.1, Ma=None, bulk_ratio=None, noise_seed=None,
           noise_amp=1e-6, prec="f32", nx=None, ny=None) -> dict:
    """Differentially heated square cavity (Sec. 4.3) in lattice units.

    T0 = rho0 = 1, ideal gas with R = c_s^2/T0, L = N - 1, Sutherland
    S = 110.5/600, first-order extrapolation, walls x = 0 at T0 (1 + eps) and
    x = L at T0 (1 - eps), adiabatic top and bottom, gravity -y per unit mass.
    The lattice viscosity is set by nu0 = mu0/rho0 (default 0.1, i.e. the
    paper's tau = 0.8); gravity then follows from
    Ra = Pr g rho0^2 (T_h - T_c) L^3 / (T0 mu0^2).  Passing Ma instead fixes
    the buoyancy velocity U = Ma c_s, g = U^2/(2 eps L), mu0 = rho0 U L sqrt(Pr/Ra).
    """
    nx = N if nx is None else nx
    ny = N if ny is None else ny
    L = N - 1
    if Ma is not None:
        U = Ma * math.sqrt(CS2)
        g = U * U / (2.0 * eps * L)
        nu0 = U * L * math.sqrt(Pr / Ra)
    else:
        g = Ra * nu0 * nu0 / (2.0 * eps * Pr * L ** 3)
    br = bulk_ratio_for_ra(Ra) if bulk_ratio is None else bulk_ratio
    c = base_case(nx=nx, ny=ny, eos="ideal", Pr=Pr, gamma=1.4, nu0=nu0, bulk_ratio=br,
                  visc_law="sutherland", suth_S=110.5 / 600.0,
                  force=(0.0, -g), per_mass=True,
                  sides=[_side(T=1.0 + eps), _side(T=1.0 - eps),
                         _side(thermal="adiabatic"), _side(thermal="adiabatic")],
                  extrap_order=1, prec=prec)
    c["Ra"], c["eps"] = Ra, eps
    # Mach number of the reference velocity sqrt(Ra) mu0 / (rho0 L) of Sec. 4.3
    c["Ma_ref"] = math.sqrt(Ra) * nu0 / L / math.sqrt(CS2)
    if noise_seed is not None:
        c["init"] = {"rho": 1.0 + noise_amp * noise(noise_seed, nx * ny).reshape(ny, nx)}
    return c


def stable_nu0_window(eps: float, Pr: float, smax: float = 1.85, suth_S: float = 110.5 / 600.0):
    """Range of nu0 = mu0/rho0 for which the relaxation rates that the fixed
    products of Sec. 4 pair up stay at or below smax at both walls of a
    cavity with T = T0 (1 +- eps), isobaric density rho0 T0 / T and
    Sutherland viscosity:
      cold wall (small nu): s_p <= smax and sigma_j <= smax,
      hot wall (large nu):  s_q <= smax and sigma_e <= smax,
    using 1/s_p - 1/2 = 3 nu, (1/s_p - 1/2)(1/s_q - 1/2) = 1/12,
    1/sigma_j - 1/2 = nu / (kappa Pr) (rho = rho0), (1/sigma_j - 1/2)
    (1/sigma_e - 1/2) = 1/4, kappa = 1/3.  Returns (lo, hi); lo > hi when
    no such window exists."""
    kappa = 1.0 / 3.0
    m = 1.0 / smax - 0.5                       # required 1/s - 1/2 margin

    def nu_factor(T):                         # nu(T) / nu0 at p = p0
        mu = T ** 1.5 * (1.0 + suth_S) / (T + suth_S)
        return mu * T                          # mu / rho with rho = 1 / T
    fc, fh = nu_factor(1.0 - eps), nu_factor(1.0 + eps)
    mu_c = (1.0 - eps) ** 1.5 * (1.0 + suth_S) / (1.0 - eps + suth_S)
    mu_h = (1.0 + eps) ** 1.5 * (1.0 + suth_S) / (1.0 + eps + suth_S)
    lo = max(m / 3.0 / fc, m * kappa * Pr / mu_c)
    hi = min((1.0 / 36.0) / m / fh, 0.25 * kappa * Pr / m / mu_h)
    return lo, hi


def batch_cases(seed=2, n=64, Ma=0.05, nu_min=0.1, smax=1.75, prec="f32") -> list:
    """Uneven cavities: N in {128,256,512,1024}, log10 Ra in U[3,8],
    eps in U[0.1,0.6], Pr in {0.71,1,7}; four draws per case from one stream.

    Each case is set up at buoyancy Mach number Ma (g and mu0 from Ra as in
    cavity(Ma=...)).  Where that viscosity falls outside the window
    [max(nu_min, lo), hi] with (lo, hi) = stable_nu0_window(eps, Pr) it is
    moved to the nearest end (the geometric mean if the window is empty)
    with the same g, i.e. run at the effective Rayleigh number
    Ra * (nu_Ma / nu0)^2, "Ra_eff".  nu_min = 0.1 (tau0 = 0.8) is where the
    linearised coupled scheme stops growing at the cold wall of an eps = 0.6
    cavity.  For Pr = 7 and eps >= 0.48 the window is empty (s_q at the hot
    wall and sigma_j at the cold wall cannot both stay below smax); those
    cases run at the geometric mean and diverge after a few hundred steps."""
    u = uniform01(seed, 4 * n).reshape(n, 4)
    sizes = (128, 256, 512, 1024)
    prs = (0.71, 1.0, 7.0)
    out = []
    for k in range(n):
        N = sizes[min(int(u[k, 0] * 4), 3)]
        Ra = 10.0 ** (3.0 + 5.0 * u[k, 1])
        eps = 0.1 + 0.5 * u[k, 2]
        Pr = prs[min(int(u[k, 3] * 3), 2)]
        c = cavity(N=N, Ra=Ra, eps=eps, Pr=Pr, Ma=Ma, prec=prec)
        c["Ra_eff"] = Ra
        lo, hi = stable_nu0_window(eps, Pr, smax)
        lo = max(lo, nu_min)
        c["nu0_window"] = (lo, hi)
        c["window_empty"] = lo > hi      # flagged before any step: may diverge
        nu = c["nu0"] if lo <= hi else math.sqrt(lo * hi)
        nu = min(max(nu, lo), hi) if lo <= hi else nu
        if nu != c["nu0"]:
            c["Ra_eff"] = Ra * (c["nu0"] / nu) ** 2
            c["nu0"] = nu
            c["Ma_ref"] = math.sqrt(c["Ra_eff"]) * nu / (N - 1) / math.sqrt(CS2)
        out.append(c)
    return out


def random_fields(case: dict, seed: int, du=0.02, drho=0.05, dT=0.05):
    """Smooth-ish random initial fields for parity tests (walls included)."""
    nx, ny = case["nx"], case["ny"]
    n = nx * ny
    r = noise(seed, 4 * n).reshape(4, ny, nx)
    rho = case.get("rho0", 1.0) * (1.0 + drho * r[0])
    ux = du * r[1]
    uy = du * r[2]
    T = case.get("T0", 1.0) * (1.0 + dT * r[3])
    return {"rho": rho, "ux": ux, "uy": uy, "T": T}
