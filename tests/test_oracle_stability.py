"""Linear stability of the oracle's uniform-state update (no GPU).

A uniform state at rest (rho_b, 0, T_b) with no force is a fixed point of the
coupled step of Secs. 2.1-2.2.  Near it the step is linear: collision
(Jacobian J of the 18 post-collision DFs with respect to the 18
pre-collision DFs, taken by central differences of the oracle's own
collision) followed by streaming, which multiplies DF q of a Fourier mode k
by exp(-i k.e_q).  The spectral radius of diag(exp(-i k.e_q)) J over k is
the per-step growth of the fastest mode.

Pins against the paper (Secs. 4.1, 4.2): at tau = 0.8 for mu0/rho0 the
ideal-gas runs with Pr = 0.1 lose stability, the decoupling and
Carnahan-Starling runs at the same parameters do not, and Pr = 0.71 is
stable; Table 1 raises the bulk-to-shear viscosity ratio to 2 and 4 for the
high-Ra cavities to enhance stability.

Finding (documented, not a pin of the paper): with the relaxation relations
of Sec. 4 the ideal-gas rest state grows at small viscosity, from about
nu0 = 0.02 (Pr = 0.71, ratio 1) on, while the decoupling EOS stays neutral.
None of the readings the paper leaves open changes this at T0, rho0 (the
local-density or reference-density viscosity coincide there).
"""
import numpy as np
import pytest

import oracle
from paper_1809_08683_amd import inputs

EX, EY, _ = oracle.lattice()
M, MINV = oracle.moment_matrix()


def _uniform_df(o, rho, T):
    d = o.derived()
    p = o.pressure(rho, T)
    eta = (p / d["cs2"] - (2 + d["alpha1"]) * rho) / d["beta1"]
    rhoE = rho * d["cv"] * T
    meq = o.meq(rho, 0.0, 0.0, eta)
    neq = o.neq(rho, rhoE, 0.0, 0.0, rhoE / rho + p / rho, T)
    return np.concatenate([MINV @ meq, MINV @ neq])


def _jacobian(o, rho=1.0, T=1.0, h=1e-6):
    x0 = _uniform_df(o, rho, T)

    def post(x):
        r = o.collide_node(x[:9], x[9:], np.zeros(4))
        return np.concatenate([r["fbar"], r["gbar"]])

    assert np.abs(post(x0) - x0).max() < 1e-14, "uniform rest state must be a fixed point"
    J = np.empty((18, 18))
    for j in range(18):
        e = np.zeros(18)
        e[j] = h
        J[:, j] = (post(x0 + e) - post(x0 - e)) / (2 * h)
    return J


def spectral_radius(o, rho=1.0, T=1.0, nk=32):
    """Largest |eigenvalue| of the one-step amplification matrix over the
    nk x nk Fourier modes of a periodic lattice (half plane by symmetry)."""
    J = _jacobian(o, rho, T)
    worst = 0.0
    for a in range(nk):
        for b in range(nk // 2 + 1):
            ph = np.exp(-1j * (2 * np.pi * a / nk * EX + 2 * np.pi * b / nk * EY))
            A = np.concatenate([ph, ph])[:, None] * J
            worst = max(worst, float(np.abs(np.linalg.eigvals(A)).max()))
    return worst


def _case(eos, nu0, Pr, bulk_ratio=1.0):
    c = inputs.base_case(nx=4, ny=4, eos=eos, nu0=nu0, Pr=Pr, bulk_ratio=bulk_ratio,
                         cv_rule=1 if eos == "cs" else 0)
    return oracle.Oracle(c)


NEUTRAL = 1.0 + 1e-7   # the conserved modes sit at |lambda| = 1 (finite-difference Jacobian)


@pytest.mark.parametrize("eos", ["decoupled", "ideal", "cs"])
def test_paper_unstable_set_is_the_ideal_gas_at_low_prandtl(eos):
    """Secs. 4.1 and 4.2: with tau = 0.8 for mu0/rho0, Pr = 0.1 loses
    stability for the ideal-gas EOS only; Pr = 0.71 is stable for all three."""
    r_low = spectral_radius(_case(eos, 0.1, 0.1))
    r_ref = spectral_radius(_case(eos, 0.1, 0.71))
    assert r_ref <= NEUTRAL
    if eos == "ideal":
        assert r_low > 1.1
    else:
        assert r_low <= NEUTRAL


def test_bulk_viscosity_ratio_of_table1_enhances_stability():
    """Table 1: the bulk/shear viscosity ratio is raised (1 -> 2 -> 4) at high
    Ra to enhance stability; the growth of the least stable mode falls with
    the ratio."""
    r = [spectral_radius(_case("ideal", 0.0124, 0.71, br)) for br in (1.0, 2.0, 4.0)]
    assert r[0] > r[1] > r[2] > 1.0


def test_small_viscosity_growth_needs_the_thermal_coupling():
    """Finding: at nu0 = 0.0124 (the viscosity a 2048^2, Ra = 1e8 cavity gets at
    buoyancy Mach 0.05) the ideal-gas rest state grows by more than 10 % per
    step; with the decoupling EOS (p independent of T, so the energy DF no
    longer feeds the density DF) the same rates are neutral."""
    assert spectral_radius(_case("decoupled", 0.0124, 0.71)) <= NEUTRAL
    assert spectral_radius(_case("ideal", 0.0124, 0.71)) > 1.1
    assert spectral_radius(_case("ideal", 0.05, 0.71)) <= NEUTRAL


def test_linear_growth_matches_the_time_stepping():
    """The amplification matrix predicts the oracle's own time stepping: a
    1e-13 perturbation of the rest state of a periodic 32x32 ideal-gas box at
    nu0 = 0.0124 grows at the predicted rate (to 1 %: a mode close to the
    fastest one still contributes after 100 steps) while it is small."""
    o = _case("ideal", 0.0124, 0.71)
    rate = spectral_radius(o, nk=32)
    c = inputs.base_case(nx=32, ny=32, eos="ideal", nu0=0.0124, Pr=0.71)
    n = 32 * 32
    box = oracle.Oracle(c).init(rho=1.0 + 1e-13 * inputs.noise(11, n).reshape(32, 32))

    def amp():
        f, g = box.df()
        return np.abs(f - f.mean(axis=(0, 1))).max()

    box.step(100)
    a0 = amp()
    box.step(40)
    a1 = amp()
    assert a1 < 1e-4
    measured = (a1 / a0) ** (1 / 40)
    assert measured == pytest.approx(rate, rel=1e-2)


@pytest.mark.parametrize("Pr", [0.71])
def test_quiescent_cavity_at_a_stable_viscosity_stays_at_rest(Pr):
    """Closed ideal-gas cavity at rest with every wall at T0 and no force, at
    nu0 = 0.1 (tau0 = 0.8): a fixed point.  Rounding accumulates at most
    linearly in time (a random walk of about 1e-16 per step), it does not
    grow from step to step."""
    c = inputs.cavity(N=16, Ra=1e3, eps=0.1, Pr=Pr, nu0=0.1, prec="f64")
    c["force"] = (0.0, 0.0)
    for s in c["sides"][:2]:
        s["T"] = 1.0
    o = oracle.Oracle(c).init()
    x0 = np.concatenate([a.ravel() for a in o.df()])
    o.step(750)
    d1 = np.abs(np.concatenate([a.ravel() for a in o.df()]) - x0).max()
    o.step(750)
    d2 = np.abs(np.concatenate([a.ravel() for a in o.df()]) - x0).max()
    assert d2 < 1e-12 and d2 < 3 * d1


def test_quiescent_cavity_at_the_buoyancy_mach_viscosity_grows_from_rounding():
    """Finding: the same cavity at nu0 = 0.0124 is not a stable fixed point:
    rounding errors grow at about the rate of the periodic analysis and the
    state leaves rest within a few hundred steps."""
    c = inputs.cavity(N=16, Ra=1e3, eps=0.1, Pr=0.71, nu0=0.0124, prec="f64")
    c["force"] = (0.0, 0.0)
    for s in c["sides"][:2]:
        s["T"] = 1.0
    o = oracle.Oracle(c).init()
    f0, _ = o.df()
    o.step(150)
    f1, _ = o.df()
    assert np.abs(f1 - f0).max() > 1e-9


def _rest_channel(Pr, nu0, order, nx=16, ny=32):
    c = inputs.couette(nx=nx, ny=ny, U=0.0, T_bottom=1.0, T_top=1.0, nu=nu0)
    c["Pr"] = Pr
    c["extrap_order"] = order
    return c


def _departure(c, rho, steps):
    o = oracle.Oracle(c).init(rho=rho)
    x0 = np.concatenate([a.ravel() for a in o.df()])
    try:
        o.step(steps)
    except oracle.OracleError:
        return np.inf
    return np.abs(np.concatenate([a.ravel() for a in o.df()]) - x0).max()


def test_walls_lower_the_stable_viscosity_at_high_prandtl():
    """Finding: isothermal walls (Sec. 3, second-order extrapolation) make the
    ideal-gas rest state unstable at Pr = 7, tau = 0.8 for perturbations that
    vary along the wall, although the periodic analysis is neutral there.
    Perturbations that are uniform along the wall (the one-dimensional
    channel flows of Secs. 4.1, 4.2, which the paper runs up to Pr = 20 at
    this tau) stay at rounding level.  The decoupling EOS is stable with the
    same walls, and so is the ideal gas at Pr = 0.71 and at nu0 = 0.3."""
    nx, ny = 16, 32
    varying = 1.0 + 1e-12 * inputs.noise(3, nx * ny).reshape(ny, nx)
    uniform = 1.0 + 1e-12 * np.repeat(inputs.noise(3, ny)[:, None], nx, axis=1)
    assert spectral_radius(_case("ideal", 0.1, 7.0)) <= NEUTRAL
    assert _departure(_rest_channel(7.0, 0.1, 2), varying, 600) > 1e-6
    assert _departure(_rest_channel(7.0, 0.1, 2), uniform, 600) < 1e-11
    assert _departure(_rest_channel(0.71, 0.1, 2), varying, 600) < 1e-11
    assert _departure(_rest_channel(7.0, 0.3, 2), varying, 600) < 1e-11
    dec = _rest_channel(7.0, 0.1, 2)
    dec["eos"] = "decoupled"
    assert _departure(dec, varying, 600) < 1e-11


def _wall_state_radius(nu0, rho_b, T_b, reading, bulk_ratio=1.0, Pr=0.71):
    """Growth of a uniform rest state (rho_b, T_b) of an eps = 0.6 cavity with
    Sutherland viscosity, under a reading of the viscosity of Sec. 4:
    'local' nu = mu(T)/rho (the oracle's), 'rho0' nu = mu(T)/rho0.  The second
    is evaluated with the oracle by scaling nu0 and Pr by rho_b/rho0, which
    gives the same rates (s_p from mu/rho0, sigma_j from lambda) at rho_b."""
    scale = rho_b if reading == "rho0" else 1.0
    c = inputs.base_case(nx=4, ny=4, eos="ideal", nu0=nu0 * scale, Pr=Pr * scale,
                         bulk_ratio=bulk_ratio, visc_law="sutherland", suth_S=110.5 / 600.0)
    return spectral_radius(oracle.Oracle(c), rho_b, T_b)


@pytest.mark.parametrize("Ma", [0.05, 0.1])
def test_no_reading_stabilises_the_512_cavity_at_low_mach(Ma):
    """Sec. 4.3, Table 1 (Ra = 1e6 on 512^2, bulk ratio 1) at buoyancy Mach
    0.05 and 0.1: nu0 = Ma c_s L sqrt(Pr/Ra).  Both readings of the local
    viscosity (local rho or rho0) coincide at the reference state T0, rho0,
    which already grows at Ma 0.05; the cold-wall state (T = 0.4, rho = 2.5
    at the mean pressure) grows under either reading at both Mach numbers."""
    nu0 = inputs.cavity(N=512, Ra=1e6, Ma=Ma)["nu0"]
    cold = (1.0 / 0.4, 0.4)
    if Ma == 0.05:
        assert _wall_state_radius(nu0, 1.0, 1.0, "local") > 1.1
    for reading in ("local", "rho0"):
        assert _wall_state_radius(nu0, *cold, reading) > 1.05


def test_benchmark_viscosity_is_stable_at_the_reference_and_cold_wall():
    """The cavity viscosity used for the step benchmark (nu0 = 0.1, tau0 =
    0.8) keeps the reference and cold-wall rest states neutral."""
    assert _wall_state_radius(0.1, 1.0, 1.0, "local") <= NEUTRAL
    assert _wall_state_radius(0.1, 1.0 / 0.4, 0.4, "local") <= NEUTRAL
