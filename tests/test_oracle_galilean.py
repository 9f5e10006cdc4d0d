"""Pins of the cubic velocity corrections R, T.grad(rho) and X.grad(p) of
Sec. 2.1 (no GPU).

Sec. 2.1 introduces R, T and X, with the cubic and quartic terms of m^eq and
F_m, to remove the additional cubic velocity terms from the recovered
momentum equation.  Those terms are what breaks Galilean invariance of the
lattice's viscous dynamics: linearised about a uniform flow U, the exact
Navier-Stokes decay of a shear wave (rate nu k^2) and of a sound wave
(rate (nu + bulk) k^2 / 2 for the decoupling EOS, bulk = nu here) do not
depend on U.  A term cubic in u shows up in the linearised lattice dynamics
as a U^2 error of the decay rates (from 3 rho U^2 du) and a U^3 error (from
U^3 grad(rho)).  So with the corrections the continuum part of both
coefficients vanishes, and without them it does not.

Measurement: a small-amplitude wave on a periodic lattice with mean flow
s*udir; the decay rate of its complex Fourier amplitude is fitted over a
time window.  Even part e(s) = (r(s) + r(-s))/2 - r(0), odd part
d(s) = (r(s) - r(-s))/2, both relative to r(0).  The U^2 coefficient comes
from s = 0.05, 0.1 (e = a2 s^2 + a4 s^4), the U^3 coefficient from s = 0.1,
0.2 (d = a1 s + a3 s^3).  Lattice (k^2) errors are removed by Richardson
extrapolation over N = 32 and 64 (the wave number halves).

Which entries each configuration exercises: shear waves with k along x
strain p_xy (R18, R88), along the diagonal p_xx (R17, R77); sound waves add
the bulk moment e (R11, R71, R81) and density and pressure gradients
parallel or oblique to U (T and X, rows 1, 7, 8).  Every single-entry sign
flip of R, T or X, the (1 - k) factor of T_1 and switching T and X off each
fail at least one of these tests (mutation table in the design notes).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1809_08683_amd import inputs

NU = 0.05


def _rate(kind, kdir, U, N, cubic=2, amp=1e-6):
    """Fitted decay rate / k^2 of a shear or (right-going) sound wave."""
    sc = (N // 32) ** 2
    t1, t2, dt = 40 * sc, 240 * sc, 8 * sc
    k = 2 * np.pi * np.asarray(kdir, float) / N
    kk = np.linalg.norm(k)
    kn = k / kk
    tn = np.array([-kn[1], kn[0]])
    c = inputs.base_case(nx=N, ny=N, eos="decoupled", nu0=NU, Pr=0.71, cubic=cubic)
    o = oracle.Oracle(c)
    y, x = np.mgrid[0:N, 0:N]
    ph = k[0] * x + k[1] * y
    cs = np.sqrt(1.0 / 3.0)
    if kind == "sound":
        dp = amp * np.cos(ph)
        o.init(rho=1 + dp / cs ** 2, ux=U[0] + dp / cs * kn[0], uy=U[1] + dp / cs * kn[1])
    else:
        o.init(ux=U[0] + amp * tn[0] * np.sin(ph), uy=U[1] + amp * tn[1] * np.sin(ph))
    o.step(t1)
    ts, amps = [], []
    while True:
        m = o.macros()
        if kind == "sound":
            un = (m["ux"] - U[0]) * kn[0] + (m["uy"] - U[1]) * kn[1]
            q = (m["p"] - 1.0 / 3.0) + cs * m["rho"] * un     # right-going characteristic
        else:
            q = (m["ux"] - U[0]) * tn[0] + (m["uy"] - U[1]) * tn[1]
        ts.append(o.time)
        amps.append(abs((q * np.exp(-1j * ph)).mean()))
        if o.time >= t2:
            break
        o.step(dt)
    return -np.polyfit(ts, np.log(amps), 1)[0] / kk ** 2


def _coefficients(kind, kdir, udir, N, cubic=2, odd=True):
    """(a2, a3): U^2 and U^3 coefficients of the relative decay-rate error."""
    ss = (0.05, 0.1, 0.2) if odd else (0.05, 0.1)
    jobs = [(0.0, 0.0)] + [(sg * s * udir[0], sg * s * udir[1]) for s in ss for sg in (1, -1)]
    with ThreadPoolExecutor(max_workers=8) as ex:    # the oracle releases the GIL
        r = list(ex.map(lambda U: _rate(kind, kdir, U, N, cubic), jobs))
    r0, rs = r[0], dict(zip([(s, sg) for s in ss for sg in (1, -1)], r[1:]))
    e = {s: ((rs[s, 1] + rs[s, -1]) / 2 - r0) / r0 for s in ss}
    a2 = (16 * e[0.05] - e[0.1]) / (16 * 0.05 ** 2 - 0.1 ** 2)
    if not odd:
        return a2, 0.0
    d = {s: (rs[s, 1] - rs[s, -1]) / (2 * r0) for s in (0.1, 0.2)}
    a3 = (d[0.2] - 2 * d[0.1]) / (0.2 ** 3 - 2 * 0.1 ** 3)
    return a2, a3


def _continuum(kind, kdir, udir, cubic=2):
    a32 = np.array(_coefficients(kind, kdir, udir, 32, cubic))
    a64 = np.array(_coefficients(kind, kdir, udir, 64, cubic))
    return (4 * a64 - a32) / 3


@pytest.mark.parametrize("kdir", [(1, 0), (1, 1)])
def test_shear_viscosity_has_no_quadratic_velocity_error(kdir):
    """Shear waves (k along x: p_xy strain; k diagonal: p_xx strain) with an
    oblique mean flow: the viscosity's U^2 error vanishes with R (within the
    small U^4 leak of the fit) and is O(10) without the corrections."""
    udir = (0.8, 0.6)
    a2, _ = _coefficients("shear", kdir, udir, 32, cubic=2, odd=False)
    a2_off, _ = _coefficients("shear", kdir, udir, 32, cubic=0, odd=False)
    assert abs(a2) < 0.5
    assert abs(a2_off) > 5.0


SOUND = [((1, 0), (0.8, 0.6)), ((1, 0), (0.6, -0.8)),
         ((0, 1), (0.6, 0.8)), ((0, 1), (-0.8, 0.6)),
         ((1, 1), (0.8, 0.6)), ((1, 1), (0.6, -0.8))]


@pytest.mark.parametrize("kdir,udir", SOUND)
def test_sound_attenuation_has_no_quadratic_or_cubic_velocity_error(kdir, udir):
    """Sound waves (bulk and normal strain, density and pressure gradients)
    with a mean flow at an angle: continuum U^2 and U^3 coefficients of the
    attenuation error vanish with R, T and X."""
    a2, a3 = _continuum("sound", kdir, udir)
    assert abs(a2) < 0.4
    assert abs(a3) < 0.6


def test_sound_pin_detects_the_uncorrected_scheme():
    """Without R, T and X the same measurement shows the cubic terms: a U^2
    coefficient of about 24 for the diagonal wave."""
    a2, _ = _continuum("sound", (1, 1), (0.8, 0.6), cubic=0)
    assert abs(a2) > 5.0
