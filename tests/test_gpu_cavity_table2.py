"""The differentially heated cavity of Sec. 4.3 against Table 2 ("Present"
rows) at the grids of Table 1: eps = 0.6, Pr = 0.71, gamma = 1.4,
Sutherland viscosity, first-order walls, FP64 path run to its steady state.
The mean hot-wall Nusselt number and the mean pressure p_ave* (the integral
of p_EOS / p0 over the cavity, trapezoidal weights on the node grid) must
agree with the printed values to 0.5 % and 0.2 %; measured: 0.06-0.2 % and
0.02-0.07 %.  (Ra >= 1e6 is out of reach at tau0 = 0.8, see the design
notes.)"""
import numpy as np
import pytest

from paper_1809_08683_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _steady_cavity(N, Ra, chunk=20000, cap=1000000, rtol=1e-7):
    c = inputs.cavity(N=N, Ra=Ra, eps=0.6, prec="f64", noise_seed=1)
    g = lbm.Context(c).init(**c["init"])
    prev, n = None, 0
    while n < cap:
        g.step(chunk)
        n += chunk
        nu = g.nusselt(0)
        if prev is not None and abs(nu - prev) < rtol * abs(nu):
            break
        prev = nu
    p = g.macros()["p"]
    g.close()
    w = np.ones(N)
    w[0] = w[-1] = 0.5
    p0 = 1.0 / 3.0          # p_EOS(rho0, T0) = rho0 R T0 with R = c_s^2 / T0
    p_ave = float((w[:, None] * w[None, :] * p).sum() / w.sum() ** 2 / p0)
    return nu, p_ave, n


@pytest.mark.parametrize("Ra", [1e3, 1e4, 1e5])
def test_cavity_against_table2(Ra, golden):
    t1, t2 = golden["cavity_table1"], golden["cavity_table2_present"]
    N = t1["N"][t1["Ra"].index(Ra)]
    i = t2["Ra"].index(Ra)
    nu, p_ave, n = _steady_cavity(N, Ra)
    e_nu = (nu - t2["Nu_ave"][i]) / t2["Nu_ave"][i]
    e_p = (p_ave - t2["p_ave"][i]) / t2["p_ave"][i]
    print(f"Ra={Ra:.0e} N={N}: {n} steps, Nu {nu:.5f} ({e_nu:+.2e}), p_ave {p_ave:.5f} ({e_p:+.2e})", flush=True)
    assert abs(e_nu) < 5e-3
    assert abs(e_p) < 2e-3
