"""GPU parity of the batched step: many independent lattices of uneven size
and parameters advanced by one launch per step (lbm_batch_create and the
lbm_case_* calls), against the FP64 CPU oracle run case by case, and against
single-case contexts on the same inputs.
"""
import numpy as np
import pytest

import oracle
from paper_1809_08683_amd import inputs, lbm

pytestmark = pytest.mark.gpu

P = inputs._periodic
W = inputs._side
FIELDS = ("rho", "ux", "uy", "T", "p")
BAR = {"f64": (1e-10, 1e-10), "f32": (2e-5, 2e-4), "f16s": (2e-3, 2e-2)}


def _cavity(N, ny=None, order=1, eps=0.3, fy=-1e-4):
    c = inputs.cavity(N=N, Ra=1e4, eps=eps, prec="f64")
    c["nu0"] = 0.1
    c["force"] = (0.0, fy)
    if ny is not None:
        c["ny"] = ny
    c["extrap_order"] = order
    return c


def mixed_cases():
    """Uneven shapes, all boundary kinds, all four equations of state."""
    return [
        _cavity(13, ny=11),
        inputs.couette(nx=7, ny=14, nu=0.1),
        inputs.base_case(nx=16, ny=12, nu0=0.1, force=(1e-4, -2e-4), per_mass=True),
        _cavity(131, ny=9, order=2),
        inputs.base_case(nx=12, ny=10, nu0=0.1, force=(0, -1e-4), per_mass=True,
                         sides=[W(T=1.05), W(T=0.95), P(), P()], extrap_order=1),
        inputs.base_case(nx=16, ny=12, nu0=0.1, eos="vdw", a=0.05, b=0.2),
        inputs.base_case(nx=16, ny=12, nu0=0.1, eos="cs", cv_rule=1),
        inputs.base_case(nx=1, ny=24, nu0=0.1, eos="decoupled", visc_law="linear"),
        _cavity(70, ny=37, eps=0.1),
    ]


def errors(gpu, ref):
    out = {}
    scale_u = max(np.abs(ref["ux"]).max(), np.abs(ref["uy"]).max(), 1e-300)
    for k in FIELDS:
        scale = scale_u if k in ("ux", "uy") else max(np.abs(ref[k]).max(), 1e-300)
        out[k] = float(np.abs(gpu[k] - ref[k]).max() / scale)
    return out


def check(gpu, ref, prec, label):
    e = errors(gpu, ref)
    print(label, " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    bar_s, bar_u = BAR[prec]
    for k, v in e.items():
        assert v <= (bar_u if k in ("ux", "uy") else bar_s), (label, k, v)


def with_prec(cases, prec):
    return [dict(c, prec=prec) for c in cases]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_matches_oracle_per_case(prec):
    cases = with_prec(mixed_cases(), prec)
    fields = [inputs.random_fields(c, 100 + k, du=0.01, drho=0.02, dT=0.02) for k, c in enumerate(cases)]
    print(f"batch of {len(cases)} cases, {prec}, 20 steps", flush=True)
    b = lbm.Batch(cases)
    for k, f in enumerate(fields):
        b.init(k, **f)
    b.step(20)
    assert b.flags() == [0] * len(cases)
    for k, (c, f) in enumerate(zip(cases, fields)):
        o = oracle.Oracle(c).init(**f)
        o.step(20)
        check(b.macros(k), o.macros(), prec, f"case {k} ({c['nx']}x{c['ny']} {c['eos']})")
    b.close()


def test_batch_equals_single_contexts():
    """Each case of a batch follows the same arithmetic as the case alone."""
    cases = with_prec(mixed_cases(), "f32")
    fields = [inputs.random_fields(c, 200 + k, du=0.01, drho=0.02, dT=0.02) for k, c in enumerate(cases)]
    b = lbm.Batch(cases)
    for k, f in enumerate(fields):
        b.init(k, **f)
    b.step(15)
    for k, (c, f) in enumerate(zip(cases, fields)):
        g = lbm.Context(c).init(**f).step(15)
        mb, mg = b.macros(k), g.macros()
        e = max(errors(mb, mg).values())
        print(f"case {k}: batch vs single max rel {e:.2e}", flush=True)
        assert e <= 1e-6, (k, e)
        g.close()
    b.close()


def test_batch_divergence_flags_only_that_case():
    """The paper's unstable set (Sec. 4.1) inside a batch: only its flag is
    raised and the other cases still follow the oracle."""
    U0 = 0.2 * np.sqrt(1 / 3)
    bad = inputs.poiseuille(nx=3, ny=33, U0=U0, nu=0.1, eos="ideal", a=0.0, b=0.0)
    bad["Pr"] = 0.1
    bad["sides"][3]["T"] = 1.0 + U0 ** 2 / ((3.5 / 3) * 10)
    good = [_cavity(13, ny=11), inputs.couette(nx=7, ny=14, nu=0.1)]
    cases = [good[0], bad, good[1]]
    fields = [inputs.random_fields(good[0], 7, du=0.01, drho=0.02, dT=0.02), None,
              inputs.random_fields(good[1], 8, du=0.01, drho=0.02, dT=0.02)]
    b = lbm.Batch(cases)
    for k, f in enumerate(fields):
        b.init(k, **(f or {}))
    steps = 0
    while b.flags()[1] == 0 and steps < 5000:
        b.step(100, allow_diverged=True)
        steps += 100
    print(f"unstable case flagged after {steps} steps", flush=True)
    assert b.flags() == [0, 1, 0]
    for k in (0, 2):
        o = oracle.Oracle(cases[k]).init(**fields[k])
        o.step(steps)
        check(b.macros(k), o.macros(), "f64", f"case {k} after {steps} steps")
    b.close()


def test_batch_sweep_configuration():
    """The uneven sweep of 64 cavities (N in {128..1024}, Ra log-uniform in
    [1e3, 1e8], eps in [0.1, 0.6], Pr in {0.71, 1, 7}), FP32, in one batch:
    no case diverges in 10 steps, every case keeps its mass, and one case of
    every size (1024^2 included) agrees with the oracle."""
    cases = inputs.batch_cases(seed=2, n=64, prec="f32")
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    print(f"64-case sweep: {nodes} nodes", flush=True)
    b = lbm.Batch(cases)
    for k, c in enumerate(cases):
        b.init(k, rho=1.0 + 1e-6 * inputs.noise(3 + k, c["nx"] * c["ny"]).reshape(c["ny"], c["nx"]))
    m0 = [b.totals(k)[0] for k in range(len(cases))]
    b.step(10)
    assert b.flags() == [0] * len(cases)
    for k in range(len(cases)):
        m1 = b.totals(k)[0]
        assert abs(m1 - m0[k]) / m0[k] < 1e-6, (k, m0[k], m1)
    sizes = [c["nx"] for c in cases]
    picks = [sizes.index(n) for n in (128, 256, 512, 1024) if n in sizes]
    assert len(picks) == 4
    for k in picks:
        c = cases[k]
        rho0 = 1.0 + 1e-6 * inputs.noise(3 + k, c["nx"] * c["ny"]).reshape(c["ny"], c["nx"])
        o = oracle.Oracle(c).init(rho=rho0)
        o.step(10)
        check(b.macros(k), o.macros(), "f32", f"sweep case {k} N={c['nx']} Ra={c['Ra']:.3g}")
    b.close()


def test_batch_step_and_nusselt_in_survey_form():
    """lbm_batch_step / lbm_batch_nusselt: every case's flag and Nu through
    the x = 0 wall, NaN for the diverged channel (the paper's unstable set of
    Sec. 4.1, Pr = 0.1, which has no x-walls anyway), the cavities' equal to
    lbm_case_nusselt."""
    U0 = 0.2 * np.sqrt(1 / 3)
    bad = inputs.base_case(nx=3, ny=33, eos="ideal", nu0=0.1, Pr=0.1, force=(8 * 0.1 * U0 / 32 ** 2, 0.0),
                           sides=[P(), P(), W(T=1.0), W(T=1.0 + U0 ** 2 / ((3.5 / 3) * 10))], extrap_order=2)
    good = [_cavity(13, ny=11), _cavity(40, ny=24, eps=0.2)]
    cases = [good[0], bad, good[1]]
    b = lbm.Batch(cases)
    for k in range(3):
        b.init(k)
    for _ in range(50):
        b.batch_step(100)
        if b.flags()[1]:
            break
    b.batch_step(10)
    nu, dv = b.batch_nusselt(0)
    assert dv == [0, 1, 0]
    assert np.isnan(nu[1])
    for k in (0, 2):
        assert nu[k] == b.nusselt(k, 0)
    b.close()
