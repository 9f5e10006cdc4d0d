"""GPU tests of the launch machinery around the step: compiled kernel
variants and work-list settings (lbm_set_launch_config), graph-captured
stepping (lbm_step_ex with LBM_STEP_GRAPH), the autotuner with its cache
(lbm_autotune) and the record of when a divergence was first seen.  The
physics may not depend on any of it: every result is compared bitwise with
plain one-launch-per-step stepping in the default configuration."""
import json

import numpy as np
import pytest

from paper_1809_08683_amd import inputs, lbm

pytestmark = pytest.mark.gpu

P = inputs._periodic
W = inputs._side
FIELDS = ("rho", "ux", "uy", "T", "p")


def _cavity(N, ny=None, order=1, eps=0.3):
    c = inputs.cavity(N=N, Ra=1e4, eps=eps, prec="f32")
    c["nu0"] = 0.1
    c["force"] = (0.0, -1e-4)
    if ny is not None:
        c["ny"] = ny
    c["extrap_order"] = order
    return c


def mixed(prec):
    cases = [_cavity(13, ny=11), inputs.couette(nx=7, ny=14, nu=0.1), _cavity(131, ny=9, order=2),
             inputs.base_case(nx=16, ny=12, nu0=0.1, eos="vdw", a=0.05, b=0.2),
             inputs.base_case(nx=12, ny=10, nu0=0.1, force=(0, -1e-4), per_mass=True,
                              sides=[W(T=1.05), W(T=0.95), P(), P()], extrap_order=1),
             _cavity(200, ny=70, eps=0.2)]
    return [dict(c, prec=prec) for c in cases]


def _batch(prec, seed0=300):
    cases = mixed(prec)
    b = lbm.Batch(cases)
    for k, c in enumerate(cases):
        b.init(k, **inputs.random_fields(c, seed0 + k, du=0.01, drho=0.02, dT=0.02))
    return b, cases


def _same(b1, b2, n):
    for k in range(n):
        m1, m2 = b1.macros(k), b2.macros(k)
        for f in FIELDS:
            assert np.array_equal(m1[f], m2[f]), (k, f)


@pytest.mark.parametrize("prec", ["f32", "f64", "f16s", "f32g16"])
def test_every_launch_configuration_gives_the_same_state(prec):
    ref, cases = _batch(prec)
    ref.step(12)
    for variant in range(5):
        for xw_scale, bands in ((1.0, 4), (0.85, 1), (1.2, 16)):
            print(f"{prec}: variant {variant} xw_scale {xw_scale} bands {bands}", flush=True)
            b, _ = _batch(prec)
            b.set_launch_config(variant, xw_scale, bands)
            b.step(5)
            b.set_launch_config((variant + 1) % 5, 1.0, 4)   # switching mid-run keeps the state
            b.step(7)
            _same(ref, b, len(cases))
            b.close()


@pytest.mark.parametrize("prec", ["f32", "f64", "f16s", "f32g16"])
def test_graph_replay_equals_plain_launches(prec):
    """The captured graph of n steps is replayed several times with eager
    work (macro and totals reads) in between; every replay matches plain
    stepping, for an even and an odd n (the odd graph starts from either
    buffer).  In the 16-bit formats this also checks the device step
    counter of the stochastic rounding, which the replays advance."""
    ref, cases = _batch(prec)
    g, _ = _batch(prec)
    for n in (6, 6, 5, 5, 5, 6):
        ref.step(n)
        g.step_ex(n, graph=True)
        assert g.time == ref.time
        _same(ref, g, len(cases))
        assert [g.totals(k) for k in range(len(cases))] == [ref.totals(k) for k in range(len(cases))]
    single = lbm.Context(dict(_cavity(64, ny=48), prec=prec)).init()
    plain = lbm.Context(dict(_cavity(64, ny=48), prec=prec)).init()
    for _ in range(3):
        single.step_ex(10, graph=True)
        plain.step(10)
    m1, m2 = single.macros(), plain.macros()
    for f in FIELDS:
        assert np.array_equal(m1[f], m2[f])


def test_autotune_keeps_the_state_and_uses_its_cache(tmp_path):
    cache = str(tmp_path / "tune.json")
    ref, cases = _batch("f32")
    b, _ = _batch("f32")
    ref.step(4)
    b.step(4)
    before = [b.macros(k) for k in range(len(cases))]
    r = b.autotune(trial_steps=5, cache_path=cache)
    print("tuned:", r, flush=True)
    assert r["trials"] == 5 * 3 * 4 and r["from_cache"] == 0
    assert r["ms_per_step"] <= r["default_ms_per_step"] * 1.0001
    assert (r["variant"], r["xw_scale"], r["bands_per_xcd"]) == (0, 1.0, 4) or \
        r["ms_per_step"] < 0.99 * r["default_ms_per_step"]
    assert b.time == 4
    for k in range(len(cases)):
        m = b.macros(k)
        for f in FIELDS:
            assert np.array_equal(m[f], before[k][f])
    ref.step(9)
    b.step(9)
    _same(ref, b, len(cases))
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, e), = entries.items()
    assert "|f32|n6|" in key and e["variant"] == r["variant"]
    b2, _ = _batch("f32")
    r2 = b2.autotune(trial_steps=5, cache_path=cache)
    assert r2["from_cache"] == 1 and r2["trials"] == 0 and r2["variant"] == r["variant"]


def test_divergence_time_is_recorded():
    """The paper's unstable set (Sec. 4.1) in a batch: the call that first
    sees the case diverged is recorded; the other cases report -1."""
    U0 = 0.2 * np.sqrt(1 / 3)
    bad = inputs.poiseuille(nx=3, ny=33, U0=U0, nu=0.1, eos="ideal", a=0.0, b=0.0)
    bad["Pr"] = 0.1
    bad["sides"][3]["T"] = 1.0 + U0 ** 2 / ((3.5 / 3) * 10)
    b = lbm.Batch([_cavity(13, ny=11), dict(bad, prec="f32")])
    b.init(0)
    b.init(1)
    t_first = None
    for _ in range(60):
        b.step(100, allow_diverged=True)
        if b.flags()[1] and t_first is None:
            t_first = b.time
    assert t_first is not None
    assert b.diverged_at(1) == t_first and b.diverged_at(0) == -1
