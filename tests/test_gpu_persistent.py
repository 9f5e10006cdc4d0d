"""Persistent stepping (lbm_step_ex with LBM_STEP_PERSISTENT): n steps in
one launch with per-case step barriers instead of launch boundaries.  It
must give bitwise the state of plain launches, alone and replayed as a
captured graph with eager work in between, in every storage format and
launch-configuration variant, on the mixed batch (uneven sizes, walls,
periodic axes) and a single cavity; a wait that cannot be satisfied ends
the call with an error instead of a hang (forced from the host with a
spin limit of zero polls)."""
import numpy as np
import pytest

from paper_1809_08683_amd import inputs, lbm
from test_gpu_runtime import FIELDS, _batch, _cavity, _same

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f64", "f16s", "f32g16"])
def test_persistent_equals_plain_launches(prec):
    ref, cases = _batch(prec)
    b, _ = _batch(prec)
    for n in (5, 1, 6, 7):
        print(f"{prec}: persistent {n} steps", flush=True)
        ref.step(n)
        b.step_ex(n, persistent=True)
        assert b.time == ref.time
        _same(ref, b, len(cases))
    ref.close()
    b.close()


@pytest.mark.parametrize("prec", ["f32", "f32g16"])
def test_persistent_graph_replays_equal_plain_launches(prec):
    ref, cases = _batch(prec)
    g, _ = _batch(prec)
    for n in (6, 6, 5, 5, 6):
        ref.step(n)
        g.step_ex(n, graph=True, persistent=True)
        _same(ref, g, len(cases))
        assert [g.totals(k) for k in range(len(cases))] == [ref.totals(k) for k in range(len(cases))]
    single = lbm.Context(dict(_cavity(200, ny=130), prec=prec)).init()
    plain = lbm.Context(dict(_cavity(200, ny=130), prec=prec)).init()
    for _ in range(3):
        single.step_ex(10, graph=True, persistent=True)
        plain.step(10)
    m1, m2 = single.macros(), plain.macros()
    for f in FIELDS:
        assert np.array_equal(m1[f], m2[f])


def test_persistent_in_every_variant():
    for variant in range(5):
        ref, cases = _batch("f32")
        b, _ = _batch("f32")
        b.set_launch_config(variant, 1.0, 4)
        print(f"variant {variant}", flush=True)
        ref.step(7)
        b.step_ex(7, persistent=True)
        _same(ref, b, len(cases))
        ref.close()
        b.close()


def test_persistent_wait_gives_up_instead_of_hanging():
    b, cases = _batch("f32")
    b.set_persistent_spin_limit(0)
    with pytest.raises(lbm.LBMError) as ei:
        b.step_ex(4, persistent=True)
    assert ei.value.status == lbm.EDEVICE
    with pytest.raises(lbm.LBMError):
        b.step(1)                       # every case must be initialised again
    b.set_persistent_spin_limit(1 << 24)
    for k, c in enumerate(cases):
        b.init(k, **inputs.random_fields(c, 300 + k, du=0.01, drho=0.02, dT=0.02))
    ref, _ = _batch("f32")
    ref.step(4)
    b.step_ex(4, persistent=True)
    _same(ref, b, len(cases))
