"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/lbm.h declares, and rejects invalid parameters before touching
the device."""
import ctypes as C
import os
import re

import pytest

from paper_1809_08683_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load_library()
    names = declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(lbm.exported_symbols()) <= set(names)


def test_workspace_bytes():
    lib = lbm.load_library()
    small = lib.lbm_workspace_bytes(16, 16, 1)
    big = lib.lbm_workspace_bytes(2048, 2048, 1)
    assert small > 0 and big > 2 * 18 * 2048 * 2048 * 4
    assert lib.lbm_workspace_bytes(2048, 2048, 2) < big < lib.lbm_workspace_bytes(2048, 2048, 0)
    assert lib.lbm_workspace_bytes(0, 16, 1) == 0 and lib.lbm_workspace_bytes(16, 16, 7) == 0


@pytest.mark.parametrize("mutate,msg", [
    (lambda c: c.update(nx=4), "at least 5"),
    (lambda c: c.update(Pr=0.0), "Pr"),
    (lambda c: c.update(nu0=-1.0), "nu0"),
    (lambda c: c.update(bulk_ratio=0.0), "bulk"),
    (lambda c: c.update(extrap_order=3), "extrap"),
    (lambda c: c.update(cubic=5), "cubic"),
    (lambda c: c["sides"][1].update(kind="periodic"), "opposite"),
    (lambda c: c["sides"][0].update(T=-1.0), "temperature"),
    (lambda c: c.update(eos="vdw", a=0.05, b=2.0), "van der Waals"),
])
def test_invalid_parameters_rejected_before_device_use(mutate, msg):
    case = inputs.cavity(N=16, Ra=1e4, prec="f32")
    mutate(case)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.Context(case)
    assert ei.value.status == lbm.EINVAL
    assert msg in str(ei.value)


def test_null_blocks_rejected():
    lib = lbm.load_library()
    h = C.c_void_p()
    assert lib.lbm_create(8, 8, None, 0.71, 1.4, None, None, None, C.byref(h)) == lbm.EINVAL
    lib.lbm_destroy(h)
    assert lib.lbm_last_error(None) == b"null context"
