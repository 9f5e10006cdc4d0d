"""Stochastic rounding of the 16-bit storage formats, checked on the host:
the random operands the kernels use (computed with the kernels' code by
lbm_rounding_operand) have uniform, independent top bits across steps,
rows and neighbouring nodes, and the library's model of the device's
rounding (lbm_round_half_stochastic; the device is held to the model
bitwise in tests/test_gpu_rounding.py) is unbiased.  A biased operand (for
instance one whose top byte cannot exceed some constant's) turns the
rounding into a systematic drift of the stored DFs."""
import numpy as np
import pytest

from paper_1809_08683_amd import lbm

STEPS = 3000
NODES = ((0, 0), (1, 1), (517, 1023), (2047, 3))


def _top_bytes(prec, x, y, rows):
    """Top 8 bits of each operand (the rounding depends on the top bits)."""
    return np.array([[lbm.rounding_operand(prec, x, y, t, q) >> 24 for q in rows] for t in range(STEPS)],
                    dtype=float)


def _top_fields(prec, x, y, rows, bits=10):
    return np.array([[lbm.rounding_operand(prec, x, y, t, q) >> (32 - bits) for q in rows] for t in range(STEPS)],
                    dtype=np.int64)


@pytest.mark.parametrize("prec,rows", [("f16s", list(range(18))), ("f32g16", list(range(9, 18)))])
def test_rounding_operands_are_uniform_and_independent(prec, rows):
    sigma = 255.0 / np.sqrt(12.0) / np.sqrt(STEPS)
    chi2_limit = 45.0       # 15 degrees of freedom: P(chi2 > 45) < 1e-4
    r_limit = 4.5 / np.sqrt(STEPS)
    prev = None
    for (x, y) in NODES:
        B = _top_bytes(prec, x, y, rows)
        for j in range(len(rows)):
            u = B[:, j]
            assert abs(u.mean() - 127.5) < 4.5 * sigma, (prec, x, y, rows[j], u.mean())
            hist = np.bincount((u // 16).astype(int), minlength=16)
            e = STEPS / 16
            assert ((hist - e) ** 2 / e).sum() < chi2_limit, (prec, x, y, rows[j])
            assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < r_limit, (prec, x, y, rows[j])
        C = np.corrcoef(B.T)
        np.fill_diagonal(C, 0.0)
        assert np.abs(C).max() < r_limit, (prec, x, y)
        if prev is not None:
            assert max(abs(np.corrcoef(prev[:, j], B[:, j])[0, 1]) for j in range(len(rows))) < r_limit
        prev = B
    a, b = _top_bytes(prec, 10, 20, rows), _top_bytes(prec, 11, 20, rows)
    assert max(abs(np.corrcoef(a[:, j], b[:, j])[0, 1]) for j in range(len(rows))) < r_limit


@pytest.mark.parametrize("prec,rows", [("f16s", list(range(18))), ("f32g16", list(range(9, 18)))])
def test_operands_of_a_node_share_no_top_bits(prec, rows):
    """The top 10 bits of a node's operands come from disjoint bits of its
    random words, so no two values of a node round alike by construction:
    their fields agree only as often as independent uniform 10-bit numbers."""
    F = _top_fields(prec, 3, 4, rows)
    n = len(rows)
    bits = (F[:, :, None] >> np.arange(10)[None, None, :]) & 1          # [step, value, bit]
    limit = 5 * 0.5 / np.sqrt(STEPS)
    for i in range(n):
        for j in range(i + 1, n):
            same = np.mean(F[:, i] == F[:, j])
            assert same < 10.0 / 1024, (prec, rows[i], rows[j], same)
            # no bit of one field follows a bit of the other (a shared bit agrees always)
            agree = np.mean(bits[:, i, :, None] == bits[:, j, None, :], axis=0)
            assert np.abs(agree - 0.5).max() < limit, (prec, rows[i], rows[j], np.abs(agree - 0.5).max())


def test_rows_without_16_bit_storage_get_no_operand():
    for t in (0, 1, 77):
        assert all(lbm.rounding_operand("f32g16", 5, 6, t, q) == 0 for q in range(9))
        assert all(lbm.rounding_operand(p, 5, 6, t, q) == 0 for p in ("f32", "f64") for q in range(18))
        assert lbm.rounding_operand("f16s", 5, 6, t, 18) == 0 and lbm.rounding_operand("f16s", 5, 6, t, -1) == 0
    assert any(lbm.rounding_operand("f16s", 5, 6, t, 0) != 0 for t in range(4))


def _fp16_neighbours(v):
    h = np.float16(v)
    if float(h) == v:
        return float(h), float(h)
    lo = h if abs(float(h)) < abs(v) else np.nextafter(h, np.float16(0))
    hi = np.nextafter(lo, np.float16(np.copysign(np.inf, v)))
    return float(lo), float(hi)


def _operands_256():
    """256 operands whose top bytes take every value, each centred in its
    bucket: the mean of a rounding over them is exact to 1/512 ulp."""
    return [(k << 24) | (1 << 23) for k in range(256)]


def test_stochastic_rounding_model_is_unbiased():
    rng = np.random.default_rng(11)
    mags = np.exp(rng.uniform(np.log(2.0 ** -27), np.log(30.0), 400)).astype(np.float32)
    signs = np.where(rng.random(400) < 0.5, -1.0, 1.0).astype(np.float32)
    ops = _operands_256()
    for v in (mags * signs).astype(np.float32):
        v = float(v)
        r = np.array([lbm.round_half_stochastic(v, o) for o in ops])
        lo, hi = _fp16_neighbours(v)
        assert set(np.unique(r)) <= {lo, hi}, (v, lo, hi, np.unique(r))
        assert all(float(np.float16(x)) == x for x in r)
        ulp = abs(hi - lo)
        assert abs(r.mean() - v) <= ulp / 512 + 1e-12 * abs(v), (v, r.mean() - v, ulp)
        if ulp > 0:
            assert abs((r == hi).mean() - abs(v - lo) / ulp) <= 1 / 256 + 1e-9


def test_model_edges():
    for v in (0.0, 1.0, -0.5, 0.125, float(np.float16(0.3)), float(np.float16(-17.25)), 2.0 ** -24, 3 * 2.0 ** -24):
        assert all(lbm.round_half_stochastic(v, o) == v for o in (0, 1 << 31, 0xFFFFFFFF))
    for v in (0.3, 1e-3, 7.77, 3e-6):
        for o in (0, 0x80000000, 0xFFFFFFFF):
            assert lbm.round_half_stochastic(-v, o) == -lbm.round_half_stochastic(v, o)
        lo, hi = _fp16_neighbours(v)
        assert lbm.round_half_stochastic(v, 0) == lo and lbm.round_half_stochastic(v, 0xFFFFFFFF) == hi
