"""Stochastic rounding of the 16-bit storage formats, checked on the host
with the kernels' own code (lbm_rounding_byte, lbm_round_half_stochastic):
the random bytes are uniform and independent across steps, rows and
neighbouring nodes, and the rounding is unbiased to 1/512 of an FP16 unit in
the last place.  A biased byte (for instance the top byte of a product with
a constant, which cannot exceed that constant's top byte) turns the
rounding into a systematic drift of the stored DFs."""
import numpy as np
import pytest

from paper_1809_08683_amd import lbm


STEPS = 3000
NODES = ((0, 0), (1, 1), (517, 1023), (2047, 3))


def _bytes(prec, x, y, rows):
    return np.array([[lbm.rounding_byte(prec, x, y, t, q) for q in rows] for t in range(STEPS)], dtype=float)


@pytest.mark.parametrize("prec,rows", [("f16s", list(range(18))), ("f32g16", list(range(9, 18)))])
def test_rounding_bytes_are_uniform_and_independent(prec, rows):
    sigma = 255.0 / np.sqrt(12.0) / np.sqrt(STEPS)
    chi2_limit = 45.0       # 15 degrees of freedom: P(chi2 > 45) < 1e-4
    r_limit = 4.5 / np.sqrt(STEPS)
    prev = None
    for (x, y) in NODES:
        B = _bytes(prec, x, y, rows)
        assert B.min() >= 0 and B.max() <= 255
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
    # the bytes of a node's neighbour in x differ
    a, b = _bytes(prec, 10, 20, rows), _bytes(prec, 11, 20, rows)
    assert max(abs(np.corrcoef(a[:, j], b[:, j])[0, 1]) for j in range(len(rows))) < r_limit


def test_rows_without_16_bit_storage_get_no_byte():
    for t in (0, 1, 77):
        assert all(lbm.rounding_byte("f32g16", 5, 6, t, q) == 0 for q in range(9))
        assert all(lbm.rounding_byte(p, 5, 6, t, q) == 0 for p in ("f32", "f64") for q in range(18))
        assert lbm.rounding_byte("f16s", 5, 6, t, 18) == 0 and lbm.rounding_byte("f16s", 5, 6, t, -1) == 0
    assert any(lbm.rounding_byte("f16s", 5, 6, t, 0) != 0 for t in range(4))


def _fp16_neighbours(v):
    h = np.float16(v)
    if float(h) == v:
        return float(h), float(h)
    lo = h if float(h) < v else np.nextafter(h, np.float16(-np.inf))
    hi = np.nextafter(lo, np.float16(np.inf))
    return float(lo), float(hi)


def test_stochastic_rounding_is_unbiased():
    rng = np.random.default_rng(11)
    mags = np.exp(rng.uniform(np.log(1e-4), np.log(30.0), 300)).astype(np.float32)
    signs = np.where(rng.random(300) < 0.5, -1.0, 1.0).astype(np.float32)
    for v in (mags * signs).astype(np.float32):
        v = float(v)
        r = np.array([lbm.round_half_stochastic(v, u) for u in range(256)])
        lo, hi = _fp16_neighbours(v)
        assert set(np.unique(r)) <= {lo, hi}, (v, lo, hi, np.unique(r))
        assert all(float(np.float16(x)) == x for x in r)
        ulp = hi - lo if hi != lo else 0.0
        assert abs(r.mean() - v) <= ulp / 512 + 1e-7 * abs(v) * 2 ** -13, (v, r.mean() - v, ulp)
        # the fraction of roundings up follows the position of v between the neighbours
        if ulp > 0:
            assert abs((r == hi).mean() - (v - lo) / ulp) <= 1 / 256 + 1e-9


def test_representable_values_zero_and_sign():
    for v in (0.0, -0.0, 1.0, -0.5, 0.125, float(np.float16(0.3)), float(np.float16(-17.25))):
        assert all(lbm.round_half_stochastic(v, u) == v for u in range(0, 256, 5))
    for v in (0.3, 1e-3, 7.77):
        for u in (0, 100, 255):
            assert lbm.round_half_stochastic(-v, u) == -lbm.round_half_stochastic(v, u)
