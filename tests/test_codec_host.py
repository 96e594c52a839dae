"""Host-side checks of the 16-bit storage arithmetic the kernels rely on
(no GPU): the fixed-point value of an FP16 code, 2^(40 - kg) times the code's
value for the power-of-two scales kg = 0..16 the library picks, is an exact
FP32 product -- equal, for every finite code, to the FP64 product rounded to
an integer -- and the sum of eight such values is exact in FP64."""
import numpy as np


def test_fp16_fixed_point_is_an_exact_fp32_product():
    codes = np.arange(65536, dtype=np.uint16)
    v = codes.view(np.float16).astype(np.float32)
    fin = np.isfinite(v)
    v = v[fin]
    for kg in range(17):
        s32 = np.float32(2.0 ** (40 - kg))
        a = (v * s32).astype(np.float64)
        b = np.rint(v.astype(np.float64) * 2.0 ** (40 - kg))
        assert np.array_equal(a, b), kg
        assert np.all(np.abs(a) < 2.0 ** 57)


def test_eight_fixed_point_values_sum_exactly():
    rng = np.random.default_rng(0)
    codes = rng.integers(0, 65536, size=(100000, 8), dtype=np.uint16)
    v = codes.view(np.float16).astype(np.float64)
    ok = np.isfinite(v).all(axis=1)
    v = v[ok] * 2.0 ** 30  # kg = 10
    exact = [sum(int(x) for x in row) for row in v[:2000]]
    assert all(int(s) == e for s, e in zip(v[:2000].sum(axis=1), exact))
