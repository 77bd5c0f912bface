"""The exact FP32 quotient the mixed-radix passes use instead of an integer
division (FastDiv in pss_kernels.hip): trunc((float(x) + 0.5f) * (1.0f / d))
must equal floor(x / d) for every 0 <= x < 2^21 and every divisor the
kernels take (line lengths and their sub-lengths 2^a 3^b 5^c up to 4096,
lines per block up to 64).  Emulated here in IEEE single precision with
numpy, whose float32 division and multiplication round to nearest like the
device's."""

import numpy as np


def _divisors():
    ds = set(range(1, 65))
    for a in range(13):
        for b in range(8):
            for c in range(6):
                v = 2 ** a * 3 ** b * 5 ** c
                if v <= 4096:
                    ds.add(v)
    return sorted(ds)


def test_fp32_quotient_is_exact_below_2_21():
    x = np.arange(1 << 21, dtype=np.int64)
    xf = x.astype(np.float32) + np.float32(0.5)
    for d in _divisors():
        rd = np.float32(1.0) / np.float32(d)
        q = (xf * rd).astype(np.int64)  # truncation toward zero, as the device's conversion
        assert np.array_equal(q, x // d), d
