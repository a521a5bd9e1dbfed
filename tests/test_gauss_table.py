"""The discrete Gaussian sampler's thresholds (Background, "Homomorphic
encryption": the error polynomials of keys and encryptions, sigma = 3.2).

Both sides invert the cumulative distribution of the discrete Gaussian
truncated at |x| <= 19: T[i] = floor(2^63 * CDF(i)).  The oracle evaluates it
in binary128, the library in double-double; both are pinned here to the exact
value computed with 60-digit decimal arithmetic, so a one-unit difference in
any threshold (which would make the two samplers disagree on some draws) fails.
Host only: no GPU involved."""
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import ckks

SIGMAS = [3.2, 3.19, 2.0, 2.5, 4.0, 6.0, 8.0]


def exact_table(sigma, K=19):
    getcontext().prec = 60
    s = Decimal(sigma)
    w = [(Decimal(1) if i == 0 else Decimal(2)) * (-(Decimal(i * i)) / (2 * s * s)).exp() for i in range(K + 1)]
    tot, acc, out = sum(w), Decimal(0), []
    for i in range(K):
        acc += w[i]
        out.append(int((acc / tot * (Decimal(2) ** 63)).to_integral_value(rounding="ROUND_FLOOR")))
    return out


def test_exact_table_closed_forms():
    # the pin itself: T[18] + the mass beyond 18 fills 2^63, T[0] is the mass at 0
    getcontext().prec = 60
    s = Decimal(3.2)
    w0 = Decimal(1)
    tot = w0 + 2 * sum((-(Decimal(i * i)) / (2 * s * s)).exp() for i in range(1, 20))
    T = exact_table(3.2)
    assert T[0] == int((w0 / tot * Decimal(2) ** 63).to_integral_value(rounding="ROUND_FLOOR"))
    assert all(a < b for a, b in zip(T, T[1:]))
    tail = 2 * (-(Decimal(361)) / (2 * s * s)).exp() / tot * Decimal(2) ** 63
    assert abs((Decimal(2) ** 63 - T[18]) - tail) < 1


@pytest.mark.parametrize("sigma", SIGMAS)
def test_oracle_table_exact(sigma):
    T = np.zeros(19, dtype=np.uint64)
    ckks.lib().orc_gauss_table(sigma, T.ctypes.data_as(ckks.u64p))
    assert [int(v) for v in T] == exact_table(sigma)


@pytest.mark.parametrize("sigma", SIGMAS)
def test_library_table_exact(sigma):
    from paper_2306_09189_amd import hecnn
    if not os.path.exists(hecnn.LIB_PATH):
        pytest.skip("library not built")
    assert [int(v) for v in hecnn.gauss_table(sigma)] == exact_table(sigma)


def test_library_rejects_small_sigma():
    from paper_2306_09189_amd import hecnn
    if not os.path.exists(hecnn.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(hecnn.HecError):
        hecnn.gauss_table(1.0)
