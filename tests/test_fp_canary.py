"""Build canary: the oracle must be compiled without multiply-add contraction,
otherwise bit-exact parity with the GPU decoder is not defined."""
import numpy as np

import oracle


def test_no_fma_contraction():
    a = np.float32(1.0) + np.float32(2.0 ** -12)
    b = a
    c = -(np.float32(1.0) + np.float32(2.0 ** -11))
    two_roundings = np.float32(np.float32(a * b) + c)  # a*b loses its 2^-24 term
    fused = np.float32(float(a) * float(b) + float(c))  # 2^-24, exact in double
    assert two_roundings != fused
    assert oracle.fp_canary(a, b, c) == two_roundings
