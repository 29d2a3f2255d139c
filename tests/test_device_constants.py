"""The device math constants are what their derivation gives (host-side check)."""
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_03484_amd", "csrc")


def _header_constants():
    vals = {}
    for f in ("dmath.hpp", "kepler.hpp"):
        for name, lit in re.findall(r"constexpr double (\w+) = (0x[0-9a-fA-Fp.+-]+);", open(os.path.join(CSRC, f)).read()):
            vals[name] = float.fromhex(lit)
    return vals


def test_reduction_constants_match_mpmath():
    sys.path.insert(0, CSRC)
    import gen_constants
    want = gen_constants.constants()
    have = _header_constants()
    for k, v in want.items():
        assert have[k] == v, k


def test_taylor_coefficients_are_inverse_factorials():
    import math
    text = open(os.path.join(CSRC, "dmath.hpp")).read()
    for name, sign, num, den in re.findall(r"constexpr double ([SC]\d+) = (-?)(1\.0) / (\d+\.0);", text):
        k = int(name[1:])
        assert float(den) == math.factorial(k), name
        assert (sign == "-") == (k % 4 in (2, 3)), name
