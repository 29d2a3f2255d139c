"""Regenerate the reduction constants of dmath.hpp / kepler.hpp from 50-digit pi.

pi/2 (and 2 pi) is split into its nearest double and the nearest double to the
remainder; 2/pi and 1/(2 pi) are rounded once.  Prints C++ hex-float literals.
"""
import mpmath


def split(x):
    hi = float(x)
    lo = float(x - mpmath.mpf(hi))
    return hi, lo


def constants():
    mpmath.mp.dps = 50
    pio2_hi, pio2_lo = split(mpmath.pi / 2)
    twopi_hi, twopi_lo = split(2 * mpmath.pi)
    return {
        "PIO2_HI": pio2_hi, "PIO2_LO": pio2_lo, "TWO_OVER_PI": float(2 / mpmath.pi),
        "TWO_PI_HI": twopi_hi, "TWO_PI_LO": twopi_lo, "INV_TWO_PI": float(1 / (2 * mpmath.pi)),
    }


if __name__ == "__main__":
    for k, v in constants().items():
        print(f"constexpr double {k} = {v.hex()};")
