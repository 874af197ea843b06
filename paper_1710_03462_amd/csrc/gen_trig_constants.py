"""Derive the argument-reduction constants of trig.h from pi itself.

pi is computed to 120 decimal digits with Machin's formula in integer
arithmetic; pi/2 is then cut into three doubles (Cody & Waite, "Software
Manual for the Elementary Functions", 1980): the first two keep 33
significant bits, so k * part is exact for |k| < 2^20, and the third is the
remainder rounded to 53 bits.  Prints C++ hex-float literals.
"""
from fractions import Fraction


def arctan_inv(x, digits):
    """arctan(1/x) * 10^digits, integer arithmetic."""
    scale = 10 ** (digits + 10)
    total, term, n, sign = 0, scale // x, 1, 1
    while term:
        total += sign * (term // n)
        term //= x * x
        n += 2
        sign = -sign
    return total // 10 ** 10


def pi_fraction(digits=120):
    return Fraction(16 * arctan_inv(5, digits) - 4 * arctan_inv(239, digits), 10 ** digits)


def truncate_bits(v, bits):
    """Truncate a positive Fraction to `bits` significant bits (exact as a double)."""
    e = 0
    while v >= 2:
        v /= 2
        e += 1
    while v < 1:
        v *= 2
        e -= 1
    m = int(v * 2 ** (bits - 1))
    return Fraction(m, 2 ** (bits - 1)) * Fraction(2) ** e


def main():
    half_pi = pi_fraction() / 2
    p1 = truncate_bits(half_pi, 33)
    p2 = truncate_bits(half_pi - p1, 33)
    p3 = float(half_pi - p1 - p2)
    two_over_pi = float(1 / half_pi)
    for name, v in (("kPio2Hi", float(p1)), ("kPio2Mid", float(p2)), ("kPio2Lo", p3),
                    ("kTwoOverPi", two_over_pi)):
        print(f"constexpr double {name} = {v.hex()};  // {v!r}")
    assert float(p1) == p1 and float(p2) == p2


if __name__ == "__main__":
    main()
