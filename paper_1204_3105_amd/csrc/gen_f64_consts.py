"""Double-double constants of the FP64 near field (near.hip), from series in
60-digit decimal arithmetic: ln 2 = 2 atanh(1/3), pi = 16 atan(1/5) -
4 atan(1/239) (Machin).  ln 2 is split so that its high part has 32
significant bits (e * ln2_hi is exact for |e| < 2^21).  c = sqrt(1/2)
rounded to double is the logarithm's reduction point; ln_c = ln c, formed as
ln(c sqrt 2) - ln(2)/2 with ln(c sqrt 2) = 2 atanh((y - 1)/(y + 1)),
y = c sqrt 2."""
import math
from decimal import Decimal, getcontext

getcontext().prec = 60


def atanh_inv(x, n=200):
    s, p = Decimal(0), x
    for k in range(n):
        s += p / (2 * k + 1)
        p *= x * x
    return s


def atan_inv(n, terms=200):
    x = Decimal(1) / n
    s, p = Decimal(0), x
    for k in range(terms):
        s += (p / (2 * k + 1)) * (1 if k % 2 == 0 else -1)
        p *= x * x
    return s


def split(v):
    hi = float(v)
    return hi, float(v - Decimal(hi))


if __name__ == "__main__":
    ln2 = 2 * atanh_inv(Decimal(1) / 3)
    pi = 16 * atan_inv(5) - 4 * atan_inv(239)
    m, e = math.frexp(float(ln2))
    hi = math.ldexp(math.floor(m * 2 ** 32), e - 32)
    print("ln2_hi %r ln2_lo %r" % (hi, float(ln2 - Decimal(hi))))
    for name, v in (("pi", pi), ("pi_2", pi / 2), ("pi_6", pi / 6)):
        print("%s %r %r" % ((name,) + split(v)))
    print("inv_sqrt3 %r tan_pi_12 %r" % (float(1 / Decimal(3).sqrt()), float(2 - Decimal(3).sqrt())))
    c = math.sqrt(0.5)
    y = Decimal(c) * Decimal(2).sqrt()
    print("sqrt_half %r ln_c %r" % (c, float(2 * atanh_inv((y - 1) / (y + 1)) - ln2 / 2)))
