"""Polynomials of the FP64 near field's logarithm and arctangent (near.hip).

Both functions are reduced to a short interval and a series remainder there:
  ln m = 2 atanh(s) = 2 s (1 + z P(z)),   z = s^2, s = (m - 1)/(m + 1),
         m in [sqrt(1/2), sqrt(2)):  z in [0, (3 - 2 sqrt2)^2];
  atan t = t (1 + w Q(w)),                w = t^2, |t| <= tan(pi/12):
         w in [0, (2 - sqrt3)^2].
P and Q are fitted here instead of truncating the Taylor series
P = sum z^k/(2k+3), Q = sum (-1)^(k+1) w^k/(2k+3): the weighted minimax
polynomial (weight z, resp. w, since that is how the remainder's error
reaches the result) of the given degree, by Lawson's iteratively reweighted
least squares on 600 Chebyshev nodes in 50-digit arithmetic (mpmath).
Prints the C initializers (coefficient k of z^k) and the error bound
max |z (P_fit - P)| of each fit, and checks the whole function in float64
Horner evaluation against mpmath on a dense grid (max error in ulp of the
result).

    python gen_f64_poly.py
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 50
LN_DEG = 6      # 7 coefficients: max |z dP| about 1.2e-18
ATAN_DEG = 7    # 8 coefficients: max |w dQ| about 1.6e-17


def p_ln(z):
    if z == 0:
        return mp.mpf(1) / 3
    s = mp.sqrt(z)
    return (mp.atanh(s) / s - 1) / z


def q_atan(w):
    if w == 0:
        return -mp.mpf(1) / 3
    s = mp.sqrt(w)
    return (mp.atan(s) / s - 1) / w


def lawson(f, b, deg, n=600, iters=60):
    """Coefficients c_0..c_deg minimising max over [0, b] of |x (sum c_k x^k - f(x))|."""
    xs = [b * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n)) / 2 for k in range(n)]
    fs = [f(x) for x in xs]
    lam = [mp.mpf(1) / n] * n
    c = None
    emax = None
    for _ in range(iters):
        A = mp.matrix(deg + 1, deg + 1)
        rhs = mp.matrix(deg + 1, 1)
        for x, fv, l in zip(xs, fs, lam):
            g = l * x * x
            pw = [x ** j for j in range(deg + 1)]
            for i in range(deg + 1):
                rhs[i] += g * pw[i] * fv
                for j in range(deg + 1):
                    A[i, j] += g * pw[i] * pw[j]
        c = mp.lu_solve(A, rhs)
        errs = [abs(x * (sum(c[j] * x ** j for j in range(deg + 1)) - fv)) for x, fv in zip(xs, fs)]
        emax = max(errs)
        lam = [l * e / emax for l, e in zip(lam, errs)]
        s = sum(lam)
        lam = [l / s for l in lam]
    return [float(c[j]) for j in range(deg + 1)], emax


def horner(c, x):
    p = np.full_like(x, c[-1])
    for ck in reversed(c[:-1]):
        p = p * x + ck   # numpy float64: one rounding per operation (no fma)
    return p


def check_ln(c):
    m = np.linspace(np.sqrt(0.5), np.sqrt(2.0), 20001)[:-1]
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    got = 2.0 * s + 2.0 * s * (z * horner(c, z))
    worst = 0.0
    for mi, gi in zip(m[::40], got[::40]):
        ref = mp.log(mp.mpf(float(mi)))
        if ref != 0:
            ulp = np.spacing(abs(float(ref)))
            worst = max(worst, float(abs(mp.mpf(float(gi)) - ref)) / ulp)
    return worst


def check_atan(c):
    t = np.linspace(0.0, 2.0 - np.sqrt(3.0), 20001)[1:]
    w = t * t
    got = t + (t * w) * horner(c, w)
    worst = 0.0
    for ti, gi in zip(t[::40], got[::40]):
        ref = mp.atan(mp.mpf(float(ti)))
        ulp = np.spacing(abs(float(ref)))
        worst = max(worst, float(abs(mp.mpf(float(gi)) - ref)) / ulp)
    return worst


if __name__ == "__main__":
    zl = (3 - 2 * mp.sqrt(2)) ** 2
    wa = (2 - mp.sqrt(3)) ** 2
    cl, el = lawson(p_ln, zl, LN_DEG)
    ca, ea = lawson(q_atan, wa, ATAN_DEG)
    print("// ln m = 2s (1 + z P(z)), z = s^2 <= (3 - 2 sqrt2)^2: max |z dP| %s; "
          "float64 Horner: max %.2f ulp" % (mp.nstr(el, 3), check_ln(cl)))
    print("static constexpr double kLnPoly[%d] = {%s};" % (len(cl), ", ".join("%.17g" % v for v in cl)))
    print("// atan t = t (1 + w Q(w)), w = t^2 <= (2 - sqrt3)^2: max |w dQ| %s; "
          "float64 Horner: max %.2f ulp" % (mp.nstr(ea, 3), check_atan(ca)))
    print("static constexpr double kAtanPoly64[%d] = {%s};" % (len(ca), ", ".join("%.17g" % v for v in ca)))
