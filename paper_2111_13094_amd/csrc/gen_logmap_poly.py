"""Generates the polynomial used by the device log map for theta / sin(theta) as a
function of z = cos(theta) on [0, 1] (the factor 1 / sinc(acos z) of the log-map equation
in Sec. 3.1). Relative-error-weighted Chebyshev least squares of degree 9, converted to
monomials in z and rounded to float32; prints the coefficients (lowest order first) and
the maximum relative error of float32 Horner evaluation (about 1.8e-7)."""
import numpy as np
from numpy.polynomial import chebyshev as C


def f(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    m = s > 1e-4
    out[m] = np.arccos(z[m]) / s[m]
    u = 1.0 - z[~m]
    out[~m] = 1.0 + u / 3.0 + 2.0 * u * u / 15.0
    return out


def main(deg=9):
    zs = np.concatenate([np.cos(np.linspace(0, np.pi / 2, 200001)), np.linspace(0, 1, 200001)])
    V = C.chebvander(2 * zs - 1, deg)
    w = 1.0 / f(zs)
    coef, *_ = np.linalg.lstsq(V * w[:, None], f(zs) * w, rcond=None)
    P = np.polynomial.Polynomial(C.cheb2poly(coef))
    cz = P(np.polynomial.Polynomial([-1.0, 2.0])).coef.astype(np.float32)
    zz = np.linspace(0, 1, 4000001).astype(np.float32)
    acc = np.float32(cz[-1])
    for c in cz[-2::-1]:
        acc = np.float32(acc * zz + c)
    ref = f(zz.astype(np.float64))
    for c in cz:
        print("%.9e" % c)
    print("max relative error (float32 Horner): %.3e" % (np.abs(acc - ref) / ref).max())


if __name__ == "__main__":
    main()
