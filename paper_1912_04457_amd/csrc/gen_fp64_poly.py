"""Coefficients of the FP64 polynomials in collide.hip (exp64, log64,
sincos_2pi): Chebyshev-node fits (mpmath.chebyfit, near-minimax) of the
smooth part of each function on its reduced range, at 60 digits, rounded to
FP64.  Prints each list highest degree first with the fit's error bound.

  exp:  e^r = 1 + r (1 + r g(r)),  g(r) = (e^r - 1 - r)/r^2,  |r| <= ln2/2
  ln:   ln m = 2 s P(s^2),         P(w) = atanh(sqrt w)/sqrt w, w <= ((sqrt2-1)/(sqrt2+1))^2
  sin:  sin(pi r) = r S(r^2),      cos(pi r) = C(r^2),           |r| <= 1/4
"""
import mpmath as mp

mp.mp.dps = 60


def fit(f, a, b, deg):
    poly, err = mp.chebyfit(f, [a, b], deg + 1, error=True)
    return [float(c) for c in poly], err


def main():
    margin = mp.mpf("1.0001")
    a = mp.log(2) / 2 * margin
    g = lambda r: (mp.exp(r) - 1 - r) / r ** 2 if abs(r) > mp.mpf(10) ** -20 else mp.mpf(1) / 2 + r / 6
    w_sin = mp.mpf(1) / 16 * margin
    S = lambda w: mp.sin(mp.pi * mp.sqrt(w)) / mp.sqrt(w) if w > 0 else mp.pi
    C = lambda w: mp.cos(mp.pi * mp.sqrt(w))
    sm = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    P = lambda w: mp.atanh(mp.sqrt(w)) / mp.sqrt(w) if w > 0 else mp.mpf(1)
    for name, f, lo, hi, deg in (("exp g", g, -a, a, 9), ("sin S", S, 0, w_sin, 6), ("cos C", C, 0, w_sin, 6),
                                 ("ln P", P, 0, sm * sm * margin, 7)):
        c, err = fit(f, lo, hi, deg)
        print(f"{name} (degree {deg}, fit error {mp.nstr(err, 3)}):")
        print("  " + ", ".join(repr(x) for x in c))


if __name__ == "__main__":
    main()
