"""Coefficients of the transport kernel's inverse error function.

erfinv(x) / x is fitted, in relative error, as a degree-8 polynomial in
t = w - 2.5 for w = -ln(1 - x^2) < 5 and in t = sqrt(w) - 3 for 5 <= w <= 16
(the two regions of Giles 2010, "Approximating the erfinv function"), then
evaluated in FP32 the way the kernel does (Horner with fused multiply-adds)
over the inputs x = 2u - 1 the kernel's uniforms u produce, to report the
largest relative error.  Run: python erfinv_fit.py
"""
import numpy as np
from scipy.special import erfinv

DEG = 8


def fit(t_lo, t_hi, w_of_t, n=20001):
    t = np.linspace(t_lo, t_hi, n)
    w = w_of_t(t)
    x = np.sqrt(-np.expm1(-w))
    f = erfinv(x) / x
    v = np.vander(t, DEG + 1, increasing=True)
    c, *_ = np.linalg.lstsq(v / f[:, None], np.ones_like(f), rcond=None)
    return c


def evaluate_f32(x, central, tail):
    x = x.astype(np.float32)
    w = (-np.log(((np.float32(1) - x) * (np.float32(1) + x)).astype(np.float32))).astype(np.float32)
    out = np.empty_like(x)
    for mask, coef, t in ((w < 5, central, lambda w: w - np.float32(2.5)),
                          (w >= 5, tail, lambda w: np.sqrt(w) - np.float32(3))):
        tt = t(w[mask]).astype(np.float32)
        p = np.full_like(tt, np.float32(coef[DEG]))
        for k in range(DEG - 1, -1, -1):
            p = (p.astype(np.float64) * tt + np.float32(coef[k])).astype(np.float32)   # one rounding: fma
        out[mask] = p * x[mask]
    return out


def main():
    central = fit(-2.5 + 1e-9, 2.5, lambda t: t + 2.5)
    tail = fit(np.sqrt(5.0) - 3.0, 1.0, lambda t: (t + 3.0) ** 2)
    for name, c in (("w < 5, t = w - 2.5", central), ("w >= 5, t = sqrt(w) - 3", tail)):
        print(name + ", highest power first:")
        print("  " + ", ".join("%.9e" % v for v in c[::-1]))
    u = (np.arange(0, 1 << 23, dtype=np.float64) + 0.5) / 2 ** 23
    x = (2 * u - 1).astype(np.float32)
    got = evaluate_f32(x, np.float32(central), np.float32(tail)).astype(np.float64)
    ref = erfinv(x.astype(np.float64))
    rel = np.abs(got - ref) / np.abs(ref)
    print("largest relative error over all 2^23 inputs: %.3e" % rel.max())


if __name__ == "__main__":
    main()
