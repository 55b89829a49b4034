"""Mittag-Leffler function for the oracle pins (mpmath, high precision).

E_alpha(z) = sum_k z^k / Gamma(alpha k + 1), summed at 60 digits; valid for the
moderate |z| <= ~10 the pins use.  Cross-checked in the tests against the
closed forms E_1(z) = exp(z) and E_{1/2}(z) = exp(z^2) erfc(-z).
"""
import mpmath as mp


def mittag_leffler(alpha, z, dps=60):
    with mp.workdps(dps):
        a = mp.mpf(alpha)
        zz = mp.mpc(z)
        s = mp.mpc(0)
        term_k = 0
        k = 0
        while True:
            t = zz ** k / mp.gamma(a * k + 1)
            s += t
            if k > 10 and abs(t) < mp.mpf(10) ** (-dps + 5) * max(1, abs(s)):
                break
            k += 1
            term_k += 1
            if k > 5000:
                raise RuntimeError("Mittag-Leffler series did not converge")
        return complex(s) if isinstance(z, complex) else float(s.real)
