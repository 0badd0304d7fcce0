"""Coefficients of the expm1 polynomial in exp_pair (rt_internal.h).

After the range reduction x = k ln2 + r, exp_pair needs expm1(u) for |u| <= ln2/2 to
full float64 relative accuracy.  It evaluates expm1(u) = u q(u) with q the degree-10
polynomial that minimises max |q(u) / (expm1(u)/u) - 1| on that interval (a little
wider, for the rounding of r), found here by the Remez exchange in 60-digit arithmetic
(mpmath).  The maximal relative error is 1.76e-17 (degree 9 would give 1.2e-15).

    python paper_1001_3301_amd/csrc/expm1_minimax.py

prints the Horner lines between the BEGIN/END markers of exp_pair, highest degree first.
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 60
DEGREE = 10
HALF_RANGE = mp.log(2) / 2 * (1 + mp.mpf("1e-6"))


def _f(u):
    return mp.expm1(u) / u if u != 0 else mp.mpf(1)


def remez(n: int = DEGREE, a=HALF_RANGE, iters: int = 30, grid: int = 4000):
    """Coefficients c_0..c_n (ascending) of the relative-minimax q, and the error."""
    m = n + 2
    x = [a * mp.cos(mp.pi * (m - 1 - i) / (m - 1)) for i in range(m)]
    pts = [a * mp.cos(mp.pi * k / grid) for k in range(grid + 1)][::-1]
    for _ in range(iters):
        # q(x_i) - f(x_i) = (-1)^i E f(x_i) at the n + 2 reference points
        A = mp.matrix(m, m)
        b = mp.matrix(m, 1)
        for i, xi in enumerate(x):
            fi = _f(xi)
            for j in range(n + 1):
                A[i, j] = xi ** j
            A[i, n + 1] = (-1) ** i * fi
            b[i] = fi
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(n + 1)]
        err = [(mp.polyval(c[::-1], g) - _f(g)) / _f(g) for g in pts]
        # next reference: the local extrema of the error, alternating in sign
        ext = [(pts[k], err[k]) for k in range(len(pts))
               if k in (0, len(pts) - 1) or (err[k] - err[k - 1]) * (err[k + 1] - err[k]) <= 0]
        alt = []
        for g, e in ext:
            if alt and mp.sign(alt[-1][1]) == mp.sign(e):
                if abs(e) > abs(alt[-1][1]):
                    alt[-1] = (g, e)
            else:
                alt.append((g, e))
        while len(alt) > m:
            alt.pop(0 if abs(alt[0][1]) < abs(alt[-1][1]) else -1)
        if len(alt) < m:
            break
        x = [g for g, _ in alt]
    return c, max(abs(e) for e in err)


def horner_lines(c) -> list[str]:
    """The C lines of exp_pair's Horner evaluation (float64 coefficients, repr exact)."""
    d = [float(v) for v in c][::-1]
    out = [f"    double p = {d[0]!r};"]
    out += [f"    p = fma(p, u, {v!r});" for v in d[1:]]
    return out


if __name__ == "__main__":
    coef, e = remez()
    print(f"// relative error {mp.nstr(e, 4)}")
    print("\n".join(horner_lines(coef)))
