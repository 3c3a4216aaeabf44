"""Rational approximations r(x) ~ x^p for the one-flavour (RHMC) actions.

The DD-RHMC boundary action needs (D_d^+ D_d)^{1/4} and (D^+ D)^{-1/2} of the
normal operators (eq. (ddrhmc) and the one-flavour action that follows it).
Both are applied as partial fractions
    r(x) = a0 + sum_k alpha_k / (x + beta_k),   beta_k > 0,
so that r(A) v needs one multi-shift solve with the shifts beta_k.

This script computes best relative-error approximations of type (n, n) on
[lo, hi] by the Remez exchange algorithm (the minimax error equioscillates at
2n + 2 points), in 150-digit arithmetic with mpmath (on x scaled by sqrt(lo hi), so
that the monomial basis stays well inside the working precision), and writes the partial
fractions with the achieved maximum relative error
    eps = max_{lo <= x <= hi} |r(x) / x^p - 1|
measured on a dense logarithmic grid.  The paper prints no coefficients; these
files are inputs that the caller passes to the library and the tests pass to
the oracle, like the seeded fields.

    python -m paper_2203_17119_amd.rational.remez --power 0.25 --lo 1e-3 --hi 64 --degree 10 -o FILE.json
"""
from __future__ import annotations

import argparse
import json

import mpmath as mp

mp.mp.dps = 150


def _horner(c, x):
    s = mp.mpf(0)
    for a in reversed(c):
        s = s * x + a
    return s


def _solve_levelled(f, xs, n, E_guess, q_prev):
    """Coefficients p (n+1), q (n+1, q0 = 1) and level E with
    P(x_i) - f(x_i) Q(x_i) = (-1)^i E f(x_i) Q_prev(x_i) at the 2n+2 nodes."""
    m = 2 * n + 2
    A = mp.matrix(m, m)
    rhs = mp.matrix(m, 1)
    for i, x in enumerate(xs):
        fx = f(x)
        qp = _horner(q_prev, x)
        for j in range(n + 1):
            A[i, j] = x ** j
        for j in range(1, n + 1):
            A[i, n + j] = -fx * x ** j
        A[i, 2 * n + 1] = -((-1) ** i) * fx * qp
        rhs[i] = fx
    sol = mp.lu_solve(A, rhs)
    p = [sol[j] for j in range(n + 1)]
    q = [mp.mpf(1)] + [sol[n + j] for j in range(1, n + 1)]
    return p, q, sol[2 * n + 1]


def remez(power: float, lo: float, hi: float, n: int, iters: int = 60, grid: int = 4000):
    """Best type-(n, n) relative approximation of x^power on [lo, hi] as partial
    fractions.  Computed for u^power on [lo/s, hi/s], s = sqrt(lo hi), then
    scaled back: x^p = s^p u^p with u = x / s."""
    s = mp.sqrt(mp.mpf(lo) * mp.mpf(hi))
    r = _remez_unit(power, mp.mpf(lo) / s, mp.mpf(hi) / s, n, iters, grid)
    sp = s ** mp.mpf(power)
    a0 = sp * r["a0"]
    alphas = [sp * s * a for a in r["alpha"]]
    betas = [s * b for b in r["beta"]]
    la, lb = mp.log(mp.mpf(lo)), mp.log(mp.mpf(hi))
    pf = lambda x: a0 + sum(al / (x + be) for al, be in zip(alphas, betas))  # noqa: E731
    dense = [mp.exp(la + (lb - la) * k / (4 * grid - 1)) for k in range(4 * grid)]
    eps = max(abs(pf(x) / x ** mp.mpf(power) - 1) for x in dense)
    return {"power": float(power), "lo": float(lo), "hi": float(hi), "degree": n,
            "a0": float(a0), "alpha": [float(a) for a in alphas], "beta": [float(b) for b in betas],
            "max_rel_error": float(eps), "remez_iterations": r["iterations"]}


def _remez_unit(power, lo, hi, n, iters, grid):
    pw = mp.mpf(power)
    f = lambda x: x ** pw  # noqa: E731
    # initial nodes: Chebyshev-like points in log x
    la, lb = mp.log(lo), mp.log(hi)
    m = 2 * n + 2
    xs = [mp.exp(la + (lb - la) * (1 - mp.cos(mp.pi * i / (m - 1))) / 2) for i in range(m)]
    q = [mp.mpf(1)] + [mp.mpf(0)] * n
    E = mp.mpf(0)
    gx = [mp.exp(la + (lb - la) * k / (grid - 1)) for k in range(grid)]
    for it in range(iters):
        for _ in range(4):  # settle the level for the current nodes
            p, q, E = _solve_levelled(f, xs, n, E, q)
        err = lambda x: _horner(p, x) / (_horner(q, x) * f(x)) - 1  # noqa: E731
        ev = [err(x) for x in gx]
        # one extremum per sign run of the error on the grid, refined by a local search
        runs, start = [], 0
        for k in range(1, grid + 1):
            if k == grid or mp.sign(ev[k]) != mp.sign(ev[start]):
                kk = max(range(start, k), key=lambda j: abs(ev[j]))
                runs.append(kk)
                start = k
        if len(runs) < m:
            raise RuntimeError(f"Remez: {len(runs)} alternations, need {m}")
        while len(runs) > m:  # drop the smallest end extremum
            if abs(ev[runs[0]]) < abs(ev[runs[-1]]):
                runs.pop(0)
            else:
                runs.pop()
        new = []
        for kk in runs:
            a = gx[max(kk - 1, 0)]
            b = gx[min(kk + 1, grid - 1)]
            g = lambda x: -abs(err(x))  # noqa: E731
            # golden-section search for the extremum inside its grid cell pair
            for _ in range(40):
                c1, c2 = a + (b - a) * mp.mpf("0.382"), a + (b - a) * mp.mpf("0.618")
                if g(c1) < g(c2):
                    b = c2
                else:
                    a = c1
            new.append((a + b) / 2)
        xs = new
        ext = [abs(err(x)) for x in xs]
        spread = (max(ext) - min(ext)) / max(ext)
        if spread < mp.mpf("1e-6"):
            break
    # partial fractions: poles z_k = roots of Q, residues P(z_k) / Q'(z_k)
    zs = mp.polyroots(list(reversed(q)), maxsteps=400, extraprec=200)
    dq = [j * q[j] for j in range(1, n + 1)]
    a0 = p[n] / q[n]
    alphas, betas = [], []
    for z in zs:
        if abs(mp.im(z)) > mp.mpf("1e-20") * (1 + abs(z)):
            raise RuntimeError("complex pole")
        z = mp.re(z)
        if z >= 0:
            raise RuntimeError("pole inside the positive axis")
        alphas.append(_horner(p, z) / _horner(dq, z))
        betas.append(-z)
    order = sorted(range(n), key=lambda k: betas[k])
    alphas = [alphas[k] for k in order]
    betas = [betas[k] for k in order]
    return {"a0": a0, "alpha": alphas, "beta": betas, "iterations": it + 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--power", type=float, required=True)
    ap.add_argument("--lo", type=float, required=True)
    ap.add_argument("--hi", type=float, required=True)
    ap.add_argument("--degree", type=int, required=True)
    ap.add_argument("-o", "--output", required=True)
    a = ap.parse_args()
    r = remez(a.power, a.lo, a.hi, a.degree)
    with open(a.output, "w") as fh:
        json.dump(r, fh, indent=1)
        fh.write("\n")
    print(f"x^{a.power} on [{a.lo}, {a.hi}], degree {a.degree}: max relative error {r['max_rel_error']:.3e}")


if __name__ == "__main__":
    main()
