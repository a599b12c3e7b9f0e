"""Locate the critical Wilson mass of the synthetic ensembles with the oracle
and place the working mass just above it.

The smallest |eigenvalue| of the Hermitian gamma5 D (equal to the smallest
singular value of D) is computed exactly (dense Hermitian eigensolver,
eigenvalues in a window around zero) on a 4^3x8 lattice of the same ensemble
parameters (temporal anisotropy xi, link spread eps, three APE-like
projections).  A scan and a golden-section search locate m_c, the m0 where
sigma_min(m0) is smallest: the low modes of D cross the imaginary axis there.
On this volume sigma_min never drops below ~6e-3 (the low eigenvalues keep
imaginary parts of that size), so a 1e-3 target cannot be reached by bisection;
the working mass is m0 = m_c + DELTA on the physical side of the crossing,
where the real parts of the low eigenvalues are of order DELTA.  The result
(m_c, m0, sigma_min at both) is written to tests/golden/m0_tuned.json and used
for every volume of that ensemble.

Run: python -m oracle.tune_m0   (a few CPU minutes)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import lattice  # noqa: E402
from oracle.gamma import gamma5_full  # noqa: E402
from oracle.wilson import WilsonOp  # noqa: E402

ENSEMBLES = {
    # name: (xi, eps, n_ape, config id)
    "aniso_xi3.5_eps0.2": (3.5, 0.2, 3, 2),
    "iso_xi1_eps0.25": (1.0, 0.25, 3, 3),
}
DIMS = [4, 4, 4, 8]
TARGET = 1e-3
DELTA = 1e-2
WINDOW = 0.25


def sigma_min_fn(U, xi):
    V = lattice.volume(DIMS)
    D0 = WilsonOp(U, DIMS, 0.0, xi).dense()
    g5 = np.tile(gamma5_full().diagonal(), V)
    H0 = g5[:, None] * D0  # gamma5 D(m0=0), Hermitian

    def f(m0):
        H = H0 + m0 * np.diag(g5)
        ev = scipy.linalg.eigvalsh(H, subset_by_value=(-WINDOW, WINDOW), driver="evr")
        return float(np.min(np.abs(ev))) if ev.size else WINDOW

    return f


def tune(xi, eps, n_ape, config, log=print):
    """Golden-section search for the m0 of smallest sigma_min in [-0.15, 0.05]; if that
    minimum lies below the target, bisect on the side above it to sigma_min = target,
    otherwise keep the minimiser (the closest approach to criticality of the lattice)."""
    U = synth.gauge_field(DIMS, eps, n_ape, config=config)
    f = sigma_min_fn(U, xi)
    cache = {}

    def g(m):
        if m not in cache:
            cache[m] = f(m)
            log(f"  m0={m:+.6f} sigma_min={cache[m]:.4e}")
        return cache[m]

    # coarse scan, then golden section around the best point
    grid = np.linspace(-0.05, 0.03, 17)
    vals = [g(float(m)) for m in grid]
    i = int(np.argmin(vals))
    a, b = float(grid[max(i - 1, 0)]), float(grid[min(i + 1, grid.size - 1)])
    r = (np.sqrt(5) - 1) / 2
    c, d = b - r * (b - a), a + r * (b - a)
    for _ in range(30):
        if g(c) < g(d):
            b = d
        else:
            a = c
        c, d = b - r * (b - a), a + r * (b - a)
        if b - a < 1e-6:
            break
    m_min = 0.5 * (a + b)
    s_min = g(m_min)
    if s_min <= TARGET:
        lo, hi = m_min, float(grid[-1])  # f(lo) <= target < f(hi) on the upper side
        for _ in range(40):
            mid = 0.5 * (lo + hi)
            if g(mid) <= TARGET:
                lo = mid
            else:
                hi = mid
            if hi - lo < 1e-8:
                break
        return m_min, s_min, hi, g(hi), "bisected to the target above the crossing"
    m0 = m_min + DELTA
    return m_min, s_min, m0, g(m0), f"sigma_min floor above the target: m0 = m_c + {DELTA}"


def main():
    out = {"lattice": DIMS, "target_sigma_min": TARGET, "delta": DELTA,
           "method": "dense gamma5 D spectrum on the small lattice, golden-section search for m_c",
           "ensembles": {}}
    for name, (xi, eps, n_ape, config) in ENSEMBLES.items():
        t = time.time()
        print(f"{name}: xi={xi} eps={eps} n_ape={n_ape}", flush=True)
        mc, smc, m0, s, how = tune(xi, eps, n_ape, config, log=lambda m: print(m, flush=True))
        out["ensembles"][name] = {"xi": xi, "eps": eps, "n_ape": n_ape, "m_c": mc, "sigma_min_at_m_c": smc,
                                  "m0": m0, "sigma_min": s, "how": how, "seconds": round(time.time() - t, 1)}
    path = os.path.join(ROOT, "tests", "golden", "m0_tuned.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
