"""Writes the oracle regression fixtures of this directory.  Calls only the
oracle (and the seeded input generators); run from the repository root:

    python tests/golden/make_golden.py

The paper prints no worked example with values, so these fixtures are not
the paper's: they freeze what the oracle computes for small, fully specified
cases, so that any later change of the oracle's arithmetic shows up as a
failing regression test and has to be justified against the paper.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def ghat_table():
    """G^ (Sec. 2.2, eq. GHat_calc and its closed forms) for N = 8, L = 6 at
    a fixed set of (k, m) pairs covering every branch, lambda = 0 and 1."""
    N, L, c = 8, 6.0, 4
    pairs = [((c, c, c), (c + 1, c, c)),          # A = 0 (zeta = 0): zero row
             ((c + 2, c, c - 2), (c + 1, c, c - 1)),  # B = 0 (xi = zeta/2)
             ((c + 2, c, c), (c + 1, c + 1, c)),  # A = B (p = 0)
             ((c + 3, c - 1, c + 1), (c, c, c)),  # Cm = 0 (xi = 0)
             ((1, 6, 3), (2, 5, 5)), ((7, 7, 7), (7, 6, 4)), ((0, 3, 5), (1, 2, 4)), ((5, 1, 6), (3, 1, 7))]
    lines = ["# G^(xi_m, zeta_k) of the oracle, N = 8, L = 6 (Sec. 2.2, eq. GHat_calc, closed forms)",
             "# columns: lambda k1 k2 k3 m1 m2 m3 value"]
    for lam in (0, 1):
        for k, m in pairs:
            v = oracle.ghat(N, L, lam, np.array(k), np.array(m))
            lines.append(f"{lam} {' '.join(map(str, k))} {' '.join(map(str, m))} {v:.17e}")
    open(os.path.join(HERE, "oracle_ghat_n8.txt"), "w").write("\n".join(lines) + "\n")


def bkw_step():
    """Q_c = P_N Q~ (Sec. 3.2 and 3.3) of the BKW distribution at t = 5.5,
    Maxwell molecules, N = 8, L = 6: its moments and the values at a few grid
    points, and f after one Euler step of 0.01 (Sec. 3.3 semi-discrete form)."""
    w = synth.WORKLOADS["bkw_n8"]
    N, L = w["N"], w["L"]
    f = synth.bkw(N, L, 5.5)[None]
    qt = oracle.collision(N, L, 0, f)
    qc, mom = oracle.project(N, L, qt)
    pts = [(0, 0, 0), (4, 4, 4), (3, 4, 5), (2, 6, 1), (7, 3, 4), (5, 5, 2)]
    lines = ["# BKW at t = 5.5, Maxwell molecules, N = 8, L = 6: oracle Q~, Q_c (Sec. 3.2, 3.3)",
             "# moments of Q~ (mass, momentum x3, energy):",
             "moments " + " ".join(f"{x:.17e}" for x in mom[0]),
             "# columns: j1 j2 j3 Q~ Q_c f+0.01*Q_c"]
    for p in pts:
        lines.append(f"{p[0]} {p[1]} {p[2]} {qt[0][p]:.17e} {qc[0][p]:.17e} {f[0][p] + 0.01 * qc[0][p]:.17e}")
    open(os.path.join(HERE, "oracle_bkw_n8.txt"), "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    oracle.build(force=False)
    ghat_table()
    bkw_step()
    print("wrote", sorted(f for f in os.listdir(HERE) if f.endswith(".txt")))
