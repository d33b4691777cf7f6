"""Oracle regression fixtures (tests/golden/, written by
tests/golden/make_golden.py from the oracle alone): the oracle still computes
what it computed when they were written.  A change of the oracle's arithmetic
must come with regenerated fixtures and the passage of the paper that
justifies it."""
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    return [ln.split() for ln in open(os.path.join(GOLDEN, name)) if ln.strip() and not ln.startswith("#")]


def test_ghat_fixture(orc):
    rows = _rows("oracle_ghat_n8.txt")
    assert len(rows) == 16
    scale = max(abs(float(r[7])) for r in rows)
    for r in rows:
        lam, k, m, v = int(r[0]), np.array(r[1:4], int), np.array(r[4:7], int), float(r[7])
        assert abs(orc.ghat(8, 6.0, lam, k, m) - v) <= 1e-15 * scale, r


def test_bkw_fixture(orc):
    rows = _rows("oracle_bkw_n8.txt")
    f = synth.bkw(8, 6.0, 5.5)[None]
    qt = orc.collision(8, 6.0, 0, f)
    qc, mom = orc.project(8, 6.0, qt)
    want = np.array(rows[0][1:], float)
    assert np.abs(mom[0] - want).max() <= 1e-14 * np.abs(want).max()
    s = np.abs(qt).max()
    for r in rows[1:]:
        p = tuple(int(x) for x in r[:3])
        assert abs(qt[0][p] - float(r[3])) <= 1e-13 * s
        assert abs(qc[0][p] - float(r[4])) <= 1e-13 * s
        assert abs(f[0][p] + 0.01 * qc[0][p] - float(r[5])) <= 1e-15 * max(1.0, abs(float(r[5])))
