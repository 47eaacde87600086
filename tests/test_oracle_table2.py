"""Pin of replacement + bilinear form against Table 2 (Appendix A.1): the
maximum relative pair error E1 (both charges replaced) and E2 (one replaced)
between a unit cube and the unit cube directly above it at gap 1, with the
charges stepping by 0.04 over 26^3 points in each cube."""
import numpy as np
import pytest

from conftest import load_golden

GRID = np.linspace(0.0, 1.0, 26)


def _points(lo):
    X, Y, Z = np.meshgrid(GRID + lo[0], GRID + lo[1], GRID + lo[2], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def _replaced(orc, n, lo, pts):
    # one replacement per point (Eq. (6)), unit charge
    return np.stack([orc.replace(n, lo, 1.0, p, [1.0]) for p in pts])


def _e1_e2(orc, n, lo2):
    lo1 = np.zeros(3)
    P, Pt = _points(lo1), _points(lo2)
    R1, R2 = _replaced(orc, n, lo1, P), _replaced(orc, n, lo2, Pt)
    K = orc.bilinear_matrix(n, lo1, 1.0, lo2, 1.0)
    W = K @ R2.T                          # [n^3, points in C~]
    # nodes of C~ for E2 (P itself not replaced)
    t = orc.nodes(n)
    Xn = np.stack([np.tile(t, n * n), np.tile(np.repeat(t, n), n), np.repeat(t, n * n)], axis=1) + lo2
    e1 = e2 = 0.0
    sq = (Pt ** 2).sum(1)
    B = 128  # small blocks keep the temporaries in cache
    for c0 in range(0, P.shape[0], B):
        p = P[c0:c0 + B]
        # |p - p~| from the Gram matrix (distances >= 1 here, so no cancellation)
        r = p @ Pt.T
        r *= -2.0
        r += (p ** 2).sum(1)[:, None]
        r += sq[None, :]
        np.sqrt(r, out=r)
        a = R1[c0:c0 + B] @ W
        a *= r
        e1 = max(e1, a.max() - 1.0, 1.0 - a.min())
        F = 1.0 / np.sqrt(((p[:, None, :] - Xn[None, :, :]) ** 2).sum(2))
        a = F @ R2.T
        a *= r
        e2 = max(e2, a.max() - 1.0, 1.0 - a.min())
    return e1, e2


@pytest.mark.parametrize("row", load_golden("table2_e1e2.txt").tolist(), ids=lambda r: f"order{int(r[0])}")
def test_table2_directly_above(orc, row):
    n, E1p, E2p = int(row[0]), row[1], row[2]
    e1, e2 = _e1_e2(orc, n, np.array([0.0, 0.0, 2.0]))
    # the paper's grid and node reading reproduce its table to a few percent
    assert abs(e1 / E1p - 1) < 0.10, (e1, E1p)
    assert abs(e2 / E2p - 1) < 0.10, (e2, E2p)
    assert e1 / e2 <= 2.0 + 1e-9          # "E1/E2 is at most 2"


@pytest.mark.slow
def test_table2_max_is_directly_above_order4(orc):
    # "E1 and E2 took their maximum when C~ was just above C" (order 4)
    best = {}
    for ix in range(-2, 3):
        for iy in range(-2, 3):
            best[(ix, iy)] = _e1_e2(orc, 4, np.array([2.0 * ix, 2.0 * iy, 2.0]))
    e1max = max(v[0] for v in best.values())
    e2max = max(v[1] for v in best.values())
    assert best[(0, 0)][0] == e1max and best[(0, 0)][1] == e2max
