"""Pins of the oracle's exact reference sums: the free-space direct sum and
the tin-foil Ewald sum used for the periodic modes."""
import math

import numpy as np
import pytest

from conftest import load_golden


def test_direct_two_and_three_charges(orc):
    pos = np.array([[0.1, 0.2, 0.3], [0.4, 0.6, 0.3], [0.1, 0.2, 0.9]])
    q = np.array([1.0, -2.0, 0.5])
    phi, field = orc.direct(pos, q)
    r01, r02, r12 = 0.5, 0.6, math.sqrt(0.09 + 0.16 + 0.36)
    assert np.isclose(phi[0], -2.0 / r01 + 0.5 / r02, rtol=1e-15)
    assert np.isclose(phi[1], 1.0 / r01 + 0.5 / r12, rtol=1e-15)
    # field at 0 from charge 1 points from 1 to 0 scaled by q1/r^3
    f0 = -2.0 * (pos[0] - pos[1]) / r01 ** 3 + 0.5 * (pos[0] - pos[2]) / r02 ** 3
    assert np.allclose(field[0], f0, rtol=1e-14)


def test_ewald_madelung_rock_salt(orc):
    M = load_golden("madelung_nacl.txt")[0, 0]
    pos = np.array([[0, 0, 0], [.5, .5, 0], [.5, 0, .5], [0, .5, .5],
                    [.5, 0, 0], [0, .5, 0], [0, 0, .5], [.5, .5, .5]], float)
    q = np.array([1, 1, 1, 1, -1, -1, -1, -1], float)
    phi, field = orc.ewald(pos, q)
    assert np.allclose(phi, -q * M / 0.5, rtol=1e-13)
    assert np.abs(field).max() < 1e-12
    # the same crystal, box scaled and shifted
    phi2, _ = orc.ewald(2.0 * pos + 0.3, q, box=2.0)
    assert np.allclose(phi2, -q * M / 1.0, rtol=1e-13)


def test_ewald_independent_of_splitting(orc):
    rng = np.random.default_rng(1)
    pos, q = rng.random((40, 3)), rng.uniform(-1, 1, 40)
    q -= q.mean()
    a = orc.ewald(pos, q, alpha=5.0, nrecip=12)
    b = orc.ewald(pos, q, alpha=8.0, nrecip=18)
    assert np.abs(a[0] - b[0]).max() < 1e-11 * np.abs(a[0]).max()
    assert np.abs(a[1] - b[1]).max() < 1e-10 * np.abs(a[1]).max()


def test_ewald_rejects_net_charge(orc):
    with pytest.raises(orc.OracleError):
        orc.ewald(np.random.default_rng(0).random((3, 3)), np.array([1.0, 1.0, -1.5]))


def test_ewald_is_cubic_image_sum_minus_shape_term(orc):
    # Summing the images in growing cubes converges to the tin-foil energy plus
    # (2 pi / 3V)|M|^2 for a neutral cell with dipole M (textbook result).
    rng = np.random.default_rng(0)
    p = rng.random((4, 3))
    q = np.array([1.0, -1.0, 0.5, -0.5])
    phi, _ = orc.ewald(p, q)
    e_ewald = 0.5 * (q * phi).sum()
    M = (q[:, None] * p).sum(0)
    shape = 2.0 * math.pi / 3.0 * (M @ M)

    def cubic(R):
        g = np.arange(-R, R + 1, dtype=float)
        m = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        E = 0.0
        for i in range(4):
            for j in range(4):
                r = np.linalg.norm(p[i] - p[j] + m, axis=1)
                if i == j:
                    r = r[r > 0]
                E += 0.5 * q[i] * q[j] * (1.0 / r).sum()
        return E

    e20, e40 = cubic(20), cubic(40)
    extrap = e40 + (e40 - e20) / 3.0       # the remainder falls as R^-2
    assert abs((extrap - e_ewald) / shape - 1.0) < 1e-4


def test_periodic_root_independent_of_splitting(orc):
    T2 = orc.periodic_root(3, alpha=2.0)
    T3 = orc.periodic_root(3, alpha=3.0)
    assert np.abs(T2 - T3).max() < 1e-12 * np.abs(T2).max()
    assert np.allclose(T2, T2.T, atol=1e-13)
