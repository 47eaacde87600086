"""Pins of the oracle's building blocks against identities the paper states
(Sec. 2.1) and textbook special cases."""
import itertools

import numpy as np
import pytest


@pytest.mark.parametrize("n", range(2, 9))
def test_lagrange_reproduces_monomials(orc, n):
    # Eq. (2): sum_i a_i^j g_i(x) = x^j for j < n, at points inside and outside
    t = orc.nodes(n)
    for x in np.linspace(-0.7, 1.7, 23):
        g, dg = orc.lagrange(t, x)
        for j in range(n):
            # tolerance: rounding of the sum, scaled by its largest terms
            assert abs(np.dot(t ** j, g) - x ** j) <= 1e-14 * max(1.0, np.abs(t ** j * g).sum())
            # derivative of the same identity
            ref = j * x ** (j - 1) if j > 0 else 0.0
            assert abs(np.dot(t ** j, dg) - ref) <= 1e-13 * max(1.0, np.abs(t ** j * dg).sum())


@pytest.mark.parametrize("n", range(2, 9))
def test_lagrange_kronecker(orc, n):
    # g_i(a_j) = delta_ij (Sec. 2.1.1)
    t = orc.nodes(n)
    for j in range(n):
        g, _ = orc.lagrange(t, t[j])
        assert np.allclose(g, np.eye(n)[j], atol=1e-14)


def test_nodes_include_end_points(orc):
    # n-division points include both end points and are equally spaced (Sec. 2.1.2)
    t = orc.nodes(4)
    assert np.allclose(t, [0, 1 / 3, 2 / 3, 1], atol=1e-15)
    ts = orc.nodes(4, sigma=1 / 1.2)  # reduced arrangement (Sec. 4.1)
    assert np.allclose(ts, 0.5 + (np.array([0, 1 / 3, 2 / 3, 1]) - 0.5) / 1.2)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_invariance_1d(orc, n):
    # Eq. (9): Rpl on S~ equals shift_{S->S~} applied to Rpl on S, for any two segments
    rng = np.random.default_rng(n)
    for _ in range(5):
        lo, L = rng.uniform(-1, 1), rng.uniform(0.2, 2)
        lo2, L2 = rng.uniform(-1, 1), rng.uniform(0.2, 2)
        a = lo + L * orc.nodes(n)
        at = lo2 + L2 * orc.nodes(n)
        G = orc.shift_1d(a, at)
        for x in rng.uniform(-1, 2, 7):
            g, _ = orc.lagrange(a, x)
            gt, _ = orc.lagrange(at, x)
            assert np.allclose(G @ g, gt, atol=1e-10 * max(1, np.abs(gt).max()))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_invariance_3d_child_to_parent(orc, n):
    # Eq. (11) for the upward pass: replacing in a child and shifting to the
    # parent equals replacing directly in the parent (to 1e-12)
    rng = np.random.default_rng(10 + n)
    t = orc.nodes(n)
    plo, ps = np.array([0.25, 0.5, 0.0]), 0.25
    for b in itertools.product((0, 1), repeat=3):
        clo = plo + ps / 2 * np.array(b)
        pos = clo + ps / 2 * rng.random((9, 3))
        q = rng.uniform(-1, 1, 9)
        child = orc.replace(n, clo, ps / 2, pos, q)
        G = [orc.shift_1d(clo[a] + ps / 2 * t, plo[a] + ps * t) for a in range(3)]
        shifted = orc.shift_3d(n, G[0], G[1], G[2], child)
        direct = orc.replace(n, plo, ps, pos, q)
        assert np.abs(shifted - direct).max() <= 1e-12 * np.abs(direct).max()


def test_invariance_3d_arbitrary_cubes(orc):
    # the invariance holds for any two cubes, nested or not (Eq. (11))
    rng = np.random.default_rng(3)
    n = 4
    t = orc.nodes(n)
    for _ in range(4):
        lo1, s1 = rng.uniform(-1, 1, 3), rng.uniform(0.3, 1.5)
        lo2, s2 = rng.uniform(-1, 1, 3), rng.uniform(0.3, 1.5)
        pos = lo1 + s1 * rng.random((6, 3))
        q = rng.uniform(-1, 1, 6)
        G = [orc.shift_1d(lo1[a] + s1 * t, lo2[a] + s2 * t) for a in range(3)]
        a = orc.shift_3d(n, G[0], G[1], G[2], orc.replace(n, lo1, s1, pos, q))
        b = orc.replace(n, lo2, s2, pos, q)
        assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()


def test_shift_round_trip(orc):
    # shift_{S->C} o shift_{C->S} = identity (Appendix A.2)
    n = 5
    t = orc.nodes(n)
    C = 0.375 + 0.125 * t
    S = t
    assert np.allclose(orc.shift_1d(S, C) @ orc.shift_1d(C, S), np.eye(n), atol=1e-9)


def test_replace_order2_is_cloud_in_cell(orc):
    # n = 2: the weights are the trilinear (cloud-in-cell) weights
    rng = np.random.default_rng(4)
    lo, s = np.array([0.5, -1.0, 2.0]), 0.5
    for _ in range(10):
        x = lo + s * rng.random(3)
        u = (x - lo) / s
        phi = orc.replace(2, lo, s, x, [1.7])
        ref = np.zeros(8)
        for k, j, i in itertools.product((0, 1), repeat=3):
            w = (u[0] if i else 1 - u[0]) * (u[1] if j else 1 - u[1]) * (u[2] if k else 1 - u[2])
            ref[i + 2 * j + 4 * k] = 1.7 * w
        assert np.allclose(phi, ref, atol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_replace_reproduces_moments(orc, n):
    # sum_a Phi_a x_a^al y_a^be z_a^ga = sum_l q_l x_l^al y_l^be z_l^ga for al,be,ga < n
    rng = np.random.default_rng(20 + n)
    lo, s = np.array([0.1, 0.2, 0.3]), 0.7
    pos = lo + s * rng.random((11, 3))
    q = rng.uniform(-1, 1, 11)
    phi = orc.replace(n, lo, s, pos, q)
    a = lo[0] + s * orc.nodes(n)
    X, Y, Z = np.meshgrid(a, a + lo[1] - lo[0], a + lo[2] - lo[0], indexing="ij")
    X, Y, Z = (V.transpose(2, 1, 0).ravel() for V in (X, Y, Z))  # index i + n j + n^2 k
    for al, be, ga in itertools.product(range(n), repeat=3):
        lhs = np.sum(phi * X ** al * Y ** be * Z ** ga)
        rhs = np.sum(q * pos[:, 0] ** al * pos[:, 1] ** be * pos[:, 2] ** ga)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, np.abs(q).sum())


def test_replace_charge_on_node_is_unit_vector(orc):
    n = 4
    lo, s = np.zeros(3), 1.0
    t = orc.nodes(n)
    phi = orc.replace(n, lo, s, [t[1], t[3], t[0]], [2.5])
    ref = np.zeros(n ** 3)
    ref[1 + n * 3 + 0] = 2.5
    assert np.allclose(phi, ref, atol=1e-14)


def test_bilinear_is_symmetric_and_exact_on_nodes(orc):
    n = 3
    lo1, lo2 = np.zeros(3), np.array([0.0, 0.0, 2.0])
    K = orc.bilinear_matrix(n, lo1, 1.0, lo2, 1.0)
    assert np.allclose(K, orc.bilinear_matrix(n, lo2, 1.0, lo1, 1.0).T, atol=0)
    rng = np.random.default_rng(5)
    v, w = rng.standard_normal(n ** 3), rng.standard_normal(n ** 3)
    assert np.isclose(orc.bilinear(n, lo1, 1.0, lo2, 1.0, v, w), v @ K @ w, rtol=1e-13)
    # two charges sitting on nodes interact exactly (their replacements are unit vectors)
    p1, p2 = np.array([0.5, 1.0, 0.0]), np.array([1.0, 0.0, 3.0])
    a = orc.replace(n, lo1, 1.0, p1, [1.0])
    b = orc.replace(n, lo2, 1.0, p2, [-2.0])
    assert np.isclose(orc.bilinear(n, lo1, 1.0, lo2, 1.0, a, b), -2.0 / np.linalg.norm(p1 - p2), rtol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_invariance_3d_reduced_nodes(orc, n):
    # Eq. (11) with the reduced arrangement of Sec. 4.1 (spacing x 1/1.2,
    # points inside the cube): replacing in a child and shifting to the
    # parent still equals replacing directly in the parent
    sig = 1 / 1.2
    rng = np.random.default_rng(40 + n)
    t = orc.nodes(n, sig)
    assert np.isclose(t.max() - t.min(), sig) and np.isclose(t.mean(), 0.5)
    plo, ps = np.array([0.5, 0.0, 0.25]), 0.25
    for b in itertools.product((0, 1), repeat=3):
        clo = plo + ps / 2 * np.array(b)
        pos = clo + ps / 2 * rng.random((9, 3))
        q = rng.uniform(-1, 1, 9)
        child = orc.replace(n, clo, ps / 2, pos, q, sigma=sig)
        G = [orc.shift_1d(clo[a] + ps / 2 * t, plo[a] + ps * t) for a in range(3)]
        shifted = orc.shift_3d(n, G[0], G[1], G[2], child)
        direct = orc.replace(n, plo, ps, pos, q, sigma=sig)
        assert np.abs(shifted - direct).max() <= 1e-12 * np.abs(direct).max()
