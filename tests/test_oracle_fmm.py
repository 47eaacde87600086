"""Pins of the oracle's replacement FMM (Sec. 2.2, Sec. 2.3, Sec. 4.2)."""
import numpy as np
import pytest

import workloads
from conftest import load_golden

FREE, FREE_C, PER, PER_C = 0, 1, 2, 3


def _inputs(n, seed, neutral=True):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    q = rng.uniform(-1, 1, n)
    if neutral:
        q -= q.mean()
    return pos, q


@pytest.mark.parametrize("mode,levels,order,N,d", [
    (FREE, 3, 4, 300, 0.0), (FREE, 2, 3, 200, 0.0), (FREE, 3, 5, 120, 0.0),
    (FREE_C, 3, 4, 200, 0.01), (FREE_C, 3, 5, 150, 0.01),
    (PER, 2, 4, 64, 0.0), (PER_C, 2, 4, 64, 0.02), (PER_C, 2, 3, 64, 0.02)])
def test_tree_equals_pairwise_closed_form(orc, mode, levels, order, N, d):
    # The upward/downward passes reproduce, to rounding, the pairwise form in
    # which every pair interacts at the level where it becomes well separated
    # (invariance property, Eq. (11)).
    pos, q = _inputs(N, 7 + mode + order)
    a = orc.fmm(pos, q, levels, order, mode, split_d=d)
    b = orc.fmm_pairwise(pos, q, levels, order, mode, split_d=d)
    assert np.abs(a["phi"] - b["phi"]).max() <= 1e-12 * np.abs(b["phi"]).max()
    assert abs(a["energy"] - b["energy"]) <= 1e-12 * np.abs(q * b["phi"]).sum()


def test_all_near_field_equals_direct_sum(orc):
    # every charge in a 2x2x2 block of finest cells: no far field at all
    rng = np.random.default_rng(2)
    pos = 0.25 + 0.25 * rng.random((80, 3))       # cells 1..2 at level 3
    q = rng.uniform(-1, 1, 80)
    a = orc.fmm(pos, q, 3, 4)
    ref_phi, ref_field = orc.direct(pos, q)
    assert np.allclose(a["phi"], ref_phi, rtol=1e-13, atol=1e-12)
    assert np.allclose(a["field"], ref_field, rtol=1e-12, atol=1e-10)


def test_charges_on_shared_nodes_interact_exactly(orc):
    # Charges at opposite corners of the box are nodes of every cell that
    # holds them, so their far interaction is the exact 1/r.
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    q = np.array([1.5, -0.5])
    for order in (2, 3, 4, 6):
        a = orc.fmm(pos, q, 3, order)
        assert np.isclose(a["energy"], 1.5 * -0.5 / np.sqrt(3.0), rtol=1e-14)


@pytest.mark.parametrize("row", load_golden("table1_errors.txt").tolist(), ids=lambda r: f"order{int(r[0])}")
def test_table1_error_magnitudes(orc, row):
    # Table 1 workload shape: 23040 random +-1 charges, 8^3 finest cells.  The
    # paper's charges are not available, so only the magnitude can be pinned.
    n = int(row[0])
    w, pos, q = workloads.workload_inputs("t1")
    ref_phi, ref_field = _direct_t1(orc)
    a = orc.fmm(pos, q, 3, n)
    e1 = np.mean(np.abs((a["phi"] - ref_phi) / ref_phi))
    e2 = np.mean(np.abs((a["field"] - ref_field) / ref_field))
    assert 0.75 < e1 / row[1] < 1.33, (e1, row[1])
    assert 0.4 < e2 / row[2] < 2.5, (e2, row[2])


_T1 = {}


def _direct_t1(orc):
    if "d" not in _T1:
        _, pos, q = workloads.workload_inputs("t1")
        _T1["d"] = orc.direct(pos, q)
    return _T1["d"]


def test_split_count_matches_continuity_experiment(orc):
    # Sec. 3.2: 475 of 23040 charges split at 2d = 1/1024 with 8^3 cells and
    # order 4; only interior cell faces split in free space.
    N, L, n, two_d, ns_paper = load_golden("split_count.txt")[0]
    w, pos, q = workloads.workload_inputs("t1")
    ns, nf = orc.split_count(pos, int(L), int(n), FREE_C, split_d=two_d / 2)
    sd = np.sqrt(ns_paper)
    assert abs(ns - ns_paper) < 3 * sd
    # expectation for uniform charges: 7 interior faces per axis
    expect = N * (1 - (1 - 7 * two_d) ** 3)
    assert abs(ns - expect) < 3 * np.sqrt(expect)
    # every split charge adds n-1 fragments per split axis (n even)
    assert nf > N + (n - 1) * ns - 1


@pytest.mark.parametrize("mode", [FREE, FREE_C, PER, PER_C])
def test_reflection_and_axis_permutation_symmetry(orc, mode):
    pos, q = _inputs(256, 3)
    d = 0.01 if mode in (FREE_C, PER_C) else 0.0
    a = orc.fmm(pos, q, 3, 4, mode, split_d=d)
    # x -> 1 - x (periodic: wrap the reflected coordinate)
    ref = pos.copy()
    ref[:, 0] = np.mod(1.0 - ref[:, 0], 1.0) if mode in (PER, PER_C) else 1.0 - ref[:, 0]
    b = orc.fmm(ref, q, 3, 4, mode, split_d=d)
    scale = np.abs(a["phi"]).max()
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-11 * scale
    assert np.abs(a["field"][:, 0] + b["field"][:, 0]).max() < 1e-9 * np.abs(a["field"]).max()
    perm = pos[:, [1, 2, 0]]
    c = orc.fmm(perm, q, 3, 4, mode, split_d=d)
    assert np.abs(a["phi"] - c["phi"]).max() < 1e-11 * scale
    assert np.abs(a["field"][:, [1, 2, 0]] - c["field"]).max() < 1e-9 * np.abs(a["field"]).max()


@pytest.mark.parametrize("mode", [FREE, PER_C])
def test_dE_dq_is_phi_exactly(orc, mode):
    # E is quadratic in the charges, so a central difference in q_i is exact
    pos, q = _inputs(128, 5)
    d = 0.02 if mode == PER_C else 0.0
    a = orc.fmm(pos, q, 2, 4, mode, split_d=d)
    for i in (0, 17, 99):
        eps = 1e-3
        dq = np.zeros_like(q)
        dq[i] = eps
        if mode == PER_C:      # stay neutral: move the charge from another one
            dq[(i + 1) % 128] = -eps
        ep = orc.fmm(pos, q + dq, 2, 4, mode, split_d=d)["energy"]
        em = orc.fmm(pos, q - dq, 2, 4, mode, split_d=d)["energy"]
        fd = (ep - em) / (2 * eps)
        ref = a["phi"][i] - (a["phi"][(i + 1) % 128] if mode == PER_C else 0.0)
        assert abs(fd - ref) < 1e-9 * np.abs(a["phi"]).max()


@pytest.mark.parametrize("mode", [FREE, FREE_C, PER, PER_C])
def test_field_is_minus_energy_gradient(orc, mode):
    # central difference of the energy in the position of one charge
    pos, q = _inputs(150, 9)
    L, n = 2, 4
    s = 0.25
    d = 0.02 if mode in (FREE_C, PER_C) else 0.0
    # charge 0 inside a split zone (continuous modes), charge 1 well inside a cell
    pos[0] = [0.5 + 0.3 * d if d else 0.6, 0.1, 0.7]
    pos[1] = [0.375, 0.62, 0.13]
    a = orc.fmm(pos, q, L, n, mode, split_d=d)
    for i in (0, 1):
        for ax in range(3):
            h = 1e-6
            p1, p2 = pos.copy(), pos.copy()
            p1[i, ax] += h
            p2[i, ax] -= h
            fd = (orc.fmm(p1, q, L, n, mode, split_d=d)["energy"] -
                  orc.fmm(p2, q, L, n, mode, split_d=d)["energy"]) / (2 * h)
            ref = -q[i] * a["field"][i, ax]
            assert abs(fd - ref) < 1e-5 * max(1.0, abs(ref)), (i, ax, fd, ref)
    assert s > 2 * d


def _energy_track(orc, pos, q, i, xs, mode, L, n, d):
    out = []
    for x in xs:
        p = pos.copy()
        p[i, 0] = x
        out.append(orc.fmm(p, q, L, n, mode, split_d=d)["energy"])
    return np.array(out)


@pytest.mark.parametrize("face,modes", [(0.5, (FREE_C, FREE)), (0.0, (PER_C, PER))])
def test_energy_continuity_across_face(orc, face, modes):
    # Sec. 3.2 / Sec. 4.2: with the split the energy is continuous when a
    # charge crosses a cell face (face 0.5) or the periodic wall (face 0);
    # without it the energy jumps.  Continuity test: the largest step in E
    # shrinks ten-fold when the step in x does; a jump does not shrink.
    pos, q = _inputs(512, 11)
    L, n = 3, 4
    d = 1.0 / 2048
    ratios = {}
    for mode in modes:
        mx = []
        for step in (d / 20, d / 200):
            xs = face + step * (np.arange(8) - 3.5)
            if mode in (PER, PER_C):
                xs = np.mod(xs, 1.0)
            E = _energy_track(orc, pos, q, 0, xs, mode, L, n, d)
            mx.append(np.abs(np.diff(E)).max())
        ratios[mode] = mx[0] / mx[1]
    cont, plain = modes
    assert ratios[cont] > 6.0, ratios
    assert ratios[plain] < 2.0, ratios


def test_periodic_matches_ewald_at_approximation_level(orc):
    pos, q = _inputs(600, 13)
    ref_phi, ref_field = orc.ewald(pos, q)
    for mode in (PER, PER_C):
        a = orc.fmm(pos, q, 3, 5, mode, split_d=1.0 / 4096)
        ephi = np.linalg.norm(a["phi"] - ref_phi) / np.linalg.norm(ref_phi)
        assert ephi < 5e-3, (mode, ephi)
        # unsplit charges: field at approximation level
        e = np.linalg.norm(a["field_paper"] - ref_field) / np.linalg.norm(ref_field)
        assert e < 5e-3, (mode, e)
        assert abs(a["energy"] - 0.5 * (q * ref_phi).sum()) < 5e-3 * np.abs(0.5 * q * ref_phi).sum()


def test_periodic_invariant_under_box_translation(orc):
    pos, q = _inputs(200, 17)
    a = orc.fmm(pos, q, 2, 4, PER_C, split_d=0.01)
    b = orc.fmm(pos + np.array([1.0, -2.0, 3.0]), q, 2, 4, PER_C, split_d=0.01)
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-11 * np.abs(a["phi"]).max()


def test_paper_force_rule_agrees_off_the_split_zones(orc):
    pos, q = _inputs(300, 19)
    a = orc.fmm(pos, q, 3, 4, FREE_C, split_d=0.004)
    same = np.all(a["field"] == a["field_paper"], axis=1)
    assert same.mean() > 0.8
    ns, _ = orc.split_count(pos, 3, 4, FREE_C, split_d=0.004)
    assert (~same).sum() <= ns


def test_error_codes(orc):
    pos, q = _inputs(20, 23)
    with pytest.raises(orc.OracleError) as e:
        orc.fmm(pos + 1.5, q, 2, 4, FREE)
    assert e.value.code == -2
    with pytest.raises(orc.OracleError) as e:
        orc.fmm(pos, q + 1.0, 2, 4, PER)
    assert e.value.code == -3
    p2 = pos.copy()
    p2[3, 1] = np.nan
    with pytest.raises(orc.OracleError) as e:
        orc.fmm(p2, q, 2, 4, FREE)
    assert e.value.code == -4
    with pytest.raises(orc.OracleError) as e:
        orc.fmm(pos, q, 1, 4, FREE)
    assert e.value.code == -1
    # x = box on the upper wall belongs to the last cell in free space
    p3 = pos.copy()
    p3[0] = [1.0, 1.0, 1.0]
    orc.fmm(p3, q, 2, 4, FREE)


def test_reduced_nodes_lower_error_at_order4_only(orc):
    # Sec. 4.1: moving the n-division points inside the cube, their spacing
    # scaled by 1/1.2, lowers Error1 at order 4 (the paper: by about 20%),
    # and the gain fades at orders >= 6.  On the Table 1 shape the oracle
    # gives ratios 0.50 (n = 4) and 1.10 (n = 6); the pin checks the
    # direction and the fading, not the size (the paper's charges are not
    # available).
    w, pos, q = workloads.workload_inputs("t1")
    ref_phi, _ = _direct_t1(orc)

    def e1(n, shrink):
        a = orc.fmm(pos, q, 3, n, node_shrink=shrink)
        return np.mean(np.abs((a["phi"] - ref_phi) / ref_phi))

    assert e1(4, 1 / 1.2) < 0.85 * e1(4, 1.0)
    assert e1(6, 1 / 1.2) > 0.9 * e1(6, 1.0)


@pytest.mark.parametrize("mode", [FREE, PER_C])
def test_reduced_nodes_tree_equals_pairwise_closed_form(orc, mode):
    # the invariance property holds for any node placement, so the tree
    # passes with shrunk nodes still reproduce the pairwise closed form
    pos, q = _inputs(150, 31 + mode)
    d = 0.02 if mode == PER_C else 0.0
    a = orc.fmm(pos, q, 2, 4, mode, split_d=d, node_shrink=1 / 1.2)
    b = orc.fmm_pairwise(pos, q, 2, 4, mode, split_d=d, node_shrink=1 / 1.2)
    assert np.abs(a["phi"] - b["phi"]).max() <= 1e-12 * np.abs(b["phi"]).max()
    c = orc.fmm(pos, q, 2, 4, mode, split_d=d)
    assert np.abs(a["phi"] - c["phi"]).max() > 1e-8 * np.abs(c["phi"]).max()
