"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Bars: FP64 mode 1e-10 relative; FP32 mode 1e-5 relative
RMS on forces (and potentials); energies relative to sum |q phi| / 2."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
os.makedirs("gpurun_out", exist_ok=True)

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2212_13080_amd as eq  # noqa: E402
import workloads  # noqa: E402
from gpu_common import case_inputs, oracle_result, rel_max, rel_rms  # noqa: E402

FREE, FREE_C, PER, PER_C = 0, 1, 2, 3
TOL = {eq.FP64: 1e-10, eq.FP32: 1e-5}


def run_gpu(pos, q, levels, order, boundary, precision, split_d=0.0, **kw):
    plan = eq.Plan(levels, order, boundary, precision, split_d=split_d, **kw)
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda()
    E, phi, field = plan.forward(pt, qt)
    dx, dq = plan.backward(qt, torch.ones((), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return dict(energy=E.item(), phi=phi.double().cpu().numpy(), field=field.double().cpu().numpy(),
                dEdx=dx.double().cpu().numpy(), dEdq=dq.double().cpu().numpy())


def check(g, r, q, tol, label=""):
    print(f"  {label}: phi {rel_max(g['phi'], r['phi']):.2e} field {rel_rms(g['field'], r['field']):.2e} "
          f"E {g['energy']:.10g} vs {r['energy']:.10g}", flush=True)
    if tol <= 1e-9:
        assert rel_max(g["phi"], r["phi"]) <= tol
        assert rel_max(g["field"], r["field"]) <= tol
    else:
        assert rel_rms(g["phi"], r["phi"]) <= tol
        assert rel_rms(g["field"], r["field"]) <= tol
    scale = 0.5 * np.abs(q * r["phi"]).sum()
    assert abs(g["energy"] - r["energy"]) <= tol * scale
    # adjoint: dE/dx = -q field, dE/dq = phi (same tolerance)
    ref_dx = -q[:, None] * r["field"]
    if tol <= 1e-9:
        assert rel_max(g["dEdx"], ref_dx) <= tol
        assert rel_max(g["dEdq"], r["phi"]) <= tol
    else:
        assert rel_rms(g["dEdx"], ref_dx) <= tol
        assert rel_rms(g["dEdq"], r["phi"]) <= tol


# (workload generator, N, levels, order, boundary, split_d) -- sizes the
# oracle finishes in seconds that still span many cells and ragged leaves
CASES = [
    ("c1", 4096, 3, 4, FREE, 0.0),
    ("c2", 32768, 4, 4, FREE, 0.0),
    ("c2", 20000, 3, 3, FREE, 0.0),
    ("c3", 16384, 3, 5, PER_C, 0.0),
    ("c3", 8000, 3, 5, PER, 0.0),
    ("c4", 8192, 3, 6, FREE_C, 0.0),
    ("c5", 12 * 10 ** 3, 4, 4, PER_C, 0.0),
    ("c1", 3000, 2, 7, FREE, 0.0),
    ("c1", 3000, 3, 2, FREE_C, 0.004),
]


@pytest.mark.parametrize("precision", [eq.FP64, eq.FP32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-N{c[1]}-l{c[2]}-n{c[3]}-b{c[4]}")
def test_parity_small(case, precision):
    key, n, levels, order, boundary, d = case
    print(f"case {case} precision {precision}", flush=True)
    pos, q, r = oracle_result(key, n, levels, order, boundary, d)
    g = run_gpu(pos, q, levels, order, boundary, precision, split_d=d)
    check(g, r, q, TOL[precision], f"{key} {precision}")


def test_parity_c2_full_size_f32():
    # the benchmark workload itself, every output compared
    w, pos, q = workloads.workload_inputs("c2")
    print(f"case c2 full N={w.n}", flush=True)
    r = oracle.fmm(pos, q, w.levels, w.order, w.boundary)
    g = run_gpu(pos, q, w.levels, w.order, w.boundary, eq.FP32)
    check(g, r, q, TOL[eq.FP32], "c2 full f32")


def test_parity_c2_full_size_f64():
    w, pos, q = workloads.workload_inputs("c2")
    print(f"case c2 full N={w.n} f64", flush=True)
    r = oracle.fmm(pos, q, w.levels, w.order, w.boundary)
    g = run_gpu(pos, q, w.levels, w.order, w.boundary, eq.FP64)
    check(g, r, q, TOL[eq.FP64], "c2 full f64")


@pytest.mark.parametrize("precision", [eq.FP64, eq.FP32], ids=["f64", "f32"])
def test_edge_cases(precision):
    rng = np.random.default_rng(77)
    # one charge: no interactions at all
    g = run_gpu(np.array([[0.3, 0.4, 0.5]]), np.array([1.0]), 2, 4, FREE, precision)
    assert g["energy"] == 0.0 and g["phi"][0] == 0.0
    # all charges in one finest cell: pure near field
    pos = 0.5 + 0.1 * rng.random((50, 3))
    q = rng.uniform(-1, 1, 50)
    r = oracle.fmm(pos, q, 3, 4, FREE)
    check(run_gpu(pos, q, 3, 4, FREE, precision), r, q, TOL[precision], "one cell")
    # charges exactly on cell faces, on the upper wall and at corners
    pos = rng.integers(0, 9, (200, 3)) / 8.0
    pos = np.unique(pos, axis=0)
    q = rng.uniform(-1, 1, pos.shape[0])
    r = oracle.fmm(pos, q, 3, 4, FREE)
    check(run_gpu(pos, q, 3, 4, FREE, precision), r, q, TOL[precision], "faces")
    qn = q - q.mean()
    pos_p = np.mod(pos, 1.0)
    pos_p, idx = np.unique(pos_p, axis=0, return_index=True)
    qn = qn[idx] - qn[idx].mean()
    for b in (PER, PER_C):
        # every charge sits on three faces: up to 4^3 pieces each
        r = oracle.fmm(pos_p, qn, 3, 4, b, split_d=0.01)
        g = run_gpu(pos_p, qn, 3, 4, b, precision, split_d=0.01, max_fragments=64 * qn.size)
        tol = TOL[precision]
        if b == PER_C and precision == eq.FP32:
            # Here every force component comes from the split derivative
            # sum_m dw_m phi(p_m) (|dw| up to ~5/(2d)), which amplifies the
            # ~1e-6 relative error of the float local vectors by about s/(2d)
            # = 6: the bound for an all-split set is 5e-5 (derived, not the
            # 1e-5 of ordinary inputs, where few charges are split).
            tol = 5e-5
        check(g, r, qn, tol, f"faces b{b}")


def test_empty_input():
    plan = eq.Plan(3, 4, FREE, eq.FP32)
    E, phi, field = plan.forward(torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                                 torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert E.item() == 0.0 and phi.numel() == 0


def test_error_codes():
    rng = np.random.default_rng(5)
    pos = torch.from_numpy(rng.random((100, 3))).cuda()
    q = torch.from_numpy(rng.uniform(-1, 1, 100)).cuda()
    plan = eq.Plan(3, 4, FREE, eq.FP32)
    with pytest.raises(eq.EqfmmError) as e:
        plan.forward(pos + 1.5, q)
    assert e.value.code == -2
    bad = pos.clone()
    bad[7, 1] = float("nan")
    with pytest.raises(eq.EqfmmError) as e:
        plan.forward(bad, q)
    assert e.value.code == -4
    pplan = eq.Plan(3, 4, PER, eq.FP32)
    with pytest.raises(eq.EqfmmError) as e:
        pplan.forward(pos, q.abs())
    assert e.value.code == -3
    # fragment capacity too small for the split charge set
    cplan = eq.Plan(3, 4, FREE_C, eq.FP32, split_d=0.02, max_fragments=101)
    with pytest.raises(eq.EqfmmError) as e:
        cplan.forward(pos, q)
    assert e.value.code == -5
    with pytest.raises(eq.EqfmmError) as e:
        eq.Plan(1, 4, FREE, eq.FP32)
    assert e.value.code == -1
    # backward without a forward on that workspace
    fresh = eq.Plan(3, 4, FREE, eq.FP32)
    with pytest.raises(eq.EqfmmError) as e:
        fresh.backward(q, torch.ones((), dtype=torch.float64, device="cuda"))
    assert e.value.code == -7
    # the plan still works after errors
    E, _, _ = plan.forward(pos, q)
    assert np.isfinite(E.item())


@pytest.mark.parametrize("case", [("c1", 4096, 3, 4, FREE), ("c3", 8000, 3, 5, PER_C), ("c4", 4096, 3, 6, FREE_C)],
                         ids=lambda c: f"{c[0]}-b{c[4]}")
def test_async_forward_parity(case):
    """eqfmm_forward_async: status 0 and the FP32 parity bar against the
    oracle, with the adjoint enqueued right behind it."""
    key, n, levels, order, boundary = case
    print(f"case {case}", flush=True)
    pos, q, r = oracle_result(key, n, levels, order, boundary)
    plan = eq.Plan(levels, order, boundary, eq.FP32)
    pt, qt = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    E, phi, field = plan.forward(pt, qt, status=status)
    dx, dq = plan.backward(qt, torch.ones((), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert status.item() == 0
    g = dict(energy=E.item(), phi=phi.double().cpu().numpy(), field=field.double().cpu().numpy(),
             dEdx=dx.double().cpu().numpy(), dEdq=dq.double().cpu().numpy())
    check(g, r, q, TOL[eq.FP32], f"{key} async")


def test_async_error_status():
    """Data-dependent errors through the status word; the kernels stay in
    range whatever the input, and the plan keeps working afterwards."""
    rng = np.random.default_rng(6)
    pos = torch.from_numpy(rng.random((100, 3))).cuda()
    q = torch.from_numpy(rng.uniform(-1, 1, 100)).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def code(plan, p, qq):
        status.fill_(99)
        plan.forward(p, qq, status=status)
        torch.cuda.synchronize()
        return status.item()

    plan = eq.Plan(3, 4, FREE, eq.FP32)
    assert code(plan, pos + 1.5, q) == -2
    bad = pos.clone()
    bad[3, 0] = float("inf")
    assert code(plan, bad, q) == -4
    assert code(eq.Plan(3, 4, PER, eq.FP32), pos, q.abs()) == -3
    small = eq.Plan(3, 4, FREE_C, eq.FP32, split_d=0.02, max_fragments=101)
    assert code(small, pos, q) == -5
    with pytest.raises(eq.EqfmmError) as e:
        eq.Plan.check_status(status)
    assert e.value.code == -5
    # a set that fits the same small capacity (charges near finest-cell
    # centres, so none is split) is computed correctly
    cells = rng.integers(0, 8, (8, 3))
    inner = torch.from_numpy((cells + 0.5 + rng.uniform(-0.08, 0.08, (8, 3))) / 8.0).cuda()
    qi = torch.from_numpy(rng.uniform(-1, 1, 8)).cuda()
    assert code(small, inner, qi) == 0
    E, phi, _ = small.forward(inner, qi)
    ref = oracle.fmm(inner.cpu().numpy(), qi.cpu().numpy(), 3, 4, FREE_C, split_d=0.02)
    assert abs(E.item() - ref["energy"]) <= 1e-5 * 0.5 * np.abs(qi.cpu().numpy() * ref["phi"]).sum()
    assert code(plan, pos, q) == 0


def test_autograd_matches_oracle_and_finite_differences():
    # energy via forward, dE/dx and dE/dq via the adjoint kernel
    w, pos, q = case_inputs("c2", 8192, 3)
    r = oracle.fmm(pos, q, 3, 4, FREE)
    plan = eq.Plan(3, 4, FREE, eq.FP64)
    pt = torch.from_numpy(pos).cuda().requires_grad_(True)
    qt = torch.from_numpy(q).cuda().requires_grad_(True)
    E, phi, field = eq.energy(pt, qt, plan)
    (3.0 * E).backward()
    gx, gq = pt.grad.cpu().numpy(), qt.grad.cpu().numpy()
    assert rel_max(gx, -3.0 * q[:, None] * r["field"]) < 1e-10
    assert rel_max(gq, 3.0 * r["phi"]) < 1e-10
    # central differences in FP64 on charges away from cell faces and from
    # close neighbours (the O(h^2) term grows as 1/r^4 near a close pair)
    rng = np.random.default_rng(3)
    s = 1.0 / 8
    u = np.mod(pos / s, 1.0)
    d2 = ((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, 1.0)
    ok = np.where(np.all((u > 0.05) & (u < 0.95), axis=1) & (d2.min(1) > 0.02 ** 2))[0]
    idx = rng.choice(ok, 16, replace=False)
    h = 1e-6
    for i in idx:
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            ep = plan.forward(torch.from_numpy(pp).cuda(), torch.from_numpy(q).cuda())[0].item()
            em = plan.forward(torch.from_numpy(pm).cuda(), torch.from_numpy(q).cuda())[0].item()
            fd = (ep - em) / (2 * h)
            assert abs(fd - gx[i, a] / 3.0) < 1e-5 * max(1.0, abs(gx[i, a] / 3.0)), (i, a, fd, gx[i, a] / 3)


BF16_CASES = [("c2", 32768, 4, 4, FREE, 0.0), ("c4", 8192, 3, 6, FREE_C, 0.0), ("c3", 16384, 3, 5, PER_C, 0.0)]


@pytest.mark.parametrize("case", BF16_CASES, ids=lambda c: f"{c[0]}-N{c[1]}-l{c[2]}-n{c[3]}-b{c[4]}")
def test_bf16_far_field_error_bound(case):
    # bf16 inputs to the far-field products (unit roundoff 2^-8), float
    # accumulation: the error is stated against the FP64 oracle, not parity
    key, n, levels, order, boundary, d = case
    pos, q, r = oracle_result(key, n, levels, order, boundary, d)
    g = run_gpu(pos, q, levels, order, boundary, eq.FP32_BF16FAR, split_d=d)
    f32 = run_gpu(pos, q, levels, order, boundary, eq.FP32, split_d=d)
    e_phi, e_fld = rel_rms(g["phi"], r["phi"]), rel_rms(g["field"], r["field"])
    e_E = abs(g["energy"] - r["energy"]) / (0.5 * np.abs(q * r["phi"]).sum())
    print(f"  bf16 {key}: phi {e_phi:.2e} field {e_fld:.2e} E {e_E:.2e}  "
          f"(f32: phi {rel_rms(f32['phi'], r['phi']):.2e} field {rel_rms(f32['field'], r['field']):.2e})",
          flush=True)
    with open("gpurun_out/bf16_errors.txt", "a") as f:
        f.write(f"{key} N={n} l={levels} n={order} b={boundary}: phi {e_phi:.3e} field {e_fld:.3e} E {e_E:.3e}\n")
    # stated bound: 5e-3 (plain modes); continuous modes 2e-2, because the
    # split derivative amplifies the far-field input rounding by ~s/(2d)
    bound = 2e-2 if boundary in (FREE_C, PER_C) else 5e-3
    assert e_phi < bound and e_fld < bound and e_E < 1e-4


# Sec. 4.1: the n-division points inside the cube, spacing scaled by 1/1.2.
# FP64 is held to 1e-10.  In FP32 the bar is 1e-5 at n = 4; at n = 5 and 6
# the bound is 1e-4: with the points inside the cube the child-to-parent
# shift extrapolates, and its absolute column sums per axis grow from 2.17
# to 3.71 (n = 5) and from 2.99 to 7.18 (n = 6), so the float rounding of
# the upward and downward passes is amplified about (3.71/2.17)^3 = 5 and
# (7.18/2.99)^3 = 14 times more per level than with the default points.
@pytest.mark.parametrize("precision", [eq.FP64, eq.FP32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", [("c2", 20000, 3, 4, FREE, 0.0, 1e-5), ("c3", 8192, 3, 5, PER_C, 0.0, 1e-4),
                                  ("c4", 8192, 3, 6, FREE_C, 0.0, 1e-4)],
                         ids=lambda c: f"{c[0]}-N{c[1]}-l{c[2]}-n{c[3]}-b{c[4]}")
def test_parity_reduced_nodes(case, precision):
    key, n, levels, order, boundary, d, tol32 = case
    print(f"case {case} precision {precision} node_shrink 1/1.2", flush=True)
    _, pos, q = case_inputs(key, n, levels)
    r = oracle.fmm(pos, q, levels, order, boundary, split_d=d, node_shrink=1 / 1.2)
    g = run_gpu(pos, q, levels, order, boundary, precision, split_d=d, node_shrink=1 / 1.2)
    check(g, r, q, TOL[eq.FP64] if precision == eq.FP64 else tol32, f"{key} {precision} shrink")


# phi is linear in q with a symmetric matrix in the free modes, so the
# gradient of sum_i c_i phi_i in q is phi evaluated with charges c.  Checked
# against the oracle (phi of c plus phi of q for the loss c.phi + E) and,
# in FP64, against central differences in q, which are exact up to rounding
# for a loss that is quadratic in q.
@pytest.mark.parametrize("precision", [eq.FP64, eq.FP32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", [("c2", 8192, 3, 4, FREE, 0.0), ("c4", 8192, 3, 6, FREE_C, 0.0)],
                         ids=lambda c: f"{c[0]}-N{c[1]}-l{c[2]}-n{c[3]}-b{c[4]}")
def test_phi_vjp_in_q(case, precision):
    key, n, levels, order, boundary, d = case
    print(f"case {case} precision {precision} phi vjp", flush=True)
    _, pos, q = case_inputs(key, n, levels)
    c = np.random.default_rng(11).uniform(-1, 1, n)
    ref = oracle.fmm(pos, c, levels, order, boundary)["phi"] + oracle.fmm(pos, q, levels, order, boundary)["phi"]
    plan = eq.Plan(levels, order, boundary, precision)
    pt = torch.from_numpy(pos).cuda()
    qt = torch.from_numpy(q).cuda().requires_grad_(True)
    ct = torch.from_numpy(c).cuda()
    E, phi, _ = eq.energy(pt, qt, plan)
    ((ct * phi.double()).sum() + E).backward()
    gq = qt.grad.cpu().numpy()
    if precision == eq.FP64:
        assert rel_max(gq, ref) <= 1e-10
        v = np.random.default_rng(12).uniform(-1, 1, n)
        h = 1e-3

        def loss(qq):
            Ev, phv, _ = plan.forward(pt, torch.from_numpy(qq).cuda())
            return float((ct * phv).sum().item() + Ev.item())

        fd = (loss(q + h * v) - loss(q - h * v)) / (2 * h)
        assert abs(fd - np.dot(gq, v)) <= 1e-9 * np.abs(gq * v).sum()
    else:
        assert rel_rms(gq, ref) <= 1e-5
    # phi is not differentiable in the positions: asking for it fails loudly
    pt2 = pt.clone().requires_grad_(True)
    E2, phi2, _ = eq.energy(pt2, qt, plan)
    with pytest.raises(NotImplementedError):
        (ct * phi2.double()).sum().backward()
