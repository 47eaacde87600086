"""The water-like periodic workload as a sequence of evaluations: 3145728
charges (1048576 rigid 3-site molecules), l_f = 7, n = 4, continuous
periodic boundary (Sec. 4.2), FP32 with the adjoint forces, 100 evaluations
with every charge moved by N(0, 1e-4) per axis (and wrapped) between them.

Checked at every step: the call succeeds (the device status word holds no
error), every output is finite, and the adjoint identities E = 1/2 sum q phi
and dE/dq = phi hold.  At the first and the last step the FP32 forces are
compared with the FP64 form on the same positions (1e-5 relative RMS).  The
time per evaluation (forward + adjoint, positions already on the device) is
recorded in the test output folder.
"""
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
os.makedirs("gpurun_out", exist_ok=True)

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2212_13080_amd as eq  # noqa: E402
import workloads  # noqa: E402
from gpu_common import rel_rms  # noqa: E402

STEPS = 100


def test_water_trajectory():
    w, pos, q = workloads.workload_inputs("c5")
    print(f"case {w.name} trajectory of {STEPS} evaluations", flush=True)
    dev = torch.device("cuda:0")
    plan = eq.Plan(w.levels, w.order, w.boundary, eq.FP32, device=dev)
    plan64 = eq.Plan(w.levels, w.order, w.boundary, eq.FP64, device=dev)
    ws = plan.workspace(w.n)
    qt = torch.from_numpy(q).to(dev)
    one = torch.ones((), dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    rng = np.random.default_rng(5)
    pt = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    gpu_s = 0.0
    for step in range(STEPS):
        if step:
            pos = workloads.water_step(rng, pos)
        pt.copy_(torch.from_numpy(pos))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, phi, field = plan.forward(pt, qt, ws=ws, status=status)
        dx, dq = plan.backward(qt, one, ws=ws)
        torch.cuda.synchronize()
        gpu_s += time.perf_counter() - t0
        plan.check_status(status)
        e = E.item()
        assert np.isfinite(e)
        for t in (phi, field, dx, dq):
            assert bool(torch.isfinite(t).all())
        qp = float(torch.dot(qt, phi.double()).item())
        assert abs(e - 0.5 * qp) <= 1e-6 * float(torch.dot(qt.abs(), phi.double().abs()).item())
        assert rel_rms(dq.double().cpu().numpy(), phi.double().cpu().numpy()) <= 1e-6
        if step in (0, STEPS - 1):
            E64, _, _ = plan64.forward(pt, qt)
            dx64, _ = plan64.backward(qt, one)
            err = rel_rms(dx.double().cpu().numpy(), dx64.cpu().numpy())
            print(f"step {step}: E {e:.9e} (FP64 {E64.item():.9e}), FP32 force rel RMS {err:.2e}", flush=True)
            assert err <= 1e-5
    ms = gpu_s * 1e3 / STEPS
    with open("gpurun_out/c5_trajectory.txt", "w") as f:
        f.write(f"{w.name}: {STEPS} evaluations (forward + adjoint), {ms:.2f} ms each, "
                f"{w.n / (ms * 1e-3):.4g} particles/s\n")
