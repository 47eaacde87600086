"""Continuity of the energy on the GPU (Sec. 2.3 for cell faces, Sec. 4.2 for
the periodic wall), on the full 2097152-charge periodic workload (l_f = 6,
n = 5) in the FP64 form.

One charge is moved along x across a finest-cell face (x = 0.5, a face on
every level) or across the periodic wall (x = 0), in steps of 1e-6, and the
total energy is evaluated at every position.  With the split the energy is
a smooth function of the position: over a step this small its second
difference is many orders below its first difference.  Without the split the
charge changes cell, near list and far-field representation at the face, and
the energy jumps by the method's truncation error: the largest second
difference is then the jump, far above the continuous mode's.

The same track in free space (x = 0.5 only) compares the free-continuous
and plain free modes.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
os.makedirs("gpurun_out", exist_ok=True)

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2212_13080_amd as eq  # noqa: E402
import workloads  # noqa: E402

STEP = 1e-6
POINTS = 9


def energy_track(mode, pos, q, i, xs, levels, order):
    plan = eq.Plan(levels, order, mode, eq.FP64, device="cuda:0")
    pt, qt = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    ws = plan.workspace(len(q))
    out = []
    for x in xs:
        pt[i, 0] = float(x)
        E, _, _ = plan.forward(pt, qt, want_phi=False, want_field=False, ws=ws)
        out.append(E.item())
    return np.array(out)


def smoothness(E):
    """Largest second difference over the largest first difference."""
    return float(np.abs(np.diff(E, 2)).max() / np.abs(np.diff(E)).max())


@pytest.mark.parametrize("face,modes", [
    (0.5, (eq.PERIODIC_CONTINUOUS, eq.PERIODIC)),
    (0.0, (eq.PERIODIC_CONTINUOUS, eq.PERIODIC)),
    (0.5, (eq.FREE_CONTINUOUS, eq.FREE)),
])
def test_energy_continuity_full_size(face, modes):
    w, pos, q = workloads.workload_inputs("c3")
    pos = pos.copy()
    i = 12345
    xs = face + STEP * (np.arange(POINTS) - (POINTS - 1) / 2)
    xs = np.mod(xs, 1.0)
    # keep the charge away from the y and z split zones: only x decides
    pos[i, 1:] = [0.3 + 0.5 / 64, 0.7 + 0.5 / 64]
    res, d2 = {}, {}
    for mode in modes:
        E = energy_track(mode, pos, q, i, xs, w.levels, w.order)
        res[mode] = smoothness(E)
        d2[mode] = float(np.abs(np.diff(E, 2)).max())
        line = (f"face {face} mode {mode}: max|dE| {np.abs(np.diff(E)).max():.3e} "
                f"max|d2E| {d2[mode]:.3e}")
        print(line, flush=True)
        with open("gpurun_out/continuity.txt", "a") as f:
            f.write(line + "\n")
    cont, plain = modes
    assert res[cont] < 1e-2, res
    # the jump of the plain mode stands far above the curvature of the
    # continuous mode's energy
    assert d2[plain] > 30 * d2[cont], d2
