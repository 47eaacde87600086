"""Benchmark of the hot path: one step = forward (energy, potential, field)
+ adjoint (dE/dx, dE/dq) of the equivalent-charge FMM on one GPU, inputs
resident in HBM.  Prints one JSON line.

Default workload: 262144 charges uniform in the unit cube, charges uniform
in [-1, 1] minus their mean, 32^3 finest cells (l_f = 5), 4 points per axis,
free boundary, FP32 arithmetic with FP64 energy reduction.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm": 8000.0,            # GB/s
    "fp32_mfma": 157.3,       # TFLOP/s
    "fp64_mfma": 78.6,
    "bf16_mfma": 2500.0,
}


def counter_traffic(workload, prec):
    """HBM bytes per far-field launch from the committed hardware-counter
    record (profiles/m2l_c2_traffic.json), or None when that record is for
    another workload or precision or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "m2l_c2_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, rec["kernel_source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if sha != rec["kernel_source_sha256"] or rec["workload"] != workload or prec != 1:
        return None
    return rec["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default=None, help="f64 | f32 | bf16far (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--node-shrink", type=float, default=1.0,
                    help="spacing of the n-division points relative to the cell (Sec. 4.1: 1/1.2)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the side-by-side timing of the other precision forms")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="run one plain device copy of MB megabytes before the timed region "
                         "(reference kernel for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU spatial decomposition is not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2212_13080_amd as eq
    import workloads

    w, pos, q = workloads.workload_inputs(args.config)
    prec = {"f64": eq.FP64, "f32": eq.FP32, "bf16far": eq.FP32_BF16FAR, None: w.precision}[args.precision]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pt = torch.from_numpy(pos).to(dev)
    qt = torch.from_numpy(q).to(dev)
    one = torch.ones((), dtype=torch.float64, device=dev)
    peak_key = {eq.FP64: "fp64_mfma", eq.FP32: "fp32_mfma", eq.FP32_BF16FAR: "bf16_mfma"}
    dtype_name = {eq.FP64: "f64", eq.FP32: "f32", eq.FP32_BF16FAR: "f32+bf16"}

    def run_form(prec, steps, warmup, stage_breakdown):
        """Time `steps` steps of one precision form; returns the timing, the
        far-field launch statistics and the last step's outputs."""
        plan = eq.Plan(w.levels, w.order, w.boundary, prec, node_shrink=args.node_shrink, device=dev)
        ws = plan.workspace(w.n)
        # Each step's forward writes its data-dependent status to this word
        # instead of blocking on it; it is checked after every
        # synchronisation (every step computes on the same inputs).
        status = torch.zeros(1, dtype=torch.int32, device=dev)

        def step():
            E, phi, field = plan.forward(pt, qt, ws=ws, status=status)
            dx, dq = plan.backward(qt, one, ws=ws)
            return E, phi, field, dx, dq

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        plan.check_status(status)
        # only the far-field launch is bracketed by events in the timed
        # region (an event pair costs a few microseconds)
        plan.profile(["m2l"])
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.check_status(status)
        prof = plan.profile_read()
        plan.profile(False)
        ms = (t1 - t0) * 1e3 / steps
        print(f"[bench] {w.name} {dtype_name[prec]}: {ms:.3f} ms/step, {w.n / (ms * 1e-3):.4g} particles/s",
              file=sys.stderr, flush=True)
        if stage_breakdown:
            # per-stage breakdown, in steps of their own after the timed region
            plan.profile(True)
            nb = min(steps, 5)
            for _ in range(nb):
                step()
            stages = plan.profile_read()
            plan.profile(False)
            plan.check_status(status)
            for k, v in stages.items():
                if v["launches"]:
                    print(f"[bench]   {k:8s} {v['ms'] / nb:8.4f} ms/step  launches/step "
                          f"{v['launches'] / nb:.0f}", file=sys.stderr, flush=True)
        # dominant kernel: the far-field products of all levels (one launch
        # per step; two in the bf16 mode)
        m2l = prof["m2l"]
        achieved = m2l["flops"] / (m2l["ms"] * 1e-3) / 1e12 if m2l["ms"] > 0 else 0.0
        roof = {"kernel": "m2l", "bound": "mfma", "achieved": round(achieved, 3),
                "peak": PEAKS[peak_key[prec]], "unit": "TFLOP/s",
                "frac": round(achieved / PEAKS[peak_key[prec]], 4),
                "avg_launch_ms": round(m2l["ms"] / max(m2l["launches"], 1), 5),
                "launches_per_step": m2l["launches"] / steps,
                "algorithmic_flops_per_step": m2l["flops"] / steps}
        del plan, ws
        return ms, roof, out

    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy * 2 ** 20 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms, roofline, out = run_form(prec, args.steps, args.warmup, True)
    value = w.n / (ms * 1e-3)
    roofline = dict(roofline, traffic=counter_traffic(w.name, prec))
    # the three forms side by side (plain FP64, FP32 + adjoint, BF16 far
    # field + adjoint), each on the same inputs
    forms = {}
    if not args.no_forms:
        for p in (eq.FP64, eq.FP32, eq.FP32_BF16FAR):
            if p == prec:
                fms, froof, fout = ms, roofline, out
            else:
                fms, froof, fout = run_form(p, max(args.steps // 4, 1), max(args.warmup // 4, 1), False)
            forms[dtype_name[p]] = {"value": round(w.n / (fms * 1e-3), 1), "ms_per_step": round(fms, 4),
                                    "m2l_frac": froof["frac"], "m2l_peak": froof["peak"],
                                    "m2l_avg_launch_ms": froof["avg_launch_ms"], "_out": fout}

    E, phi, field, dx, dq = out
    result = {
        "metric": "energy+force particles/s at 1e-5 rel. force error vs FP64 plain; % roofline",
        "value": round(value, 1), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_name[prec],
        "data": "synthetic",
        "config": {"workload": w.name, "n_charges": w.n, "levels": w.levels, "order": w.order,
                   "boundary": workloads.BOUNDARY_NAMES[w.boundary], "node_shrink": args.node_shrink},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # whole evaluations of the same workload, repeated until about 10 s
        # of host time (at most 50)
        runs, t0 = 0, time.perf_counter()
        while True:
            ref = oracle.fmm(pos, q, w.levels, w.order, w.boundary, node_shrink=args.node_shrink)
            runs += 1
            tc = time.perf_counter() - t0
            if tc >= 10.0 or runs >= 50:
                break
        result["cpu_baseline"] = {"value": round(w.n * runs / tc, 1), "unit": "particles/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": f"{runs} full evaluations of the same workload ({w.n} charges, "
                                            f"potential+field+energy), {tc:.2f} s"}
        Fr = q[:, None] * ref["field"]

        def errors(o):
            F = -o[3].double().cpu().numpy()
            return (float(np.linalg.norm(F - Fr) / np.linalg.norm(Fr)),
                    float(abs(o[0].item() - ref["energy"]) / abs(ref["energy"])))

        result["rel_rms_force_err"], result["rel_energy_err"] = errors(out)
        for f in forms.values():
            f["rel_rms_force_err"], f["rel_energy_err"] = errors(f["_out"])
    for f in forms.values():
        f.pop("_out")
    if forms:
        result["forms"] = forms
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
