"""Helpers shared by the GPU tests (loaded only by tests marked gpu)."""
import functools

import numpy as np

import oracle
import workloads


def rel_rms(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@functools.lru_cache(maxsize=16)
def oracle_result(key, n, levels, order, boundary, split_d=0.0):
    """Oracle FMM on the seeded inputs of workload `key` at the given size."""
    w, pos, q = case_inputs(key, n, levels)
    r = oracle.fmm(pos, q, levels, order, boundary, split_d=split_d)
    return pos, q, r


def case_inputs(key, n, levels):
    w = workloads.WORKLOADS[key]
    if n == w.n and levels == w.levels:
        return workloads.workload_inputs(key)
    return workloads.small_variant(key, n, levels)
