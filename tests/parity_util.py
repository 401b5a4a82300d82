"""Shared helpers of the GPU parity tests (not a test module).

The oracle is plain single-threaded C called through ctypes, which releases
the GIL, so independent oracle calls (instances of a batch, tolerances of
one input) run side by side in threads.  Each call is still the plain
oracle; only the calls overlap.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

INT_KEYS = ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status")
VALUE_TOL = 1e-13


def threads() -> int:
    # the GPU machine gives a job 16 CPUs whatever os.cpu_count() reports
    return max(1, min(16, os.cpu_count() or 1))


def parallel(jobs: dict) -> dict:
    """Run {key: callable} in a thread pool; returns {key: result}."""
    with ThreadPoolExecutor(threads()) as ex:
        futs = {k: ex.submit(f) for k, f in jobs.items()}
        return {k: f.result() for k, f in futs.items()}


def check_instances(res, offsets, x, y, tols, opt=None):
    """Every instance j of a batched launch (results res[j], host vectors x,
    y, instance [offsets[j], offsets[j+1])) against the oracle on that
    instance alone: integer outputs bit for bit, the value within
    1e-13 * sum |x_i y_i|.  Returns the number of instances checked."""
    B = len(tols)

    def one(j):
        a, b = int(offsets[j]), int(offsets[j + 1])
        xs, ys = x[a:b], y[a:b]
        o = oracle.qdot(xs, ys, float(tols[j]), opt=opt)
        bad = [k for k in INT_KEYS if res[j][k] != o[k]]
        if o["status"] != oracle.OK:
            return j, bad, 0.0, 0.0
        return j, bad, abs(res[j]["value"] - o["value"]), oracle.abs_dot(xs, ys)

    with ThreadPoolExecutor(threads()) as ex:
        out = list(ex.map(one, range(B)))
    for j, bad, diff, scale in out:
        assert not bad, (j, bad, [(k, res[j][k]) for k in bad])
        assert diff <= VALUE_TOL * scale, (j, diff, scale)
    return len(out)


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()
