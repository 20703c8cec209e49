"""The 64-instance batch at its full size (2.79e6 cells, 7.7e8 particles per step), as the
benchmark runs it (each instance numbered along a Morton curve, energy-exact sampling): the
FP64 batch against the oracle run instance by instance, over its first two steps, for a
sample of instances that spans the sizes, the two kinds and the Knudsen range (the oracle
runs them in parallel processes on the host); every count of every sampled instance
identical, fields within 1e-12.  The FP32 batch's error against the same oracle runs is
stated per instance (written to gpurun_out/fp32_error_batch64.json)."""
import json
import multiprocessing as mp
import os
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

from parity import BATCH_TOTALS, INT_KEYS, compare_fields

pytestmark = pytest.mark.gpu

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
STEPS = 2
# instances of the batch: the two with the most particles (tubes of 1.4e5 and 1.7e5 cells), the
# smallest cavities and tubes, the smallest and largest Knudsen numbers (6: 1e-4, 59: 0.82),
# the two cavities where the printed pairs of Sec. 2.4(b) fail later on (37, 51), and others
SAMPLE = (0, 1, 2, 5, 6, 13, 20, 27, 36, 37, 46, 51, 55, 59, 60, 62, 63)


def _say(*a):
    print("[gpu-batch-full]", *a, flush=True)
    sys.stdout.flush()


def _instance(k):
    w = wl.morton_numbered(wl.batched_instance(wl.batched_specs()[k]))
    w.params.sampling = 1
    return w


def _oracle_run(k):
    """Worker (a fresh process: no GPU): instance k alone in the oracle, with its instance
    index, for STEPS steps; W, P and the statistics after each step."""
    import oracle

    w = _instance(k)
    o = oracle.Oracle(w.mesh, w.params, instance=k)
    o.set_state(w.W0)
    out = []
    for _ in range(STEPS):
        o.step()
        W, P, _ = o.state()
        out.append((W, P, o.stats()))
    vol, _, _ = o.geometry()
    return k, vol, out


@pytest.mark.timeout(900)
def test_full_batch_first_steps_against_oracle_per_instance():
    from paper_2007_13091_amd.ugkwp import Solver

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ctx = mp.get_context("spawn")
    old = os.environ.get("PYTHONPATH", "")
    os.environ["PYTHONPATH"] = root + (os.pathsep + old if old else "")
    pool = ctx.Pool(processes=min(len(SAMPLE), 12))
    pending = pool.map_async(_oracle_run, SAMPLE, chunksize=1)
    _say("oracle runs started for instances", SAMPLE)
    ws = [_instance(k) for k in range(64)]
    results = {}
    # capacity for two steps: about N_ref per cell, plus the ceiling's two per cell and step
    caps = [int(1.1 * w.params.n_ref * w.mesh.n_cells + 8 * w.mesh.n_cells) + 65536 for w in ws]
    for prec in (0, 1):
        g = Solver([w.mesh for w in ws], [w.params for w in ws], precision=prec, capacity=caps)
        g.init_state(np.concatenate([w.W0 for w in ws]))
        steps = []
        for n in range(STEPS):
            g.step(1)
            stats = {k: g.instance_stats(k) for k in SAMPLE}
            steps.append((g.moments(0), g.moments(1), stats))
            _say("batch precision", prec, "step", n)
        cells = {k: g.instance_cells(k) for k in SAMPLE}
        g.close()
        del g
        results[prec] = (steps, cells)
    import torch

    torch.cuda.empty_cache()
    oracle_out = dict((k, (vol, out)) for k, vol, out in pending.get(timeout=800))
    pool.close()
    pool.join()
    errs = []
    for k in SAMPLE:
        vol, out = oracle_out[k]
        steps64, cells = results[0]
        c0, c1 = cells[k]
        for n in range(STEPS):
            Wo, Po, so = out[n]
            Wg, Wpg, sg = steps64[n]
            for key in INT_KEYS:
                if key in BATCH_TOTALS:
                    continue
                assert sg[k][key] == so[key], f"instance {k} step {n} {key}: gpu {sg[k][key]} oracle {so[key]}"
            compare_fields(Wg[c0:c1], Wo, Wpg[c0:c1] * vol[:, None], Po, vol, what=f"instance {k} step {n}")
        steps32, cells32 = results[1]
        W32 = steps32[-1][0][c0:c1]
        Wo = out[-1][0]
        rho32, rhoo = W32[:, 0], Wo[:, 0]
        T = lambda W: (2 / 3) * (W[:, 4] - 0.5 * (W[:, 1:4] ** 2).sum(1) / W[:, 0]) / W[:, 0]
        U = lambda W: np.linalg.norm(W[:, 1:4] / W[:, 0:1], axis=1)
        e = {"instance": k, "cells": int(c1 - c0), "n_ref": ws[k].params.n_ref, "mu_ref": ws[k].params.mu_ref,
             "step": STEPS}
        for name, a, b, sc in (("rho", rho32, rhoo, rhoo.mean()), ("U", U(W32), U(Wo), np.sqrt(T(Wo).mean())),
                               ("T", T(W32), T(Wo), T(Wo).mean())):
            d = np.abs(a - b) / sc
            e[name] = {"L1": float(d.mean()), "Linf": float(d.max())}
        errs.append(e)
        _say("instance", k, "parity ok; FP32 L1 rho", e["rho"]["L1"])
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "fp32_error_batch64.json"), "w") as fh:
        json.dump({"protocol": f"FP32 batch vs the FP64 oracle per instance after {STEPS} steps from the initial "
                               "state (same Philox draws)", "instances": errs}, fh, indent=1)
    for e in errs:
        # far below the method's own noise, 1/sqrt(N_ref) per cell: in the tubes of 1.4e5-1.7e5
        # cells (h ~ 6e-6 to 2.4e-5) an FP32 position resolves only 1/400 to 1/100 of a cell,
        # and the particles that FP32 rounding puts on the other side of a face dominate
        bound = 0.1 / np.sqrt(e["n_ref"])
        for q in ("rho", "U", "T"):
            assert e[q]["L1"] < bound, e
