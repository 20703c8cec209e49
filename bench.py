"""Benchmark of the UGKWP hot path on one MI355X.

Headline workload: the batched form (64 independent shock-tube and cavity instances, 2.8e6
box cells, 50-500 particles per cell, Knudsen numbers 1e-4 to 1) in the FP32 form (flux and
transport in FP32; per-cell sums, W - W^p and energy -> T in FP64), every instance in one
launch per kernel, launch shapes autotuned, against the same 64 instances run one by one in
the FP64 plain form on the same GPU.  A step is one full time step of the scheme: wave flux,
sampling, free-flight times, free transport, particle sums and the cell update.

Prints ONE JSON line: particle moves/s (value) and cell-steps/s of the batched FP32 form;
the FP64 plain comparison; the FP32 form's one-step error against the FP64 plain form from the
same state, per instance; the roofline position of both particle kernels (timed live with hip
events on the library's stream over the timed steps) and of the whole step; the lid-driven
cavity legs (second order, after 1000 steps); side numbers; and the CPU oracle's rate on a
bounded sample of the batch (its first instances, one step each from their warm states).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# algorithmic bytes of one particle move: the particle state read once and written once
# (FP64: x 24 + u 24 + m 8 + cell 4 + uid 8 = 68 B; FP32 form: 12 + 12 + 4 + 4 + 8 = 40 B)
BYTES_PER_MOVE = {"double": 136, "float": 80}
# algorithmic bytes of the gather (S6): a survivor's record read and written with its cell,
# plus its bucket key read (FP64: 64 + 64 + 4 + 4 = 136 B; FP32: 36 + 40 + 4 = 80 B); a
# collided particle's velocity and mass read with its key (FP64: 48 + 4 = 52 B; FP32: 36 + 4)
BYTES_PER_SURVIVOR = {"double": 136, "float": 80}
BYTES_PER_COLLIDED = {"double": 52, "float": 40}
# algorithmic bytes of a first-order cell-step: W and P read and written, volume and the
# projections Delta S read (192 B), plus the face geometry (normal, area, owner and neighbour)
# of its share of the faces: box hex 3 faces (FP64 40 B each, FP32 24 B); second order adds
# the least-squares data of the cell (48 B) and the face-centre offsets (24 B per face)
BYTES_PER_CELL = {("hex", "double", 0): 312, ("hex", "float", 0): 264,
                  ("hex", "double", 2): 312 + 48 + 3 * 24, ("hex", "float", 2): 264 + 24 + 3 * 12}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CAVITY_START = 1000  # the cavity legs time the steps after this many (the paper's cavity runs
#                      thousands of steps; the survey's window is steps 1001-2000)
BATCH_START = 100    # the batched legs time the steps after this many


def code_text(src):
    """C++ source without its comments and with runs of white space made one space, so that
    an edit of a comment or of the layout leaves the digest alone (the sources hold no string
    literal with comment markers)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_digest(read=None):
    """Digest of the kernel sources' code (comments and layout aside); `read(name)` gives a
    source's text, by default the file in the package."""
    if read is None:
        def read(f):
            with open(os.path.join(ROOT, "paper_2007_13091_amd", "csrc", f)) as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_common.hpp"):
        h.update(code_text(read(f)).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from committed rocprofv3 counter runs,
    if the kernel source has not changed since they were taken (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("source_digest") != kernel_source_digest():
        return None
    return e.get("bytes_per_launch")


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)


def kernel_names(rtype, cfg, multi, ke=False):
    """Names of the two particle kernels as the profiler lists them (cfg: launch shapes; ke:
    the gas has internal degrees of freedom)."""
    return {"stream": f"k_stream<{rtype}, {cfg[0]}, {'true' if multi else 'false'}, {cfg[1]}>",
            "gather": f"k_gather<{rtype}, 1, {'true' if ke else 'false'}>"}


def timed_steps(s, steps):
    """K steps, eager launches, bracketed by device synchronisation, with hip events on the
    library's stream around the two particle kernels (transport and gather) in every step.
    Returns wall seconds, particle moves, the two kernels' average launch times (ms) and the
    statistics before and after."""
    import torch

    s.profile(True, slots=["stream", "gather"])
    s.profile_read()
    st0 = s.step(0, stats=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.step(0, stats=True)
    prof = s.profile_read()
    s.profile(False)
    kms = {k: prof[k][0] / max(prof[k][1], 1) for k in ("stream", "gather")}
    return t1 - t0, st1["moved_total"] - st0["moved_total"], kms, st0, st1


def kernel_roofline(kms, moves_per_step, last, rtype, names, workload):
    """Roofline position of the transport and the gather: algorithmic bytes per launch over
    the average launch time.  Transport: the particle moves of a step; gather: the survivors
    and collided particles of a step (those of the last timed step)."""
    algo = {"stream": BYTES_PER_MOVE[rtype] * moves_per_step,
            "gather": BYTES_PER_SURVIVOR[rtype] * last["n_alive"] + BYTES_PER_COLLIDED[rtype] * last["n_collided"]}
    out = {}
    for k in ("stream", "gather"):
        ach = algo[k] / (kms[k] * 1e-3) / 1e9
        out[k] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(names[k], workload),
                  "kernel": names[k], "kernel_avg_ms": round(kms[k], 4), "algorithmic_bytes_per_launch": int(algo[k])}
    dom = max(("stream", "gather"), key=lambda k: kms[k])
    return dom, out


def whole_step(ms_per_step, moves_per_step, cells, rtype, recon=0):
    """The whole step against HBM: the particle moves' and the cells' algorithmic bytes over
    the wall time of a step."""
    algo = BYTES_PER_MOVE[rtype] * moves_per_step + BYTES_PER_CELL[("hex", rtype, recon)] * cells
    ach = algo / (ms_per_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": int(algo)}


def _prim(W):
    rho = W[:, 0]
    U = W[:, 1:4] / rho[:, None]
    T = (2 / 3) * (W[:, 4] - 0.5 * rho * (U * U).sum(1)) / rho
    return rho, np.linalg.norm(U, axis=1), T


def field_error(Wa, Wb):
    """L1 (mean over cells) and Linf of rho, |U| and T of Wa against Wb, relative to the mean
    density, the thermal speed and the mean temperature of Wb."""
    ra, ua, ta = _prim(Wa)
    rb, ub, tb = _prim(Wb)
    out = {}
    for name, a, b, sc in (("rho", ra, rb, rb.mean()), ("U", ua, ub, np.sqrt(tb.mean())), ("T", ta, tb, tb.mean())):
        d = np.abs(a - b) / sc
        out[name] = {"L1": float(d.mean()), "Linf": float(d.max())}
    return out


def batch_workloads(sampling):
    from paper_2007_13091_amd import workloads as wl

    ws = [wl.morton_numbered(w) for w in wl.batched()]
    for w in ws:
        w.params.sampling = sampling
    return ws


def collisionless_fraction(w):
    """Smallest and largest e = exp(-dt/tau) over the cells of a box-hex workload's initial
    state: dt from the CFL rule with h = (volume / cells)^(1/3) (uniform cubic cells),
    tau = mu_ref T^omega / p."""
    xyz = np.asarray(w.mesh.xyz)
    h = (np.prod(xyz.max(0) - xyz.min(0)) / w.mesh.n_cells) ** (1.0 / 3.0)
    W = np.asarray(w.W0)
    K = int(round(2.0 / (w.params.gamma - 1.0) - 3.0))
    rho = W[:, 0]
    U = W[:, 1:4] / rho[:, None]
    T = (2.0 / (3.0 + K)) * (W[:, 4] / rho - 0.5 * (U * U).sum(1))
    dt = w.params.cfl * h / (np.abs(U) + 3.0 * np.sqrt(T)[:, None]).sum(1).max()
    tau = w.params.mu_ref * T ** w.params.omega / (rho * T)
    e = np.exp(-dt / tau)
    return float(e.min()), float(e.max())


def batch_capacity(w, steps):
    # Within a step a cell holds its old particles and the newly sampled ones (the collided are
    # removed only at its end).  The sample is about N_ref (1 - e) + 2 (the share of the hydro
    # wave's collisionless part, N_sam = 2 ceil(r)); the old ones are what the last steps kept:
    # a cell keeps the share e, so its count settles near N_ref + 2/(1 - e), and before that it
    # drifts up by up to two per step
    e_lo, e_hi = collisionless_fraction(w)
    drift = min(2.2 * steps, 2.2 / max(1.0 - e_hi, 1e-9) + 8.0)
    per_cell = 1.15 * w.params.n_ref * (2.0 - e_lo) + drift + 8.0
    return int(per_cell * w.mesh.n_cells) + 65536


def batch_capacities(ws, steps):
    """Capacities of the batch's instances for `steps` steps: the estimate above, or the plain
    bound 1.3 N_ref + 2.2 per step per cell where that is larger and the batch's total still fits
    a 32-bit particle index."""
    est = [batch_capacity(w, steps) for w in ws]
    plain = [max(e, int((1.3 * w.params.n_ref + 2.2 * steps) * w.mesh.n_cells) + 65536) for e, w in zip(est, ws)]
    return plain if sum(plain) < 2 ** 31 - 1024 else est


def batched_run(steps, warmup, start, sampling, cpu_sample_moves=0):
    """The batched FP32 form: `start` steps (of which the autotuner's trials), `warmup` more,
    then `steps` timed; then the same `steps` replayed from a captured hip graph (side number).
    Then each instance alone in the FP64 plain form, `start + warmup` steps, `steps` timed, and
    the FP32 form's one-step error from that instance's state (exported from the FP64 run and
    imported into both forms)."""
    import torch

    from paper_2007_13091_amd.ugkwp import Solver

    ws = batch_workloads(sampling)
    meshes, params = [w.mesh for w in ws], [w.params for w in ws]
    W0 = np.concatenate([w.W0 for w in ws])
    nc = int(sum(w.mesh.n_cells for w in ws))
    tuning = 13 * 2
    total = start + warmup + 2 * steps + 2
    caps = batch_capacities(ws, total)
    stream = torch.cuda.Stream()
    s = Solver(meshes, params, capacity=caps, precision=1, stream=stream)
    s.init_state(W0)
    s.step(max(start - tuning, 1), stats=False)
    cfg = s.autotune(steps_per_trial=1)
    # the warm-up steps time the first-order flux kernel (the hip events bracket it alone)
    s.profile(True, slots=["flux"])
    s.profile_read()
    s.step(warmup, stats=True)
    fl = s.profile_read()["flux"]
    s.profile(False)
    el, moves, kms, st0, st1 = timed_steps(s, steps)
    done_steps = int(st1["step"])
    names = kernel_names("float", cfg, True)
    workload = "batch64"
    dom, kr = kernel_roofline(kms, moves / steps, st1, "float", names, workload)
    faces = sum((6 * w.mesh.n_cells + int(w.mesh.bface_nodes.shape[0])) // 2 for w in ws)
    flux_ms = fl[0] / max(fl[1], 1)
    flux_name = f"k_flux<float, {cfg[3]}>"
    flux_ach = BYTES_PER_FACE_FP32 * faces / (flux_ms * 1e-3) / 1e9
    flux_roof = {"kernel": flux_name, "kernel_avg_ms": round(flux_ms, 4), "bound": "hbm", "achieved": round(flux_ach, 1),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(flux_ach / HBM_PEAK_GBS, 4),
                 "bytes_per_face": BYTES_PER_FACE_FP32, "faces": faces,
                 "traffic": measured_traffic(flux_name, workload), "timed": "the warm-up steps"}
    s.graph(True)
    s.step(1, stats=False)  # capture
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    s.step(steps, stats=False)
    torch.cuda.synchronize()
    tg = (time.perf_counter() - tg0) / steps * 1e3
    s.close()
    del s
    torch.cuda.empty_cache()
    ms = el / steps * 1e3
    out = {"value": moves / el, "ms_per_step": ms, "cell_steps_per_s": nc * steps / el,
           "particles_per_step": int(moves / steps), "steps": steps, "timed_after_step": done_steps - steps,
           "launch_config": {"stream_bs": cfg[0], "stream_ilp": cfg[1], "sample_wpb": cfg[2], "flux_bs": cfg[3]},
           "dominant": dom, "kernels": kr, "whole_step": whole_step(ms, moves / steps, nc, "float"),
           "flux": flux_roof,
           "graph_replay_ms_per_step": round(tg, 4), "cells": nc, "instances": len(ws)}
    # FP64 plain, one instance after the other (eager launches), then the one-step error
    pm, pt, pc = 0, 0.0, 0
    kt = {"stream": 0.0, "gather": 0.0}
    last64 = {"n_alive": 0, "n_collided": 0}
    errs = []
    flips = 0
    sample, sample_moves = [], 0  # warm states of the first instances, for the CPU baseline
    for k, (w, cap) in enumerate(zip(ws, caps)):
        g = Solver(w.mesh, w.params, capacity=cap, precision=0)
        g.init_state(w.W0)
        g.step(done_steps - steps, stats=False)
        e, mv, km, a, b = timed_steps(g, steps)
        pm += mv
        pt += e
        pc += w.mesh.n_cells * steps
        for q in kt:
            kt[q] += km[q] * steps
        last64["n_alive"] += b["n_alive"]
        last64["n_collided"] += b["n_collided"]
        st = g.export_state()
        if sample_moves < cpu_sample_moves:
            sample.append((k, w, st))
            sample_moves += mv / steps
        f = Solver(w.mesh, w.params, capacity=cap, precision=1)
        f.import_state(st)
        s64, s32 = g.step(1), f.step(1)
        flips += abs(s64["n_collided"] - s32["n_collided"]) + abs(s64["n_alive"] - s32["n_alive"])
        err = field_error(f.moments(0), g.moments(0))
        errs.append({"instance": k, "cells": w.mesh.n_cells, "n_ref": w.params.n_ref,
                     "mu_ref": w.params.mu_ref, "step": int(s64["step"]), **err})
        f.close()
        g.close()
        del f, g
        torch.cuda.empty_cache()
    p_ms = pt / steps * 1e3
    kms64 = {q: kt[q] / (len(ws) * steps) for q in kt}
    out["fp64_plain_one_by_one"] = {
        "value": pm / pt, "unit": "particle moves/s", "cell_steps_per_s": pc / pt, "ms_per_step": p_ms,
        "kernel_ms_per_step_sum": {q: round(kt[q] / steps, 4) for q in kt},
        "whole_step": whole_step(p_ms, pm / steps, nc, "double"),
        "kernels": {q: {"kernel_avg_ms_mean_over_instances": round(kms64[q], 4),
                        "achieved": round((BYTES_PER_MOVE["double"] * pm / steps if q == "stream" else
                                           BYTES_PER_SURVIVOR["double"] * last64["n_alive"] +
                                           BYTES_PER_COLLIDED["double"] * last64["n_collided"])
                                          / (kt[q] / steps * 1e-3) / 1e9, 1),
                        "unit": "GB/s", "peak": HBM_PEAK_GBS} for q in kt}}
    for q in kt:
        ach = out["fp64_plain_one_by_one"]["kernels"][q]["achieved"]
        out["fp64_plain_one_by_one"]["kernels"][q]["frac"] = round(ach / HBM_PEAK_GBS, 4)
    out["speedup_vs_fp64_plain_one_by_one"] = out["value"] / (pm / pt)
    worst = {v: max(e[v]["L1"] for e in errs) for v in ("rho", "U", "T")}
    worst_inf = {v: max(e[v]["Linf"] for e in errs) for v in ("rho", "U", "T")}
    out["stated_error"] = {
        "protocol": "one step of the FP32 form against one step of the FP64 plain form from the same state "
                    "(each instance's FP64 state after the timed steps, exported and imported into both; the same "
                    "Philox draws); FP64 plain matches the oracle to 1e-12 (parity tests)",
        "worst_over_instances_L1": worst, "worst_over_instances_Linf": worst_inf,
        "decision_flips": int(flips), "per_instance": errs}
    return out, sample


def cavity_leg(precision, steps, warmup, start, sampling=0, recon=2, prandtl=1.0):
    """The lid-driven cavity (Sec. 4.2) at 32^3, 400 particles per cell, second order
    (least-squares gradients with the Venkatakrishnan limiter, as the paper's cavity): `start`
    steps, `warmup` more, then `steps` timed.  sampling 2: the first-order g_p; prandtl != 1:
    the Shakhov model (with sampling 2 or 3)."""
    import torch

    from paper_2007_13091_amd import workloads as wl
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.morton_numbered(wl.cavity())
    w.params.sampling = sampling
    w.params.recon = recon
    w.params.prandtl = prandtl
    nc = w.mesh.n_cells
    s = Solver(w.mesh, w.params, precision=precision)
    s.init_state(w.W0)
    cfg = s.launch_config()
    s.step(start, stats=False)
    s.step(warmup, stats=True)
    el, moves, kms, st0, st1 = timed_steps(s, steps)
    rtype = "double" if precision == 0 else "float"
    names = kernel_names(rtype, cfg, False)
    workload = f"cavity32_recon{recon}" + ("_gp" if sampling == 2 else "") + ("_shakhov" if prandtl != 1.0 else "")
    dom, kr = kernel_roofline(kms, moves / steps, st1, rtype, names, workload)
    ms = el / steps * 1e3
    s.close()
    del s
    torch.cuda.empty_cache()
    leg = {"value": moves / el, "unit": "particle moves/s", "ms_per_step": ms, "cell_steps_per_s": nc * steps / el,
           "particles_per_step": int(moves / steps), "steps": steps, "timed_after_step": int(st1["step"]) - steps,
           "dominant": dom, "kernels": kr, "whole_step": whole_step(ms, moves / steps, nc, rtype, recon)}
    return leg


def cpu_baseline(sample):
    """The oracle as it stands on a sample of the batch: the first instances (in instance
    order), each from the state the GPU's FP64 plain run reached after its timed steps
    (imported into the oracle, with its instance index), one step each, timed.  Twice: the
    serial build on one core, then the OpenMP build (the same results bit for bit) on every
    thread OpenMP is given; the value is the OpenMP one."""
    import oracle

    def run(omp):
        moved, cells, el = 0, 0, 0.0
        for k, w, st in sample:
            o = oracle.Oracle(w.mesh, w.params, instance=k, omp=omp)
            o.set_state(w.W0)
            o.import_state(st)
            t0 = time.perf_counter()
            o.step()
            el += time.perf_counter() - t0
            so = o.stats()
            moved += so["n_alive"] + so["n_collided"] + so["n_escaped"]
            cells += w.mesh.n_cells
            del o
        return moved, cells, el

    m1, c1, e1 = run(False)
    nth = oracle.threads(0)
    mp, cp, ep = run(True)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    names = [k for k, _, _ in sample]
    step = int(np.asarray(sample[0][2]["step"]).reshape(-1)[0]) if sample else 0
    return {"value": mp / ep if ep > 0 else None, "unit": "particle moves/s", "cores": nth, "kind": "oracle",
            "build": "OpenMP (per-face, per-cell and per-particle loops parallel; sums in serial order)",
            "cpu_model": model, "cell_steps_per_s": cp / ep if ep > 0 else None,
            "single_core": {"value": m1 / e1 if e1 > 0 else None, "cores": 1, "seconds": round(e1, 2),
                            "cell_steps_per_s": c1 / e1 if e1 > 0 else None},
            "sample": f"instances {names} of the batch (FP64, first order, energy-exact sampling), one step each from "
                      f"the GPU run's state at step {step}: {mp} particle moves and {cp} cell-steps, {ep:.1f} s on "
                      f"{nth} threads, {e1:.1f} s on one"}


# algorithmic bytes of the first-order flux per face: both cells' W (2 x 40), the face's
# geometry (normal, area, owner and neighbour: 48) and its flux out (40)
BYTES_PER_FACE = 168
# in the FP32 form the face geometry is FP32 (normal 12, area 4, owner and neighbour 8): 144 B
BYTES_PER_FACE_FP32 = 144
GKS_CAPACITY = 65536


def gks_side(steps, warmup):
    """Side number: the GKS limit of the scheme, the cavity at Kn 1e-6, FP64 plain.  There
    exp(-dt/tau) underflows to 0, so no particle is ever sampled and a step is the wave part
    alone.  Cell-steps/s, and the flux kernel's position against HBM (its time from hip events
    over the warm-up steps)."""
    import torch

    from paper_2007_13091_amd import workloads as wl
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.morton_numbered(wl.cavity(kn=1e-6))
    # no particle is ever sampled: a small capacity keeps the particle kernels' grids, which
    # cover the capacity, from launching blocks that find nothing to do
    s = Solver(w.mesh, w.params, capacity=GKS_CAPACITY)
    s.init_state(w.W0)
    s.step(1, stats=False)
    s.profile(True)
    s.profile_read()
    s.step(max(warmup - 1, 1), stats=False)
    warm = s.profile_read()
    s.profile(False)
    st0 = s.step(0, stats=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.step(0, stats=True)
    s.close()
    del s
    torch.cuda.empty_cache()
    el = t1 - t0
    nc = w.mesh.n_cells
    faces = (6 * nc + int(w.mesh.bface_nodes.shape[0])) // 2  # box hexes: shared faces counted twice
    flux_ms = warm["flux"][0] / max(warm["flux"][1], 1)
    achieved = BYTES_PER_FACE * faces / (flux_ms * 1e-3) / 1e9
    return {"workload": "cavity 32^3 (Morton-numbered) at Kn 1e-6 (GKS limit: no particles), FP64 plain",
            "cell_steps_per_s": nc * steps / el, "ms_per_step": el / steps * 1e3, "steps": steps,
            "particles_per_step": int((st1["moved_total"] - st0["moved_total"]) / steps), "capacity": GKS_CAPACITY,
            "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in warm.items()},
            "flux_roofline": {"kernel": "k_flux<double, 128>", "kernel_avg_ms": round(flux_ms, 4),
                              "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_face": BYTES_PER_FACE,
                              "faces": faces}}


def configs_run(gks_steps=3000, only=None, recon=None):
    """The other configurations, timed (not part of the default run): the shock tube over its
    40 steps (FP64; launch-bound at 200 cells), and the Mach 10 cube (1.2e6 tets) and the
    Mach 15 vehicle at Kn 1e-3 (3.1e6 tets) in both forms, started wave-only for `gks_steps`
    steps (the paper's continuum start), timed over the wave-particle steps that follow, until
    the near-wake turns non-physical."""
    import torch

    from paper_2007_13091_amd import workloads as wl
    from paper_2007_13091_amd.ugkwp import Solver

    def one(w, precision, warm, steps):
        s = Solver(w.mesh, w.params, precision=precision)
        s.init_state(w.W0)
        st0 = s.step(warm, stats=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, stats=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st1 = s.step(0, stats=True)
        s.close()
        del s
        torch.cuda.empty_cache()
        el = t1 - t0
        moves = st1["moved_total"] - st0["moved_total"]
        return {"value": moves / el, "unit": "particle moves/s", "cell_steps_per_s": w.mesh.n_cells * steps / el,
                "ms_per_step": el / steps * 1e3, "particles_per_step": int(moves / steps), "steps": steps,
                "after_steps": warm}

    out = {}
    if only in (None, "sod"):
        w = wl.morton_numbered(wl.sod())
        out["sod_50x2x2_fp64"] = one(w, 0, 1, 39)
    for name, make in (("cube_mach10", lambda: wl.cube()), ("vehicle_mach15_kn1e-3", lambda: wl.vehicle(kn=1e-3))):
        if only not in (None, name.split("_")[0]):
            continue
        w = wl.morton_numbered(make())
        w.params.gks_steps = gks_steps
        w.params.sampling = 1
        if recon is not None:
            w.params.recon = recon
        for prec in (0, 1):
            out[f"{name}_{'fp64' if prec == 0 else 'fp32'}"] = one(w, prec, gks_steps + 1, 4)
    return out


# algorithmic bytes of the time averaging per cell: W and the running sum read, the sum
# written, the volume read (5 x 8 x 3 + 8)
BYTES_PER_AVG_CELL = 128


def averaging_side(steps, warmup):
    """Side number: the cost of time averaging (Sec. 2.4(c)) on the FP64 cavity: the same
    solver timed over `steps` steps without averaging and then over `steps` steps averaging
    every step, and the averaging kernels' position against HBM (k_avg_cells and k_avg_fin are
    timed with k_finalize in one group; the group's time without averaging is subtracted)."""
    import torch

    from paper_2007_13091_amd import workloads as wl
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.morton_numbered(wl.cavity())
    s = Solver(w.mesh, w.params)
    s.init_state(w.W0)
    s.step(warmup, stats=False)
    s.profile(True, slots=["finalize"])
    s.profile_read()
    s.step(warmup, stats=False)
    fin0 = s.profile_read()["finalize"]
    s.profile(False)

    def timed():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, stats=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    ms_plain = timed()
    s.set_averaging(0)
    s.profile(True, slots=["finalize"])
    s.profile_read()
    s.step(warmup, stats=False)
    fin1 = s.profile_read()["finalize"]
    s.profile(False)
    ms = timed()
    _, res, n = s.average()
    s.close()
    del s
    torch.cuda.empty_cache()
    nc = w.mesh.n_cells
    avg_ms = fin1[0] / max(fin1[1], 1) - fin0[0] / max(fin0[1], 1)
    achieved = BYTES_PER_AVG_CELL * nc / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    return {"workload": "cavity 32^3 (Morton-numbered), FP64 plain, every step averaged", "ms_per_step": ms,
            "ms_per_step_without": ms_plain, "steps_averaged": int(n[0]), "last_relative_change": float(res[0]),
            "averaging_kernels_ms": round(avg_ms, 4),
            "roofline": {"bound": "hbm", "achieved": None if achieved is None else round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
                         "bytes_per_cell": BYTES_PER_AVG_CELL, "cells": nc}}


BATCH_WORKLOAD = ("64 independent instances alternating shock tube (Nx x 2 x 2 box hexes) and lid-driven cavity (n^3), "
                  "cells log-uniform in [2e3, 2e5] (2.79e6 in all), Kn log-uniform in [1e-4, 1], 50-500 particles per "
                  "cell, CFL 0.5, each numbered along a Morton curve; FP32 form, all instances in one launch per kernel, "
                  "launch shapes autotuned; energy-exact sampling (the printed pairs turn 2 of the 64 instances "
                  "non-physical)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch-start", type=int, default=BATCH_START,
                    help="steps of the batch before its warm-up (the autotuner's trials are among them)")
    ap.add_argument("--cavity-start", type=int, default=CAVITY_START)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-moves", type=float, default=2e8,
                    help="particle moves per step of the batch instances the CPU baseline steps once each")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-cavity", action="store_true")
    ap.add_argument("--no-gks", action="store_true")
    ap.add_argument("--no-avg", action="store_true")
    ap.add_argument("--configs", action="store_true",
                    help="time the tube, the cube and the vehicle (their own JSON object; not the bench line)")
    ap.add_argument("--config", choices=["sod", "cube", "vehicle"], default=None,
                    help="with --configs: only this configuration (for profiling it alone)")
    ap.add_argument("--recon", type=int, choices=[0, 1, 2], default=None,
                    help="with --configs: the reconstruction of the cube and vehicle (default: first order)")
    ap.add_argument("--gks-steps", type=int, default=3000,
                    help="with --configs: wave-only steps before the timed UGKWP steps of the cube and vehicle")
    ap.add_argument("--gks-only", action="store_true",
                    help="run only the GKS-limit leg and print its JSON object (for profiling it alone)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched FP32 leg (no FP64 comparison) and print its JSON object")
    ap.add_argument("--cavity-only", type=int, default=-1, metavar="PRECISION",
                    help="run only the cavity leg in that precision (0 FP64, 1 FP32) and print its JSON object")
    ap.add_argument("--cavity-sampling", type=int, choices=[0, 1, 2, 3], default=0,
                    help="with --cavity-only: the hydro-particle sampling")
    ap.add_argument("--cavity-prandtl", type=float, default=1.0,
                    help="with --cavity-only: the Prandtl number (1 BGK, else the Shakhov model)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.configs:
        print(json.dumps({"configs": configs_run(args.gks_steps, args.config, args.recon)}), flush=True)
        return
    if args.gks_only:
        print(json.dumps({"gks_limit": gks_side(args.steps, args.warmup)}), flush=True)
        return
    if args.cavity_only >= 0:
        leg = cavity_leg(args.cavity_only, args.steps, args.warmup, args.cavity_start, sampling=args.cavity_sampling,
                         prandtl=args.cavity_prandtl)
        print(json.dumps({"cavity": leg}), flush=True)
        return
    if args.batched_only:
        import torch

        from paper_2007_13091_amd.ugkwp import Solver

        ws = batch_workloads(1)
        caps = batch_capacities(ws, args.batch_start + args.warmup + args.steps + 2)
        s = Solver([w.mesh for w in ws], [w.params for w in ws], capacity=caps, precision=1,
                   stream=torch.cuda.Stream())
        s.init_state(np.concatenate([w.W0 for w in ws]))
        s.step(max(args.batch_start - 26, 1), stats=False)
        cfg = s.autotune(steps_per_trial=1)
        s.step(args.warmup, stats=True)
        el, moves, kms, _, st1 = timed_steps(s, args.steps)
        print(json.dumps({"batched_only": {"value": moves / el, "ms_per_step": el / args.steps * 1e3,
                                           "kernel_ms": kms, "launch_config": list(cfg)}}), flush=True)
        return

    b, sample = batched_run(args.steps, args.warmup, args.batch_start, sampling=1,
                            cpu_sample_moves=0 if args.no_cpu_baseline else args.cpu_moves)
    plain = b["fp64_plain_one_by_one"]
    roof = dict(b["kernels"][b["dominant"]])
    roof["other_kernel"] = b["kernels"]["gather" if b["dominant"] == "stream" else "stream"]
    roof["whole_step"] = b["whole_step"]
    roof["flux_kernel"] = b["flux"]
    out = {
        "metric": "particle moves/s + cell-steps/s, FP32/batched vs FP64 plain at stated error",
        "value": b["value"],
        "unit": "particle moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "instances": b["instances"], "cells": b["cells"],
                   "particles_per_step": b["particles_per_step"], "timed_after_step": b["timed_after_step"],
                   "launch_config": b["launch_config"]},
        "cell_steps_per_s": b["cell_steps_per_s"],
        "fp64_plain_one_by_one": plain,
        "speedup_vs_fp64_plain": b["speedup_vs_fp64_plain_one_by_one"],
        "stated_error": b["stated_error"],
        "graph_replay_ms_per_step": b["graph_replay_ms_per_step"],
        "roofline": roof,
    }
    if not args.no_cavity:
        c64 = cavity_leg(0, args.steps, args.warmup, args.cavity_start)
        c32 = cavity_leg(1, args.steps, args.warmup, args.cavity_start)
        c32["speedup_vs_fp64_plain"] = c32["value"] / c64["value"]
        # the first-order g_p, with the BGK model and with the Shakhov model at Pr = 2/3
        gp = cavity_leg(0, args.steps, args.warmup, args.cavity_start, sampling=2)
        sh = cavity_leg(0, args.steps, args.warmup, args.cavity_start, sampling=2, prandtl=2.0 / 3.0)
        sh["ms_per_step_vs_bgk_gp"] = sh["ms_per_step"] / gp["ms_per_step"]
        out["cavity32"] = {"workload": "lid-driven cavity, 32^3 box hexes (Morton-numbered), 400 particles/cell, "
                                       "Kn 0.075, diffuse walls, lid 0.16 sqrt(gamma T_w), second order "
                                       "(Venkatakrishnan), the printed pairs of Sec. 2.4(b)",
                           "fp64_plain": c64, "fp32_form": c32,
                           "fp64_gp_bgk": gp, "fp64_gp_shakhov_pr_2_3": sh}
    if not args.no_gks:
        out["gks_limit"] = gks_side(args.steps, args.warmup)
    if not args.no_avg:
        out["time_averaging"] = averaging_side(args.steps, args.warmup)
    if sample:
        out["cpu_baseline"] = cpu_baseline(sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
