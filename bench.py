"""Benchmark of the UGKWP hot path on one MI355X.

Workload: the lid-driven cubic cavity (paper Sec. 4.2) at the hot-path size: unit cube of
32^3 box hexes, diffuse isothermal walls at T_w = 1, lid z = 1 moving at 0.16 sqrt(gamma T_w),
Kn 0.075 (VHS, omega = 0.81), 400 particles per cell (about 1.3e7 particles), CFL 0.95,
synthetic initial state (gas at rest).  A step is one full time step of the scheme: wave
flux, sampling, free-flight times, free transport, particle sums and the cell update.

Prints ONE JSON line: particle moves/s (value) and cell-steps/s, the dominant kernel's
roofline position (timed live with hip events on the library's stream), and the CPU
oracle's rate on a bounded sample of the same workload.
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
BYTES_PER_MOVE_FP64 = 136
BYTES_PER_MOVE_FP32 = 80
# algorithmic bytes of the gather (S6): a survivor's record read and written with its cell,
# plus its bucket key read (FP64: 64 + 64 + 4 + 4 = 136 B; FP32: 36 + 40 + 4 = 80 B); a
# collided particle's velocity and mass read with its key (FP64: 48 + 4 = 52 B; FP32: 36 + 4)
BYTES_PER_SURVIVOR = {"double": 136, "float": 80}
BYTES_PER_COLLIDED = {"double": 52, "float": 40}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


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


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter runs, if the kernel
    source has not changed since they were taken (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("source_digest") != kernel_source_digest():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(steps=12):
    """The oracle as it stands, single-threaded, on the same workload from the same initial
    state: the first `steps` steps (the first samples every particle, the rest are typical)."""
    import oracle
    from paper_2007_13091_amd import workloads as wl

    w = wl.morton_numbered(wl.cavity())
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    moved = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step()
        st = o.stats()
        moved += st["n_alive"] + st["n_collided"] + st["n_escaped"]
    el = time.perf_counter() - t0
    return {"value": moved / el, "unit": "particle moves/s", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} steps of the 32^3 cavity (Morton-numbered, 400 particles/cell) from the initial state, "
                      f"{moved} particle moves in {el:.1f} s; cell-steps/s {steps * w.mesh.n_cells / el:.3g}"}


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)


def timed_run(w, precision, warmup, steps):
    """W untimed steps (every kernel group timed with hip events, to find the dominant one),
    then K timed steps bracketed by device synchronisation, with hip events on the library's
    stream around the dominant kernel only (events around every group cost about 5% of a
    step).  Returns the per-group times of the warm-up and the dominant group's time over the
    timed steps."""
    import torch

    from paper_2007_13091_amd.ugkwp import Solver

    s = Solver(w.mesh, w.params, precision=precision)
    s.init_state(w.W0)
    cfg = s.launch_config()
    s.step(1, stats=False)
    s.profile(True)
    s.profile_read()  # clear
    st0 = s.step(max(warmup - 1, 1), stats=True)
    warm = s.profile_read()
    # the heavier of the two kernels that carry the step's particle traffic (the others are
    # a few percent of a step; under a counter-collecting profiler their launch overheads
    # can look larger in a short warm-up)
    dom = max(("stream", "gather"), key=lambda k: warm[k][0])
    s.profile(True, slots=[dom])
    moved0 = st0["moved_total"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.step(0, stats=True)
    prof = s.profile_read()
    s.profile(False)
    s.close()
    del s
    torch.cuda.empty_cache()
    kern = {k: v for k, v in warm.items()}
    kern[dom] = prof[dom]
    return t1 - t0, st1["moved_total"] - moved0, kern, cfg, dom, st1


# algorithmic bytes of the first-order flux per face: both cells' W (2 x 40), the face's
# geometry (normal, area, owner and neighbour: 48) and its flux out (40)
BYTES_PER_FACE = 168


GKS_CAPACITY = 65536


def gks_side(steps, warmup):
    """Side number: the GKS limit of the scheme, the cavity at Kn 1e-6, FP64 plain.  There
    exp(-dt/tau) underflows to 0, so no particle is ever sampled and a step is the wave part
    alone (at Kn 1e-4 the sampling rule, N_sam = 2 ceil(N_ref rho^hp / (2 (rho^p + rho^hp))),
    still draws N_ref particles of tiny mass per cell once the previous ones have collided).
    Cell-steps/s, and the flux kernel's position against HBM (its time from hip events over
    the warm-up steps)."""
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


def configs_run():
    """The other configurations, timed (not part of the default run): the shock tube over
    its 40 steps (FP64; launch-bound at 200 cells), and the Mach 10 cube (1.2e6 tets) and the
    Mach 15 vehicle at Kn 1e-3 (3.1e6 tets) in both forms over the steps after the first
    (sampling from an empty start) and before their wakes empty (the impulsive start)."""
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
    w = wl.morton_numbered(wl.sod())
    out["sod_50x2x2_fp64"] = one(w, 0, 1, 39)
    w = wl.morton_numbered(wl.cube())
    out["cube_mach10_fp64"] = one(w, 0, 1, 3)
    out["cube_mach10_fp32"] = one(w, 1, 1, 3)
    w = wl.morton_numbered(wl.vehicle(kn=1e-3))
    out["vehicle_mach15_kn1e-3_fp64"] = one(w, 0, 1, 2)
    out["vehicle_mach15_kn1e-3_fp32"] = one(w, 1, 1, 2)
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


def stated_fp32_error():
    """The FP32 form's error against the FP64 oracle, as measured by tests/test_gpu_fp32.py
    and committed under profiles/ (L1 and Linf of rho, |U|, T, with the seed-to-seed noise)."""
    f = os.path.join(ROOT, "profiles", "fp32_error_cavity16.json")
    try:
        with open(f) as fh:
            rows = json.load(fh)
        last = rows[-1]
        return {"workload": "cavity 16^3, 400 particles/cell", "step": last["step"],
                "fp32_vs_fp64_oracle": last["fp32_vs_oracle"], "fp64_seed_noise": last["noise_floor"]}
    except (OSError, ValueError, KeyError, IndexError):
        return None


def batched_run(steps, warmup, plain_steps):
    """The batched form on 64 independent tube and cavity instances (log-uniform cell counts in
    [2e3, 2e5], Kn in [1e-4, 1], 50 to 500 particles per cell; each instance's cells numbered
    along a Morton curve): FP32 transport, all instances in
    one launch per kernel, launch shapes autotuned on real steps, steps replayed from a
    captured hip graph.  Against it: the FP64 plain form run instance by instance (each alone,
    eager launches), timed over `plain_steps` steps after the same number of warm-up steps."""
    import torch

    from paper_2007_13091_amd import workloads as wl
    from paper_2007_13091_amd.ugkwp import Solver

    ws = [wl.morton_numbered(w) for w in wl.batched()]
    meshes, params = [w.mesh for w in ws], [w.params for w in ws]
    W0 = np.concatenate([w.W0 for w in ws])
    nc = int(sum(w.mesh.n_cells for w in ws))
    # capacity: N_sam = 2 ceil(r) adds at least two particles per cell and step wherever the
    # hydro wave has a collisionless part, and rarefied cells lose only their collided share,
    # so counts drift up by up to two per cell and step on top of about N_ref
    total_steps = warmup + 13 * 2 + 1 + steps
    caps = [int(1.3 * w.params.n_ref * w.mesh.n_cells + 2.2 * total_steps * w.mesh.n_cells) + 65536 for w in ws]
    stream = torch.cuda.Stream()
    s = Solver(meshes, params, capacity=caps, precision=1, stream=stream)
    s.init_state(W0)
    s.step(max(warmup, 1), stats=False)
    cfg = s.autotune(steps_per_trial=1)
    s.graph(True)
    st0 = s.step(1, stats=True)
    s.profile(True)
    s.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.step(0, stats=True)
    done_steps = st1["step"]
    s.close()
    del s
    torch.cuda.empty_cache()
    el = t1 - t0
    moves = st1["moved_total"] - st0["moved_total"]
    out = {"value": moves / el, "unit": "particle moves/s", "dtype": "f32 transport, f64 sums",
           "ms_per_step": el / steps * 1e3, "cell_steps_per_s": nc * steps / el, "steps": steps,
           "warmup_and_tuning_steps": int(done_steps - steps),
           "instances": len(ws), "cells": nc, "particles_per_step": int(moves / steps),
           "launch_config": {"stream_bs": cfg[0], "stream_ilp": cfg[1], "sample_wpb": cfg[2], "flux_bs": cfg[3]},
           "graph_replay": True}
    # FP64 plain, one instance after the other, each on the current stream with eager launches
    pm, pt, pc = 0, 0.0, 0
    for w, cap in zip(ws, caps):
        g = Solver(w.mesh, w.params, capacity=cap, precision=0)
        g.init_state(w.W0)
        a = g.step(int(done_steps - steps), stats=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        g.step(plain_steps, stats=False)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        b = g.step(0, stats=True)
        pm += b["moved_total"] - a["moved_total"]
        pt += tb - ta
        pc += w.mesh.n_cells * plain_steps
        g.close()
        del g
    torch.cuda.empty_cache()
    out["fp64_plain_one_by_one"] = {"value": pm / pt, "unit": "particle moves/s", "cell_steps_per_s": pc / pt,
                                    "steps": plain_steps}
    out["speedup_vs_fp64_plain_one_by_one"] = out["value"] / (pm / pt)
    return out


def roofline(prof, dom, moves_per_launch, last, rtype, cfg):
    """Roofline position of the dominant kernel group dom (transport or gather): its
    algorithmic bytes per launch over its average duration.  Transport: the particle moves
    of a step; gather: the survivors and collided particles of a step (last: statistics of
    the last timed step).  cfg: the solver's launch shapes (they name the kernel instance)."""
    dom_ms, dom_n = prof[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    if dom == "stream":
        algo = (BYTES_PER_MOVE_FP64 if rtype == "double" else BYTES_PER_MOVE_FP32) * moves_per_launch
        kname = f"k_stream<{rtype}, {cfg[0]}, false, {cfg[1]}>"
    elif dom == "gather":
        algo = BYTES_PER_SURVIVOR[rtype] * last["n_alive"] + BYTES_PER_COLLIDED[rtype] * last["n_collided"]
        kname = f"k_gather<{rtype}, 1>"  # one wave (cell) per block
    else:
        raise RuntimeError(f"no algorithmic byte count for kernel group {dom}")
    achieved = algo / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kname),
            "kernel": kname, "kernel_avg_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(algo)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-gks", action="store_true")
    ap.add_argument("--no-avg", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=40)
    ap.add_argument("--batched-warmup", type=int, default=8)
    ap.add_argument("--configs", action="store_true",
                    help="time the tube, the cube and the vehicle (their own JSON object; not the bench line)")
    ap.add_argument("--gks-only", action="store_true",
                    help="run only the GKS-limit leg and print its JSON object (for profiling it alone)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched leg and print its JSON object (for profiling it alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.configs:
        print(json.dumps({"configs": configs_run()}), flush=True)
        return
    if args.gks_only:
        print(json.dumps({"gks_limit": gks_side(args.steps, args.warmup)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_form": batched_run(args.batched_steps, args.batched_warmup, args.batched_steps)}),
              flush=True)
        return

    from paper_2007_13091_amd import workloads as wl

    w = wl.morton_numbered(wl.cavity())
    nc = w.mesh.n_cells
    el, moves, prof, cfg, dom, last = timed_run(w, 0, args.warmup, args.steps)
    value = moves / el
    moves_per_launch = moves / args.steps
    roof = roofline(prof, dom, moves_per_launch, last, "double", cfg)
    out = {
        "metric": "particle moves/s + cell-steps/s, FP32/batched vs FP64 plain at stated error",
        "value": value,
        "unit": "particle moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lid-driven cavity, 32^3 box hexes numbered along a Morton curve, 400 particles/cell, "
                               "Kn 0.075, diffuse walls, lid 0.16 sqrt(gamma T_w); FP64 plain form",
                   "cells": nc, "faces": int(w.mesh.n_cells * 3 + 3 * 32 * 32), "particles_per_step": int(moves_per_launch)},
        "cell_steps_per_s": nc * args.steps / el,
        "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_fp32:
        el32, moves32, prof32, cfg32, dom32, last32 = timed_run(w, 1, args.warmup, args.steps)
        out["fp32_form"] = {"value": moves32 / el32, "unit": "particle moves/s", "dtype": "f32 transport, f64 sums",
                            "ms_per_step": el32 / args.steps * 1e3, "cell_steps_per_s": nc * args.steps / el32,
                            "speedup_vs_fp64_plain": (moves32 / el32) / value,
                            "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof32.items()},
                            "roofline": roofline(prof32, dom32, moves32 / args.steps, last32, "float", cfg32),
                            "stated_error": stated_fp32_error()}
    if not args.no_batched:
        out["batched_form"] = batched_run(args.batched_steps, args.batched_warmup, args.batched_steps)
    if not args.no_gks:
        out["gks_limit"] = gks_side(args.steps, args.warmup)
    if not args.no_avg:
        out["time_averaging"] = averaging_side(args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
