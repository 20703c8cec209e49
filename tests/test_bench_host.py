"""CPU checks of bench.py's host logic: the source digest that ties the committed traffic
counters to the kernels ignores comments and layout but not code, unknown kernels report no
traffic, and a multi-GPU request is refused with a message (this build measures one GPU)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_digest_ignores_comments_and_layout_but_not_code():
    b = _bench()
    src = {f: open(os.path.join(ROOT, "paper_2007_13091_amd", "csrc", f)).read()
           for f in ("kernels.hip", "device_common.hpp")}
    base = b.kernel_source_digest(lambda f: src[f])
    assert base == b.kernel_source_digest()
    commented = dict(src)
    commented["kernels.hip"] = "// a new comment\n/* and a block\n   comment */\n" + src["kernels.hip"].replace(
        "\n", "\n    \n", 3)
    assert b.kernel_source_digest(lambda f: commented[f]) == base
    changed = dict(src)
    changed["device_common.hpp"] = src["device_common.hpp"].replace("kWallSeg = 64", "kWallSeg = 32")
    assert changed["device_common.hpp"] != src["device_common.hpp"]
    assert b.kernel_source_digest(lambda f: changed[f]) != base


def test_unknown_kernel_has_no_measured_traffic():
    assert _bench().measured_traffic("k_no_such_kernel<double>", "batch64") is None
    assert _bench().measured_traffic("k_gather<float, 1, false>", "no_such_workload") is None


def test_roofline_and_error_helpers():
    b = _bench()
    # 1e6 moves in FP32 at 80 B each over 0.02 ms: 4000 GB/s, half of the peak
    dom, kr = b.kernel_roofline({"stream": 0.02, "gather": 0.01}, 1e6, {"n_alive": 9e5, "n_collided": 1e5}, "float",
                                {"stream": "k_stream<float, 256, true, 1>", "gather": "k_gather<float, 1, false>"}, "none")
    assert dom == "stream" and abs(kr["stream"]["frac"] - 0.5) < 1e-12
    assert kr["gather"]["algorithmic_bytes_per_launch"] == 80 * 900000 + 40 * 100000
    ws = b.whole_step(1.0, 1e7, 32768, "double")
    assert ws["algorithmic_bytes_per_step"] == 136 * 10 ** 7 + 312 * 32768
    import numpy as np
    W = np.tile([1.0, 0.1, 0.0, 0.0, 1.6], (4, 1))
    e = b.field_error(W, W)
    assert all(e[v]["L1"] == 0 and e[v]["Linf"] == 0 for v in ("rho", "U", "T"))


def test_kernel_names_match_the_instantiations():
    b = _bench()
    n = b.kernel_names("float", (256, 1), True)
    assert n == {"stream": "k_stream<float, 256, true, 1>", "gather": "k_gather<float, 1, false>"}
    src = open(os.path.join(ROOT, "paper_2007_13091_amd", "csrc", "kernels.hip")).read()
    assert "k_gather<float, WPB, false>" in src and "k_stream<R, " in src


def test_batch_capacity_covers_the_drift_and_fits_an_index():
    from paper_2007_13091_amd import workloads as wl

    b = _bench()
    specs = wl.batched_specs()
    total = 0
    for k in (0, 6, 19, 63):
        w = wl.batched_instance(specs[k])
        e_lo, e_hi = b.collisionless_fraction(w)
        assert 0.0 <= e_lo <= e_hi <= 1.0
        cap = b.batch_capacity(w, 127)
        # the old particles (N_ref plus a drift of up to two per cell and step, or their settled
        # count) and a new sample of N_ref (1 - e) within the step
        settled = w.params.n_ref + 2.0 / max(1.0 - e_hi, 1e-9)
        old = min(w.params.n_ref + 2 * 127, settled)
        assert cap >= (old + w.params.n_ref * (1.0 - e_lo) + 2) * w.mesh.n_cells
        total += cap
    # a continuum-limit cavity settles: its capacity does not grow with the steps, and it holds
    # two full samples
    w = wl.cavity(n=8, n_ref=100, kn=1e-7)
    assert b.collisionless_fraction(w)[1] < 1e-3
    assert b.batch_capacity(w, 1000) == b.batch_capacity(w, 100)
    assert b.batch_capacity(w, 100) >= 2 * 100 * w.mesh.n_cells
    assert sum(b.batch_capacity(wl.batched_instance(sp), 127) for sp in specs) < 2 ** 31 - 1024


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
