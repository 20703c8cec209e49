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
    assert _bench().measured_traffic("k_no_such_kernel<double>") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
