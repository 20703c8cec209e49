"""Launch shapes, graph replay and the autotuner change nothing in the results: every launch
shape of the tunable kernels gives bit-identical fields and particles; a step replayed from a
captured hip graph equals the eagerly launched step at every step (with eager work and
synchronisation between replays); an autotuned run equals a plain run of as many steps."""
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-launch]", *a, flush=True)
    sys.stdout.flush()


def _state(s):
    p = s.particles()
    o = np.argsort(p["uid"])
    return s.moments(0), {k: v[o] for k, v in p.items()}


def _same(a, b, what):
    np.testing.assert_array_equal(a[0], b[0], err_msg=f"{what}: W")
    for k in ("uid", "cell", "x", "u", "m", "e"):
        np.testing.assert_array_equal(a[1][k], b[1][k], err_msg=f"{what}: particles {k}")


SHAPES = [(128, 1, 1, 64), (512, 2, 8, 256), (256, 2, 2, 128), (256, 1, 4, 64), (512, 1, 1, 256), (128, 2, 8, 128)]


@pytest.mark.parametrize("gas", ["monatomic", "diatomic-gp"])
@pytest.mark.parametrize("precision", [0, 1])
def test_every_launch_shape_gives_identical_results(precision, gas):
    from paper_2007_13091_amd.ugkwp import Solver

    g = 5.0 / 3.0 if gas == "monatomic" else 7.0 / 5.0
    ws = [wl.cavity(n=8, n_ref=200), wl.free_stream_box(n=(4, 3, 3), n_ref=60, kn=0.2, perturb=0.2, tets=True,
                                                         jitter=0.15, gamma=g)]
    if gas != "monatomic":
        ws[0] = wl.closed_box(n=(6, 5, 4), n_ref=120, kn=0.1, bc=wl.BC_DIFFUSE, perturb=0.3, gamma=g)
        ws[0].params.recon, ws[0].params.sampling = 2, 2
    ref = None
    for shape in [None] + SHAPES:
        _say("precision", precision, "shape", shape)
        s = Solver([w.mesh for w in ws], [w.params for w in ws], precision=precision)
        s.init_state(np.concatenate([w.W0 for w in ws]))
        if shape is not None:
            assert s.launch_config(shape) == shape
        s.step(5)
        st = _state(s)
        if ref is None:
            ref = st
        else:
            _same(st, ref, f"shape {shape}")
        s.close()


def test_graph_replay_equals_eager_every_step():
    import torch
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.free_stream_box(n=(5, 4, 3), U=(0.9, -0.3, 0.2), n_ref=60, kn=0.05, perturb=0.3)
    stream = torch.cuda.Stream()
    a = Solver(w.mesh, w.params, stream=stream)
    b = Solver(w.mesh, w.params, stream=stream)
    a.init_state(w.W0)
    b.init_state(w.W0)
    b.graph(True)
    for k in range(7):
        a.step(1, stats=False)
        b.step(1, stats=False)
        torch.cuda.synchronize()
        # eager work between replays
        x = torch.ones(1000, device="cuda").cumsum(0)
        assert float(x[-1]) == 1000.0
        _same(_state(b), _state(a), f"graph replay step {k}")
        if k == 3:
            b.graph(False)
            b.step(1, stats=False)
            a.step(1, stats=False)
            b.graph(True)
    sa, sb = a.step(2), b.step(2)
    for key in ("n_alive", "n_sampled", "n_injected", "n_collided", "n_escaped", "crossings", "wall_hits", "step",
                "max_crossings_seen"):
        assert sa[key] == sb[key], key
    _same(_state(b), _state(a), "graph replay end")


@pytest.mark.parametrize("case", ["diatomic-gp-diffuse", "batch-mixed-modes", "batch-shakhov"])
def test_graph_replay_with_internal_energy_and_gp_sampling(case):
    # the internal-energy instantiations and the g_p sampling kernel, captured and replayed
    import torch
    from paper_2007_13091_amd.ugkwp import Solver

    if case == "diatomic-gp-diffuse":
        w = wl.closed_box(n=(4, 3, 3), n_ref=60, kn=0.2, bc=wl.BC_DIFFUSE, tets=True, jitter=0.15, perturb=0.3,
                          gamma=7.0 / 5.0)
        w.params.recon, w.params.sampling = 2, 2
        meshes, params, W0 = w.mesh, w.params, w.W0
    elif case == "batch-mixed-modes":
        ws = wl.small_batch(4)
        for k, x in enumerate(ws):
            x.params.recon = 1 if k % 2 == 0 else 0
            x.params.sampling = 2 if k % 2 == 0 else 1
        meshes, params, W0 = [x.mesh for x in ws], [x.params for x in ws], np.concatenate([x.W0 for x in ws])
    else:
        # the heat-flux kernel and the Shakhov terms (sampling 3 and 2), next to a BGK instance
        ws = wl.small_batch(4)
        for k, x in enumerate(ws):
            x.params.prandtl = 2.0 / 3.0 if k < 3 else 1.0
            x.params.sampling = (3, 2, 3, 0)[k]
            x.params.recon = 2 if k == 1 else 0
        meshes, params, W0 = [x.mesh for x in ws], [x.params for x in ws], np.concatenate([x.W0 for x in ws])
    stream = torch.cuda.Stream()
    a = Solver(meshes, params, stream=stream)
    b = Solver(meshes, params, stream=stream)
    a.init_state(W0)
    b.init_state(W0)
    b.graph(True)
    for k in range(5):
        a.step(1, stats=False)
        b.step(1, stats=False)
        torch.cuda.synchronize()
        x = torch.ones(1000, device="cuda").cumsum(0)
        assert float(x[-1]) == 1000.0
        _same(_state(b), _state(a), f"{case} graph replay step {k}")
    assert a.step(0)["n_alive"] > 0


def test_graph_needs_a_created_stream():
    from paper_2007_13091_amd.ugkwp import Solver, UgkwpError
    import torch

    w = wl.cavity(n=4, n_ref=50)
    s = Solver(w.mesh, w.params, stream=torch.cuda.default_stream())
    with pytest.raises(UgkwpError, match="stream"):
        s.graph(True)


def test_autotuned_run_equals_plain_run():
    from paper_2007_13091_amd.ugkwp import Solver

    ws = wl.small_batch(4)
    a = Solver([w.mesh for w in ws], [w.params for w in ws], precision=1)
    b = Solver([w.mesh for w in ws], [w.params for w in ws], precision=1)
    W0 = np.concatenate([w.W0 for w in ws])
    a.init_state(W0)
    b.init_state(W0)
    cfg = a.autotune(steps_per_trial=1)
    _say("autotuned", cfg)
    n = a.instance_stats(0)["step"]
    assert n == 2 * 13
    b.step(n)
    _same(_state(a), _state(b), "autotuned vs plain")
    assert a.launch_config() == cfg


def test_profile_events_change_nothing_and_mask_selects_slots():
    """Timing every kernel group, or one of them, leaves the results bit-identical to an
    untimed run; a mask times only the named group."""
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.cavity(n=8, n_ref=200)
    runs = []
    for slots in ("off", None, ["stream"]):
        _say("profile slots", slots)
        s = Solver(w.mesh, w.params)
        s.init_state(w.W0)
        if slots != "off":
            s.profile(True, slots=slots)
        s.step(4)
        if slots != "off":
            prof = s.profile_read()
            timed = {k for k, v in prof.items() if v[1] > 0}
            if slots is None:
                assert {"stream", "gather", "flux", "sample"} <= timed
                assert all(v[1] == 4 for k, v in prof.items() if k in ("stream", "gather"))
            else:
                assert timed == {"stream"} and prof["stream"][1] == 4 and prof["stream"][0] > 0
        runs.append(_state(s))
        s.close()
    _same(runs[1], runs[0], "all groups timed")
    _same(runs[2], runs[0], "stream timed")


def test_autotune_cache_hit_and_miss(tmp_path):
    # a miss tunes on real steps and appends a JSON line; the same workload then hits without a
    # step; another workload (the FP32 form) misses; unreadable lines are ignored
    import json

    from paper_2007_13091_amd.ugkwp import Solver

    ws = wl.small_batch(3)
    W0 = np.concatenate([w.W0 for w in ws])
    cache = tmp_path / "tune.jsonl"
    cache.write_text("not json\n")

    def solver(precision=0):
        s = Solver([w.mesh for w in ws], [w.params for w in ws], precision=precision)
        s.init_state(W0)
        return s

    a = solver()
    cfg, hit = a.autotune(1, cache=cache)
    assert not hit and a.instance_stats(0)["step"] == 2 * 13
    b = solver()
    cfg2, hit2 = b.autotune(1, cache=cache)
    assert hit2 and cfg2 == cfg and b.instance_stats(0)["step"] == 0
    assert tuple(b.launch_config()) == cfg
    c = solver(precision=1)
    _, hit3 = c.autotune(1, cache=cache)
    assert not hit3
    lines = cache.read_text().splitlines()
    assert len(lines) == 3
    rec = [json.loads(x) for x in lines[1:]]
    assert rec[0]["launch"] == list(cfg) and rec[0]["key"] != rec[1]["key"]
