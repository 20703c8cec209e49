"""Wave-only steps with no particle anywhere take a shorter launch sequence (no sampling,
transport, bucket or gather kernels: they would find nothing to do).  Its results must be those
of the full step bit for bit:

* an instance alone (the short sequence for its first gks_steps steps) against the same
  instance in a batch with an instance that has no wave-only phase (so every step of the batch
  takes the full sequence): W, the particles and the counts agree at every step, through the
  switch to wave-particle steps, in both forms and at second order;
* graph replay across the switch equals eager launches;
* a state exported in the wave-only phase (no particles) and imported continues bit for bit;
  one imported with particles takes the full sequence and agrees with the uninterrupted run.
"""
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-wave-only]", *a, flush=True)
    sys.stdout.flush()


def _case(name):
    if name == "sod":
        w = wl.sod(nx=30, ny=2, nz=2, n_ref=80, kn=1e-2)
        w.params.gks_steps = 5
    elif name == "cavity-recon2":
        w = wl.cavity(n=8, n_ref=100, kn=0.02)
        w.params.recon = 2
        w.params.gks_steps = 4
    else:
        w = wl.free_stream_box(n=(4, 3, 3), U=(2.5, 0.4, -0.3), T=1.2, n_ref=60, kn=0.1, perturb=0.2, tets=True,
                               jitter=0.15, walls={"zlo": wl.BC(wl.BC_DIFFUSE, Tw=1.0)})
        w.params.gks_steps = 4
    return w


def _particles(s, lo, hi):
    p = s.particles()
    sel = (p["cell"] >= lo) & (p["cell"] < hi)
    o = np.argsort(p["uid"][sel])
    return {k: v[sel][o] for k, v in p.items()}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["sod", "cavity-recon2", "farfield-tets"])
def test_short_sequence_equals_full_step(name, precision):
    from paper_2007_13091_amd.ugkwp import Solver

    a = _case(name)
    b = wl.cavity(n=4, n_ref=40, kn=0.05)  # no wave-only phase: the batch takes full steps
    alone = Solver(a.mesh, a.params, precision=precision)
    batch = Solver([a.mesh, b.mesh], [a.params, b.params], precision=precision)
    alone.init_state(a.W0)
    batch.init_state(np.concatenate([a.W0, b.W0]))
    nc = a.mesh.n_cells
    for n in range(a.params.gks_steps + 3):
        _say(name, precision, "step", n)
        sa = alone.step(1)
        batch.step(1)
        sb = batch.instance_stats(0)
        for k in ("n_alive", "n_sampled", "n_collided", "n_escaped", "n_injected", "step"):
            assert sa[k] == sb[k], (name, n, k, sa[k], sb[k])
        assert sa["dt"] == sb["dt"] and sa["t"] == sb["t"]
        np.testing.assert_array_equal(alone.moments(0), batch.moments(0)[:nc], err_msg=f"{name} step {n}")
        pa, pb = _particles(alone, 0, nc), _particles(batch, 0, nc)
        for k in ("uid", "cell", "x", "u", "m"):
            np.testing.assert_array_equal(pa[k], pb[k], err_msg=f"{name} step {n} {k}")
        if n < a.params.gks_steps:
            assert sa["n_alive"] == 0 and sa["n_sampled"] == 0
    assert alone.step(0)["n_alive"] > 0


def test_graph_replay_across_the_switch():
    import torch
    from paper_2007_13091_amd.ugkwp import Solver

    w = _case("farfield-tets")
    stream = torch.cuda.Stream()
    a = Solver(w.mesh, w.params, stream=stream)
    b = Solver(w.mesh, w.params, stream=stream)
    a.init_state(w.W0)
    b.init_state(w.W0)
    b.graph(True)
    for n in range(w.params.gks_steps + 3):
        a.step(1, stats=False)
        b.step(1, stats=False)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.moments(0), b.moments(0), err_msg=f"graph step {n}")
    pa, pb = _particles(a, 0, w.mesh.n_cells), _particles(b, 0, w.mesh.n_cells)
    for k in ("uid", "x", "u", "m"):
        np.testing.assert_array_equal(pa[k], pb[k])
    assert a.step(0)["n_alive"] > 0


def test_import_in_the_wave_only_phase():
    from paper_2007_13091_amd.ugkwp import Solver

    w = _case("sod")
    ref = Solver(w.mesh, w.params)
    ref.init_state(w.W0)
    ref.step(2)
    st = ref.export_state()
    assert st["particles"]["uid"].size == 0
    c = Solver(w.mesh, w.params)
    c.init_state(w.W0)
    c.import_state(st)
    for n in range(w.params.gks_steps + 2):
        sr, sc = ref.step(1), c.step(1)
        assert sr["n_alive"] == sc["n_alive"] and sr["n_sampled"] == sc["n_sampled"]
        np.testing.assert_array_equal(ref.moments(0), c.moments(0), err_msg=f"imported, step {n}")
    # a state with particles, imported while the wave-only phase still runs: its particles must
    # still stream and collide (full steps), as in the oracle
    import oracle
    from parity import compare_fields, compare_stats

    ref.step(4)
    st2 = ref.export_state()
    assert st2["particles"]["uid"].size > 0
    w2 = _case("sod")
    w2.params.gks_steps = 1000
    st2["step"] = np.array([7])
    d = Solver(w2.mesh, w2.params)
    d.init_state(w2.W0)
    d.import_state(st2)
    o = oracle.Oracle(w2.mesh, w2.params)
    o.set_state(w2.W0)
    o.import_state(st2)
    vol, _, _ = o.geometry()
    for n in range(3):
        sd = d.step(1)
        o.step()
        compare_stats(sd, o.stats(), what=f"imported with particles, step {n}")
        assert sd["n_sampled"] == 0 and sd["n_collided"] > 0
        Wo, Po, _ = o.state()
        compare_fields(d.moments(0), Wo, d.moments(1) * vol[:, None], Po, vol, what=f"imported with particles {n}")
