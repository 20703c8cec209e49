"""State export and import through the C ABI (checkpoint and restart between steps).

* Resume: a run exported after k steps and imported into a fresh context continues bit for
  bit like the run that was never interrupted (both forms; a batch of instances; the Shakhov
  model, whose heat fluxes a pass of their own recomputes after the import in the order the
  gather sums them).
* Import of a state the oracle reached (particles in the oracle's order, grouped by cell for
  the library), then GPU-vs-oracle parity over the next steps: the imported particles are
  the old particles of the next step, with their free-flight draws keyed by their ids.
* Refusals: unsorted cells, more particles than the capacity, a non-physical W, a step
  beyond the particle-id field; a refused import leaves the state untouched.
"""
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

from parity import compare_fields, compare_particles, compare_stats

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-state]", *a, flush=True)
    sys.stdout.flush()


def _solver(w, precision=0, capacity=0):
    from paper_2007_13091_amd.ugkwp import Solver

    ws = w if isinstance(w, list) else [w]
    s = Solver([x.mesh for x in ws], [x.params for x in ws], precision=precision, capacity=capacity)
    s.init_state(np.concatenate([x.W0 for x in ws]))
    return s


def _same(a, b, what):
    sa, sb = a.export_state(), b.export_state()
    np.testing.assert_array_equal(sa["W"], sb["W"], err_msg=what)
    np.testing.assert_array_equal(sa["P"], sb["P"], err_msg=what)
    np.testing.assert_array_equal(sa["step"], sb["step"], err_msg=what)
    np.testing.assert_array_equal(sa["t"], sb["t"], err_msg=what)
    for k in ("x", "u", "m", "cell", "uid"):
        np.testing.assert_array_equal(sa["particles"][k], sb["particles"][k], err_msg=f"{what} {k}")


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", ["tets-diffuse", "farfield", "batch", "shakhov"])
def test_resume_is_bitwise(case, precision):
    if case == "tets-diffuse":
        w = wl.closed_box(n=(4, 3, 3), n_ref=60, kn=0.3, bc=wl.BC_DIFFUSE, tets=True, jitter=0.15, perturb=0.2)
    elif case == "shakhov":
        # the heat fluxes the gather leaves for the next step, recomputed after the import by a
        # pass of their own summed in the same order
        w = wl.cavity(n=6, n_ref=80)
        w.params.recon, w.params.sampling, w.params.prandtl = 2, 2, 2.0 / 3.0
    elif case == "farfield":
        w = wl.free_stream_box(n=(5, 4, 3), U=(0.9, -0.3, 0.2), n_ref=80, kn=0.05, perturb=0.3)
    else:
        w = wl.small_batch(5)
    _say("resume", case, precision)
    a = _solver(w, precision)
    a.step(6)
    st = a.export_state()
    assert st["particles"]["uid"].size > 0
    b = _solver(w, precision)
    b.step(2)  # a different state, replaced by the import
    b.import_state(st)
    _same(a, b, f"{case} after import")
    for n in range(4):
        sa, sb = a.step(1), b.step(1)
        for k in ("n_alive", "n_sampled", "n_collided", "n_escaped", "n_injected", "crossings", "wall_hits",
                  "max_crossings_seen"):
            assert sa[k] == sb[k], (case, n, k)
        _same(a, b, f"{case} step {n} after import")


@pytest.mark.parametrize("sampling", [0, 1])
def test_import_oracle_state_then_parity(sampling):
    import oracle

    w = wl.closed_box(n=(4, 3, 3), n_ref=60, kn=0.2, bc=wl.BC_DIFFUSE, tets=True, jitter=0.15, perturb=0.3)
    w.params.sampling = sampling
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    o.step(5)
    st = o.export_state()
    p = st["particles"]
    order = np.argsort(p["cell"], kind="stable")
    gst = dict(W=st["W"], P=st["P"], step=st["step"], t=st["t"],
               particles={k: v[order] for k, v in p.items()})
    g = _solver(w)
    g.import_state(gst)
    vol, _, _ = o.geometry()
    for n in range(4):
        sg = g.step(1)
        o.step()
        compare_stats(sg, o.stats(), what=f"imported step {n}")
        Wo, Po, _ = o.state()
        compare_fields(g.moments(0), Wo, g.moments(1) * vol[:, None], Po, vol, what=f"imported step {n}")
        compare_particles(g.particles(), o.particles(), vscale=3.0, what=f"imported step {n}")
        assert sg["step"] == o.step_index and abs(sg["t"] - o.time) <= 1e-12 * o.time


def test_import_refusals_leave_the_state():
    from paper_2007_13091_amd.ugkwp import E_ARG, E_CAPACITY, E_NONPHYS, UgkwpError

    w = wl.closed_box(n=(3, 3, 2), n_ref=40, kn=0.1, perturb=0.2)
    a = _solver(w, capacity=5000)
    b = _solver(w, capacity=5000)
    a.step(3)
    b.step(3)
    good = a.export_state()
    n = good["particles"]["uid"].size
    assert 0 < n < 5000

    def bad(**kw):
        st = {k: (dict(v) if k == "particles" else v) for k, v in good.items()}
        for k, v in kw.items():
            if k in good["particles"]:
                st["particles"][k] = v
            else:
                st[k] = v
        return st

    cells = good["particles"]["cell"].copy()
    cells[[0, -1]] = cells[[-1, 0]]
    with pytest.raises(UgkwpError) as e:
        a.import_state(bad(cell=cells))
    assert e.value.status == E_ARG
    reps = 5000 // n + 1  # more particles than the capacity of 5000
    big = {k: np.concatenate([v] * reps) for k, v in good["particles"].items()}
    big["cell"] = np.sort(big["cell"])
    st = dict(good)
    st["particles"] = big
    with pytest.raises(UgkwpError) as e:
        a.import_state(st)
    assert e.value.status == E_CAPACITY
    W = good["W"].copy()
    W[2, 4] = 0.0
    with pytest.raises(UgkwpError) as e:
        a.import_state(bad(W=W))
    assert e.value.status == E_NONPHYS
    with pytest.raises(UgkwpError) as e:
        a.import_state(bad(step=np.array([1 << 19])))
    assert e.value.status == E_ARG
    # the refused imports changed nothing: a and b still step alike
    a.step(2)
    b.step(2)
    _same(a, b, "after refused imports")
