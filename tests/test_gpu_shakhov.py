"""GPU parity of the Shakhov collision model (prandtl != 1) against the oracle.

Both sides compute each cell's heat flux from its particles at the start of the step (sums in
different orders, FP64), add q1 (1 - Pr) q_f.n to the energy flux of the wave part at every
interior and far-field face, and draw the hydro particles from g^+ by acceptance-rejection with
the same Philox draws, every acceptance taken in FP64: counts identical, fields and particles
within 1e-12.  Cases:
* a periodic box whose mass starts in particles with a heat flux (imported on both sides):
  parity, and the GPU's heat flux relaxing like the scheme's recursion for a homogeneous gas;
* the second-order cavity with g_p plus the correction (sampling 2), diffuse walls;
* tetrahedra with far-field faces (sampling 3);
* a batch mixing Shakhov and BGK instances;
* the FP32 form (conservation, and its distance from FP64).
"""
import math
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

from parity import compare_fields, compare_particles, compare_stats
from test_gpu_batch import _run_batch
from test_gpu_parity import run_pair
from test_oracle_shakhov import _boxes, _particles_with_heat_flux, _sums

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-shakhov]", *a, flush=True)
    sys.stdout.flush()


def _hot_periodic(pr, nper, seed=12, dt_over_tau=0.2):
    import oracle

    w = wl.periodic_box(n=(2, 2, 2), n_ref=nper, kn=0.05, cfl=0.5, seed=seed, perturb=0.0, drift=(0, 0, 0))
    o0 = oracle.Oracle(w.mesh, w.params)
    vol, _, dS = o0.geometry()
    w.params.mu_ref = w.params.cfl * (vol / (3.0 * dS).sum(1)).min() / dt_over_tau
    w.params.sampling = 3
    w.params.prandtl = pr
    lo, ext = _boxes(w.mesh)
    p = _particles_with_heat_flux(np.random.default_rng(seed), vol, lo, ext, range(len(vol)), nper, 1.0)
    P = _sums(p, len(vol))
    st = dict(W=P / vol[:, None], P=P, particles=p, step=0, t=0.0)
    return w, st, vol


@pytest.mark.parametrize("pr", [2.0 / 3.0, 1.0])
def test_shakhov_homogeneous_relaxation(pr):
    import oracle
    from paper_2007_13091_amd.ugkwp import Solver

    w, st, vol = _hot_periodic(pr, 4000)
    g = Solver(w.mesh, w.params)
    g.init_state(st["W"])
    g.import_state(st)
    o = oracle.Oracle(w.mesh, w.params)
    o.import_state(st)
    name = f"homogeneous Pr={pr:.3f}"
    Q = [o.heat_flux()[:, 0].mean()]
    for n in range(6):
        _say(name, "step", n)
        sg = g.step(1)
        o.step()
        compare_stats(sg, o.stats(), what=f"{name} step {n}")
        Wo, Po, _ = o.state()
        compare_fields(g.moments(0), Wo, g.moments(1) * vol[:, None], Po, vol, what=f"{name} step {n}")
        pg = g.particles()
        compare_particles(pg, o.particles(), vscale=3.0, what=f"{name} step {n}")
        # the heat flux of the GPU's particles, summed here
        Wg = g.moments(0)
        cv = pg["u"] - (Wg[:, 1:4] / Wg[:, :1])[pg["cell"]]
        h = 0.5 * pg["m"] * (cv * cv).sum(1)
        Q.append((np.bincount(pg["cell"], weights=h * cv[:, 0], minlength=len(vol)) / vol).mean())
    e = math.exp(-0.2)
    pred = [Q[0]]
    for k in range(6):
        pred.append(pred[-1] * (e if k == 0 else e * (1 + (1 - e) * (1 - pr))))
    np.testing.assert_allclose(Q, pred, rtol=0.12)


def _shakhov(w, sampling=3, recon=None, pr=2.0 / 3.0):
    w.params.prandtl = pr
    w.params.sampling = sampling
    if recon is not None:
        w.params.recon = recon
    return w


def test_shakhov_cavity_second_order_gp():
    w = _shakhov(wl.cavity(n=8, n_ref=100), sampling=2, recon=2)
    s, o = run_pair(w, 10, every=5, name="cavity8-shakhov-gp")
    assert np.abs(o.heat_flux()).max() > 0


def test_shakhov_tets_far_field():
    w = _shakhov(wl.free_stream_box(n=(5, 4, 3), U=(0.9, -0.3, 0.2), n_ref=80, kn=0.05, perturb=0.3, tets=True,
                                    jitter=0.1), pr=0.72)
    s, o = run_pair(w, 6, name="farfield-shakhov")
    assert s.step(0)["n_escaped"] > 0


def test_shakhov_tube_first_order():
    w = _shakhov(wl.sod(nx=40, ny=2, nz=2, n_ref=80, kn=1e-2))
    run_pair(w, 12, every=4, name="sod-shakhov")


def test_shakhov_in_a_mixed_batch():
    ws = wl.small_batch(6)
    for k, w in enumerate(ws):
        if k % 2 == 0:
            _shakhov(w, sampling=3 if k % 4 == 0 else 2, recon=None if k % 4 == 0 else 2, pr=0.6 + 0.05 * k)
    _run_batch(ws, 5, name="mixed-shakhov-batch")


def test_shakhov_fp32_form():
    from paper_2007_13091_amd.ugkwp import Solver

    w = _shakhov(wl.periodic_box(n=(4, 3, 3), n_ref=80, kn=0.2, perturb=0.3))
    out = []
    for prec in (0, 1):
        g = Solver(w.mesh, w.params, precision=prec)
        g.init_state(w.W0)
        vol, _, _ = g.geometry()
        t0 = (w.W0 * vol[:, None]).sum(0)
        g.step(8)
        W = g.moments(0)
        t = (W * vol[:, None]).sum(0)
        np.testing.assert_allclose(t, t0, rtol=1e-12, atol=1e-12)
        out.append(W)
    # the FP32 form stays near FP64 in density (different draws decide only where it rounds)
    assert np.abs(out[1][:, 0] / out[0][:, 0] - 1).max() < 0.05


def test_shakhov_cavity_full_size():
    """The bench's Shakhov leg at its size: 32^3 cavity (Morton-numbered), 400 particles per
    cell, second order, g_p plus the correction, Pr = 2/3; the first step has no particles
    (q = 0), the next two draw from g^+ and add the flux term."""
    w = _shakhov(wl.morton_numbered(wl.cavity()), sampling=2, recon=2)
    s, o = run_pair(w, 3, every=1, name="cavity32-shakhov-gp")
    assert np.abs(o.heat_flux()).max() > 0
