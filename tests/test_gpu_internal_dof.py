"""GPU parity with internal degrees of freedom (Sec. 2.1, Sec. 2.3): a diatomic gas (gamma = 7/5,
K = 2) and K = 4, against the oracle: the primitives, wave flux (first and second order),
sampled internal energies, their re-emission at diffuse walls and their inflow at far-field
faces, and the particle sums that carry them.  Counts identical, fields within 1e-12, every
particle's internal energy variable within 1e-12 of the thermal scale."""
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

from test_gpu_parity import run_pair

pytestmark = pytest.mark.gpu

DIATOMIC = 7.0 / 5.0


def _say(*a):
    print("[gpu-kdof]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("sampling", [0, 1])
def test_diatomic_shock_tube(sampling):
    w = wl.sod(nx=50, ny=2, nz=2, n_ref=100, kn=1e-3, gamma=DIATOMIC)
    run_pair(w, 20, every=5, name="sod-diatomic", sampling=sampling)


def test_diatomic_tets_diffuse_walls():
    w = wl.closed_box(n=(4, 3, 3), n_ref=80, kn=0.3, bc=wl.BC_DIFFUSE, tets=True, jitter=0.15, perturb=0.3,
                      gamma=DIATOMIC)
    s, _ = run_pair(w, 6, name="tets-diffuse-diatomic")
    assert s.step(0)["wall_hits"] > 0


def test_diatomic_far_field_inflow():
    w = wl.free_stream_box(n=(5, 4, 3), U=(0.9, -0.3, 0.2), n_ref=80, kn=0.1, perturb=0.3, gamma=DIATOMIC)
    s, _ = run_pair(w, 6, name="farfield-diatomic")
    assert s.step(0)["n_injected"] > 0


@pytest.mark.parametrize("recon", [1, 2])
def test_diatomic_second_order(recon):
    w = wl.sod(nx=30, ny=2, nz=2, n_ref=60, kn=1e-2, gamma=DIATOMIC)
    w.params.recon = recon
    run_pair(w, 10, every=5, name=f"sod-diatomic-recon{recon}")


def test_k4_closed_box_energy_exact():
    w = wl.closed_box(n=(4, 3, 2), n_ref=60, kn=0.1, perturb=0.3, gamma=9.0 / 7.0)
    run_pair(w, 6, name="box-k4", sampling=1)


def test_diatomic_fp32_form_conserves():
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.closed_box(n=(4, 3, 3), n_ref=80, kn=0.1, perturb=0.2, gamma=DIATOMIC)
    g = Solver(w.mesh, w.params, precision=1)
    g.init_state(w.W0)
    vol, _, _ = g.geometry()
    t0 = (w.W0 * vol[:, None]).sum(0)
    g.step(10)
    t = (g.moments(0) * vol[:, None]).sum(0)
    assert abs(t[0] - t0[0]) < 1e-12 * t0[0] and abs(t[4] - t0[4]) < 1e-12 * t0[4]
    assert g.particles()["e"].min() > 0


def test_mixed_gamma_batch_is_refused():
    from paper_2007_13091_amd.ugkwp import E_ARG, UgkwpError, workspace_bytes

    a = wl.sod(nx=10, ny=2, nz=2, n_ref=20)
    b = wl.sod(nx=10, ny=2, nz=2, n_ref=20, gamma=DIATOMIC)
    with pytest.raises(UgkwpError) as e:
        workspace_bytes([a.mesh, b.mesh], [a.params, b.params])
    assert e.value.status == E_ARG
