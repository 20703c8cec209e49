"""The OpenMP build of the oracle (used only to time the CPU baseline on many cores) gives
the same results as the serial build, bit for bit: its parallel loops write per-item
outputs and every sum keeps the serial order.  Checked over several steps on each mesh kind,
boundary condition, order of reconstruction, sampling mode and internal-DOF count."""
import numpy as np
import pytest

import oracle
from paper_2007_13091_amd import workloads as wl


def _cases():
    a = wl.closed_box(n=(4, 3, 3), n_ref=60, kn=0.2, bc=wl.BC_DIFFUSE, tets=True, jitter=0.15, perturb=0.3)
    b = wl.free_stream_box(n=(5, 4, 3), U=(1.2, -0.3, 0.2), n_ref=50, kn=0.05, perturb=0.3, tets=True, jitter=0.1)
    c = wl.sod(nx=24, ny=2, nz=2, n_ref=40)
    c.params.recon = 2
    d = wl.cavity(n=6, n_ref=50)
    d.params.sampling = 1
    e = wl.closed_box(n=(4, 4, 3), n_ref=40, kn=0.1, perturb=0.2, gamma=7.0 / 5.0)
    f = wl.free_stream_box(n=(4, 3, 3), U=(1.5, 0.2, 0.0), n_ref=40, kn=0.2)
    f.params.gks_steps = 2
    return {"tets-diffuse": a, "farfield-tets": b, "tube-recon2": c, "cavity-exact": d, "diatomic": e,
            "wave-only-start": f}


@pytest.mark.parametrize("name", list(_cases()))
def test_openmp_build_is_bitwise_the_serial_build(name):
    w = _cases()[name]
    assert oracle.threads(4) == 4
    a = oracle.Oracle(w.mesh, w.params)
    b = oracle.Oracle(w.mesh, w.params, omp=True)
    a.set_state(w.W0)
    b.set_state(w.W0)
    for n in range(5):
        a.step()
        b.step()
        assert a.stats() == b.stats(), (name, n)
        for x, y in zip(a.state(), b.state()):
            np.testing.assert_array_equal(x, y, err_msg=f"{name} step {n}")
        pa, pb = a.particles(), b.particles()
        for k in pa:
            np.testing.assert_array_equal(pa[k], pb[k], err_msg=f"{name} step {n} {k}")
    assert a.stats()["n_alive"] > 0


def test_serial_build_runs_one_thread():
    assert oracle.threads(0, omp=False) == 1
