"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the same seeded inputs.

Bar: particle ids, cells, counts and every collided/escaped/sampled decision identical;
fields within 1e-12 relative (see tests/parity.py).  Cases span several tiles of every
kernel plus ragged tails, the edge cases of the method (no particles at all, N_min raising
the sample count, diffuse walls, a moving lid, tetrahedra with jittered nodes,
free-molecular flow), the capacity and crossing limits, and the cavity at its full size in
the launch configuration the benchmark times.
"""
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

from parity import compare_fields, compare_particles, compare_stats

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


def _solver(w, capacity=0):
    from paper_2007_13091_amd.ugkwp import Solver

    s = Solver(w.mesh, w.params, capacity=capacity)
    s.init_state(w.W0)
    return s


def _oracle(w):
    import oracle

    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    return o


def run_pair(w, steps, every=1, capacity=0, length=1.0, vscale=3.0, name="", sampling=None, min_steps=None):
    """GPU and oracle side by side for `steps` steps.  min_steps: the run may end earlier with a
    non-physical state (E_NONPHYS), provided both sides report it at the same step and at
    least min_steps steps were compared before it."""
    if sampling is not None:
        w.params.sampling = sampling
        name = f"{name} sampling={sampling}"
    s = _solver(w, capacity)
    o = _oracle(w)
    vol, _, _ = o.geometry()
    vg, _, dSg = s.geometry()
    _, _, dSo = o.geometry()
    np.testing.assert_allclose(vg, vol, rtol=1e-14)
    np.testing.assert_allclose(dSg, dSo, rtol=1e-14, atol=1e-300)
    for n in range(steps):
        _say(name, "step", n)
        if min_steps is None:
            sg = s.step(1)
            o.step()
        else:
            import oracle
            from paper_2007_13091_amd.ugkwp import E_NONPHYS, UgkwpError

            try:
                sg = s.step(1)
            except UgkwpError as e:
                assert e.status == E_NONPHYS, f"{name}: {e}"
                with pytest.raises(oracle.OracleError) as eo:
                    o.step()
                assert eo.value.status == oracle.E_NONPHYS, f"{name}: oracle did not fail at step {n}"
                assert n >= min_steps, f"{name}: non-physical after only {n} steps"
                _say(name, "both sides non-physical at step", n)
                return s, o
            o.step()
        compare_stats(sg, o.stats(), what=f"{name} step {n}")
        if (n + 1) % every == 0 or n == steps - 1:
            Wo, Po, _ = o.state()
            compare_fields(s.moments(0), Wo, s.moments(1) * vol[:, None], Po, vol, what=f"{name} step {n}")
            compare_particles(s.particles(), o.particles(), length=length, vscale=vscale, what=f"{name} step {n}")
    return s, o


@pytest.mark.parametrize("sampling", [0, 1])
def test_sod_40_steps(sampling):
    w = wl.sod()  # 50x2x2 boxes, 200 particles/cell, Kn 1e-3, specular walls
    run_pair(w, 40, every=1, name="sod", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
@pytest.mark.parametrize("tets", [False, True])
def test_single_cell_and_one_column_meshes(tets, sampling):
    # degenerate sizes: one box cell (or the six tetrahedra of one box), and a one-cell-wide
    # column with diffuse walls, where every particle leaves its cell only through walls or
    # along the column
    w = wl.closed_box(n=(1, 1, 1), n_ref=64, kn=0.05, tets=tets)
    run_pair(w, 5, name="single box" if not tets else "one box of tets", sampling=sampling)
    w = wl.closed_box(n=(1, 1, 7), n_ref=30, kn=0.5, bc=wl.BC_DIFFUSE, tets=tets)
    run_pair(w, 5, name="column", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
def test_sod_tets_jittered_box(sampling):
    w = wl.closed_box(n=(4, 3, 3), n_ref=60, kn=0.02, tets=True, jitter=0.15)
    run_pair(w, 8, name="tet-box", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
def test_cavity_small_diffuse_lid(sampling):
    w = wl.cavity(n=8, n_ref=400)
    run_pair(w, 10, every=2, name="cavity8", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
def test_diffuse_box_rarefied_many_bounces(sampling):
    w = wl.closed_box(n=(3, 2, 2), n_ref=300, kn=2.0, bc=wl.BC_DIFFUSE, perturb=0.3)
    run_pair(w, 6, name="diffuse-kn2", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
@pytest.mark.parametrize("tets", [False, True])
def test_periodic_box(tets, sampling):
    """Periodic faces (test support): every face interior, particles re-entering through
    the partner face at x + shift."""
    w = wl.periodic_box(n=(5, 4, 3), n_ref=80, kn=0.05, tets=tets)
    s, _ = run_pair(w, 8, every=2, name="periodic" + ("-tets" if tets else ""), sampling=sampling)
    assert s.step(0)["wall_hits"] == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_periodic_box_conserves_all_five_totals(precision):
    from paper_2007_13091_amd.ugkwp import Solver

    w = wl.periodic_box(n=(6, 5, 4), n_ref=100, kn=0.02)
    s = Solver(w.mesh, w.params, precision=precision)
    s.init_state(w.W0)
    vol, _, _ = s.geometry()
    t0 = (s.moments(0) * vol[:, None]).sum(0)
    st = s.step(20)
    assert st["crossings"] > 0 and st["n_escaped"] == 0
    t1 = (s.moments(0) * vol[:, None]).sum(0)
    _say("periodic totals", precision, t0, t1)
    np.testing.assert_allclose(t1, t0, rtol=5e-14, atol=0)


@pytest.mark.parametrize("sampling", [0, 1])
def test_free_molecular_sod(sampling):
    w = wl.sod(nx=20, ny=2, nz=2, n_ref=100)
    w.params.mu_ref = 1e30
    run_pair(w, 10, name="sod-free-molecular", sampling=sampling)


def test_continuum_limit_no_particles():
    w = wl.sod(nx=50, ny=2, nz=2, n_ref=100)
    w.params.mu_ref = 1e-14  # exp(-dt/tau) underflows: no particle is ever sampled
    s, o = run_pair(w, 12, every=4, name="sod-gks-only")
    assert s.particle_count() == 0


@pytest.mark.parametrize("sampling", [0, 1])
def test_n_min_raises_sample_count(sampling):
    w = wl.closed_box(n=(3, 3, 2), n_ref=20, kn=0.01, perturb=0.2)
    w.params.n_min = 64
    run_pair(w, 5, name="n_min", sampling=sampling)


def test_numerical_dissipation_c2():
    w = wl.sod(nx=30, ny=2, nz=2, n_ref=50, kn=1e-4)
    w.params.c2 = 10.0
    run_pair(w, 10, every=5, name="sod-c2")


@pytest.mark.parametrize("sampling", [0, 1])
def test_farfield_box_transitional(sampling):
    # far field on all six sides, non-uniform inside: wave flux against W_inf, particles
    # leaving are removed and free-stream particles enter
    w = wl.free_stream_box(n=(5, 4, 3), U=(0.9, -0.3, 0.2), n_ref=120, kn=0.05, perturb=0.3)
    run_pair(w, 8, name="farfield-hex", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
def test_farfield_box_tets_jittered(sampling):
    w = wl.free_stream_box(n=(4, 3, 3), U=(0.5, 0.4, -0.3), T=1.2, n_ref=80, kn=0.2, perturb=0.2, tets=True,
                           jitter=0.15)
    run_pair(w, 6, name="farfield-tet", sampling=sampling)


def test_farfield_free_molecular_inflow_only():
    # collisionless: everything that enters is a particle; the hydro part comes only from
    # the free stream
    w = wl.free_stream_box(n=(4, 3, 2), U=(0.6, 0.0, 0.0), n_ref=150, kn=1e6)
    run_pair(w, 6, name="farfield-free-molecular")


@pytest.mark.parametrize("sampling", [0, 1])
def test_supersonic_inflow_with_diffuse_walls(sampling):
    # Mach 3 stream along x over a diffuse cold wall (z = 0), specular side planes
    U = 3.0 * np.sqrt(5.0 / 3.0)
    w = wl.free_stream_box(n=(6, 2, 4), U=(U, 0.0, 0.0), n_ref=60, kn=0.1, perturb=0.1,
                           walls={"zlo": wl.BC(wl.BC_DIFFUSE, Tw=1.0), "ylo": wl.BC(wl.BC_SPECULAR),
                                  "yhi": wl.BC(wl.BC_SPECULAR)})
    run_pair(w, 8, name="supersonic-wall", sampling=sampling)


@pytest.mark.parametrize("sampling", [0, 1])
def test_cube_small_mach10(sampling):
    # the Mach 10 cube case (far-field outer box, diffuse cube, jittered tets, N_min = N_ref,
    # C2 = 10) on a coarse mesh, over the steps before the wake behind the cube empties
    w = wl.small_cube(n_ref=50)
    run_pair(w, 5, name="cube-small", length=4.0, vscale=15.0, sampling=sampling, min_steps=3)


@pytest.mark.timeout(600)
def test_cube_full_size_first_steps():
    # the full 1.2e6-tetrahedron cube with 6e7 particles, in the launch configuration of the
    # timed runs: every field, count and particle against the oracle over the first two steps
    w = wl.cube()
    _say("cube full size", w.mesh.n_cells, "cells")
    run_pair(w, 2, name="cube-full", length=12.0, vscale=15.0)


@pytest.mark.parametrize("sampling", [0, 1])
@pytest.mark.parametrize("kn", [1e-3, 1.0])
def test_vehicle_small_mach15(kn, sampling):
    # the Mach 15 sphere-cone (staircase body, diffuse wall at 0.2 T_0, far field) on a coarse
    # mesh at both ends of its Knudsen range, over the steps before its wake empties
    w = wl.small_vehicle(kn=kn)
    run_pair(w, 5, name=f"vehicle-small-kn{kn}", length=4.0, vscale=25.0, sampling=sampling, min_steps=3)


@pytest.mark.timeout(900)
def test_vehicle_full_size_first_step():
    # 3.1e6 tetrahedra and 1.6e8 particles: every field, count and particle after one step
    w = wl.vehicle()
    _say("vehicle full size", w.mesh.n_cells, "cells")
    run_pair(w, 1, name="vehicle-full", length=8.0, vscale=25.0)


@pytest.mark.parametrize("sampling", [0, 1])
@pytest.mark.parametrize("recon", [1, 2])
def test_second_order_sod(recon, sampling):
    # second order: least-squares gradients with Barth-Jespersen (1) or Venkatakrishnan (2)
    w = wl.sod(n_ref=100)
    w.params.recon = recon
    run_pair(w, 20, every=5, name=f"sod-recon{recon}", sampling=sampling)


@pytest.mark.parametrize("recon", [1, 2])
def test_second_order_farfield_tets(recon):
    w = wl.free_stream_box(n=(4, 3, 3), U=(0.5, 0.4, -0.3), T=1.2, n_ref=60, kn=0.05, perturb=0.2, tets=True,
                           jitter=0.15)
    w.params.recon = recon
    run_pair(w, 6, name=f"farfield-tet-recon{recon}")


@pytest.mark.parametrize("sampling", [0, 1])
def test_second_order_cavity_diffuse_walls(sampling):
    w = wl.cavity(n=8, n_ref=200, kn=0.01)
    w.params.recon = 2
    run_pair(w, 8, every=2, name="cavity-recon2", sampling=sampling)


def test_second_order_specular_tets_near_continuum():
    w = wl.closed_box(n=(4, 3, 3), n_ref=40, kn=1e-3, perturb=0.3, tets=True, jitter=0.15)
    w.params.recon = 1
    w.params.c2 = 1.0
    run_pair(w, 8, name="tet-box-recon1")


def test_deterministic_rerun_bitwise():
    w = wl.cavity(n=6, n_ref=300)
    a = _solver(w)
    b = _solver(w)
    a.step(5)
    b.step(5)
    np.testing.assert_array_equal(a.moments(0), b.moments(0))
    pa, pb = a.particles(), b.particles()
    np.testing.assert_array_equal(pa["uid"], pb["uid"])
    np.testing.assert_array_equal(pa["x"], pb["x"])


def test_capacity_error_is_reported_and_poisons():
    from paper_2007_13091_amd.ugkwp import E_CAPACITY, E_STATE, UgkwpError

    w = wl.closed_box(n=(3, 3, 2), n_ref=100)
    s = _solver(w, capacity=500)
    with pytest.raises(UgkwpError) as e:
        s.step(1)
    assert e.value.status == E_CAPACITY
    with pytest.raises(UgkwpError) as e:
        s.step(1)
    assert e.value.status == E_STATE
    s.init_state(w.W0)  # clears the poison; a smaller workload now fits
    assert s.particle_count() == 0


def test_crossing_limit_is_reported():
    from paper_2007_13091_amd.ugkwp import E_LOST, UgkwpError

    w = wl.closed_box(n=(4, 4, 4), n_ref=50, kn=1.0)
    w.params.max_crossings = 1
    w.params.cfl = 1.0
    s = _solver(w)
    with pytest.raises(UgkwpError) as e:
        for _ in range(3):
            s.step(1)
    assert e.value.status == E_LOST


def test_crossing_limit_after_diffuse_reemission_is_reported():
    """A particle whose first crossing is a diffuse wall stops there and is finished by the
    wall kernel; in a 2 x 2 x 2 rarefied box many re-emitted particles cross again within
    the step, exceeding a limit of one crossing in that kernel."""
    from paper_2007_13091_amd.ugkwp import E_LOST, UgkwpError

    w = wl.closed_box(n=(2, 2, 2), n_ref=200, kn=2.0, bc=wl.BC_DIFFUSE, perturb=0.2)
    w.params.max_crossings = 1
    w.params.cfl = 1.0
    s = _solver(w)
    with pytest.raises(UgkwpError) as e:
        for _ in range(3):
            s.step(1)
    assert e.value.status == E_LOST


def test_nonphysical_initial_state_rejected():
    from paper_2007_13091_amd.ugkwp import E_NONPHYS, Solver, UgkwpError

    w = wl.closed_box(n=(2, 2, 2))
    s = Solver(w.mesh, w.params)
    W = w.W0.copy()
    W[3, 0] = -1.0
    with pytest.raises(UgkwpError) as e:
        s.init_state(W)
    assert e.value.status == E_NONPHYS


@pytest.mark.parametrize("morton,sampling", [(True, 0), (False, 0), (True, 1)])
def test_cavity_full_size(morton, sampling, steps=2):
    """32^3 cavity, 400 particles/cell (~1.3e7 particles): the benchmark's configuration (cells
    numbered along a Morton curve), and the same cavity numbered x fastest."""
    w = wl.morton_numbered(wl.cavity()) if morton else wl.cavity()
    run_pair(w, steps, every=1, name="cavity32 morton" if morton else "cavity32", sampling=sampling)


@pytest.mark.parametrize("case", ["sod", "cavity-recon2", "farfield-tets"])
def test_wave_only_start_then_switch(case):
    """The wave-only start (no particles for the first gks_steps steps, the waves carry the
    whole hydro transport) and the switch to wave-particle steps, against the oracle."""
    if case == "sod":
        w = wl.sod(nx=30, ny=2, nz=2, n_ref=80, kn=1e-2)
        w.params.gks_steps = 4
    elif case == "cavity-recon2":
        w = wl.cavity(n=8, n_ref=120, kn=0.02)
        w.params.recon = 2
        w.params.gks_steps = 3
    else:
        w = wl.free_stream_box(n=(4, 3, 3), U=(2.5, 0.4, -0.3), T=1.2, n_ref=60, kn=0.1, perturb=0.2, tets=True,
                               jitter=0.15, walls={"zlo": wl.BC(wl.BC_DIFFUSE, Tw=1.0)})
        w.params.gks_steps = 3
    s, o = run_pair(w, w.params.gks_steps + 4, name=f"wave-only-{case}")
    assert s.step(0)["n_alive"] > 0
