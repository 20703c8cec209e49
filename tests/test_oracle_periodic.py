"""Oracle pins for periodic faces (test support: a tagged face leads to the face at x + shift;
not a boundary condition of the paper).

With every side of a box periodic no face is a wall, so the scheme must keep all five totals
(mass, the three momenta, energy) constant to rounding: a check that the wave flux is applied
with opposite signs to the two cells of each face, which a closed box (momentum not
conserved) cannot make.  Free transport through periodic faces has a closed form: a particle
ends at x0 + u t wrapped into the box, in the cell holding that point."""
import numpy as np
import pytest

import oracle
from paper_2007_13091_amd import workloads as wl


def _totals(o):
    vol, _, _ = o.geometry()
    W, _, _ = o.state()
    return (W * vol[:, None]).sum(0)


@pytest.mark.parametrize("tets", [False, True])
def test_periodic_box_conserves_all_five_totals(tets):
    w = wl.periodic_box(n=(4, 3, 3), n_ref=60, kn=0.05, tets=tets)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    # every face is interior: cells x faces per cell / 2
    per_cell = 4 if tets else 6
    assert o.nf == o.nc * per_cell // 2
    t0 = _totals(o)
    assert abs(t0[1]) > 0.1 and abs(t0[2]) > 0.05  # a drifting gas: the momenta are not zero
    for _ in range(30):
        o.step()
    t1 = _totals(o)
    st = o.stats()
    assert st["wall_hits"] == 0 and st["n_escaped"] == 0 and st["crossings"] > 0
    np.testing.assert_allclose(t1, t0, rtol=2e-14, atol=0)


def test_closed_specular_box_does_not_conserve_momentum():
    # the contrast that makes the periodic pin meaningful: walls take momentum
    w = wl.closed_box(n=(4, 3, 3), n_ref=60, kn=0.05)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    t0 = _totals(o)
    for _ in range(10):
        o.step()
    t1 = _totals(o)
    assert abs(t1[0] - t0[0]) <= 1e-13 * abs(t0[0]) and abs(t1[4] - t0[4]) <= 1e-13 * abs(t0[4])
    assert np.max(np.abs(t1[1:4] - t0[1:4])) > 1e-6


def _cell_of(w, p):
    """Index of the box hex holding point p (cells numbered x fastest)."""
    hi = (1.0, 0.75, 0.5)
    n = (4, 3, 3)
    ijk = [min(int(p[a] / (hi[a] / n[a])), n[a] - 1) for a in range(3)]
    return ijk[0] + n[0] * (ijk[1] + n[1] * ijk[2])


@pytest.mark.parametrize("u", [(3.7, 0.0, 0.0), (-2.3, 1.9, 0.0), (1.3, -2.9, 4.1)])
def test_free_flight_wraps_around_periodic_faces(u):
    w = wl.periodic_box(n=(4, 3, 3), n_ref=10)
    o = oracle.Oracle(w.mesh, w.params)
    hi = np.array([1.0, 0.75, 0.5])
    x0 = np.array([0.41, 0.33, 0.27])
    t = 0.9
    rc, x, uo, cell, ncross = o.track(x0, u, _cell_of(w, x0), t)
    assert rc == 0
    np.testing.assert_array_equal(uo, np.array(u))  # no wall: the velocity is untouched
    expect = np.mod(x0 + np.array(u) * t, hi)
    np.testing.assert_allclose(x, expect, rtol=0, atol=1e-12)
    assert cell == _cell_of(w, expect)
    # one crossing per cell boundary passed on each axis
    h = hi / np.array([4, 3, 3])
    passed = sum(abs(int(np.floor((x0[a] + u[a] * t) / h[a])) - int(np.floor(x0[a] / h[a]))) for a in range(3))
    assert ncross == passed


def test_unpaired_periodic_face_is_a_mesh_error():
    w = wl.periodic_box(n=(3, 2, 2))
    # the x-high side becomes a wall: the x-low periodic faces have no partner
    w.mesh.bcs = list(w.mesh.bcs) + [wl.BC(wl.BC_SPECULAR)]
    xhi = w.mesh.bface_bc == 1
    w.mesh.bface_bc = np.where(xhi, len(w.mesh.bcs) - 1, w.mesh.bface_bc).astype(np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(w.mesh, w.params)


def test_second_order_refused_with_periodic_faces():
    w = wl.periodic_box(n=(3, 2, 2))
    w.params.recon = 1
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(w.mesh, w.params)


def test_step_counts_total_and_most_crossings():
    # a free-molecular periodic box whose mass is all in imported particles (W = P / Omega, so no
    # hydro part and nothing sampled): in one step every particle flies u dt in a straight line,
    # and the step's crossing total and maximum are the per-particle counts of cell boundaries
    # passed on each axis
    w = wl.periodic_box(n=(4, 3, 3), n_ref=10, kn=1e6, perturb=0.0, drift=(0.0, 0.0, 0.0))
    o = oracle.Oracle(w.mesh, w.params)
    hi = np.array([1.0, 0.75, 0.5])
    h = hi / np.array([4, 3, 3])
    rng = np.random.default_rng(4)
    n = 400
    x = rng.uniform(0, 1, (n, 3)) * hi
    u = rng.normal(0, 3.0, (n, 3))
    cell = np.array([_cell_of(w, p) for p in x])
    order = np.argsort(cell, kind="stable")
    x, u, cell = x[order], u[order], cell[order]
    vol, _, _ = o.geometry()
    m = np.full(n, vol.sum() / n)
    P = np.zeros((o.nc, 5))
    np.add.at(P[:, 0], cell, m)
    for d in range(3):
        np.add.at(P[:, 1 + d], cell, m * u[:, d])
    np.add.at(P[:, 4], cell, 0.5 * m * (u * u).sum(1))
    uid = (np.uint64(1) << np.uint64(62)) + np.arange(n, dtype=np.uint64)
    o.import_state(dict(W=P / vol[:, None], P=P, particles=dict(x=x, u=u, m=m, cell=cell, uid=uid), step=0, t=0.0))
    o.step()
    st = o.stats()
    assert st["n_sampled"] == 0 and st["n_collided"] == 0 and st["n_alive"] == n
    dt = st["dt"]
    passed = np.abs(np.floor((x + u * dt) / h) - np.floor(x / h)).sum(1).astype(np.int64)
    assert passed.max() >= 2
    assert st["crossings"] == int(passed.sum())
    assert st["max_crossings_seen"] == int(passed.max())
