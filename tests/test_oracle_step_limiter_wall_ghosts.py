"""Pins of four parts of the oracle that whole-step invariants do not fix.

* The time step of Sec. 2.4(a), the relaxation time tau = mu_ref T^omega / p and the
  collisionless fraction exp(-dt/tau) at the start of the shock tube, against a worked
  example computed by hand (tests/golden/sod_step0.json).  Dropping the 1/2 in Delta S, or
  using the sound speed sqrt(gamma T) for 3 sqrt(T), moves dt by a factor 2 or 1.7.
* The Venkatakrishnan limiter: with eps -> 0 it reduces to phi(y) = (y^2 + 2y)/(y^2 + y + 2)
  of y = M / D (the algebraic form of the limiter in one ratio); with K = 1 it follows the
  full formula with eps^2 = (K h)^3; Barth-Jespersen gives min(1, y).  Both on a 3-cell row
  where M and D are known in closed form.
* The diffuse wall's re-emission law (Sec. 2.4(e)): the normal speed of a re-emitted particle
  follows the flux-weighted half-Maxwellian, i.e. a Rayleigh law of scale sqrt(T_w), and the
  tangential components are N(U_w, T_w) (KS tests on many single-particle reflections); a
  closed diffuse box at rest at T = T_w stays at T_w within its noise.
* The ghost states of the least-squares gradients at boundary faces: a field symmetric about
  a specular wall has zero normal gradient there; a uniform state gives zero gradients in the
  boundary cells for every wall type; a shear profile that meets a moving diffuse wall at the
  wall's velocity is reconstructed exactly in the cell next to the wall (the ghost continues
  the line, 2 U_w - U).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2007_13091_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sod_step0.json")


def _prim(W):
    rho = W[:, 0]
    U = W[:, 1:4] / rho[:, None]
    T = (2 / 3) * (W[:, 4] - 0.5 * rho * (U * U).sum(1)) / rho
    return rho, U, T


# ----------------------------------------------------------------------------------------
# time step, relaxation time and collisionless fraction (worked example)
# ----------------------------------------------------------------------------------------
def test_sod_step0_dt_tau_and_collisionless_fraction():
    with open(GOLD) as fh:
        g = json.load(fh)
    w = wl.sod()
    assert abs(w.params.cfl - g["cfl"]) == 0
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    dt = o.sample_only()
    tol = g["rel_tol"]
    assert abs(dt / g["dt"] - 1) < tol, dt
    vol, xc, _ = o.geometry()
    np.testing.assert_allclose(vol, g["cell_edge"] ** 3, rtol=1e-12)
    p = o.particles()
    rho = w.W0[:, 0]
    # the sample of a cell with no particles holds exactly exp(-dt/tau) rho Omega
    e = np.bincount(p["cell"], weights=p["m"], minlength=o.nc) / (rho * vol)
    left, right = xc[:, 0] < 0.5, xc[:, 0] > 0.5
    for sel, ek, tk in ((left, "exp_left", "tau_left"), (right, "exp_right", "tau_right")):
        assert np.all(np.abs(e[sel] / g[ek] - 1) < tol), (ek, e[sel].min(), e[sel].max())
        tau = -dt / np.log(e[sel])
        assert np.all(np.abs(tau / g[tk] - 1) < tol), (tk, tau.min(), tau.max())


# ----------------------------------------------------------------------------------------
# Venkatakrishnan and Barth-Jespersen limiters on a row of three box cells
# ----------------------------------------------------------------------------------------
def _row_gradient(a, b, recon, K):
    """Three unit boxes along x, specular walls; rho = 1 - a, 1, 1 + b, at rest, T = 1.  The
    middle cell's unlimited x-gradient of rho is (a + b)/2 (its y and z ghosts are mirror
    images with the same density); returns its limited value."""
    bcs = [wl.BC(wl.BC_SPECULAR)]
    mesh = wl.box_hex_mesh((3, 1, 1), (0.0, 0.0, 0.0), (3.0, 1.0, 1.0), {s: 0 for s in wl.SIDES}, bcs)
    rho = np.array([1.0 - a, 1.0, 1.0 + b])
    W0 = wl.conservative(rho, np.zeros((3, 3)), np.ones(3))
    prm = wl.Params(mu_ref=0.1, n_ref=10, recon=recon, venkat_k=K)
    o = oracle.Oracle(mesh, prm)
    o.set_state(W0)
    gW, gH, Wh = o.gradients()
    return gW[1, 0, :], (a + b) / 2.0


def _venkat_ratio(y):
    return (y * y + 2 * y) / (y * y + y + 2)


@pytest.mark.parametrize("a,b", [(0.3, 0.05), (0.05, 0.3), (0.2, 0.2), (0.01, 0.4), (0.45, 0.12)])
def test_venkatakrishnan_small_eps_is_the_ratio_form(a, b):
    g, g0 = _row_gradient(a, b, recon=2, K=1e-9)
    # faces +x and -x: D = +-(a + b)/4, M = b and -a; y = M / D
    phi = min(_venkat_ratio(4 * b / (a + b)), _venkat_ratio(4 * a / (a + b)))
    assert abs(g[0] / g0 - phi) < 1e-12, (g[0] / g0, phi)
    assert g[1] == 0.0 and g[2] == 0.0


@pytest.mark.parametrize("a,b", [(0.3, 0.05), (0.05, 0.3), (0.45, 0.12)])
def test_venkatakrishnan_with_eps_from_cell_size(a, b):
    # K = 1, h = Omega^(1/3) = 1: eps^2 = 1, comparable to M^2 and D^2 here
    K = 1.0
    g, g0 = _row_gradient(a, b, recon=2, K=K)
    eps2 = (K * 1.0) ** 3

    def venkat(M, D):
        return ((M * M + eps2) * D + 2 * D * D * M) / (D * (M * M + 2 * D * D + M * D + eps2))

    D = (a + b) / 4
    phi = min(venkat(b, D), venkat(-a, -D))
    assert abs(g[0] / g0 - phi) < 1e-12, (g[0] / g0, phi)
    # a larger K (larger eps) limits less: phi grows towards 1
    g2, _ = _row_gradient(a, b, recon=2, K=3.0)
    assert g2[0] / g0 > g[0] / g0
    assert abs(g2[0] / g0 - 1) < abs(g[0] / g0 - 1)


@pytest.mark.parametrize("a,b", [(0.3, 0.05), (0.05, 0.3), (0.2, 0.2)])
def test_barth_jespersen_is_min_one_ratio(a, b):
    g, g0 = _row_gradient(a, b, recon=1, K=1.0)
    phi = min(1.0, 4 * b / (a + b), 4 * a / (a + b))
    assert abs(g[0] / g0 - phi) < 1e-12


# ----------------------------------------------------------------------------------------
# diffuse re-emission law
# ----------------------------------------------------------------------------------------
def test_diffuse_reemission_law():
    Tw, Uw = 2.3, (0.0, 0.4, -0.2)
    bcs = [wl.BC(wl.BC_DIFFUSE, Tw=Tw, Uw=Uw), wl.BC(wl.BC_SPECULAR)]
    side = {s: 1 for s in wl.SIDES}
    side["xlo"] = 0
    mesh = wl.box_hex_mesh((1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), side, bcs)
    prm = wl.Params(mu_ref=0.1, n_ref=10)
    o = oracle.Oracle(mesh, prm)
    o.set_state(wl.conservative(np.ones(1), np.zeros((1, 3)), np.ones(1)))
    n = 20000
    u = np.zeros((n, 3))
    for i in range(n):
        # hits the wall x = 0 after 1e-6, re-emitted, flies 1e-6 more (no other face reached)
        rc, x, ui, cell, ncross = o.track([1e-6, 0.5, 0.5], [-1.0, 0.0, 0.0], 0, 2e-6, uid=1000 + i, step=3)
        assert rc == 0 and ncross == 1 and cell == 0
        u[i] = ui
    s = math.sqrt(Tw)
    # normal component, into the gas (+x): Rayleigh with scale sqrt(T_w)
    assert np.all(u[:, 0] > 0)
    assert stats.kstest(u[:, 0], stats.rayleigh(scale=s).cdf).pvalue > 1e-4
    # not the half-normal, nor the Rayleigh of the wrong scale
    assert stats.kstest(u[:, 0], stats.halfnorm(scale=s).cdf).pvalue < 1e-10
    assert stats.kstest(u[:, 0], stats.rayleigh(scale=s / math.sqrt(2)).cdf).pvalue < 1e-10
    # tangential components: N(U_w, T_w)
    assert stats.kstest(u[:, 1], stats.norm(loc=Uw[1], scale=s).cdf).pvalue > 1e-4
    assert stats.kstest(u[:, 2], stats.norm(loc=Uw[2], scale=s).cdf).pvalue > 1e-4
    assert abs(np.corrcoef(u[:, 1], u[:, 2])[0, 1]) < 4 / math.sqrt(n)


@pytest.mark.parametrize("sampling", [0, 1])
def test_diffuse_box_at_wall_temperature_stays_there(sampling):
    # a rarefied gas at rest at T = T_w in a closed diffuse box: an equilibrium; over 20 steps
    # the box-mean temperature stays within 4 sigma of T_w (sigma from the cells' spread)
    w = wl.closed_box(n=(4, 4, 3), n_ref=200, kn=0.5, bc=wl.BC_DIFFUSE, perturb=0.0)
    w.params.sampling = sampling
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    for _ in range(20):
        o.step()
    assert o.stats()["wall_hits"] > 0
    W, _, _ = o.state()
    vol, _, _ = o.geometry()
    _, U, T = _prim(W)
    sig = T.std() / math.sqrt(T.size)
    assert abs(np.average(T, weights=vol) - 1.0) < 4 * sig + 1e-12, (T.mean(), sig)
    assert np.abs(U).max() < 10 * T.std() + 0.05


# ----------------------------------------------------------------------------------------
# ghost states of the gradients at boundary faces
# ----------------------------------------------------------------------------------------
def test_specular_ghost_mirror_symmetric_field_has_zero_normal_gradient():
    # two unit boxes along x between specular walls, the second the mirror image of the first
    # about x = 1: the first cell's neighbour and its ghost at the wall x = 0 hold the same
    # state, so its x-gradient vanishes for every component
    bcs = [wl.BC(wl.BC_SPECULAR)]
    mesh = wl.box_hex_mesh((2, 1, 1), (0.0, 0.0, 0.0), (2.0, 1.0, 1.0), {s: 0 for s in wl.SIDES}, bcs)
    W0 = wl.conservative(np.array([1.3, 1.3]), np.array([[0.4, 0.1, -0.2], [-0.4, 0.1, -0.2]]), np.array([0.9, 0.9]))
    for recon in (1, 2):
        o = oracle.Oracle(mesh, wl.Params(mu_ref=0.1, n_ref=10, recon=recon))
        o.set_state(W0)
        gW, gH, _ = o.gradients()
        assert np.abs(gW[:, :, 0]).max() < 1e-15
        assert np.abs(gH[:, :, 0]).max() < 1e-15
    # without the mirror (a ghost equal to the cell itself) the normal momentum's gradient
    # would be (W1 - W0)/2 = -0.52: the test above would see it


@pytest.mark.parametrize("recon", [1, 2])
def test_uniform_state_has_zero_gradient_at_every_wall_type(recon):
    # a uniform gas moving along y: diffuse walls at x moving with the gas, far field at y
    # (the free stream is the gas itself), specular walls at z (the velocity is tangential)
    U = (0.0, 0.35, 0.0)
    Wu = wl.conservative(np.array(1.2), np.array(U), np.array(0.8))
    bcs = [wl.BC(wl.BC_DIFFUSE, Tw=0.8, Uw=U), wl.BC(wl.BC_FARFIELD, Winf=tuple(Wu)), wl.BC(wl.BC_SPECULAR)]
    side = {"xlo": 0, "xhi": 0, "ylo": 1, "yhi": 1, "zlo": 2, "zhi": 2}
    for tets in (False, True):
        if tets:
            mesh = wl.tet_box_mesh((3, 3, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 0.7), side, bcs, jitter=0.1, seed=3)
        else:
            mesh = wl.box_hex_mesh((3, 3, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 0.7), side, bcs)
        W0 = np.tile(Wu, (mesh.n_cells, 1))
        o = oracle.Oracle(mesh, wl.Params(mu_ref=0.1, n_ref=10, recon=recon))
        o.set_state(W0)
        gW, gH, _ = o.gradients()
        assert np.abs(gW).max() < 1e-13 and np.abs(gH).max() < 1e-13, (tets, np.abs(gW).max())


def test_diffuse_ghost_continues_a_shear_profile():
    # tangential velocity U_y = U_w + s x next to a diffuse wall at x = 0 moving at U_w: the
    # ghost at x = -1/2 holds 2 U_w - U(1/2) = U(-1/2), so the row's least-squares gradient in
    # the first cell is exactly s rho (a ghost equal to the cell would give s rho / 2)
    Uw, s, rho = 0.2, 0.1, 1.1
    bcs = [wl.BC(wl.BC_DIFFUSE, Tw=1.0, Uw=(0.0, Uw, 0.0)), wl.BC(wl.BC_SPECULAR)]
    side = {"xlo": 0, "xhi": 1, "ylo": 1, "yhi": 1, "zlo": 1, "zhi": 1}
    mesh = wl.box_hex_mesh((3, 3, 1), (0.0, 0.0, 0.0), (3.0, 3.0, 1.0), side, bcs)
    xc = wl.cell_centroids(mesh)
    U = np.zeros((mesh.n_cells, 3))
    U[:, 1] = Uw + s * xc[:, 0]
    W0 = wl.conservative(np.full(mesh.n_cells, rho), U, np.full(mesh.n_cells, 1.0))
    o = oracle.Oracle(mesh, wl.Params(mu_ref=0.1, n_ref=10, recon=1))
    o.set_state(W0)
    gW, _, _ = o.gradients()
    c = int(np.where((np.abs(xc[:, 0] - 0.5) < 1e-12) & (np.abs(xc[:, 1] - 1.5) < 1e-12))[0][0])
    assert abs(gW[c, 2, 0] - s * rho) < 1e-14, gW[c, 2, 0]
    assert abs(gW[c, 0, 0]) < 1e-15
