"""Pins of the energy-exact pair sampling (the oracle's reading of the hydro-particle
sampling): per cell, the sampled particles carry exactly the momentum and the thermal
energy of the Maxwellian they are drawn from.

* every cell's sample has mean velocity U and temperature (about U) T of the cell's W,
  to roundoff; these are the plain definitions, computed from the particles;
* pairs stay antithetic (u + u' = 2U);
* the marginal velocity law over many cells is still the Maxwellian (the common factor
  tends to 1 as 1/sqrt(N));
* a Mach 10 free-molecular box, which reaches T <= 0 within ten steps when the thermal energy
  of the samples is left to chance, stays physical."""
import math

import numpy as np
from scipy import stats

import oracle
from paper_2007_13091_amd import workloads as wl


def _prim(W):
    rho = W[:, 0]
    U = W[:, 1:4] / rho[:, None]
    T = (2 / 3) * (W[:, 4] - 0.5 * rho * (U * U).sum(1)) / rho
    return rho, U, T


def _sampled_state(w):
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    o.sample_only()
    return o, o.particles()


def test_each_cell_sample_has_exact_mean_velocity_and_temperature():
    w = wl.closed_box(n=(4, 3, 3), n_ref=24, kn=0.05, perturb=0.3)
    o, p = _sampled_state(w)
    _, U, T = _prim(w.W0)
    c = p["cell"].astype(np.int64)
    m, u = p["m"], p["u"]
    nc = w.mesh.n_cells
    M = np.bincount(c, weights=m, minlength=nc)
    assert np.all(M > 0)
    Ubar = np.stack([np.bincount(c, weights=m * u[:, d], minlength=nc) for d in range(3)], 1) / M[:, None]
    dev = u - U[c]
    Ts = np.bincount(c, weights=m * (dev * dev).sum(1), minlength=nc) / (3 * M)
    assert np.abs(Ubar - U).max() <= 1e-13 * np.sqrt(T).max()
    assert np.abs(Ts / T - 1).max() <= 1e-13


def test_pairs_stay_antithetic():
    w = wl.closed_box(n=(3, 2, 2), n_ref=20, kn=0.05, perturb=0.3)
    o, p = _sampled_state(w)
    _, U, _ = _prim(w.W0)
    k = (p["uid"] & np.uint64(0xFFFFF)).astype(np.int64)
    cell = p["cell"].astype(np.int64)
    key = cell * (1 << 20) + (k // 2)
    order = np.lexsort((k, key))
    a, b = order[0::2], order[1::2]
    assert np.all(key[a] == key[b])
    np.testing.assert_allclose(p["u"][a] + p["u"][b], 2 * U[cell[a]], rtol=0, atol=1e-13 * 4)


def test_velocity_law_over_many_cells_is_maxwellian():
    # uniform gas at rest, T = 1: the pooled x-velocities of 200 cells x 40 particles
    w = wl.closed_box(n=(10, 5, 4), n_ref=40, kn=0.05, perturb=0.0)
    o, p = _sampled_state(w)
    ks = stats.kstest(p["u"][:, 0], "norm")
    assert ks.pvalue > 1e-3, ks
    # the per-cell factors sit near 1: the second moment pools to exactly 3 T
    assert abs((p["u"] ** 2).sum(1).mean() - 3.0) < 1e-12


def test_mach10_free_molecular_box_stays_physical():
    U = 10 * math.sqrt(5 / 3)
    w = wl.free_stream_box(n=(4, 3, 3), U=(U, 0, 0), n_ref=30, kn=1e6, cfl=0.9)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    for _ in range(40):
        o.step()
    W, _, _ = o.state()
    _, _, T = _prim(W)
    assert T.min() > 0.3, T.min()
