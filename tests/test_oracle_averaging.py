"""Oracle pins for time averaging (Sec. 2.4(c)): Wbar^n = sum_{m > N_avg} dt^m W^m /
sum_{m > N_avg} dt^m over the steps after N_avg, and its relative change between successive
steps in the volume-weighted L1 norm of the whole field (the paper leaves the norm open).

What fixes the oracle's running sums without restating them:
* a state that does not change averages to itself, with zero change;
* a single averaged step is that step's state, and the change is infinite (undefined);
* every W^n of a closed specular box holds the same mass and energy, so any average with
  weights that sum to one does too: a wrong normaliser fails;
* the closed form Wbar^n - Wbar^{n-1} = (dt^n / D^{n-1}) (W^n - Wbar^n), with D^{n-1} the
  sum of the earlier recorded steps, holds only for the dt-weighted mean: with the ~1% step
  to step variation of dt in the shock tube a plain mean, a shifted weight or a wrong D fails
  it (the change of the average is formed here from that closed form, not as the oracle
  forms it, a difference of two averages);
* the step count: steps n > N_avg exactly."""
import numpy as np
import pytest

import oracle
from paper_2007_13091_amd import workloads as wl


def _l1(vol, X):
    return float((vol[:, None] * np.abs(X)).sum())


def test_steady_state_averages_to_itself():
    w = wl.closed_box(n=(3, 3, 3), perturb=0.0)
    w.params.mu_ref = 1e-14  # no particles: the uniform gas at rest stays as it is
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    o.set_averaging(1)
    for _ in range(6):
        o.step()
    Wb, res, n = o.average()
    assert n == 5
    np.testing.assert_allclose(Wb, w.W0, rtol=0, atol=1e-14)
    assert res <= 1e-15


def test_one_averaged_step_is_that_state_and_nothing_before_it():
    w = wl.sod(nx=12, ny=1, nz=1, n_ref=30)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    o.set_averaging(3)
    for _ in range(3):
        o.step()
        with pytest.raises(oracle.OracleError):
            o.average()
    o.step()
    Wb, res, n = o.average()
    W, _, _ = o.state()
    assert n == 1 and res == np.inf
    # (dt W) / dt: within one rounding of W
    np.testing.assert_allclose(Wb, W, rtol=2.3e-16, atol=0)


@pytest.mark.parametrize("tets", [False, True])
def test_average_of_a_closed_box_holds_its_mass_and_energy(tets):
    w = wl.closed_box(n=(3, 3, 2), n_ref=40, kn=0.05, tets=tets, jitter=0.1 if tets else 0.0)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    vol, _, _ = o.geometry()
    o.set_averaging(2)
    for _ in range(10):
        o.step()
    Wb, res, n = o.average()
    W, _, _ = o.state()
    assert n == 8 and 0 < res < 1
    tot0 = (vol[:, None] * w.W0.reshape(-1, 5)).sum(0)
    totb = (vol[:, None] * Wb).sum(0)
    assert abs(totb[0] - tot0[0]) <= 1e-13 * tot0[0]
    assert abs(totb[4] - tot0[4]) <= 1e-13 * tot0[4]
    # the average is not the last state (particles make the field fluctuate)
    assert np.abs(Wb - W).max() > 1e-6


def test_change_of_the_average_follows_the_dt_weighted_closed_form():
    w = wl.sod(n_ref=60)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    vol, _, _ = o.geometry()
    o.set_averaging(2)
    o.step(2)
    dts, prev = [], None
    for _ in range(8):
        o.step()
        dt = o.stats()["dt"]
        Wb, res, n = o.average()
        W, _, _ = o.state()
        if prev is not None:
            D_prev = sum(dts)
            dWb = (dt / D_prev) * (W - Wb)
            # the difference of two averages against the closed form
            scale = np.abs(W - Wb).max() * dt / D_prev
            np.testing.assert_allclose(Wb - prev, dWb, rtol=0, atol=1e-9 * scale)
            np.testing.assert_allclose(res, _l1(vol, dWb) / _l1(vol, Wb), rtol=1e-8)
        dts.append(dt)
        prev = Wb
    assert n == 8
    # the weights matter: dt varies by far more than the tolerance above
    assert (max(dts) - min(dts)) / max(dts) > 1e-3


def test_plain_mean_differs_from_the_dt_weighted_average():
    # the same run averaged by hand both ways: the oracle's average is the weighted one
    w = wl.sod(n_ref=60)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    o.set_averaging(0)
    Ws, dts = [], []
    for _ in range(12):
        o.step()
        Ws.append(o.state()[0])
        dts.append(o.stats()["dt"])
    Wb, _, n = o.average()
    assert n == 12
    Ws, dts = np.array(Ws), np.array(dts)
    weighted = (dts[:, None, None] * Ws).sum(0) / dts.sum()
    plain = Ws.mean(0)
    err_w = np.abs(Wb - weighted).max()
    err_p = np.abs(Wb - plain).max()
    assert err_w <= 1e-14 * np.abs(weighted).max()
    assert err_p > 1e3 * max(err_w, 1e-300)


def test_averaging_off_and_reset():
    w = wl.sod(nx=12, ny=1, nz=1, n_ref=30)
    o = oracle.Oracle(w.mesh, w.params)
    o.set_state(w.W0)
    o.step(2)
    with pytest.raises(oracle.OracleError):
        o.average()  # off by default
    o.set_averaging(0)  # steps from now on (their counter is past 0)
    o.step(2)
    assert o.average()[2] == 2
    o.set_averaging(-1)
    o.step()
    with pytest.raises(oracle.OracleError):
        o.average()
    o.set_averaging(0)
    o.step()
    assert o.average()[2] == 1
    o.set_state(w.W0)  # a new state clears the sums and keeps the setting
    with pytest.raises(oracle.OracleError):
        o.average()
    o.step()
    assert o.average()[2] == 1
