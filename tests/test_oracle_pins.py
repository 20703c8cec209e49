"""Pins of the CPU oracle's building blocks against things other than itself.

Each test fixes one part of oracle/ugkwp_oracle.c with a value that the mathematics or an
independent library routine determines: numpy's Philox for the generator, quadrature of
Maxwellians for the moments, quadrature of the printed time coefficients c1..c5 (paper,
Eq. of f_ij(t)) for q1..q5 (paper, Eq. of q1..q5), the Euler flux for a uniform state,
rotation and mirror invariance, and an independent quadrature of the whole first-order
interface flux.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle

RNG = np.random.Generator(np.random.Philox(key=np.array([2024, 11], dtype=np.uint64)))


# ----------------------------------------------------------------------------------------
# Philox4x64-10 and the particle-id layout
# ----------------------------------------------------------------------------------------
def _numpy_philox(ctr, key):
    # numpy increments the 256-bit counter before each block: start one below
    v = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    c = [(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("trial", range(12))
def test_philox_matches_numpy(trial):
    ctr = RNG.integers(0, 2**63, size=4, dtype=np.uint64) * np.uint64(2) + np.uint64(trial % 2)
    if trial == 0:
        ctr = np.array([0, 0, 0, 0], dtype=np.uint64)
    key = RNG.integers(0, 2**63, size=2, dtype=np.uint64)
    np.testing.assert_array_equal(oracle.philox(ctr, key), _numpy_philox(ctr, key))


def test_uid_layout():
    uid = oracle.make_uid(1, 5, 123456, 77)
    assert uid >> 63 == 1
    assert (uid >> 44) & 0x7FFFF == 5
    assert (uid >> 20) & 0xFFFFFF == 123456
    assert uid & 0xFFFFF == 77
    assert oracle.make_uid(0, 0, 0, 0) == 0


# ----------------------------------------------------------------------------------------
# Maxwellian moments: full and half range
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("U,T", [(0.0, 1.0), (0.7, 0.3), (-1.3, 2.5), (4.0, 0.2), (-0.05, 7.0)])
def test_moments_against_quadrature(U, T):
    lam = 1.0 / (2.0 * T)
    mp.mp.dps = 40
    f = lambda u, k: u**k * mp.sqrt(lam / mp.pi) * mp.exp(-lam * (u - U) ** 2)
    for rng in (-1, 0, 1):
        m = oracle.moments(rng, U, lam)
        for k in range(7):
            if rng > 0:
                ref = mp.quad(lambda u: f(u, k), [0, U if U > 0 else 1, mp.inf])
            elif rng < 0:
                ref = mp.quad(lambda u: f(u, k), [-mp.inf, U if U < 0 else -1, 0])
            else:
                ref = mp.quad(lambda u: f(u, k), [-mp.inf, U, mp.inf])
            scale = max(1.0, float(abs(U) + math.sqrt(T))) ** k
            assert abs(m[k] - float(ref)) <= 4e-15 * max(scale, abs(float(ref))), (rng, k, m[k], float(ref))


def test_half_moments_sum_to_full():
    for _ in range(50):
        U = RNG.uniform(-5, 5)
        lam = 1.0 / (2.0 * RNG.uniform(0.05, 10))
        mp_, mn, mf = oracle.moments(1, U, lam), oracle.moments(-1, U, lam), oracle.moments(0, U, lam)
        scale = (abs(U) + math.sqrt(1 / (2 * lam)) + 1) ** np.arange(7)
        assert np.all(np.abs(mp_ + mn - mf) <= 4e-15 * scale)


# ----------------------------------------------------------------------------------------
# q1..q5: time integrals of the printed c1..c5 over [0, dt]
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("x", [1e-8, 1e-5, 1e-3, 0.03, 0.3, 0.999, 1.0, 1.7, 10.0, 1e3, 1e8])
def test_qcoef_against_integrated_c(x):
    mp.mp.dps = 50
    tau = mp.mpf("0.37")
    dt = tau * mp.mpf(x)
    E = lambda t: mp.exp(-t / tau)
    c = [lambda t: 1 - E(t),
         lambda t: t * E(t) - tau * (1 - E(t)),
         lambda t: t - tau * (1 - E(t)),
         lambda t: E(t),
         lambda t: -t * E(t)]
    pts = [0, min(dt, 50 * tau), dt] if dt > 50 * tau else [0, dt]
    qs = [mp.quad(ci, pts) for ci in c]
    e = E(dt)
    ref = [qs[0], qs[1], qs[2], qs[3] - dt * e, qs[4] + dt * dt * e / 2]
    got = oracle.qcoef(float(dt), float(tau))
    for k in range(5):
        # each coefficient is O(tau dt-scale); compare relative to its own size where it is
        # well resolved, else relative to the natural scale of its time power
        nat = float(dt if k in (0, 3) else dt * dt)
        err = abs(got[k] - float(ref[k]))
        assert err <= 1e-13 * abs(float(ref[k])) + 1e-15 * nat, (k, got[k], float(ref[k]))


def test_qcoef_limits():
    # dt >> tau: q1 -> dt, q3 -> dt^2/2; dt << tau: q4 -> dt, q5 -> -dt^2/2 (paper, after Eq. q1..q5)
    dt = 0.01
    q = oracle.qcoef(dt, 1e-12)
    assert abs(q[0] - dt) < 1e-11 and abs(q[2] - dt * dt / 2) < 1e-12
    q = oracle.qcoef(dt, 1e12)
    x = dt / 1e12
    e = math.exp(-x)
    assert abs((q[3] + dt * e) - dt) < 1e-15 and abs((q[4] - dt * dt * e / 2) + dt * dt / 2) < 1e-16


# ----------------------------------------------------------------------------------------
# interface flux
# ----------------------------------------------------------------------------------------
def _W(rho, U, T):
    U = np.asarray(U, dtype=float)
    return np.array([rho, *(rho * U), 0.5 * rho * U @ U + 1.5 * rho * T])


def _euler_flux(W, n):
    rho = W[0]
    U = W[1:4] / rho
    T = (2 / 3) * (W[4] - 0.5 * rho * U @ U) / rho
    p = rho * T
    un = U @ n
    return np.array([rho * un, *(rho * un * U + p * n), (W[4] + p) * un])


def _unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("trial", range(8))
def test_uniform_state_flux_is_scaled_euler_flux(trial):
    rho = RNG.uniform(0.1, 3)
    U = RNG.uniform(-2, 2, 3)
    T = RNG.uniform(0.2, 4)
    n = _unit(RNG.normal(size=3))
    W = _W(rho, U, T)
    mu, om, dt = RNG.uniform(1e-4, 1e-1), 0.81, RNG.uniform(1e-4, 1e-2)
    tau = mu * T**om / (rho * T)
    e = math.exp(-dt / tau)
    FE = _euler_flux(W, n)
    # hydro density = total: q1 + q4 - dt e = dt (1 - e)
    F = oracle.flux_interior(W, W, rho, rho, n, dt, mu, om, 0.0)
    np.testing.assert_allclose(F, dt * (1 - e) * FE, rtol=1e-12, atol=1e-14 * np.abs(FE).max() * dt)
    # no hydro density: equilibrium part only, q1 = dt - tau (1 - e)
    F0 = oracle.flux_interior(W, W, 0.0, 0.0, n, dt, mu, om, 0.0)
    q1 = dt - tau * (1 - e)
    np.testing.assert_allclose(F0, q1 * FE, rtol=1e-11, atol=1e-14 * np.abs(FE).max() * dt)


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


@pytest.mark.parametrize("trial", range(8))
def test_flux_rotation_and_mirror(trial):
    Wl = _W(RNG.uniform(0.2, 2), RNG.uniform(-1.5, 1.5, 3), RNG.uniform(0.3, 3))
    Wr = _W(RNG.uniform(0.2, 2), RNG.uniform(-1.5, 1.5, 3), RNG.uniform(0.3, 3))
    hl, hr = Wl[0] * RNG.uniform(0, 1), Wr[0] * RNG.uniform(0, 1)
    n = _unit(RNG.normal(size=3))
    args = (0.004, 0.02, 0.81, 3.0)
    F = oracle.flux_interior(Wl, Wr, hl, hr, n, *args)
    R = _rot(RNG)
    rW = lambda W: np.array([W[0], *(R @ W[1:4]), W[4]])
    FR = oracle.flux_interior(rW(Wl), rW(Wr), hl, hr, R @ n, *args)
    np.testing.assert_allclose(FR, rW(F), rtol=1e-12, atol=1e-13 * np.abs(F).max())
    Fm = oracle.flux_interior(Wr, Wl, hr, hl, -n, *args)
    np.testing.assert_allclose(Fm, -F, rtol=1e-13, atol=1e-15 * np.abs(F).max())


def _gl(a, b, k=80):
    x, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _quad_flux(Wl, Wr, hl, hr, n, dt, mu, om, c2):
    """Independent quadrature of the first-order interface flux in a face frame built here
    (any orthonormal frame works): half-range u_n by Gauss-Legendre on each side of 0,
    transverse velocities by Gauss-Hermite."""
    n = _unit(n)
    a = np.array([1.0, 0, 0]) if abs(n[0]) < 0.9 else np.array([0, 1.0, 0])
    t1 = _unit(np.cross(n, a)); t2 = np.cross(n, t1)
    B = np.stack([n, t1, t2])
    xh, wh = np.polynomial.hermite.hermgauss(40)

    def side(W):
        rho = W[0]; U = B @ (W[1:4] / rho); T = (2 / 3) * (W[4] - 0.5 * (W[1:4] @ W[1:4]) / rho) / rho
        return rho, U, T

    def maxw_grid(U, T, rng):
        s = math.sqrt(2 * T)
        lo, hi = U[0] - 12 * math.sqrt(T), U[0] + 12 * math.sqrt(T)
        if rng > 0:
            lo = max(lo, 0.0)
        elif rng < 0:
            hi = min(hi, 0.0)
        if hi <= lo:
            return None
        un, wn = _gl(lo, hi, 120)
        fn = np.exp(-(un - U[0]) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T)
        v = U[1] + s * xh; w = U[2] + s * xh
        wv = wh / math.sqrt(math.pi)
        UN, V, Wt = np.meshgrid(un, v, w, indexing="ij")
        Wgt = (wn * fn)[:, None, None] * wv[None, :, None] * wv[None, None, :]
        return UN, V, Wt, Wgt

    def mom(U, T, rng, weight_un):
        g = maxw_grid(U, T, rng)
        if g is None:
            return np.zeros(5)
        UN, V, Wt, Wg = g
        psi = [np.ones_like(UN), UN, V, Wt, 0.5 * (UN**2 + V**2 + Wt**2)]
        f = Wg * (UN if weight_un else 1.0)
        return np.array([(f * p).sum() for p in psi])

    rl, Ul, Tl = side(Wl)
    rr, Ur, Tr = side(Wr)
    W0 = rl * mom(Ul, Tl, 1, False) + rr * mom(Ur, Tr, -1, False)
    r0 = W0[0]; U0 = W0[1:4] / r0; T0 = (2 / 3) * (W0[4] - 0.5 * r0 * U0 @ U0) / r0
    tau = mu * T0**om / (r0 * T0) + c2 * abs(rl * Tl - rr * Tr) / (rl * Tl + rr * Tr) * dt
    e = math.exp(-dt / tau)
    q1 = dt - tau * (1 - e)
    q4m = tau * (1 - e) - dt * e
    Ff = q1 * r0 * mom(U0, T0, 0, True) + q4m * (hl * mom(Ul, Tl, 1, True) + hr * mom(Ur, Tr, -1, True))
    return np.array([Ff[0], *(Ff[1] * n + Ff[2] * t1 + Ff[3] * t2), Ff[4]])


@pytest.mark.parametrize("trial", range(5))
def test_flux_against_independent_quadrature(trial):
    Wl = _W(RNG.uniform(0.2, 2), RNG.uniform(-1.5, 1.5, 3), RNG.uniform(0.3, 3))
    Wr = _W(RNG.uniform(0.2, 2), RNG.uniform(-1.5, 1.5, 3), RNG.uniform(0.3, 3))
    hl, hr = Wl[0] * RNG.uniform(0, 1), Wr[0] * RNG.uniform(0, 1)
    n = _unit(RNG.normal(size=3))
    args = (RNG.uniform(1e-3, 1e-2), RNG.uniform(1e-3, 1e-1), 0.81, 2.0 * trial)
    F = oracle.flux_interior(Wl, Wr, hl, hr, n, *args)
    G = _quad_flux(Wl, Wr, hl, hr, n, *args)
    np.testing.assert_allclose(F, G, rtol=1e-10, atol=1e-11 * np.abs(G).max())


def test_specular_wall_flux_is_pressure_for_gas_at_rest():
    rho, T, dt, mu = 0.8, 1.3, 3e-3, 0.02
    n = _unit([0.3, -0.4, 0.866])
    W = _W(rho, [0, 0, 0], T)
    tau = mu * T**0.81 / (rho * T)
    e = math.exp(-dt / tau)
    F = oracle.flux_specular(W, rho, n, dt, mu, 0.81, 0.0)
    np.testing.assert_allclose(F, np.array([0, *(dt * (1 - e) * rho * T * n), 0]), rtol=1e-13, atol=1e-17)


def test_specular_wall_flux_matches_mirror_quadrature():
    W = _W(0.9, [0.4, -0.2, 0.3], 1.1)
    n = _unit([1.0, 0.5, -0.2])
    Ug = W[1:4] / W[0] - 2 * (W[1:4] / W[0] @ n) * n
    Wg = _W(0.9, Ug, 1.1)
    G = _quad_flux(W, Wg, 0.5, 0.5, n, 2e-3, 0.01, 0.81, 0.0)
    F = oracle.flux_specular(W, 0.5, n, 2e-3, 0.01, 0.81, 0.0)
    Gn = G[1:4] @ n
    np.testing.assert_allclose(F, np.array([0, *(Gn * n), 0]), rtol=1e-10, atol=1e-13)


def test_diffuse_wall_flux_at_equilibrium_is_pressure():
    # gas at rest at the wall temperature: emitted half = mirror of incoming half
    rho, T, dt, tau = 1.2, 0.9, 2e-3, 4e-3
    n = _unit([0.0, 0.0, 1.0])
    W = _W(rho, [0, 0, 0], T)
    e = math.exp(-dt / tau)
    F = oracle.flux_diffuse(W, rho, tau, n, dt, T, [0, 0, 0])
    np.testing.assert_allclose(F, np.array([0, 0, 0, dt * (1 - e) * rho * T, 0]), rtol=1e-13, atol=1e-18)


def test_diffuse_wall_flux_zero_mass_and_emitted_moments():
    rho, T, dt, tau = 0.7, 1.4, 2e-3, 3e-3
    n = _unit([0.2, 0.9, -0.1])
    U = np.array([0.3, 0.5, -0.4])
    W = _W(rho, U, T)
    Tw, Uw = 0.8, np.array([0.0, 0.0, 0.0])
    F = oracle.flux_diffuse(W, 0.3, tau, n, dt, Tw, Uw)
    assert F[0] == 0.0
    # incoming by quadrature of the one-sided integrals; outgoing from the closed form of a
    # half Maxwellian at rest: <u_n> = -sqrt(Tw/2pi), <u_n^2> = Tw/2, <u_n |u|^2/2> = -sqrt(Tw/2pi) * 2 Tw
    e = math.exp(-dt / tau)
    q1 = dt - tau * (1 - e); q4m = tau * (1 - e) - dt * e
    # one-sided incoming moments, computed directly from the erfc closed form
    s = math.sqrt(T); un = U @ n
    z = un / math.sqrt(2 * T)
    m0 = 0.5 * math.erfc(-z); m1 = un * m0 + s * math.exp(-z * z) / math.sqrt(2 * math.pi)
    fin_mass = (q1 * rho + q4m * 0.3) * m1
    rhow = fin_mass / (dt * math.sqrt(Tw / (2 * math.pi)))
    out_n = dt * rhow * Tw / 2
    m2 = un * m1 + T * m0
    in_n = (q1 * rho + q4m * 0.3) * m2
    assert abs(F[1:4] @ n - (in_n + out_n)) < 1e-13 * abs(in_n + out_n)
