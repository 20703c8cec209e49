"""Comparison helpers for GPU-vs-oracle parity (no arithmetic of the method here).

Bar: integers (particle ids, cells, counts, collided/escaped decisions, crossings) equal;
floating-point fields within 1e-12 relative.  For vector components that can be near zero
(momenta, particle velocities and positions) the relative error is taken against the
natural scale of the quantity (rho sqrt(T) for momentum, the thermal speed for velocities,
the domain size for positions), so that a value of 0 +- roundoff does not read as a large
relative error.
"""
import numpy as np

RTOL = 1e-12
INT_KEYS = ("n_alive", "n_sampled", "n_injected", "n_collided", "n_escaped", "crossings", "wall_hits",
            "max_crossings_seen")
BATCH_TOTALS = ("crossings", "wall_hits", "max_crossings_seen")  # reported for the whole batch only


def _field_err(a, b, W_ref):
    rho = np.abs(W_ref[:, 0])
    ke = 0.5 * (W_ref[:, 1:4] ** 2).sum(1) / np.maximum(rho, 1e-300)
    T = np.maximum((2 / 3) * (W_ref[:, 4] - ke) / np.maximum(rho, 1e-300), 0)
    mscale = rho * (np.sqrt(T) + np.sqrt((W_ref[:, 1:4] ** 2).sum(1)) / np.maximum(rho, 1e-300))
    scale = np.stack([rho, mscale, mscale, mscale, np.abs(W_ref[:, 4])], 1)
    return np.abs(a - b) / np.maximum(scale, 1e-300)


def compare_fields(Wg, Wo, Pg, Po, vol, rtol=RTOL, what=""):
    ew = _field_err(Wg, Wo, Wo)
    assert ew.max() <= rtol, f"{what} W rel err {ew.max():.3e} at cell {np.unravel_index(ew.argmax(), ew.shape)}"
    # particle sums: scale by the particle density of the cell (P / Omega)
    Pv = Po / vol[:, None]
    has = Po[:, 0] > 0
    if np.any(has):
        ep = _field_err(Pg[has] / vol[has, None], Pv[has], Pv[has])
        assert ep.max() <= rtol, f"{what} P rel err {ep.max():.3e}"
    assert np.all((Pg[:, 0] > 0) == has), f"{what} particle-holding cells differ"


def compare_particles(pg, po, length=1.0, vscale=1.0, rtol=RTOL, what=""):
    assert pg["uid"].shape == po["uid"].shape, f"{what} particle counts {pg['uid'].shape} vs {po['uid'].shape}"
    ig = np.argsort(pg["uid"], kind="stable")
    io = np.argsort(po["uid"], kind="stable")
    np.testing.assert_array_equal(pg["uid"][ig], po["uid"][io], err_msg=f"{what} particle ids")
    np.testing.assert_array_equal(pg["cell"][ig].astype(np.int64), po["cell"][io].astype(np.int64),
                                  err_msg=f"{what} particle cells")
    if pg["uid"].size == 0:
        return
    dx = np.abs(pg["x"][ig] - po["x"][io]).max() / length
    du = np.abs(pg["u"][ig] - po["u"][io]).max() / vscale
    # particle masses: m = rho^hp Omega / N_sam, and rho^h = rho - rho^p cancels where particles
    # hold most of the mass; compare against the mean particle mass of the cell
    cells = po["cell"][io].astype(np.int64)
    nc = int(cells.max()) + 1 if cells.size else 0
    msum = np.bincount(cells, weights=np.abs(po["m"][io]), minlength=nc)
    mcnt = np.bincount(cells, minlength=nc)
    mscale = msum[cells] / np.maximum(mcnt[cells], 1)
    dm = (np.abs(pg["m"][ig] - po["m"][io]) / mscale).max() if cells.size else 0.0
    assert dx <= rtol and du <= rtol and dm <= rtol, f"{what} particle state dx {dx:.2e} du {du:.2e} dm {dm:.2e}"
    if "e" in pg and "e" in po:
        # internal energy variables (K > 0), against the thermal scale vscale^2
        de = np.abs(pg["e"][ig] - po["e"][io]).max() / (vscale * vscale)
        assert de <= rtol, f"{what} particle internal energies de {de:.2e}"


def compare_stats(sg, so, what=""):
    for k in INT_KEYS:
        assert sg[k] == so[k], f"{what} {k}: gpu {sg[k]} oracle {so[k]}"
    assert abs(sg["dt"] - so["dt"]) <= RTOL * so["dt"], f"{what} dt {sg['dt']} vs {so['dt']}"
