"""The allocation-free entry point ugkwp_init_mesh_static (the library's own static workspace
instead of a caller's buffer) against ugkwp_init_mesh with a caller's workspace: the same
results bit for bit, on two calls in a row (the shock tube at its full size, then a smaller
tube in the same array), plus its refusals (a mesh too large for the array, a second live
context on the same GPU)."""
import sys

import numpy as np
import pytest

from paper_2007_13091_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-no-alloc]", *a, flush=True)
    sys.stdout.flush()


def _pair(w, steps, precision=0):
    from paper_2007_13091_amd.ugkwp import Solver

    a = Solver(w.mesh, w.params, precision=precision)
    b = Solver(w.mesh, w.params, precision=precision, static_workspace=True)
    assert b.ws is None  # no device memory allocated for it
    a.init_state(w.W0)
    b.init_state(w.W0)
    for n in range(steps):
        sa, sb = a.step(1), b.step(1)
        for k in ("n_alive", "n_sampled", "n_collided", "crossings", "wall_hits"):
            assert sa[k] == sb[k], (n, k, sa[k], sb[k])
    np.testing.assert_array_equal(a.moments(0), b.moments(0))
    np.testing.assert_array_equal(a.moments(1), b.moments(1))
    pa, pb = a.particles(), b.particles()
    for k in ("x", "u", "m", "cell", "uid"):
        np.testing.assert_array_equal(pa[k], pb[k])
    a.close()
    return b


@pytest.mark.parametrize("precision", [0, 1])
def test_static_workspace_matches_caller_workspace_twice(precision):
    from paper_2007_13091_amd.ugkwp import lib

    w = wl.sod()  # 200 box cells, 200 particles per cell: 21 MiB of workspace
    _say("first call: shock tube", w.mesh.n_cells, "cells, precision", precision)
    b = _pair(w, 8, precision)
    b.close()
    assert lib().ugkwp_static_workspace_bytes() == 32 << 20
    w2 = wl.sod(nx=20, n_ref=64, kn=0.01)  # smaller, in the array the first one left
    _say("second call: smaller tube", w2.mesh.n_cells, "cells")
    b2 = _pair(w2, 6, precision)
    b2.close()


def test_static_workspace_refusals():
    from paper_2007_13091_amd.ugkwp import E_CAPACITY, E_STATE, Solver, UgkwpError

    big = wl.cavity(n=8, n_ref=400)  # 68 MiB of workspace
    with pytest.raises(UgkwpError) as e:
        Solver(big.mesh, big.params, static_workspace=True)
    assert e.value.status == E_CAPACITY
    w = wl.sod(nx=20, n_ref=64)
    a = Solver(w.mesh, w.params, static_workspace=True)
    with pytest.raises(UgkwpError) as e:
        Solver(w.mesh, w.params, static_workspace=True)
    assert e.value.status == E_STATE
    a.init_state(w.W0)
    a.step(2)
    a.close()
    # released: a new context may take the array
    b = Solver(w.mesh, w.params, static_workspace=True)
    b.init_state(w.W0)
    assert b.step(1)["n_sampled"] > 0
    b.close()
