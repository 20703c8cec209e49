"""Seeded synthetic inputs: meshes, boundary tables, parameters and initial states.

This module holds no arithmetic of the method itself.  It builds the inputs that both the
GPU library and the CPU oracle consume: unstructured meshes given as node coordinates plus
cell connectivity (4-node tetrahedra, 8-node axis-aligned boxes in VTK node order),
tagged boundary faces, a boundary-condition table, solver parameters and the initial
conservative state W = (rho, rho U, rho E) per cell (R = 1, monatomic, rho E = rho |U|^2/2 +
3 rho T / 2).

Workloads follow the paper's test cases (Sec. 4): the shock tube in a square column
(Sec. 4.1), the lid-driven cubic cavity (Sec. 4.2), and the flow past a cube (Sec. 4.3),
at the sizes of the hot-path configurations described in the design notes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_SPECULAR = 0
BC_DIFFUSE = 1
BC_FARFIELD = 2
BC_PERIODIC = 3  # test support: a face leads to the face at x + shift (not a condition of the paper)

CELL_TET = 4
CELL_HEX = 8

# box sides in the order the generators tag them
SIDES = ("xlo", "xhi", "ylo", "yhi", "zlo", "zhi")


@dataclass
class BC:
    type: int
    Tw: float = 1.0
    Uw: tuple = (0.0, 0.0, 0.0)
    Winf: tuple = (0.0, 0.0, 0.0, 0.0, 0.0)
    shift: tuple = (0.0, 0.0, 0.0)  # periodic: a point x of a tagged face matches x + shift


@dataclass
class Mesh:
    xyz: np.ndarray            # [n_nodes, 3] float64
    cell_type: np.ndarray      # [n_cells] uint8 (4 or 8)
    cell_node_off: np.ndarray  # [n_cells + 1] int64
    cell_nodes: np.ndarray     # [sum nodes] int64
    bface_nodes: np.ndarray    # [n_bfaces, 4] int64, -1 pads a triangle
    bface_bc: np.ndarray       # [n_bfaces] int32, index into bcs
    bcs: list = field(default_factory=list)

    @property
    def n_cells(self) -> int:
        return int(self.cell_type.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    def bc_arrays(self):
        t = np.array([b.type for b in self.bcs], dtype=np.int32)
        tw = np.array([b.Tw for b in self.bcs], dtype=np.float64)
        uw = np.array([b.Uw for b in self.bcs], dtype=np.float64).reshape(-1, 3)
        wi = np.array([b.Winf for b in self.bcs], dtype=np.float64).reshape(-1, 5)
        sh = np.array([b.shift for b in self.bcs], dtype=np.float64).reshape(-1, 3)
        return t, tw, np.ascontiguousarray(uw), np.ascontiguousarray(wi), np.ascontiguousarray(sh)


@dataclass
class Params:
    mu_ref: float
    omega: float = 0.81
    cfl: float = 0.5
    c2: float = 0.0
    n_ref: int = 200
    n_min: int = 0
    max_crossings: int = 1000
    seed: int = 1
    gamma: float = 5.0 / 3.0
    recon: int = 0          # 0 first order, 1 LSQ + Barth-Jespersen, 2 LSQ + Venkatakrishnan
    venkat_k: float = 1.0   # Venkatakrishnan constant K
    sampling: int = 0       # hydro-particle velocities: 0 the pairs U +- sqrt(T) X of Sec. 2.4(b),
                            # 1 the energy-exact variant (one factor per cell on the deviations),
                            # 2 the first-order g_p of Sec. 2.3 (needs recon 1 or 2),
                            # 3 independent draws from the collision model's equilibrium
    gks_steps: int = 0      # steps from the initial state run wave-only (no particles): the
                            # continuum start of the paper's hypersonic cases
    prandtl: float = 1.0    # collision model: 1 the BGK model of the paper, otherwise the Shakhov
                            # model with this Prandtl number (K = 0, sampling 2 or 3)


def mu_ref_from_kn(kn: float, omega: float) -> float:
    """Reference viscosity of a VHS gas for a Knudsen number at rho = T = L = 1 (R = 1)."""
    return 15.0 * math.sqrt(2.0 * math.pi) * kn / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))


def internal_dof(gamma: float) -> int:
    """K internal degrees of freedom of gamma = (K + 5)/(K + 3) (5/3: K = 0; 7/5: K = 2)."""
    K = 2.0 / (gamma - 1.0) - 3.0
    Ki = int(round(K))
    if abs(K - Ki) > 1e-9 or Ki < 0:
        raise ValueError(f"gamma = {gamma} is not (K + 5)/(K + 3) for an integer K >= 0")
    return Ki


def conservative(rho, U, T, K=0):
    """W = (rho, rho U, rho E) with R = 1 and K internal degrees of freedom:
    rho E = rho |U|^2/2 + (3 + K)/2 rho T (K = 0: monatomic)."""
    rho = np.asarray(rho, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    W = np.empty(rho.shape + (5,), dtype=np.float64)
    W[..., 0] = rho
    W[..., 1:4] = rho[..., None] * U
    W[..., 4] = 0.5 * rho * (U * U).sum(-1) + 0.5 * (3 + K) * rho * T
    return W


# --------------------------------------------------------------------------------------
# box-hex meshes
# --------------------------------------------------------------------------------------
def _axis_nodes(lo, hi, n, grading=None):
    if grading is None:
        return np.linspace(lo, hi, n + 1)
    return np.asarray(grading, dtype=np.float64)


def box_hex_mesh(n, lo, hi, side_bc, bcs, coords=None) -> Mesh:
    """Structured box of axis-aligned hexahedra given as unstructured connectivity.

    n: (nx, ny, nz); lo, hi: corners; side_bc: dict side name -> index into bcs;
    coords: optional explicit node coordinates per axis (graded meshes).
    Cells are numbered x fastest, then y, then z.
    """
    nx, ny, nz = n
    ax = [coords[a] if coords is not None else _axis_nodes(lo[a], hi[a], n[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(), Z.transpose(2, 1, 0).ravel()], 1)

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i = i.transpose(2, 1, 0).ravel()
    j = j.transpose(2, 1, 0).ravel()
    k = k.transpose(2, 1, 0).ravel()
    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    cn = np.stack([nid(i + a, j + b, k + c) for (a, b, c) in corners], 1).astype(np.int64)
    nc = cn.shape[0]
    bf, bt = _box_boundary(n, nid, side_bc)
    return Mesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                cell_type=np.full(nc, CELL_HEX, dtype=np.uint8),
                cell_node_off=np.arange(0, 8 * nc + 1, 8, dtype=np.int64),
                cell_nodes=cn.ravel(), bface_nodes=bf, bface_bc=bt, bcs=list(bcs))


def _box_boundary(n, nid, side_bc, tri_split=False):
    nx, ny, nz = n
    faces, tags = [], []

    def quad(p, q, r, s, tag):
        if tri_split:
            # Kuhn split: the diagonal of each boundary quad runs through its lowest and highest
            # corner (p and r in the order given), which matches the tetrahedra of tet_box_mesh
            faces.append((p, q, r, -1)); tags.append(tag)
            faces.append((p, r, s, -1)); tags.append(tag)
        else:
            faces.append((p, q, r, s)); tags.append(tag)

    for jj in range(ny):
        for kk in range(nz):
            quad(nid(0, jj, kk), nid(0, jj + 1, kk), nid(0, jj + 1, kk + 1), nid(0, jj, kk + 1), side_bc["xlo"])
            quad(nid(nx, jj, kk), nid(nx, jj + 1, kk), nid(nx, jj + 1, kk + 1), nid(nx, jj, kk + 1), side_bc["xhi"])
    for ii in range(nx):
        for kk in range(nz):
            quad(nid(ii, 0, kk), nid(ii + 1, 0, kk), nid(ii + 1, 0, kk + 1), nid(ii, 0, kk + 1), side_bc["ylo"])
            quad(nid(ii, ny, kk), nid(ii + 1, ny, kk), nid(ii + 1, ny, kk + 1), nid(ii, ny, kk + 1), side_bc["yhi"])
    for ii in range(nx):
        for jj in range(ny):
            quad(nid(ii, jj, 0), nid(ii + 1, jj, 0), nid(ii + 1, jj + 1, 0), nid(ii, jj + 1, 0), side_bc["zlo"])
            quad(nid(ii, jj, nz), nid(ii + 1, jj, nz), nid(ii + 1, jj + 1, nz), nid(ii, jj + 1, nz), side_bc["zhi"])
    return np.array(faces, dtype=np.int64).reshape(-1, 4), np.array(tags, dtype=np.int32)


# Kuhn (Freudenthal) split of a box into 6 tetrahedra along the diagonal from corner 0 to
# corner 6: one tetrahedron per ordering of the three axes.  Conforming between neighbours.
_KUHN = []
for _perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
    _b = [0, 0, 0]
    _path = [tuple(_b)]
    for _a in _perm:
        _b[_a] = 1
        _path.append(tuple(_b))
    _KUHN.append(_path)


def tet_box_mesh(n, lo, hi, side_bc, bcs, jitter=0.0, seed=1, coords=None) -> Mesh:
    """Box of hexahedra, each split into 6 tetrahedra (Kuhn split along the 0-6 diagonal).

    jitter: interior nodes move uniformly within +-jitter*h per axis (h: local spacing),
    seeded; boundary nodes stay on their planes (they move only within them).
    """
    nx, ny, nz = n
    ax = [coords[a] if coords is not None else _axis_nodes(lo[a], hi[a], n[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(), Z.transpose(2, 1, 0).ravel()], 1)
    if jitter > 0.0:
        rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x4D455348], dtype=np.uint64)))
        for a in range(3):
            h = np.diff(ax[a])
            hloc = np.minimum(np.concatenate([[h[0]], h]), np.concatenate([h, [h[-1]]]))
            idx = [np.arange(n[0] + 1), np.arange(n[1] + 1), np.arange(n[2] + 1)]
            I, J, K = np.meshgrid(*idx, indexing="ij")
            I = I.transpose(2, 1, 0).ravel(); J = J.transpose(2, 1, 0).ravel(); K = K.transpose(2, 1, 0).ravel()
            pos = (I, J, K)[a]
            inner = (pos > 0) & (pos < n[a])
            d = rng.uniform(-jitter, jitter, size=xyz.shape[0]) * hloc[pos]
            xyz[:, a] = np.where(inner, xyz[:, a] + d, xyz[:, a])

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i = i.transpose(2, 1, 0).ravel(); j = j.transpose(2, 1, 0).ravel(); k = k.transpose(2, 1, 0).ravel()
    tets = []
    for path in _KUHN:
        tets.append(np.stack([nid(i + a, j + b, k + c) for (a, b, c) in path], 1))
    cn = np.stack(tets, 1).reshape(-1, 4).astype(np.int64)
    nc = cn.shape[0]
    bf, bt = _box_boundary(n, nid, side_bc, tri_split=True)
    return Mesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                cell_type=np.full(nc, CELL_TET, dtype=np.uint8),
                cell_node_off=np.arange(0, 4 * nc + 1, 4, dtype=np.int64),
                cell_nodes=cn.ravel(), bface_nodes=bf, bface_bc=bt, bcs=list(bcs))


def cell_centroids(mesh: Mesh) -> np.ndarray:
    """Node average per cell (inputs only: used to place initial states)."""
    off = mesh.cell_node_off
    nn = np.diff(off)
    out = np.zeros((mesh.n_cells, 3))
    for k in np.unique(nn):
        sel = np.nonzero(nn == k)[0]
        idx = mesh.cell_nodes[off[sel][:, None] + np.arange(k)[None, :]]
        out[sel] = mesh.xyz[idx].mean(1)
    return out


# --------------------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    mesh: Mesh
    params: Params
    W0: np.ndarray  # [n_cells, 5]
    steps: int


def morton_numbered(w: Workload, bits: int = 10) -> Workload:
    """The same workload with its cells numbered along a Morton (Z-order) curve through their
    centroids (quantised to 2^bits levels per axis over the cells' bounding box; ties keep
    their order).  Cells close in space then get close indices: the neighbours a particle
    crosses into, and the cells that exchange particles, sit close in memory and are
    processed close in time, so their data stay in the L2.  The mesh, its boundary faces and
    the initial state are the same; only the numbering of the cells changes (and with it the
    random draws, which are keyed by cell index)."""
    m = w.mesh
    cnt = np.diff(m.cell_node_off)
    cid = np.repeat(np.arange(m.n_cells), cnt)
    cen = np.stack([np.bincount(cid, weights=m.xyz[m.cell_nodes, d], minlength=m.n_cells) for d in range(3)], 1)
    cen /= cnt[:, None]
    lo, hi = cen.min(0), cen.max(0)
    top = (1 << bits) - 1
    q = np.clip(((cen - lo) / np.maximum(hi - lo, 1e-300) * top).astype(np.int64), 0, top)
    key = np.zeros(m.n_cells, dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            key |= ((q[:, d] >> b) & 1) << (3 * b + d)
    order = np.argsort(key, kind="stable")
    lens = cnt[order]
    noff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx = np.repeat(m.cell_node_off[:-1][order] - noff[:-1], lens) + np.arange(int(noff[-1]))
    mesh = Mesh(m.xyz, m.cell_type[order], noff, m.cell_nodes[idx].astype(np.int64), m.bface_nodes, m.bface_bc,
                list(m.bcs))
    return Workload(w.name + " (Morton-numbered)", mesh, w.params, w.W0.reshape(-1, 5)[order].copy(), w.steps)


def sod(nx=50, ny=2, nz=2, n_ref=200, kn=1e-3, cfl=0.5, steps=40, seed=1, tets=False, gamma=5.0 / 3.0) -> Workload:
    """Shock tube in a square column (paper Sec. 4.1) at the hot-path size: [0,1]x[0,0.04]^2,
    rho = 1, p = 1 left of x = 0.5 and rho = 0.125, p = 0.1 right; all walls specular; monatomic
    unless gamma says otherwise (7/5: the paper's diatomic gas, K = 2)."""
    h = 1.0 / nx
    lo, hi = (0.0, 0.0, 0.0), (1.0, ny * h, nz * h)
    bcs = [BC(BC_SPECULAR)]
    side = {s: 0 for s in SIDES}
    mesh = (tet_box_mesh if tets else box_hex_mesh)((nx, ny, nz), lo, hi, side, bcs)
    xc = cell_centroids(mesh)
    left = xc[:, 0] < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    W0 = conservative(rho, np.zeros((mesh.n_cells, 3)), p / rho, K=internal_dof(gamma))
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=0.0, n_ref=n_ref, n_min=0, seed=seed,
                 gamma=gamma)
    return Workload("sod", mesh, prm, W0, steps)


def cavity(n=32, n_ref=400, kn=0.075, cfl=0.95, steps=2000, seed=1, Tw=1.0) -> Workload:
    """Lid-driven cubic cavity (paper Sec. 4.2) at the hot-path size: unit cube, n^3 boxes,
    diffuse isothermal walls at T_w, lid z = 1 moving at U = (0.16 sqrt(gamma T_w), 0, 0)."""
    lid = 0.16 * math.sqrt(5.0 / 3.0 * Tw)
    bcs = [BC(BC_DIFFUSE, Tw=Tw), BC(BC_DIFFUSE, Tw=Tw, Uw=(lid, 0.0, 0.0))]
    side = {s: 0 for s in SIDES}
    side["zhi"] = 1
    mesh = box_hex_mesh((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), side, bcs)
    nc = mesh.n_cells
    W0 = conservative(np.ones(nc), np.zeros((nc, 3)), np.ones(nc))
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=0.0, n_ref=n_ref, n_min=0, seed=seed)
    return Workload("cavity", mesh, prm, W0, steps)


def closed_box(n=(4, 3, 2), n_ref=50, kn=0.05, cfl=0.5, seed=7, bc=BC_SPECULAR, perturb=0.2, tets=False,
               jitter=0.0, gamma=5.0 / 3.0) -> Workload:
    """Small closed box with a seeded non-uniform initial state (for conservation checks)."""
    bcs = [BC(bc, Tw=1.0)]
    side = {s: 0 for s in SIDES}
    if tets:
        mesh = tet_box_mesh(n, (0.0, 0.0, 0.0), (1.0, 0.75, 0.5), side, bcs, jitter=jitter, seed=seed)
    else:
        mesh = box_hex_mesh(n, (0.0, 0.0, 0.0), (1.0, 0.75, 0.5), side, bcs)
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x57415445], dtype=np.uint64)))
    nc = mesh.n_cells
    rho = 1.0 + perturb * rng.uniform(-1, 1, nc)
    U = 0.3 * perturb * rng.uniform(-1, 1, (nc, 3))
    T = 1.0 + perturb * rng.uniform(-1, 1, nc)
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=0.0, n_ref=n_ref, n_min=0, seed=seed,
                 gamma=gamma)
    return Workload("closed_box", mesh, prm, conservative(rho, U, T, K=internal_dof(gamma)), 10)


def periodic_box(n=(4, 3, 3), n_ref=50, kn=0.05, cfl=0.5, seed=5, perturb=0.2, drift=(0.3, -0.2, 0.1),
                 tets=False) -> Workload:
    """Fully periodic box [0,1]x[0,0.75]x[0,0.5] (every side leads to the opposite one), with a
    seeded non-uniform initial state drifting at `drift` on average: no face is a wall, so
    mass, all three momenta and energy are conserved exactly by the scheme."""
    hi = (1.0, 0.75, 0.5)
    bcs = []
    side = {}
    for a, (lo_s, hi_s) in enumerate((("xlo", "xhi"), ("ylo", "yhi"), ("zlo", "zhi"))):
        sh = [0.0, 0.0, 0.0]
        sh[a] = hi[a]
        side[lo_s] = len(bcs)
        bcs.append(BC(BC_PERIODIC, shift=tuple(sh)))
        sh[a] = -hi[a]
        side[hi_s] = len(bcs)
        bcs.append(BC(BC_PERIODIC, shift=tuple(sh)))
    if tets:
        mesh = tet_box_mesh(n, (0.0, 0.0, 0.0), hi, side, bcs, jitter=0.0, seed=seed)
    else:
        mesh = box_hex_mesh(n, (0.0, 0.0, 0.0), hi, side, bcs)
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x50455249], dtype=np.uint64)))
    nc = mesh.n_cells
    rho = 1.0 + perturb * rng.uniform(-1, 1, nc)
    U = np.array(drift)[None, :] + 0.3 * perturb * rng.uniform(-1, 1, (nc, 3))
    T = 1.0 + perturb * rng.uniform(-1, 1, nc)
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=0.0, n_ref=n_ref, n_min=0, seed=seed)
    return Workload("periodic_box", mesh, prm, conservative(rho, U, T), 10)


def free_stream_box(n=(4, 3, 3), U=(0.8, 0.3, 0.0), T=1.0, rho=1.0, n_ref=100, kn=0.5, cfl=0.5, seed=11,
                    tets=False, jitter=0.0, perturb=0.0, walls=None, gamma=5.0 / 3.0) -> Workload:
    """Box of [0,1]x[0,0.75]x[0,0.5] with far-field faces on its sides, filled with the free stream
    it is bathed in (perturb > 0: a seeded non-uniform initial state instead).  walls: optional
    dict side name -> BC for sides that are not far field."""
    K = internal_dof(gamma)
    Winf = conservative(np.array([rho]), np.array([U]), np.array([T]), K=K)[0]
    bcs = [BC(BC_FARFIELD, Winf=tuple(float(v) for v in Winf))]
    side = {s_: 0 for s_ in SIDES}
    for nm, b in (walls or {}).items():
        side[nm] = len(bcs)
        bcs.append(b)
    gen = tet_box_mesh if tets else box_hex_mesh
    kw = dict(jitter=jitter, seed=seed) if tets else {}
    mesh = gen(n, (0.0, 0.0, 0.0), (1.0, 0.75, 0.5), side, bcs, **kw)
    nc_ = mesh.n_cells
    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        r = rho * (1.0 + perturb * rng.uniform(-1, 1, nc_))
        Uc = np.asarray(U, dtype=np.float64)[None, :] * (1.0 + perturb * rng.uniform(-1, 1, (nc_, 3)))
        Tc = T * (1.0 + perturb * rng.uniform(-1, 1, nc_))
        W0 = conservative(r, Uc, Tc, K=K)
    else:
        W0 = np.tile(Winf, (nc_, 1))
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=0.0, n_ref=n_ref, n_min=0, seed=seed,
                 gamma=gamma)
    return Workload("free_stream_box", mesh, prm, W0, 10)


# --------------------------------------------------------------------------------------
# flow past a cube (paper Sec. 4.3)
# --------------------------------------------------------------------------------------
def graded_axis(lo, hi, a, b, h0, growth, hmax):
    """Node coordinates on [lo, hi]: uniform spacing h0 on [a, b] (b - a a multiple of h0),
    spacing growing geometrically by `growth` up to hmax outside it; each outer run is scaled
    to end exactly on lo / hi."""
    n_in = int(round((b - a) / h0))
    core = np.linspace(a, b, n_in + 1)

    def run(length):
        if length <= 0:
            return np.zeros(0)
        steps, h, tot = [], h0, 0.0
        while tot < length - 1e-12:
            h = min(h * growth, hmax)
            steps.append(h)
            tot += h
        st = np.array(steps)
        if tot - length > 0.5 * st[-1] and len(st) > 1:
            st = st[:-1]
        return np.cumsum(st) * (length / st.sum())

    right = b + run(hi - b)
    left = a - run(a - lo)
    out = np.concatenate([left[::-1], core, right])
    out[0], out[-1] = lo, hi
    return out


def cube_mesh(lo=(-4.0, -5.0, -5.0), hi=(8.0, 5.0, 5.0), half=0.5, h0=0.05, growth=1.16, hmax=0.4, jitter=0.15,
              seed=1, bc_far=0, bc_wall=1, bcs=()) -> Mesh:
    """Graded box of hexahedra minus the cube [-half, half]^3 (whose faces lie on grid planes),
    each remaining hexahedron split into 6 Kuhn tetrahedra.  Interior nodes move uniformly within
    +-jitter h per axis (seeded, h the smaller adjacent spacing); nodes on the cube stay, nodes on
    the outer box move only within its planes.  Outer faces carry bc_far, cube faces bc_wall."""
    ax = [graded_axis(lo[d], hi[d], -half, half, h0, growth, hmax) for d in range(3)]
    n = [len(a) - 1 for a in ax]
    nx, ny, nz = n
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(), Z.transpose(2, 1, 0).ravel()], 1)
    idx = [np.arange(n[0] + 1), np.arange(n[1] + 1), np.arange(n[2] + 1)]
    I, J, K = np.meshgrid(*idx, indexing="ij")
    pos = [I.transpose(2, 1, 0).ravel(), J.transpose(2, 1, 0).ravel(), K.transpose(2, 1, 0).ravel()]
    # grid index range of the cube per axis
    cr = [(int(np.argmin(np.abs(ax[d] + half))), int(np.argmin(np.abs(ax[d] - half)))) for d in range(3)]
    on_cube = np.ones(xyz.shape[0], dtype=bool)
    for d in range(3):
        on_cube &= (pos[d] >= cr[d][0]) & (pos[d] <= cr[d][1])
    if jitter > 0.0:
        rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x43554245], dtype=np.uint64)))
        base = xyz.copy()
        for d in range(3):
            h = np.diff(ax[d])
            hloc = np.minimum(np.concatenate([[h[0]], h]), np.concatenate([h, [h[-1]]]))
            inner = (pos[d] > 0) & (pos[d] < n[d]) & ~on_cube
            dd = rng.uniform(-jitter, jitter, size=xyz.shape[0]) * hloc[pos[d]]
            xyz[:, d] = np.where(inner, base[:, d] + dd, base[:, d])

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i = i.transpose(2, 1, 0).ravel(); j = j.transpose(2, 1, 0).ravel(); k = k.transpose(2, 1, 0).ravel()
    inside = ((i >= cr[0][0]) & (i < cr[0][1]) & (j >= cr[1][0]) & (j < cr[1][1]) & (k >= cr[2][0]) & (k < cr[2][1]))
    keep = ~inside
    i, j, k = i[keep], j[keep], k[keep]
    tets = [np.stack([nid(i + a, j + b, k + c) for (a, b, c) in path], 1) for path in _KUHN]
    cn = np.stack(tets, 1).reshape(-1, 4).astype(np.int64)
    nc = cn.shape[0]
    side = {s_: bc_far for s_ in SIDES}
    bf, bt = _box_boundary(n, nid, side, tri_split=True)
    # cube surface: the faces of the removed block, split like the tetrahedra that touch them
    faces, tags = [], []
    (i0, i1), (j0, j1), (k0, k1) = cr

    def quad(p, q, r, s_):
        faces.append((p, q, r, -1)); faces.append((p, r, s_, -1)); tags.extend([bc_wall, bc_wall])

    for jj in range(j0, j1):
        for kk in range(k0, k1):
            for ii in (i0, i1):
                quad(nid(ii, jj, kk), nid(ii, jj + 1, kk), nid(ii, jj + 1, kk + 1), nid(ii, jj, kk + 1))
    for ii in range(i0, i1):
        for kk in range(k0, k1):
            for jj in (j0, j1):
                quad(nid(ii, jj, kk), nid(ii + 1, jj, kk), nid(ii + 1, jj, kk + 1), nid(ii, jj, kk + 1))
    for ii in range(i0, i1):
        for jj in range(j0, j1):
            for kk in (k0, k1):
                quad(nid(ii, jj, kk), nid(ii + 1, jj, kk), nid(ii + 1, jj + 1, kk), nid(ii, jj + 1, kk))
    bf = np.concatenate([bf, np.array(faces, dtype=np.int64).reshape(-1, 4)])
    bt = np.concatenate([bt, np.array(tags, dtype=np.int32)])
    return Mesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                cell_type=np.full(nc, CELL_TET, dtype=np.uint8),
                cell_node_off=np.arange(0, 4 * nc + 1, 4, dtype=np.int64),
                cell_nodes=cn.ravel(), bface_nodes=bf, bface_bc=bt, bcs=list(bcs))


def cube(mach=10.0, kn=0.1, n_ref=50, cfl=0.9, c2=10.0, Tw=1.0, h0=0.05, growth=1.16, hmax=0.4,
         lo=(-4.0, -5.0, -5.0), hi=(8.0, 5.0, 5.0), jitter=0.15, seed=1, steps=1200) -> Workload:
    """Mach 10 flow past a cube (paper Sec. 4.3) at the hot-path size: [-4,8]x[-5,5]^2 minus the
    unit cube, about 1.2e6 jittered tetrahedra; free stream rho = 1, T = 1, U = (Ma sqrt(5/3), 0, 0);
    far field on the outer box, diffuse cube walls at T_w; N_ref = N_min; impulsive start."""
    U = mach * math.sqrt(5.0 / 3.0)
    Winf = conservative(np.array([1.0]), np.array([[U, 0.0, 0.0]]), np.array([1.0]))[0]
    bcs = [BC(BC_FARFIELD, Winf=tuple(float(v) for v in Winf)), BC(BC_DIFFUSE, Tw=Tw)]
    mesh = cube_mesh(lo=lo, hi=hi, h0=h0, growth=growth, hmax=hmax, jitter=jitter, seed=seed, bcs=bcs)
    W0 = np.tile(Winf, (mesh.n_cells, 1))
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=c2, n_ref=n_ref, n_min=n_ref, seed=seed)
    return Workload("cube", mesh, prm, W0, steps)


def small_cube(**kw) -> Workload:
    """The cube case on a coarse mesh ([-1.5,2.5]x[-1.5,1.5]^2, h = 0.25 at the cube) for parity runs."""
    args = dict(h0=0.25, growth=1.5, hmax=0.6, lo=(-1.5, -1.5, -1.5), hi=(2.5, 1.5, 1.5), n_ref=30)
    args.update(kw)
    return cube(**args)


# --------------------------------------------------------------------------------------
# batches of independent instances
# --------------------------------------------------------------------------------------
def batched_specs(n_inst=64, cells=(2e3, 2e5), kn=(1e-4, 1.0), n_ref=(50, 500), seed=1):
    """The seeded draws of `batched`: per instance (kind, target cell count, Kn, N_ref), kind
    'sod' for even and 'cavity' for odd instances."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x42415443], dtype=np.uint64)))
    out = []
    for k in range(n_inst):
        nc = math.exp(rng.uniform(math.log(cells[0]), math.log(cells[1])))
        knk = math.exp(rng.uniform(math.log(kn[0]), math.log(kn[1])))
        nr = int(rng.integers(n_ref[0], n_ref[1] + 1))
        out.append(("sod" if k % 2 == 0 else "cavity", nc, knk, nr))
    return out


def batched_instance(spec, cfl=0.5, seed=1) -> Workload:
    """One instance of `batched` from its draws (kind, cells, Kn, N_ref)."""
    kind, nc, knk, nr = spec
    if kind == "sod":
        return sod(nx=max(2, math.ceil(nc / 4)), ny=2, nz=2, n_ref=nr, kn=knk, cfl=cfl, seed=seed)
    return cavity(n=max(2, int(round(nc ** (1.0 / 3.0)))), n_ref=nr, kn=knk, cfl=cfl, seed=seed)


def batched(n_inst=64, cells=(2e3, 2e5), kn=(1e-4, 1.0), n_ref=(50, 500), cfl=0.5, seed=1):
    """Independent instances alternating shock tube and cavity: cell counts log-uniform in
    `cells`, Knudsen numbers log-uniform in `kn`, N_ref uniform integers in `n_ref` (seeded).
    Tube: N_x x 2 x 2 boxes with N_x = ceil(cells / 4), h = 1 / N_x, the Sod data.  Cavity: n^3
    boxes with n = round(cells^(1/3)), the lid-driven cavity data.  All CFL `cfl`, N_min 0."""
    return [batched_instance(sp, cfl=cfl, seed=seed) for sp in batched_specs(n_inst, cells, kn, n_ref, seed)]


def small_batch(n_inst=6, seed=1):
    """A batch small enough for the oracle: 20 to 200 cells, 20 to 60 particles per cell."""
    return batched(n_inst=n_inst, cells=(20, 200), kn=(1e-3, 1.0), n_ref=(20, 60), seed=seed)


# --------------------------------------------------------------------------------------
# a body cut out of a graded box (the sphere-cone vehicle, paper Sec. 4.4)
# --------------------------------------------------------------------------------------
def carved_tet_mesh(ax, inside, jitter=0.15, seed=1, bc_far=0, bc_wall=1, bcs=()) -> Mesh:
    """Box of hexahedra on the node coordinates ax[0..2] with every hexahedron whose centroid
    satisfies inside(x, y, z) removed (a staircase body), the rest split into 6 Kuhn
    tetrahedra.  Faces between kept and removed hexahedra carry bc_wall, the outer box bc_far;
    boundary quads are split along their lowest-highest diagonal like the tetrahedra.
    Interior nodes move within +-jitter h per axis (seeded); nodes on the body stay, nodes on
    the outer box move only within its planes."""
    n = [len(a) - 1 for a in ax]
    nx, ny, nz = n
    cx = [0.5 * (a[1:] + a[:-1]) for a in ax]
    CX, CY, CZ = np.meshgrid(cx[0], cx[1], cx[2], indexing="ij")
    removed = inside(CX, CY, CZ)  # [nx, ny, nz]
    keep = ~removed

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    # nodes touching a removed hexahedron lie on the body: they do not move
    on_body = np.zeros((nx + 1, ny + 1, nz + 1), dtype=bool)
    ri, rj, rk = np.nonzero(removed)
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                on_body[ri + a, rj + b, rk + c] = True
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(), Z.transpose(2, 1, 0).ravel()], 1)
    I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    pos = [I.transpose(2, 1, 0).ravel(), J.transpose(2, 1, 0).ravel(), K.transpose(2, 1, 0).ravel()]
    fixed = on_body.transpose(2, 1, 0).ravel()
    if jitter > 0.0:
        rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x43415256], dtype=np.uint64)))
        base = xyz.copy()
        for d in range(3):
            h = np.diff(ax[d])
            hloc = np.minimum(np.concatenate([[h[0]], h]), np.concatenate([h, [h[-1]]]))
            inner = (pos[d] > 0) & (pos[d] < n[d]) & ~fixed
            dd = rng.uniform(-jitter, jitter, size=xyz.shape[0]) * hloc[pos[d]]
            xyz[:, d] = np.where(inner, base[:, d] + dd, base[:, d])
    # tetrahedra of the kept hexahedra, in (i fastest, then j, k) order
    ki, kj, kk = np.nonzero(keep.transpose(2, 1, 0))  # z, y, x order so that x runs fastest
    i, j, k = kk, kj, ki
    tets = [np.stack([nid(i + a, j + b, k + c) for (a, b, c) in path], 1) for path in _KUHN]
    cn = np.stack(tets, 1).reshape(-1, 4).astype(np.int64)
    nc = cn.shape[0]
    faces, tags = [], []

    def add_quads(d, p, q, r, tag):
        # quad on the node plane p of axis d spanning cells q, r of the two other axes
        e1, e2 = [a for a in range(3) if a != d]
        def node(pp, qq, rr):
            idx = [None, None, None]
            idx[d], idx[e1], idx[e2] = pp, qq, rr
            return nid(idx[0], idx[1], idx[2])
        n00, n10, n11, n01 = node(p, q, r), node(p, q + 1, r), node(p, q + 1, r + 1), node(p, q, r + 1)
        t1 = np.stack([n00, n10, n11, -np.ones_like(n00)], 1)
        t2 = np.stack([n00, n11, n01, -np.ones_like(n00)], 1)
        f = np.stack([t1, t2], 1).reshape(-1, 4)
        faces.append(f)
        tags.append(np.full(f.shape[0], tag, dtype=np.int32))

    for d in range(3):
        kd = np.moveaxis(keep, d, 0)  # [n_d, ., .]
        # outer planes
        for p, sl in ((0, 0), (n[d], n[d] - 1)):
            qq, rr = np.nonzero(kd[sl])
            add_quads(d, np.full(qq.shape, p), qq, rr, bc_far)
        # interior planes between cells a = p - 1 and b = p
        a, b = kd[:-1], kd[1:]
        pp, qq, rr = np.nonzero(a != b)
        add_quads(d, pp + 1, qq, rr, bc_wall)
    bf = np.concatenate(faces).astype(np.int64)
    bt = np.concatenate(tags)
    return Mesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                cell_type=np.full(nc, CELL_TET, dtype=np.uint8),
                cell_node_off=np.arange(0, 4 * nc + 1, 4, dtype=np.int64),
                cell_nodes=cn.ravel(), bface_nodes=bf, bface_bc=bt, bcs=list(bcs))


def sphere_cone_inside(rn=0.3, half_angle_deg=20.0, length=2.0, nose=0.0):
    """Inside test of a sphere-cone along +x: spherical nose of radius rn with its tip at
    x = nose, a cone of the given half angle tangent to it, a flat base at x = nose + length."""
    th = math.radians(half_angle_deg)
    xt = nose + rn * (1.0 - math.sin(th))
    rt = rn * math.cos(th)

    def inside(x, y, z):
        r = np.sqrt(y * y + z * z)
        xs = x - nose
        sph = (xs - rn) ** 2 + r * r <= rn * rn
        cone = (x >= xt) & (x <= nose + length) & (r <= rt + (x - xt) * math.tan(th))
        return (xs >= 0.0) & ((x < xt) & sph | cone)

    return inside


def vehicle(mach=15.0, kn=1e-3, n_ref=50, cfl=0.95, c2=10.0, h0=0.0435, growth=1.15, hmax=0.3,
            lo=(-2.0, -3.0, -3.0), hi=(6.0, 3.0, 3.0), refine=((-0.2, 2.2), (-1.1, 1.1), (-1.1, 1.1)),
            jitter=0.15, seed=1, steps=1200) -> Workload:
    """Mach 15 flow past a blunt sphere-cone (nose radius 0.3, half angle 20 degrees, length 2,
    axis along x) in [-2,6]x[-3,3]^2: graded hexahedra (h0 in the refined box around the body,
    growing to hmax), the body's hexahedra removed, Kuhn tetrahedra with jitter; diffuse wall at
    T_w = 0.2 T_0 (T_0 = 1 + (gamma - 1)/2 Ma^2 the stagnation temperature), far field outside;
    free stream rho = 1, T = 1; N_ref = N_min."""
    ax = []
    for d in range(3):
        a, b = refine[d]
        nce = max(1, int(round((b - a) / h0)))
        b = a + nce * h0
        ax.append(graded_axis(lo[d], hi[d], a, b, h0, growth, hmax))
    U = mach * math.sqrt(5.0 / 3.0)
    T0 = 1.0 + (5.0 / 3.0 - 1.0) / 2.0 * mach * mach
    Winf = conservative(np.array([1.0]), np.array([[U, 0.0, 0.0]]), np.array([1.0]))[0]
    bcs = [BC(BC_FARFIELD, Winf=tuple(float(v) for v in Winf)), BC(BC_DIFFUSE, Tw=0.2 * T0)]
    mesh = carved_tet_mesh(ax, sphere_cone_inside(), jitter=jitter, seed=seed, bcs=bcs)
    W0 = np.tile(Winf, (mesh.n_cells, 1))
    prm = Params(mu_ref=mu_ref_from_kn(kn, 0.81), omega=0.81, cfl=cfl, c2=c2, n_ref=n_ref, n_min=n_ref, seed=seed)
    return Workload("vehicle", mesh, prm, W0, steps)


def small_vehicle(**kw) -> Workload:
    """The vehicle case on a coarse mesh for parity runs."""
    args = dict(h0=0.2, growth=1.5, hmax=0.8, lo=(-1.0, -1.6, -1.6), hi=(3.0, 1.6, 1.6),
                refine=((-0.2, 2.2), (-1.0, 1.0), (-1.0, 1.0)), n_ref=30)
    args.update(kw)
    return vehicle(**args)
