// Host-side mesh preparation (see mesh_prep.hpp).
//
// Cells are the control volumes Omega_i of the finite-volume form (paper, Eq. FVmacroEq);
// faces S_ij carry the unit normal n_ij from cell i to cell j and the area |S_ij|.  Every
// interior face is owned by the first cell (lowest index) that lists it; the neighbour
// uses exactly the reversed plane of the owner so that both cells classify a point on the
// face the same way during particle tracking.
#include "mesh_prep.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>

namespace ugkwp {
namespace {

// local faces of an axis-aligned box in VTK node order: -x, +x, -y, +y, -z, +z
const int kHexFace[6][4] = {{0, 3, 7, 4}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};
// local faces of a tetrahedron: face i lies opposite node i
const int kTetFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

using Key = std::array<int64_t, 4>;

struct KeyHash {
    size_t operator()(const Key &k) const {
        uint64_t h = 0x9E3779B97F4A7C15ULL;
        for (int64_t v : k) {
            h ^= (uint64_t)v + 0x9E3779B97F4A7C15ULL + (h << 6) + (h >> 2);
        }
        return (size_t)h;
    }
};

Key make_key(const int64_t *ids, int n) {
    Key k{-1, -1, -1, -1};
    for (int i = 0; i < n; ++i) k[i] = ids[i];
    std::sort(k.begin(), k.begin() + n);
    return k;
}

}  // namespace

int32_t prepare_mesh(const ugkwp_mesh &m, HostMesh &H, std::string &err) {
    if (m.n_cells <= 0 || m.n_nodes <= 0 || !m.xyz || !m.cell_type || !m.cell_node_off || !m.cell_nodes) {
        err = "mesh: empty or missing arrays";
        return UGKWP_E_ARG;
    }
    if (m.n_cells >= (int64_t(1) << 24)) {
        err = "mesh: at most 2^24 - 1 cells (particle ids hold the birth cell in 24 bits)";
        return UGKWP_E_ARG;
    }
    if (m.n_bfaces < 0 || (m.n_bfaces > 0 && (!m.bface_nodes || !m.bface_bc)) || m.n_bc < 0 ||
        (m.n_bc > 0 && !m.bc)) {
        err = "mesh: bad boundary arrays";
        return UGKWP_E_ARG;
    }
    for (int32_t b = 0; b < m.n_bc; ++b) {
        const ugkwp_bc &bc = m.bc[b];
        if (bc.type < UGKWP_BC_SPECULAR || bc.type > UGKWP_BC_PERIODIC) {
            err = "mesh: unknown boundary type";
            return UGKWP_E_ARG;
        }
        if (bc.type == UGKWP_BC_PERIODIC &&
            !(std::isfinite(bc.shift[0]) && std::isfinite(bc.shift[1]) && std::isfinite(bc.shift[2]) &&
              std::fabs(bc.shift[0]) + std::fabs(bc.shift[1]) + std::fabs(bc.shift[2]) > 0.0)) {
            err = "mesh: a periodic boundary needs a finite, nonzero shift";
            return UGKWP_E_ARG;
        }
        if (bc.type == UGKWP_BC_DIFFUSE && !(bc.T_w > 0.0)) {
            err = "mesh: diffuse wall needs T_w > 0";
            return UGKWP_E_ARG;
        }
        if (bc.type == UGKWP_BC_FARFIELD) {
            const double *w = bc.W_inf;
            double ke = 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0];
            if (!(w[0] > 0.0) || !(w[4] - ke > 0.0)) {
                err = "mesh: far-field state must have rho > 0 and T > 0";
                return UGKWP_E_ARG;
            }
        }
    }
    const int32_t nc = (int32_t)m.n_cells;
    H.nc = nc;
    H.vol.assign(nc, 0.0);
    H.lfx.assign((size_t)nc * kMaxFaces * 3, 0.0);
    H.xc.assign(3 * (size_t)nc, 0.0);
    H.dS.assign(3 * (size_t)nc, 0.0);
    H.nfc.assign(nc, 0);
    H.ctype.assign(nc, 0);
    H.plane.assign((size_t)nc * kMaxFaces * 4, 0.0);
    H.nb.assign((size_t)nc * kMaxFaces, -1);
    H.nblf.assign((size_t)nc * kMaxFaces, -1);
    H.cface.assign((size_t)nc * kMaxFaces, 0);
    H.orig.assign(3 * (size_t)nc, 0.0);
    H.box.assign(6 * (size_t)nc, 0.0);
    H.edge.assign(9 * (size_t)nc, 0.0);
    H.bcs.assign(m.bc, m.bc + m.n_bc);
    std::vector<double> larea((size_t)nc * kMaxFaces, 0.0);

    auto node = [&](int64_t i) { return m.xyz + 3 * i; };

    for (int32_t c = 0; c < nc; ++c) {
        int64_t o0 = m.cell_node_off[c], o1 = m.cell_node_off[c + 1];
        if (o1 - o0 != m.cell_type[c] || (m.cell_type[c] != 4 && m.cell_type[c] != 8)) {
            err = "mesh: cell " + std::to_string(c) + " is neither a 4-node tetrahedron nor an 8-node box";
            return UGKWP_E_MESH;
        }
        const int64_t *cn = m.cell_nodes + o0;
        for (int i = 0; i < m.cell_type[c]; ++i)
            if (cn[i] < 0 || cn[i] >= m.n_nodes) {
                err = "mesh: node index out of range in cell " + std::to_string(c);
                return UGKWP_E_MESH;
            }
        double *P = &H.plane[(size_t)c * kMaxFaces * 4];
        if (m.cell_type[c] == 8) {
            H.ctype[c] = 8;
            H.nfc[c] = 6;
            const double *a = node(cn[0]), *g = node(cn[6]);
            double lo[3] = {a[0], a[1], a[2]}, hi[3] = {g[0], g[1], g[2]};
            for (int i = 0; i < 8; ++i) {
                const double *p = node(cn[i]);
                bool bx = (i == 1 || i == 2 || i == 5 || i == 6), by = (i == 2 || i == 3 || i == 6 || i == 7),
                     bz = (i >= 4);
                if (p[0] != (bx ? hi[0] : lo[0]) || p[1] != (by ? hi[1] : lo[1]) || p[2] != (bz ? hi[2] : lo[2])) {
                    err = "mesh: hex " + std::to_string(c) + " is not an axis-aligned box in VTK node order";
                    return UGKWP_E_MESH;
                }
            }
            double ext[3];
            for (int d = 0; d < 3; ++d) {
                ext[d] = hi[d] - lo[d];
                if (!(ext[d] > 0.0)) {
                    err = "mesh: degenerate hex " + std::to_string(c);
                    return UGKWP_E_MESH;
                }
                H.xc[3 * c + d] = 0.5 * (lo[d] + hi[d]);
                H.orig[3 * c + d] = lo[d];
                H.box[6 * c + d] = lo[d];
                H.box[6 * c + 3 + d] = hi[d];
                H.edge[9 * c + 4 * d] = ext[d];
            }
            H.vol[c] = ext[0] * ext[1] * ext[2];
            double area[3] = {ext[1] * ext[2], ext[0] * ext[2], ext[0] * ext[1]};
            for (int lf = 0; lf < 6; ++lf) {
                int ax = lf >> 1;
                bool up = lf & 1;
                P[4 * lf + 0] = P[4 * lf + 1] = P[4 * lf + 2] = 0.0;
                P[4 * lf + ax] = up ? 1.0 : -1.0;
                P[4 * lf + 3] = up ? hi[ax] : -lo[ax];
                larea[(size_t)c * kMaxFaces + lf] = area[ax];
                for (int d = 0; d < 3; ++d)
                    H.lfx[((size_t)c * kMaxFaces + lf) * 3 + d] = d == ax ? (up ? hi[ax] : lo[ax]) : H.xc[3 * c + d];
            }
        } else {
            H.ctype[c] = 4;
            H.nfc[c] = 4;
            const double *v[4] = {node(cn[0]), node(cn[1]), node(cn[2]), node(cn[3])};
            double e[3][3];
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 3; ++d) e[k][d] = v[k + 1][d] - v[0][d];
            double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                         e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                         e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
            if (!(std::fabs(det) > 0.0)) {
                err = "mesh: degenerate tetrahedron " + std::to_string(c);
                return UGKWP_E_MESH;
            }
            H.vol[c] = std::fabs(det) / 6.0;
            for (int d = 0; d < 3; ++d) {
                H.xc[3 * c + d] = 0.25 * (v[0][d] + v[1][d] + v[2][d] + v[3][d]);
                H.orig[3 * c + d] = v[0][d];
                for (int k = 0; k < 3; ++k) H.edge[9 * c + 3 * k + d] = e[k][d];
            }
            for (int lf = 0; lf < 4; ++lf) {
                const double *p = v[kTetFace[lf][0]], *q = v[kTetFace[lf][1]], *r = v[kTetFace[lf][2]], *o = v[lf];
                double a[3], b[3], N[3];
                for (int d = 0; d < 3; ++d) {
                    a[d] = q[d] - p[d];
                    b[d] = r[d] - p[d];
                }
                N[0] = a[1] * b[2] - a[2] * b[1];
                N[1] = a[2] * b[0] - a[0] * b[2];
                N[2] = a[0] * b[1] - a[1] * b[0];
                double side = N[0] * (o[0] - p[0]) + N[1] * (o[1] - p[1]) + N[2] * (o[2] - p[2]);
                if (side > 0.0) {
                    N[0] = -N[0];
                    N[1] = -N[1];
                    N[2] = -N[2];
                }
                double len = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
                double cen[3];
                for (int d = 0; d < 3; ++d) {
                    P[4 * lf + d] = N[d] / len;
                    cen[d] = (p[d] + q[d] + r[d]) / 3.0;
                }
                P[4 * lf + 3] = P[4 * lf] * cen[0] + P[4 * lf + 1] * cen[1] + P[4 * lf + 2] * cen[2];
                larea[(size_t)c * kMaxFaces + lf] = 0.5 * len;
                for (int d = 0; d < 3; ++d) H.lfx[((size_t)c * kMaxFaces + lf) * 3 + d] = cen[d];
            }
        }
    }

    // boundary faces by sorted node key
    struct BFace {
        int32_t bc;
        int64_t b;
    };
    std::unordered_map<Key, BFace, KeyHash> bmap;
    bmap.reserve((size_t)m.n_bfaces * 2 + 1);
    for (int64_t b = 0; b < m.n_bfaces; ++b) {
        const int64_t *bn = m.bface_nodes + 4 * b;
        int nn = bn[3] < 0 ? 3 : 4;
        if (m.bface_bc[b] < 0 || m.bface_bc[b] >= m.n_bc) {
            err = "mesh: boundary face " + std::to_string(b) + " has no valid tag";
            return UGKWP_E_MESH;
        }
        if (!bmap.emplace(make_key(bn, nn), BFace{m.bface_bc[b], b}).second) {
            err = "mesh: boundary face listed twice";
            return UGKWP_E_MESH;
        }
    }

    // interior faces: first occurrence owns the face
    struct Open {
        int32_t cell;
        int32_t lf;
    };
    std::unordered_map<Key, Open, KeyHash> open;
    open.reserve((size_t)nc * 3);
    std::vector<int32_t> fown, fnb;
    std::vector<double> fn, farea;
    int64_t matched_b = 0;
    for (int32_t c = 0; c < nc; ++c) {
        const int64_t *cn = m.cell_nodes + m.cell_node_off[c];
        for (int lf = 0; lf < H.nfc[c]; ++lf) {
            int64_t ids[4];
            int nn = H.ctype[c] == 8 ? 4 : 3;
            for (int i = 0; i < nn; ++i) ids[i] = H.ctype[c] == 8 ? cn[kHexFace[lf][i]] : cn[kTetFace[lf][i]];
            Key k = make_key(ids, nn);
            auto it = open.find(k);
            if (it == open.end()) {
                open.emplace(k, Open{c, lf});
                continue;
            }
            Open own = it->second;
            open.erase(it);
            int32_t f = (int32_t)fown.size();
            size_t so = (size_t)own.cell * kMaxFaces + own.lf, sn = (size_t)c * kMaxFaces + lf;
            fown.push_back(own.cell);
            fnb.push_back(c);
            for (int d = 0; d < 3; ++d) fn.push_back(H.plane[4 * so + d]);
            for (int d = 0; d < 3; ++d) H.fx.push_back(H.lfx[so * 3 + d]);
            farea.push_back(larea[so]);
            H.nb[so] = c;
            H.nblf[so] = lf;
            H.nb[sn] = own.cell;
            H.nblf[sn] = own.lf;
            H.cface[so] = f + 1;
            H.cface[sn] = -(f + 1);
            for (int d = 0; d < 4; ++d) H.plane[4 * sn + d] = -H.plane[4 * so + d];
        }
    }
    // what is left open must be a tagged boundary face; visit in cell order for a stable numbering
    H.bf_lf.assign((size_t)m.n_bfaces, 0);
    std::vector<std::pair<int32_t, int32_t>> rest;
    rest.reserve(open.size());
    for (auto &kv : open) rest.emplace_back(kv.second.cell, kv.second.lf);
    std::sort(rest.begin(), rest.end());
    // periodic faces are paired after the others: (cell, local face, bc)
    struct Per {
        int32_t c, lf, bc;
    };
    std::vector<Per> per;
    for (auto &cl : rest) {
        int32_t c = cl.first, lf = cl.second;
        const int64_t *cn = m.cell_nodes + m.cell_node_off[c];
        int64_t ids[4];
        int nn = H.ctype[c] == 8 ? 4 : 3;
        for (int i = 0; i < nn; ++i) ids[i] = H.ctype[c] == 8 ? cn[kHexFace[lf][i]] : cn[kTetFace[lf][i]];
        auto it = bmap.find(make_key(ids, nn));
        if (it == bmap.end()) {
            err = "mesh: face " + std::to_string(lf) + " of cell " + std::to_string(c) +
                  " is neither shared nor a tagged boundary face";
            return UGKWP_E_MESH;
        }
        ++matched_b;
        size_t so = (size_t)c * kMaxFaces + lf;
        int32_t f = (int32_t)fown.size();
        const int32_t bci = it->second.bc;
        const int64_t b = it->second.b;
        if (m.bc[bci].type == UGKWP_BC_PERIODIC) {
            H.bf_lf[(size_t)b] = (uint8_t)lf;
            per.push_back(Per{c, lf, bci});
            continue;
        }
        fown.push_back(c);
        fnb.push_back(-1 - bci);
        for (int d = 0; d < 3; ++d) fn.push_back(H.plane[4 * so + d]);
        for (int d = 0; d < 3; ++d) H.fx.push_back(H.lfx[so * 3 + d]);
        farea.push_back(larea[so]);
        H.bf_lf[(size_t)b] = (uint8_t)lf;
        if (m.bc[bci].type == UGKWP_BC_FARFIELD) {
            if (b >= (int64_t(1) << 24)) {
                err = "mesh: far-field faces need an input index below 2^24 (particle ids hold it in 24 bits)";
                return UGKWP_E_MESH;
            }
            // the entry face as listed: corner p0 and the edges to p1 and to p2 (triangle) or p3
            // (parallelogram p0 p1 p2 p3), area from their cross product
            const int64_t *bn = m.bface_nodes + 4 * b;
            const int tri = bn[3] < 0;
            const double *p0 = m.xyz + 3 * bn[0], *p1 = m.xyz + 3 * bn[1], *pq = m.xyz + 3 * (tri ? bn[2] : bn[3]);
            double g[10], e1[3], e2[3];
            for (int d = 0; d < 3; ++d) {
                g[d] = p0[d];
                e1[d] = p1[d] - p0[d];
                e2[d] = pq[d] - p0[d];
                g[3 + d] = e1[d];
                g[6 + d] = e2[d];
            }
            const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                         cz = e1[0] * e2[1] - e1[1] * e2[0];
            const double cr = std::sqrt(cx * cx + cy * cy + cz * cz);
            g[9] = tri ? 0.5 * cr : cr;
            H.ff_cell.push_back(c);
            H.ff_lf.push_back(lf);
            H.ff_bf.push_back((int32_t)b);
            H.ff_bc.push_back(bci);
            H.ff_tri.push_back(tri);
            H.ff_geo.insert(H.ff_geo.end(), g, g + 10);
        }
        H.nb[so] = -1 - bci;
        H.nblf[so] = -1;
        H.cface[so] = f + 1;
    }
    if (matched_b != m.n_bfaces) {
        err = "mesh: a boundary face does not belong to any cell";
        return UGKWP_E_MESH;
    }
    // periodic pairs: face A (condition b) leads to the periodic face B whose centre is A's
    // centre plus b's shift and whose condition has the opposite shift.  Centres are matched
    // through a hash of their coordinates quantised at 1e-9 of the domain's extent (the 27
    // neighbouring quanta are searched, so a rounding split cannot hide a partner).  The
    // pair becomes one interior face owned by the earlier of the two in (cell, face) order.
    if (!per.empty()) {
        double ext = 0.0;
        for (int64_t i = 0; i < 3 * m.n_nodes; ++i) ext = std::max(ext, std::fabs(m.xyz[i]));
        const double q = 1e-9 * (ext > 0.0 ? ext : 1.0);
        auto qkey = [q](const double *x, int dx, int dy, int dz) {
            const int64_t a = (int64_t)std::llround(x[0] / q) + dx, b = (int64_t)std::llround(x[1] / q) + dy,
                          c = (int64_t)std::llround(x[2] / q) + dz;
            return std::array<int64_t, 3>{a, b, c};
        };
        struct QHash {
            size_t operator()(const std::array<int64_t, 3> &k) const {
                return (size_t)(k[0] * 0x9E3779B97F4A7C15ULL ^ k[1] * 0xC2B2AE3D27D4EB4FULL ^ k[2] * 0x165667B19E3779F9ULL);
            }
        };
        std::unordered_map<std::array<int64_t, 3>, std::vector<int32_t>, QHash> at;
        for (int32_t i = 0; i < (int32_t)per.size(); ++i)
            at[qkey(&H.lfx[((size_t)per[i].c * kMaxFaces + per[i].lf) * 3], 0, 0, 0)].push_back(i);
        std::vector<char> done(per.size(), 0);
        for (int32_t i = 0; i < (int32_t)per.size(); ++i) {
            if (done[i]) continue;
            const Per &A = per[i];
            const double *s = m.bc[A.bc].shift;
            const double *xa = &H.lfx[((size_t)A.c * kMaxFaces + A.lf) * 3];
            const double t[3] = {xa[0] + s[0], xa[1] + s[1], xa[2] + s[2]};
            int32_t jb = -1;
            for (int dx = -1; dx <= 1 && jb < 0; ++dx)
                for (int dy = -1; dy <= 1 && jb < 0; ++dy)
                    for (int dz = -1; dz <= 1 && jb < 0; ++dz) {
                        auto hit = at.find(qkey(t, dx, dy, dz));
                        if (hit == at.end()) continue;
                        for (int32_t j : hit->second) {
                            if (j == i || done[j]) continue;
                            const double *sb = m.bc[per[j].bc].shift;
                            const double *xb = &H.lfx[((size_t)per[j].c * kMaxFaces + per[j].lf) * 3];
                            if (std::fabs(sb[0] + s[0]) + std::fabs(sb[1] + s[1]) + std::fabs(sb[2] + s[2]) > 1e-12 * ext)
                                continue;
                            if (std::fabs(xb[0] - t[0]) + std::fabs(xb[1] - t[1]) + std::fabs(xb[2] - t[2]) > 3e-9 * ext)
                                continue;
                            jb = j;
                            break;
                        }
                    }
            if (jb < 0) {
                err = "mesh: periodic face " + std::to_string(A.lf) + " of cell " + std::to_string(A.c) +
                      " has no partner at its centre plus the shift";
                return UGKWP_E_MESH;
            }
            const Per &B = per[jb];
            done[i] = done[jb] = 1;
            const size_t sa = (size_t)A.c * kMaxFaces + A.lf, sb = (size_t)B.c * kMaxFaces + B.lf;
            const int32_t f = (int32_t)fown.size();
            fown.push_back(A.c);
            fnb.push_back(B.c);
            for (int d = 0; d < 3; ++d) fn.push_back(H.plane[4 * sa + d]);
            for (int d = 0; d < 3; ++d) H.fx.push_back(xa[d]);
            farea.push_back(larea[sa]);
            H.nb[sa] = B.c;
            H.nblf[sa] = B.lf + kPeriodicEntry * (A.bc + 1);
            H.nb[sb] = A.c;
            H.nblf[sb] = A.lf + kPeriodicEntry * (B.bc + 1);
            H.cface[sa] = f + 1;
            H.cface[sb] = -(f + 1);
            ++H.nper;
        }
    }
    H.nff = (int32_t)H.ff_cell.size();
    H.nf = (int32_t)fown.size();
    H.fown.swap(fown);
    H.fnb.swap(fnb);
    H.fn.swap(fn);
    H.farea.swap(farea);
    // projections of the control volume: Delta S^d = 1/2 sum_faces |S n_d|
    for (int32_t c = 0; c < nc; ++c)
        for (int lf = 0; lf < H.nfc[c]; ++lf) {
            size_t s = (size_t)c * kMaxFaces + lf;
            for (int d = 0; d < 3; ++d) H.dS[3 * c + d] += 0.5 * std::fabs(larea[s] * H.plane[4 * s + d]);
        }
    return UGKWP_OK;
}


int32_t concat_meshes(const std::vector<HostMesh> &parts, HostMesh &out, std::vector<InstRange> &ranges,
                      std::string &err) {
    int64_t nc = 0, nf = 0, nff = 0, nbf = 0, nbc = 0;
    for (const HostMesh &h : parts) {
        nc += h.nc;
        nf += h.nf;
        nff += h.nff;
        nbf += (int64_t)h.bf_lf.size();
        nbc += (int64_t)h.bcs.size();
    }
    if (nc > 2147483647LL - 1 || nf > 2147483647LL - 1 || nbf > 2147483647LL - 1) {
        err = "batch: more than 2^31 - 1 cells, faces or boundary faces in total";
        return UGKWP_E_ARG;
    }
    // a periodic slot's entry, lf + kPeriodicEntry (bc + 1), must fit in 32 bits
    if (nbc >= (int64_t(1) << 27)) {
        err = "batch: 2^27 or more boundary conditions in total";
        return UGKWP_E_ARG;
    }
    HostMesh o;
    o.nc = (int32_t)nc;
    o.nf = (int32_t)nf;
    o.nff = (int32_t)nff;
    ranges.clear();
    int32_t coff = 0, foff = 0, boff = 0, ffoff = 0;
    int64_t bfoff = 0;
    auto app = [](auto &dst, const auto &src) { dst.insert(dst.end(), src.begin(), src.end()); };
    for (const HostMesh &h : parts) {
        ranges.push_back(InstRange{coff, coff + h.nc, ffoff, ffoff + h.nff, bfoff});
        app(o.vol, h.vol);
        app(o.xc, h.xc);
        app(o.dS, h.dS);
        app(o.nfc, h.nfc);
        app(o.ctype, h.ctype);
        app(o.plane, h.plane);
        app(o.box, h.box);
        app(o.orig, h.orig);
        app(o.edge, h.edge);
        // a periodic entry carries its boundary condition's index, offset like the others
        for (int32_t v : h.nblf)
            o.nblf.push_back(v >= kPeriodicEntry ? (v % kPeriodicEntry) + kPeriodicEntry * (v / kPeriodicEntry + boff)
                                                 : v);
        o.nper += h.nper;
        for (int32_t v : h.nb) o.nb.push_back(v >= 0 ? v + coff : -1 - (-1 - v + boff));
        for (int32_t v : h.cface) o.cface.push_back(v > 0 ? v + foff : (v < 0 ? v - foff : 0));
        for (int32_t v : h.fown) o.fown.push_back(v + coff);
        for (int32_t v : h.fnb) o.fnb.push_back(v >= 0 ? v + coff : -1 - (-1 - v + boff));
        app(o.fn, h.fn);
        app(o.farea, h.farea);
        app(o.lfx, h.lfx);
        app(o.fx, h.fx);
        app(o.bcs, h.bcs);
        for (int32_t v : h.ff_cell) o.ff_cell.push_back(v + coff);
        app(o.ff_lf, h.ff_lf);
        app(o.ff_bf, h.ff_bf);
        for (int32_t v : h.ff_bc) o.ff_bc.push_back(v + boff);
        app(o.ff_tri, h.ff_tri);
        app(o.ff_geo, h.ff_geo);
        app(o.bf_lf, h.bf_lf);
        coff += h.nc;
        foff += h.nf;
        boff += (int32_t)h.bcs.size();
        ffoff += h.nff;
        bfoff += (int64_t)h.bf_lf.size();
    }
    out = std::move(o);
    return UGKWP_OK;
}

}  // namespace ugkwp
