// Host-side mesh preparation for the UGKWP library: validation, face matching and the
// geometry the kernels read (cell volumes and centroids, outward face planes, face normals
// and areas, the projections Delta S of the time-step formula, sampling frames).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "ugkwp.h"
#include "device_common.hpp"  // kPeriodicEntry

namespace ugkwp {

constexpr int kMaxFaces = 6;  // faces per cell slot (box hex); tetrahedra use 4

struct HostMesh {
    int32_t nc = 0, nf = 0;
    std::vector<double> vol;     // [nc]
    std::vector<double> xc;      // [nc][3]
    std::vector<double> dS;      // [nc][3]
    std::vector<uint8_t> nfc;    // faces per cell (4 or 6)
    std::vector<uint8_t> ctype;  // 4 or 8
    std::vector<double> plane;   // [nc][6][4]: outward unit normal n and d with n.x = d on the face
    std::vector<int32_t> nb;     // [nc][6]: neighbour cell, or -1 - bc index at a boundary
    std::vector<int32_t> nblf;   // [nc][6]: the face's local index in the neighbour (-1 at a boundary)
    std::vector<int32_t> cface;  // [nc][6]: global face f as f + 1 (owner) or -(f + 1) (neighbour)
    std::vector<double> box;     // [nc][6]  lo[3], hi[3] of a box hex (the exact node coordinates)
    std::vector<double> orig;    // [nc][3]  sampling frame: x = orig + s e1 + t e2 + w e3
    std::vector<double> edge;    // [nc][3][3]
    std::vector<int32_t> fown;   // [nf]
    std::vector<int32_t> fnb;    // [nf]: neighbour cell, or -1 - bc index
    std::vector<double> fn;      // [nf][3]  unit normal, owner -> neighbour (out of the domain at walls)
    std::vector<double> farea;   // [nf]
    std::vector<double> lfx;     // [nc][6][3] centre of each local face
    std::vector<double> fx;      // [nf][3] face centre (the owner's local face)
    std::vector<ugkwp_bc> bcs;
    // far-field faces, in (cell, local face) order: where free-stream particles enter
    int32_t nff = 0;
    std::vector<int32_t> ff_cell, ff_lf, ff_bf, ff_bc, ff_tri;  // [nff]; ff_bf: input boundary-face index
    std::vector<double> ff_geo;  // [nff][10]: corner p0, edges p1 - p0 and (p2 or p3) - p0, area
    std::vector<uint8_t> bf_lf;  // [n_bfaces]: local face of an input boundary face in its cell
    int32_t nper = 0;            // periodic face pairs (each one interior face)
};


// Returns UGKWP_OK or UGKWP_E_ARG / UGKWP_E_MESH with a message in *err.
int32_t prepare_mesh(const ugkwp_mesh &m, HostMesh &out, std::string &err);

// Where instance k of a batch sits in the concatenated mesh.
struct InstRange {
    int32_t cell0, cell1;  // cells
    int32_t ff0, ff1;      // far-field faces
    int64_t bf0;           // input boundary faces (index into bf_lf)
};

// Concatenate the prepared meshes of a batch into one mesh of disconnected parts: cell,
// face and boundary-condition indices are offset; far-field faces keep the instance-local
// index of their input boundary face.  Fails with UGKWP_E_ARG if the total exceeds 32-bit
// indices.
int32_t concat_meshes(const std::vector<HostMesh> &parts, HostMesh &out, std::vector<InstRange> &ranges,
                      std::string &err);

}  // namespace ugkwp
