// Internal declarations shared by the preprocessor and the device library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gks.h"

namespace gks {

// Preprocessed mesh in the library's internal (Morton) cell order.
struct HostMesh {
    int64_t n = 0;   // cells
    int64_t nf = 0;  // faces
    double L[3] = {1, 1, 1};
    int64_t n_grown = 0;
    std::vector<int64_t> perm;  // internal -> caller index
    // cells
    std::vector<int8_t> type;
    std::vector<double> vol, xc, m2, hcfl;  // m2: [n][6] xx xy xz yy yz zz (centred means)
    // stencil: members of cell i are st_idx[st_ptr[i] .. st_ptr[i+1]); per member a
    // sub-stencil membership mask, a row of the quadratic pseudo-inverse (9, zero for
    // members only a sub-stencil uses) and its centroid offset scaled by h = |Omega_i|^(1/3)
    // (3); per cell the inverses G_m^{-1}/h of the sub-stencil normal matrices
    // (6 unique entries xx xy xz yy yz zz for each of 8 slots)
    std::vector<int32_t> st_ptr, st_idx;
    std::vector<uint8_t> st_mask;
    std::vector<uint8_t> st_flip;  // per member: bit d set if the member is mirrored across a wall on axis d
    std::vector<double> pinv, dsc, ginv;
    // faces
    std::vector<int32_t> owner, nbr;  // nbr = -1 - axis for a reflective wall on that axis
    std::vector<double> fgeo;  // [9][4 nf]: d_owner(3), d_neighbour(3), weighted vector area(3) per Gauss point
    // cell -> faces in F_p order, encoded 2 * face + side (side 1: the cell is the neighbour)
    std::vector<int32_t> cf_ptr, cf_idx;
    // transposed stencil CSR: entries e with st_idx[e] == i are tr_idx[tr_ptr[i] .. tr_ptr[i+1])
    std::vector<int32_t> tr_ptr, tr_idx;
};

gks_status preprocess(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types,
                      const int64_t *cells, const double *box, int periodic, int min_big, HostMesh &H);

gks_status fail(gks_status s, const std::string &msg);

}  // namespace gks

struct gks_host_mesh {
    gks::HostMesh h;
};
