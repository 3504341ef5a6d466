// Host preprocessor of the gas-kinetic solver: connectivity, geometry,
// stencils, FP64 least-squares pseudo-inverses and the device layouts.
//
// Follows Section 2 of Yang, Pan & Xu (arXiv 2203.09047):
//   - face labels F_p of the four cell types (the prism's third face is read
//     as p1 p2 p5 p4; the printed p6 cannot close the cell);
//   - tetrahedron, pyramid and prism as degenerate hexahedra, each mapped by
//     the trilinear interpolation of Eq. trilinear on [-1/2,1/2]^3 and
//     integrated with the 3x3x3 Gauss rule; the vertex labels p1..p8 are
//     cyclic (bottom p1..p4, top p5..p8 above them) and are placed on the
//     reference corners in that order;
//   - faces as bilinear patches on [-1/2,1/2]^2 with 2x2 Gauss points at
//     +-sqrt(3)/6, weight 1/4 each (Eq. flux-qud); a triangle with vertices
//     a < b < c (canonical node ids) is the degenerate quadrilateral a b c c;
//   - big stencil: the face neighbours and their face neighbours, as a set,
//     without the cell itself; sub-stencils per cell type; a sub-stencil that
//     names the neighbours of a neighbour takes all of that neighbour's face
//     neighbours except the cell itself;
//   - least-squares fits of the quadratic (9 coefficients) and of the linear
//     polynomials (3 coefficients) in the zero-mean basis about the cell
//     centroid; a fit whose scaled matrix has fewer rows than unknowns or
//     sigma_min < 1e-6 sigma_max is grown by face neighbours of its members,
//     one at a time, until it is well posed; optionally (min_big > 0) a big
//     stencil with fewer than min_big members is grown the same way to
//     min_big members (kept smaller if the candidates run out).
// The pseudo-inverses come from a one-sided Jacobi SVD of the scaled matrix.
// Cells are reordered along a Morton curve of their centroids; each face is
// owned by its lower-numbered cell and oriented towards the other one.
#include "gks_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

namespace gks {


namespace {

constexpr int kTet = 0, kPyr = 1, kPrism = 2, kHex = 3;
constexpr int kFaces[4] = {4, 5, 5, 6};
constexpr int kVerts[4] = {4, 5, 6, 8};

// F_p as 0-based vertex slots; -1 marks a triangle.
constexpr int kFaceSlots[4][6][4] = {
    {{0, 1, 2, -1}, {0, 1, 3, -1}, {1, 2, 3, -1}, {2, 0, 3, -1}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}, {0, 1, 2, 3}, {0, 0, 0, 0}},
    {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}, {0, 0, 0, 0}},
    {{0, 1, 2, 3}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}, {4, 5, 6, 7}},
};

// Degenerate-hexahedron slots: vertex slot used at each of the 8 hexahedron corners.
constexpr int kHexSlot[4][8] = {
    {0, 1, 2, 2, 3, 3, 3, 3},
    {0, 1, 2, 3, 4, 4, 4, 4},
    {0, 1, 2, 2, 3, 4, 5, 5},
    {0, 1, 2, 3, 4, 5, 6, 7},
};

// Sub-stencils: three face labels (0-based) and the face whose neighbour's ring joins (-1 none).
struct SubDef {
    int f[3];
    int ring;
};
constexpr SubDef kSubHex[8] = {{{0, 1, 2}, -1}, {{0, 2, 3}, -1}, {{0, 3, 4}, -1}, {{0, 4, 1}, -1},
                               {{5, 1, 2}, -1}, {{5, 2, 3}, -1}, {{5, 3, 4}, -1}, {{5, 4, 1}, -1}};
constexpr SubDef kSubPrism[6] = {{{0, 2, 3}, -1}, {{0, 3, 4}, -1}, {{0, 4, 2}, -1},
                                 {{1, 2, 3}, -1}, {{1, 3, 4}, -1}, {{1, 4, 2}, -1}};
constexpr SubDef kSubTet[4] = {{{0, 1, 2}, 0}, {{0, 1, 3}, 1}, {{1, 2, 3}, 2}, {{2, 0, 3}, 3}};
constexpr SubDef kSubPyr[8] = {{{0, 1, 2}, 0}, {{1, 2, 3}, 1}, {{2, 3, 0}, 2}, {{3, 0, 1}, 3},
                               {{0, 1, 4}, 0}, {{1, 2, 4}, 1}, {{2, 3, 4}, 2}, {{3, 0, 4}, 3}};

// A stencil member or face neighbour: the image x -> sg x + of L of a cell, sg = +-1 per axis
// (a reflection across a wall plane), of an offset in units of the box (periodic images; 0 or 2
// for the mirror across the wall at 0 or at L).  The image's momentum components carry the signs sg.
struct Member {
    int64_t cell = -1;  // external index
    int sg[3] = {1, 1, 1};
    int of[3] = {0, 0, 0};
    bool operator==(const Member &o) const
    {
        return cell == o.cell && sg[0] == o.sg[0] && sg[1] == o.sg[1] && sg[2] == o.sg[2] && of[0] == o.of[0] &&
               of[1] == o.of[1] && of[2] == o.of[2];
    }
};

Member image(int64_t cell) { return Member{cell, {1, 1, 1}, {0, 0, 0}}; }

// rel seen from base's cell, then base's image map
Member shifted(const Member &base, const Member &rel)
{
    Member r;
    r.cell = rel.cell;
    for (int d = 0; d < 3; ++d) {
        r.sg[d] = base.sg[d] * rel.sg[d];
        r.of[d] = base.sg[d] * rel.of[d] + base.of[d];
    }
    return r;
}

bool contains(const std::vector<Member> &v, const Member &m) { return std::find(v.begin(), v.end(), m) != v.end(); }

struct Key4Hash {
    size_t operator()(const std::array<int64_t, 4> &k) const
    {
        uint64_t h = 1469598103934665603ull;
        for (int64_t v : k) {
            h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        }
        return (size_t)h;
    }
};

struct CellGeom {
    double vol;
    double xc[3];
    double S[3][3];  // mean of (x - xc)(x - xc)^T over the cell
};

// 3x3x3 Gauss on the trilinear map of the degenerate hexahedron.
CellGeom cell_geometry(const double X[8][3])
{
    static const double r = 0.5 * std::sqrt(0.6);
    static const double node[3] = {-r, 0.0, r};
    static const double wt[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};
    // corner sign pattern of the cyclic hexahedron labels
    static const double sgn[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                     {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    double pts[27][3], w[27];
    int q = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c, ++q) {
                const double xi[3] = {node[a], node[b], node[c]};
                double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                double x[3] = {0, 0, 0};
                for (int m = 0; m < 8; ++m) {
                    double l[3], d[3];
                    for (int k = 0; k < 3; ++k) {
                        l[k] = 0.5 + sgn[m][k] * xi[k];
                        d[k] = sgn[m][k];
                    }
                    const double phi = l[0] * l[1] * l[2];
                    const double g[3] = {d[0] * l[1] * l[2], l[0] * d[1] * l[2], l[0] * l[1] * d[2]};
                    for (int i = 0; i < 3; ++i) {
                        x[i] += phi * X[m][i];
                        for (int j = 0; j < 3; ++j) J[i][j] += g[j] * X[m][i];
                    }
                }
                const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                   J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                w[q] = wt[a] * wt[b] * wt[c] * std::fabs(det);
                for (int i = 0; i < 3; ++i) pts[q][i] = x[i];
            }
    CellGeom g{};
    double s1[3] = {0, 0, 0};
    for (int k = 0; k < 27; ++k) {
        g.vol += w[k];
        for (int i = 0; i < 3; ++i) s1[i] += w[k] * pts[k][i];
    }
    for (int i = 0; i < 3; ++i) g.xc[i] = s1[i] / g.vol;
    for (int k = 0; k < 27; ++k) {
        const double d[3] = {pts[k][0] - g.xc[0], pts[k][1] - g.xc[1], pts[k][2] - g.xc[2]};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) g.S[i][j] += w[k] * d[i] * d[j];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g.S[i][j] /= g.vol;
    return g;
}

// 2x2 Gauss points of the bilinear patch through v0 v1 v2 v3 (cyclic), with
// the weighted vector area (1/4) X_eta x X_zeta at each point.
void face_points(const double V[4][3], double gp[4][3], double va[4][3])
{
    const double g = std::sqrt(3.0) / 6.0;
    const double pe[4] = {-g, g, g, -g};
    const double pz[4] = {-g, -g, g, g};
    for (int k = 0; k < 4; ++k) {
        const double e = pe[k], z = pz[k];
        // corners (-,-) (+,-) (+,+) (-,+)
        const double w[4] = {(0.5 - e) * (0.5 - z), (0.5 + e) * (0.5 - z), (0.5 + e) * (0.5 + z),
                             (0.5 - e) * (0.5 + z)};
        const double we[4] = {-(0.5 - z), (0.5 - z), (0.5 + z), -(0.5 + z)};
        const double wz[4] = {-(0.5 - e), -(0.5 + e), (0.5 + e), (0.5 - e)};
        double x[3] = {0, 0, 0}, xe[3] = {0, 0, 0}, xz[3] = {0, 0, 0};
        for (int m = 0; m < 4; ++m)
            for (int i = 0; i < 3; ++i) {
                x[i] += w[m] * V[m][i];
                xe[i] += we[m] * V[m][i];
                xz[i] += wz[m] * V[m][i];
            }
        gp[k][0] = x[0];
        gp[k][1] = x[1];
        gp[k][2] = x[2];
        va[k][0] = 0.25 * (xe[1] * xz[2] - xe[2] * xz[1]);
        va[k][1] = 0.25 * (xe[2] * xz[0] - xe[0] * xz[2]);
        va[k][2] = 0.25 * (xe[0] * xz[1] - xe[1] * xz[0]);
    }
}

// One-sided Jacobi SVD of a row-major n x k matrix: on return the pseudo-inverse
// P (k x n, row-major) and sigma_min / sigma_max.
double jacobi_pinv(const std::vector<double> &A, int n, int k, std::vector<double> &P)
{
    std::vector<double> U(A);  // n x k, columns are rotated
    std::vector<double> V((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) V[(size_t)j * k + j] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                double a = 0, b = 0, c = 0;
                for (int r = 0; r < n; ++r) {
                    const double up = U[(size_t)r * k + p], uq = U[(size_t)r * k + q];
                    a += up * up;
                    b += uq * uq;
                    c += up * uq;
                }
                if (c == 0.0 || std::fabs(c) <= 1e-15 * std::sqrt(a * b)) continue;
                rotated = true;
                const double zeta = (b - a) / (2.0 * c);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int r = 0; r < n; ++r) {
                    const double up = U[(size_t)r * k + p], uq = U[(size_t)r * k + q];
                    U[(size_t)r * k + p] = cs * up - sn * uq;
                    U[(size_t)r * k + q] = sn * up + cs * uq;
                }
                for (int r = 0; r < k; ++r) {
                    const double vp = V[(size_t)r * k + p], vq = V[(size_t)r * k + q];
                    V[(size_t)r * k + p] = cs * vp - sn * vq;
                    V[(size_t)r * k + q] = sn * vp + cs * vq;
                }
            }
        if (!rotated) break;
    }
    std::vector<double> s2(k);
    double smin = INFINITY, smax = 0.0;
    for (int j = 0; j < k; ++j) {
        double s = 0;
        for (int r = 0; r < n; ++r) s += U[(size_t)r * k + j] * U[(size_t)r * k + j];
        s2[j] = s;
        smin = std::min(smin, std::sqrt(s));
        smax = std::max(smax, std::sqrt(s));
    }
    const double ratio = smax > 0 ? smin / smax : 0.0;
    P.assign((size_t)k * n, 0.0);
    if (ratio > 0)
        for (int i = 0; i < k; ++i)
            for (int r = 0; r < n; ++r) {
                double s = 0;
                for (int l = 0; l < k; ++l) s += V[(size_t)i * k + l] * U[(size_t)r * k + l] / s2[l];
                P[(size_t)i * n + r] = s;
            }
    return ratio;
}

uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

}  // namespace

// ---------------------------------------------------------------------------
gks_status preprocess(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types,
                      const int64_t *cells, const double *box, int periodic, int min_big, HostMesh &H)
{
    if (!nodes || !types || !cells || !box || n_nodes <= 0 || n_cells <= 0) return fail(GKS_EINVAL, "null or empty mesh");
    if (n_cells >= (int64_t)1 << 30) return fail(GKS_EINVAL, "too many cells for 32-bit indices");
    for (int i = 0; i < 3; ++i)
        if (!(box[i] > 0)) return fail(GKS_EINVAL, "box lengths must be positive");
    const int64_t n = n_cells;
    for (int64_t c = 0; c < n; ++c) {
        if (types[c] < 0 || types[c] > 3) return fail(GKS_EINVAL, "bad cell type");
        for (int s = 0; s < kVerts[types[c]]; ++s)
            if (cells[8 * c + s] < 0 || cells[8 * c + s] >= n_nodes) return fail(GKS_EINVAL, "bad node id");
    }
    // canonical node ids: the smallest id among nodes at the same wrapped position
    std::vector<int64_t> canon(n_nodes);
    {
        std::unordered_map<std::array<int64_t, 4>, int64_t, Key4Hash> pos;
        pos.reserve((size_t)n_nodes * 2);
        const double q = 1048576.0;
        for (int64_t v = 0; v < n_nodes; ++v) {
            std::array<int64_t, 4> k{};
            for (int i = 0; i < 3; ++i) {
                const int64_t m = (int64_t)std::llround(q);
                int64_t t = (int64_t)std::llround(nodes[3 * v + i] / box[i] * q);
                k[i] = periodic ? ((t % m) + m) % m : t;
            }
            k[3] = 0;
            auto it = pos.find(k);
            if (it == pos.end()) {
                pos.emplace(k, v);
                canon[v] = v;
            } else {
                canon[v] = std::min(it->second, v);
                it->second = canon[v];
            }
        }
        // second pass: every node takes the final minimum of its position
        for (int64_t v = 0; v < n_nodes; ++v) {
            std::array<int64_t, 4> k{};
            for (int i = 0; i < 3; ++i) {
                const int64_t m = (int64_t)std::llround(q);
                int64_t t = (int64_t)std::llround(nodes[3 * v + i] / box[i] * q);
                k[i] = periodic ? ((t % m) + m) % m : t;
            }
            canon[v] = pos[k];
        }
    }
    // per-cell geometry
    std::vector<CellGeom> geo(n);
    std::vector<double> area(n, 0.0);
    for (int64_t c = 0; c < n; ++c) {
        double X[8][3];
        for (int m = 0; m < 8; ++m)
            for (int i = 0; i < 3; ++i) X[m][i] = nodes[3 * cells[8 * c + kHexSlot[types[c]][m]] + i];
        geo[c] = cell_geometry(X);
        if (!(geo[c].vol > 0)) return fail(GKS_EMESH, "cell with non-positive volume");
    }
    // faces: match local faces by their canonical vertex sets
    struct Half {
        int64_t cell;
        int lf;
    };
    std::vector<std::array<Member, 6>> nb(n);
    struct RawFace {
        Half a, b;
        int sh[3];      // image of b's vertices as seen from a
        int wall = -1;  // b absent: the wall's axis (its side in wall_hi)
        int wall_hi = 0;
    };
    std::vector<RawFace> raw;
    {
        std::unordered_map<std::array<int64_t, 4>, int64_t, Key4Hash> open;
        open.reserve((size_t)n * 3);
        for (int64_t c = 0; c < n; ++c)
            for (int lf = 0; lf < kFaces[types[c]]; ++lf) {
                const int *sl = kFaceSlots[types[c]][lf];
                const int nv = sl[3] < 0 ? 3 : 4;
                std::array<int64_t, 4> k{-1, -1, -1, -1};
                for (int i = 0; i < nv; ++i) k[i] = canon[cells[8 * c + sl[i]]];
                std::sort(k.begin(), k.begin() + nv);
                auto it = open.find(k);
                if (it == open.end()) {
                    open.emplace(k, (int64_t)raw.size());
                    raw.push_back(RawFace{Half{c, lf}, Half{-1, -1}, {0, 0, 0}, -1, 0});
                } else {
                    RawFace &f = raw[it->second];
                    if (f.b.cell >= 0) return fail(GKS_EMESH, "face shared by more than two cells");
                    f.b = Half{c, lf};
                }
            }
        for (auto &f : raw) {
            const int *sa = kFaceSlots[types[f.a.cell]][f.a.lf];
            if (f.b.cell < 0) {
                if (periodic) return fail(GKS_EMESH, "face with one cell (mesh not closed periodically)");
                // a reflective wall: every vertex on the plane x_axis = 0 or L; the neighbour is the
                // owner's mirror image across it
                const int nv = sa[3] < 0 ? 3 : 4;
                for (int d = 0; d < 3 && f.wall < 0; ++d) {
                    bool lo = true, hi = true;
                    for (int i = 0; i < nv; ++i) {
                        const double x = nodes[3 * cells[8 * f.a.cell + sa[i]] + d];
                        if (std::fabs(x) > 1e-12 * box[d]) lo = false;
                        if (std::fabs(x - box[d]) > 1e-12 * box[d]) hi = false;
                    }
                    if (lo || hi) {
                        f.wall = d;
                        f.wall_hi = hi ? 1 : 0;
                    }
                }
                if (f.wall < 0) return fail(GKS_EMESH, "boundary face not on a wall of the box");
                Member g = image(f.a.cell);
                g.sg[f.wall] = -1;
                g.of[f.wall] = f.wall_hi ? 2 : 0;
                nb[f.a.cell][f.a.lf] = g;
                continue;
            }
            const int *sb = kFaceSlots[types[f.b.cell]][f.b.lf];
            const int64_t va0 = cells[8 * f.a.cell + sa[0]];
            int64_t match = -1;
            for (int i = 0; i < (sb[3] < 0 ? 3 : 4); ++i) {
                const int64_t vb = cells[8 * f.b.cell + sb[i]];
                if (canon[vb] == canon[va0]) match = vb;
            }
            for (int i = 0; i < 3; ++i) f.sh[i] = (int)std::lround((nodes[3 * va0 + i] - nodes[3 * match + i]) / box[i]);
            nb[f.a.cell][f.a.lf] = Member{f.b.cell, {1, 1, 1}, {f.sh[0], f.sh[1], f.sh[2]}};
            nb[f.b.cell][f.b.lf] = Member{f.a.cell, {1, 1, 1}, {-f.sh[0], -f.sh[1], -f.sh[2]}};
        }
    }
    // Morton order of the centroids
    std::vector<int64_t> perm(n), inv(n);
    {
        std::vector<std::pair<uint64_t, int64_t>> code(n);
        for (int64_t c = 0; c < n; ++c) {
            uint64_t m = 0;
            for (int i = 0; i < 3; ++i) {
                double u = geo[c].xc[i] / box[i];
                u -= std::floor(u);
                const uint64_t b = std::min<uint64_t>((uint64_t)(u * 2097152.0), 2097151);
                m |= spread3(b) << i;
            }
            code[c] = {m, c};
        }
        std::sort(code.begin(), code.end());
        for (int64_t i = 0; i < n; ++i) {
            perm[i] = code[i].second;
            inv[code[i].second] = i;
        }
    }

    // stencils and fits, per cell in internal order
    H.n = n;
    H.L[0] = box[0];
    H.L[1] = box[1];
    H.L[2] = box[2];
    H.perm = perm;
    H.type.resize(n);
    H.vol.resize(n);
    H.xc.resize(3 * n);
    H.m2.resize(6 * n);
    H.hcfl.resize(n);
    H.st_ptr.assign(n + 1, 0);
    H.st_idx.clear();
    H.st_mask.clear();
    H.st_flip.clear();
    H.pinv.clear();
    H.dsc.clear();
    H.ginv.clear();
    H.n_grown = 0;

    auto member_row = [&](const CellGeom &g0, const Member &m, int k, double h, double *row) {
        const CellGeom &gm0 = geo[m.cell];
        // the image's moments: reflections flip the mixed second moments they touch
        CellGeom gm = gm0;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) gm.S[p][q] = m.sg[p] * m.sg[q] * gm0.S[p][q];
        double D[3];
        for (int i = 0; i < 3; ++i) D[i] = m.sg[i] * gm0.xc[i] + m.of[i] * box[i] - g0.xc[i];
        // means over the member of (x - x0)^n minus the means over the cell itself
        const double vals[9] = {D[0],
                                D[1],
                                D[2],
                                gm.S[0][0] + D[0] * D[0] - g0.S[0][0],
                                gm.S[0][1] + D[0] * D[1] - g0.S[0][1],
                                gm.S[0][2] + D[0] * D[2] - g0.S[0][2],
                                gm.S[1][1] + D[1] * D[1] - g0.S[1][1],
                                gm.S[1][2] + D[1] * D[2] - g0.S[1][2],
                                gm.S[2][2] + D[2] * D[2] - g0.S[2][2]};
        for (int j = 0; j < k; ++j) row[j] = vals[j] / (j < 3 ? h : h * h);
    };
    // min_rows: a well-posed fit is still grown while it has fewer members (best effort: kept when the
    // candidates run out)
    auto fit = [&](int64_t c, std::vector<Member> &list, int k, double h, std::vector<double> &P,
                   int min_rows) -> int {
        const CellGeom &g0 = geo[c];
        const Member self = image(c);
        std::vector<Member> cand;
        for (const Member &m : list)
            for (int p = 0; p < kFaces[types[m.cell]]; ++p) {
                Member s = shifted(m, nb[m.cell][p]);
                if (s == self || contains(list, s) || contains(cand, s)) continue;
                cand.push_back(s);
            }
        size_t used = 0;
        for (;;) {
            const int rows = (int)list.size();
            bool posed = false;
            if (rows >= k) {
                std::vector<double> A((size_t)rows * k);
                for (int r = 0; r < rows; ++r) member_row(g0, list[r], k, h, &A[(size_t)r * k]);
                posed = jacobi_pinv(A, rows, k, P) >= 1e-6;
            }
            const bool out_of_candidates = used >= cand.size();
            if (posed && (rows >= min_rows || out_of_candidates)) {
                // undo the column scaling: coefficient j = scaled unknown j / h^deg
                for (int j = 0; j < k; ++j) {
                    const double s = j < 3 ? h : h * h;
                    for (int r = 0; r < rows; ++r) P[(size_t)j * rows + r] /= s;
                }
                return (int)used;
            }
            if (out_of_candidates) return -1;
            list.push_back(cand[used++]);
        }
    };

    struct CellOut {
        std::vector<int32_t> idx;
        std::vector<uint8_t> mask, flip;
        std::vector<double> pinv, dsc, ginv;
        int grown = 0;
        int err = 0;  // 0 ok, 1 big fit singular, 2 sub fit singular, 3 too large
    };
    std::vector<CellOut> outs(n);
    auto process = [&](int64_t i, CellOut &out) {
        const int64_t c = perm[i];
        const int t = types[c];
        const CellGeom &g = geo[c];
        const Member self = image(c);
        H.type[i] = (int8_t)t;
        H.vol[i] = g.vol;
        for (int d = 0; d < 3; ++d) H.xc[3 * i + d] = g.xc[d];
        const double m2v[6] = {g.S[0][0], g.S[0][1], g.S[0][2], g.S[1][1], g.S[1][2], g.S[2][2]};
        for (int d = 0; d < 6; ++d) H.m2[6 * i + d] = m2v[d];
        // big stencil
        std::vector<Member> big;
        for (int p = 0; p < kFaces[t]; ++p)
            if (!contains(big, nb[c][p])) big.push_back(nb[c][p]);
        for (int p = 0; p < kFaces[t]; ++p) {
            const Member &J = nb[c][p];
            for (int q = 0; q < kFaces[types[J.cell]]; ++q) {
                Member s = shifted(J, nb[J.cell][q]);
                if (s == self || contains(big, s)) continue;
                big.push_back(s);
            }
        }
        // sub-stencils
        const SubDef *sd;
        int M;
        switch (t) {
        case kHex: sd = kSubHex; M = 8; break;
        case kPrism: sd = kSubPrism; M = 6; break;
        case kTet: sd = kSubTet; M = 4; break;
        default: sd = kSubPyr; M = 8; break;
        }
        std::vector<std::vector<Member>> subs(M);
        for (int m = 0; m < M; ++m) {
            for (int q = 0; q < 3; ++q)
                if (!contains(subs[m], nb[c][sd[m].f[q]])) subs[m].push_back(nb[c][sd[m].f[q]]);
            if (sd[m].ring >= 0) {
                const Member &J = nb[c][sd[m].ring];
                for (int q = 0; q < kFaces[types[J.cell]]; ++q) {
                    Member s = shifted(J, nb[J.cell][q]);
                    if (s == self || contains(subs[m], s)) continue;
                    subs[m].push_back(s);
                }
            }
        }
        const double h = std::cbrt(g.vol);
        std::vector<double> P0;
        int gr = fit(c, big, 9, h, P0, min_big);
        if (gr < 0) {
            out.err = 1;
            return;
        }
        out.grown += gr;
        const int nls = (int)big.size();
        std::vector<std::vector<double>> Pm(M);
        for (int m = 0; m < M; ++m) {
            int gm = fit(c, subs[m], 3, h, Pm[m], 0);
            if (gm < 0) {
                out.err = 2;
                return;
            }
            out.grown += gm;
        }
        // member list = big stencil, then members only a sub-stencil uses
        std::vector<Member> members = big;
        std::vector<std::vector<int>> slot(M);
        for (int m = 0; m < M; ++m)
            for (const Member &s : subs[m]) {
                auto it = std::find(members.begin(), members.end(), s);
                int k = (int)(it - members.begin());
                if (it == members.end()) members.push_back(s);
                slot[m].push_back(k);
            }
        if (members.size() > 255) {
            out.err = 3;
            return;
        }
        // scaled centroid offsets of the members: the linear sub-stencil fits are
        // b^m = (1/h) G_m^{-1} sum_{k in S_m} D_k (Q_k - Q_0), G_m = sum_{k in S_m} D_k D_k^T
        std::vector<std::array<double, 3>> Ds(members.size());
        for (size_t k = 0; k < members.size(); ++k)
            for (int d = 0; d < 3; ++d)
                Ds[k][d] = (members[k].sg[d] * geo[members[k].cell].xc[d] + members[k].of[d] * box[d] - g.xc[d]) / h;
        out.ginv.assign(48, 0.0);
        for (int m = 0; m < M; ++m) {
            double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k : slot[m])
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) G[p][q] += Ds[k][p] * Ds[k][q];
            const double c00 = G[1][1] * G[2][2] - G[1][2] * G[2][1];
            const double c01 = G[0][2] * G[2][1] - G[0][1] * G[2][2];
            const double c02 = G[0][1] * G[1][2] - G[0][2] * G[1][1];
            const double c11 = G[0][0] * G[2][2] - G[0][2] * G[2][0];
            const double c12 = G[0][2] * G[1][0] - G[0][0] * G[1][2];
            const double c22 = G[0][0] * G[1][1] - G[0][1] * G[1][0];
            const double det = G[0][0] * c00 + G[0][1] * (G[1][2] * G[2][0] - G[1][0] * G[2][2]) +
                               G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
            const double s = 1.0 / (det * h);
            const double inv6[6] = {c00 * s, c01 * s, c02 * s, c11 * s, c12 * s, c22 * s};
            for (int q = 0; q < 6; ++q) out.ginv[6 * m + q] = inv6[q];
        }
        for (size_t k = 0; k < members.size(); ++k) {
            uint8_t mask = 0;
            for (int m = 0; m < M; ++m)
                for (size_t e = 0; e < slot[m].size(); ++e)
                    if (slot[m][e] == (int)k) mask |= (uint8_t)(1u << m);
            out.idx.push_back((int32_t)members[k].cell);  // external for now
            out.mask.push_back(mask);
            // bit d: mirrored on axis d; bit 3 + d: at the plane x_d = L; bit 6: mirrored twice on an axis
            // (at 0 and at L: a translation by 2L, which only the reflective condition leaves invariant)
            unsigned fl = 0;
            for (int d = 0; d < 3; ++d) {
                if (members[k].sg[d] < 0) fl |= 1u << d | (members[k].of[d] == 2 ? 1u << (3 + d) : 0u);
                else if (!periodic && (members[k].of[d] == 2 || members[k].of[d] == -2)) fl |= 1u << 6;
            }
            out.flip.push_back((uint8_t)fl);
            for (int j = 0; j < 9; ++j)
                out.pinv.push_back((int)k < nls ? P0[(size_t)j * nls + k] : 0.0);
            for (int d = 0; d < 3; ++d) out.dsc.push_back(Ds[k][d]);
        }
    };
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) process(i, outs[i]);
    for (int64_t i = 0; i < n; ++i) {
        CellOut &o = outs[i];
        if (o.err == 1) return fail(GKS_ESINGULAR, "big-stencil fit stays rank deficient at cell " + std::to_string(perm[i]));
        if (o.err == 2) return fail(GKS_ESINGULAR, "sub-stencil fit stays rank deficient at cell " + std::to_string(perm[i]));
        if (o.err == 3) return fail(GKS_EINVAL, "stencil too large at cell " + std::to_string(perm[i]));
        H.n_grown += o.grown;
        H.st_ptr[i + 1] = H.st_ptr[i] + (int32_t)o.idx.size();
        H.st_idx.insert(H.st_idx.end(), o.idx.begin(), o.idx.end());
        H.st_mask.insert(H.st_mask.end(), o.mask.begin(), o.mask.end());
        H.st_flip.insert(H.st_flip.end(), o.flip.begin(), o.flip.end());
        H.pinv.insert(H.pinv.end(), o.pinv.begin(), o.pinv.end());
        H.dsc.insert(H.dsc.end(), o.dsc.begin(), o.dsc.end());
        H.ginv.insert(H.ginv.end(), o.ginv.begin(), o.ginv.end());
        CellOut().idx.swap(o.idx);
        std::vector<double>().swap(o.pinv);
        std::vector<double>().swap(o.dsc);
        std::vector<double>().swap(o.ginv);
        std::vector<uint8_t>().swap(o.mask);
        std::vector<uint8_t>().swap(o.flip);
    }
    for (auto &v : H.st_idx) v = (int32_t)inv[v];

    // faces in internal numbering: owner = lower index; sorted by (owner, neighbour)
    const int64_t nf = (int64_t)raw.size();
    std::vector<int64_t> forder(nf);
    std::vector<std::pair<int64_t, int64_t>> fkey(nf);
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t a = inv[raw[f].a.cell];
        const int64_t b = raw[f].b.cell >= 0 ? inv[raw[f].b.cell] : INT64_MAX;  // walls after the owner's faces
        fkey[f] = {std::min(a, b), std::max(a, b)};
        forder[f] = f;
    }
    std::stable_sort(forder.begin(), forder.end(), [&](int64_t x, int64_t y) { return fkey[x] < fkey[y]; });
    H.nf = nf;
    H.owner.resize(nf);
    H.nbr.resize(nf);
    H.fgeo.assign((size_t)9 * 4 * nf, 0.0);
    std::vector<double> area_sum(n, 0.0);
    std::vector<std::vector<std::pair<int, int>>> cf(n);  // (face, side) per internal cell, in F_p order
    for (int64_t i = 0; i < n; ++i) cf[i].resize(kFaces[H.type[i]], {-1, -1});
    for (int64_t fo = 0; fo < nf; ++fo) {
        const RawFace &r = raw[forder[fo]];
        const bool wall = r.b.cell < 0;
        const bool a_owns = wall || inv[r.a.cell] < inv[r.b.cell];
        const Half own = a_owns ? r.a : r.b;
        const Half oth = a_owns ? r.b : r.a;
        // the neighbour's image as seen from the owner: a periodic image, or the owner's mirror
        Member img = wall ? nb[own.cell][own.lf] : image(oth.cell);
        if (!wall)
            for (int d = 0; d < 3; ++d) img.of[d] = a_owns ? r.sh[d] : -r.sh[d];
        H.owner[fo] = (int32_t)inv[own.cell];
        H.nbr[fo] = wall ? -1 - (2 * r.wall + r.wall_hi) : (int32_t)inv[oth.cell];
        const int *sl = kFaceSlots[types[own.cell]][own.lf];
        double V[4][3];
        if (sl[3] >= 0) {
            for (int m = 0; m < 4; ++m)
                for (int d = 0; d < 3; ++d) V[m][d] = nodes[3 * cells[8 * own.cell + sl[m]] + d];
        } else {
            int64_t v[3] = {cells[8 * own.cell + sl[0]], cells[8 * own.cell + sl[1]], cells[8 * own.cell + sl[2]]};
            std::sort(v, v + 3, [&](int64_t x, int64_t y) { return canon[x] < canon[y]; });
            const int64_t order[4] = {v[0], v[1], v[2], v[2]};
            for (int m = 0; m < 4; ++m)
                for (int d = 0; d < 3; ++d) V[m][d] = nodes[3 * order[m] + d];
        }
        double gp[4][3], va[4][3];
        face_points(V, gp, va);
        const CellGeom &go = geo[own.cell], &gn = geo[img.cell];
        double orient = 0;
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) orient += va[k][d] * (gp[k][d] - go.xc[d]);
        const double s = orient < 0 ? -1.0 : 1.0;
        double ar = 0;
        for (int k = 0; k < 4; ++k) {
            for (int d = 0; d < 3; ++d) {
                const double dl = gp[k][d] - go.xc[d];
                const double dr = gp[k][d] - (img.sg[d] * gn.xc[d] + img.of[d] * box[d]);
                H.fgeo[(size_t)(0 + d) * 4 * nf + 4 * fo + k] = dl;
                H.fgeo[(size_t)(3 + d) * 4 * nf + 4 * fo + k] = dr;
                H.fgeo[(size_t)(6 + d) * 4 * nf + 4 * fo + k] = s * va[k][d];
            }
            ar += std::sqrt(va[k][0] * va[k][0] + va[k][1] * va[k][1] + va[k][2] * va[k][2]);
        }
        area_sum[inv[own.cell]] += ar;
        cf[inv[own.cell]][own.lf] = {(int)fo, 0};
        if (!wall) {
            area_sum[inv[oth.cell]] += ar;
            cf[inv[oth.cell]][oth.lf] = {(int)fo, 1};
        }
    }
    H.cf_ptr.assign(n + 1, 0);
    H.cf_idx.clear();
    for (int64_t i = 0; i < n; ++i) {
        for (auto &e : cf[i]) H.cf_idx.push_back((int32_t)(2 * e.first + e.second));
        H.cf_ptr[i + 1] = (int32_t)H.cf_idx.size();
        H.hcfl[i] = 6.0 * H.vol[i] / area_sum[i];
    }
    // transposed stencil: for each cell, the stencil entries (of all cells) that name it, in entry order
    H.tr_ptr.assign(n + 1, 0);
    for (int32_t v : H.st_idx) H.tr_ptr[v + 1]++;
    for (int64_t i = 0; i < n; ++i) H.tr_ptr[i + 1] += H.tr_ptr[i];
    H.tr_idx.assign(H.st_idx.size(), 0);
    {
        std::vector<int32_t> fill(H.tr_ptr.begin(), H.tr_ptr.end() - 1);
        for (size_t e = 0; e < H.st_idx.size(); ++e) H.tr_idx[fill[H.st_idx[e]]++] = (int32_t)e;
    }
    return GKS_OK;
}

}  // namespace gks
