/*
 * Seeded synthetic inputs for the gas-kinetic solver: hybrid-lattice meshes
 * and cell-averaged initial fields.
 *
 * This module holds no arithmetic of the numerical method.  It only produces
 * what both the FP64 reference and the GPU library consume: node coordinates,
 * cell types with their vertex lists, and cell averages of analytic fields.
 * Cell averages are computed by splitting each (flat-faced) cell into
 * tetrahedra and applying a collapsed (Duffy) tensor Gauss-Legendre rule,
 * which is unrelated to the trilinear 3x3x3 rule the method uses.
 *
 * Cell vertex order follows the paper's labels (Section 2): tetrahedron
 * p1..p4; pyramid base p1..p4 (cyclic) and apex p5; prism bottom p1p2p3 and
 * top p4p5p6 with p4 above p1; hexahedron bottom p1..p4 (cyclic) and top
 * p5..p8 above them.
 *
 * Lattice realisation (one draw per lattice hexahedron):
 *   type T = splitmix64(seed ^ index) mod 4 in {HEX, PRISM, TET, PYR};
 *   HEX   -> 1 hexahedron, demands quadrilateral faces everywhere;
 *   PRISM -> 2 prisms split by the local plane x = y, demands triangles on
 *            the two z faces and quadrilaterals on the four side faces;
 *   TET   -> 6 tetrahedra sharing the main diagonal, demands triangles;
 *   PYR   -> no demand.
 * Each lattice face takes the demand of its higher-priority side
 * (HEX > PRISM > TET > PYR; quadrilateral when neither side demands).  A
 * lattice hexahedron whose six faces all match its own demand is realised as
 * drawn; any other one, and every PYR, becomes 6 pyramids with apex at the
 * centre, each pyramid on a triangulated face being split into 2 tetrahedra.
 * Every triangulated lattice face uses the diagonal from its minimum corner
 * to its maximum corner, so the mesh is conforming, periodic images match,
 * and the construction never cascades.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { T_TET = 0, T_PYR = 1, T_PRISM = 2, T_HEX = 3 };
/* draw codes */
enum { D_HEX = 0, D_PRISM = 1, D_TET = 2, D_PYR = 3 };
/* mesh kinds (K_HEXPRISM: whole columns along z of hexahedra, 40 % of them, or of prisms; the
   cavity meshes' cell mix) */
enum { K_HYBRID = 0, K_HEX = 1, K_TET = 2, K_PYR = 3, K_PRISM = 4, K_HEXPRISM = 5 };

uint64_t gin_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    int N;
    int periodic;
    int kind;
    uint64_t seed;
    int8_t *draw; /* per lattice hex */
    int8_t *native;
} lat_t;

static int64_t hidx(const lat_t *L, int i, int j, int k) { return (int64_t)i + (int64_t)L->N * ((int64_t)j + (int64_t)L->N * k); }

static int draw_of(const lat_t *L, int i, int j, int k)
{
    switch (L->kind) {
    case K_HEX: return D_HEX;
    case K_TET: return D_TET;
    case K_PYR: return D_PYR;
    case K_PRISM: return D_PRISM;
    default: break;
    }
    uint64_t r = gin_splitmix64(L->seed ^ (uint64_t)hidx(L, i, j, k));
    return (int)(r % 4u);
}

static int priority(int d)
{
    switch (d) {
    case D_HEX: return 3;
    case D_PRISM: return 2;
    case D_TET: return 1;
    default: return 0;
    }
}

/* demand of a drawn type on lattice face axis a (0=x,1=y,2=z): 0 none, 1 quad, 2 tri */
static int demand(int d, int axis)
{
    switch (d) {
    case D_HEX: return 1;
    case D_PRISM: return axis == 2 ? 2 : 1;
    case D_TET: return 2;
    default: return 0;
    }
}

/* face type (1 quad, 2 tri) of the lattice face of hex (i,j,k) on side s of axis a */
static int face_type(const lat_t *L, int i, int j, int k, int axis, int s)
{
    int d0 = L->draw[hidx(L, i, j, k)];
    int n[3] = {i, j, k};
    n[axis] += s ? 1 : -1;
    int has_nb = 1;
    if (n[axis] < 0 || n[axis] >= L->N) {
        if (L->periodic) n[axis] = (n[axis] + L->N) % L->N;
        else has_nb = 0;
    }
    int best = d0;
    if (has_nb) {
        int d1 = L->draw[hidx(L, n[0], n[1], n[2])];
        if (priority(d1) > priority(best)) best = d1;
    }
    int dm = demand(best, axis);
    return dm == 0 ? 1 : dm;
}

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static void lat_init(lat_t *L, int N, int kind, uint64_t seed, int periodic)
{
    L->N = N;
    L->kind = kind;
    L->seed = seed;
    L->periodic = periodic;
    int64_t nh = (int64_t)N * N * N;
    L->draw = (int8_t *)malloc((size_t)nh);
    L->native = (int8_t *)malloc((size_t)nh);
    if (kind == K_HEXPRISM) {
        /* the columns (i, j) with the round(0.4 N^2) smallest seeded hashes hold hexahedra, the others
           prisms (split alike in every layer, so every face matches) */
        const int64_t nc = (int64_t)N * N, nhex = (4 * nc + 5) / 10;
        uint64_t *h = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nc), *srt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nc);
        for (int64_t c = 0; c < nc; c++) h[c] = srt[c] = gin_splitmix64(seed ^ (0xC0C0C0C0ull + (uint64_t)c));
        qsort(srt, (size_t)nc, sizeof(uint64_t), cmp_u64);
        const uint64_t cut = nhex < nc ? srt[nhex] : ~0ull;
        for (int k = 0; k < N; k++)
            for (int j = 0; j < N; j++)
                for (int i = 0; i < N; i++)
                    L->draw[hidx(L, i, j, k)] = (int8_t)(h[i + (int64_t)N * j] < cut ? D_HEX : D_PRISM);
        free(h);
        free(srt);
    } else {
        for (int k = 0; k < N; k++)
            for (int j = 0; j < N; j++)
                for (int i = 0; i < N; i++) L->draw[hidx(L, i, j, k)] = (int8_t)draw_of(L, i, j, k);
    }
    for (int k = 0; k < N; k++)
        for (int j = 0; j < N; j++)
            for (int i = 0; i < N; i++) {
                int d = L->draw[hidx(L, i, j, k)];
                int ok = (d != D_PYR);
                for (int a = 0; a < 3 && ok; a++)
                    for (int s = 0; s < 2 && ok; s++)
                        if (face_type(L, i, j, k, a, s) != demand(d, a)) ok = 0;
                L->native[hidx(L, i, j, k)] = (int8_t)ok;
            }
}

static void lat_free(lat_t *L)
{
    free(L->draw);
    free(L->native);
}

/* lattice node id */
static int64_t nid(int N, int i, int j, int k) { return (int64_t)i + (int64_t)(N + 1) * ((int64_t)j + (int64_t)(N + 1) * k); }

/* local cube corner c = (bx,by,bz) bits -> node id */
static int64_t corner(int N, int i, int j, int k, int bx, int by, int bz) { return nid(N, i + bx, j + by, k + bz); }

typedef struct {
    int64_t ncell;
    int64_t hist[4];
    int8_t *types;   /* may be NULL when counting */
    int64_t *cells;  /* [ncell][8] */
} sink_t;

static void emit(sink_t *S, int type, const int64_t *v, int nv)
{
    if (S->types) {
        S->types[S->ncell] = (int8_t)type;
        int64_t *c = S->cells + 8 * S->ncell;
        for (int q = 0; q < 8; q++) c[q] = q < nv ? v[q] : -1;
    }
    S->hist[type]++;
    S->ncell++;
}

/* the four corners of lattice face (axis, side) of hex (i,j,k), in cyclic order */
static void face_quad(int N, int i, int j, int k, int axis, int s, int64_t q[4], int bits[4][3])
{
    int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
    int cyc[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int c = 0; c < 4; c++) {
        int b[3];
        b[axis] = s;
        b[a1] = cyc[c][0];
        b[a2] = cyc[c][1];
        q[c] = corner(N, i, j, k, b[0], b[1], b[2]);
        if (bits) memcpy(bits[c], b, sizeof b);
    }
}

static void realise(const lat_t *L, int i, int j, int k, int64_t center_id, sink_t *S)
{
    int N = L->N;
    int d = L->draw[hidx(L, i, j, k)];
    if (L->native[hidx(L, i, j, k)]) {
        if (d == D_HEX) {
            int64_t v[8] = {corner(N, i, j, k, 0, 0, 0), corner(N, i, j, k, 1, 0, 0), corner(N, i, j, k, 1, 1, 0),
                            corner(N, i, j, k, 0, 1, 0), corner(N, i, j, k, 0, 0, 1), corner(N, i, j, k, 1, 0, 1),
                            corner(N, i, j, k, 1, 1, 1), corner(N, i, j, k, 0, 1, 1)};
            emit(S, T_HEX, v, 8);
        } else if (d == D_PRISM) {
            /* split by the plane x = y: triangles (00,10,11) and (00,11,01) */
            int tri[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {1, 1}, {0, 1}}};
            for (int t = 0; t < 2; t++) {
                int64_t v[6];
                for (int c = 0; c < 3; c++) {
                    v[c] = corner(N, i, j, k, tri[t][c][0], tri[t][c][1], 0);
                    v[c + 3] = corner(N, i, j, k, tri[t][c][0], tri[t][c][1], 1);
                }
                emit(S, T_PRISM, v, 6);
            }
        } else { /* D_TET: 6 tetrahedra along the main diagonal */
            static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
            for (int p = 0; p < 6; p++) {
                int b[3] = {0, 0, 0};
                int64_t v[4];
                v[0] = corner(N, i, j, k, 0, 0, 0);
                b[perm[p][0]] = 1;
                v[1] = corner(N, i, j, k, b[0], b[1], b[2]);
                b[perm[p][1]] = 1;
                v[2] = corner(N, i, j, k, b[0], b[1], b[2]);
                v[3] = corner(N, i, j, k, 1, 1, 1);
                emit(S, T_TET, v, 4);
            }
        }
        return;
    }
    /* fallback: 6 pyramids with apex at the centre; triangulated faces -> 2 tets */
    for (int a = 0; a < 3; a++)
        for (int s = 0; s < 2; s++) {
            int64_t q[4];
            int bits[4][3];
            face_quad(N, i, j, k, a, s, q, bits);
            if (face_type(L, i, j, k, a, s) == 1) {
                int64_t v[5] = {q[0], q[1], q[2], q[3], center_id};
                emit(S, T_PYR, v, 5);
            } else {
                /* diagonal from the minimum corner (cyclic slot 0) to the maximum one (slot 2) */
                int64_t v1[4] = {q[0], q[1], q[2], center_id};
                int64_t v2[4] = {q[0], q[2], q[3], center_id};
                emit(S, T_TET, v1, 4);
                emit(S, T_TET, v2, 4);
            }
        }
}

/*
 * Count (types == NULL) or build a lattice mesh on the box [0,Lx]x[0,Ly]x[0,Lz].
 * nodes: [(N+1)^3 + n_center][3]; types: [ncell]; cells: [ncell][8] (-1 padded).
 * Returns 0 on success.
 */
int gin_lattice(int N, int kind, uint64_t seed, int periodic, const double *box, int64_t *n_nodes, int64_t *n_cells,
                int64_t *hist, double *nodes, int8_t *types, int64_t *cells)
{
    if (N < 1 || kind < 0 || kind > 5) return 1;
    lat_t L;
    lat_init(&L, N, kind, seed, periodic);
    int64_t nlat = (int64_t)(N + 1) * (N + 1) * (N + 1);
    int64_t ncenter = 0;
    for (int64_t h = 0; h < (int64_t)N * N * N; h++)
        if (!L.native[h]) ncenter++;
    *n_nodes = nlat + ncenter;
    sink_t S;
    memset(&S, 0, sizeof S);
    S.types = types;
    S.cells = cells;
    if (nodes) {
        for (int k = 0; k <= N; k++)
            for (int j = 0; j <= N; j++)
                for (int i = 0; i <= N; i++) {
                    double *x = nodes + 3 * nid(N, i, j, k);
                    x[0] = box[0] * (double)i / N;
                    x[1] = box[1] * (double)j / N;
                    x[2] = box[2] * (double)k / N;
                }
    }
    int64_t cid = nlat;
    for (int k = 0; k < N; k++)
        for (int j = 0; j < N; j++)
            for (int i = 0; i < N; i++) {
                int64_t center = -1;
                if (!L.native[hidx(&L, i, j, k)]) {
                    center = cid++;
                    if (nodes) {
                        double *x = nodes + 3 * center;
                        x[0] = box[0] * (i + 0.5) / N;
                        x[1] = box[1] * (j + 0.5) / N;
                        x[2] = box[2] * (k + 0.5) / N;
                    }
                }
                realise(&L, i, j, k, center, &S);
            }
    *n_cells = S.ncell;
    if (hist)
        for (int t = 0; t < 4; t++) hist[t] = S.hist[t];
    lat_free(&L);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Cell averages of analytic fields                                         */
/* ---------------------------------------------------------------------- */

enum { F_WAVE = 0, F_TGV = 1, F_RIEMANN = 2, F_WAVE_PERTURBED = 3, F_UNIFORM = 4 };

typedef struct {
    int kind;
    double gamma;
    double p[16];      /* field parameters, meaning per kind */
    int nmodes;        /* F_WAVE_PERTURBED */
    const double *modes; /* [nmodes][3 + 6]: integer wave vector, A(3), B(3) */
} field_t;

/* primitive (rho, u, v, w, p) at x */
static void field_prim(const field_t *f, const double *x, double *w)
{
    const double *P = f->p;
    switch (f->kind) {
    case F_WAVE:
    case F_WAVE_PERTURBED: {
        /* rho = 1 + amp sin(k.x - k.U t), U const, p const; P = amp, kx,ky,kz, U,V,W, p0, t */
        double ph = P[1] * (x[0] - P[4] * P[8]) + P[2] * (x[1] - P[5] * P[8]) + P[3] * (x[2] - P[6] * P[8]);
        w[0] = 1.0 + P[0] * sin(ph);
        w[1] = P[4];
        w[2] = P[5];
        w[3] = P[6];
        w[4] = P[7];
        if (f->kind == F_WAVE_PERTURBED) {
            for (int m = 0; m < f->nmodes; m++) {
                const double *md = f->modes + 9 * m;
                double a = 2.0 * M_PI * (md[0] * x[0] + md[1] * x[1] + md[2] * x[2]);
                double c = cos(a), s = sin(a);
                for (int q = 0; q < 3; q++) w[1 + q] += md[3 + q] * c + md[6 + q] * s;
            }
        }
        break;
    }
    case F_TGV: {
        /* P = V0, rho0, p0 */
        double V0 = P[0], r0 = P[1], p0 = P[2];
        w[1] = V0 * sin(x[0]) * cos(x[1]) * cos(x[2]);
        w[2] = -V0 * cos(x[0]) * sin(x[1]) * cos(x[2]);
        w[3] = 0.0;
        w[4] = p0 + r0 * V0 * V0 / 16.0 * (cos(2 * x[0]) + cos(2 * x[1])) * (cos(2 * x[2]) + 2.0);
        w[0] = r0 * w[4] / p0;
        break;
    }
    case F_RIEMANN: {
        /* plane n.x = c; P = nx,ny,nz,c, left(rho,u,v,w,p), right(rho,u,v,w,p) */
        double s = P[0] * x[0] + P[1] * x[1] + P[2] * x[2] - P[3];
        const double *st = s < 0 ? P + 4 : P + 9;
        for (int q = 0; q < 5; q++) w[q] = st[q];
        break;
    }
    default: {
        for (int q = 0; q < 5; q++) w[q] = P[q];
        break;
    }
    }
}

static void field_cons(const field_t *f, const double *x, double *q)
{
    double w[5];
    field_prim(f, x, w);
    q[0] = w[0];
    q[1] = w[0] * w[1];
    q[2] = w[0] * w[2];
    q[3] = w[0] * w[3];
    q[4] = w[4] / (f->gamma - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
}

/* Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n */
static void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

static void sub3(const double *a, const double *b, double *c)
{
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}

/* integrate conserved variables over a tetrahedron; returns volume */
static double tet_integrate(const field_t *f, const double *v0, const double *v1, const double *v2, const double *v3,
                            int n, const double *gx, const double *gw, double *acc)
{
    double e1[3], e2[3], e3[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    sub3(v3, v0, e3);
    double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                 e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    double adet = fabs(det);
    for (int ia = 0; ia < n; ia++)
        for (int ib = 0; ib < n; ib++)
            for (int ic = 0; ic < n; ic++) {
                double a = gx[ia], b = gx[ib], c = gx[ic];
                double s3 = c, s2 = b * (1.0 - c), s1 = a * (1.0 - b) * (1.0 - c);
                double jac = (1.0 - b) * (1.0 - c) * (1.0 - c);
                double wt = gw[ia] * gw[ib] * gw[ic] * jac * adet;
                double x[3];
                for (int q = 0; q < 3; q++) x[q] = v0[q] + s1 * e1[q] + s2 * e2[q] + s3 * e3[q];
                double qv[5];
                field_cons(f, x, qv);
                for (int q = 0; q < 5; q++) acc[q] += wt * qv[q];
            }
    return adet / 6.0;
}

/*
 * Cell averages of the conserved variables (rho, rho U, rho V, rho W, rho E),
 * output layout [5][ncell].  order = points per direction of the collapsed
 * Gauss-Legendre rule on each sub-tetrahedron (1..12).
 */
int gin_cell_averages(int64_t ncell, const double *nodes, const int8_t *types, const int64_t *cells, int kind,
                      double gamma, const double *params, int nmodes, const double *modes, int order, double *out)
{
    if (order < 1 || order > 12) return 1;
    field_t f;
    f.kind = kind;
    f.gamma = gamma;
    for (int q = 0; q < 16; q++) f.p[q] = params[q];
    f.nmodes = nmodes;
    f.modes = modes;
    double gx[12], gw[12];
    gauss_legendre01(order, gx, gw);
    /* tetrahedral splits of each type in local vertex slots */
    static const int tet_split[1][4] = {{0, 1, 2, 3}};
    static const int pyr_split[2][4] = {{0, 1, 2, 4}, {0, 2, 3, 4}};
    static const int pri_split[3][4] = {{0, 1, 2, 3}, {1, 2, 3, 4}, {2, 3, 4, 5}};
    static const int hex_split[6][4] = {{0, 1, 2, 4}, {1, 2, 4, 5}, {2, 4, 5, 6}, {0, 2, 3, 4}, {2, 3, 4, 6}, {3, 4, 6, 7}};
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < ncell; c++) {
        const int64_t *v = cells + 8 * c;
        const int(*sp)[4];
        int ns;
        switch (types[c]) {
        case T_TET: sp = tet_split; ns = 1; break;
        case T_PYR: sp = pyr_split; ns = 2; break;
        case T_PRISM: sp = pri_split; ns = 3; break;
        default: sp = hex_split; ns = 6; break;
        }
        double acc[5] = {0, 0, 0, 0, 0};
        double vol = 0.0;
        for (int t = 0; t < ns; t++)
            vol += tet_integrate(&f, nodes + 3 * v[sp[t][0]], nodes + 3 * v[sp[t][1]], nodes + 3 * v[sp[t][2]],
                                 nodes + 3 * v[sp[t][3]], order, gx, gw, acc);
        for (int q = 0; q < 5; q++) out[q * ncell + c] = acc[q] / vol;
    }
    return 0;
}
