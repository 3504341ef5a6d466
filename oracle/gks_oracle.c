/*
 * FP64 reference ("oracle") for the third-order gas-kinetic scheme on hybrid
 * unstructured meshes (Yang, Pan & Xu, arXiv 2203.09047).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded
 * implementation written from the paper so that the GPU library can be
 * checked against it.  Only the test suite, the smoke check and the CPU leg of
 * the benchmark may load it.  It shares no code, table or helper with the GPU
 * library; both consume the same mesh records and initial cell averages.
 *
 * What it follows, in the paper's order:
 *   - cell and face labels of the four element types (Section 2);
 *   - big stencil and sub-stencils (Section 2);
 *   - quadratic least-squares polynomial P_0 and linear polynomials P_m
 *     (Section 2, Eq. lin-def), nonlinear combination (Eq. weno), linear
 *     weights, nonlinear weights and smoothness indicators (Eq. indicator);
 *   - 3x3x3 Gauss integration on the trilinear map (Eq. trilinear) with the
 *     element types as degenerate hexahedra (Section 2);
 *   - bilinear face map and 2x2 Gauss flux integration (Eq. flux-qud);
 *   - the BGK model and its moments (Eq. bgk-3d, Eq. compatibility), the
 *     time-dependent distribution at a face Gauss point (Eq. flux-1), the
 *     slopes from reconstructed directional derivatives and compatibility,
 *     the interface equilibrium and its slopes (Section 3.2);
 *   - the collision time of the opening of Section 5;
 *   - the semi-discrete operator (Eq. semi, Eq. finite) and the two-stage
 *     fourth-order time stepping the paper cites for unsteady flow
 *     (Section 3.3: Li & Du 2016; Pan, Xu, Li & Li 2016).
 *
 * Readings where the paper is silent or garbled (identical on the GPU side):
 *   - hexahedron vertices p1..p8 map cyclically to reference corners:
 *     p1(-,-,-) p2(+,-,-) p3(+,+,-) p4(-,+,-), p5..p8 the same at zeta=+1/2;
 *   - prism face F3 is {p1 p2 p5 p4} (the printed p6 is a typo);
 *   - face Gauss nodes are at +-sqrt(3)/6 on [-1/2,1/2]^2 with weights 1/4;
 *     a triangle (a,b,c), sorted by canonical node id, is the quad (a,b,c,c);
 *   - big stencil = set of face neighbours and their face neighbours, minus
 *     the cell itself; sub-stencil rings of a neighbour use all of that
 *     neighbour's other face neighbours;
 *   - the sub-stencil constraint is: cell average of P_m over each member
 *     equals that member's average;
 *   - WENO acts on conservative variables componentwise; every multi-index
 *     of the smoothness indicator counts once; exponent p (default 1) and
 *     epsilon (default 1e-6) of the nonlinear weights are parameters;
 *   - tangential frame: e = coordinate axis with the smallest |n1.e|,
 *     n2 = unit(e - (e.n1) n1), n3 = n1 x n2;
 *   - time step dt = CFL min_i h_i / (|U_i| + c_i), h_i = 6|Omega_i| / sum|S_f|;
 *   - collision time per Gauss point from that point's p_l, p_r (and the
 *     pressure of g0 for the viscous part);
 *   - Prandtl number fix: the energy flux gains (1/Pr - 1) q with q the heat
 *     flux of the time-integrated distribution about the g0 velocity;
 *   - flux and its time derivative from the two time integrals over dt/2
 *     and dt (two-stage fourth-order GKS).
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Scalar type of every quantity that depends on the conserved state.  The default build is plain
 * FP64.  Built with -DORC_COMPLEX_STEP, the same code runs on complex numbers x + i h v with a tiny
 * h: the imaginary parts then carry h times the directional derivative along v of every quantity,
 * exact to rounding since no difference of nearby values is formed (the complex-step derivative of
 * Squire & Trapp 1998 and Martins, Sturdza & Alonso 2003; with h = 1e-200 every product of two
 * imaginary parts underflows to zero, so the arithmetic is that of dual numbers).  Each elementary
 * function below extends its FP64 value by its first-order Taylor term in the imaginary part, |x|
 * by sign(Re x) x with sign(0) = 0, and every branch and comparison looks at the real part, so the
 * real parts are those of the FP64 build.  Geometry, stencils, least-squares operators and the
 * time step stay FP64 in both builds.
 */
#ifdef ORC_COMPLEX_STEP
#include <complex.h>
typedef double _Complex real;
static inline double RE(real x) { return creal(x); }
static inline real r_sqrt(real x)
{
    const double s = sqrt(creal(x));
    return CMPLX(s, cimag(x) / (2.0 * s));
}
static inline real r_exp(real x)
{
    const double e = exp(creal(x));
    return CMPLX(e, cimag(x) * e);
}
static inline real r_expm1(real x) { return CMPLX(expm1(creal(x)), cimag(x) * exp(creal(x))); }
/* d erfc(a) / da = -2/sqrt(pi) exp(-a^2) */
static inline real r_erfc(real x)
{
    const double a = creal(x);
    return CMPLX(erfc(a), -cimag(x) * M_2_SQRTPI * exp(-a * a));
}
static inline real r_abs(real x)
{
    const double a = creal(x);
    return a > 0.0 ? x : (a < 0.0 ? -x : CMPLX(0.0, 0.0));
}
static inline real r_pow(real x, double e)
{
    const double a = creal(x);
    return CMPLX(pow(a, e), cimag(x) * e * pow(a, e - 1.0));
}
#else
typedef double real;
static inline double RE(real x) { return x; }
static inline real r_sqrt(real x) { return sqrt(x); }
static inline real r_exp(real x) { return exp(x); }
static inline real r_expm1(real x) { return expm1(x); }
static inline real r_erfc(real x) { return erfc(x); }
static inline real r_abs(real x) { return fabs(x); }
static inline real r_pow(real x, double e) { return pow(x, e); }
#endif

enum { TET = 0, PYR = 1, PRISM = 2, HEX = 3 };

/* Boundary conditions of the six box planes of a mesh with walls (plane 2 d + hi: axis d, at 0 or at
 * L).  Every one keeps the paper's ghost-cell construction (Section 2): the ghost across a plane is
 * the mirror image of an interior cell, its flow variables set by the condition from the mirrored
 * cell's.  At a face Gauss point on the plane the state beyond it is the condition applied to the
 * inner reconstructed state, with the mirror's sign on the derivatives across the plane. */
enum { BC_SLIP = 0,       /* reflective: normal momentum negated (the Riemann problems' walls) */
       BC_NOSLIP = 1,     /* no-slip adiabatic wall moving with velocity uw: U -> 2 uw - U, rho and p kept */
       BC_ISOTHERMAL = 2, /* no-slip wall at temperature Tw: U -> 2 uw - U, T -> 2 Tw - T, p kept (the cavity) */
       BC_FARFIELD = 3,   /* far field by Riemann invariants against the free stream far (the sphere's inlet/outlet) */
       BC_EXTRAPOLATE = 4 /* zero-gradient outflow: the ghost repeats the mirrored cell (non-reflecting ends) */ };

typedef struct {
    int type;
    double uw[3]; /* wall velocity (no-slip types) */
    double Tw;    /* wall temperature p / rho (isothermal) */
    double far[5]; /* free stream rho, U, V, W, p (far field) */
} orc_bc;

typedef struct {
    double gamma, cfl, mu, Pr;
    double weno_eps, weno_gamma_m, weno_p;
    double tau_eps, tau_C;
    int viscous;
    int force_linear; /* use the linear weights gamma_m instead of the nonlinear ones */
    int fallback;     /* 1: a side state at a Gauss point with rho <= 0 or p <= 0 is replaced by its
                         cell's average with zero slopes (first order there), and counted */
    double fallback_floor; /* with fallback: also when rho or p is at most this fraction of the
                              cell average's */
    int smooth;       /* 1: the smooth-flow distribution (Eq. flux-2) instead of the full one (Eq. flux-1) */
    double mu_power;  /* viscous: mu (T / T_ref)^mu_power at the interface temperature T = p0 / rho0 (gas
                         constant 1), the power law of the paper's hypersonic sphere case; 0: constant mu */
    double T_ref;
    orc_bc bc[6];     /* the box planes' conditions on meshes with walls (plane 2 axis + hi) */
} orc_params;

/* ------------------------------------------------------------------ */
/* element tables (Section 2)                                           */
/* ------------------------------------------------------------------ */
static const int NFACE[4] = {4, 5, 5, 6};
/* faces in the paper's labels (1-based vertex labels), 0 marks "triangle" */
static const int FACE_LAB[4][6][4] = {
    /* tetrahedron */
    {{1, 2, 3, 0}, {1, 2, 4, 0}, {2, 3, 4, 0}, {3, 1, 4, 0}},
    /* pyramid */
    {{1, 2, 5, 0}, {2, 3, 5, 0}, {3, 4, 5, 0}, {4, 1, 5, 0}, {1, 2, 3, 4}},
    /* prism (F3 corrected to p1 p2 p5 p4) */
    {{1, 2, 3, 0}, {4, 5, 6, 0}, {1, 2, 5, 4}, {2, 3, 6, 5}, {3, 1, 4, 6}},
    /* hexahedron */
    {{1, 2, 3, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 4, 8, 7}, {4, 1, 5, 8}, {5, 6, 7, 8}},
};
/* degenerate-hexahedron relabelling (Section 2), 1-based */
static const int DEGEN[4][8] = {
    {1, 2, 3, 3, 4, 4, 4, 4},
    {1, 2, 3, 4, 5, 5, 5, 5},
    {1, 2, 3, 3, 4, 5, 6, 6},
    {1, 2, 3, 4, 5, 6, 7, 8},
};
/* reference corner of each hexahedron slot (cyclic bottom, then top) */
static const int CORNER[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                 {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

/* the nine monomials of degree 1 and 2: x y z xx xy xz yy yz zz */
static const int MONO[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {1, 1, 0},
                               {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};

/* ------------------------------------------------------------------ */
/* mesh state                                                           */
/* ------------------------------------------------------------------ */
/* A stencil member or face neighbour: the image x -> sg x + of L of a cell,
 * sg = +-1 per axis (a reflection across a wall plane) and of an offset in
 * units of the box (periodic images; 0 or 2 for the mirror across the wall at
 * 0 or at L).  Momentum components of the image carry the signs sg. */
typedef struct {
    int64_t cell;
    int sg[3];
    int of[3];
} sref;

#define MAXST 96
#define MAXSUB 16

typedef struct {
    int n;          /* rows */
    int k;          /* unknowns */
    double *qr;     /* n x k, column-major Householder factors */
    double *tau;    /* k */
    double scale[9]; /* unknown j of the scaled fit equals scale[j] times the coefficient */
    int ok;
} lsq;

typedef struct {
    int type;
    double vol, xc[3], m2[6]; /* m2: means of (x-xc)(x-xc): xx xy xz yy yz zz */
    double area_sum;
    int nf;
    int64_t face[6];
    int fside[6];  /* 0 owner, 1 neighbour */
    sref nb[6];    /* neighbour across face p (paper's F_p order) */
    int K;
    int grown; /* members appended to make the fits well posed */
    sref st[MAXST];
    lsq ls0;
    int M;
    int subn[8];
    sref sub[8][MAXSUB];
    lsq ls[8];
} ocell;

typedef struct {
    int64_t owner, nbr;
    int owner_lf;
    sref nb;                 /* the neighbour seen from the owner: an image of nbr, or at a wall
                                (nbr = -1) the owner's mirror image across it */
    int64_t key[4];          /* canonical node ids (sorted), -1 for triangles */
    double gp[4][3];         /* Gauss points in the owner's frame */
    double va[4][3];         /* vector area 1/4 X_eta x X_zeta, owner -> neighbour */
} oface;

typedef struct {
    int64_t n_nodes, n_cells, n_faces;
    double L[3];
    int periodic;
    const double *nodes;
    double *nodes_copy;
    int8_t *types;
    int64_t *cells;
    int64_t *canon;
    ocell *c;
    oface *f;
    /* per-stage WENO data */
    real *a;  /* [n][5][9] */
    real *b;  /* [n][5][8][3] */
    real *w;  /* [n][5][9] normalised weights omega_0..omega_M */
    int64_t n_fallback; /* Gauss-point sides that fell back to first order since the last query */
    /* option: a big stencil with fewer members than this is grown like an
     * ill-posed fit (0: the paper's neighbours-of-neighbours set as it is) */
    int min_big;
    /* stencils built for a subset of the cells only: per-cell reconstructions of those cells,
       no residual or step */
    int partial;
} orc;

static char g_err[256];
static void seterr(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* small dense linear algebra                                           */
/* ------------------------------------------------------------------ */
/* Householder QR of a column-major n x k matrix (n >= k), in place. */
static void house_qr(double *A, int n, int k, double *tau)
{
    for (int j = 0; j < k; j++) {
        double nrm = 0.0;
        for (int i = j; i < n; i++) nrm += A[i + n * j] * A[i + n * j];
        nrm = sqrt(nrm);
        if (nrm == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        double alpha = A[j + n * j] > 0 ? -nrm : nrm;
        double v0 = A[j + n * j] - alpha;
        /* v = (1, A[j+1..]/v0) */
        for (int i = j + 1; i < n; i++) A[i + n * j] /= v0;
        tau[j] = -v0 / alpha;
        A[j + n * j] = alpha;
        for (int c = j + 1; c < k; c++) {
            double s = A[j + n * c];
            for (int i = j + 1; i < n; i++) s += A[i + n * j] * A[i + n * c];
            s *= tau[j];
            A[j + n * c] -= s;
            for (int i = j + 1; i < n; i++) A[i + n * c] -= s * A[i + n * j];
        }
    }
}

/* least-squares solve with the factors of house_qr; b (length n) is overwritten */
static void house_solve(const double *A, int n, int k, const double *tau, real *b, real *x)
{
    for (int j = 0; j < k; j++) {
        real s = b[j];
        for (int i = j + 1; i < n; i++) s += A[i + n * j] * b[i];
        s *= tau[j];
        b[j] -= s;
        for (int i = j + 1; i < n; i++) b[i] -= s * A[i + n * j];
    }
    for (int j = k - 1; j >= 0; j--) {
        real s = b[j];
        for (int c = j + 1; c < k; c++) s -= A[j + n * c] * x[c];
        x[j] = s / A[j + n * j];
    }
}

/* Gaussian elimination with partial pivoting, n <= 8, row-major A */
static int gauss_solve(int n, real *A, real *b, real *x)
{
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(RE(A[r * n + c])) > fabs(RE(A[p * n + c]))) p = r;
        if (RE(A[p * n + c]) == 0.0) return 1;
        if (p != c) {
            for (int q = 0; q < n; q++) {
                real t = A[c * n + q];
                A[c * n + q] = A[p * n + q];
                A[p * n + q] = t;
            }
            real t = b[c];
            b[c] = b[p];
            b[p] = t;
        }
        for (int r = c + 1; r < n; r++) {
            real f = A[r * n + c] / A[c * n + c];
            for (int q = c; q < n; q++) A[r * n + q] -= f * A[c * n + q];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        real s = b[r];
        for (int q = r + 1; q < n; q++) s -= A[r * n + q] * x[q];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* geometry: trilinear map and 3x3x3 Gauss rule (Eq. trilinear)        */
/* ------------------------------------------------------------------ */
static void cell_slots(const orc *o, int64_t c, double X[8][3])
{
    int t = o->types[c];
    for (int s = 0; s < 8; s++) {
        int64_t nd = o->cells[8 * c + DEGEN[t][s] - 1];
        for (int q = 0; q < 3; q++) X[s][q] = o->nodes[3 * nd + q];
    }
}

/* position and |Jacobian| of the trilinear map at (xi,eta,zeta) in [-1/2,1/2]^3 */
static double trilinear(double X[8][3], const double r[3], double x[3])
{
    double J[3][3] = {{0}};
    x[0] = x[1] = x[2] = 0.0;
    for (int s = 0; s < 8; s++) {
        double f[3], d[3];
        for (int q = 0; q < 3; q++) {
            f[q] = 0.5 * (1.0 + 2.0 * CORNER[s][q] * r[q]);
            d[q] = CORNER[s][q];
        }
        double psi = f[0] * f[1] * f[2];
        double dpsi[3] = {d[0] * f[1] * f[2], f[0] * d[1] * f[2], f[0] * f[1] * d[2]};
        for (int q = 0; q < 3; q++) {
            x[q] += X[s][q] * psi;
            for (int p = 0; p < 3; p++) J[q][p] += X[s][q] * dpsi[p];
        }
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    return fabs(det);
}

static void cell_moments(const orc *o, int64_t c, ocell *C)
{
    const double g = 0.5 * sqrt(3.0 / 5.0);
    const double gx[3] = {-g, 0.0, g};
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double X[8][3];
    cell_slots(o, c, X);
    double vol = 0.0, m1[3] = {0, 0, 0};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) {
                double r[3] = {gx[i], gx[j], gx[k]}, x[3];
                double wj = gw[i] * gw[j] * gw[k] * trilinear(X, r, x);
                vol += wj;
                for (int q = 0; q < 3; q++) m1[q] += wj * x[q];
            }
    for (int q = 0; q < 3; q++) C->xc[q] = m1[q] / vol;
    double m2[6] = {0};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) {
                double r[3] = {gx[i], gx[j], gx[k]}, x[3];
                double wj = gw[i] * gw[j] * gw[k] * trilinear(X, r, x);
                double d[3] = {x[0] - C->xc[0], x[1] - C->xc[1], x[2] - C->xc[2]};
                m2[0] += wj * d[0] * d[0];
                m2[1] += wj * d[0] * d[1];
                m2[2] += wj * d[0] * d[2];
                m2[3] += wj * d[1] * d[1];
                m2[4] += wj * d[1] * d[2];
                m2[5] += wj * d[2] * d[2];
            }
    C->vol = vol;
    for (int q = 0; q < 6; q++) C->m2[q] = m2[q] / vol;
}

/* ------------------------------------------------------------------ */
/* mesh connectivity                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t key[4];
    int64_t cell;
    int lf;
} frec;

static int cmp_key4(const int64_t *a, const int64_t *b)
{
    for (int q = 0; q < 4; q++) {
        if (a[q] < b[q]) return -1;
        if (a[q] > b[q]) return 1;
    }
    return 0;
}

static int cmp_frec(const void *pa, const void *pb)
{
    const frec *a = pa, *b = pb;
    int c = cmp_key4(a->key, b->key);
    if (c) return c;
    if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
    return a->lf - b->lf;
}

typedef struct {
    int64_t q[3];
    int64_t id;
} nrec;

static int cmp_nrec(const void *pa, const void *pb)
{
    const nrec *a = pa, *b = pb;
    for (int k = 0; k < 3; k++)
        if (a->q[k] != b->q[k]) return a->q[k] < b->q[k] ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

static int cmp_i64(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return a < b ? -1 : (a > b);
}

/* node ids of local face lf of cell c, in the face table's order; returns 3 or 4 */
static int face_nodes(const orc *o, int64_t c, int lf, int64_t v[4])
{
    int t = o->types[c];
    int n = FACE_LAB[t][lf][3] ? 4 : 3;
    for (int q = 0; q < n; q++) v[q] = o->cells[8 * c + FACE_LAB[t][lf][q] - 1];
    return n;
}

static int same_sref(const sref *a, const sref *b)
{
    return a->cell == b->cell && a->sg[0] == b->sg[0] && a->sg[1] == b->sg[1] && a->sg[2] == b->sg[2] &&
           a->of[0] == b->of[0] && a->of[1] == b->of[1] && a->of[2] == b->of[2];
}

static sref sref_self(int64_t c)
{
    sref s = {c, {1, 1, 1}, {0, 0, 0}};
    return s;
}

static int add_unique(sref *list, int *n, int cap, sref s)
{
    for (int q = 0; q < *n; q++)
        if (same_sref(&list[q], &s)) return 0;
    if (*n >= cap) return -1;
    list[(*n)++] = s;
    return 1;
}

/* rel seen from base's cell, then base's image map: x -> sg_b (sg_r x + of_r L) + of_b L */
static sref compose(sref base, sref rel)
{
    sref r;
    r.cell = rel.cell;
    for (int q = 0; q < 3; q++) {
        r.sg[q] = base.sg[q] * rel.sg[q];
        r.of[q] = base.sg[q] * rel.of[q] + base.of[q];
    }
    return r;
}

/* centroid of a stencil member in the frame of the cell owning the stencil */
static void image_centroid(const orc *o, sref s, double x[3])
{
    for (int q = 0; q < 3; q++) x[q] = s.sg[q] * o->c[s.cell].xc[q] + s.of[q] * o->L[q];
}

/* mean over the member's cell of (x - x0)^n for the nine monomials */
static void member_means(const orc *o, sref s, const double x0[3], double out[9])
{
    const ocell *K = &o->c[s.cell];
    double xk[3];
    image_centroid(o, s, xk);
    double D[3] = {xk[0] - x0[0], xk[1] - x0[1], xk[2] - x0[2]};
    /* second central moments of the member (a reflection flips the mixed ones it touches) */
    double S[3][3] = {{K->m2[0], K->m2[1], K->m2[2]}, {K->m2[1], K->m2[3], K->m2[4]}, {K->m2[2], K->m2[4], K->m2[5]}};
    for (int p = 0; p < 3; p++)
        for (int q = 0; q < 3; q++) S[p][q] *= s.sg[p] * s.sg[q];
    for (int n = 0; n < 9; n++) {
        int e[3] = {MONO[n][0], MONO[n][1], MONO[n][2]};
        int deg = e[0] + e[1] + e[2];
        if (deg == 1) {
            out[n] = e[0] ? D[0] : (e[1] ? D[1] : D[2]);
        } else {
            int ax[2], na = 0;
            for (int q = 0; q < 3; q++)
                for (int r = 0; r < e[q]; r++) ax[na++] = q;
            out[n] = S[ax[0]][ax[1]] + D[ax[0]] * D[ax[1]];
        }
    }
}

/* Householder factors of an already scaled n x k row-major matrix */
static int lsq_build(lsq *L, int n, int k, const double *A_rowmajor)
{
    L->n = n;
    L->k = k;
    L->ok = 0;
    if (n < k) return 1;
    L->qr = malloc(sizeof(double) * n * k);
    L->tau = malloc(sizeof(double) * k);
    for (int j = 0; j < k; j++)
        for (int i = 0; i < n; i++) L->qr[i + n * j] = A_rowmajor[i * k + j];
    house_qr(L->qr, n, k, L->tau);
    L->ok = 1;
    return 0;
}

static void lsq_apply(const lsq *L, const real *rhs, real *x)
{
    real b[MAXST];
    for (int i = 0; i < L->n; i++) b[i] = rhs[i];
    real y[9];
    house_solve(L->qr, L->n, L->k, L->tau, b, y);
    for (int j = 0; j < L->k; j++) x[j] = y[j] / L->scale[j];
}

static void lsq_free(lsq *L)
{
    free(L->qr);
    free(L->tau);
}

/* face-neighbour ring of neighbour j (seen from cell i): all of j's face neighbours except i */
static int ring_of(const orc *o, int64_t i, sref j, sref *out)
{
    int n = 0;
    const ocell *J = &o->c[j.cell];
    for (int p = 0; p < J->nf; p++) {
        sref s = compose(j, J->nb[p]);
        sref self = sref_self(i);
        if (same_sref(&s, &self)) continue;
        out[n++] = s;
    }
    return n;
}

/* sub-stencil neighbour labels (1-based F_p) and the neighbour whose ring joins it (0 = none) */
static const int SUB_HEX[8][4] = {{1, 2, 3, 0}, {1, 3, 4, 0}, {1, 4, 5, 0}, {1, 5, 2, 0},
                                  {6, 2, 3, 0}, {6, 3, 4, 0}, {6, 4, 5, 0}, {6, 5, 2, 0}};
static const int SUB_PRISM[6][4] = {{1, 3, 4, 0}, {1, 4, 5, 0}, {1, 5, 3, 0}, {2, 3, 4, 0}, {2, 4, 5, 0}, {2, 5, 3, 0}};
static const int SUB_TET[4][4] = {{1, 2, 3, 1}, {1, 2, 4, 2}, {2, 3, 4, 3}, {3, 1, 4, 4}};
static const int SUB_PYR[8][4] = {{1, 2, 3, 1}, {2, 3, 4, 2}, {3, 4, 1, 3}, {4, 1, 2, 4},
                                  {1, 2, 5, 1}, {2, 3, 5, 2}, {3, 4, 5, 3}, {4, 1, 5, 4}};

/*
 * Scaled least-squares matrix rows of a member list: for each member k and
 * each of the first k monomials, mean over Omega_k of (x-x0)^n minus the mean
 * over Omega_0, with (x-x0) measured in units of h.
 */
static void lsq_rows(const orc *o, const ocell *C, const sref *list, int n, int k, double h, double *A)
{
    double S[3][3] = {{C->m2[0], C->m2[1], C->m2[2]}, {C->m2[1], C->m2[3], C->m2[4]}, {C->m2[2], C->m2[4], C->m2[5]}};
    for (int r = 0; r < n; r++) {
        double mk[9];
        member_means(o, list[r], C->xc, mk);
        for (int j = 0; j < k; j++) {
            double own = 0.0;
            int deg = MONO[j][0] + MONO[j][1] + MONO[j][2];
            if (deg == 2) {
                int ax[2], na = 0;
                for (int q = 0; q < 3; q++)
                    for (int t = 0; t < MONO[j][q]; t++) ax[na++] = q;
                own = S[ax[0]][ax[1]];
            }
            A[r * k + j] = (mk[j] - own) / (deg == 1 ? h : h * h);
        }
    }
}

/* eigenvalues of a symmetric k x k matrix (k <= 9) by cyclic Jacobi rotations */
static void sym_eig(double *G, int k, double *ev)
{
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < k; p++)
            for (int q = 0; q < k; q++) {
                tot += G[p * k + q] * G[p * k + q];
                if (p != q) off += G[p * k + q] * G[p * k + q];
            }
        if (off <= 1e-34 * tot) break;
        for (int p = 0; p < k; p++)
            for (int q = p + 1; q < k; q++) {
                double apq = G[p * k + q];
                if (apq == 0.0) continue;
                double th = (G[q * k + q] - G[p * k + p]) / (2.0 * apq);
                double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < k; r++) {
                    double grp = G[r * k + p], grq = G[r * k + q];
                    G[r * k + p] = c * grp - s * grq;
                    G[r * k + q] = s * grp + c * grq;
                }
                for (int r = 0; r < k; r++) {
                    double gpr = G[p * k + r], gqr = G[q * k + r];
                    G[p * k + r] = c * gpr - s * gqr;
                    G[q * k + r] = s * gpr + c * gqr;
                }
            }
    }
    for (int p = 0; p < k; p++) ev[p] = G[p * k + p];
}

/*
 * A least-squares fit is accepted when it has at least as many rows as
 * unknowns and the singular values of the scaled matrix satisfy
 * sigma_min >= 1e-6 sigma_max (squared: eigenvalues of A^T A).
 */
static int well_posed(const double *A, int n, int k)
{
    if (n < k) return 0;
    double G[81], ev[9];
    for (int p = 0; p < k; p++)
        for (int q = 0; q < k; q++) {
            double s = 0.0;
            for (int r = 0; r < n; r++) s += A[r * k + p] * A[r * k + q];
            G[p * k + q] = s;
        }
    sym_eig(G, k, ev);
    double lo = INFINITY, hi = 0.0;
    for (int p = 0; p < k; p++) {
        if (ev[p] < lo) lo = ev[p];
        if (ev[p] > hi) hi = ev[p];
    }
    return hi > 0.0 && lo >= 1e-12 * hi;
}

/*
 * Grow a member list until its fit is well posed and has at least min_rows
 * members: candidates are the face neighbours of the current members (members
 * in order, faces in F_p order), excluding the cell itself and existing
 * members; they are appended one at a time.  When the candidates run out a
 * well-posed fit is kept below min_rows.  Returns the number appended, or -1
 * when the candidates run out before the fit is well posed.
 */
static int grow_until_posed(const orc *o, int64_t i, const ocell *C, sref *list, int *n, int cap, int k, double h,
                            int min_rows)
{
    sref self = sref_self(i);
    sref cand[MAXST * 6];
    int nc = 0;
    for (int r = 0; r < *n; r++) {
        const ocell *J = &o->c[list[r].cell];
        for (int p = 0; p < J->nf; p++) {
            sref s = compose(list[r], J->nb[p]);
            if (same_sref(&s, &self)) continue;
            int dup = 0;
            for (int q = 0; q < *n && !dup; q++) dup = same_sref(&list[q], &s);
            for (int q = 0; q < nc && !dup; q++) dup = same_sref(&cand[q], &s);
            if (!dup) cand[nc++] = s;
        }
    }
    int added = 0;
    double A[MAXST * 9];
    for (;;) {
        lsq_rows(o, C, list, *n, k, h, A);
        const int posed = well_posed(A, *n, k);
        if (posed && *n >= min_rows) return added;
        if (added >= nc || *n >= cap) return posed ? added : -1;
        list[(*n)++] = cand[added++];
    }
}

static int build_stencils(orc *o, int64_t i)
{
    ocell *C = &o->c[i];
    sref self = sref_self(i);
    C->K = 0;
    for (int p = 0; p < C->nf; p++)
        if (add_unique(C->st, &C->K, MAXST, C->nb[p]) < 0) return 1;
    for (int p = 0; p < C->nf; p++) {
        const ocell *J = &o->c[C->nb[p].cell];
        for (int q = 0; q < J->nf; q++) {
            sref s = compose(C->nb[p], J->nb[q]);
            if (same_sref(&s, &self)) continue;
            if (add_unique(C->st, &C->K, MAXST, s) < 0) return 1;
        }
    }
    const int(*tab)[4];
    switch (C->type) {
    case HEX: tab = SUB_HEX; C->M = 8; break;
    case PRISM: tab = SUB_PRISM; C->M = 6; break;
    case TET: tab = SUB_TET; C->M = 4; break;
    default: tab = SUB_PYR; C->M = 8; break;
    }
    for (int m = 0; m < C->M; m++) {
        C->subn[m] = 0;
        for (int q = 0; q < 3; q++) add_unique(C->sub[m], &C->subn[m], MAXSUB, C->nb[tab[m][q] - 1]);
        if (tab[m][3]) {
            sref ring[8];
            int nr = ring_of(o, i, C->nb[tab[m][3] - 1], ring);
            for (int q = 0; q < nr; q++)
                if (!same_sref(&ring[q], &self)) add_unique(C->sub[m], &C->subn[m], MAXSUB, ring[q]);
        }
    }
    /* least-squares fits in (x - x0)/h; ill-posed ones are grown by the next ring */
    double h = cbrt(C->vol);
    C->grown = 0;
    int g = grow_until_posed(o, i, C, C->st, &C->K, MAXST, 9, h, o->min_big);
    if (g < 0) return 2;
    C->grown += g;
    double A[MAXST * 9];
    lsq_rows(o, C, C->st, C->K, 9, h, A);
    if (lsq_build(&C->ls0, C->K, 9, A)) return 2;
    for (int m = 0; m < C->M; m++) {
        g = grow_until_posed(o, i, C, C->sub[m], &C->subn[m], MAXSUB, 3, h, 0);
        if (g < 0) return 3;
        C->grown += g;
        lsq_rows(o, C, C->sub[m], C->subn[m], 3, h, A);
        if (lsq_build(&C->ls[m], C->subn[m], 3, A)) return 3;
        for (int j = 0; j < 3; j++) C->ls[m].scale[j] = h;
    }
    for (int j = 0; j < 9; j++) C->ls0.scale[j] = (j < 3) ? h : h * h;
    return 0;
}

/* bilinear face map (Eq. flux-qud): quad x1..x4 cyclic, corners (-,-) (+,-) (+,+) (-,+) */
static void face_gauss(const double Xq[4][3], double gp[4][3], double va[4][3])
{
    static const int cs[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
    const double g = sqrt(3.0) / 6.0;
    static const int gs[4][2] = {{-1, -1}, {1, -1}, {-1, 1}, {1, 1}};
    for (int k = 0; k < 4; k++) {
        double r[2] = {gs[k][0] * g, gs[k][1] * g};
        double x[3] = {0, 0, 0}, xe[3] = {0, 0, 0}, xz[3] = {0, 0, 0};
        for (int m = 0; m < 4; m++) {
            double fe = 0.5 * (1.0 + 2.0 * cs[m][0] * r[0]);
            double fz = 0.5 * (1.0 + 2.0 * cs[m][1] * r[1]);
            for (int q = 0; q < 3; q++) {
                x[q] += Xq[m][q] * fe * fz;
                xe[q] += Xq[m][q] * cs[m][0] * fz;
                xz[q] += Xq[m][q] * fe * cs[m][1];
            }
        }
        double cr[3] = {xe[1] * xz[2] - xe[2] * xz[1], xe[2] * xz[0] - xe[0] * xz[2], xe[0] * xz[1] - xe[1] * xz[0]};
        for (int q = 0; q < 3; q++) {
            gp[k][q] = x[q];
            va[k][q] = 0.25 * cr[q];
        }
    }
}

void orc_destroy(orc *o);

/* want (optional): build the stencils and fits of the cells with want[c] != 0 only */
orc *orc_create_cells(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types, const int64_t *cells,
                      const double *box, int periodic, int min_big, const unsigned char *want)
{
    orc *o = calloc(1, sizeof(orc));
    o->min_big = min_big;
    o->partial = want != NULL;
    o->n_nodes = n_nodes;
    o->n_cells = n_cells;
    o->periodic = periodic;
    for (int q = 0; q < 3; q++) o->L[q] = box[q];
    o->nodes_copy = malloc(sizeof(double) * 3 * n_nodes);
    memcpy(o->nodes_copy, nodes, sizeof(double) * 3 * n_nodes);
    o->nodes = o->nodes_copy;
    o->types = malloc(n_cells);
    memcpy(o->types, types, n_cells);
    o->cells = malloc(sizeof(int64_t) * 8 * n_cells);
    memcpy(o->cells, cells, sizeof(int64_t) * 8 * n_cells);
    /* canonical node ids: smallest id among nodes at the same (wrapped) position */
    o->canon = malloc(sizeof(int64_t) * n_nodes);
    {
        const double S = 16777216.0;
        nrec *nr = malloc(sizeof(nrec) * n_nodes);
        for (int64_t n = 0; n < n_nodes; n++) {
            for (int q = 0; q < 3; q++) {
                long long v = llround(o->nodes[3 * n + q] / o->L[q] * S);
                if (periodic) v = ((v % (long long)S) + (long long)S) % (long long)S;
                nr[n].q[q] = v;
            }
            nr[n].id = n;
        }
        qsort(nr, n_nodes, sizeof(nrec), cmp_nrec);
        for (int64_t a = 0; a < n_nodes;) {
            int64_t b = a;
            while (b < n_nodes && !memcmp(nr[b].q, nr[a].q, sizeof nr[a].q)) b++;
            for (int64_t q = a; q < b; q++) o->canon[nr[q].id] = nr[a].id;
            a = b;
        }
        free(nr);
    }
    o->c = calloc(n_cells, sizeof(ocell));
    int64_t nrec_total = 0;
    for (int64_t c = 0; c < n_cells; c++) {
        if (types[c] < 0 || types[c] > 3) {
            seterr("bad cell type");
            orc_destroy(o);
            return NULL;
        }
        o->c[c].type = types[c];
        o->c[c].nf = NFACE[(int)types[c]];
        nrec_total += o->c[c].nf;
        cell_moments(o, c, &o->c[c]);
    }
    frec *fr = malloc(sizeof(frec) * nrec_total);
    int64_t r = 0;
    for (int64_t c = 0; c < n_cells; c++)
        for (int lf = 0; lf < o->c[c].nf; lf++) {
            int64_t v[4];
            int n = face_nodes(o, c, lf, v);
            for (int q = 0; q < 4; q++) fr[r].key[q] = q < n ? o->canon[v[q]] : -1;
            qsort(fr[r].key, n, sizeof(int64_t), cmp_i64);
            fr[r].cell = c;
            fr[r].lf = lf;
            r++;
        }
    qsort(fr, nrec_total, sizeof(frec), cmp_frec);
    o->f = malloc(sizeof(oface) * (nrec_total + 1));
    int64_t nf = 0;
    for (int64_t a = 0; a < nrec_total;) {
        const int pair = a + 1 < nrec_total && !cmp_key4(fr[a].key, fr[a + 1].key);
        if ((pair && a + 2 < nrec_total && !cmp_key4(fr[a].key, fr[a + 2].key)) || (!pair && periodic)) {
            seterr("face is not shared by exactly two cells (boundary faces need periodic matching)");
            free(fr);
            orc_destroy(o);
            return NULL;
        }
        oface *F = &o->f[nf];
        F->owner = fr[a].cell;
        F->owner_lf = fr[a].lf;
        F->nbr = pair ? fr[a + 1].cell : -1;
        memcpy(F->key, fr[a].key, sizeof F->key);
        int64_t vo[4];
        int n = face_nodes(o, F->owner, fr[a].lf, vo);
        if (pair) {
            /* image shift: owner vertex minus the neighbour's vertex of the same canonical id */
            int64_t vn[4];
            face_nodes(o, F->nbr, fr[a + 1].lf, vn);
            int64_t m = -1;
            for (int q = 0; q < n && m < 0; q++)
                if (o->canon[vn[q]] == o->canon[vo[0]]) m = vn[q];
            F->nb = sref_self(F->nbr);
            for (int q = 0; q < 3; q++) F->nb.of[q] = (int)lround((o->nodes[3 * vo[0] + q] - o->nodes[3 * m + q]) / o->L[q]);
        } else {
            /* a wall: every vertex on the plane x_axis = 0 or L; the neighbour is the owner's mirror */
            int axis = -1, side = 0;
            for (int q = 0; q < 3 && axis < 0; q++) {
                int lo = 1, hi = 1;
                for (int v = 0; v < n; v++) {
                    const double x = o->nodes[3 * vo[v] + q];
                    if (fabs(x) > 1e-12 * o->L[q]) lo = 0;
                    if (fabs(x - o->L[q]) > 1e-12 * o->L[q]) hi = 0;
                }
                if (lo || hi) {
                    axis = q;
                    side = hi;
                }
            }
            if (axis < 0) {
                seterr("boundary face not on a wall of the box");
                free(fr);
                orc_destroy(o);
                return NULL;
            }
            F->nb = sref_self(F->owner);
            F->nb.sg[axis] = -1;
            F->nb.of[axis] = side ? 2 : 0;
        }
        /* face geometry from the owner's vertices */
        double Xq[4][3];
        if (n == 4) {
            for (int v = 0; v < 4; v++)
                for (int q = 0; q < 3; q++) Xq[v][q] = o->nodes[3 * vo[v] + q];
        } else {
            /* triangle (a,b,c) sorted by canonical id becomes the quad (a,b,c,c) */
            int64_t srt[3] = {vo[0], vo[1], vo[2]};
            for (int u = 0; u < 3; u++)
                for (int v = u + 1; v < 3; v++)
                    if (o->canon[srt[v]] < o->canon[srt[u]]) {
                        int64_t t = srt[u];
                        srt[u] = srt[v];
                        srt[v] = t;
                    }
            for (int q = 0; q < 3; q++) {
                Xq[0][q] = o->nodes[3 * srt[0] + q];
                Xq[1][q] = o->nodes[3 * srt[1] + q];
                Xq[2][q] = o->nodes[3 * srt[2] + q];
                Xq[3][q] = o->nodes[3 * srt[2] + q];
            }
        }
        face_gauss(Xq, F->gp, F->va);
        /* orient owner -> neighbour */
        double s = 0.0;
        for (int k = 0; k < 4; k++)
            for (int q = 0; q < 3; q++) s += F->va[k][q] * (F->gp[k][q] - o->c[F->owner].xc[q]);
        if (s < 0)
            for (int k = 0; k < 4; k++)
                for (int q = 0; q < 3; q++) F->va[k][q] = -F->va[k][q];
        ocell *Co = &o->c[F->owner];
        Co->face[fr[a].lf] = nf;
        Co->fside[fr[a].lf] = 0;
        Co->nb[fr[a].lf] = F->nb;
        double ar = 0.0;
        for (int k = 0; k < 4; k++) ar += sqrt(F->va[k][0] * F->va[k][0] + F->va[k][1] * F->va[k][1] + F->va[k][2] * F->va[k][2]);
        Co->area_sum += ar;
        if (pair) {
            ocell *Cn = &o->c[F->nbr];
            Cn->face[fr[a + 1].lf] = nf;
            Cn->fside[fr[a + 1].lf] = 1;
            Cn->nb[fr[a + 1].lf] = sref_self(F->owner);
            for (int q = 0; q < 3; q++) Cn->nb[fr[a + 1].lf].of[q] = -F->nb.of[q];
            Cn->area_sum += ar;
        }
        nf++;
        a += pair ? 2 : 1;
    }
    free(fr);
    o->n_faces = nf;
    /* each iteration writes only its own cell's stencils and fits: the same result at any thread
       count; the failure reported is the lowest failing cell's */
    int64_t bad = -1;
    int bad_code = 0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < n_cells; c++) {
        if (want && !want[c]) continue;
        int e = build_stencils(o, c);
        if (e) {
#pragma omp critical
            if (bad < 0 || c < bad) {
                bad = c;
                bad_code = e;
            }
        }
    }
    if (bad >= 0) {
        char m[160];
        snprintf(m, sizeof m, "stencil construction failed at cell %lld (code %d)", (long long)bad, bad_code);
        seterr(m);
        orc_destroy(o);
        return NULL;
    }
    o->a = malloc(sizeof(real) * n_cells * 45);
    o->b = malloc(sizeof(real) * n_cells * 120);
    o->w = malloc(sizeof(real) * n_cells * 45);
    return o;
}

orc *orc_create(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types, const int64_t *cells,
                const double *box, int periodic, int min_big)
{
    return orc_create_cells(n_nodes, nodes, n_cells, types, cells, box, periodic, min_big, NULL);
}

/* a cell whose stencils were not built (an oracle made for a subset of the cells) */
static int unbuilt(const orc *o, int64_t i)
{
    if (o->partial && o->c[i].K == 0) {
        seterr("stencils of this cell were not built");
        return 1;
    }
    return 0;
}

void orc_destroy(orc *o)
{
    if (!o) return;
    if (o->c)
        for (int64_t c = 0; c < o->n_cells; c++) {
            if (o->c[c].ls0.qr) lsq_free(&o->c[c].ls0);
            for (int m = 0; m < 8; m++)
                if (o->c[c].ls[m].qr) lsq_free(&o->c[c].ls[m]);
        }
    free(o->c);
    free(o->f);
    free(o->canon);
    free(o->nodes_copy);
    free(o->types);
    free(o->cells);
    free(o->a);
    free(o->b);
    free(o->w);
    free(o);
}

int64_t orc_n_faces(const orc *o) { return o->n_faces; }

/* Gauss-point sides that fell back to first order since the last call (then reset) */
/* threads of the two parallel loops (reconstruction, face fluxes); results do not depend on it */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t orc_fallback_count(orc *o)
{
    const int64_t c = o->n_fallback;
    o->n_fallback = 0;
    return c;
}

void orc_cell_geometry(const orc *o, double *vol, double *xc, double *m2, double *area)
{
    for (int64_t c = 0; c < o->n_cells; c++) {
        if (vol) vol[c] = o->c[c].vol;
        for (int q = 0; q < 3; q++)
            if (xc) xc[3 * c + q] = o->c[c].xc[q];
        for (int q = 0; q < 6; q++)
            if (m2) m2[6 * c + q] = o->c[c].m2[q];
        if (area) area[c] = o->c[c].area_sum;
    }
}

void orc_face_info(const orc *o, int64_t *owner, int64_t *nbr, int64_t *key, double *gp, double *va, int *sh)
{
    for (int64_t f = 0; f < o->n_faces; f++) {
        const oface *F = &o->f[f];
        if (owner) owner[f] = F->owner;
        if (nbr) nbr[f] = F->nbr;
        for (int q = 0; q < 4; q++)
            if (key) key[4 * f + q] = F->key[q];
        for (int k = 0; k < 4; k++)
            for (int q = 0; q < 3; q++) {
                if (gp) gp[12 * f + 3 * k + q] = F->gp[k][q];
                if (va) va[12 * f + 3 * k + q] = F->va[k][q];
            }
        for (int q = 0; q < 3; q++)
            if (sh) sh[3 * f + q] = F->nb.of[q];
    }
}

/* stencil sizes: K and M, and sub-stencil sizes */
int orc_stencil_grown(const orc *o, int64_t c) { return o->c[c].grown; }

void orc_stencil_info(const orc *o, int64_t c, int *K, int *M, int *subn)
{
    *K = o->c[c].K;
    *M = o->c[c].M;
    for (int m = 0; m < o->c[c].M; m++) subn[m] = o->c[c].subn[m];
}

/* ------------------------------------------------------------------ */
/* WENO reconstruction (Section 2, Eq. weno, Eq. indicator)            */
/* ------------------------------------------------------------------ */
static real Qat(const orc *o, const real *Q, int comp, int64_t cell) { return Q[comp * o->n_cells + cell]; }

static void prim_of(double gam, const real v[5], real *rho, real U[3], real *p)
{
    *rho = v[0];
    for (int d = 0; d < 3; d++) U[d] = v[1 + d] / v[0];
    *p = (gam - 1.0) * (v[4] - 0.5 * v[0] * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
}

static void cons_of(double gam, real rho, const real U[3], real p, real v[5])
{
    v[0] = rho;
    for (int d = 0; d < 3; d++) v[1 + d] = rho * U[d];
    v[4] = p / (gam - 1.0) + 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
}

/*
 * Far field by Riemann invariants along the outward normal (axis d, sign sn) against the free stream:
 * U_n +- 2c/(gamma-1) carried out of the domain by the interior and into it by the free stream
 * (subsonic), the entropy p / rho^gamma and the tangential velocity from the upwind side; supersonic
 * inflow takes the free stream, supersonic outflow the interior state.
 */
static void farfield_state(const orc_params *P, int d, double sn, const real v[5], real g[5])
{
    const double gam = P->gamma;
    const double *f = P->bc[2 * d + (sn > 0)].far;
    real rho, U[3], p;
    prim_of(gam, v, &rho, U, &p);
    const real c = r_sqrt(gam * p / rho);
    const real un = sn * U[d];
    const double fU[3] = {f[1], f[2], f[3]};
    const double cf = sqrt(gam * f[4] / f[0]), unf = sn * fU[d];
    if (RE(un) >= RE(c)) { /* supersonic outflow */
        for (int j = 0; j < 5; j++) g[j] = v[j];
        return;
    }
    real gU[3], grho, gp;
    if (unf <= -cf) { /* supersonic inflow */
        const real fr = f[0], fp = f[4];
        const real fu[3] = {fU[0], fU[1], fU[2]};
        cons_of(gam, fr, fu, fp, g);
        return;
    }
    const real Rp = un + 2.0 * c / (gam - 1.0), Rm = unf - 2.0 * cf / (gam - 1.0);
    const real unb = 0.5 * (Rp + Rm), cb = 0.25 * (gam - 1.0) * (Rp - Rm);
    real s;
    if (RE(unb) > 0.0) { /* outflow: entropy and tangential velocity of the interior */
        s = p / r_pow(rho, gam);
        for (int q = 0; q < 3; q++) gU[q] = U[q];
    } else {
        s = f[4] / pow(f[0], gam);
        for (int q = 0; q < 3; q++) gU[q] = fU[q];
    }
    gU[d] = sn * unb;
    grho = r_pow(cb * cb / (gam * s), 1.0 / (gam - 1.0));
    gp = grho * cb * cb / gam;
    cons_of(gam, grho, gU, gp, g);
}

/* the ghost state across box plane `plane` of the state v (cell average, global frame) */
static void bc_state(const orc_params *P, int plane, const real v[5], real g[5])
{
    const orc_bc *B = &P->bc[plane];
    const int d = plane / 2;
    const double gam = P->gamma;
    switch (B->type) {
    case BC_SLIP:
        for (int j = 0; j < 5; j++) g[j] = v[j];
        g[1 + d] = -v[1 + d];
        return;
    case BC_FARFIELD: farfield_state(P, d, plane % 2 ? 1.0 : -1.0, v, g); return;
    case BC_EXTRAPOLATE:
        for (int j = 0; j < 5; j++) g[j] = v[j];
        return;
    default: {
        real rho, U[3], p, gU[3];
        prim_of(gam, v, &rho, U, &p);
        for (int q = 0; q < 3; q++) gU[q] = 2.0 * B->uw[q] - U[q];
        const real grho = B->type == BC_ISOTHERMAL ? p / (2.0 * B->Tw - p / rho) : rho;
        cons_of(gam, grho, gU, p, g);
    }
    }
}

/*
 * Cell average of a member: its cell's, through the boundary condition of every wall plane the member
 * is mirrored across (axis order; an axis mirrored twice, at 0 and at L, is a translation by 2L and
 * crosses both planes: first the one at 0 for +2L, first the one at L for -2L).
 */
static void member_state(const orc *o, const orc_params *P, const real *Q, sref s, real v[5])
{
    for (int c = 0; c < 5; c++) v[c] = Qat(o, Q, c, s.cell);
    for (int d = 0; d < 3; d++) {
        int planes[2], np = 0;
        if (s.sg[d] < 0)
            planes[np++] = 2 * d + (s.of[d] == 2);
        else if (s.of[d] == 2 && !o->periodic) {
            planes[np++] = 2 * d;
            planes[np++] = 2 * d + 1;
        } else if (s.of[d] == -2 && !o->periodic) {
            planes[np++] = 2 * d + 1;
            planes[np++] = 2 * d;
        }
        for (int k = 0; k < np; k++) {
            real g[5];
            bc_state(P, planes[k], v, g);
            for (int c = 0; c < 5; c++) v[c] = g[c];
        }
    }
}

static real member_value(const orc *o, const orc_params *P, const real *Q, int comp, sref s)
{
    if (s.sg[0] > 0 && s.sg[1] > 0 && s.sg[2] > 0 &&
        (o->periodic || (abs(s.of[0]) < 2 && abs(s.of[1]) < 2 && abs(s.of[2]) < 2)))
        return Qat(o, Q, comp, s.cell); /* not mirrored */
    real v[5];
    member_state(o, P, Q, s, v);
    return v[comp];
}

/*
 * Value and gradient (global frame) beyond box plane `plane` at a Gauss point on it, from the inner
 * reconstructed ones: the ghost field is the condition applied to the mirrored inner field, so its
 * value is the condition of the inner value and its gradient the condition's derivative applied to
 * the inner gradient, with the derivative across the plane negated (the mirror).  The far field's
 * ghost is uniform (zero gradient).  The flux's reflective walls evaluate the image's reconstruction
 * instead (the same state).
 */
static void bc_ghost_point(const orc_params *P, int plane, const real v[5], const real gv[5][3], real g[5], real gg[5][3])
{
    const orc_bc *B = &P->bc[plane];
    const int d = plane / 2;
    const double gam = P->gamma;
    if (B->type == BC_FARFIELD) {
        farfield_state(P, d, plane % 2 ? 1.0 : -1.0, v, g);
        for (int c = 0; c < 5; c++)
            for (int q = 0; q < 3; q++) gg[c][q] = 0.0;
        return;
    }
    if (B->type == BC_EXTRAPOLATE || B->type == BC_SLIP) {
        /* linear conditions: the sign of the normal momentum (reflective), the mirror on the gradient */
        for (int c = 0; c < 5; c++) {
            const double s = B->type == BC_SLIP && c == 1 + d ? -1.0 : 1.0;
            g[c] = s * v[c];
            for (int q = 0; q < 3; q++) gg[c][q] = (q == d ? -s : s) * gv[c][q];
        }
        return;
    }
    /* no-slip: primitive variables and their derivatives along x, y, z */
    real rho, U[3], p, drho[3], dU[3][3], dp[3];
    prim_of(gam, v, &rho, U, &p);
    for (int q = 0; q < 3; q++) {
        drho[q] = gv[0][q];
        real udu = 0.0;
        for (int a = 0; a < 3; a++) {
            dU[a][q] = (gv[1 + a][q] - U[a] * gv[0][q]) / rho;
            udu += U[a] * dU[a][q];
        }
        dp[q] = (gam - 1.0) * (gv[4][q] - 0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) * gv[0][q] - rho * udu);
    }
    real gU[3], gdU[3][3], grho = rho, gdrho[3];
    for (int a = 0; a < 3; a++) {
        gU[a] = 2.0 * B->uw[a] - U[a];
        for (int q = 0; q < 3; q++) gdU[a][q] = -dU[a][q];
    }
    for (int q = 0; q < 3; q++) gdrho[q] = drho[q];
    if (B->type == BC_ISOTHERMAL) {
        const real T = p / rho, Tg = 2.0 * B->Tw - T;
        grho = p / Tg;
        for (int q = 0; q < 3; q++) {
            const real dT = (dp[q] - T * drho[q]) / rho;
            gdrho[q] = (dp[q] + grho * dT) / Tg; /* d(p / Tg) with dTg = -dT */
        }
    }
    cons_of(gam, grho, gU, p, g);
    const real u2 = gU[0] * gU[0] + gU[1] * gU[1] + gU[2] * gU[2];
    for (int q = 0; q < 3; q++) {
        real udu = 0.0;
        for (int a = 0; a < 3; a++) udu += gU[a] * gdU[a][q];
        gg[0][q] = gdrho[q];
        for (int a = 0; a < 3; a++) gg[1 + a][q] = gU[a] * gdrho[q] + grho * gdU[a][q];
        gg[4][q] = dp[q] / (gam - 1.0) + 0.5 * u2 * gdrho[q] + grho * udu;
    }
    for (int c = 0; c < 5; c++) gg[c][d] = -gg[c][d];
}

static void weno_cell(orc *o, const orc_params *P, const real *Q, int64_t i)
{
    ocell *C = &o->c[i];
    real *a = o->a + 45 * i, *b = o->b + 120 * i, *w = o->w + 45 * i;
    double S[3][3] = {{C->m2[0], C->m2[1], C->m2[2]}, {C->m2[1], C->m2[3], C->m2[4]}, {C->m2[2], C->m2[4], C->m2[5]}};
    int M = C->M;
    double gm = P->weno_gamma_m, g0 = 1.0 - gm * M;
    for (int comp = 0; comp < 5; comp++) {
        real q0 = Qat(o, Q, comp, i);
        real rhs[MAXST];
        /* P_0: least squares on the big stencil */
        for (int k = 0; k < C->K; k++) rhs[k] = member_value(o, P, Q, comp, C->st[k]) - q0;
        real *ac = a + 9 * comp;
        lsq_apply(&C->ls0, rhs, ac);
        /* P_m on the sub-stencils */
        for (int m = 0; m < M; m++) {
            for (int k = 0; k < C->subn[m]; k++) rhs[k] = member_value(o, P, Q, comp, C->sub[m][k]) - q0;
            lsq_apply(&C->ls[m], rhs, b + 24 * comp + 3 * m);
        }
        /* smoothness indicators over Omega_0, each multi-index once */
        double vol = C->vol;
        double v13 = cbrt(vol);
        /* first derivatives of P_0 are linear: d/dx = a_x + 2a_xx X + a_xy Y + a_xz Z, ... */
        real G[3][4] = {
            {ac[0], 2 * ac[3], ac[4], ac[5]},
            {ac[1], ac[4], 2 * ac[6], ac[7]},
            {ac[2], ac[5], ac[7], 2 * ac[8]},
        };
        real beta0 = 0.0;
        for (int d = 0; d < 3; d++) {
            real lin = 0.0;
            for (int p = 0; p < 3; p++)
                for (int q = 0; q < 3; q++) lin += G[d][1 + p] * S[p][q] * G[d][1 + q];
            real integral = vol * (G[d][0] * G[d][0] + lin);
            beta0 += integral / v13;
        }
        real sec[6] = {2 * ac[3], 2 * ac[6], 2 * ac[8], ac[4], ac[5], ac[7]};
        for (int d = 0; d < 6; d++) beta0 += v13 * vol * sec[d] * sec[d];
        real beta[8];
        real tw = 0.0;
        for (int m = 0; m < M; m++) {
            const real *bm = b + 24 * comp + 3 * m;
            beta[m] = vol * (bm[0] * bm[0] + bm[1] * bm[1] + bm[2] * bm[2]) / v13;
            tw += r_abs(beta0 - beta[m]) / M;
        }
        real om[9], sum = 0.0;
        if (P->force_linear) {
            om[0] = g0;
            for (int m = 0; m < M; m++) om[1 + m] = gm;
        } else {
            om[0] = g0 * (1.0 + r_pow(tw / (beta0 + P->weno_eps), P->weno_p));
            for (int m = 0; m < M; m++) om[1 + m] = gm * (1.0 + r_pow(tw / (beta[m] + P->weno_eps), P->weno_p));
        }
        for (int m = 0; m <= M; m++) sum += om[m];
        for (int m = 0; m <= M; m++) w[9 * comp + m] = om[m] / sum;
    }
}

/* value and gradient at x (cell's own frame) of P_m (m = 0..M) or of Eq. weno (m < 0) */
static void weno_eval(const orc *o, const orc_params *P, const real *Q, int64_t i, int which, const double x[3],
                      real val[5], real grad[5][3])
{
    const ocell *C = &o->c[i];
    const real *a = o->a + 45 * i, *b = o->b + 120 * i, *w = o->w + 45 * i;
    double X[3] = {x[0] - C->xc[0], x[1] - C->xc[1], x[2] - C->xc[2]};
    double S[3][3] = {{C->m2[0], C->m2[1], C->m2[2]}, {C->m2[1], C->m2[3], C->m2[4]}, {C->m2[2], C->m2[4], C->m2[5]}};
    /* basis p_n(x) = (x-x0)^n - mean over Omega_0, and its gradient */
    double pb[9], dp[9][3];
    for (int n = 0; n < 9; n++) {
        const int *e = MONO[n];
        double mono = 1.0, mean = 0.0;
        for (int q = 0; q < 3; q++) mono *= pow(X[q], e[q]);
        if (n >= 3) {
            int ax[2], na = 0;
            for (int q = 0; q < 3; q++)
                for (int r = 0; r < e[q]; r++) ax[na++] = q;
            mean = S[ax[0]][ax[1]];
        }
        pb[n] = mono - mean;
        for (int d = 0; d < 3; d++) {
            if (e[d] == 0) {
                dp[n][d] = 0.0;
                continue;
            }
            double t = e[d];
            for (int q = 0; q < 3; q++) t *= pow(X[q], q == d ? e[q] - 1 : e[q]);
            dp[n][d] = t;
        }
    }
    int M = C->M;
    double gm = P->weno_gamma_m, g0 = 1.0 - gm * M;
    for (int comp = 0; comp < 5; comp++) {
        real q0 = Qat(o, Q, comp, i);
        const real *ac = a + 9 * comp;
        /* every candidate polynomial at x */
        real pv[9], pg[9][3];
        pv[0] = q0;
        pg[0][0] = pg[0][1] = pg[0][2] = 0.0;
        for (int n = 0; n < 9; n++) {
            pv[0] += ac[n] * pb[n];
            for (int d = 0; d < 3; d++) pg[0][d] += ac[n] * dp[n][d];
        }
        for (int m = 0; m < M; m++) {
            const real *bm = b + 24 * comp + 3 * m;
            pv[1 + m] = q0;
            for (int d = 0; d < 3; d++) pg[1 + m][d] = 0.0;
            for (int n = 0; n < 3; n++) {
                pv[1 + m] += bm[n] * pb[n];
                for (int d = 0; d < 3; d++) pg[1 + m][d] += bm[n] * dp[n][d];
            }
        }
        if (which >= 0) {
            val[comp] = pv[which];
            for (int d = 0; d < 3; d++) grad[comp][d] = pg[which][d];
            continue;
        }
        /* Eq. weno */
        const real *wc = w + 9 * comp;
        real v = pv[0] / g0, g[3] = {pg[0][0] / g0, pg[0][1] / g0, pg[0][2] / g0};
        for (int m = 0; m < M; m++) {
            v -= gm / g0 * pv[1 + m];
            for (int d = 0; d < 3; d++) g[d] -= gm / g0 * pg[1 + m][d];
        }
        v *= wc[0];
        for (int d = 0; d < 3; d++) g[d] *= wc[0];
        for (int m = 0; m < M; m++) {
            v += wc[1 + m] * pv[1 + m];
            for (int d = 0; d < 3; d++) g[d] += wc[1 + m] * pg[1 + m][d];
        }
        val[comp] = v;
        for (int d = 0; d < 3; d++) grad[comp][d] = g[d];
    }
}

/* every cell's reconstruction; each iteration writes only its own cell's coefficients, so the
   OpenMP loop gives the same result as the serial one */
static void weno_all(orc *o, const orc_params *P, const real *Q)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < o->n_cells; i++) weno_cell(o, P, Q, i);
}

/* exported: evaluate at point x of cell i (m=-1: Eq. weno; m>=0: P_m) */
int orc_weno_eval(orc *o, const orc_params *P, const real *Q, int64_t i, int m, const double *x, real *val, real *grad)
{
    if (unbuilt(o, i)) return 7;
    weno_cell(o, P, Q, i);
    real g[5][3];
    weno_eval(o, P, Q, i, m, x, val, g);
    for (int c = 0; c < 5; c++)
        for (int d = 0; d < 3; d++) grad[3 * c + d] = g[c][d];
    return 0;
}

/* normalised nonlinear weights of cell i (for inspection) */
int orc_weno_weights(orc *o, const orc_params *P, const real *Q, int64_t i, real *w)
{
    if (unbuilt(o, i)) return 7;
    weno_cell(o, P, Q, i);
    /* omega_0..omega_M per component; the slots beyond M are zero */
    for (int c = 0; c < 5; c++)
        for (int m = 0; m < 9; m++) w[9 * c + m] = m <= o->c[i].M ? o->w[45 * i + 9 * c + m] : 0.0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* BGK moments (Eq. bgk-3d, Eq. compatibility)                         */
/* ------------------------------------------------------------------ */
/* polynomial in (u, v, w, varsigma^2): sum of c u^a v^b w^e (varsigma^2)^d */
#define MAXT 48
typedef struct {
    int n;
    real c[MAXT];
    int e[MAXT][4];
} vpoly;

static void vp_zero(vpoly *p) { p->n = 0; }
static void vp_add(vpoly *p, real c, int a, int b, int w, int d)
{
    if (c == 0.0) return;
    p->c[p->n] = c;
    p->e[p->n][0] = a;
    p->e[p->n][1] = b;
    p->e[p->n][2] = w;
    p->e[p->n][3] = d;
    p->n++;
}

/* psi_j, j = 0..4: 1, u, v, w, (u^2 + v^2 + w^2 + varsigma^2)/2 */
static void vp_psi(vpoly *p, int j)
{
    vp_zero(p);
    switch (j) {
    case 0: vp_add(p, 1.0, 0, 0, 0, 0); break;
    case 1: vp_add(p, 1.0, 1, 0, 0, 0); break;
    case 2: vp_add(p, 1.0, 0, 1, 0, 0); break;
    case 3: vp_add(p, 1.0, 0, 0, 1, 0); break;
    default:
        vp_add(p, 0.5, 2, 0, 0, 0);
        vp_add(p, 0.5, 0, 2, 0, 0);
        vp_add(p, 0.5, 0, 0, 2, 0);
        vp_add(p, 0.5, 0, 0, 0, 1);
        break;
    }
}

/* a . psi for a slope vector a[5] */
static void vp_slope(vpoly *p, const real a[5])
{
    vp_zero(p);
    vp_add(p, a[0], 0, 0, 0, 0);
    vp_add(p, a[1], 1, 0, 0, 0);
    vp_add(p, a[2], 0, 1, 0, 0);
    vp_add(p, a[3], 0, 0, 1, 0);
    vp_add(p, 0.5 * a[4], 2, 0, 0, 0);
    vp_add(p, 0.5 * a[4], 0, 2, 0, 0);
    vp_add(p, 0.5 * a[4], 0, 0, 2, 0);
    vp_add(p, 0.5 * a[4], 0, 0, 0, 1);
}

/* (a_1 . psi) u + (a_2 . psi) v + (a_3 . psi) w for three slope vectors */
static void vp_advect(vpoly *p, const real a[3][5])
{
    vp_zero(p);
    for (int m = 0; m < 3; m++) {
        vpoly s;
        vp_slope(&s, a[m]);
        for (int t = 0; t < s.n; t++) {
            int e[4] = {s.e[t][0], s.e[t][1], s.e[t][2], s.e[t][3]};
            e[m]++;
            vp_add(p, s.c[t], e[0], e[1], e[2], e[3]);
        }
    }
}

#define MAXO 14
/* normalised moments of a Maxwellian: <u^n> (full, u>0, u<0), <v^n>, <w^n>, <varsigma^(2d)> */
typedef struct {
    real rho, U, V, W, lam;
    real uf[MAXO], up[MAXO], un[MAXO], v[MAXO], w[MAXO], s[6];
} maxw;

static void moments_1d_full(real U, real lam, real *m)
{
    m[0] = 1.0;
    m[1] = U;
    for (int n = 0; n + 2 < MAXO; n++) m[n + 2] = U * m[n + 1] + (n + 1) / (2.0 * lam) * m[n];
}

static void maxw_init(maxw *g, real rho, real U, real V, real W, real lam, double K)
{
    g->rho = rho;
    g->U = U;
    g->V = V;
    g->W = W;
    g->lam = lam;
    moments_1d_full(U, lam, g->uf);
    moments_1d_full(V, lam, g->v);
    moments_1d_full(W, lam, g->w);
    /* half spaces: <u^0> = erfc(-+ sqrt(lam) U)/2, <u^1> = U<u^0> +- exp(-lam U^2)/(2 sqrt(pi lam)) */
    real e = r_exp(-lam * U * U) / (2.0 * r_sqrt(M_PI * lam));
    g->up[0] = 0.5 * r_erfc(-r_sqrt(lam) * U);
    g->un[0] = 0.5 * r_erfc(r_sqrt(lam) * U);
    g->up[1] = U * g->up[0] + e;
    g->un[1] = U * g->un[0] - e;
    for (int n = 0; n + 2 < MAXO; n++) {
        g->up[n + 2] = U * g->up[n + 1] + (n + 1) / (2.0 * lam) * g->up[n];
        g->un[n + 2] = U * g->un[n + 1] + (n + 1) / (2.0 * lam) * g->un[n];
    }
    /* internal degrees of freedom: <(varsigma^2)^d> = prod_{j<d} (K/2 + j) / lam^d */
    g->s[0] = 1.0;
    for (int d = 1; d < 6; d++) g->s[d] = g->s[d - 1] * (0.5 * K + (d - 1)) / lam;
}

/* half = 0 full space, +1 u > 0, -1 u < 0; moment of u^upow * P * R */
static real mom2(const maxw *g, int half, int upow, const vpoly *P, const vpoly *R)
{
    const real *mu = half > 0 ? g->up : (half < 0 ? g->un : g->uf);
    real s = 0.0;
    for (int i = 0; i < P->n; i++)
        for (int j = 0; j < R->n; j++) {
            int a = P->e[i][0] + R->e[j][0] + upow;
            int b = P->e[i][1] + R->e[j][1];
            int w = P->e[i][2] + R->e[j][2];
            int d = P->e[i][3] + R->e[j][3];
            s += P->c[i] * R->c[j] * mu[a] * g->v[b] * g->w[w] * g->s[d];
        }
    return s;
}

/* <u^upow P psi> (normalised, 5-vector) */
static void mom_psi(const maxw *g, int half, int upow, const vpoly *P, real out[5])
{
    for (int j = 0; j < 5; j++) {
        vpoly pj;
        vp_psi(&pj, j);
        out[j] = mom2(g, half, upow, P, &pj);
    }
}

/* solve <a psi> = b for the slope a: M_jk = <psi_j psi_k> (normalised) */
static int slope_solve(const maxw *g, const real b[5], real a[5])
{
    real A[25], r[5];
    for (int j = 0; j < 5; j++) {
        vpoly pj;
        vp_psi(&pj, j);
        for (int k = 0; k < 5; k++) {
            vpoly pk;
            vp_psi(&pk, k);
            A[5 * j + k] = mom2(g, 0, 0, &pj, &pk);
        }
        r[j] = b[j];
    }
    return gauss_solve(5, A, r, a);
}

static void cons_to_prim(double gam, const real q[5], real *rho, real U[3], real *lam, real *p)
{
    *rho = q[0];
    for (int d = 0; d < 3; d++) U[d] = q[1 + d] / q[0];
    *p = (gam - 1.0) * (q[4] - 0.5 * q[0] * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    *lam = q[0] / (2.0 * *p);
}

/*
 * Flux at one face Gauss point in the local frame (Section 3.2, Eq. flux-1).
 * ql, qr: conservative states on the left (owner) and right; dql, dqr: their
 * derivatives along n1, n2, n3 ([3][5]).  Returns the time integrals F(dt/2)
 * and F(dt) of the flux per unit area, fitted to Fbar0 = flux at t_n and
 * Fbar1 = its time derivative.  dbg (optional, 80 doubles): rho0 U0 V0 W0
 * lam0, al[3][5], ar[3][5], abar[3][5], Al[5], Ar[5], Abar[5], tau, F(dt/2)[5],
 * F(dt)[5].
 */
int orc_gp_flux(const orc_params *P, const real *ql, const real *dql, const real *qr, const real *dqr, double dt,
                real *Fbar, real *dbg)
{
    double gam = P->gamma, K = (5.0 - 3.0 * gam) / (gam - 1.0);
    real rl, rr, Ul[3], Ur[3], laml, lamr, pl, pr;
    cons_to_prim(gam, ql, &rl, Ul, &laml, &pl);
    cons_to_prim(gam, qr, &rr, Ur, &lamr, &pr);
    if (!(RE(rl) > 0 && RE(rr) > 0 && RE(pl) > 0 && RE(pr) > 0)) return 4;
    maxw gl, gr, g0;
    maxw_init(&gl, rl, Ul[0], Ul[1], Ul[2], laml, K);
    maxw_init(&gr, rr, Ur[0], Ur[1], Ur[2], lamr, K);
    vpoly one;
    vp_zero(&one);
    vp_add(&one, 1.0, 0, 0, 0, 0);
    /* interface equilibrium: Q0 = rho_l <psi>_{u>0,l} + rho_r <psi>_{u<0,r} */
    real hl[5], hr[5], q0[5];
    mom_psi(&gl, 1, 0, &one, hl);
    mom_psi(&gr, -1, 0, &one, hr);
    for (int j = 0; j < 5; j++) q0[j] = rl * hl[j] + rr * hr[j];
    real r0, U0[3], lam0, p0;
    cons_to_prim(gam, q0, &r0, U0, &lam0, &p0);
    if (!(RE(r0) > 0 && RE(p0) > 0)) return 4;
    maxw_init(&g0, r0, U0[0], U0[1], U0[2], lam0, K);
    /* slopes from the directional derivatives: <a_m> = dQ/dn_m */
    real al[3][5], ar[3][5];
    for (int m = 0; m < 3; m++) {
        real bl[5], br[5];
        for (int j = 0; j < 5; j++) {
            bl[j] = dql[5 * m + j] / rl;
            br[j] = dqr[5 * m + j] / rr;
        }
        if (slope_solve(&gl, bl, al[m]) || slope_solve(&gr, br, ar[m])) return 5;
    }
    /* time slopes from compatibility: <a_1 u + a_2 v + a_3 w + A> = 0 */
    real Al[5], Ar[5];
    {
        vpoly adv;
        real b[5];
        vp_advect(&adv, al);
        mom_psi(&gl, 0, 0, &adv, b);
        for (int j = 0; j < 5; j++) b[j] = -b[j];
        if (slope_solve(&gl, b, Al)) return 5;
        vp_advect(&adv, ar);
        mom_psi(&gr, 0, 0, &adv, b);
        for (int j = 0; j < 5; j++) b[j] = -b[j];
        if (slope_solve(&gr, b, Ar)) return 5;
    }
    /* equilibrium slopes: rho0 <abar_m psi> = rho_l <a^l_m psi>_{u>0} + rho_r <a^r_m psi>_{u<0} */
    real ab[3][5], Ab[5];
    for (int m = 0; m < 3; m++) {
        vpoly sl, sr;
        vp_slope(&sl, al[m]);
        vp_slope(&sr, ar[m]);
        real ml[5], mr[5], b[5];
        mom_psi(&gl, 1, 0, &sl, ml);
        mom_psi(&gr, -1, 0, &sr, mr);
        for (int j = 0; j < 5; j++) b[j] = (rl * ml[j] + rr * mr[j]) / r0;
        if (slope_solve(&g0, b, ab[m])) return 5;
    }
    {
        vpoly adv;
        real b[5];
        vp_advect(&adv, ab);
        mom_psi(&g0, 0, 0, &adv, b);
        for (int j = 0; j < 5; j++) b[j] = -b[j];
        if (slope_solve(&g0, b, Ab)) return 5;
    }
    /* collision time (opening of Section 5) */
    real jump = r_abs((pl - pr) / (pl + pr)) * dt;
    real mu = P->mu;
    if (P->viscous && P->mu_power != 0.0) mu *= r_pow((p0 / r0) / P->T_ref, P->mu_power);
    real tau = P->viscous ? mu / p0 + P->tau_C * jump : P->tau_eps * dt + P->tau_C * jump;
    /* moment vectors shared by both time integrals; upow = 1 gives flux moments, 0 conserved moments */
    real Mg0[2][5], Mg0a[2][5], Mg0A[2][5], Mh[2][5], Mha[2][5], MhA[2][5];
    {
        vpoly adv0, A0, advl, advr, Alp, Arp;
        vp_advect(&adv0, ab);
        vp_slope(&A0, Ab);
        vp_advect(&advl, al);
        vp_advect(&advr, ar);
        vp_slope(&Alp, Al);
        vp_slope(&Arp, Ar);
        for (int up = 0; up < 2; up++) {
            real x[5], y[5];
            mom_psi(&g0, 0, up, &one, Mg0[up]);
            mom_psi(&g0, 0, up, &adv0, Mg0a[up]);
            mom_psi(&g0, 0, up, &A0, Mg0A[up]);
            mom_psi(&gl, 1, up, &one, x);
            mom_psi(&gr, -1, up, &one, y);
            for (int j = 0; j < 5; j++) Mh[up][j] = rl * x[j] + rr * y[j];
            mom_psi(&gl, 1, up, &advl, x);
            mom_psi(&gr, -1, up, &advr, y);
            for (int j = 0; j < 5; j++) Mha[up][j] = rl * x[j] + rr * y[j];
            mom_psi(&gl, 1, up, &Alp, x);
            mom_psi(&gr, -1, up, &Arp, y);
            for (int j = 0; j < 5; j++) MhA[up][j] = rl * x[j] + rr * y[j];
        }
    }
    real Fd[2][5];
    for (int s = 0; s < 2; s++) {
        double d = s == 0 ? 0.5 * dt : dt;
        real eta = r_exp(-d / tau), om = -r_expm1(-d / tau);
        real T1 = d - tau * om;
        real T2 = 2.0 * tau * tau * om - tau * d * (1.0 + eta);
        real T3 = 0.5 * d * d - tau * d + tau * tau * om;
        real T4 = tau * om;
        real T5 = 2.0 * tau * tau * om - tau * d * eta;
        real W[2][5];
        if (P->smooth) {
            /* Eq. flux-2 with the -tau Abar term that the smooth limit of Eq. flux-1 carries (the
               printed line drops it): f = g0 (1 - tau (abar.u + Abar) + Abar t), integrated over
               [0, d]: d <.>g0 - tau d <.(abar.u + Abar)>g0 + d^2/2 <.Abar>g0 */
            for (int up = 0; up < 2; up++)
                for (int j = 0; j < 5; j++)
                    W[up][j] = r0 * (d * Mg0[up][j] - tau * d * (Mg0a[up][j] + Mg0A[up][j]) + 0.5 * d * d * Mg0A[up][j]);
        } else {
            for (int up = 0; up < 2; up++)
                for (int j = 0; j < 5; j++)
                    W[up][j] = r0 * (T1 * Mg0[up][j] + T2 * Mg0a[up][j] + T3 * Mg0A[up][j]) + T4 * Mh[up][j] -
                               T5 * Mha[up][j] - tau * T4 * MhA[up][j];
        }
        for (int j = 0; j < 5; j++) Fd[s][j] = W[1][j];
        if (P->viscous && P->Pr != 1.0) {
            /* heat flux about U0 of the time-integrated distribution */
            const real *Fm = W[1], *Wm = W[0];
            real U2 = U0[0] * U0[0] + U0[1] * U0[1] + U0[2] * U0[2];
            real q2 = 2.0 * Fm[4] - 2.0 * (U0[0] * Fm[1] + U0[1] * Fm[2] + U0[2] * Fm[3]) + U2 * Fm[0] -
                        U0[0] * 2.0 * Wm[4] + 2.0 * U0[0] * (U0[0] * Wm[1] + U0[1] * Wm[2] + U0[2] * Wm[3]) -
                        U0[0] * U2 * Wm[0];
            Fd[s][4] += (1.0 / P->Pr - 1.0) * 0.5 * q2;
        }
    }
    for (int j = 0; j < 5; j++) {
        Fbar[j] = (4.0 * Fd[0][j] - Fd[1][j]) / dt;
        Fbar[5 + j] = 4.0 * (Fd[1][j] - 2.0 * Fd[0][j]) / (dt * dt);
    }
    if (dbg) {
        real *z = dbg;
        z[0] = r0;
        z[1] = U0[0];
        z[2] = U0[1];
        z[3] = U0[2];
        z[4] = lam0;
        for (int m = 0; m < 3; m++)
            for (int j = 0; j < 5; j++) {
                z[5 + 5 * m + j] = al[m][j];
                z[20 + 5 * m + j] = ar[m][j];
                z[35 + 5 * m + j] = ab[m][j];
            }
        for (int j = 0; j < 5; j++) {
            z[50 + j] = Al[j];
            z[55 + j] = Ar[j];
            z[60 + j] = Ab[j];
            z[66 + j] = Fd[0][j];
            z[71 + j] = Fd[1][j];
        }
        z[65] = tau;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* face fluxes and the semi-discrete operator (Eq. flux-qud, Eq. finite) */
/* ------------------------------------------------------------------ */
static void local_frame(const double va[3], double n[3][3])
{
    double a = sqrt(va[0] * va[0] + va[1] * va[1] + va[2] * va[2]);
    for (int q = 0; q < 3; q++) n[0][q] = va[q] / a;
    int e = 0;
    for (int q = 1; q < 3; q++)
        if (fabs(n[0][q]) < fabs(n[0][e])) e = q;
    double t[3] = {0, 0, 0};
    t[e] = 1.0;
    double d = n[0][e];
    for (int q = 0; q < 3; q++) t[q] -= d * n[0][q];
    double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int q = 0; q < 3; q++) n[1][q] = t[q] / tn;
    n[2][0] = n[0][1] * n[1][2] - n[0][2] * n[1][1];
    n[2][1] = n[0][2] * n[1][0] - n[0][0] * n[1][2];
    n[2][2] = n[0][0] * n[1][1] - n[0][1] * n[1][0];
}

static void to_local(const double n[3][3], const real val[5], const real grad[5][3], real q[5], real dq[3][5])
{
    q[0] = val[0];
    q[4] = val[4];
    for (int m = 0; m < 3; m++) q[1 + m] = val[1] * n[m][0] + val[2] * n[m][1] + val[3] * n[m][2];
    for (int m = 0; m < 3; m++) {
        real dn[5];
        for (int c = 0; c < 5; c++) dn[c] = grad[c][0] * n[m][0] + grad[c][1] * n[m][1] + grad[c][2] * n[m][2];
        dq[m][0] = dn[0];
        dq[m][4] = dn[4];
        for (int k = 0; k < 3; k++) dq[m][1 + k] = dn[1] * n[k][0] + dn[2] * n[k][1] + dn[3] * n[k][2];
    }
}

static int physical_state(const orc_params *P, const real q[5])
{
    if (!(RE(q[0]) > 0.0)) return 0;
    const real p = (P->gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
    return RE(p) > 0.0;
}

/* a side state that keeps its reconstruction: rho and p positive and, with a floor, above that
   fraction of the side cell's average density and pressure */
static int admissible_state(const orc *o, const orc_params *P, const real *Q, sref s, const real q[5])
{
    if (!physical_state(P, q)) return 0;
    if (P->fallback_floor > 0.0) {
        real v[5];
        member_state(o, P, Q, s, v);
        const real pav = (P->gamma - 1.0) * (v[4] - 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0]);
        const real p = (P->gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
        if (!(RE(q[0]) > P->fallback_floor * RE(v[0])) || !(RE(p) > P->fallback_floor * RE(pav))) return 0;
    }
    return 1;
}

/* first-order fallback of one side: the member's cell average in the local frame, zero slopes */
static void fallback_state(const orc *o, const orc_params *P, const real *Q, sref s, const double n[3][3], real q[5],
                           real dq[3][5])
{
    real v[5], g[5][3];
    member_state(o, P, Q, s, v);
    for (int c = 0; c < 5; c++) g[c][0] = g[c][1] = g[c][2] = 0.0;
    to_local(n, v, g, q, dq);
}

static int face_flux_all(orc *o, const orc_params *P, const real *Q, double dt, real *out)
{
    if (o->partial) {
        seterr("stencils built for a subset of the cells: no residual");
        return 7;
    }
    weno_all(o, P, Q);
    /* each iteration writes only its own face's fluxes; the fallback count is an integer sum */
    int err = 0;
    int64_t nfb = 0;
#pragma omp parallel for schedule(static) reduction(+ : nfb) reduction(max : err)
    for (int64_t f = 0; f < o->n_faces; f++) {
        const oface *F = &o->f[f];
        real acc[10] = {0};
        /* a wall face: its box plane, and whether its condition is other than the reflective one */
        const sref *T = &F->nb;
        int plane = -1;
        if (F->nbr < 0)
            for (int d = 0; d < 3; d++)
                if (T->sg[d] < 0) plane = 2 * d + (T->of[d] == 2);
        const int general = plane >= 0 && P->bc[plane].type != BC_SLIP;
        for (int k = 0; k < 4; k++) {
            real vl[5], gl[5][3], vr[5], gr[5][3];
            weno_eval(o, P, Q, F->owner, -1, F->gp[k], vl, gl);
            double n[3][3];
            local_frame(F->va[k], n);
            real ql[5], qr[5], dql[3][5], dqr[3][5];
            to_local(n, vl, gl, ql, dql);
            if (!general) {
                /* the neighbour's polynomial as its image: P(T^-1 x), momentum signed by the reflections */
                double xr[3];
                for (int q = 0; q < 3; q++) xr[q] = T->sg[q] * (F->gp[k][q] - T->of[q] * o->L[q]);
                weno_eval(o, P, Q, T->cell, -1, xr, vr, gr);
                for (int c = 0; c < 5; c++)
                    for (int q = 0; q < 3; q++) gr[c][q] *= T->sg[q];
                for (int c = 0; c < 3; c++) {
                    vr[1 + c] *= T->sg[c];
                    for (int q = 0; q < 3; q++) gr[1 + c][q] *= T->sg[c];
                }
                to_local(n, vr, gr, qr, dqr);
                if (P->fallback) {
                    if (!admissible_state(o, P, Q, sref_self(F->owner), ql)) {
                        fallback_state(o, P, Q, sref_self(F->owner), n, ql, dql);
                        nfb++;
                    }
                    if (!admissible_state(o, P, Q, F->nb, qr)) {
                        fallback_state(o, P, Q, F->nb, n, qr, dqr);
                        nfb++;
                    }
                }
            } else {
                /* the state beyond the plane: its condition applied to the inner state (after the inner
                   side's fallback, whose ghost then falls back too) */
                if (P->fallback && !admissible_state(o, P, Q, sref_self(F->owner), ql)) {
                    member_state(o, P, Q, sref_self(F->owner), vl);
                    for (int c = 0; c < 5; c++) gl[c][0] = gl[c][1] = gl[c][2] = 0.0;
                    to_local(n, vl, gl, ql, dql);
                    nfb += 2;
                }
                bc_ghost_point(P, plane, vl, gl, vr, gr);
                to_local(n, vr, gr, qr, dqr);
            }
            real Fb[10];
            const int e = orc_gp_flux(P, ql, &dql[0][0], qr, &dqr[0][0], dt, Fb, NULL);
            if (e) {
                if (e > err) err = e;
                break;
            }
            double area = sqrt(F->va[k][0] * F->va[k][0] + F->va[k][1] * F->va[k][1] + F->va[k][2] * F->va[k][2]);
            for (int s = 0; s < 2; s++) {
                const real *Fl = Fb + 5 * s;
                real g[5];
                g[0] = Fl[0];
                g[4] = Fl[4];
                for (int q = 0; q < 3; q++) g[1 + q] = Fl[1] * n[0][q] + Fl[2] * n[1][q] + Fl[3] * n[2][q];
                for (int c = 0; c < 5; c++) acc[5 * s + c] += area * g[c];
            }
        }
        for (int c = 0; c < 10; c++) out[10 * f + c] = acc[c];
    }
    o->n_fallback += nfb;
    return err;
}

/* face fluxes [F][10]: (Fbar0, Fbar1), area-integrated, owner -> neighbour */
int orc_face_flux(orc *o, const orc_params *P, const real *Q, double dt, real *out)
{
    return face_flux_all(o, P, Q, dt, out);
}

/* L and dL/dt per cell, layout [5][n] each */
int orc_residual(orc *o, const orc_params *P, const real *Q, double dt, real *L, real *dL)
{
    int64_t n = o->n_cells;
    real *ff = malloc(sizeof(real) * 10 * o->n_faces);
    int e = face_flux_all(o, P, Q, dt, ff);
    if (e) {
        free(ff);
        return e;
    }
    for (int64_t i = 0; i < n; i++) {
        const ocell *C = &o->c[i];
        real s0[5] = {0}, s1[5] = {0};
        for (int p = 0; p < C->nf; p++) {
            double sg = C->fside[p] == 0 ? 1.0 : -1.0;
            const real *fx = ff + 10 * C->face[p];
            for (int c = 0; c < 5; c++) {
                s0[c] += sg * fx[c];
                s1[c] += sg * fx[5 + c];
            }
        }
        for (int c = 0; c < 5; c++) {
            L[c * n + i] = -s0[c] / C->vol;
            dL[c * n + i] = -s1[c] / C->vol;
        }
    }
    free(ff);
    return 0;
}

/* time step: CFL min_i h_i / (|U_i| + c_i), h_i = 6 |Omega_i| / sum of face areas */
double orc_timestep(const orc *o, const orc_params *P, const real *Q)
{
    int64_t n = o->n_cells;
    double dt = INFINITY;
    for (int64_t i = 0; i < n; i++) {
        double q[5], U[3];
        for (int c = 0; c < 5; c++) q[c] = RE(Q[c * n + i]);
        const double rho = q[0];
        for (int d = 0; d < 3; d++) U[d] = q[1 + d] / q[0];
        const double p = (P->gamma - 1.0) * (q[4] - 0.5 * q[0] * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
        if (!(rho > 0 && p > 0)) return -1.0;
        double h = 6.0 * o->c[i].vol / o->c[i].area_sum;
        double s = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) + sqrt(P->gamma * p / rho);
        double d = P->cfl * h / s;
        if (d < dt) dt = d;
    }
    return dt;
}

/* two-stage fourth-order step for a generic operator Q -> (L, dL/dt) */
typedef int (*orc_op)(void *ctx, const real *Q, real *L, real *dL);

int orc_s2o4(int64_t len, real *Q, double dt, orc_op op, void *ctx)
{
    real *L0 = malloc(sizeof(real) * len), *D0 = malloc(sizeof(real) * len);
    real *Qs = malloc(sizeof(real) * len), *L1 = malloc(sizeof(real) * len), *D1 = malloc(sizeof(real) * len);
    int e = op(ctx, Q, L0, D0);
    if (!e) {
        for (int64_t k = 0; k < len; k++) Qs[k] = Q[k] + 0.5 * dt * L0[k] + 0.125 * dt * dt * D0[k];
        e = op(ctx, Qs, L1, D1);
    }
    if (!e)
        for (int64_t k = 0; k < len; k++) Q[k] = Q[k] + dt * L0[k] + dt * dt / 6.0 * (D0[k] + 2.0 * D1[k]);
    free(L0);
    free(D0);
    free(Qs);
    free(L1);
    free(D1);
    return e;
}

typedef struct {
    orc *o;
    const orc_params *P;
    double dt;
} step_ctx;

static int scheme_op(void *vctx, const real *Q, real *L, real *dL)
{
    step_ctx *s = vctx;
    return orc_residual(s->o, s->P, Q, s->dt, L, dL);
}

int orc_step(orc *o, const orc_params *P, real *Q, double dt)
{
    step_ctx s = {o, P, dt};
    return orc_s2o4(5 * o->n_cells, Q, dt, scheme_op, &s);
}

/*
 * Advance nsteps steps (or up to t_end when t_end > 0, the last step shortened).
 * dt_fixed > 0 uses that step size instead of the CFL one.  dts (optional)
 * receives the step sizes.  Returns 0 or a status code.
 */
int orc_run(orc *o, const orc_params *P, real *Q, int nsteps, double t_end, double dt_fixed, double *dts, int *steps_done,
            double *t_out)
{
    double t = 0.0;
    int k = 0;
    for (;;) {
        if (t_end > 0) {
            if (t >= t_end * (1.0 - 1e-14)) break;
        } else if (k >= nsteps)
            break;
        double dt = dt_fixed > 0 ? dt_fixed : orc_timestep(o, P, Q);
        if (!(dt > 0)) return 4;
        if (t_end > 0 && t + dt > t_end) dt = t_end - t;
        int e = orc_step(o, P, Q, dt);
        if (e) return e;
        if (dts) dts[k] = dt;
        t += dt;
        k++;
    }
    if (steps_done) *steps_done = k;
    if (t_out) *t_out = t;
    return 0;
}

/* ------------------------------------------------------------------ */
/* raw entry points used by the pin tests                               */
/* ------------------------------------------------------------------ */
/* volume, centroid and second central moment means of one cell given its vertices in the paper's order */
void orc_cell_moments_raw(int type, const double *verts, double *vol, double *xc, double *m2)
{
    orc tmp;
    memset(&tmp, 0, sizeof tmp);
    int8_t t = (int8_t)type;
    int64_t cells[8];
    for (int q = 0; q < 8; q++) cells[q] = q;
    tmp.nodes = verts;
    tmp.types = &t;
    tmp.cells = cells;
    ocell C;
    memset(&C, 0, sizeof C);
    cell_moments(&tmp, 0, &C);
    *vol = C.vol;
    for (int q = 0; q < 3; q++) xc[q] = C.xc[q];
    for (int q = 0; q < 6; q++) m2[q] = C.m2[q];
}

/* Gauss points and weighted vector areas of the bilinear patch through quad (x1..x4 cyclic) */
void orc_face_gauss_raw(const double *quad, double *gp, double *va)
{
    double Xq[4][3], g[4][3], v[4][3];
    for (int m = 0; m < 4; m++)
        for (int q = 0; q < 3; q++) Xq[m][q] = quad[3 * m + q];
    face_gauss(Xq, g, v);
    for (int k = 0; k < 4; k++)
        for (int q = 0; q < 3; q++) {
            gp[3 * k + q] = g[k][q];
            va[3 * k + q] = v[k][q];
        }
}

/* boundary condition of box plane `plane` applied to a cell average (g) and at a Gauss point on the
   plane (gp, ggp [5][3]: the value and gradient beyond it from the inner v, gv [5][3]) */
void orc_bc_ghost(const orc_params *P, int plane, const real *v, const real *gv, real *g, real *gp, real *ggp)
{
    real gvv[5][3], gg[5][3];
    for (int c = 0; c < 5; c++)
        for (int q = 0; q < 3; q++) gvv[c][q] = gv[3 * c + q];
    bc_state(P, plane, v, g);
    bc_ghost_point(P, plane, v, gvv, gp, gg);
    for (int c = 0; c < 5; c++)
        for (int q = 0; q < 3; q++) ggp[3 * c + q] = gg[c][q];
}

/* normalised Maxwellian moments <u^n> full / u>0 / u<0 (n < 14) and <varsigma^(2d)> (d < 6) */
void orc_maxwell_moments(double U, double lam, double K, double *full, double *pos, double *neg, double *s)
{
    maxw g;
    maxw_init(&g, 1.0, U, 0.0, 0.0, lam, K);
    for (int n = 0; n < MAXO; n++) {
        full[n] = RE(g.uf[n]);
        pos[n] = RE(g.up[n]);
        neg[n] = RE(g.un[n]);
    }
    for (int d = 0; d < 6; d++) s[d] = RE(g.s[d]);
}

/* big-stencil members of cell c (cell ids and image shifts); returns K */
int orc_stencil_members(const orc *o, int64_t c, int64_t *ids, int *sh)
{
    const ocell *C = &o->c[c];
    for (int k = 0; k < C->K; k++) {
        ids[k] = C->st[k].cell;
        for (int q = 0; q < 3; q++) sh[3 * k + q] = C->st[k].of[q];
    }
    return C->K;
}

/* sub-stencil m members of cell c; returns their count */
/* reflection signs of the big stencil's members [K][3] (+1: no reflection on that axis) */
int orc_stencil_signs(const orc *o, int64_t c, int *sg)
{
    const ocell *C = &o->c[c];
    for (int k = 0; k < C->K; k++)
        for (int q = 0; q < 3; q++) sg[3 * k + q] = C->st[k].sg[q];
    return C->K;
}

int orc_substencil_members(const orc *o, int64_t c, int m, int64_t *ids, int *sh)
{
    const ocell *C = &o->c[c];
    if (m < 0 || m >= C->M) return 0;
    for (int k = 0; k < C->subn[m]; k++) {
        ids[k] = C->sub[m][k].cell;
        for (int q = 0; q < 3; q++) sh[3 * k + q] = C->sub[m][k].of[q];
    }
    return C->subn[m];
}

/* faces of cell c in the paper's F_p order and the side (0 owner, 1 neighbour); returns the face count */
int orc_cell_faces(const orc *o, int64_t c, int64_t *faces, int *side)
{
    const ocell *C = &o->c[c];
    for (int p = 0; p < C->nf; p++) {
        faces[p] = C->face[p];
        side[p] = C->fside[p];
    }
    return C->nf;
}
