/*
 * gks.h -- C ABI of the MI355X third-order gas-kinetic scheme on hybrid
 * unstructured meshes (Yang, Pan & Xu, arXiv 2203.09047).
 *
 * The library computes the explicit hot path of the method on one gfx950 GPU:
 *   WENO reconstruction per cell (Section 2: least-squares quadratic on the
 *   big stencil, linear polynomials on the sub-stencils, linear weights,
 *   smoothness indicators of Eq. indicator, nonlinear combination Eq. weno),
 *   the BGK time-dependent flux at the four Gauss points of every face
 *   (Section 3.2, Eq. flux-1, integrated over the face with Eq. flux-qud),
 *   and the two-stage fourth-order time step (Section 3.3, applied to the
 *   semi-discrete operator of Eq. semi / Eq. finite).
 *
 * Conventions shared by every entry point:
 *   - Cell indices are the library's internal order (cells sorted along a
 *     Morton space-filling curve of their centroids).  gks_host_mesh_perm()
 *     maps internal index -> index in the caller's mesh records.
 *   - Conserved variables Q are structure-of-arrays FP64 [5][n_cells]:
 *     rho, rho U, rho V, rho W, rho E.
 *   - Every device pointer is owned by the caller.  The library never
 *     allocates device memory in a compute call; the mesh arena and the work
 *     buffer are sized by gks_mesh_sizes() and passed in.  Host objects
 *     (gks_host_mesh, gks_mesh handles) are allocated with malloc/new and
 *     released by their destroy calls.
 *   - Compute calls are asynchronous on the given stream (NULL = default
 *     stream of the current device) and only enqueue kernels.
 *   - Errors are status codes; no call aborts or throws across the ABI.
 *     gks_last_error() returns a thread-local message for the last failure.
 *   - Non-physical states (rho <= 0 or p <= 0 at a cell or a Gauss point,
 *     or a NaN) set a sticky flag in the work buffer; gks_poll_status()
 *     synchronises the stream and reports GKS_ENONPHYS.  Nothing is
 *     repaired silently.
 */
#ifndef GKS_H
#define GKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *gks_stream_t; /* a hipStream_t */

typedef enum {
    GKS_OK = 0,
    GKS_EINVAL = 1,     /* bad pointer, size or parameter */
    GKS_EDEVICE = 2,    /* HIP runtime error (see gks_last_error) */
    GKS_ESINGULAR = 3,  /* a least-squares fit stayed rank deficient after growing its stencil */
    GKS_ENONPHYS = 4,   /* sticky: non-physical state met in a kernel */
    GKS_EMESH = 5       /* mesh records are not a conforming (periodic) mesh */
} gks_status;

typedef enum { GKS_FP64 = 0, GKS_FP32_MIXED = 1 } gks_precision;

/*
 * Boundary condition of one box plane of a mesh with walls (gks_preprocess
 * with periodic = 0).  Section 2 builds stencils across a boundary from ghost
 * cells: the mirror images of interior cells, whose flow variables the
 * condition sets from the mirrored cell's.  At a face Gauss point on the
 * plane the state beyond it is the condition applied to the inner
 * reconstructed state (its gradient by the chain rule, the derivative across
 * the plane negated); the far field's ghost is uniform.
 *   GKS_BC_SLIP        reflective wall: normal momentum negated (the default);
 *   GKS_BC_NOSLIP      adiabatic no-slip wall moving with velocity uw:
 *                      U -> 2 uw - U, density and pressure kept;
 *   GKS_BC_ISOTHERMAL  no-slip wall at temperature Tw = p / rho (gas constant 1):
 *                      U -> 2 uw - U, T -> 2 Tw - T, pressure kept (the
 *                      paper's cavity: "isothermal and nonslip");
 *   GKS_BC_FARFIELD    Riemann invariants U_n +- 2c/(gamma-1) along the outward
 *                      normal against the free stream far = (rho, U, V, W, p):
 *                      the outgoing one from the interior, the incoming one
 *                      from the free stream, entropy and tangential velocity
 *                      from the upwind side; supersonic inflow takes the free
 *                      stream, supersonic outflow the interior (the sphere's
 *                      inlet and outlet);
 *   GKS_BC_EXTRAPOLATE the ghost repeats the mirrored cell (zero-gradient
 *                      outflow; the Riemann problems' non-reflecting ends).
 */
typedef enum {
    GKS_BC_SLIP = 0,
    GKS_BC_NOSLIP = 1,
    GKS_BC_ISOTHERMAL = 2,
    GKS_BC_FARFIELD = 3,
    GKS_BC_EXTRAPOLATE = 4
} gks_bc_type;

typedef struct {
    int type;      /* gks_bc_type */
    double uw[3];  /* wall velocity (no-slip types; tangential to the plane) */
    double Tw;     /* wall temperature p / rho (isothermal; > 0) */
    double far[5]; /* free stream rho, U, V, W, p (far field; rho, p > 0) */
} gks_boundary;

/*
 * Scheme parameters.  Defaults (gks_default_params) follow the paper:
 * gamma = 1.4; linear weights gamma_m = 0.0125 for every sub-stencil and
 * gamma_0 = 1 - 0.0125 M (Section 2); nonlinear weights
 * w_m = gamma_m (1 + (tau_w / (beta_m + weno_eps))^weno_p) with weno_p = 1
 * and weno_eps = 1e-6 (the paper leaves epsilon unspecified); collision time
 * tau = tau_eps dt + tau_C |p_l - p_r| / (p_l + p_r) dt for inviscid flow and
 * mu / p_0 + tau_C |p_l - p_r| / (p_l + p_r) dt for viscous flow with
 * tau_eps = 0.01, tau_C = 1 (opening of Section 5); CFL time step
 * dt = cfl min_i h_i / (|U_i| + c_i) with h_i = 6 |Omega_i| / (sum of face areas).
 * Pr != 1 adds (1/Pr - 1) q to the energy flux, q being the heat flux of the
 * time-integrated distribution about the interface velocity.
 */
typedef struct {
    double gamma;
    double cfl;
    double mu;
    double Pr;
    double weno_eps;
    double weno_gamma_m;
    double weno_p;
    double tau_eps;
    double tau_C;
    int viscous;      /* 0: Euler, 1: Navier-Stokes collision time */
    int precision;    /* gks_precision */
    int force_linear; /* 1: use the linear weights (testing of the quadratic reproduction) */
    int dt_given;     /* 1: gks_s2o4_step uses *dt_dev as given instead of computing the CFL step */
    int first_order_fallback; /* 1: a reconstructed side state at a Gauss point with rho <= 0 or
                                 p <= 0 is replaced by its cell's average with zero slopes (first
                                 order there) and counted (gks_fallback_count); 0: the paper's scheme */
    double fallback_floor;    /* with first_order_fallback: a side state also falls back when its
                                 rho or p is at most fallback_floor times its cell average's
                                 (0: positivity only; must lie in [0, 1)) */
    int smooth_flux;          /* 1: the smooth-flow distribution of Eq. flux-2 at the Gauss points,
                                 f = g0 (1 - tau (abar . u + Abar) + Abar t) (with the -tau Abar term
                                 that the smooth limit of Eq. flux-1 carries; the printed equation
                                 drops it), for smooth flows; 0: Eq. flux-1 (the default) */
    double mu_power;          /* viscous only: mu (T0 / T_ref)^mu_power in the collision time, T0 = p0 / rho0
                                 the interface temperature (gas constant 1): the power law of the
                                 paper's hypersonic case (Section 5, exponent 0.7 there); 0 (the
                                 default): constant mu.  The adjoint refuses it (GKS_EINVAL) */
    double T_ref;             /* the temperature at which the viscosity is mu (> 0 when used; default 1) */
    double dt_max;            /* > 0: the CFL step is capped at dt_max on the device (the time left to an
                                 end time, so that the last step lands on it); 0 (the default): no cap */
    gks_boundary bc[6];       /* conditions of the box planes x = 0, x = L, y = 0, y = L, z = 0, z = L
                                 (index 2 axis + hi) on a mesh with walls; ignored on periodic meshes.
                                 Default: all GKS_BC_SLIP.  Conditions other than the reflective one
                                 are refused (GKS_EINVAL) on a mesh so thin that a stencil reaches across
                                 both walls of an axis */
} gks_params;

typedef struct gks_host_mesh gks_host_mesh;
typedef struct gks_mesh gks_mesh;

void gks_default_params(gks_params *p);

/*
 * Build the host-side preprocessed mesh (Section 2: face labels of the four
 * cell types, degenerate-hexahedron trilinear maps, 3x3x3 volume Gauss rule,
 * bilinear faces with 2x2 Gauss points, big stencil and sub-stencils, FP64
 * least-squares pseudo-inverses; plus the Morton reorder of the cells).
 *   nodes  [n_nodes][3] FP64 coordinates;
 *   types  [n_cells] int8: 0 tetrahedron, 1 pyramid, 2 prism, 3 hexahedron;
 *   cells  [n_cells][8] int64 node ids in the paper's vertex order, -1 padded;
 *   box    [3] periodic box lengths (the domain is [0,box_x] x [0,box_y] x [0,box_z]);
 *   periodic: 1, every face is shared by exactly two cells, opposite faces of
 *     the box matched as periodic images; 0, a face of one cell must lie on a
 *     face of the box (a wall): the cell's neighbour across it is its own
 *     mirror image (the image's neighbours are the mirrors of the cell's
 *     neighbours), its state given by the plane's condition (gks_params.bc,
 *     reflective by default: the cell's with the normal momentum negated);
 *   min_big_stencil: 0 keeps the paper's big stencil (face neighbours and
 *     their face neighbours); k > 0 also grows a big stencil with fewer than
 *     k members, by the rule used for ill-posed fits (face neighbours of the
 *     members, in order), to k members where the mesh has them.  The paper's
 *     rule gives 12-member stencils on some tetrahedra of mixed meshes, on
 *     which the linear scheme is unstable; 16 is the size it gives a
 *     tetrahedron whose neighbours share no other cell.
 * All arrays are read only during the call.  Returns GKS_EMESH for a
 * non-conforming mesh and GKS_ESINGULAR when a fit cannot be made well posed.
 */
gks_status gks_preprocess(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types,
                          const int64_t *cells, const double *box, int periodic, int min_big_stencil,
                          gks_host_mesh **out);
void gks_host_mesh_free(gks_host_mesh *h);

/*
 * n_cells, n_faces, stencil entries (members of all cells), sub-stencil
 * entries (members of all sub-stencils of all cells), and the number of
 * members appended by rank growth.
 * Any pointer may be NULL.
 */
gks_status gks_host_mesh_counts(const gks_host_mesh *h, int64_t *n_cells, int64_t *n_faces, int64_t *n_stencil,
                                int64_t *n_subcoef, int64_t *n_grown);
/* perm[n_cells]: internal index -> caller's cell index */
gks_status gks_host_mesh_perm(const gks_host_mesh *h, int64_t *perm);
/* per cell (internal order): volume, centroid [n][3]; either pointer may be NULL */
gks_status gks_host_mesh_geometry(const gks_host_mesh *h, double *vol, double *xc);
/* per face: owner and neighbour (internal indices; a wall face on box plane 2 axis + hi has neighbour
   -1 - (2 axis + hi)) */
gks_status gks_host_mesh_faces(const gks_host_mesh *h, int32_t *owner, int32_t *nbr);
/*
 * Face Gauss-point geometry [9][4 n_faces] (Gauss point 4 f + g): offset from
 * the owner's centroid (3), offset from the neighbour's (image) centroid (3),
 * weighted vector area (3), as the flux kernel reads it.
 */
gks_status gks_host_mesh_face_geometry(const gks_host_mesh *h, double *fgeo);

/*
 * Bytes of the device mesh arena and of the work buffer for a precision, and
 * of one step's coefficient tape (the optional coeff_tape of gks_s2o4_step,
 * read back by gks_adjoint_step: both stages' per-cell quadratics,
 * 2 x n_cells x 50 elements of the precision).  The work buffer holds the
 * stage state, reconstruction coefficients, face fluxes, time-step partials
 * and the status word.  Any output pointer may be NULL.
 */
gks_status gks_mesh_sizes(const gks_host_mesh *h, int precision, size_t *mesh_bytes, size_t *work_bytes,
                          size_t *tape_bytes_per_step);

/*
 * Upload the mesh into the caller's device arena (mesh_bytes from
 * gks_mesh_sizes, 256-byte aligned) on the stream and synchronise it.
 * The returned handle refers to the arena; it does not own it.
 */
gks_status gks_init_mesh(const gks_host_mesh *h, int precision, void *mesh_arena, size_t mesh_bytes,
                         gks_stream_t stream, gks_mesh **out);
void gks_destroy_mesh(gks_mesh *m);

/* Clear the sticky status word of a work buffer (enqueued on the stream). */
gks_status gks_reset_status(gks_mesh *m, void *work, gks_stream_t stream);

/*
 * CFL time step (reading of the paper's time-step step of its solution
 * algorithm, which gives no formula): *dt_dev = cfl min_i h_i / (|U_i| + c_i),
 * computed in FP64 with a deterministic two-pass minimum, and capped at
 * p->dt_max when that is positive.
 */
gks_status gks_timestep(gks_mesh *m, const double *Q, const gks_params *p, double *dt_dev, void *work,
                        gks_stream_t stream);

/*
 * WENO reconstruction (Section 2, Eq. weno).  Every candidate polynomial is a
 * polynomial in the same zero-mean basis, so the nonlinear combination of
 * Eq. weno is itself one quadratic per cell and component.  Output coeff
 * [n_cells][5][10] (FP64, or FP32 for GKS_FP32_MIXED): for component c,
 * entry 0 is the constant term and entries 1..9 the coefficients of the
 * monomials x y z xx xy xz yy yz zz of (x - x_c), so that the reconstructed
 * value at x is coeff[0] + sum_n coeff[n] (x - x_c)^n; in FP32_MIXED mode
 * entry 0 excludes the cell average, which is added back in FP64.
 */
gks_status gks_reconstruct(gks_mesh *m, const double *Q, void *coeff, const gks_params *p, void *work,
                           gks_stream_t stream);

/*
 * Face fluxes (Section 3.2, Eq. flux-1 at each Gauss point, Eq. flux-qud over
 * the face).  For each face the time integrals F(dt/2) and F(dt) of the
 * area-integrated flux give Fbar0 = (4 F(dt/2) - F(dt)) / dt (flux at the
 * start of the step) and Fbar1 = 4 (F(dt) - 2 F(dt/2)) / dt^2 (its time
 * derivative).  face_flux is [n_faces][10] (FP64, or FP32 for
 * GKS_FP32_MIXED), oriented owner -> neighbour.  dt_dev is read on the device.
 */
gks_status gks_flux(gks_mesh *m, const void *coeff, const double *Q, const double *dt_dev, void *face_flux,
                    const gks_params *p, void *work, gks_stream_t stream);

/*
 * Semi-discrete operator (Eq. finite) and its time derivative:
 * L_i = -(1/|Omega_i|) sum_p s_p Fbar0_p, dL_i = -(1/|Omega_i|) sum_p s_p Fbar1_p,
 * each [5][n_cells] FP64, gathered per cell in a fixed face order.
 */
gks_status gks_residual(gks_mesh *m, const void *face_flux, double *L, double *dL, const gks_params *p,
                        gks_stream_t stream);

/*
 * One two-stage fourth-order step (Section 3.3):
 *   Q* = Q + dt/2 L(Q) + dt^2/8 dL(Q),
 *   Q <- Q + dt L(Q) + dt^2/6 (dL(Q) + 2 dL(Q*)),
 * with the same dt in both stages.  Q is updated in place.  If p->dt_given
 * is 0 the CFL step is computed first into *dt_dev; otherwise *dt_dev is
 * used as given.  Q_star (optional, may be NULL) receives Q* [5][n_cells].
 * coeff_tape (optional, may be NULL): device buffer of 2 x n_cells x 50
 * elements of the mesh precision that receives both stages' reconstructions
 * (the per-cell quadratics of Q and of Q*, layout [2][n_cells][5][10]); the
 * adjoint step can reuse it instead of reconstructing again.
 */
gks_status gks_s2o4_step(gks_mesh *m, double *Q, double *dt_dev, const gks_params *p, void *work, double *Q_star,
                         void *coeff_tape, gks_stream_t stream);

/*
 * Allocation-free variant of gks_s2o4_step, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and results, with the work buffer
 * replaced by a static device array of the library (64 MiB, held by every
 * device the library runs on until the process ends).  Meshes whose work
 * buffer (gks_mesh_sizes) exceeds 64 MiB are refused with GKS_EINVAL (about
 * 100 k hybrid cells in FP64, 200 k in FP32_MIXED).  The call allocates
 * nothing and only enqueues kernels and copies on the stream.
 *   status_dev: caller-owned device int32[2] that takes the role of the work
 *     buffer's status word: word 0 becomes nonzero when a non-physical state
 *     is met, word 1 counts first-order fallbacks.  Sticky: the call never
 *     clears it (the caller zeroes it before the first call).
 * Other arguments as gks_s2o4_step.  Every call on one device shares that
 * device's array, so calls that overlap in time on one device (different
 * streams, threads or meshes) race and must be serialised by the caller.
 */
gks_status gks_s2o4_step_noalloc(gks_mesh *m, double *Q, double *dt_dev, const gks_params *p, int32_t *status_dev,
                                 double *Q_star, void *coeff_tape, gks_stream_t stream);

/*
 * One implicit step of the steady solver (Section 3.3: Eq. impEuler with the
 * flux-split operator of Eq. euler-scheme, solved by the Jacobi iteration of
 * Eq. jacobi with kmax sweeps).  Res = L + dt_f/2 dL/dt is the GKS residual
 * (reconstruction + Eq. flux-1, or Eq. flux-2 with smooth_flux) integrated
 * over the flux step dt_f = *dt_dev (the CFL step unless p->dt_given); the
 * implicit pseudo-time step is dt = dt_factor * dt_f.  Per cell i, with T
 * the Euler flux along the outward face normal, S the face area and
 * r = |U_nb . n| + c_nb at t_n:
 *   D_i dQ_i^(k) = |Omega_i| Res_i - 1/2 sum_f [T(Q_nb + dQ_nb^(k-1)) - T(Q_nb) - r dQ_nb^(k-1)] S,
 *   D_i = |Omega_i| / dt + 1/2 sum_f r S,  dQ^(0) = |Omega| Res / D,
 * and Q += dQ^(kmax) in place.  On a mesh with walls the neighbour across a
 * face on a box plane is the ghost of Section 2's construction, the plane's
 * condition (p->bc) on the cell's own state, Q_nb = B(Q_i), and its increment
 * dQ_nb = B(Q_i + dQ_i) - B(Q_i) with the cell's previous iterate.  The work
 * buffer's coefficient area holds the iteration.  dt_factor > 0,
 * 0 <= kmax <= 1000 (GKS_EINVAL otherwise).  The paper times this path with
 * kmax = 3 (the lid-driven cavity with the smooth-flow flux, and the sphere).
 */
gks_status gks_implicit_step(gks_mesh *m, double *Q, double *dt_dev, double dt_factor, int kmax, const gks_params *p,
                             void *work, gks_stream_t stream);

/*
 * Discrete adjoint of one S2O4 step (FP64 meshes only), the dt of the step
 * being a constant.  With the step written as
 *   Q* = Q + dt/2 L(Q) + dt^2/8 D(Q),  Q' = Q + dt L(Q) + dt^2/6 (D(Q) + 2 D(Q*)),
 * and lam' = dJ/dQ' [5][n_cells] (device), it computes
 *   lam* = dt^2/3 J_D(Q*)^T lam',
 *   lam  = lam' + lam* + J_L(Q)^T (dt lam' + dt/2 lam*) + J_D(Q)^T (dt^2/6 lam' + dt^2/8 lam*)
 * into lam_n, where J_L, J_D are the Jacobians of the reconstruction -> flux ->
 * Eq. finite operator (including the nonlinear WENO weights and the collision
 * time; |x| is differentiated as sign(x), sign(0) = 0).  Qn and Qstar are the
 * step's start state and stage state (as produced by gks_s2o4_step), dt_dev
 * the step's dt.  adj_work: caller-owned device buffer of the size that
 * gks_adjoint_work_bytes() reports, 256-byte aligned.  coeff_tape (optional,
 * may be NULL): the step's coefficient tape from gks_s2o4_step
 * (tape_bytes_per_step of gks_mesh_sizes); when given, the two
 * reconstructions of Qn and Qstar are read from it instead of recomputed.
 * Periodic meshes only (GKS_EINVAL on a mesh with walls), with the
 * first-order fallback, the smooth flux and the viscosity power law off
 * (GKS_EINVAL otherwise: the adjoint differentiates Eq. flux-1 without the
 * fallback's switch).  Every gather runs in a fixed order (no atomics): the
 * result is bitwise reproducible, and the same with or without the tape.
 * The same conventions define the tangent of the FP64 reference it is
 * tested against.
 */
gks_status gks_adjoint_work_bytes(const gks_host_mesh *h, size_t *bytes);
gks_status gks_adjoint_step(gks_mesh *m, const double *Qn, const double *Qstar, const double *dt_dev,
                            const double *lam_np1, double *lam_n, const gks_params *p, void *adj_work,
                            const double *coeff_tape, gks_stream_t stream);

/*
 * Flow functional J = sum_i |Omega_i| |rho U_i|^2 / (2 rho_i) (kinetic energy)
 * into *J_dev (deterministic two-pass sum), and its gradient dJ/dQ [5][n]
 * into dJdQ when not NULL.  Uses the time-step partials of the work buffer.
 */
gks_status gks_kinetic_energy(gks_mesh *m, const double *Q, double *J_dev, double *dJdQ, void *work,
                              gks_stream_t stream);

/* Synchronise the stream and report GKS_ENONPHYS if the sticky flag is set. */
gks_status gks_poll_status(gks_mesh *m, void *work, gks_stream_t stream);

/* Synchronise and read (then reset) the number of Gauss-point side states
 * that fell back to first order since the last read (first_order_fallback). */
gks_status gks_fallback_count(gks_mesh *m, void *work, int64_t *count, gks_stream_t stream);

/*
 * Gauss-point flux in the local frame for a batch (kernel-level testing of the
 * flux of Section 3.2).  ql, qr [n][5]: conserved states with the momentum in
 * the (n1, n2, n3) frame; dql, dqr [n][3][5]: their derivatives along n1, n2,
 * n3; dt [n]; out [n][10]: (Fbar0, Fbar1) per unit area.  Device pointers;
 * FP64, or FP32 arithmetic for GKS_FP32_MIXED (inputs and outputs stay FP64).
 */
gks_status gks_gp_flux_batch(int64_t n, const double *ql, const double *dql, const double *qr, const double *dqr,
                             const double *dt, double *out, const gks_params *p, gks_stream_t stream);

/*
 * Testing aid for the FP64 flux of periodic meshes without the fallback (the
 * flux of Section 3.2 at the Gauss points of Eq. flux-qud) and for the first
 * kernel of its reverse in gks_adjoint_step.  Those kernels stage the
 * coefficients of the cells owning a chunk of faces in a window of up to 92
 * consecutive cells in device shared memory (faces are sorted by owner) and
 * read an owner beyond the window from memory directly.  cells in [0, 92]
 * narrows the window of this mesh handle (0: every owner read directly), so
 * that tests can run the direct path; the results are bitwise the same for every
 * value.  Default 92.  GKS_EINVAL for a null handle or a value outside the range.
 */
gks_status gks_set_flux_window(gks_mesh *m, int cells);

/*
 * Optional per-kernel timing with HIP events recorded on the launch stream
 * around every kernel the library enqueues (host-side events owned by the
 * mesh handle; no device memory).  gks_profile_read synchronises on the last
 * event, returns the summed milliseconds and launch counts per kernel id
 * (arrays of GKS_K_COUNT) and clears the record.
 */
enum {
    GKS_K_TIMESTEP = 0,
    GKS_K_RECONSTRUCT = 1,
    GKS_K_FLUX = 2,
    GKS_K_STAGE1 = 3,
    GKS_K_STAGE2 = 4,
    GKS_K_RESIDUAL = 5,
    GKS_K_FLUX_ADJ = 6,
    GKS_K_RECONSTRUCT_ADJ = 7,
    GKS_K_GATHER_ADJ = 8,
    GKS_K_IMPLICIT = 9,
    GKS_K_COUNT = 10
};
gks_status gks_profile(gks_mesh *m, int enable);
gks_status gks_profile_read(gks_mesh *m, double *total_ms, int64_t *launches);

/*
 * Host (CPU) execution of the same templated Gauss-point flux and of its
 * hand-written reverse (vector-Jacobian product), for testing the adjoint
 * against finite differences.  gks_gp_flux_host runs in FP32 arithmetic when
 * p->precision is GKS_FP32_MIXED (inputs and outputs stay FP64), else FP64;
 * the reverse is FP64.  Arguments as gks_gp_flux_batch for
 * one point (host pointers); outb [10] is the cotangent of (Fbar0, Fbar1),
 * qlb, qrb [5] and dqlb, dqrb [3][5] receive the input cotangents.
 */
gks_status gks_gp_flux_host(const double *ql, const double *dql, const double *qr, const double *dqr, double dt,
                            const gks_params *p, double *out);
gks_status gks_gp_flux_vjp_host(const double *ql, const double *dql, const double *qr, const double *dqr, double dt,
                                const gks_params *p, const double *outb, double *qlb, double *dqlb, double *qrb,
                                double *dqrb);

/*
 * Host execution of the WENO combination of one cell and component (after the
 * stencil sums) and of its reverse, FP64, for testing the adjoint:
 * a [9] quadratic coefficients, r [8][3] sub-stencil sums sum_k D_k (Q_k - Q_0),
 * gi [8][6] inverses of the sub-stencil normal matrices (divided by h),
 * M sub-stencils, v23 = |Omega|^(2/3), S [6] centred second moments, q0 the cell
 * average; c [10] the combined quadratic.  The reverse maps cb [10] to
 * ab [9], rb [8][3] and the direct cotangent of q0.
 */
gks_status gks_weno_combine_host(const double *a, const double *r, const double *gi, int M, double v23,
                                 const double *S, double q0, const gks_params *p, double *c);
gks_status gks_weno_combine_vjp_host(const double *a, const double *r, const double *gi, int M, double v23,
                                     const double *S, const gks_params *p, const double *cb, double *ab, double *rb,
                                     double *q0b);

/*
 * Floating-point operations of one face Gauss point of the flux kernel
 * (two-sided state evaluation, frame, BGK flux with both time integrals,
 * rotation back), counted by executing the kernel's templated body on the
 * host with an operation-counting number type: additions/subtractions,
 * multiplications, divisions, and transcendental calls (erfc, exp, expm1,
 * sqrt).  viscous/Pr select the collision-time and Prandtl branches.
 */
gks_status gks_gp_op_count(int viscous, double Pr, int64_t *adds, int64_t *muls, int64_t *divs, int64_t *transc);

const char *gks_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GKS_H */
