// Device library of the gas-kinetic solver for gfx950 (MI355X): kernels and C ABI.
//
// Kernels (one stage of the two-stage fourth-order step runs K1 -> K2 -> K3):
//   K0 timestep  : CFL time step, FP64 two-pass deterministic minimum.
//   K1 reconstruct: one lane per (cell, conserved component).  Streams the
//                  cell's stencil once: differences Q_k - Q_0, the quadratic
//                  fit a = A^+ (Q_k - Q_0) and the linear sub-stencil fits
//                  b^m; smoothness indicators (Eq. indicator), nonlinear
//                  weights, and Eq. weno collapsed into one quadratic.
//   K2 flux      : one lane per (face, Gauss point); reconstructed states on
//                  both sides, local frame, BGK flux of Eq. flux-1 with both
//                  time integrals, rotated back and weighted (Eq. flux-qud);
//                  the four Gauss points of a face are summed across lanes in
//                  a fixed butterfly order.
//   K3 update    : one lane per cell; gathers its face fluxes in F_p order
//                  (no atomics, so results are bitwise reproducible), forms
//                  L and dL/dt (Eq. finite) in FP64 and applies a stage of
//                  the two-stage fourth-order step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gks_flux.h"
#include "gks_flux_adj.h"
#include "gks_weno.h"
#include "gks_internal.h"
#include "gks_opcount.h"

namespace gks {

static thread_local std::string g_err;

gks_status fail(gks_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

static gks_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GKS_OK;
    return fail(GKS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// device mesh
// ---------------------------------------------------------------------------
struct DevMesh {
    int n, nf;
    int precision;
    // cells
    const int8_t *M;        // number of sub-stencils
    const double *vol;      // |Omega|
    const double *vol23;    // |Omega|^(2/3)
    const double *m2;       // [6][n] centred second moments (means)
    const double *hcfl;     // 6 |Omega| / sum of face areas
    const int32_t *st_ptr;  // [n+1]
    const int2 *st_rec;     // members: {cell, sub-stencil membership mask}
    int nnz;                // stencil members
    const void *pinv;       // [nnz][9] (member-major), FP64 or FP32
    const void *dsc;        // [nnz][3] scaled member centroid offsets, FP64 or FP32
    const void *ginv;       // [48][n] inverses of the sub-stencil normal matrices / h, FP64 or FP32
    const int32_t *st_cell; // [nnz] member cells (as in st_rec)
    const uint8_t *st_flip; // [nnz] bit d: the member is the mirror image across a wall on axis d (bit 3 + d:
                            // the wall at L; bit 6: mirrored at both walls of an axis)
    int walls;              // the mesh has walls (faces with nbr = -1 - plane, plane = 2 axis + hi)
    int double_mirror;      // some member is mirrored at both walls of an axis
    // sub-stencil lists: the members of sub-stencil s of cell i are entries
    // ss_ptr[8 i + s] .. ss_ptr[8 i + s + 1], each the member's position in the cell's
    // stencil and B = G_s^{-1} D_k / h, so that b^s = sum B (Q_k - Q_0)
    const int32_t *ss_ptr;  // [8 n + 1]
    const uint8_t *ss_loc;  // [nss]
    const void *ss_B;       // [nss][3], FP64 or FP32
    int nss;
    // faces
    const int32_t *owner, *nbr;
    const double *fgeo;     // [9][4 nf]
    const double *fnS;      // [4][nf]: unit normal (owner -> neighbour) and area of each face
    const int32_t *cf_ptr, *cf_idx;
    const int32_t *tr_ptr, *tr_idx;  // transposed stencil (adjoint gathers)
};

// work buffer: status word, time-step partials, Q*, coefficients, face fluxes
struct Work {
    int *status;
    double *dtpart;
    double *Qs;
    void *coeff;
    void *ff;
};

constexpr int kBlock = 256;
constexpr int kDtBlocks = 1024;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t work_layout(int64_t n, int64_t nf, int precision, Work *w, char *base)
{
    const size_t es = precision == GKS_FP32_MIXED ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return base ? (void *)(base + o) : nullptr;
    };
    void *st = take(256);
    void *dp = take(sizeof(double) * (kDtBlocks + 1));
    void *qs = take(sizeof(double) * 5 * n);
    void *co = take(es * 50 * n);
    void *ff = take(es * 10 * nf);
    if (w) {
        w->status = (int *)st;
        w->dtpart = (double *)dp;
        w->Qs = (double *)qs;
        w->coeff = co;
        w->ff = ff;
    }
    return off;
}

// Static scratch of the allocation-free step (gks_s2o4_step_noalloc): the same layout as a
// caller's work buffer, held by every device the library runs on until the process ends.  Host
// code never uses the array's name as an address: gks_init_mesh resolves each device's copy with
// hipGetSymbolAddress, with that device current, and the entry point passes that pointer.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// resolve (once) the scratch address of the current device
static gks_status scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(GKS_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return GKS_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(GKS_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    return GKS_OK;
}

static void *scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// ---------------------------------------------------------------------------
// K0: time step
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_dt_partial(int n, const double *__restrict__ Q, const double *__restrict__ hcfl,
                                                       double gam, double cfl, double *__restrict__ part, int *status)
{
    __shared__ double red[kBlock];
    double best = INFINITY;
    bool bad = false;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double r = Q[i], mx = Q[n + i], my = Q[2 * n + i], mz = Q[3 * n + i], E = Q[4 * n + i];
        const double ir = 1.0 / r;
        const double ke = 0.5 * (mx * mx + my * my + mz * mz) * ir;
        const double p = (gam - 1.0) * (E - ke);
        if (!(r > 0.0) || !(p > 0.0)) {
            bad = true;
            continue;
        }
        const double s = sqrt((mx * mx + my * my + mz * mz)) * ir + sqrt(gam * p * ir);
        best = fmin(best, cfl * hcfl[i] / s);
    }
    if (bad) status[0] = 1;
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// the minimum of the per-block partials, capped at dt_max when dt_max > 0 (the time left to an end time)
__global__ void __launch_bounds__(kBlock) k_dt_final(int nb, const double *__restrict__ part, double *dt, double dt_max)
{
    __shared__ double red[kBlock];
    double best = INFINITY;
    for (int i = threadIdx.x; i < nb; i += kBlock) best = fmin(best, part[i]);
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dt[0] = dt_max > 0.0 ? fmin(red[0], dt_max) : red[0];
}

// ---------------------------------------------------------------------------
// K1: WENO reconstruction, one lane per (cell, component)
// ---------------------------------------------------------------------------
// K1: reconstruction.  Four lanes cooperate on one (cell, conserved component):
// lane l streams members l, l+4, ... of the cell's stencil for the quadratic
// fit, so a cell's 20 lanes read consecutive pseudo-inverse entries, and lane l
// then fits sub-stencils l and l+4 from their member lists.  Partial sums are
// combined over the quad with DPP lane permutations, so every lane of the quad
// holds bitwise-identical totals (deterministic, no atomics).
// ---------------------------------------------------------------------------
// sign of conserved component c of a stencil member mirrored across the walls in flip (bit d: axis d)
__device__ __forceinline__ double mirror_sign(unsigned flip, int c)
{
    return c >= 1 && c <= 3 && (flip >> (c - 1) & 1u) ? -1.0 : 1.0;
}

constexpr int kK1Lanes = 4;
constexpr int kK1CellLanes = 5 * kK1Lanes;
// 12 cells = 240 lanes = 4 waves (the last one 48 lanes).  The forward reconstruction stages
// 40.8 KB per block in FP64 (four blocks per CU) and 31.6 KB in FP32 (five), its reverse
// 27.5 KB (five).  Blocks of 16 cells leave more of the CU waiting at the staging barrier and
// measured 19% slower (8 cells: 8% slower).
constexpr int kK1Cells = 12;
constexpr int kK1Block = kK1Cells * kK1CellLanes;
// Staged in LDS per block (the cells' stencil and sub-stencil ranges are contiguous): the
// members' cell averages, pseudo-inverse rows (forward kernel) and sub-stencil lists.  The
// reverse and the FP32 forward kernel stage up to 26 members and 50 sub-stencil entries per
// cell on average (the hybrid lattices' largest blocks hold 312 and 576; the FP64 forward
// kernel's limits are below).  A block whose ranges are longer reads them from global memory.
constexpr int kK1Stage = 26 * kK1Cells;
constexpr int kK1SubStage = 50 * kK1Cells;

// DPP lane permutations (VALU, no LDS traffic) of a 32-bit value within a quad of lanes
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) { return dpp_f32<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) { return dpp_f64<CTRL>(v); }

constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]

// Sum over a quad of lanes; every lane gets the bitwise-identical total
// (each step adds the same two partial sums, only in swapped order).
template <typename T>
__device__ __forceinline__ T quad_sum(T v)
{
    v += dpp_t<kDppQuadXor1>(v);
    v += dpp_t<kDppQuadXor2>(v);
    return v;
}

// Block index remap so that each of the 8 XCDs (which receive blocks round-robin)
// works through one contiguous range of blocks, keeping neighbour gathers in its L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}
// The WENO combination (Eq. weno, Eq. indicator) of one (cell, component) held by a
// quad of lanes: a[9] is the same on every lane, bs[h] is this lane's sub-stencil
// l + 4 h.  The indicator differences, the nonlinear weights and the linear parts
// of the sub-stencils are summed over the quad; every lane returns the same c[10].
template <typename T>
__device__ __forceinline__ void weno_combine_quad(const T a[9], const T bs[2][3], int l, int M, T v23, const T S[6],
                                                  double q0, bool with_q0, const WenoParams &wp, T c[10])
{
    const T H[3][3] = {{T(2) * a[3], a[4], a[5]}, {a[4], T(2) * a[6], a[7]}, {a[5], a[7], T(2) * a[8]}};
    const T Sm[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
    T beta0 = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T quad = T(0);
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) quad += H[d][p] * Sm[p][q] * H[d][q];
        beta0 += a[d] * a[d] + quad;
    }
    const T sec = T(4) * (a[3] * a[3] + a[6] * a[6] + a[8] * a[8]) + a[4] * a[4] + a[5] * a[5] + a[7] * a[7];
    beta0 = v23 * beta0 + v23 * v23 * sec;
    const T gm = (T)wp.gm, g0 = T(1) - gm * T(M), eps = (T)wp.eps, pw = (T)wp.p;
    T beta[2], tw = T(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        beta[h] = v23 * (bs[h][0] * bs[h][0] + bs[h][1] * bs[h][1] + bs[h][2] * bs[h][2]);
        if (l + 4 * h < M) tw += wabs(beta0 - beta[h]);
    }
    tw = quad_sum(tw) / T(M);
    T w0, ws[2];
    if (wp.force_linear) {
        w0 = g0;
        ws[0] = ws[1] = gm;
    } else {
        w0 = g0 * (T(1) + wpow(tw / (beta0 + eps), pw));
#pragma unroll
        for (int h = 0; h < 2; ++h) ws[h] = gm * (T(1) + wpow(tw / (beta[h] + eps), pw));
    }
    T wsum = T(0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (l + 4 * h < M) wsum += ws[h];
    const T isum = T(1) / (w0 + quad_sum(wsum));
    const T f0 = w0 * isum / g0;
#pragma unroll
    for (int j = 0; j < 9; ++j) c[1 + j] = f0 * a[j];
    const T sub0 = f0 * gm;
    T lin[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (l + 4 * h < M) {
            const T fs = ws[h] * isum - sub0;
            lin[0] += fs * bs[h][0];
            lin[1] += fs * bs[h][1];
            lin[2] += fs * bs[h][2];
        }
    c[1] += quad_sum(lin[0]);
    c[2] += quad_sum(lin[1]);
    c[3] += quad_sum(lin[2]);
    const T corr = -(c[4] * S[0] + c[5] * S[1] + c[6] * S[2] + c[7] * S[3] + c[8] * S[4] + c[9] * S[5]);
    c[0] = with_q0 ? (T)q0 + corr : corr;
}

// DPP broadcast of lane o of each quad of lanes to the whole quad
template <int O>
__device__ __forceinline__ double quad_bcast(double v)
{
    return dpp_f64<O | (O << 2) | (O << 4) | (O << 6)>(v);
}

/*
 * Reverse of weno_combine_quad (FP64): cb[10] (the same on every lane of the
 * quad) -> ab[9] (the same on every lane), bsb[h] (this lane's sub-stencils
 * l + 4 h) and q0b.  The forward quantities are recomputed; every sum over
 * sub-stencils is a quad sum, so the lanes stay bitwise identical.
 */
__device__ __forceinline__ void weno_combine_quad_b(const double a[9], const double bs[2][3], int l, int M, double v23,
                                                    const double S[6], const WenoParams &wp, const double cb_in[10],
                                                    double ab[9], double bsb[2][3], double &q0b)
{
    const double H[3][3] = {{2.0 * a[3], a[4], a[5]}, {a[4], 2.0 * a[6], a[7]}, {a[5], a[7], 2.0 * a[8]}};
    const double Sm[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
    double beta0 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double quad = 0.0;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) quad += H[d][p] * Sm[p][q] * H[d][q];
        beta0 += a[d] * a[d] + quad;
    }
    const double sec = 4.0 * (a[3] * a[3] + a[6] * a[6] + a[8] * a[8]) + a[4] * a[4] + a[5] * a[5] + a[7] * a[7];
    beta0 = v23 * beta0 + v23 * v23 * sec;
    const double gm = wp.gm, g0 = 1.0 - gm * M, eps = wp.eps, pw = wp.p;
    const bool lin = wp.force_linear != 0;
    bool on[2];
    double beta[2], xs[2], ws[2], tw = 0.0, wsum = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        on[h] = l + 4 * h < M;
        beta[h] = v23 * (bs[h][0] * bs[h][0] + bs[h][1] * bs[h][1] + bs[h][2] * bs[h][2]);
        if (on[h]) tw += wabs(beta0 - beta[h]);
    }
    tw = quad_sum(tw) / M;
    const double x0 = lin ? 0.0 : tw / (beta0 + eps);
    const double w0 = lin ? g0 : g0 * (1.0 + wpow(x0, pw));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        xs[h] = lin ? 0.0 : tw / (beta[h] + eps);
        ws[h] = lin ? gm : gm * (1.0 + wpow(xs[h], pw));
        if (on[h]) wsum += ws[h];
    }
    const double isum = 1.0 / (w0 + quad_sum(wsum));
    const double f0 = w0 * isum / g0;
    const double sub0 = f0 * gm;
    // reverse of c[0] = q0 - sum c_n S_n and of c[1 + j] = f0 a_j
    double cb[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) cb[j] = cb_in[j];
    q0b = cb[0];
#pragma unroll
    for (int q = 0; q < 6; ++q) cb[4 + q] += -S[q] * cb[0];
    double f0b = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        ab[j] = f0 * cb[1 + j];
        f0b += a[j] * cb[1 + j];
    }
    // contributions of c[1..3] += f_m b^m (f_m = w_m / sum - f0 gm) to f0 and to the sum
    double fsb[2], sumb = 0.0, f0bp = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        fsb[h] = bs[h][0] * cb[1] + bs[h][1] * cb[2] + bs[h][2] * cb[3];
        if (on[h]) {
            sumb += -fsb[h] * ws[h] * isum * isum;
            f0bp += -fsb[h] * gm;
        }
    }
    f0b += quad_sum(f0bp);
    sumb = quad_sum(sumb) - f0b * w0 * isum * isum / g0;
    const double w0b = f0b * isum / g0 + sumb;
    // tau_w
    double twb = 0.0, beta0b = 0.0;
    if (!lin) {
        const double dp0 = pw == 1.0 ? 1.0 : pw * wpow(x0, pw - 1.0);
        const double x0b = w0b * g0 * dp0;
        beta0b += -x0b * x0 / (beta0 + eps);
        double twp = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (on[h]) {
                const double dps = pw == 1.0 ? 1.0 : pw * wpow(xs[h], pw - 1.0);
                twp += (fsb[h] * isum + sumb) * gm * dps / (beta[h] + eps);
            }
        twb = (x0b / (beta0 + eps) + quad_sum(twp)) / M;
    }
    // this lane's sub-stencils
    double beta0bp = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (on[h]) {
            const double fs = ws[h] * isum - sub0;
            const double wsb = fsb[h] * isum + sumb;
            double betab = 0.0;
            if (!lin) {
                const double dps = pw == 1.0 ? 1.0 : pw * wpow(xs[h], pw - 1.0);
                betab += -wsb * gm * dps * xs[h] / (beta[h] + eps);
            }
            const double sg = wsgn(beta0 - beta[h]);
            beta0bp += twb * sg;
            betab += -twb * sg;
#pragma unroll
            for (int q = 0; q < 3; ++q) bsb[h][q] = fs * cb[1 + q] + 2.0 * v23 * betab * bs[h][q];
        } else {
            bsb[h][0] = bsb[h][1] = bsb[h][2] = 0.0;
        }
    }
    beta0b += quad_sum(beta0bp);
    // beta0 = v23 sum_d (a_d^2 + H_d S H_d) + v23^2 sec
    const double g1 = v23 * beta0b, g2 = v23 * v23 * beta0b;
#pragma unroll
    for (int d = 0; d < 3; ++d) ab[d] += 2.0 * g1 * a[d];
    double Hb[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) t += Sm[p][q] * H[d][q];
            Hb[d][p] = 2.0 * g1 * t;
        }
    ab[3] += 2.0 * Hb[0][0] + 8.0 * g2 * a[3];
    ab[4] += Hb[0][1] + Hb[1][0] + 2.0 * g2 * a[4];
    ab[5] += Hb[0][2] + Hb[2][0] + 2.0 * g2 * a[5];
    ab[6] += 2.0 * Hb[1][1] + 8.0 * g2 * a[6];
    ab[7] += Hb[1][2] + Hb[2][1] + 2.0 * g2 * a[7];
    ab[8] += 2.0 * Hb[2][2] + 8.0 * g2 * a[8];
}

// 16-byte windows of the per-member and per-entry arrays that one block stages: a window of
// bytes [b0, b1) is copied from its 16-byte aligned start; the at most 15 bytes read beyond b1
// lie in the array's padding or the next array of the mesh arena.  Every lane copies a whole
// number of rows (those past a window's end repeat its last row; those past the buffer go to
// its last row, which nothing reads), so the copies need no branch into which the compiler could
// sink their loads.
// The forward kernel's staging limits per block.  FP64 blocks fit four per CU in 40.96 KB of LDS,
// which holds members and sub-stencil entries in one of three splits, chosen per mesh as the one
// that stages the most of its blocks (k1_staging_class): 240 members and 552 entries (the hybrid
// lattice: 2.4% of its blocks exceed them and read global memory; the kernel measures 11% faster
// than with the FP32 limits at three blocks per CU), 288 and 300 (hexahedra and prisms) or 228 and
// 576 (pyramids).  FP32 blocks stage up to 312 members and 600 entries (31.6 KB, five per CU).
constexpr int kK1Classes = 3;
constexpr int kK1StageOf[kK1Classes] = {20 * kK1Cells, 24 * kK1Cells, 19 * kK1Cells};
constexpr int kK1SubStageOf[kK1Classes] = {46 * kK1Cells, 25 * kK1Cells, 48 * kK1Cells};
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <typename T, int CAP = 0>
struct K1Windows {
    static constexpr int kStage = sizeof(T) == 8 ? kK1StageOf[CAP] : kK1Stage;
    static constexpr int kSubStage = sizeof(T) == 8 ? kK1SubStageOf[CAP] : kK1SubStage;
    static constexpr int kP = (kStage * 9 * (int)sizeof(T) + 30) / 16;     // pseudo-inverse rows
    static constexpr int kB = (kSubStage * 3 * (int)sizeof(T) + 30) / 16;  // sub-stencil B rows
    static constexpr int kL = (kSubStage + 6) / 4;                          // sub-stencil member bytes, 4 B words
    static constexpr int kPIter = (kP + kK1Block - 1) / kK1Block;
    static constexpr int kBIter = (kB + kK1Block - 1) / kK1Block;
    static constexpr int kLIter = (kL + kK1Block - 1) / kK1Block;
    static constexpr int kEIter = (kStage + kK1Block - 1) / kK1Block;
};

// GEN: some plane of a mesh with walls has a condition other than the reflective one (a separate
// instantiation keeps the periodic and reflective-wall kernel free of the conditions' code)
template <typename T, bool GEN, int CAP>
__global__ void __launch_bounds__(kK1Block) __attribute__((amdgpu_waves_per_eu(3)))
k_reconstruct(DevMesh m, const double *__restrict__ Q, T *__restrict__ coeff, WenoParams wp, BoundarySet bcs)
{
    using W = K1Windows<T, CAP>;
    __shared__ double sq[5][W::kStage + 1];  // the last column takes the stores of lanes past the range
    __shared__ u32x4 sP[W::kP + 1];
    __shared__ u32x4 sBw[W::kB + 1];
    __shared__ unsigned sLw[W::kL + 1];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int t = blk * kK1Block + threadIdx.x;
    const int n = m.n;
    const int ic = t / kK1CellLanes;
    const int lane = t - kK1CellLanes * ic;
    const int comp = lane >> 2;
    const int l = lane & 3;
    const bool valid = ic < n;
    const int i = valid ? ic : n - 1;  // tail lanes shadow the last cell and write nothing
    const T *B = (const T *)m.ss_B;
    const int cb0 = blk * kK1Cells, cb1 = min(cb0 + kK1Cells, n);
    const int e0 = m.st_ptr[cb0], e1 = m.st_ptr[cb1];
    const int s0 = m.ss_ptr[8 * cb0], s1 = m.ss_ptr[8 * cb1];
    // uniform over the block; non-empty windows keep the clamped row indices below in range
    const bool staged = e1 > e0 && s1 > s0 && e1 - e0 <= W::kStage && s1 - s0 <= W::kSubStage;
    // the lane's own ranges and cell data, loaded before the staging so that no load after it
    // waits on them
    const int k0 = m.st_ptr[i], k1 = m.st_ptr[i + 1];
    int pr[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        pr[h][0] = m.ss_ptr[8 * i + l + 4 * h];
        pr[h][1] = m.ss_ptr[8 * i + l + 4 * h + 1];
    }
    const double *Qc = Q + (size_t)comp * n;
    const double q0 = Qc[i];
    const T S[6] = {(T)m.m2[i], (T)m.m2[n + i], (T)m.m2[2 * n + i], (T)m.m2[3 * n + i], (T)m.m2[4 * n + i],
                    (T)m.m2[5 * n + i]};
    const int Mi = m.M[i];
    const T v23i = (T)m.vol23[i];
    const T *pinv = (const T *)m.pinv;
    // byte offsets of the block's rows inside the staged windows
    const size_t pA = (sizeof(T) * 9 * (size_t)e0) & ~(size_t)15;
    const size_t bA = (sizeof(T) * 3 * (size_t)s0) & ~(size_t)15;
    const int lA = s0 & ~3;
    if (staged) {
        // one round of independent loads for the whole block: the member indices and flips, and
        // the pseudo-inverse, B and member-byte windows as 16-byte (4-byte) rows; then the
        // members' averages, which need the indices
        const int pC = (int)((sizeof(T) * 9 * (size_t)e1 - pA + 15) >> 4);
        const int bC = (int)((sizeof(T) * 3 * (size_t)s1 - bA + 15) >> 4);
        const int lC = (s1 - lA + 3) >> 2;
        const char *pinv_b = (const char *)m.pinv + pA;
        const char *B_b = (const char *)m.ss_B + bA;
        const unsigned *L_w = (const unsigned *)(m.ss_loc + lA);
        int cx[W::kEIter];
        unsigned cf[W::kEIter];
        u32x4 rp[W::kPIter], rb[W::kBIter];
        unsigned rl[W::kLIter];
#pragma unroll
        for (int r = 0; r < W::kEIter; ++r) {
            const int e = min(e0 + (int)threadIdx.x + r * kK1Block, e1 - 1);
            cx[r] = m.st_cell[e];
            cf[r] = m.st_flip[e];
        }
#pragma unroll
        for (int r = 0; r < W::kPIter; ++r) {
            const int c = min((int)threadIdx.x + r * kK1Block, pC - 1);
            rp[r] = *(const u32x4 *)(pinv_b + 16 * (size_t)c);
        }
#pragma unroll
        for (int r = 0; r < W::kBIter; ++r) {
            const int c = min((int)threadIdx.x + r * kK1Block, bC - 1);
            rb[r] = *(const u32x4 *)(B_b + 16 * (size_t)c);
        }
#pragma unroll
        for (int r = 0; r < W::kLIter; ++r) {
            const int c = min((int)threadIdx.x + r * kK1Block, lC - 1);
            rl[r] = L_w[c];
        }
        double v[W::kEIter][5];
#pragma unroll
        for (int r = 0; r < W::kEIter; ++r)
#pragma unroll
            for (int c = 0; c < 5; ++c) v[r][c] = Q[(size_t)c * n + cx[r]];
#pragma unroll
        for (int r = 0; r < W::kPIter; ++r) sP[min((int)threadIdx.x + r * kK1Block, W::kP)] = rp[r];
#pragma unroll
        for (int r = 0; r < W::kBIter; ++r) sBw[min((int)threadIdx.x + r * kK1Block, W::kB)] = rb[r];
#pragma unroll
        for (int r = 0; r < W::kLIter; ++r) sLw[min((int)threadIdx.x + r * kK1Block, W::kL)] = rl[r];
#pragma unroll
        for (int r = 0; r < W::kEIter; ++r) {
            const int e = (int)threadIdx.x + r * kK1Block;
            const int ew = e0 + e < e1 ? e : W::kStage;
            const unsigned fl = cf[r];
            if constexpr (GEN) {
                if (fl & 7u) ghost_average(bcs, fl, v[r]);  // a ghost: its planes' conditions
#pragma unroll
                for (int c = 0; c < 5; ++c) sq[c][ew] = v[r][c];
            } else {
#pragma unroll
                for (int c = 0; c < 5; ++c) sq[c][ew] = mirror_sign(fl, c) * v[r][c];
            }
        }
        __syncthreads();
    }
    // the staged rows, indexed by member and sub-stencil entry
    const T *sPinv = (const T *)((const char *)sP + (sizeof(T) * 9 * (size_t)e0 - pA));
    const T *sB = (const T *)((const char *)sBw + (sizeof(T) * 3 * (size_t)s0 - bA));
    const unsigned char *sl = (const unsigned char *)sLw + (s0 - lA);
    // a member's average from memory (blocks too large to stage)
    auto member = [&](int k) -> double {
        const unsigned fl = m.st_flip[k];
        const int x = m.st_cell[k];
        if constexpr (GEN) {
            if (!(fl & 7u)) return Qc[x];
            double v[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) v[c] = Q[(size_t)c * n + x];
            ghost_average(bcs, fl, v);
            return v[comp];
        } else {
            return mirror_sign(fl, comp) * Qc[x];
        }
    };
    // Q_k - Q_0 of stencil entry k, in FP64, then rounded to T
    auto diff = [&](int k) -> T { return (T)((staged ? sq[comp][k - e0] : member(k)) - q0); };
    T a[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = T(0);
    if (staged) {
#pragma unroll 2
        for (int k = k0 + l; k < k1; k += kK1Lanes) {
            const T d = diff(k);
            const T *row = sPinv + 9 * (k - e0);
#pragma unroll
            for (int j = 0; j < 9; ++j) a[j] += row[j] * d;
        }
    } else {
#pragma unroll 2
        for (int k = k0 + l; k < k1; k += kK1Lanes) {
            const T d = diff(k);
#pragma unroll
            for (int j = 0; j < 9; ++j) a[j] += pinv[(size_t)9 * k + j] * d;
        }
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = quad_sum(a[j]);
    // linear sub-stencil fits l and l + 4: b^s = sum B (Q_k - Q_0)
    T bs[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        bs[h][0] = bs[h][1] = bs[h][2] = T(0);
        const int p0 = pr[h][0], p1 = pr[h][1];
        if (staged) {
            for (int e = p0 - s0; e < p1 - s0; ++e) {
                const T d = diff(k0 + sl[e]);
                bs[h][0] += sB[3 * e] * d;
                bs[h][1] += sB[3 * e + 1] * d;
                bs[h][2] += sB[3 * e + 2] * d;
            }
        } else {
            for (int e = p0; e < p1; ++e) {
                const T d = diff(k0 + m.ss_loc[e]);
                bs[h][0] += B[(size_t)3 * e] * d;
                bs[h][1] += B[(size_t)3 * e + 1] * d;
                bs[h][2] += B[(size_t)3 * e + 2] * d;
            }
        }
    }
    T c[10];
    weno_combine_quad<T>(a, bs, l, Mi, v23i, S, q0, sizeof(T) == 8, wp, c);
    // lane l writes entries l, l + 4 and (lanes 0, 1) l + 8 of this component
    T v0 = c[0], v1 = c[4], v2 = c[8];
#pragma unroll
    for (int j = 1; j < 4; ++j)
        if (l == j) {
            v0 = c[j];
            v1 = c[4 + j];
        }
    if (l == 1) v2 = c[9];
    if (valid) {
        T *out = coeff + (size_t)50 * i + 10 * comp;
        out[l] = v0;
        out[4 + l] = v1;
        if (l < 2) out[8 + l] = v2;
    }
}

// ---------------------------------------------------------------------------
// K2: face flux, one lane per (face, Gauss point)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int mask)
{
    return __shfl_xor(v, mask, 64);
}

// EXT: walls or the first-order fallback can occur (a separate instantiation keeps the periodic
// kernel free of both branches).  The FP32 periodic kernels are held to 168 registers, 3 waves/SIMD
// (without spill; at their natural 173 they run 2 waves/SIMD and measure 6% slower)
template <typename T, bool PR, bool EXT, bool SM>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !EXT ? 3 : 1)))
k_flux(DevMesh m, const T *__restrict__ coeff, const double *__restrict__ Q, const double *__restrict__ dt_dev,
       T *__restrict__ ff, FluxParams<T> fp, int *status)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int f = t >> 2;
    const bool live = f < m.nf;
    const int fs = live ? f : m.nf - 1;  // tail lanes compute a valid face and write nothing
    const int nf4 = 4 * m.nf;
    const int tt = 4 * fs + (t & 3);
    const int o = m.owner[fs], nb = m.nbr[fs];
    T geo[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) geo[q] = (T)m.fgeo[(size_t)q * nf4 + tt];
    double ql0[5], qr0[5];
    if (sizeof(T) == 4 || EXT) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            ql0[c] = Q[(size_t)c * m.n + o];
            qr0[c] = nb >= 0 ? Q[(size_t)c * m.n + nb] : 0.0;
        }
    }
    const T dt = (T)dt_dev[0];
    T out[10];
    // nb < 0: a wall on box plane -1 - nb, the right state is its condition's ghost of the left one
    int nfb = 0;
    const bool ok = face_gp<T, PR, EXT, SM>(coeff + (size_t)50 * o, nb >= 0 ? coeff + (size_t)50 * nb : nullptr, ql0,
                                            qr0, geo, dt, fp, out, nfb, nb < 0 ? -1 - nb : 0);
    if (live && !ok) status[0] = 1;
    if (EXT && live && nfb) atomicAdd(status + 1, nfb);  // integer count: the same total in any order
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        out[j] += shfl_xor_t(out[j], 1);
        out[j] += shfl_xor_t(out[j], 2);
    }
    if (live) {
        const int g4 = t & 3;
        T *dst = ff + (size_t)10 * f;
#pragma unroll
        for (int j = 0; j < 10; ++j)
            if ((j & 3) == g4) dst[j] = out[j];
    }
}

// FP64, periodic, no fallback (the benchmark path).  At 1 wave/SIMD nothing hides a wave's memory
// latency, so a grid of one block per CU walks contiguous chunks of Gauss points 256 at a time and
// keeps every load of a chunk off its critical path:
// - the next chunk's neighbour coefficients and face geometry (per wave) and the coefficient rows
//   of the cells that own its faces (per block: faces are sorted by owner, so these are a window
//   of consecutive cells starting at the owner of the chunk's first face) travel from memory
//   straight into shared memory (global_load_lds, 16 B per lane and instruction, lane L of a wave
//   writing bytes [16 L, 16 L + 16) of the instruction's 1 KiB row) while the current chunk
//   computes; an owner beyond the window (win_cells <= kWinCells cells) is read from memory directly;
// - the next chunk's owner and neighbour indices are loaded one chunk ahead into registers;
// - the neighbour's side is computed first, so the owner's coefficients need no register before
//   the owner's side;
// - a chunk's results are stored at the start of the next chunk, after its wait for memory.
constexpr int kPfRows = 25;  // 16-byte rows of one cell's 50 coefficients
constexpr int kGeoRows = 5;  // rows of the 9 geometry values: q = 2k in bytes [0, 512), 2k + 1 in [512, 1024)
constexpr int kPfWaveBytes = (kPfRows + kGeoRows) * 1024;  // one wave's buffers
constexpr int kWinRows = 36;                                // owner window, 4 waves x 9 rows
constexpr int kWinCells = kWinRows * 1024 / 400;            // 92 whole cells
constexpr int kFluxLds = (kBlock / 64) * kPfWaveBytes + kWinRows * 1024;
static_assert(kFluxLds <= 160 * 1024, "one block of the chunked flux fits a CU's shared memory");
static_assert(kWinCells == 92, "the window size is part of gks_set_flux_window's contract");

template <bool PR_ANY, bool SM>
__global__ void __launch_bounds__(kBlock) k_flux_chunked(DevMesh m, const double *__restrict__ coeff,
                                                         const double *__restrict__ dt_dev, double *__restrict__ ff,
                                                         FluxParams<double> fp, int *status, int chunk, int win_cells)
{
    __shared__ __attribute__((aligned(16))) char pf[kFluxLds];
    typedef __attribute__((address_space(3))) void *lds_ptr;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int nf4 = 4 * m.nf;
    const int b0 = (int)min((int64_t)blk * chunk, (int64_t)nf4), b1 = min(b0 + chunk, nf4);
    const double dt = dt_dev[0];
    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wave-uniform
    char *cbuf = pf + wv * kPfWaveBytes;
    char *gbuf = cbuf + kPfRows * 1024;
    char *win = pf + (kBlock / 64) * kPfWaveBytes;
    const size_t coeff_last = (size_t)400 * m.n - 16;  // last 16-byte piece of the coefficients
    auto face_of = [&](int t) { return min(t >> 2, m.nf - 1); };  // tail lanes shadow the last face
    auto tt_of = [&](int t) { return 4 * face_of(t) + (t & 3); };
    // the wave's rows of the chunk starting at cbase: the lane's neighbour cell nb, and the geometry
    // (instruction lane l fetches the values of wave lanes 2 (l & 31) and 2 (l & 31) + 1: t is even,
    // so both lie in one face, also where the tail shadows the last face)
    auto prefetch = [&](int cbase, int nb) {
        const double *src = coeff + (size_t)50 * nb;
#pragma unroll
        for (int k = 0; k < kPfRows; ++k) __builtin_amdgcn_global_load_lds(src + 2 * k, (lds_ptr)(cbuf + k * 1024), 16, 0, 0);
        const int tg = tt_of(cbase + 64 * wv + 2 * (lane & 31));
#pragma unroll
        for (int k = 0; k < kGeoRows; ++k) {
            const int q = min(2 * k + (lane >> 5), 8);
            __builtin_amdgcn_global_load_lds(m.fgeo + (size_t)q * nf4 + tg, (lds_ptr)(gbuf + k * 1024), 16, 0, 0);
        }
    };
    // the wave's rows (wv, wv + 4, ...) of the owner window starting at cell w0
    auto prefetch_win = [&](int w0) {
#pragma unroll
        for (int k = 0; k < kWinRows / 4; ++k) {
            const int r = 4 * k + wv;
            const size_t off = min((size_t)400 * w0 + (size_t)(1024 * r + 16 * lane), coeff_last);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const char *>(coeff) + off, (lds_ptr)(win + r * 1024), 16, 0, 0);
        }
    };
    int own = 0, nb1 = 0, w0 = 0;  // this chunk's owner and window; the next chunk's neighbour
    if (b0 < b1) {
        const int t0 = b0 + (int)threadIdx.x;
        own = m.owner[face_of(t0)];
        w0 = m.owner[face_of(b0)];
        prefetch(b0, m.nbr[face_of(t0)]);
        prefetch_win(w0);
        nb1 = m.nbr[face_of(t0 + kBlock)];
    }
    const int g4 = (int)threadIdx.x & 3;
    bool pend = false;  // results of the previous chunk not yet stored
    double sv0 = 0.0, sv1 = 0.0, sv2 = 0.0, *sdst = ff;
    auto store_pending = [&]() {
        if (pend) {
            sdst[g4] = sv0;
            sdst[g4 + 4] = sv1;
            if (g4 < 2) sdst[g4 + 8] = sv2;
        }
    };
    for (int base = b0; base < b1; base += kBlock) {  // uniform over the block
        const int t = base + (int)threadIdx.x;
        const bool live = t < b1;
        // this wave's rows and indices have landed (vmcnt covers the shared-memory loads) ...
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        // ... and so have every wave's rows of the owner window
        __syncthreads();
        double geo[9], cr[50];
#pragma unroll
        for (int q = 0; q < 9; ++q) geo[q] = *reinterpret_cast<const double *>(gbuf + (q >> 1) * 1024 + (q & 1) * 512 + 8 * lane);
#pragma unroll
        for (int k = 0; k < kPfRows; ++k) {
            const double2 v = *reinterpret_cast<const double2 *>(cbuf + k * 1024 + 16 * lane);
            cr[2 * k] = v.x;
            cr[2 * k + 1] = v.y;
        }
        // read before the next chunk's rows overwrite them
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        store_pending();
        // the loads for the next chunk are issued unconditionally (after the last chunk they fetch
        // the last face's rows again, unused): a conditional load would make the compiler's waits
        // for this chunk's loads cover them too
        const int own_n = m.owner[face_of(t + kBlock)];
        const int w0_n = m.owner[face_of(base + kBlock)];
        const int nb2 = m.nbr[face_of(t + 2 * kBlock)];
        prefetch(base + kBlock, nb1);
        auto load_r = [&](double c[50]) {
#pragma unroll
            for (int q = 0; q < 50; ++q) c[q] = cr[q];
        };
        auto load_l = [&](double c[50]) {
            const int idx = own - w0;  // >= 0: owners do not decrease along the faces
            // (one unconditional shared-memory read and a rare overwrite from memory through a
            // volatile pointer: plain loads on both paths fold into loads through a generic pointer,
            // whose waits also cover the next window's rows)
            const char *src = win + 400 * min(idx, kWinCells - 1);
#pragma unroll
            for (int k = 0; k < kPfRows; ++k) {
                const double2 v = *reinterpret_cast<const double2 *>(src + 16 * k);
                c[2 * k] = v.x;
                c[2 * k + 1] = v.y;
            }
            if (idx >= win_cells) {
                const volatile double *g = coeff + (size_t)50 * own;
#pragma unroll
                for (int q = 0; q < 50; ++q) c[q] = g[q];
            }
            // every wave has read the window before the next chunk's rows overwrite it
            __syncthreads();
            prefetch_win(w0_n);
        };
        double out[10];
        const bool ok = face_gp_pre<double, PR_ANY, SM>(load_l, load_r, nullptr, nullptr, geo, dt, fp, out);
        if (live && !ok) status[0] = 1;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            out[j] += shfl_xor_t(out[j], 1);
            out[j] += shfl_xor_t(out[j], 2);
        }
        sv0 = g4 == 0 ? out[0] : g4 == 1 ? out[1] : g4 == 2 ? out[2] : out[3];
        sv1 = g4 == 0 ? out[4] : g4 == 1 ? out[5] : g4 == 2 ? out[6] : out[7];
        sv2 = g4 == 0 ? out[8] : out[9];
        sdst = ff + (size_t)10 * (t >> 2);
        pend = live;
        own = own_n;
        w0 = w0_n;
        nb1 = nb2;
    }
    store_pending();
    // no shared-memory load may still be in flight when the block's shared memory is released
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// ---------------------------------------------------------------------------
// K3: per-cell gather of face fluxes and stage updates
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void gather(const DevMesh &m, const T *__restrict__ ff, int i, double L[5], double D[5])
{
#pragma unroll
    for (int c = 0; c < 5; ++c) L[c] = D[c] = 0.0;
    const int p0 = m.cf_ptr[i], p1 = m.cf_ptr[i + 1];
    for (int p = p0; p < p1; ++p) {
        const int code = m.cf_idx[p];
        const double s = (code & 1) ? 1.0 : -1.0;  // owner: -F, neighbour: +F (L = -sum outward / vol)
        const T *src = ff + (size_t)10 * (code >> 1);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            L[c] += s * (double)src[c];
            D[c] += s * (double)src[5 + c];
        }
    }
    const double iv = 1.0 / m.vol[i];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        L[c] *= iv;
        D[c] *= iv;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_residual(DevMesh m, const T *__restrict__ ff, double *__restrict__ Lout,
                                                     double *__restrict__ Dout)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= m.n) return;
    double L[5], D[5];
    gather(m, ff, i, L, D);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        Lout[(size_t)c * m.n + i] = L[c];
        Dout[(size_t)c * m.n + i] = D[c];
    }
}

// stage 1: Q* = Q + dt/2 L + dt^2/8 D into Qs;  Q <- Q + dt L + dt^2/6 D (partial update)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_stage1(DevMesh m, const T *__restrict__ ff, double *__restrict__ Q,
                                                   double *__restrict__ Qs, const double *__restrict__ dt_dev)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= m.n) return;
    const double dt = dt_dev[0];
    double L[5], D[5];
    gather(m, ff, i, L, D);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const double q = Q[(size_t)c * m.n + i];
        Qs[(size_t)c * m.n + i] = q + 0.5 * dt * L[c] + 0.125 * dt * dt * D[c];
        Q[(size_t)c * m.n + i] = q + dt * L[c] + dt * dt / 6.0 * D[c];
    }
}

// stage 2: Q <- Q + dt^2/3 D(Q*)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_stage2(DevMesh m, const T *__restrict__ ff, double *__restrict__ Q,
                                                   const double *__restrict__ dt_dev)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= m.n) return;
    const double dt = dt_dev[0];
    double L[5], D[5];
    gather(m, ff, i, L, D);
#pragma unroll
    for (int c = 0; c < 5; ++c) Q[(size_t)c * m.n + i] += dt * dt / 3.0 * D[c];
}


// ---------------------------------------------------------------------------
// Implicit Jacobi step of the steady solver (Section 3.3, Eq. euler-scheme and Eq. jacobi):
// D_i dQ_i + 1/2 sum_f [T(Q_nb + dQ_nb) - T(Q_nb) - r dQ_nb] S = |Omega_i| Res_i with
// D_i = |Omega_i| / dt + 1/2 sum_f r S, T the Euler flux along the cell's outward face normal,
// r = |U_nb . n| + c_nb at t_n and Res = L + dt_f/2 dL/dt the GKS residual over the explicit step
// dt_f (dt = factor x dt_f); every gather runs over the cell's faces in F_p order.  Across a face
// on a box plane the neighbour is the ghost of Section 2's construction, the plane's condition on
// the cell's own state, B(Q_i), and its increment B(Q_i + dQ_i) - B(Q_i) with the cell's previous
// iterate.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double euler_flux_n(const double q[5], double nx, double ny, double nz, double gam,
                                               double T[5])
{
    const double ir = 1.0 / q[0];
    const double u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
    const double un = u * nx + v * ny + w * nz;
    const double p = (gam - 1.0) * (q[4] - 0.5 * (q[1] * u + q[2] * v + q[3] * w));
    T[0] = q[0] * un;
    T[1] = q[1] * un + p * nx;
    T[2] = q[2] * un + p * ny;
    T[3] = q[3] * un + p * nz;
    T[4] = (q[4] + p) * un;
    return fabs(un) + sqrt(gam * p * ir);  // spectral radius of the normal flux Jacobian
}

// the neighbour across a cell's face (code = 2 face + side) and the cell's outward unit normal; a
// wall face gives -1 - its box plane
__device__ __forceinline__ int face_side(const DevMesh &m, int code, double &nx, double &ny, double &nz, double &S)
{
    const int f = code >> 1;
    const double sg = (code & 1) ? -1.0 : 1.0;  // side 0: the owner, normal owner -> neighbour
    nx = sg * m.fnS[f];
    ny = sg * m.fnS[m.nf + f];
    nz = sg * m.fnS[2 * m.nf + f];
    S = m.fnS[3 * m.nf + f];
    return (code & 1) ? m.owner[f] : m.nbr[f];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_implicit_init(DevMesh m, const T *__restrict__ ff, const double *__restrict__ Q,
                                                          const double *__restrict__ dt_dev, double factor, double gam,
                                                          double *__restrict__ b, double *__restrict__ diag,
                                                          double *__restrict__ dq, BoundarySet bcs)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= m.n) return;
    const int n = m.n;
    double L[5], D[5];
    gather(m, ff, i, L, D);
    const double dtf = dt_dev[0], vol = m.vol[i];
    double sumr = 0.0;
    for (int p = m.cf_ptr[i]; p < m.cf_ptr[i + 1]; ++p) {
        double nx, ny, nz, S, q[5], Tn[5];
        const int nb = face_side(m, m.cf_idx[p], nx, ny, nz, S);
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = Q[(size_t)c * n + (nb >= 0 ? nb : i)];
        if (nb < 0) bc_average(bcs, -1 - nb, q);  // the ghost
        sumr += euler_flux_n(q, nx, ny, nz, gam, Tn) * S;
    }
    const double d = vol / (factor * dtf) + 0.5 * sumr;
    diag[i] = d;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const double bc = vol * (L[c] + 0.5 * dtf * D[c]);
        b[(size_t)c * n + i] = bc;
        dq[(size_t)c * n + i] = bc / d;
    }
}

__global__ void __launch_bounds__(kBlock) k_implicit_sweep(DevMesh m, const double *__restrict__ Q, double gam,
                                                           const double *__restrict__ b, const double *__restrict__ diag,
                                                           const double *__restrict__ dq_in, double *__restrict__ dq_out,
                                                           BoundarySet bcs)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= m.n) return;
    const int n = m.n;
    double off[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int p = m.cf_ptr[i]; p < m.cf_ptr[i + 1]; ++p) {
        double nx, ny, nz, S, q[5], d[5], q1[5], T0[5], T1[5];
        const int nb = face_side(m, m.cf_idx[p], nx, ny, nz, S);
        const int x = nb >= 0 ? nb : i;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            q[c] = Q[(size_t)c * n + x];
            d[c] = dq_in[(size_t)c * n + x];
            q1[c] = q[c] + d[c];
        }
        if (nb < 0) {  // the ghost and its increment: the condition on the cell's state and updated state
            bc_average(bcs, -1 - nb, q);
            bc_average(bcs, -1 - nb, q1);
#pragma unroll
            for (int c = 0; c < 5; ++c) d[c] = q1[c] - q[c];
        }
        const double r = euler_flux_n(q, nx, ny, nz, gam, T0);
        euler_flux_n(q1, nx, ny, nz, gam, T1);
#pragma unroll
        for (int c = 0; c < 5; ++c) off[c] += (T1[c] - T0[c] - r * d[c]) * S;
    }
    const double di = diag[i];
#pragma unroll
    for (int c = 0; c < 5; ++c) dq_out[(size_t)c * n + i] = (b[(size_t)c * n + i] - 0.5 * off[c]) / di;
}

__global__ void __launch_bounds__(kBlock) k_implicit_update(int len, double *__restrict__ Q, const double *__restrict__ dq)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < len) Q[t] += dq[t];
}

// ===========================================================================
// Discrete adjoint of one S2O4 step (FP64)
// ===========================================================================
//
// The step is Q* = Q + dt/2 L(Q) + dt^2/8 D(Q),
//             Q' = Q + dt L(Q) + dt^2/6 (D(Q) + 2 D(Q*)), dt frozen.
// Given lam' = dJ/dQ', the step's reverse is
//   lam* = dt^2/3 J_D(Q*)^T lam',
//   lam  = lam' + lam* + J_L(Q)^T (dt lam' + dt/2 lam*) + J_D(Q)^T (dt^2/6 lam' + dt^2/8 lam*).
// Each J^T product is one vector-Jacobian product of the operator Q -> (L, D):
// face-flux cotangents from the cell cotangents (reverse of Eq. finite), the
// reverse of every Gauss-point flux (recomputed in registers), a per-cell
// gather of the coefficient cotangents, the reverse of the reconstruction
// per (cell, component), and a gather over the transposed stencil.  All
// gathers run in a fixed order: no atomics, bitwise reproducible.

constexpr int kAccB = 47;  // accumulator cotangents per Gauss point (slots of AccSlot, Prandtl slots included)

struct AdjWork {
    double *abuf;   // [47][4F]   accumulator cotangents per Gauss point (slot-major)
    double *cbf;    // [F][2][50] coefficient cotangents per face side
    double *cbc;    // [N][50]    per cell
    double *dbar;   // [nnz][5]   cotangents of the stencil differences Q_k - Q_0 (entry-major: a
                    //            cell's 5 gathering lanes read one 40-byte record per entry)
    double *own;    // [5][N]     direct cotangent of each cell's own average
    double *lstar;  // [5][N]     lam*
    double *vjp;    // [5][N]     result of the latest vector-Jacobian product
    double *coeff;  // [N][50]    recomputed reconstruction
};

static size_t adj_layout(int64_t n, int64_t nf, int64_t nnz, AdjWork *w, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return base ? (double *)(base + o) : nullptr;
    };
    double *ab = take(8 * kAccB * 4 * nf);
    double *cbf = take(8 * 100 * nf), *cbc = take(8 * 50 * n), *dbar = take(8 * 5 * nnz), *own = take(8 * 5 * n),
           *ls = take(8 * 5 * n), *vj = take(8 * 5 * n), *co = take(8 * 50 * n);
    if (w) *w = AdjWork{ab, cbf, cbc, dbar, own, ls, vj, co};
    return off;
}

// reverse of the flux, part 1 (lane per face Gauss point): both half-space passes forward,
// then the reverse of the interface equilibrium, its slopes, the collision time, the time
// integrals and the rotation/weighting, down to the half-space accumulators.  The kernel runs
// 1 wave/SIMD, so it walks chunks of Gauss points the way k_flux_chunked does (one block per CU,
// the same shared-memory rows: the next chunk's neighbour coefficients and geometry per wave, an
// owner window per block, all by global_load_lds while the current chunk computes, and the
// neighbour's side first, as there).  A chunk's cell cotangents and volumes are requested after
// the neighbour's side pass and used after the owner's.
template <bool PR>
__global__ void __launch_bounds__(kBlock) k_flux_adj_a(DevMesh m, const double *__restrict__ coeff,
                                                       const double *__restrict__ dt_dev, const double *__restrict__ lp,
                                                       const double *__restrict__ ls, double cL1, double cL2, double cD1,
                                                       double cD2, FluxParams<double> fp, double *__restrict__ abuf,
                                                       int chunk, int win_cells)
{
    __shared__ __attribute__((aligned(16))) char pf[kFluxLds];
    typedef __attribute__((address_space(3))) void *lds_ptr;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int nf4 = 4 * m.nf;
    const int n = m.n;
    const int b0 = (int)min((int64_t)blk * chunk, (int64_t)nf4), b1 = min(b0 + chunk, nf4);
    const double dt = dt_dev[0];
    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wave-uniform
    char *cbuf = pf + wv * kPfWaveBytes;
    char *gbuf = cbuf + kPfRows * 1024;
    char *win = pf + (kBlock / 64) * kPfWaveBytes;
    const size_t coeff_last = (size_t)400 * n - 16;  // last 16-byte piece of the coefficients
    auto face_of = [&](int t) { return min(t >> 2, m.nf - 1); };  // tail lanes shadow the last face
    auto tt_of = [&](int t) { return 4 * face_of(t) + (t & 3); };
    // the same row layout as k_flux_chunked's
    auto prefetch = [&](int cbase, int nb) {
        const double *src = coeff + (size_t)50 * nb;
#pragma unroll
        for (int k = 0; k < kPfRows; ++k) __builtin_amdgcn_global_load_lds(src + 2 * k, (lds_ptr)(cbuf + k * 1024), 16, 0, 0);
        const int tg = tt_of(cbase + 64 * wv + 2 * (lane & 31));
#pragma unroll
        for (int k = 0; k < kGeoRows; ++k) {
            const int q = min(2 * k + (lane >> 5), 8);
            __builtin_amdgcn_global_load_lds(m.fgeo + (size_t)q * nf4 + tg, (lds_ptr)(gbuf + k * 1024), 16, 0, 0);
        }
    };
    auto prefetch_win = [&](int w0) {
#pragma unroll
        for (int k = 0; k < kWinRows / 4; ++k) {
            const int r = 4 * k + wv;
            const size_t off = min((size_t)400 * w0 + (size_t)(1024 * r + 16 * lane), coeff_last);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const char *>(coeff) + off, (lds_ptr)(win + r * 1024), 16, 0, 0);
        }
    };
    int own = 0, nbc = 0, nb1 = 0, w0 = 0;  // this chunk's owner, neighbour and window; the next chunk's neighbour
    if (b0 < b1) {
        const int t0 = b0 + (int)threadIdx.x;
        own = m.owner[face_of(t0)];
        nbc = m.nbr[face_of(t0)];
        w0 = m.owner[face_of(b0)];
        prefetch(b0, nbc);
        prefetch_win(w0);
        nb1 = m.nbr[face_of(t0 + kBlock)];
    }
    const double *ls_or_lp = ls ? ls : lp;  // the second set read from lp again when there is none, unused then
    for (int base = b0; base < b1; base += kBlock) {  // uniform over the block
        const int t = base + (int)threadIdx.x;
        // tail lanes (t >= b1, only in the last chunk of the grid) compute the Gauss point they
        // shadow, bit for bit as its own lane does, and store the same values to its slots: a
        // conditional store would keep the whole reverse pass's registers live across branches
        const int tt = tt_of(t);
        // the parameters pass through an empty asm each chunk, so that values derived from them are
        // formed where they are used instead of being held in registers across the loop
        FluxParams<double> fpl = fp;
        double dtl = dt;
        asm volatile("" : "+s"(fpl.gamma), "+s"(fpl.K), "+s"(fpl.mu), "+s"(fpl.Pr), "+s"(fpl.tau_eps), "+s"(fpl.tau_C),
                     "+s"(dtl));
        // this wave's rows and indices have landed (vmcnt covers the shared-memory loads) ...
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        // ... and so have every wave's rows of the owner window
        __syncthreads();
        double geo[9], cr[50];
#pragma unroll
        for (int q = 0; q < 9; ++q) geo[q] = *reinterpret_cast<const double *>(gbuf + (q >> 1) * 1024 + (q & 1) * 512 + 8 * lane);
#pragma unroll
        for (int k = 0; k < kPfRows; ++k) {
            const double2 v = *reinterpret_cast<const double2 *>(cbuf + k * 1024 + 16 * lane);
            cr[2 * k] = v.x;
            cr[2 * k + 1] = v.y;
        }
        // read before the next chunk's rows overwrite them
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        const int own_n = m.owner[face_of(t + kBlock)];
        const int w0_n = m.owner[face_of(base + kBlock)];
        const int nb2 = m.nbr[face_of(t + 2 * kBlock)];
        // issued unconditionally (after the last chunk they fetch the last face's rows again, unused),
        // as in k_flux_chunked
        prefetch(base + kBlock, nb1);
        double n3[3][3];
        const double area = local_frame(geo[6], geo[7], geo[8], n3);
        FluxAcc<double, PR> A;
        acc_zero(A);
        {
            double q[5], dq[3][5];
            side_state(cr, nullptr, geo[3], geo[4], geo[5], n3, q, dq);
            side_pass<double, PR>(q, dq, -1.0, fpl, A, 1);
        }
        // the chunk's cell cotangents and volumes, used after the owner's side pass
        double po[5], pn[5], so[5], sn[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            po[c] = lp[(size_t)c * n + own];
            pn[c] = lp[(size_t)c * n + nbc];
            so[c] = ls_or_lp[(size_t)c * n + own];
            sn[c] = ls_or_lp[(size_t)c * n + nbc];
        }
        const double vo = m.vol[own], vnb = m.vol[nbc];
        {
            double q[5], dq[3][5], cl[50];
            const int idx = own - w0;  // >= 0: owners do not decrease along the faces
            // (as in k_flux_chunked: one unconditional shared-memory read, a rare overwrite from memory)
            const char *src = win + 400 * min(idx, kWinCells - 1);
#pragma unroll
            for (int k = 0; k < kPfRows; ++k) {
                const double2 v = *reinterpret_cast<const double2 *>(src + 16 * k);
                cl[2 * k] = v.x;
                cl[2 * k + 1] = v.y;
            }
            if (idx >= win_cells) {
                const volatile double *g = coeff + (size_t)50 * own;
#pragma unroll
                for (int q = 0; q < 50; ++q) cl[q] = g[q];
            }
            // every wave has read the window before the next chunk's rows overwrite it
            __syncthreads();
            prefetch_win(w0_n);
            side_state(cl, nullptr, geo[0], geo[1], geo[2], n3, q, dq);
            side_pass<double, PR>(q, dq, 1.0, fpl, A, 0);
        }
        const double io = 1.0 / vo, inb = 1.0 / vnb;
        double outb[10];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            double Lo = cL1 * po[c], Ln = cL1 * pn[c];
            double Do = cD1 * po[c], Dn = cD1 * pn[c];
            if (ls) {
                Lo += cL2 * so[c];
                Ln += cL2 * sn[c];
                Do += cD2 * so[c];
                Dn += cD2 * sn[c];
            }
            outb[c] = dtl * (-Lo * io + Ln * inb);
            outb[5 + c] = dtl * dtl * (-Do * io + Dn * inb);
        }
        // rotation back and weighting: out = area R^T F
        double Fb[10];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Fb[5 * s] = area * outb[5 * s];
            Fb[5 * s + 4] = area * outb[5 * s + 4];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                Fb[5 * s + 1 + k] =
                    area * (outb[5 * s + 1] * n3[k][0] + outb[5 * s + 2] * n3[k][1] + outb[5 * s + 3] * n3[k][2]);
        }
        finish_flux_b<double, PR>(A, dtl, fpl, Fb, [&](int slot, double v) {
            abuf[(size_t)slot * nf4 + tt] = v;
        });
        own = own_n;
        nbc = nb1;
        w0 = w0_n;
        nb1 = nb2;
    }
    // no shared-memory load may still be in flight when the block's shared memory is released
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// reverse of the flux, part 2 (lane per face Gauss point and side): the reverse of that
// side's half-space pass and of its state evaluation; the four Gauss points of a side
// (a quad of lanes) are summed in a fixed order.  The reverse pass reads the accumulator
// cotangents one at a time deep inside its arithmetic, where a wave alone on its SIMD would
// wait for each; so the wave's 8 faces x 4 Gauss points of every slot (32 consecutive values
// per slot) travel from memory into shared memory at the start (global_load_lds, 16 B per lane
// and instruction: instruction lane l fetches 2 values of slot 4 r + (l >> 4) in row r) and
// arrive while the side's state and forward pass are computed.
constexpr int kAdjRows = (kAccB + 3) / 4;  // 1 KiB rows of 4 slots x 32 values

template <bool PR>
__global__ void __launch_bounds__(kBlock) k_flux_adj_b(DevMesh m, const double *__restrict__ coeff,
                                                       FluxParams<double> fp, const double *__restrict__ abuf,
                                                       double *__restrict__ cbf)
{
    __shared__ __attribute__((aligned(16))) double sab[(kBlock / 64) * kAdjRows * 128];
    typedef __attribute__((address_space(3))) void *lds_ptr;
    const int t = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int f0 = __builtin_amdgcn_readfirstlane(t >> 3) & ~7;  // the wave's first face (wave-uniform)
    if (f0 >= m.nf) return;                                       // the whole wave is past the last face
    const int f = t >> 3;
    const bool live = f < m.nf;
    const int fs = live ? f : m.nf - 1;
    const int side = (t >> 2) & 1;
    const int g = t & 3;
    const int nf4 = 4 * m.nf;
    const size_t tg = (size_t)4 * fs + g;
    const int lane = (int)threadIdx.x & 63;
    double *wab = sab + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) * (kAdjRows * 128);
    // the cell index first: its wait then need not cover the slots
    const int cell = side ? m.nbr[fs] : m.owner[fs];
    {
        const int e = min(4 * f0 + 2 * (lane & 15), nf4 - 2);  // past the last face: shadows, unused
#pragma unroll
        for (int r = 0; r < kAdjRows; ++r) {
            const int slot = min(4 * r + (lane >> 4), kAccB - 1);
            __builtin_amdgcn_global_load_lds(abuf + (size_t)slot * nf4 + e, (lds_ptr)(wab + 128 * r), 16, 0, 0);
        }
    }
    const int col = (int)tg - 4 * f0;  // in [0, 32): the lane's value within a slot's 32
    double geo[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) geo[q] = m.fgeo[(size_t)q * nf4 + tg];
    double n3[3][3];
    local_frame(geo[6], geo[7], geo[8], n3);
    const double X = side ? geo[3] : geo[0], Y = side ? geo[4] : geo[1], Z = side ? geo[5] : geo[2];
    double c[50];
    load_cell(coeff + (size_t)50 * cell, c);
    double q[5], dq[3][5];
    side_state(c, nullptr, X, Y, Z, n3, q, dq);
    double qb[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, dqb[3][5];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
        for (int j = 0; j < 5; ++j) dqb[mm][j] = 0.0;
    // the slots have landed (vmcnt covers the shared-memory loads)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    side_pass_b<double, PR>(q, dq, side ? -1.0 : 1.0, fp, [&](int slot) { return wab[32 * slot + col]; }, side, qb,
                            dqb);
    double cb[50];
#pragma unroll
    for (int j = 0; j < 50; ++j) cb[j] = 0.0;
    side_state_b(X, Y, Z, n3, qb, dqb, cb);
    // the quad's sums, each lane keeping the ones it stores (j = 4 r + g): an exchange with lane
    // g ^ 1 keeps the values of j's parity, one with lane g ^ 2 those of j mod 4.  Every sum is
    // (v0 + v1) + (v2 + v3) up to the order of the two operands of an addition: bitwise the same on
    // whichever lane forms it, and the same as a full quad sum.
    const bool odd = (g & 1) != 0, hi = (g & 2) != 0;
    double h[25], k[13];
#pragma unroll
    for (int i = 0; i < 25; ++i) {
        const double send = odd ? cb[2 * i] : cb[2 * i + 1];
        h[i] = (odd ? cb[2 * i + 1] : cb[2 * i]) + dpp_f64<kDppQuadXor1>(send);
    }
#pragma unroll
    for (int r = 0; r < 12; ++r) {
        const double send = hi ? h[2 * r] : h[2 * r + 1];
        k[r] = (hi ? h[2 * r + 1] : h[2 * r]) + dpp_f64<kDppQuadXor2>(send);
    }
    k[12] = h[24] + dpp_f64<kDppQuadXor2>(h[24]);  // j = 48 + g, stored by g < 2
    if (live) {
        double *dst = cbf + (size_t)100 * f + 50 * side;
#pragma unroll
        for (int r = 0; r < 12; ++r) dst[4 * r + g] = k[r];
        if (g < 2) dst[48 + g] = k[12];
    }
}

// per cell: sum of its face sides' coefficient cotangents, F_p order; a lane per cell and pair of
// coefficients (16-byte loads and stores: face-side records and cell rows are 400 bytes)
__global__ void __launch_bounds__(kBlock) k_cbar_gather(DevMesh m, const double *__restrict__ cbf, double *__restrict__ cbc)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int i = t / 25, j = 2 * (t - 25 * (t / 25));
    if (i >= m.n) return;
    double sx = 0.0, sy = 0.0;
    for (int p = m.cf_ptr[i]; p < m.cf_ptr[i + 1]; ++p) {
        const int code = m.cf_idx[p];
        const double2 v = *reinterpret_cast<const double2 *>(cbf + (size_t)100 * (code >> 1) + 50 * (code & 1) + j);
        sx += v.x;
        sy += v.y;
    }
    *reinterpret_cast<double2 *>(cbc + (size_t)50 * i + j) = make_double2(sx, sy);
}

// reverse of the reconstruction: quad of lanes per (cell, component)
__global__ void __launch_bounds__(kK1Block) __attribute__((amdgpu_waves_per_eu(3))) k_reconstruct_adj(DevMesh m, const double *__restrict__ Q,
                                                              const double *__restrict__ cbc, WenoParams wp,
                                                              double *__restrict__ dbar, double *__restrict__ own)
{
    // forward recomputation exactly as in k_reconstruct (FP64): staged gathers and lists
    __shared__ double sq[5][kK1Stage];
    __shared__ double sB[3][kK1SubStage];
    __shared__ unsigned char sl[kK1SubStage];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int t = blk * kK1Block + threadIdx.x;
    const int n = m.n;
    const int ic = t / kK1CellLanes;
    const int lane = t - kK1CellLanes * ic;
    const int comp = lane >> 2;
    const int l = lane & 3;
    const bool valid = ic < n;
    const int i = valid ? ic : n - 1;
    const double *B = (const double *)m.ss_B;
    const int cb0 = blk * kK1Cells, cb1 = min(cb0 + kK1Cells, n);
    const int e0 = m.st_ptr[cb0], e1 = m.st_ptr[cb1];
    const int s0 = m.ss_ptr[8 * cb0], s1 = m.ss_ptr[8 * cb1];
    const bool staged = e1 - e0 <= kK1Stage && s1 - s0 <= kK1SubStage;  // uniform over the block
    // the lane's own ranges, loaded before the staging so that no load after it waits on them
    const int k0 = m.st_ptr[i], k1 = m.st_ptr[i + 1];
    int pr[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        pr[h][0] = m.ss_ptr[8 * i + l + 4 * h];
        pr[h][1] = m.ss_ptr[8 * i + l + 4 * h + 1];
    }
    if (staged) {
        for (int e = e0 + (int)threadIdx.x; e < e1; e += kK1Block) {
            const int x = m.st_cell[e];
            const unsigned fl = m.st_flip[e];
#pragma unroll
            for (int c = 0; c < 5; ++c) sq[c][e - e0] = mirror_sign(fl, c) * Q[(size_t)c * n + x];
        }
        for (int e = s0 + (int)threadIdx.x; e < s1; e += kK1Block) {
            sl[e - s0] = m.ss_loc[e];
#pragma unroll
            for (int j = 0; j < 3; ++j) sB[j][e - s0] = B[(size_t)3 * e + j];
        }
        __syncthreads();
    }
    const double *pinv = (const double *)m.pinv;
    const double *dsc = (const double *)m.dsc;
    const double *Qc = Q + (size_t)comp * n;
    const double q0 = Qc[i];
    auto diff = [&](int k) -> double {
        return (staged ? sq[comp][k - e0] : mirror_sign(m.st_flip[k], comp) * Qc[m.st_cell[k]]) - q0;
    };
    double a[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = 0.0;
#pragma unroll 2
    for (int k = k0 + l; k < k1; k += kK1Lanes) {
        const double d = diff(k);
#pragma unroll
        for (int j = 0; j < 9; ++j) a[j] += pinv[(size_t)9 * k + j] * d;
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = quad_sum(a[j]);
    double bs[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        bs[h][0] = bs[h][1] = bs[h][2] = 0.0;
        const int p0 = pr[h][0], p1 = pr[h][1];
        if (staged) {
            for (int e = p0 - s0; e < p1 - s0; ++e) {
                const double d = diff(k0 + sl[e]);
                bs[h][0] += sB[0][e] * d;
                bs[h][1] += sB[1][e] * d;
                bs[h][2] += sB[2][e] * d;
            }
        } else {
            for (int e = p0; e < p1; ++e) {
                const double d = diff(k0 + m.ss_loc[e]);
                bs[h][0] += B[(size_t)3 * e] * d;
                bs[h][1] += B[(size_t)3 * e + 1] * d;
                bs[h][2] += B[(size_t)3 * e + 2] * d;
            }
        }
    }
    const double S[6] = {m.m2[i], m.m2[n + i], m.m2[2 * n + i], m.m2[3 * n + i], m.m2[4 * n + i], m.m2[5 * n + i]};
    double cb[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) cb[j] = cbc[(size_t)50 * i + 10 * comp + j];
    double ab[9], bsb[2][3], q0b;
    weno_combine_quad_b(a, bs, l, m.M[i], m.vol23[i], S, wp, cb, ab, bsb, q0b);
    // b^s = sum_k (G_s^-1 D_k / h) d_k, so d_k receives D_k . r_s with r_s = (G_s^-1 / h) bsb_s for
    // every sub-stencil s that holds member k; lane l forms r for its sub-stencils l, l + 4, and the
    // quad shares all eight
    const double *gip = (const double *)m.ginv;
    double rown[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double g[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) g[q] = gip[(size_t)(6 * (l + 4 * h) + q) * n + i];
        sym3_apply(g, bsb[h], rown[h]);
    }
    double rb[8][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        rb[0][q] = quad_bcast<0>(rown[0][q]);
        rb[1][q] = quad_bcast<1>(rown[0][q]);
        rb[2][q] = quad_bcast<2>(rown[0][q]);
        rb[3][q] = quad_bcast<3>(rown[0][q]);
        rb[4][q] = quad_bcast<0>(rown[1][q]);
        rb[5][q] = quad_bcast<1>(rown[1][q]);
        rb[6][q] = quad_bcast<2>(rown[1][q]);
        rb[7][q] = quad_bcast<3>(rown[1][q]);
    }
    // members: dbar_k = sum_j A+[k][j] ab_j + D_k . sum_{s in mask} r_s
    double sumk = 0.0;
    for (int k = k0 + l; k < k1; k += kK1Lanes) {
        const unsigned mask = (unsigned)m.st_rec[k].y;
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) v += pinv[(size_t)9 * k + j] * ab[j];
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (mask & (1u << s)) {
                sx += rb[s][0];
                sy += rb[s][1];
                sz += rb[s][2];
            }
        v += dsc[(size_t)3 * k] * sx + dsc[(size_t)3 * k + 1] * sy + dsc[(size_t)3 * k + 2] * sz;
        if (valid) dbar[(size_t)5 * k + comp] = v;
        sumk += v;
    }
    sumk = quad_sum(sumk);
    if (valid && l == 0) own[(size_t)comp * n + i] = q0b - sumk;
}

// per cell: own cotangent plus every stencil entry that names the cell; out = scale * that (+ add)
__global__ void __launch_bounds__(kBlock) k_transpose_gather(DevMesh m, const double *__restrict__ dbar,
                                                             const double *__restrict__ own, double *__restrict__ out)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int i = t / 5, c = t - 5 * (t / 5);
    if (i >= m.n) return;
    double s = own[(size_t)c * m.n + i];
    for (int p = m.tr_ptr[i]; p < m.tr_ptr[i + 1]; ++p) s += dbar[(size_t)5 * m.tr_idx[p] + c];
    out[(size_t)c * m.n + i] = s;
}

// lam = lam' + lam* + vjp
__global__ void __launch_bounds__(kBlock) k_adj_combine(int len, const double *__restrict__ lp,
                                                        const double *__restrict__ ls, const double *__restrict__ v,
                                                        double *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < len) out[i] = lp[i] + ls[i] + v[i];
}

// kinetic energy J = sum_i |Omega_i| |m_i|^2 / (2 rho_i): per-block partial sums, then one block
__global__ void __launch_bounds__(kBlock) k_ke_partial(int n, const double *__restrict__ Q, const double *__restrict__ vol,
                                                       double *__restrict__ part, double *__restrict__ grad)
{
    __shared__ double red[kBlock];
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double r = Q[i], mx = Q[n + i], my = Q[2 * n + i], mz = Q[3 * n + i];
        const double ir = 1.0 / r, m2 = mx * mx + my * my + mz * mz;
        acc += 0.5 * vol[i] * m2 * ir;
        if (grad) {
            grad[i] = -0.5 * vol[i] * m2 * ir * ir;
            grad[n + i] = vol[i] * mx * ir;
            grad[2 * n + i] = vol[i] * my * ir;
            grad[3 * n + i] = vol[i] * mz * ir;
            grad[4 * n + i] = 0.0;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBlock) k_sum_final(int nb, const double *__restrict__ part, double *out)
{
    __shared__ double red[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// batch of single Gauss-point fluxes (kernel-level tests)
template <typename T, bool PR>
__global__ void __launch_bounds__(kBlock) k_gp_batch(int64_t n, const double *__restrict__ ql, const double *__restrict__ dql,
                                                     const double *__restrict__ qr, const double *__restrict__ dqr,
                                                     const double *__restrict__ dt, double *__restrict__ out,
                                                     FluxParams<T> fp)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    T a[5], b[5], da[3][5], db[3][5], F[10];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        a[j] = (T)ql[5 * i + j];
        b[j] = (T)qr[5 * i + j];
    }
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            da[mm][j] = (T)dql[15 * i + 5 * mm + j];
            db[mm][j] = (T)dqr[15 * i + 5 * mm + j];
        }
    if (fp.smooth)
        gp_flux<T, PR, true>(a, da, b, db, (T)dt[i], fp, F);
    else
        gp_flux<T, PR>(a, da, b, db, (T)dt[i], fp, F);
#pragma unroll
    for (int j = 0; j < 10; ++j) out[10 * i + j] = (double)F[j];
}

template <typename T>
static FluxParams<T> flux_params(const gks_params *p)
{
    FluxParams<T> f;
    f.gamma = (T)p->gamma;
    f.K = (T)((5.0 - 3.0 * p->gamma) / (p->gamma - 1.0));
    f.mu = (T)p->mu;
    f.Pr = (T)p->Pr;
    f.tau_eps = (T)p->tau_eps;
    f.tau_C = (T)p->tau_C;
    f.viscous = p->viscous;
    f.fallback = p->first_order_fallback;
    f.floor = p->fallback_floor;
    f.smooth = p->smooth_flux;
    f.mu_power = (T)p->mu_power;
    f.iT_ref = p->mu_power != 0.0 ? (T)(1.0 / p->T_ref) : T(1);
    for (int b = 0; b < 6; ++b) {
        f.bc_type[b] = p->bc[b].type;
        f.bc_Tw[b] = (T)p->bc[b].Tw;
        for (int q = 0; q < 3; ++q) f.bc_uw[b][q] = (T)p->bc[b].uw[q];
        for (int q = 0; q < 5; ++q) f.bc_far[b][q] = (T)p->bc[b].far[q];
    }
    return f;
}

static BoundarySet boundary_set(const gks_params *p)
{
    BoundarySet b;
    b.gamma = p->gamma;
    b.any_general = 0;
    for (int k = 0; k < 6; ++k) {
        b.type[k] = p->bc[k].type;
        b.Tw[k] = p->bc[k].Tw;
        for (int q = 0; q < 3; ++q) b.uw[k][q] = p->bc[k].uw[q];
        for (int q = 0; q < 5; ++q) b.far[k][q] = p->bc[k].far[q];
        if (b.type[k] != kBcSlip) b.any_general = 1;
    }
    return b;
}

}  // namespace gks

// ===========================================================================
// C ABI
// ===========================================================================
using namespace gks;

struct gks_mesh {
    DevMesh d;
    int64_t n, nf;
    int precision;
    int n_cu = 256;  // compute units of the device the mesh lives on (grid of the chunked flux kernel)
    int dev = 0;     // the device the mesh lives on
    int flux_win = kWinCells;  // owner window of the chunked flux kernel (narrowed by tests only)
    int k1_class = 0;          // staging split of the FP64 reconstruction (k1_staging_class)
    // optional per-kernel HIP-event timing (gks_profile)
    bool prof = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> rec;  // kernel id, index of its start event
};

namespace {
// records a start event before and a stop event after one launch when profiling is on
struct ProfScope {
    gks_mesh *m;
    hipStream_t st;
    size_t idx = (size_t)-1;
    ProfScope(gks_mesh *m_, int id, hipStream_t s) : m(m_), st(s)
    {
        if (!m->prof) return;
        while (m->pool.size() < m->used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            m->pool.push_back(e);
        }
        idx = m->used;
        m->used += 2;
        m->rec.push_back({id, idx});
        (void)hipEventRecord(m->pool[idx], st);
    }
    ~ProfScope()
    {
        if (idx != (size_t)-1) (void)hipEventRecord(m->pool[idx + 1], st);
    }
};
}  // namespace

static hipStream_t S(gks_stream_t s) { return (hipStream_t)s; }

static unsigned grid_for(int64_t threads, int block) { return (unsigned)((threads + block - 1) / block); }

extern "C" {

void gks_default_params(gks_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->gamma = 1.4;
    p->cfl = 0.5;
    p->mu = 0.0;
    p->Pr = 1.0;
    p->weno_eps = 1e-6;
    p->weno_gamma_m = 0.0125;
    p->weno_p = 1.0;
    p->tau_eps = 0.01;
    p->tau_C = 1.0;
    p->mu_power = 0.0;
    p->T_ref = 1.0;
}

const char *gks_last_error(void) { return g_err.c_str(); }

gks_status gks_preprocess(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types,
                          const int64_t *cells, const double *box, int periodic, int min_big_stencil,
                          gks_host_mesh **out)
{
    if (!out) return fail(GKS_EINVAL, "null output");
    if (min_big_stencil < 0 || min_big_stencil > 64) return fail(GKS_EINVAL, "min_big_stencil out of range 0..64");
    *out = nullptr;
    gks_host_mesh *h = new (std::nothrow) gks_host_mesh;
    if (!h) return fail(GKS_EINVAL, "out of host memory");
    gks_status s;
    try {
        s = preprocess(n_nodes, nodes, n_cells, types, cells, box, periodic, min_big_stencil, h->h);
    } catch (const std::exception &e) {
        s = fail(GKS_EINVAL, std::string("preprocessing failed: ") + e.what());
    }
    if (s != GKS_OK) {
        delete h;
        return s;
    }
    *out = h;
    return GKS_OK;
}

void gks_host_mesh_free(gks_host_mesh *h) { delete h; }

gks_status gks_host_mesh_counts(const gks_host_mesh *h, int64_t *n_cells, int64_t *n_faces, int64_t *n_stencil,
                                int64_t *n_subcoef, int64_t *n_grown)
{
    if (!h) return fail(GKS_EINVAL, "null mesh");
    if (n_cells) *n_cells = h->h.n;
    if (n_faces) *n_faces = h->h.nf;
    if (n_stencil) *n_stencil = (int64_t)h->h.st_idx.size();
    if (n_subcoef) {
        int64_t nss = 0;
        for (uint8_t mk : h->h.st_mask) nss += __builtin_popcount((unsigned)mk);
        *n_subcoef = nss;
    }
    if (n_grown) *n_grown = h->h.n_grown;
    return GKS_OK;
}

gks_status gks_host_mesh_perm(const gks_host_mesh *h, int64_t *perm)
{
    if (!h || !perm) return fail(GKS_EINVAL, "null argument");
    std::memcpy(perm, h->h.perm.data(), sizeof(int64_t) * h->h.n);
    return GKS_OK;
}

gks_status gks_host_mesh_geometry(const gks_host_mesh *h, double *vol, double *xc)
{
    if (!h) return fail(GKS_EINVAL, "null mesh");
    if (vol) std::memcpy(vol, h->h.vol.data(), sizeof(double) * h->h.n);
    if (xc) std::memcpy(xc, h->h.xc.data(), sizeof(double) * 3 * h->h.n);
    return GKS_OK;
}

gks_status gks_host_mesh_face_geometry(const gks_host_mesh *h, double *fgeo)
{
    if (!h || !fgeo) return fail(GKS_EINVAL, "null argument");
    std::memcpy(fgeo, h->h.fgeo.data(), sizeof(double) * h->h.fgeo.size());
    return GKS_OK;
}

gks_status gks_host_mesh_faces(const gks_host_mesh *h, int32_t *owner, int32_t *nbr)
{
    if (!h) return fail(GKS_EINVAL, "null mesh");
    if (owner) std::memcpy(owner, h->h.owner.data(), sizeof(int32_t) * h->h.nf);
    if (nbr) std::memcpy(nbr, h->h.nbr.data(), sizeof(int32_t) * h->h.nf);
    return GKS_OK;
}

// The FP64 reconstruction's staging split for a mesh: the class whose limits hold the most of its
// 12-cell blocks (members and sub-stencil entries counted in the library's cell order).
static int k1_staging_class(const HostMesh &H)
{
    const int64_t n = H.n;
    int64_t staged[kK1Classes] = {0};
    for (int64_t c0 = 0; c0 < n; c0 += kK1Cells) {
        const int64_t c1 = std::min<int64_t>(c0 + kK1Cells, n);
        const int64_t e0 = H.st_ptr[c0], e1 = H.st_ptr[c1];
        int64_t subs = 0;
        for (int64_t k = e0; k < e1; ++k) subs += __builtin_popcount((unsigned)H.st_mask[k]);
        for (int c = 0; c < kK1Classes; ++c)
            if (e1 - e0 <= kK1StageOf[c] && subs <= kK1SubStageOf[c]) ++staged[c];
    }
    int best = 0;
    for (int c = 1; c < kK1Classes; ++c)
        if (staged[c] > staged[best]) best = c;
    return best;
}

// mesh arena layout (offsets only when base == nullptr)
static size_t mesh_layout(const HostMesh &H, int precision, DevMesh *d, char *base,
                          std::vector<std::pair<size_t, std::pair<const void *, size_t>>> *copies,
                          std::vector<std::vector<char>> *owned)
{
    const size_t es = precision == GKS_FP32_MIXED ? 4 : 8;
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) -> void * {
        size_t o = off;
        off = align256(off + (bytes ? bytes : 1));
        if (copies && bytes) copies->push_back({o, {src, bytes}});
        return base ? (void *)(base + o) : nullptr;
    };
    auto put_vec = [&](std::vector<char> &&v) -> void * {
        if (!owned) return put(nullptr, v.size());
        owned->push_back(std::move(v));
        return put(owned->back().data(), owned->back().size());
    };
    const int64_t n = H.n, nf = H.nf;
    std::vector<char> M(n), v23(8 * n), m2t(8 * 6 * n);
    if (owned) {
        for (int64_t i = 0; i < n; ++i) {
            const int t = H.type[i];
            M[i] = (char)(t == 3 ? 8 : t == 2 ? 6 : t == 0 ? 4 : 8);
            double v = std::cbrt(H.vol[i]);
            v = v * v;
            std::memcpy(&v23[8 * i], &v, 8);
            for (int q = 0; q < 6; ++q) std::memcpy(&m2t[8 * (q * n + i)], &H.m2[6 * i + q], 8);
        }
    }
    // [rows][width] row-major host data -> [width][rows] on the device, FP64 or FP32
    auto convert_t = [&](const std::vector<double> &v, size_t width) {
        std::vector<char> out(v.size() * es);
        if (owned) {
            const size_t rows = v.size() / width;
            for (size_t r = 0; r < rows; ++r)
                for (size_t j = 0; j < width; ++j) {
                    const double x = v[r * width + j];
                    const size_t o = j * rows + r;
                    if (es == 8)
                        std::memcpy(&out[8 * o], &x, 8);
                    else {
                        const float f = (float)x;
                        std::memcpy(&out[4 * o], &f, 4);
                    }
                }
        }
        return out;
    };
    // host data as stored (row-major), FP64 or FP32
    auto convert_n = [&](const std::vector<double> &v) {
        std::vector<char> out(v.size() * es);
        if (owned)
            for (size_t o = 0; o < v.size(); ++o) {
                if (es == 8)
                    std::memcpy(&out[8 * o], &v[o], 8);
                else {
                    const float f = (float)v[o];
                    std::memcpy(&out[4 * o], &f, 4);
                }
            }
        return out;
    };
    DevMesh dm{};
    dm.n = (int)n;
    dm.nf = (int)nf;
    dm.precision = precision;
    dm.M = (const int8_t *)put_vec(std::move(M));
    dm.vol = (const double *)put(H.vol.data(), 8 * n);
    dm.vol23 = (const double *)put_vec(std::move(v23));
    dm.m2 = (const double *)put_vec(std::move(m2t));
    dm.hcfl = (const double *)put(H.hcfl.data(), 8 * n);
    dm.st_ptr = (const int32_t *)put(H.st_ptr.data(), 4 * (n + 1));
    {
        std::vector<char> rec(owned ? 8 * H.st_idx.size() : 0);
        if (owned)
            for (size_t k = 0; k < H.st_idx.size(); ++k) {
                std::memcpy(&rec[8 * k], &H.st_idx[k], 4);
                const int32_t mk = H.st_mask[k];
                std::memcpy(&rec[8 * k + 4], &mk, 4);
            }
        dm.st_rec = owned ? (const int2 *)put_vec(std::move(rec)) : (const int2 *)put(nullptr, 8 * H.st_idx.size());
    }
    dm.nnz = (int)H.st_idx.size();
    dm.pinv = put_vec(convert_n(H.pinv));
    dm.dsc = put_vec(convert_n(H.dsc));
    dm.ginv = put_vec(convert_t(H.ginv, 48));
    dm.st_cell = (const int32_t *)put(H.st_idx.data(), 4 * H.st_idx.size());
    dm.st_flip = (const uint8_t *)put(H.st_flip.data(), H.st_flip.size());
    dm.walls = 0;
    for (int32_t b : H.nbr)
        if (b < 0) dm.walls = 1;
    dm.double_mirror = 0;
    for (uint8_t fl : H.st_flip)
        if (fl & 64u) dm.double_mirror = 1;
    {
        // sub-stencil lists in slot order, members in stencil order
        int64_t nss = 0;
        for (size_t k = 0; k < H.st_mask.size(); ++k) nss += __builtin_popcount((unsigned)H.st_mask[k]);
        std::vector<char> ptr(owned ? 4 * (8 * n + 1) : 0), loc(owned ? nss : 0);
        std::vector<double> B(owned ? 3 * nss : 0);
        if (owned) {
            int32_t e = 0;
            for (int64_t i = 0; i < n; ++i) {
                const double *g = &H.ginv[48 * i];
                for (int sl = 0; sl < 8; ++sl) {
                    std::memcpy(&ptr[4 * (8 * i + sl)], &e, 4);
                    for (int32_t k = H.st_ptr[i]; k < H.st_ptr[i + 1]; ++k) {
                        if (!(H.st_mask[k] >> sl & 1)) continue;
                        const double *gs = g + 6 * sl, *D = &H.dsc[3 * k];
                        loc[e] = (char)(k - H.st_ptr[i]);
                        B[3 * e + 0] = gs[0] * D[0] + gs[1] * D[1] + gs[2] * D[2];
                        B[3 * e + 1] = gs[1] * D[0] + gs[3] * D[1] + gs[4] * D[2];
                        B[3 * e + 2] = gs[2] * D[0] + gs[4] * D[1] + gs[5] * D[2];
                        ++e;
                    }
                }
            }
            std::memcpy(&ptr[4 * 8 * n], &e, 4);
        }
        dm.ss_ptr = owned ? (const int32_t *)put_vec(std::move(ptr)) : (const int32_t *)put(nullptr, 4 * (8 * n + 1));
        dm.ss_loc = owned ? (const uint8_t *)put_vec(std::move(loc)) : (const uint8_t *)put(nullptr, nss);
        dm.ss_B = owned ? put_vec(convert_n(B)) : put(nullptr, es * 3 * nss);
        dm.nss = (int)nss;
    }
    dm.owner = (const int32_t *)put(H.owner.data(), 4 * nf);
    dm.nbr = (const int32_t *)put(H.nbr.data(), 4 * nf);
    dm.fgeo = (const double *)put(H.fgeo.data(), 8 * H.fgeo.size());
    {
        // face normal from the summed weighted vector areas of the Gauss points, area as their sum of norms
        std::vector<char> fn(owned ? 8 * 4 * nf : 0);
        if (owned)
            for (int64_t f = 0; f < nf; ++f) {
                double A[3] = {0.0, 0.0, 0.0}, S = 0.0;
                for (int g = 0; g < 4; ++g) {
                    double v[3];
                    for (int q = 0; q < 3; ++q) {
                        v[q] = H.fgeo[(size_t)(6 + q) * 4 * nf + 4 * f + g];
                        A[q] += v[q];
                    }
                    S += std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                }
                const double a = std::sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
                const double row[4] = {A[0] / a, A[1] / a, A[2] / a, S};
                for (int q = 0; q < 4; ++q) std::memcpy(&fn[8 * ((size_t)q * nf + f)], &row[q], 8);
            }
        dm.fnS = owned ? (const double *)put_vec(std::move(fn)) : (const double *)put(nullptr, 8 * 4 * nf);
    }
    dm.cf_ptr = (const int32_t *)put(H.cf_ptr.data(), 4 * (n + 1));
    dm.cf_idx = (const int32_t *)put(H.cf_idx.data(), 4 * H.cf_idx.size());
    dm.tr_ptr = (const int32_t *)put(H.tr_ptr.data(), 4 * (n + 1));
    dm.tr_idx = (const int32_t *)put(H.tr_idx.data(), 4 * H.tr_idx.size());
    if (d) *d = dm;
    return off;
}

gks_status gks_mesh_sizes(const gks_host_mesh *h, int precision, size_t *mesh_bytes, size_t *work_bytes,
                          size_t *tape_bytes_per_step)
{
    if (!h || (precision != GKS_FP64 && precision != GKS_FP32_MIXED)) return fail(GKS_EINVAL, "bad argument");
    if (mesh_bytes) *mesh_bytes = mesh_layout(h->h, precision, nullptr, nullptr, nullptr, nullptr);
    if (work_bytes) *work_bytes = work_layout(h->h.n, h->h.nf, precision, nullptr, nullptr);
    if (tape_bytes_per_step) *tape_bytes_per_step = (precision == GKS_FP64 ? 8 : 4) * size_t(2) * 50 * (size_t)h->h.n;
    return GKS_OK;
}

gks_status gks_init_mesh(const gks_host_mesh *h, int precision, void *mesh_arena, size_t mesh_bytes,
                         gks_stream_t stream, gks_mesh **out)
{
    if (!h || !mesh_arena || !out || (precision != GKS_FP64 && precision != GKS_FP32_MIXED))
        return fail(GKS_EINVAL, "bad argument");
    if (((uintptr_t)mesh_arena & 255) != 0) return fail(GKS_EINVAL, "mesh arena must be 256-byte aligned");
    const size_t need = mesh_layout(h->h, precision, nullptr, nullptr, nullptr, nullptr);
    if (mesh_bytes < need) return fail(GKS_EINVAL, "mesh arena too small");
    std::vector<std::pair<size_t, std::pair<const void *, size_t>>> copies;
    std::vector<std::vector<char>> owned;
    owned.reserve(16);
    DevMesh d;
    mesh_layout(h->h, precision, &d, (char *)mesh_arena, &copies, &owned);
    for (auto &c : copies) {
        gks_status s = hip_check(hipMemcpyAsync((char *)mesh_arena + c.first, c.second.first, c.second.second,
                                                hipMemcpyHostToDevice, S(stream)),
                                 "mesh upload");
        if (s) return s;
    }
    gks_status s = hip_check(hipStreamSynchronize(S(stream)), "mesh upload sync");
    if (s) return s;
    gks_mesh *m = new (std::nothrow) gks_mesh;
    if (!m) return fail(GKS_EINVAL, "out of host memory");
    m->d = d;
    m->n = h->h.n;
    m->nf = h->h.nf;
    m->precision = precision;
    m->k1_class = k1_staging_class(h->h);
    int dev = 0, ncu = 0;
    if ((s = hip_check(hipGetDevice(&dev), "current device")) || (s = scratch_setup(dev))) {
        delete m;
        return s;
    }
    m->dev = dev;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        m->n_cu = ncu;
    *out = m;
    return GKS_OK;
}

void gks_destroy_mesh(gks_mesh *m)
{
    if (!m) return;
    for (hipEvent_t e : m->pool) (void)hipEventDestroy(e);
    delete m;
}

gks_status gks_set_flux_window(gks_mesh *m, int cells)
{
    if (!m) return fail(GKS_EINVAL, "null mesh");
    if (cells < 0 || cells > kWinCells) return fail(GKS_EINVAL, "flux window outside [0, 92] cells");
    m->flux_win = cells;
    return GKS_OK;
}

gks_status gks_profile(gks_mesh *m, int enable)
{
    if (!m) return fail(GKS_EINVAL, "null mesh");
    m->prof = enable != 0;
    return GKS_OK;
}

gks_status gks_profile_read(gks_mesh *m, double *total_ms, int64_t *launches)
{
    if (!m || !total_ms || !launches) return fail(GKS_EINVAL, "null argument");
    for (int k = 0; k < GKS_K_COUNT; ++k) {
        total_ms[k] = 0.0;
        launches[k] = 0;
    }
    if (!m->rec.empty()) {
        gks_status s = hip_check(hipEventSynchronize(m->pool[m->rec.back().second + 1]), "profile sync");
        if (s) return s;
    }
    for (auto &r : m->rec) {
        float ms = 0.0f;
        gks_status s = hip_check(hipEventElapsedTime(&ms, m->pool[r.second], m->pool[r.second + 1]), "profile read");
        if (s) return s;
        total_ms[r.first] += ms;
        launches[r.first] += 1;
    }
    m->rec.clear();
    m->used = 0;
    return GKS_OK;
}

static gks_status check_params(const gks_mesh *m, const gks_params *p)
{
    if (!m || !p) return fail(GKS_EINVAL, "null mesh or params");
    if (p->precision != m->precision) return fail(GKS_EINVAL, "params precision differs from the mesh precision");
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0)) return fail(GKS_EINVAL, "bad gamma or cfl");
    if (p->viscous && !(p->mu >= 0.0)) return fail(GKS_EINVAL, "bad viscosity");
    if (!(p->Pr > 0.0)) return fail(GKS_EINVAL, "bad Prandtl number");
    if (!(p->dt_max >= 0.0) || !std::isfinite(p->dt_max)) return fail(GKS_EINVAL, "dt_max must be finite and >= 0");
    bool general = false;
    for (int k = 0; k < 6; ++k) {
        const gks_boundary &b = p->bc[k];
        if (b.type < GKS_BC_SLIP || b.type > GKS_BC_EXTRAPOLATE) return fail(GKS_EINVAL, "unknown boundary condition");
        if (b.type != GKS_BC_SLIP) general = true;
        if (b.type == GKS_BC_ISOTHERMAL && !(b.Tw > 0.0 && std::isfinite(b.Tw)))
            return fail(GKS_EINVAL, "isothermal wall temperature must be finite and > 0");
        if (b.type == GKS_BC_FARFIELD && !(b.far[0] > 0.0 && b.far[4] > 0.0 && std::isfinite(b.far[1]) &&
                                           std::isfinite(b.far[2]) && std::isfinite(b.far[3])))
            return fail(GKS_EINVAL, "far-field state needs rho > 0, p > 0 and a finite velocity");
        if ((b.type == GKS_BC_NOSLIP || b.type == GKS_BC_ISOTHERMAL) &&
            !(std::isfinite(b.uw[0]) && std::isfinite(b.uw[1]) && std::isfinite(b.uw[2])))
            return fail(GKS_EINVAL, "wall velocity must be finite");
    }
    if (general && m->d.walls && m->d.double_mirror)
        return fail(GKS_EINVAL, "a stencil of this mesh reaches across both walls of an axis: only the reflective "
                                "condition is defined there");
    if (!(p->fallback_floor >= 0.0 && p->fallback_floor < 1.0)) return fail(GKS_EINVAL, "fallback_floor outside [0, 1)");
    if (!std::isfinite(p->mu_power) || (p->mu_power != 0.0 && !(p->T_ref > 0.0 && std::isfinite(p->T_ref))))
        return fail(GKS_EINVAL, "bad viscosity power law (mu_power, T_ref)");
    return GKS_OK;
}

static Work work_of(const gks_mesh *m, void *work)
{
    Work w;
    work_layout(m->n, m->nf, m->precision, &w, (char *)work);
    return w;
}

gks_status gks_reset_status(gks_mesh *m, void *work, gks_stream_t stream)
{
    if (!m || !work) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    return hip_check(hipMemsetAsync(w.status, 0, 2 * sizeof(int), S(stream)), "status reset");
}

static gks_status launch_timestep(gks_mesh *m, const double *Q, const gks_params *p, double *dt_dev, Work &w,
                                  hipStream_t st)
{
    ProfScope ps(m, GKS_K_TIMESTEP, st);
    int nb = (int)std::min<int64_t>(kDtBlocks, grid_for(m->n, kBlock));
    k_dt_partial<<<nb, kBlock, 0, st>>>((int)m->n, Q, m->d.hcfl, p->gamma, p->cfl, w.dtpart, w.status);
    k_dt_final<<<1, kBlock, 0, st>>>(nb, w.dtpart, dt_dev, p->dt_max);
    return hip_check(hipGetLastError(), "timestep launch");
}

gks_status gks_timestep(gks_mesh *m, const double *Q, const gks_params *p, double *dt_dev, void *work,
                        gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!Q || !dt_dev || !work) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    return launch_timestep(m, Q, p, dt_dev, w, S(stream));
}

static WenoParams weno_params(const gks_params *p)
{
    return WenoParams{p->weno_eps, p->weno_gamma_m, p->weno_p, p->force_linear};
}

static gks_status launch_reconstruct(gks_mesh *m, const double *Q, void *coeff, const gks_params *p, hipStream_t st)
{
    const unsigned grid = grid_for((int64_t)kK1CellLanes * m->n, kK1Block);
    ProfScope ps(m, GKS_K_RECONSTRUCT, st);
    const BoundarySet bcs = boundary_set(p);
    const bool gen = m->d.walls && bcs.any_general;
    const WenoParams wp = weno_params(p);
    if (m->precision == GKS_FP64) {
        double *c = (double *)coeff;
        switch (m->k1_class * 2 + (int)gen) {
        case 0: k_reconstruct<double, false, 0><<<grid, kK1Block, 0, st>>>(m->d, Q, c, wp, bcs); break;
        case 1: k_reconstruct<double, true, 0><<<grid, kK1Block, 0, st>>>(m->d, Q, c, wp, bcs); break;
        case 2: k_reconstruct<double, false, 1><<<grid, kK1Block, 0, st>>>(m->d, Q, c, wp, bcs); break;
        case 3: k_reconstruct<double, true, 1><<<grid, kK1Block, 0, st>>>(m->d, Q, c, wp, bcs); break;
        case 4: k_reconstruct<double, false, 2><<<grid, kK1Block, 0, st>>>(m->d, Q, c, wp, bcs); break;
        default: k_reconstruct<double, true, 2><<<grid, kK1Block, 0, st>>>(m->d, Q, c, wp, bcs); break;
        }
    } else {
        if (gen)
            k_reconstruct<float, true, 0><<<grid, kK1Block, 0, st>>>(m->d, Q, (float *)coeff, wp, bcs);
        else
            k_reconstruct<float, false, 0><<<grid, kK1Block, 0, st>>>(m->d, Q, (float *)coeff, wp, bcs);
    }
    return hip_check(hipGetLastError(), "reconstruct launch");
}

extern "C++" template <typename T, bool PR, bool SM>
static void launch_flux_t(gks_mesh *m, bool ext, unsigned grid, const T *coeff, const double *Q, const double *dt_dev,
                          T *ff, const FluxParams<T> &fp, int *status, hipStream_t st)
{
    if (ext) {
        k_flux<T, PR, true, SM><<<grid, kBlock, 0, st>>>(m->d, coeff, Q, dt_dev, ff, fp, status);
    } else if constexpr (sizeof(T) == 8 && !SM) {
        // the full FP64 flux runs 1 wave/SIMD: chunked with prefetch; the smooth one fits 2 waves/SIMD
        // one Gauss point per lane and measures faster that way (1.35 vs 1.53 ms at N = 64)
        const int64_t ncu = m->n_cu;
        const int64_t nf4 = 4 * (int64_t)m->nf;
        const int64_t per = ((nf4 + ncu * kBlock - 1) / (ncu * kBlock)) * kBlock;
        const int nblk = (int)((nf4 + per - 1) / per);
        k_flux_chunked<PR, SM><<<nblk, kBlock, 0, st>>>(m->d, coeff, dt_dev, ff, fp, status, (int)per, m->flux_win);
    } else {
        k_flux<T, PR, false, SM><<<grid, kBlock, 0, st>>>(m->d, coeff, Q, dt_dev, ff, fp, status);
    }
}

extern "C++" template <typename T, bool PR>
static void launch_flux_s(gks_mesh *m, bool ext, bool smooth, unsigned grid, const T *coeff, const double *Q,
                          const double *dt_dev, T *ff, const FluxParams<T> &fp, int *status, hipStream_t st)
{
    if (smooth)
        launch_flux_t<T, PR, true>(m, ext, grid, coeff, Q, dt_dev, ff, fp, status, st);
    else
        launch_flux_t<T, PR, false>(m, ext, grid, coeff, Q, dt_dev, ff, fp, status, st);
}

static gks_status launch_flux(gks_mesh *m, const void *coeff, const double *Q, const double *dt_dev, void *ff,
                              const gks_params *p, Work &w, hipStream_t st)
{
    const unsigned grid = grid_for(4 * m->nf, kBlock);
    ProfScope ps(m, GKS_K_FLUX, st);
    const bool pr = p->viscous && p->Pr != 1.0;
    // wall faces (neighbour < 0), the fallback and the viscosity power law exist only in the EXT
    // instantiation
    const bool ext = m->d.walls || p->first_order_fallback || (p->viscous && p->mu_power != 0.0);
    const bool sm = p->smooth_flux != 0;
    if (m->precision == GKS_FP64) {
        auto fp = flux_params<double>(p);
        const double *c = (const double *)coeff;
        if (pr)
            launch_flux_s<double, true>(m, ext, sm, grid, c, Q, dt_dev, (double *)ff, fp, w.status, st);
        else
            launch_flux_s<double, false>(m, ext, sm, grid, c, Q, dt_dev, (double *)ff, fp, w.status, st);
    } else {
        auto fp = flux_params<float>(p);
        const float *c = (const float *)coeff;
        if (pr)
            launch_flux_s<float, true>(m, ext, sm, grid, c, Q, dt_dev, (float *)ff, fp, w.status, st);
        else
            launch_flux_s<float, false>(m, ext, sm, grid, c, Q, dt_dev, (float *)ff, fp, w.status, st);
    }
    return hip_check(hipGetLastError(), "flux launch");
}

gks_status gks_reconstruct(gks_mesh *m, const double *Q, void *coeff, const gks_params *p, void *work,
                           gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!Q || !coeff) return fail(GKS_EINVAL, "null argument");
    (void)work;
    return launch_reconstruct(m, Q, coeff, p, S(stream));
}

gks_status gks_flux(gks_mesh *m, const void *coeff, const double *Q, const double *dt_dev, void *face_flux,
                    const gks_params *p, void *work, gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!coeff || !Q || !dt_dev || !face_flux || !work) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    return launch_flux(m, coeff, Q, dt_dev, face_flux, p, w, S(stream));
}

gks_status gks_residual(gks_mesh *m, const void *face_flux, double *L, double *dL, const gks_params *p,
                        gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!face_flux || !L || !dL) return fail(GKS_EINVAL, "null argument");
    const unsigned grid = grid_for(m->n, kBlock);
    ProfScope ps(m, GKS_K_RESIDUAL, S(stream));
    if (m->precision == GKS_FP64)
        k_residual<double><<<grid, kBlock, 0, S(stream)>>>(m->d, (const double *)face_flux, L, dL);
    else
        k_residual<float><<<grid, kBlock, 0, S(stream)>>>(m->d, (const float *)face_flux, L, dL);
    return hip_check(hipGetLastError(), "residual launch");
}

// one S2O4 step on the buffers of w (a caller's work buffer or the static scratch)
static gks_status run_s2o4(gks_mesh *m, double *Q, double *dt_dev, const gks_params *p, Work &w, double *Q_star,
                           void *coeff_tape, hipStream_t st)
{
    gks_status s;
    if (!p->dt_given && (s = launch_timestep(m, Q, p, dt_dev, w, st))) return s;
    const unsigned gc = grid_for(m->n, kBlock);
    // the stages' coefficients: the work buffer, or the caller's tape
    const size_t es = m->precision == GKS_FP64 ? 8 : 4;
    void *c1 = coeff_tape ? coeff_tape : w.coeff;
    void *c2 = coeff_tape ? (void *)((char *)coeff_tape + es * 50 * (size_t)m->n) : w.coeff;
    // stage 1
    if ((s = launch_reconstruct(m, Q, c1, p, st))) return s;
    if ((s = launch_flux(m, c1, Q, dt_dev, w.ff, p, w, st))) return s;
    {
    ProfScope ps(m, GKS_K_STAGE1, st);
    if (m->precision == GKS_FP64)
        k_stage1<double><<<gc, kBlock, 0, st>>>(m->d, (const double *)w.ff, Q, w.Qs, dt_dev);
    else
        k_stage1<float><<<gc, kBlock, 0, st>>>(m->d, (const float *)w.ff, Q, w.Qs, dt_dev);
    }
    if ((s = hip_check(hipGetLastError(), "stage-1 launch"))) return s;
    // stage 2
    if ((s = launch_reconstruct(m, w.Qs, c2, p, st))) return s;
    if ((s = launch_flux(m, c2, w.Qs, dt_dev, w.ff, p, w, st))) return s;
    {
    ProfScope ps(m, GKS_K_STAGE2, st);
    if (m->precision == GKS_FP64)
        k_stage2<double><<<gc, kBlock, 0, st>>>(m->d, (const double *)w.ff, Q, dt_dev);
    else
        k_stage2<float><<<gc, kBlock, 0, st>>>(m->d, (const float *)w.ff, Q, dt_dev);
    }
    if ((s = hip_check(hipGetLastError(), "stage-2 launch"))) return s;
    if (Q_star)
        return hip_check(hipMemcpyAsync(Q_star, w.Qs, sizeof(double) * 5 * m->n, hipMemcpyDeviceToDevice, st),
                         "Q* copy");
    return GKS_OK;
}

gks_status gks_s2o4_step(gks_mesh *m, double *Q, double *dt_dev, const gks_params *p, void *work, double *Q_star,
                         void *coeff_tape, gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!Q || !dt_dev || !work) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    return run_s2o4(m, Q, dt_dev, p, w, Q_star, coeff_tape, S(stream));
}

gks_status gks_s2o4_step_noalloc(gks_mesh *m, double *Q, double *dt_dev, const gks_params *p, int32_t *status_dev,
                                 double *Q_star, void *coeff_tape, gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!Q || !dt_dev || !status_dev) return fail(GKS_EINVAL, "null argument");
    const size_t need = work_layout(m->n, m->nf, m->precision, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(GKS_EINVAL, "mesh too large for the allocation-free step: it needs " + std::to_string(need) +
                                    " bytes of scratch, the library holds " + std::to_string(kScratchBytes));
    void *base = scratch_of(m->dev);
    if (!base) return fail(GKS_EDEVICE, "no scratch address for the mesh's device");
    Work w;
    work_layout(m->n, m->nf, m->precision, &w, (char *)base);
    // the sticky status word and the fallback count are the caller's; nothing in the scratch has to
    // start at zero (every other part is written before it is read)
    w.status = status_dev;
    return run_s2o4(m, Q, dt_dev, p, w, Q_star, coeff_tape, S(stream));
}

gks_status gks_implicit_step(gks_mesh *m, double *Q, double *dt_dev, double dt_factor, int kmax, const gks_params *p,
                             void *work, gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!Q || !dt_dev || !work) return fail(GKS_EINVAL, "null argument");
    if (!(dt_factor > 0.0) || kmax < 0 || kmax > 1000) return fail(GKS_EINVAL, "dt_factor must be > 0 and kmax in 0..1000");
    hipStream_t st = S(stream);
    Work w = work_of(m, work);
    if (!p->dt_given && (s = launch_timestep(m, Q, p, dt_dev, w, st))) return s;
    if ((s = launch_reconstruct(m, Q, w.coeff, p, st))) return s;
    if ((s = launch_flux(m, w.coeff, Q, dt_dev, w.ff, p, w, st))) return s;
    // the coefficients are consumed: their area holds b [5][n], the diagonal [n] and dQ [2][5][n]
    // (16 doubles per cell, within the 50 coefficients of either precision)
    const int64_t n = m->n;
    double *b = (double *)w.coeff, *diag = b + 5 * n, *dq[2] = {diag + n, diag + 6 * n};
    const unsigned gc = grid_for(n, kBlock);
    const BoundarySet bcs = boundary_set(p);
    {
        ProfScope ps(m, GKS_K_IMPLICIT, st);
        if (m->precision == GKS_FP64)
            k_implicit_init<double><<<gc, kBlock, 0, st>>>(m->d, (const double *)w.ff, Q, dt_dev, dt_factor, p->gamma, b,
                                                          diag, dq[0], bcs);
        else
            k_implicit_init<float><<<gc, kBlock, 0, st>>>(m->d, (const float *)w.ff, Q, dt_dev, dt_factor, p->gamma, b,
                                                         diag, dq[0], bcs);
        for (int k = 0; k < kmax; ++k)
            k_implicit_sweep<<<gc, kBlock, 0, st>>>(m->d, Q, p->gamma, b, diag, dq[k & 1], dq[(k + 1) & 1], bcs);
        const int len = (int)(5 * n);
        k_implicit_update<<<grid_for(len, kBlock), kBlock, 0, st>>>(len, Q, dq[kmax & 1]);
    }
    return hip_check(hipGetLastError(), "implicit step launch");
}

gks_status gks_adjoint_work_bytes(const gks_host_mesh *h, size_t *bytes)
{
    if (!h || !bytes) return fail(GKS_EINVAL, "null argument");
    *bytes = adj_layout(h->h.n, h->h.nf, (int64_t)h->h.st_idx.size(), nullptr, nullptr);
    return GKS_OK;
}

static gks_status launch_vjp(gks_mesh *m, const double *Qe, const double *coeff_in, const double *dt_dev,
                             const double *lp, const double *ls, double cL1, double cL2, double cD1, double cD2,
                             const gks_params *p, AdjWork &aw, hipStream_t st, double *out)
{
    gks_status s;
    const double *coeff = coeff_in;
    if (!coeff) {
        if ((s = launch_reconstruct(m, Qe, aw.coeff, p, st))) return s;
        coeff = aw.coeff;
    }
    const bool pr = p->viscous && p->Pr != 1.0;
    const FluxParams<double> fp = flux_params<double>(p);
    {
        ProfScope ps(m, GKS_K_FLUX_ADJ, st);
        const unsigned gb = grid_for(8 * m->nf, kBlock);
        // part 1 walks chunks of Gauss points, one block per compute unit (as the chunked flux)
        const int64_t ncu = m->n_cu;
        const int64_t nf4 = 4 * (int64_t)m->nf;
        const int64_t per = ((nf4 + ncu * kBlock - 1) / (ncu * kBlock)) * kBlock;
        const int na = (int)((nf4 + per - 1) / per);
        if (pr) {
            k_flux_adj_a<true><<<na, kBlock, 0, st>>>(m->d, coeff, dt_dev, lp, ls, cL1, cL2, cD1, cD2, fp, aw.abuf,
                                                      (int)per, m->flux_win);
            k_flux_adj_b<true><<<gb, kBlock, 0, st>>>(m->d, coeff, fp, aw.abuf, aw.cbf);
        } else {
            k_flux_adj_a<false><<<na, kBlock, 0, st>>>(m->d, coeff, dt_dev, lp, ls, cL1, cL2, cD1, cD2, fp, aw.abuf,
                                                       (int)per, m->flux_win);
            k_flux_adj_b<false><<<gb, kBlock, 0, st>>>(m->d, coeff, fp, aw.abuf, aw.cbf);
        }
    }
    {
        ProfScope ps(m, GKS_K_GATHER_ADJ, st);
        k_cbar_gather<<<grid_for(25 * m->n, kBlock), kBlock, 0, st>>>(m->d, aw.cbf, aw.cbc);
    }
    {
        ProfScope ps(m, GKS_K_RECONSTRUCT_ADJ, st);
        k_reconstruct_adj<<<grid_for((int64_t)kK1CellLanes * m->n, kK1Block), kK1Block, 0, st>>>(
            m->d, Qe, aw.cbc, weno_params(p), aw.dbar, aw.own);
    }
    {
        ProfScope ps(m, GKS_K_GATHER_ADJ, st);
        k_transpose_gather<<<grid_for(5 * m->n, kBlock), kBlock, 0, st>>>(m->d, aw.dbar, aw.own, out);
    }
    return hip_check(hipGetLastError(), "adjoint launch");
}

gks_status gks_adjoint_step(gks_mesh *m, const double *Qn, const double *Qstar, const double *dt_dev,
                            const double *lam_np1, double *lam_n, const gks_params *p, void *adj_work,
                            const double *coeff_tape, gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (m->precision != GKS_FP64) return fail(GKS_EINVAL, "the adjoint runs on an FP64 mesh");
    if (m->d.walls) return fail(GKS_EINVAL, "the adjoint is built for periodic meshes (this one has walls)");
    if (p->first_order_fallback) return fail(GKS_EINVAL, "the adjoint does not differentiate the first-order fallback");
    if (p->smooth_flux) return fail(GKS_EINVAL, "the adjoint differentiates the full flux (Eq. flux-1) only");
    if (p->viscous && p->mu_power != 0.0) return fail(GKS_EINVAL, "the adjoint covers a constant viscosity only");
    if (!Qn || !Qstar || !dt_dev || !lam_np1 || !lam_n || !adj_work) return fail(GKS_EINVAL, "null argument");
    if (((uintptr_t)adj_work & 255) != 0) return fail(GKS_EINVAL, "adjoint work buffer must be 256-byte aligned");
    AdjWork aw;
    adj_layout(m->n, m->nf, m->d.nnz, &aw, (char *)adj_work);
    hipStream_t st = S(stream);
    // lam* = dt^2/3 J_D(Q*)^T lam'
    const double *cn = coeff_tape, *cs = coeff_tape ? coeff_tape + 50 * (size_t)m->n : nullptr;
    if ((s = launch_vjp(m, Qstar, cs, dt_dev, lam_np1, nullptr, 0.0, 0.0, 1.0 / 3.0, 0.0, p, aw, st, aw.lstar)))
        return s;
    // J_L(Q)^T (dt lam' + dt/2 lam*) + J_D(Q)^T (dt^2/6 lam' + dt^2/8 lam*)
    if ((s = launch_vjp(m, Qn, cn, dt_dev, lam_np1, aw.lstar, 1.0, 0.5, 1.0 / 6.0, 0.125, p, aw, st, aw.vjp)))
        return s;
    const int len = (int)(5 * m->n);
    k_adj_combine<<<grid_for(len, kBlock), kBlock, 0, st>>>(len, lam_np1, aw.lstar, aw.vjp, lam_n);
    return hip_check(hipGetLastError(), "adjoint combine launch");
}

gks_status gks_kinetic_energy(gks_mesh *m, const double *Q, double *J_dev, double *dJdQ, void *work, gks_stream_t stream)
{
    if (!m || !Q || !J_dev || !work) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    hipStream_t st = S(stream);
    const int nb = (int)std::min<int64_t>(kDtBlocks, grid_for(m->n, kBlock));
    k_ke_partial<<<nb, kBlock, 0, st>>>((int)m->n, Q, m->d.vol, w.dtpart, dJdQ);
    k_sum_final<<<1, kBlock, 0, st>>>(nb, w.dtpart, J_dev);
    return hip_check(hipGetLastError(), "kinetic energy launch");
}

gks_status gks_poll_status(gks_mesh *m, void *work, gks_stream_t stream)
{
    if (!m || !work) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    int flag = 0;
    gks_status s = hip_check(hipMemcpyAsync(&flag, w.status, sizeof(int), hipMemcpyDeviceToHost, S(stream)), "status read");
    if (s) return s;
    if ((s = hip_check(hipStreamSynchronize(S(stream)), "status sync"))) return s;
    if (flag) return fail(GKS_ENONPHYS, "non-physical state (rho <= 0 or p <= 0) met in a kernel");
    return GKS_OK;
}

gks_status gks_fallback_count(gks_mesh *m, void *work, int64_t *count, gks_stream_t stream)
{
    if (!m || !work || !count) return fail(GKS_EINVAL, "null argument");
    Work w = work_of(m, work);
    int c = 0;
    gks_status s = hip_check(hipMemcpyAsync(&c, w.status + 1, sizeof(int), hipMemcpyDeviceToHost, S(stream)),
                             "fallback count read");
    if (s) return s;
    if ((s = hip_check(hipStreamSynchronize(S(stream)), "fallback count sync"))) return s;
    *count = c;
    return hip_check(hipMemsetAsync(w.status + 1, 0, sizeof(int), S(stream)), "fallback count reset");
}

gks_status gks_gp_flux_batch(int64_t n, const double *ql, const double *dql, const double *qr, const double *dqr,
                             const double *dt, double *out, const gks_params *p, gks_stream_t stream)
{
    if (n < 0 || !p || (n > 0 && (!ql || !dql || !qr || !dqr || !dt || !out))) return fail(GKS_EINVAL, "bad argument");
    if (n == 0) return GKS_OK;
    const unsigned grid = grid_for(n, kBlock);
    const bool pr = p->viscous && p->Pr != 1.0;
    hipStream_t st = S(stream);
    if (p->precision == GKS_FP32_MIXED) {
        if (pr)
            k_gp_batch<float, true><<<grid, kBlock, 0, st>>>(n, ql, dql, qr, dqr, dt, out, flux_params<float>(p));
        else
            k_gp_batch<float, false><<<grid, kBlock, 0, st>>>(n, ql, dql, qr, dqr, dt, out, flux_params<float>(p));
    } else {
        if (pr)
            k_gp_batch<double, true><<<grid, kBlock, 0, st>>>(n, ql, dql, qr, dqr, dt, out, flux_params<double>(p));
        else
            k_gp_batch<double, false><<<grid, kBlock, 0, st>>>(n, ql, dql, qr, dqr, dt, out, flux_params<double>(p));
    }
    return hip_check(hipGetLastError(), "gp flux launch");
}

gks_status gks_gp_flux_host(const double *ql, const double *dql, const double *qr, const double *dqr, double dt,
                            const gks_params *p, double *out)
{
    if (!ql || !dql || !qr || !dqr || !p || !out) return fail(GKS_EINVAL, "null argument");
    const bool pr = p->viscous && p->Pr != 1.0;
    bool ok;
    if (p->precision == GKS_FP32_MIXED) {
        const FluxParams<float> fp = flux_params<float>(p);
        float l[5], r[5], dl[3][5], dr[3][5], o[10];
        for (int j = 0; j < 5; ++j) {
            l[j] = (float)ql[j];
            r[j] = (float)qr[j];
        }
        for (int m = 0; m < 3; ++m)
            for (int j = 0; j < 5; ++j) {
                dl[m][j] = (float)dql[5 * m + j];
                dr[m][j] = (float)dqr[5 * m + j];
            }
        if (fp.smooth)
            ok = pr ? gp_flux<float, true, true>(l, dl, r, dr, (float)dt, fp, o)
                    : gp_flux<float, false, true>(l, dl, r, dr, (float)dt, fp, o);
        else
            ok = pr ? gp_flux<float, true>(l, dl, r, dr, (float)dt, fp, o) : gp_flux<float, false>(l, dl, r, dr, (float)dt, fp, o);
        for (int j = 0; j < 10; ++j) out[j] = o[j];
    } else {
        const FluxParams<double> fp = flux_params<double>(p);
        double dl[3][5], dr[3][5];
        for (int m = 0; m < 3; ++m)
            for (int j = 0; j < 5; ++j) {
                dl[m][j] = dql[5 * m + j];
                dr[m][j] = dqr[5 * m + j];
            }
        if (fp.smooth)
            ok = pr ? gp_flux<double, true, true>(ql, dl, qr, dr, dt, fp, out)
                    : gp_flux<double, false, true>(ql, dl, qr, dr, dt, fp, out);
        else
            ok = pr ? gp_flux<double, true>(ql, dl, qr, dr, dt, fp, out) : gp_flux<double, false>(ql, dl, qr, dr, dt, fp, out);
    }
    return ok ? GKS_OK : fail(GKS_ENONPHYS, "non-physical state");
}

gks_status gks_gp_flux_vjp_host(const double *ql, const double *dql, const double *qr, const double *dqr, double dt,
                                const gks_params *p, const double *outb, double *qlb, double *dqlb, double *qrb,
                                double *dqrb)
{
    if (!ql || !dql || !qr || !dqr || !p || !outb || !qlb || !dqlb || !qrb || !dqrb)
        return fail(GKS_EINVAL, "null argument");
    if (p->smooth_flux) return fail(GKS_EINVAL, "the reverse covers the full flux (Eq. flux-1) only");
    if (p->viscous && p->mu_power != 0.0) return fail(GKS_EINVAL, "the reverse covers a constant viscosity only");
    const FluxParams<double> fp = flux_params<double>(p);
    double dl[3][5], dr[3][5], dlb[3][5] = {}, drb[3][5] = {};
    double a[5] = {}, b[5] = {};
    for (int m = 0; m < 3; ++m)
        for (int j = 0; j < 5; ++j) {
            dl[m][j] = dql[5 * m + j];
            dr[m][j] = dqr[5 * m + j];
        }
    if (p->viscous && p->Pr != 1.0)
        gp_flux_b<double, true>(ql, dl, qr, dr, dt, fp, outb, a, dlb, b, drb);
    else
        gp_flux_b<double, false>(ql, dl, qr, dr, dt, fp, outb, a, dlb, b, drb);
    for (int j = 0; j < 5; ++j) {
        qlb[j] = a[j];
        qrb[j] = b[j];
    }
    for (int m = 0; m < 3; ++m)
        for (int j = 0; j < 5; ++j) {
            dqlb[5 * m + j] = dlb[m][j];
            dqrb[5 * m + j] = drb[m][j];
        }
    return GKS_OK;
}

gks_status gks_weno_combine_host(const double *a, const double *r, const double *gi, int M, double v23,
                                 const double *S, double q0, const gks_params *p, double *c)
{
    if (!a || !r || !gi || !S || !p || !c || M < 1 || M > 8) return fail(GKS_EINVAL, "bad argument");
    double b[8][3];
    for (int s = 0; s < 8; ++s) sym3_apply(gi + 6 * s, r + 3 * s, b[s]);
    weno_combine<double>(a, b, M, v23, S, q0, true, weno_params(p), c);
    return GKS_OK;
}

gks_status gks_weno_combine_vjp_host(const double *a, const double *r, const double *gi, int M, double v23,
                                     const double *S, const gks_params *p, const double *cb, double *ab, double *rb,
                                     double *q0b)
{
    if (!a || !r || !gi || !S || !p || !cb || !ab || !rb || !q0b || M < 1 || M > 8) return fail(GKS_EINVAL, "bad argument");
    double rr[8][3], rrb[8][3];
    for (int s = 0; s < 8; ++s)
        for (int q = 0; q < 3; ++q) rr[s][q] = r[3 * s + q];
    auto getg = [&](int s, double g[6]) {
        for (int q = 0; q < 6; ++q) g[q] = gi[6 * s + q];
    };
    double qb = 0.0;
    weno_combine_b<double>(a, rr, getg, M, v23, S, weno_params(p), cb, ab, rrb, qb);
    for (int s = 0; s < 8; ++s)
        for (int q = 0; q < 3; ++q) rb[3 * s + q] = rrb[s][q];
    *q0b = qb;
    return GKS_OK;
}

gks_status gks_gp_op_count(int viscous, double Pr, int64_t *adds, int64_t *muls, int64_t *divs, int64_t *transc)
{
    if (!adds || !muls || !divs || !transc) return fail(GKS_EINVAL, "null argument");
    // one Gauss point of the flux kernel on a generic smooth state, executed on the host
    Cnt cl[50], cr[50], geo[9];
    const double base[5] = {1.1, 0.3, -0.2, 0.1, 2.9};
    for (int c = 0; c < 5; ++c)
        for (int j = 0; j < 10; ++j) {
            cl[10 * c + j] = Cnt(j == 0 ? base[c] : 0.01 * (j + c));
            cr[10 * c + j] = Cnt(j == 0 ? 0.95 * base[c] : -0.01 * (j + 2 * c));
        }
    const double g[9] = {0.02, 0.01, -0.015, -0.03, 0.012, 0.011, 0.002, 0.0012, -0.0007};
    for (int q = 0; q < 9; ++q) geo[q] = Cnt(g[q]);
    gks_params p;
    gks_default_params(&p);
    p.viscous = viscous;
    p.mu = viscous ? 1e-3 : 0.0;
    p.Pr = Pr;
    FluxParams<Cnt> fp;
    fp.gamma = Cnt(p.gamma);
    fp.K = Cnt((5.0 - 3.0 * p.gamma) / (p.gamma - 1.0));
    fp.mu = Cnt(p.mu);
    fp.Pr = Cnt(p.Pr);
    fp.tau_eps = Cnt(p.tau_eps);
    fp.tau_C = Cnt(p.tau_C);
    fp.mu_power = Cnt(0.0);  // constant viscosity (the benchmark's)
    fp.iT_ref = Cnt(1.0);
    fp.viscous = p.viscous;
    fp.fallback = 0;
    fp.floor = 0.0;
    fp.smooth = 0;
    op_counts() = OpCounts();
    Cnt out[10];
    int nfb = 0;
    const bool ok = (viscous && Pr != 1.0) ? face_gp<Cnt, true, false>(cl, cr, nullptr, nullptr, geo, Cnt(0.01), fp, out, nfb)
                                           : face_gp<Cnt, false, false>(cl, cr, nullptr, nullptr, geo, Cnt(0.01), fp, out, nfb);
    const OpCounts c = op_counts();
    *adds = c.add;
    *muls = c.mul;
    *divs = c.div;
    *transc = c.transc;
    return ok ? GKS_OK : fail(GKS_EINVAL, "counting state was non-physical");
}

}  // extern "C"
