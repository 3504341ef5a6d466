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
#include <new>
#include <string>
#include <vector>

#include "gks_flux.h"
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
    const void *pinv;       // [9][nnz] (coefficient-major), FP64 or FP32
    const void *dsc;        // [3][nnz] scaled member centroid offsets, FP64 or FP32
    const void *ginv;       // [48][n] inverses of the sub-stencil normal matrices / h, FP64 or FP32
    // faces
    const int32_t *owner, *nbr;
    const double *fgeo;     // [9][4 nf]
    const int32_t *cf_ptr, *cf_idx;
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

__global__ void __launch_bounds__(kBlock) k_dt_final(int nb, const double *__restrict__ part, double *dt)
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
    if (threadIdx.x == 0) dt[0] = red[0];
}

// ---------------------------------------------------------------------------
// K1: WENO reconstruction, one lane per (cell, component)
// ---------------------------------------------------------------------------
struct WenoParams {
    double eps, gm, p;
    int force_linear;
};

template <typename T>
__device__ __forceinline__ T wpow(T x, T p)
{
    if (p == T(1)) return x;
    if (p == T(2)) return x * x;
    return (T)pow((double)x, (double)p);
}

// Four lanes cooperate on one (cell, conserved component): lane l streams
// members l, l+4, ... of the cell's stencil, so a cell's 20 lanes read
// consecutive operator entries and each lane's chain of dependent loads is short;
// the partial fits are summed over the quad with DPP lane permutations, so every
// lane of the quad holds bitwise-identical totals (deterministic, no atomics).
constexpr int kK1Lanes = 4;
constexpr int kK1CellLanes = 5 * kK1Lanes;
constexpr int kK1Block = 16 * kK1CellLanes;  // 16 cells, 5 waves

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
template <typename T>
__global__ void __launch_bounds__(kK1Block) k_reconstruct(DevMesh m, const double *__restrict__ Q, T *__restrict__ coeff,
                                                          WenoParams wp)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * kK1Block + threadIdx.x;
    const int n = m.n;
    const int ic = t / kK1CellLanes;
    const int lane = t - kK1CellLanes * ic;
    const int comp = lane >> 2;
    const int l = lane & 3;
    const bool valid = ic < n;
    const int i = valid ? ic : n - 1;  // tail lanes shadow the last cell and write nothing
    const T *pinv = (const T *)m.pinv;
    const T *dsc = (const T *)m.dsc;
    const int nnz = m.nnz;
    const int k0 = m.st_ptr[i], k1 = m.st_ptr[i + 1];
    const double *Qc = Q + (size_t)comp * n;
    const double q0 = Qc[i];
    T a[9], r[8][3];
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = T(0);
#pragma unroll
    for (int s = 0; s < 8; ++s) r[s][0] = r[s][1] = r[s][2] = T(0);
#pragma unroll 2
    for (int k = k0 + l; k < k1; k += kK1Lanes) {
        const int2 rec = m.st_rec[k];
        const T d = (T)(Qc[rec.x] - q0);
#pragma unroll
        for (int j = 0; j < 9; ++j) a[j] += pinv[(size_t)j * nnz + k] * d;
        const T dx = dsc[k] * d, dy = dsc[(size_t)nnz + k] * d, dz = dsc[(size_t)2 * nnz + k] * d;
        const unsigned mask = (unsigned)rec.y;
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (mask & (1u << s)) {
                r[s][0] += dx;
                r[s][1] += dy;
                r[s][2] += dz;
            }
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = quad_sum(a[j]);
    // linear sub-stencil fits: b^m = G_m^{-1} r_m / h (normal equations of the scaled offsets)
    const T *gi = (const T *)m.ginv;
    T b[8][3];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const T r0 = quad_sum(r[s][0]), r1 = quad_sum(r[s][1]), r2 = quad_sum(r[s][2]);
        const T g00 = gi[(size_t)(6 * s + 0) * n + i], g01 = gi[(size_t)(6 * s + 1) * n + i],
                g02 = gi[(size_t)(6 * s + 2) * n + i], g11 = gi[(size_t)(6 * s + 3) * n + i],
                g12 = gi[(size_t)(6 * s + 4) * n + i], g22 = gi[(size_t)(6 * s + 5) * n + i];
        b[s][0] = g00 * r0 + g01 * r1 + g02 * r2;
        b[s][1] = g01 * r0 + g11 * r1 + g12 * r2;
        b[s][2] = g02 * r0 + g12 * r1 + g22 * r2;
    }
    const int M = m.M[i];
    const T v23 = (T)m.vol23[i];
    const T S00 = (T)m.m2[i], S01 = (T)m.m2[n + i], S02 = (T)m.m2[2 * n + i], S11 = (T)m.m2[3 * n + i],
            S12 = (T)m.m2[4 * n + i], S22 = (T)m.m2[5 * n + i];
    const T gm = (T)wp.gm, g0 = T(1) - gm * T(M), eps = (T)wp.eps, pw = (T)wp.p;
    // smoothness indicators (Eq. indicator) over the cell: a = x y z xx xy xz yy yz zz
    const T H[3][3] = {{T(2) * a[3], a[4], a[5]}, {a[4], T(2) * a[6], a[7]}, {a[5], a[7], T(2) * a[8]}};
    T beta0 = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T h0 = H[d][0], h1 = H[d][1], h2 = H[d][2];
        const T quad = h0 * (S00 * h0 + S01 * h1 + S02 * h2) + h1 * (S01 * h0 + S11 * h1 + S12 * h2) +
                       h2 * (S02 * h0 + S12 * h1 + S22 * h2);
        beta0 += a[d] * a[d] + quad;
    }
    const T sec = T(4) * (a[3] * a[3] + a[6] * a[6] + a[8] * a[8]) + a[4] * a[4] + a[5] * a[5] + a[7] * a[7];
    beta0 = v23 * beta0 + v23 * v23 * sec;
    T beta[8];
    T tw = T(0);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        beta[s] = v23 * (b[s][0] * b[s][0] + b[s][1] * b[s][1] + b[s][2] * b[s][2]);
        if (s < M) tw += fabs(beta0 - beta[s]);
    }
    tw /= T(M);
    // nonlinear weights and Eq. weno folded into one quadratic
    T w0, ws[8];
    if (wp.force_linear) {
        w0 = g0;
#pragma unroll
        for (int s = 0; s < 8; ++s) ws[s] = gm;
    } else {
        w0 = g0 * (T(1) + wpow(tw / (beta0 + eps), pw));
#pragma unroll
        for (int s = 0; s < 8; ++s) ws[s] = gm * (T(1) + wpow(tw / (beta[s] + eps), pw));
    }
    T sum = w0;
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (s < M) sum += ws[s];
    const T isum = T(1) / sum;
    const T f0 = w0 * isum / g0;
    T c[10];
#pragma unroll
    for (int j = 0; j < 9; ++j) c[1 + j] = f0 * a[j];
    const T sub0 = f0 * gm;
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (s < M) {
            const T fs = ws[s] * isum - sub0;
            c[1] += fs * b[s][0];
            c[2] += fs * b[s][1];
            c[3] += fs * b[s][2];
        }
    // constant term: cell average minus the means of the quadratic monomials
    const T corr = -(c[4] * S00 + c[5] * S01 + c[6] * S02 + c[7] * S11 + c[8] * S12 + c[9] * S22);
    if constexpr (sizeof(T) == 8)
        c[0] = (T)q0 + corr;
    else
        c[0] = corr;
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

template <typename T, bool PR>
__global__ void __launch_bounds__(kBlock) k_flux(DevMesh m, const T *__restrict__ coeff, const double *__restrict__ Q,
                                                 const double *__restrict__ dt_dev, T *__restrict__ ff, FluxParams<T> fp,
                                                 int *status)
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
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            ql0[c] = Q[(size_t)c * m.n + o];
            qr0[c] = Q[(size_t)c * m.n + nb];
        }
    }
    const T dt = (T)dt_dev[0];
    T out[10];
    const bool ok = face_gp<T, PR>(coeff + (size_t)50 * o, coeff + (size_t)50 * nb, ql0, qr0, geo, dt, fp, out);
    if (live && !ok) status[0] = 1;
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
    return f;
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
}

const char *gks_last_error(void) { return g_err.c_str(); }

gks_status gks_preprocess(int64_t n_nodes, const double *nodes, int64_t n_cells, const int8_t *types,
                          const int64_t *cells, const double *box, int periodic, gks_host_mesh **out)
{
    if (!out) return fail(GKS_EINVAL, "null output");
    *out = nullptr;
    gks_host_mesh *h = new (std::nothrow) gks_host_mesh;
    if (!h) return fail(GKS_EINVAL, "out of host memory");
    gks_status s;
    try {
        s = preprocess(n_nodes, nodes, n_cells, types, cells, box, periodic, h->h);
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
    if (n_subcoef) *n_subcoef = (int64_t)h->h.ginv.size() / 6;
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

gks_status gks_host_mesh_faces(const gks_host_mesh *h, int32_t *owner, int32_t *nbr)
{
    if (!h) return fail(GKS_EINVAL, "null mesh");
    if (owner) std::memcpy(owner, h->h.owner.data(), sizeof(int32_t) * h->h.nf);
    if (nbr) std::memcpy(nbr, h->h.nbr.data(), sizeof(int32_t) * h->h.nf);
    return GKS_OK;
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
    dm.pinv = put_vec(convert_t(H.pinv, 9));
    dm.dsc = put_vec(convert_t(H.dsc, 3));
    dm.ginv = put_vec(convert_t(H.ginv, 48));
    dm.owner = (const int32_t *)put(H.owner.data(), 4 * nf);
    dm.nbr = (const int32_t *)put(H.nbr.data(), 4 * nf);
    dm.fgeo = (const double *)put(H.fgeo.data(), 8 * H.fgeo.size());
    dm.cf_ptr = (const int32_t *)put(H.cf_ptr.data(), 4 * (n + 1));
    dm.cf_idx = (const int32_t *)put(H.cf_idx.data(), 4 * H.cf_idx.size());
    if (d) *d = dm;
    return off;
}

gks_status gks_mesh_sizes(const gks_host_mesh *h, int precision, size_t *mesh_bytes, size_t *work_bytes)
{
    if (!h || (precision != GKS_FP64 && precision != GKS_FP32_MIXED)) return fail(GKS_EINVAL, "bad argument");
    if (mesh_bytes) *mesh_bytes = mesh_layout(h->h, precision, nullptr, nullptr, nullptr, nullptr);
    if (work_bytes) *work_bytes = work_layout(h->h.n, h->h.nf, precision, nullptr, nullptr);
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
    *out = m;
    return GKS_OK;
}

void gks_destroy_mesh(gks_mesh *m)
{
    if (!m) return;
    for (hipEvent_t e : m->pool) (void)hipEventDestroy(e);
    delete m;
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
    return hip_check(hipMemsetAsync(w.status, 0, sizeof(int), S(stream)), "status reset");
}

static gks_status launch_timestep(gks_mesh *m, const double *Q, const gks_params *p, double *dt_dev, Work &w,
                                  hipStream_t st)
{
    ProfScope ps(m, GKS_K_TIMESTEP, st);
    int nb = (int)std::min<int64_t>(kDtBlocks, grid_for(m->n, kBlock));
    k_dt_partial<<<nb, kBlock, 0, st>>>((int)m->n, Q, m->d.hcfl, p->gamma, p->cfl, w.dtpart, w.status);
    k_dt_final<<<1, kBlock, 0, st>>>(nb, w.dtpart, dt_dev);
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
    if (m->precision == GKS_FP64)
        k_reconstruct<double><<<grid, kK1Block, 0, st>>>(m->d, Q, (double *)coeff, weno_params(p));
    else
        k_reconstruct<float><<<grid, kK1Block, 0, st>>>(m->d, Q, (float *)coeff, weno_params(p));
    return hip_check(hipGetLastError(), "reconstruct launch");
}

static gks_status launch_flux(gks_mesh *m, const void *coeff, const double *Q, const double *dt_dev, void *ff,
                              const gks_params *p, Work &w, hipStream_t st)
{
    const unsigned grid = grid_for(4 * m->nf, kBlock);
    ProfScope ps(m, GKS_K_FLUX, st);
    const bool pr = p->viscous && p->Pr != 1.0;
    if (m->precision == GKS_FP64) {
        auto fp = flux_params<double>(p);
        if (pr)
            k_flux<double, true><<<grid, kBlock, 0, st>>>(m->d, (const double *)coeff, Q, dt_dev, (double *)ff, fp, w.status);
        else
            k_flux<double, false><<<grid, kBlock, 0, st>>>(m->d, (const double *)coeff, Q, dt_dev, (double *)ff, fp, w.status);
    } else {
        auto fp = flux_params<float>(p);
        if (pr)
            k_flux<float, true><<<grid, kBlock, 0, st>>>(m->d, (const float *)coeff, Q, dt_dev, (float *)ff, fp, w.status);
        else
            k_flux<float, false><<<grid, kBlock, 0, st>>>(m->d, (const float *)coeff, Q, dt_dev, (float *)ff, fp, w.status);
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

gks_status gks_s2o4_step(gks_mesh *m, double *Q, double *dt_dev, const gks_params *p, void *work, double *Q_star,
                         gks_stream_t stream)
{
    gks_status s = check_params(m, p);
    if (s) return s;
    if (!Q || !dt_dev || !work) return fail(GKS_EINVAL, "null argument");
    hipStream_t st = S(stream);
    Work w = work_of(m, work);
    if (!p->dt_given && (s = launch_timestep(m, Q, p, dt_dev, w, st))) return s;
    const unsigned gc = grid_for(m->n, kBlock);
    // stage 1
    if ((s = launch_reconstruct(m, Q, w.coeff, p, st))) return s;
    if ((s = launch_flux(m, w.coeff, Q, dt_dev, w.ff, p, w, st))) return s;
    {
    ProfScope ps(m, GKS_K_STAGE1, st);
    if (m->precision == GKS_FP64)
        k_stage1<double><<<gc, kBlock, 0, st>>>(m->d, (const double *)w.ff, Q, w.Qs, dt_dev);
    else
        k_stage1<float><<<gc, kBlock, 0, st>>>(m->d, (const float *)w.ff, Q, w.Qs, dt_dev);
    }
    if ((s = hip_check(hipGetLastError(), "stage-1 launch"))) return s;
    // stage 2
    if ((s = launch_reconstruct(m, w.Qs, w.coeff, p, st))) return s;
    if ((s = launch_flux(m, w.coeff, w.Qs, dt_dev, w.ff, p, w, st))) return s;
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
    fp.viscous = p.viscous;
    op_counts() = OpCounts();
    Cnt out[10];
    const bool ok = (viscous && Pr != 1.0) ? face_gp<Cnt, true>(cl, cr, nullptr, nullptr, geo, Cnt(0.01), fp, out)
                                           : face_gp<Cnt, false>(cl, cr, nullptr, nullptr, geo, Cnt(0.01), fp, out);
    const OpCounts c = op_counts();
    *adds = c.add;
    *muls = c.mul;
    *divs = c.div;
    *transc = c.transc;
    return ok ? GKS_OK : fail(GKS_EINVAL, "counting state was non-physical");
}

}  // extern "C"
