// Gas-kinetic flux at one face Gauss point, in the local frame (n1, n2, n3).
//
// Section 3.2 of Yang, Pan & Xu (arXiv 2203.09047): the distribution of
// Eq. flux-1 built from the Maxwellians g_l, g_r of the reconstructed states
// on both sides, the interface equilibrium g_0 (its conserved moments are the
// half-space moments u > 0 of g_l plus u < 0 of g_r), the spatial slopes
// <a_m> = dQ/dn_m and time slopes from <a_1 u + a_2 v + a_3 w + A> = 0 on both
// sides and for g_0.  Its flux moments are integrated in closed form over
// [0, delta] for delta = dt/2 and dt, which gives the flux at the start of
// the step and its time derivative (two-stage fourth-order GKS).
//
// Moments of a normalised Maxwellian with velocity (U, V, W) and
// lambda = rho / (2 p) factorise over u, v, w and the K internal degrees of
// freedom; the full-space ones obey <u^(k+2)> = U <u^(k+1)> + (k+1)/(2 lambda) <u^k>,
// the half-space ones start from erfc and exp and obey the same recursion.
// The slope solves <psi psi^T> a = b use their closed-form inverse.
#pragma once

#include <hip/hip_runtime.h>

#include "gks_bc.h"

namespace gks {

template <typename T>
struct FluxParams {
    T gamma, K, mu, Pr, tau_eps, tau_C;
    T mu_power, iT_ref;  // viscosity mu (T0 / T_ref)^mu_power at the interface temperature (0: constant)
    int viscous;
    int fallback;  // first-order fallback of non-physical side states
    int smooth;    // the smooth-flow distribution (Eq. flux-2) instead of Eq. flux-1
    double floor;  // ... and of states whose rho or p is at most floor times the cell average's
    // the box planes' boundary conditions (meshes with walls; plane 2 axis + hi)
    int bc_type[6];
    T bc_uw[6][3], bc_Tw[6], bc_far[6][5];
};

// Moments <u^k> (k <= 6), <v^k>, <w^k> (k <= 5), <s^2>, <s^4> of one normalised Maxwellian.
template <typename T>
struct Mom {
    T u[7], v[6], w[6], s1, s2;
};

template <typename T>
__host__ __device__ __forceinline__ void recur7(T *m, T U, T h)  // h = 1 / (2 lambda)
{
#pragma unroll
    for (int k = 0; k + 2 < 7; ++k) m[k + 2] = U * m[k + 1] + T(k + 1) * h * m[k];
}

template <typename T>
__host__ __device__ __forceinline__ void recur6(T *m, T U, T h)
{
#pragma unroll
    for (int k = 0; k + 2 < 6; ++k) m[k + 2] = U * m[k + 1] + T(k + 1) * h * m[k];
}

template <typename T>
__host__ __device__ __forceinline__ T erfc_t(T x);
template <>
__host__ __device__ __forceinline__ double erfc_t<double>(double x) { return erfc(x); }
template <>
__host__ __device__ __forceinline__ float erfc_t<float>(float x) { return erfcf(x); }
template <typename T>
__host__ __device__ __forceinline__ T exp_t(T x);
template <>
__host__ __device__ __forceinline__ double exp_t<double>(double x) { return exp(x); }
template <>
__host__ __device__ __forceinline__ float exp_t<float>(float x) { return expf(x); }
template <typename T>
__host__ __device__ __forceinline__ T pow_t(T x, T y);
template <>
__host__ __device__ __forceinline__ double pow_t<double>(double x, double y) { return pow(x, y); }
template <>
__host__ __device__ __forceinline__ float pow_t<float>(float x, float y) { return powf(x, y); }
template <typename T>
__host__ __device__ __forceinline__ T expm1_t(T x);
template <>
__host__ __device__ __forceinline__ double expm1_t<double>(double x) { return expm1(x); }
template <>
__host__ __device__ __forceinline__ float expm1_t<float>(float x) { return expm1f(x); }
template <typename T>
__host__ __device__ __forceinline__ T sqrt_t(T x);
template <>
__host__ __device__ __forceinline__ double sqrt_t<double>(double x) { return sqrt(x); }
template <>
__host__ __device__ __forceinline__ float sqrt_t<float>(float x) { return sqrtf(x); }

// Full-space v, w, internal moments (shared by full and half-space sets of one state); h = 1 / (2 lambda).
template <typename T>
__host__ __device__ __forceinline__ void mom_common(Mom<T> &m, T V, T W, T h, T K)
{
    m.v[0] = T(1);
    m.v[1] = V;
    recur6(m.v, V, h);
    m.w[0] = T(1);
    m.w[1] = W;
    recur6(m.w, W, h);
    m.s1 = K * h;
    m.s2 = K * (K + T(2)) * h * h;
}

template <typename T>
__host__ __device__ __forceinline__ void mom_full_u(Mom<T> &m, T U, T h)
{
    m.u[0] = T(1);
    m.u[1] = U;
    recur7(m.u, U, h);
}

// erfc(x): for |x| < 1 from the Maclaurin series of erf (erf x = 2/sqrt(pi) sum_n (-1)^n x^(2n+1) /
// (n! (2n+1)), Abramowitz & Stegun 7.1.5), truncated where the next term is below the type's rounding
// (the coefficients are that formula, evaluated by the compiler); beyond, the library's erfc.
constexpr double erf_series_coef(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return (n % 2 ? -1.0 : 1.0) / (f * (2 * n + 1));
}

// the library's erfc out of line: lanes that need it are rare, and inlined it would hold registers
// across the whole flux
template <typename T>
__host__ __device__ __attribute__((noinline)) T erfc_outline(T x)
{
    return erfc_t(x);
}

template <typename T>
__host__ __device__ __forceinline__ T erfc_half(T x)
{
    constexpr int N = sizeof(T) == 8 ? 18 : 10;  // |term N+1| < 5e-18 (FP64), 1e-9 (FP32) for |x| < 1
    if (x < T(1) && x > T(-1)) {
        const T z = x * x;
        T s = T(erf_series_coef(N));
#pragma unroll
        for (int n = N - 1; n >= 0; --n) s = s * z + T(erf_series_coef(n));
        return T(1) - T(M_2_SQRTPI) * x * s;
    }
    return erfc_outline(x);
}

// sign = +1: u > 0, -1: u < 0.  One square root gives both sqrt(lambda) and its inverse:
// sqrt(2 h) = 1 / sqrt(lambda).
template <typename T>
__host__ __device__ __forceinline__ void mom_half_u(Mom<T> &m, T U, T lam, T h, T sign)
{
    const T isl = sqrt_t(T(2) * h);
    const T sl = lam * isl;
    const T e = exp_t(-lam * U * U) * (T(0.25 * M_2_SQRTPI) * isl);  // exp(-lambda U^2) / (2 sqrt(pi lambda))
    m.u[0] = T(0.5) * erfc_half(-sign * sl * U);
    m.u[1] = U * m.u[0] + sign * e;
    recur7(m.u, U, h);
}

// The symmetric moment matrix Q = <u^k v^l w^n psi psi^T> of one moment set, upper triangle by
// rows (00 01 02 03 04 11 12 13 14 22 23 24 33 34 44), psi = (1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2).
// The flux needs <u^k v^l w^n psi> (Q's first column, psi_0 = 1) and, for slopes a,
// <u^k v^l w^n (a . psi) psi> = Q a: each matrix is formed once and applied to every slope.
template <typename T>
struct Q5 {
    T e[15];
};

template <int k, int l, int n, typename T>
__host__ __device__ __forceinline__ void qmat(const Mom<T> &M, Q5<T> &Q)
{
    const T *u = M.u + k, *v = M.v + l, *w = M.w + n;
    // products of the v and w moments that the entries share
    const T a00 = v[0] * w[0], a10 = v[1] * w[0], a01 = v[0] * w[1], a20 = v[2] * w[0], a11 = v[1] * w[1];
    const T a02 = v[0] * w[2], a30 = v[3] * w[0], a21 = v[2] * w[1], a12 = v[1] * w[2], a03 = v[0] * w[3];
    const T a40 = v[4] * w[0], a22 = v[2] * w[2], a04 = v[0] * w[4];
    Q.e[0] = u[0] * a00;
    Q.e[1] = u[1] * a00;
    Q.e[2] = u[0] * a10;
    Q.e[3] = u[0] * a01;
    Q.e[5] = u[2] * a00;
    Q.e[6] = u[1] * a10;
    Q.e[7] = u[1] * a01;
    Q.e[9] = u[0] * a20;
    Q.e[10] = u[0] * a11;
    Q.e[12] = u[0] * a02;
    const T tr = Q.e[5] + Q.e[9] + Q.e[12];  // <u^k v^l w^n (u^2 + v^2 + w^2)>
    Q.e[4] = T(0.5) * (tr + M.s1 * Q.e[0]);
    Q.e[8] = T(0.5) * (u[3] * a00 + u[1] * (a20 + a02) + M.s1 * Q.e[1]);
    Q.e[11] = T(0.5) * (u[2] * a10 + u[0] * (a30 + a12) + M.s1 * Q.e[2]);
    Q.e[13] = T(0.5) * (u[2] * a01 + u[0] * (a21 + a03) + M.s1 * Q.e[3]);
    Q.e[14] = T(0.25) * (u[4] * a00 + u[0] * (a40 + a04 + T(2) * a22) + T(2) * u[2] * (a20 + a02) +
                         M.s2 * Q.e[0] + T(2) * M.s1 * tr);
}

// o = Q a
template <typename T>
__host__ __device__ __forceinline__ void qmul(const Q5<T> &Q, const T a[5], T o[5])
{
    const T *e = Q.e;
    o[0] = e[0] * a[0] + e[1] * a[1] + e[2] * a[2] + e[3] * a[3] + e[4] * a[4];
    o[1] = e[1] * a[0] + e[5] * a[1] + e[6] * a[2] + e[7] * a[3] + e[8] * a[4];
    o[2] = e[2] * a[0] + e[6] * a[1] + e[9] * a[2] + e[10] * a[3] + e[11] * a[4];
    o[3] = e[3] * a[0] + e[7] * a[1] + e[10] * a[2] + e[12] * a[3] + e[13] * a[4];
    o[4] = e[4] * a[0] + e[8] * a[1] + e[11] * a[2] + e[13] * a[3] + e[14] * a[4];
}

// o += Q a
template <typename T>
__host__ __device__ __forceinline__ void qmul_add(const Q5<T> &Q, const T a[5], T o[5])
{
    T t[5];
    qmul(Q, a, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += t[j];
}

// y += s * (first column of Q) = s * P<k,l,n>
template <typename T>
__host__ __device__ __forceinline__ void qcol0_axpy(const Q5<T> &Q, T s, T y[5])
{
    y[0] += s * Q.e[0];
    y[1] += s * Q.e[1];
    y[2] += s * Q.e[2];
    y[3] += s * Q.e[3];
    y[4] += s * Q.e[4];
}

// o += <u^k x (a . psi) psi> for x = v (DIR = 2) or w (DIR = 3), from Qa = <u^k (a . psi) psi> and
// P = <u^k psi>.  x is a Gaussian of mean X and variance h in every moment set (also the half-space
// ones), so <x f(x)> = X <f> + h <df/dx> (Stein's identity) with d(psi)/dx = e_DIR + x e_4:
//   o_j += X Qa_j + h (a_DIR + a_4 X) P_j,  o_DIR += h (Qa_0 + h a_4 P_0),
//   o_4 += h (<u^k x (a . psi)> + h a_4 P_0 X),  <u^k x (a . psi)> = X Qa_0 + h P_0 (a_DIR + a_4 X).
template <int DIR, typename T>
__host__ __device__ __forceinline__ void stein_add(const T Qa[5], const T P[5], T X, T h, const T a[5], T o[5])
{
    const T c = a[DIR] + a[4] * X;
    const T hc = h * c;
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += X * Qa[j] + hc * P[j];
    const T ha4u = h * a[4] * P[0];
    o[DIR] += h * (Qa[0] + ha4u);
    o[4] += h * (X * Qa[0] + hc * P[0] + ha4u * X);
}

// o += <u^2 (a . psi) psi> of a full-space set (u Gaussian of mean U and variance h) from
// Q1a = <u (a . psi) psi>, B = <(a . psi) psi>, P1 = <u psi>, P2 = <u^2 psi>: Stein's identity in u
// on u (a . psi) psi_j, whose u-derivative has the extra term (a . psi) psi_j:
//   o_j += U Q1a_j + h (B_j + [j = 1] Q1a_0 + [j = 4] s2 + a_1 P1_j + a_4 P2_j),
//   s2 = <u^2 (a . psi)> = U Q1a_0 + h (B_0 + a_1 P1_0 + a_4 P2_0).
template <typename T>
__host__ __device__ __forceinline__ void stein_u2_add(const T Q1a[5], const T B[5], const T P1[5], const T P2[5], T U,
                                                      T h, const T a[5], T o[5])
{
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += U * Q1a[j] + h * (B[j] + a[1] * P1[j] + a[4] * P2[j]);
    o[1] += h * Q1a[0];
    o[4] += h * (U * Q1a[0] + h * (B[0] + a[1] * P1[0] + a[4] * P2[0]));
}

// <u^k (a_1 . psi u + a_2 . psi v + a_3 . psi w) psi> for the three spatial slopes a (k = 0: the
// compatibility condition's right-hand side; k = 1: the flux) =
// <u^(k+1) psi psi^T> a_1 + <u^k v psi psi^T> a_2 + <u^k w psi psi^T> a_3
template <int k, typename T>
__host__ __device__ __forceinline__ void qadv(const Mom<T> &M, const T a[3][5], T o[5])
{
    Q5<T> Q;
    qmat<k + 1, 0, 0>(M, Q);
    qmul(Q, a[0], o);
    qmat<k, 1, 0>(M, Q);
    qmul_add(Q, a[1], o);
    qmat<k, 0, 1>(M, Q);
    qmul_add(Q, a[2], o);
}

// F_m'(W) d added to f: the Jacobian of the Euler flux F_m along the frame's axis m applied to an
// increment d of the conserved variables (u = (U, V, W), g1 = gamma - 1, k2 = |u|^2 / 2, H = E + p).
template <typename T>
__host__ __device__ __forceinline__ void euler_jac_add(int m, T rho, T ir, const T u[3], T g1, T k2, T H, const T d[5],
                                                       T f[5])
{
    T du[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) du[k] = (d[1 + k] - u[k] * d[0]) * ir;
    const T dp = g1 * (d[4] - (u[0] * d[1] + u[1] * d[2] + u[2] * d[3]) + k2 * d[0]);
    f[0] += d[1 + m];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[1 + k] += d[1 + m] * u[k] + rho * u[m] * du[k];
    f[1 + m] += dp;
    f[4] += du[m] * H + u[m] * (d[4] + dp);
}

// (1/rho) sum_m dF_m/dn_m: the divergence of the Euler fluxes along the frame's axes from the
// derivatives dq[m] of the conserved variables (E = q[4]; gam = (K + 5) / (K + 3)).  For a Maxwellian
// it equals qadv<0> of the slopes <psi psi^T> a_m = dq[m] / rho, since <u_m psi dg/dn_m> = dF_m/dn_m:
// the right-hand side of the compatibility condition that gives the time slope, at a fraction of
// the moment-matrix cost.
template <typename T>
__host__ __device__ __forceinline__ void euler_div(T rho, T ir, T U, T V, T W, T p, T E, T gam, const T dq[3][5], T o[5])
{
    const T u[3] = {U, V, W};
    T f[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int m = 0; m < 3; ++m)
        euler_jac_add(m, rho, ir, u, gam - T(1), T(0.5) * (U * U + V * V + W * W), E + p, dq[m], f);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = f[j] * ir;
}

// Closed-form solution of <psi psi^T> a = b for a Maxwellian (U, V, W, lambda).
template <typename T>
__host__ __device__ __forceinline__ void slope_solve(const T b[5], T U, T V, T W, T lam, T h, T K, T a[5])
{
    // h = 1 / (2 lambda) is the moments' recursion factor and 1 / (K + 3) a constant of the launch:
    // no division of its own
    const T q = U * U + V * V + W * W + (K + T(3)) * h;
    const T R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = b[3] - W * b[0];
    const T R5 = T(2) * b[4] - q * b[0];
    a[4] = T(4) * lam * lam * (T(1) / (K + T(3))) * (R5 - T(2) * (U * R2 + V * R3 + W * R4));
    a[1] = T(2) * lam * R2 - U * a[4];
    a[2] = T(2) * lam * R3 - V * a[4];
    a[3] = T(2) * lam * R4 - W * a[4];
    a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - T(0.5) * a[4] * q;
}

// primitive variables; returns false for a non-physical state
template <typename T>
__host__ __device__ __forceinline__ bool to_prim(const T q[5], T gam, T &rho, T &U, T &V, T &W, T &lam, T &p, T &h)
{
    rho = q[0];
    const T ir = T(1) / rho;
    U = q[1] * ir;
    V = q[2] * ir;
    W = q[3] * ir;
    p = (gam - T(1)) * (q[4] - T(0.5) * rho * (U * U + V * V + W * W));
    lam = rho / (T(2) * p);
    h = p * ir;  // 1 / (2 lambda)
    return rho > T(0) && p > T(0);
}

/*
 * The Gauss-point flux is assembled in three passes so that only one side's
 * moments and slopes are live at a time: side_pass() for the left state
 * (half space u > 0) and for the right state (u < 0) accumulates every
 * half-space moment the flux needs; finish_flux() builds g_0 from them, its
 * slopes, the collision time and both time integrals.  PR selects the
 * Prandtl-number correction, which needs the conserved moments of the
 * time-integrated distribution as well.
 */
template <typename T, bool PR>
struct FluxAcc {
    T q0[5];      // sum_s rho_s <psi>_half            (conserved variables of g_0)
    T bab[3][5];  // sum_s rho_s <a^s_m psi psi>_half   (right-hand sides of the g_0 slopes)
    T Mh[5];      // sum_s rho_s <u psi>_half
    T Mha[5];     // sum_s rho_s <u (a^s . u) psi>_half
    T MhA[5];     // sum_s rho_s <u A^s psi>_half
    T Wha[PR ? 5 : 1];  // sum_s rho_s <(a^s . u) psi>_half
    T WhA[PR ? 5 : 1];  // sum_s rho_s <A^s psi>_half
    T p[2];       // side pressures
};

template <typename T, bool PR>
__host__ __device__ __forceinline__ void acc_zero(FluxAcc<T, PR> &A)
{
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        A.q0[j] = A.Mh[j] = A.Mha[j] = A.MhA[j] = T(0);
        A.bab[0][j] = A.bab[1][j] = A.bab[2][j] = T(0);
        if constexpr (PR) A.Wha[j] = A.WhA[j] = T(0);
    }
}

template <typename T>
__host__ __device__ __forceinline__ void axpy5(T *y, T a, const T *x)
{
#pragma unroll
    for (int j = 0; j < 5; ++j) y[j] += a * x[j];
}

// One side of the interface: sign = +1 for the left state (u > 0), -1 for the right (u < 0).
// SM: the smooth-flow flux needs only the half-space moments of the side state and of its spatial
// slopes (g_0 and its slopes); the side's time slope and non-equilibrium terms are skipped.
template <typename T, bool PR, bool SM = false>
__host__ __device__ __forceinline__ bool side_pass(const T q[5], const T dq[3][5], T sign, const FluxParams<T> &fp,
                                                   FluxAcc<T, PR> &A, int side)
{
    const T K = fp.K;
    T rho, U, V, W, lam, p, h;
    const bool ok = to_prim(q, fp.gamma, rho, U, V, W, lam, p, h);
    A.p[side] = p;
    if (!ok) return false;
    Mom<T> M;
    mom_common(M, V, W, h, K);
    // spatial slopes <a_m> = dQ/dn_m / rho, time slope from <a_1 u + a_2 v + a_3 w + A> = 0
    T a[3][5], Ab[5];
    const T ir = T(1) / rho;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T b[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = dq[m][j] * ir;
        slope_solve(b, U, V, W, lam, h, K, a[m]);
    }
    if constexpr (!SM) {
        T b[5];
        euler_div(rho, ir, U, V, W, p, q[4], fp.gamma, dq, b);
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = -b[j];
        slope_solve(b, U, V, W, lam, h, K, Ab);
    }
    // the half-space moments of u; each moment matrix serves every slope, and the v and w terms of
    // qadv come from the <psi psi^T> and <u psi psi^T> products by Stein's identity
    mom_half_u(M, U, lam, h, sign);
    T t[5], P0[5], t1[5], t2[5];
    Q5<T> Q;
    qmat<0, 0, 0>(M, Q);
#pragma unroll
    for (int j = 0; j < 5; ++j) P0[j] = Q.e[j];
    axpy5(A.q0, rho, P0);
    qmul(Q, a[0], t);
    axpy5(A.bab[0], rho, t);
    qmul(Q, a[1], t1);
    axpy5(A.bab[1], rho, t1);
    qmul(Q, a[2], t2);
    axpy5(A.bab[2], rho, t2);
    if constexpr (SM) return true;
    if constexpr (PR) {
        qmul(Q, Ab, t);
        axpy5(A.WhA, rho, t);
    }
    T P1[5], ma[5], wa[5];  // qadv<1> and (PR) qadv<0> of the half-space set
    qmat<1, 0, 0>(M, Q);
#pragma unroll
    for (int j = 0; j < 5; ++j) P1[j] = Q.e[j];
    axpy5(A.Mh, rho, P1);
    qmul(Q, Ab, t);
    axpy5(A.MhA, rho, t);
    if constexpr (PR) {
        qmul(Q, a[0], wa);
        stein_add<2>(t1, P0, V, h, a[1], wa);
        stein_add<3>(t2, P0, W, h, a[2], wa);
        axpy5(A.Wha, rho, wa);
    }
    qmul(Q, a[1], t1);
    qmul(Q, a[2], t2);
    qmat<2, 0, 0>(M, Q);
    qmul(Q, a[0], ma);
    stein_add<2>(t1, P1, V, h, a[1], ma);
    stein_add<3>(t2, P1, W, h, a[2], ma);
    axpy5(A.Mha, rho, ma);
    return true;
}

/*
 * out[0..4]: flux per unit area at the start of the step, out[5..9]: its time
 * derivative.  Returns false if the interface state is non-physical.
 */
// SM: the time integrals of Eq. flux-2, f = g0 (1 - tau (abar . u + Abar) + Abar t) (with the -tau Abar
// term that the smooth limit of Eq. flux-1 carries), instead of those of Eq. flux-1.
// PL: the viscosity law fp.mu_power can be active (a separate instantiation keeps the fast periodic
// kernels free of its branch and of pow's registers).
template <typename T, bool PR, bool SM = false, bool PL = true>
__host__ __device__ __forceinline__ bool finish_flux(const FluxAcc<T, PR> &A, T dt, const FluxParams<T> &fp, T out[10])
{
    const T K = fp.K;
    T r0, U0, V0, W0, lam0, p0, h0;
    const bool ok = to_prim(A.q0, fp.gamma, r0, U0, V0, W0, lam0, p0, h0);
    T ab[3][5];
    const T ir0 = T(1) / r0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T b[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = A.bab[m][j] * ir0;
        slope_solve(b, U0, V0, W0, lam0, h0, K, ab[m]);
    }
    // qadv<0>(G, ab): the negated right-hand side of g_0's time slope Ab (<psi psi^T> Ab = -pv)
    T pv[5];
    euler_div(r0, ir0, U0, V0, W0, p0, A.q0[4], fp.gamma, A.bab, pv);
    // collision time
    const T dp = (A.p[0] - A.p[1]) / (A.p[0] + A.p[1]);
    const T jump = (dp < T(0) ? -dp : dp) * dt;
    // viscosity at the interface temperature T0 = p0 / rho0 = 1 / (2 lambda0) (power law when asked)
    T mu = fp.mu;
    if constexpr (PL)
        if (fp.viscous && fp.mu_power != T(0)) mu *= pow_t(h0 * fp.iT_ref, fp.mu_power);
    const T tau = fp.viscous ? mu / p0 + fp.tau_C * jump : fp.tau_eps * dt + fp.tau_C * jump;
    // <u psi> of g_0 is its Euler flux along n1 over r0, and <u (Ab . psi) psi> that flux's Jacobian
    // applied to <psi psi^T> Ab = -pv (d/dt of <u psi g_0>); with PR, <psi> = W_0 / r0 and
    // <(Ab . psi) psi> = -pv
    T M0[5], Ma[5] = {T(0), T(0), T(0), T(0), T(0)}, MA[5] = {T(0), T(0), T(0), T(0), T(0)};
    {
        const T E0 = A.q0[4];
        M0[0] = U0;
        M0[1] = U0 * U0 + h0;
        M0[2] = U0 * V0;
        M0[3] = U0 * W0;
        M0[4] = U0 * (E0 * ir0 + h0);
        const T u0[3] = {U0, V0, W0};
        T npv[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) npv[j] = -pv[j];
        euler_jac_add(0, r0, ir0, u0, fp.gamma - T(1), T(0.5) * (U0 * U0 + V0 * V0 + W0 * W0), E0 + p0, npv, MA);
    }
    // <u (ab . u psi) psi> = qadv<1> of g_0 by Stein's identity in u, v and w (g_0 is Gaussian in
    // each), from <psi psi^T> ab[m] = bab[m] / r0, <psi> = W_0 / r0, <u psi> = M0 and <u^2 psi>
    {
        T Pw[5], P2[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) Pw[j] = A.q0[j] * ir0;
#pragma unroll
        for (int j = 0; j < 5; ++j) P2[j] = U0 * M0[j] + h0 * Pw[j];
        P2[1] += h0 * U0;
        P2[4] += h0 * (U0 * U0 + h0);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            T B[5], Q1a[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int j = 0; j < 5; ++j) B[j] = A.bab[m][j] * ir0;
            stein_add<1>(B, Pw, U0, h0, ab[m], Q1a);  // <u (ab[m] . psi) psi>
            if (m == 0)
                stein_u2_add(Q1a, B, M0, P2, U0, h0, ab[0], Ma);
            else if (m == 1)
                stein_add<2>(Q1a, M0, V0, h0, ab[1], Ma);
            else
                stein_add<3>(Q1a, M0, W0, h0, ab[2], Ma);
        }
    }
    T W0m[PR ? 5 : 1], Wam[PR ? 5 : 1], WAm[PR ? 5 : 1];
    if constexpr (PR) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            W0m[j] = A.q0[j] * ir0;
            Wam[j] = pv[j];
            WAm[j] = -pv[j];
        }
    }
    T Fd[2][5];
    const T itau = T(1) / tau;
    // exp(-dt / tau) = eta^2 and 1 - exp(-dt / tau) = om (1 + eta) for eta = exp(-dt / (2 tau)), om = 1 - eta
    T eta_h = T(0), om_h = T(0);
    if constexpr (!SM) {
        eta_h = exp_t(T(-0.5) * dt * itau);
        om_h = -expm1_t(T(-0.5) * dt * itau);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T d = s == 0 ? T(0.5) * dt : dt;
        T T1, T2, T3, T4 = T(0), T5 = T(0);
        if constexpr (SM) {
            T1 = d;
            T2 = -tau * d;
            T3 = T(0.5) * d * d - tau * d;
        } else {
            const T eta = s == 0 ? eta_h : eta_h * eta_h;
            const T om = s == 0 ? om_h : om_h * (T(1) + eta_h);
            T1 = d - tau * om;
            T2 = T(2) * tau * tau * om - tau * d * (T(1) + eta);
            T3 = T(0.5) * d * d - tau * d + tau * tau * om;
            T4 = tau * om;
            T5 = T(2) * tau * tau * om - tau * d * eta;
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            Fd[s][j] = r0 * (T1 * M0[j] + T2 * Ma[j] + T3 * MA[j]);
            if constexpr (!SM) Fd[s][j] += T4 * A.Mh[j] - T5 * A.Mha[j] - tau * T4 * A.MhA[j];
        }
        if constexpr (PR) {
            T Wv[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                Wv[j] = r0 * (T1 * W0m[j] + T2 * Wam[j] + T3 * WAm[j]);
                if constexpr (!SM) Wv[j] += T4 * A.q0[j] - T5 * A.Wha[j] - tau * T4 * A.WhA[j];
            }
            const T *F = Fd[s];
            const T U2 = U0 * U0 + V0 * V0 + W0 * W0;
            // heat flux about the interface velocity of the time-integrated distribution (times 2)
            const T q2 = T(2) * F[4] - T(2) * (U0 * F[1] + V0 * F[2] + W0 * F[3]) + U2 * F[0] -
                         U0 * (T(2) * Wv[4] - T(2) * (U0 * Wv[1] + V0 * Wv[2] + W0 * Wv[3]) + U2 * Wv[0]);
            Fd[s][4] += (T(1) / fp.Pr - T(1)) * T(0.5) * q2;
        }
    }
    const T idt = T(1) / dt;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        out[j] = (T(4) * Fd[0][j] - Fd[1][j]) * idt;
        out[5 + j] = T(4) * (Fd[1][j] - T(2) * Fd[0][j]) * idt * idt;
    }
    return ok;
}

/*
 * Gauss-point flux from the two local-frame states and their n1, n2, n3
 * derivatives.  Returns false if a state (left, right or interface) is
 * non-physical; the output is then zero.
 */
template <typename T, bool PR, bool SM = false>
__host__ __device__ bool gp_flux(const T ql[5], const T dql[3][5], const T qr[5], const T dqr[3][5], T dt,
                                 const FluxParams<T> &fp, T out[10])
{
    FluxAcc<T, PR> A;
    acc_zero(A);
    bool ok = side_pass<T, PR, SM>(ql, dql, T(1), fp, A, 0);
    ok = side_pass<T, PR, SM>(qr, dqr, T(-1), fp, A, 1) && ok;
    if (!ok) {
#pragma unroll
        for (int j = 0; j < 10; ++j) out[j] = T(0);
        return false;
    }
    return finish_flux<T, PR, SM>(A, dt, fp, out);
}

// Local frame at a Gauss point: n1 = unit weighted vector area; e = the coordinate
// axis with the smallest |n1 . e| (lowest index on ties), n2 = unit(e - (e.n1) n1),
// n3 = n1 x n2.  Returns |vector area|.
template <typename T>
__host__ __device__ __forceinline__ T local_frame(T vx, T vy, T vz, T n[3][3])
{
    const T area = sqrt_t(vx * vx + vy * vy + vz * vz);
    const T ia = T(1) / area;
    n[0][0] = vx * ia;
    n[0][1] = vy * ia;
    n[0][2] = vz * ia;
    const T ax = n[0][0] < T(0) ? -n[0][0] : n[0][0];
    const T ay = n[0][1] < T(0) ? -n[0][1] : n[0][1];
    const T az = n[0][2] < T(0) ? -n[0][2] : n[0][2];
    int e = 0;
    T best = ax;
    if (ay < best) {
        e = 1;
        best = ay;
    }
    if (az < best) e = 2;
    T t[3] = {T(0), T(0), T(0)};
    t[e] = T(1);
    const T d = n[0][e];
    t[0] = t[0] - d * n[0][0];
    t[1] = t[1] - d * n[0][1];
    t[2] = t[2] - d * n[0][2];
    const T it = T(1) / sqrt_t(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    n[1][0] = t[0] * it;
    n[1][1] = t[1] * it;
    n[1][2] = t[2] * it;
    n[2][0] = n[0][1] * n[1][2] - n[0][2] * n[1][1];
    n[2][1] = n[0][2] * n[1][0] - n[0][0] * n[1][2];
    n[2][2] = n[0][0] * n[1][1] - n[0][1] * n[1][0];
    return area;
}

// Value and gradient at offset (X, Y, Z) of one cell's per-component quadratic, rotated
// into the local frame (momentum components and derivative directions).
template <typename T>
__host__ __device__ __forceinline__ void side_state(const T *__restrict__ c, const double *q0, T X, T Y, T Z,
                                                    const T n[3][3], T q[5], T dq[3][5])
{
    T v[5], g[5][3];
    const T XX = X * X, XY = X * Y, XZ = X * Z, YY = Y * Y, YZ = Y * Z, ZZ = Z * Z;
#pragma unroll
    for (int comp = 0; comp < 5; ++comp) {
        const T *cc = c + 10 * comp;
        const T lin = cc[1] * X + cc[2] * Y + cc[3] * Z;
        const T qua = cc[4] * XX + cc[5] * XY + cc[6] * XZ + cc[7] * YY + cc[8] * YZ + cc[9] * ZZ;
        if constexpr (sizeof(T) == 8)
            v[comp] = cc[0] + lin + qua;
        else
            v[comp] = (T)(q0[comp] + (double)(cc[0] + lin + qua));
        g[comp][0] = cc[1] + T(2) * cc[4] * X + cc[5] * Y + cc[6] * Z;
        g[comp][1] = cc[2] + cc[5] * X + T(2) * cc[7] * Y + cc[8] * Z;
        g[comp][2] = cc[3] + cc[6] * X + cc[8] * Y + T(2) * cc[9] * Z;
    }
    q[0] = v[0];
    q[4] = v[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) q[1 + k] = v[1] * n[k][0] + v[2] * n[k][1] + v[3] * n[k][2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T dn[5];
#pragma unroll
        for (int cc = 0; cc < 5; ++cc) dn[cc] = g[cc][0] * n[m][0] + g[cc][1] * n[m][1] + g[cc][2] * n[m][2];
        dq[m][0] = dn[0];
        dq[m][4] = dn[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) dq[m][1 + k] = dn[1] * n[k][0] + dn[2] * n[k][1] + dn[3] * n[k][2];
    }
}

/*
 * All the work of one face Gauss point: states on both sides from their
 * quadratics (cl, cr: [5][10]) at offsets geo[0..2] (owner) and geo[3..5]
 * (neighbour), frame from the weighted vector area geo[6..8], the BGK flux,
 * rotation back to global axes and weighting (Eq. flux-qud).  out: the Gauss
 * point's (Fbar0, Fbar1) contribution to the face, owner -> neighbour.
 * ql0, qr0: FP64 cell averages (used by the FP32 variant only).
 */
// Copy one cell's 50 coefficients with 16-byte loads (the per-cell block is 16-byte aligned).
template <typename T>
__host__ __device__ __forceinline__ void load_cell(const T *__restrict__ src, T dst[50])
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(T) == 8) {
        const double2 *s2 = reinterpret_cast<const double2 *>(src);
#pragma unroll
        for (int q = 0; q < 25; ++q) {
            const double2 v = s2[q];
            dst[2 * q] = v.x;
            dst[2 * q + 1] = v.y;
        }
    } else {
        const float2 *s2 = reinterpret_cast<const float2 *>(src);  // 200-byte blocks: 8-byte alignment
#pragma unroll
        for (int q = 0; q < 25; ++q) {
            const float2 v = s2[q];
            dst[2 * q] = v.x;
            dst[2 * q + 1] = v.y;
        }
    }
#else
    for (int q = 0; q < 50; ++q) dst[q] = src[q];
#endif
}

// The state beyond a reflective wall at a Gauss point: the mirror image of the inner one.  In the
// local frame whose n1 is the wall normal the image negates the normal momentum, the normal
// derivatives of the other variables and the tangential derivatives of the normal momentum.
template <typename T>
__host__ __device__ __forceinline__ void wall_mirror(const T q[5], const T dq[3][5], T qr[5], T dqr[3][5])
{
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const T s = j == 1 ? T(-1) : T(1);
        qr[j] = s * q[j];
        dqr[0][j] = -s * dq[0][j];
        dqr[1][j] = s * dq[1][j];
        dqr[2][j] = s * dq[2][j];
    }
}

// The state beyond box plane `plane` at a Gauss point on it, in the local frame whose n1 is the plane's
// outward normal: its condition applied to the inner state (q, dq: value and derivatives along n1, n2,
// n3), the derivatives along n1 negated (the mirror), the far field's ghost uniform.
template <typename T>
__host__ __device__ __forceinline__ void bc_gauss_point(const FluxParams<T> &fp, int plane, const T n[3][3], const T q[5],
                                                        const T dq[3][5], T qr[5], T dqr[3][5])
{
    const int type = fp.bc_type[plane];
    if (type == kBcSlip) {
        wall_mirror(q, dq, qr, dqr);
        return;
    }
    if (type == kBcExtrapolate) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            qr[j] = q[j];
            dqr[0][j] = -dq[0][j];
            dqr[1][j] = dq[1][j];
            dqr[2][j] = dq[2][j];
        }
        return;
    }
    const T g1 = fp.gamma - T(1);
    const T rho = q[0], ir = T(1) / rho;
    const T U[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const T u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const T p = g1 * (q[4] - T(0.5) * rho * u2);
    T rb, Ub[3];
    if (type == kBcFarField) {
        T Uf[3], pb;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Uf[k] = fp.bc_far[plane][1] * n[k][0] + fp.bc_far[plane][2] * n[k][1] + fp.bc_far[plane][3] * n[k][2];
        farfield_frame<T>(fp.gamma, rho, U, p, fp.bc_far[plane][0], Uf, fp.bc_far[plane][4], rb, Ub, pb);
        qr[0] = rb;
#pragma unroll
        for (int k = 0; k < 3; ++k) qr[1 + k] = rb * Ub[k];
        qr[4] = pb / g1 + T(0.5) * rb * (Ub[0] * Ub[0] + Ub[1] * Ub[1] + Ub[2] * Ub[2]);
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int j = 0; j < 5; ++j) dqr[m][j] = T(0);
        return;
    }
    // no-slip: the wall velocity in the local frame, U -> 2 u_w - U, p kept; rho kept (adiabatic) or
    // rho -> p / (2 T_w - p / rho) (isothermal)
#pragma unroll
    for (int k = 0; k < 3; ++k)
        Ub[k] = T(2) * (fp.bc_uw[plane][0] * n[k][0] + fp.bc_uw[plane][1] * n[k][1] + fp.bc_uw[plane][2] * n[k][2]) - U[k];
    const bool iso = type == kBcIsothermal;
    const T Tg = iso ? T(2) * fp.bc_Tw[plane] - p * ir : T(1);
    rb = iso ? p / Tg : rho;
    const T ub2 = Ub[0] * Ub[0] + Ub[1] * Ub[1] + Ub[2] * Ub[2];
    qr[0] = rb;
#pragma unroll
    for (int k = 0; k < 3; ++k) qr[1 + k] = rb * Ub[k];
    qr[4] = p / g1 + T(0.5) * rb * ub2;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        // derivatives along n_m of the inner primitives, then of the ghost's
        const T dr = dq[m][0];
        T dU[3], udu = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dU[k] = (dq[m][1 + k] - U[k] * dr) * ir;
            udu += U[k] * dU[k];
        }
        const T dp = g1 * (dq[m][4] - T(0.5) * u2 * dr - rho * udu);
        const T drb = iso ? (dp + rb * (dp - p * ir * dr) * ir) / Tg : dr;
        T ubdu = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) ubdu -= Ub[k] * dU[k];
        const T s = m == 0 ? T(-1) : T(1);  // the mirror across the plane
        dqr[m][0] = s * drb;
#pragma unroll
        for (int k = 0; k < 3; ++k) dqr[m][1 + k] = s * (Ub[k] * drb - rb * dU[k]);
        dqr[m][4] = s * (dp / g1 + T(0.5) * ub2 * drb + rb * ubdu);
    }
}

// With fp.fallback: a side state with rho <= 0 or p <= 0, or with rho or p at most fp.floor times
// that of its cell's average qav (FP64, global frame), becomes qav in the local frame with zero
// slopes.  Returns whether it did.
template <typename T>
__host__ __device__ __forceinline__ bool fallback_side(const FluxParams<T> &fp, const double *qav, const T n[3][3],
                                                       T q[5], T dq[3][5])
{
    if (!fp.fallback) return false;
    const T p = (fp.gamma - T(1)) * (q[4] - T(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
    double rmin = 0.0, pmin = 0.0;
    if (fp.floor > 0.0) {
        const double pav = ((double)fp.gamma - 1.0) * (qav[4] - 0.5 * (qav[1] * qav[1] + qav[2] * qav[2] + qav[3] * qav[3]) / qav[0]);
        rmin = fp.floor * qav[0];
        pmin = fp.floor * pav;
    }
    if ((double)q[0] > rmin && (double)p > pmin && q[0] > T(0) && p > T(0)) return false;
    const T v1 = (T)qav[1], v2 = (T)qav[2], v3 = (T)qav[3];
    q[0] = (T)qav[0];
    q[4] = (T)qav[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) q[1 + k] = v1 * n[k][0] + v2 * n[k][1] + v3 * n[k][2];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int j = 0; j < 5; ++j) dq[m][j] = T(0);
    return true;
}

// The flux of one Gauss point of an interior face, each cell's coefficients fetched by a loader
// (load_l(T[50]), load_r(T[50])) just before that side's state is formed; the neighbour's side
// is taken first, so a caller can have the owner's coefficients in flight meanwhile (ql0, qr0:
// the FP64 cell averages that FP32 coefficients exclude; unused in FP64).  The arithmetic of
// face_gp without walls or the fallback, up to the order in which the two sides' moments are
// added to the accumulators.
template <typename T, bool PR, bool SM, typename LoadL, typename LoadR>
__host__ __device__ __forceinline__ bool face_gp_pre(LoadL load_l, LoadR load_r, const double *ql0,
                                                     const double *qr0, const T geo[9], T dt,
                                                     const FluxParams<T> &fp, T out[10])
{
    T n3[3][3];
    const T area = local_frame(geo[6], geo[7], geo[8], n3);
    FluxAcc<T, PR> A;
    acc_zero(A);
    bool ok;
    {
        T q[5], dq[3][5], cr[50];
        load_r(cr);
        side_state(cr, qr0, geo[3], geo[4], geo[5], n3, q, dq);
        ok = side_pass<T, PR, SM>(q, dq, T(-1), fp, A, 1);
    }
    {
        T q[5], dq[3][5], cl[50];
        load_l(cl);
        side_state(cl, ql0, geo[0], geo[1], geo[2], n3, q, dq);
        ok = side_pass<T, PR, SM>(q, dq, T(1), fp, A, 0) && ok;
    }
    T F[10];
    if (ok) {
        ok = finish_flux<T, PR, SM, false>(A, dt, fp, F);
    } else {
#pragma unroll
        for (int j = 0; j < 10; ++j) F[j] = T(0);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T *Fl = F + 5 * s;
        out[5 * s] = area * Fl[0];
        out[5 * s + 4] = area * Fl[4];
#pragma unroll
        for (int q = 0; q < 3; ++q) out[5 * s + 1 + q] = area * (Fl[1] * n3[0][q] + Fl[2] * n3[1][q] + Fl[3] * n3[2][q]);
    }
    return ok;
}

// EXT: walls, the first-order fallback and the viscosity power law can occur; without it cr_g is never
// null and fp.fallback and fp.mu_power are ignored.  With it, cr_g == nullptr means the face is a
// reflective wall and the right state is the mirror of the left one.  ql0, qr0: the two cells' FP64 averages (read for FP32 coefficients and for
// the fallback); nfb counts the sides that fell back.
template <typename T, bool PR, bool EXT, bool SM = false>
__host__ __device__ __forceinline__ bool face_gp(const T *__restrict__ cl_g, const T *__restrict__ cr_g, const double *ql0,
                                                 const double *qr0, const T geo[9], T dt, const FluxParams<T> &fp,
                                                 T out[10], int &nfb, int wall_plane = 0)
{
    T n3[3][3];
    const T area = local_frame(geo[6], geo[7], geo[8], n3);
    FluxAcc<T, PR> A;
    acc_zero(A);
    bool ok;
    {
        T q[5], dq[3][5], cl[50];
        load_cell(cl_g, cl);
        side_state(cl, ql0, geo[0], geo[1], geo[2], n3, q, dq);
        if (EXT) nfb += fallback_side(fp, ql0, n3, q, dq);
        ok = side_pass<T, PR, SM>(q, dq, T(1), fp, A, 0);
    }
    {
        T q[5], dq[3][5], cr[50];
        if constexpr (!EXT) {
            load_cell(cr_g, cr);
            side_state(cr, qr0, geo[3], geo[4], geo[5], n3, q, dq);
        } else if (cr_g) {
            load_cell(cr_g, cr);
            side_state(cr, qr0, geo[3], geo[4], geo[5], n3, q, dq);
            nfb += fallback_side(fp, qr0, n3, q, dq);
        } else {
            T qi[5], dqi[3][5];
            load_cell(cl_g, cr);
            side_state(cr, ql0, geo[0], geo[1], geo[2], n3, qi, dqi);
            nfb += fallback_side(fp, ql0, n3, qi, dqi);  // the ghost of a fallen-back side falls back too
            bc_gauss_point(fp, wall_plane, n3, qi, dqi, q, dq);
        }
        ok = side_pass<T, PR, SM>(q, dq, T(-1), fp, A, 1) && ok;
    }
    T F[10];
    if (ok) {
        ok = finish_flux<T, PR, SM, EXT>(A, dt, fp, F);
    } else {
#pragma unroll
        for (int j = 0; j < 10; ++j) F[j] = T(0);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T *Fl = F + 5 * s;
        out[5 * s] = area * Fl[0];
        out[5 * s + 4] = area * Fl[4];
#pragma unroll
        for (int q = 0; q < 3; ++q) out[5 * s + 1 + q] = area * (Fl[1] * n3[0][q] + Fl[2] * n3[1][q] + Fl[3] * n3[2][q]);
    }
    return ok;
}

}  // namespace gks
