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

namespace gks {

template <typename T>
struct FluxParams {
    T gamma, K, mu, Pr, tau_eps, tau_C;
    int viscous;
};

// Moments <u^k> (k <= 6), <v^k>, <w^k> (k <= 5), <s^2>, <s^4> of one normalised Maxwellian.
template <typename T>
struct Mom {
    T u[7], v[6], w[6], s1, s2;
};

template <typename T>
__device__ __forceinline__ void recur7(T *m, T U, T h)  // h = 1 / (2 lambda)
{
#pragma unroll
    for (int k = 0; k + 2 < 7; ++k) m[k + 2] = U * m[k + 1] + T(k + 1) * h * m[k];
}

template <typename T>
__device__ __forceinline__ void recur6(T *m, T U, T h)
{
#pragma unroll
    for (int k = 0; k + 2 < 6; ++k) m[k + 2] = U * m[k + 1] + T(k + 1) * h * m[k];
}

template <typename T>
__device__ __forceinline__ T erfc_t(T x);
template <>
__device__ __forceinline__ double erfc_t<double>(double x) { return erfc(x); }
template <>
__device__ __forceinline__ float erfc_t<float>(float x) { return erfcf(x); }
template <typename T>
__device__ __forceinline__ T exp_t(T x);
template <>
__device__ __forceinline__ double exp_t<double>(double x) { return exp(x); }
template <>
__device__ __forceinline__ float exp_t<float>(float x) { return expf(x); }
template <typename T>
__device__ __forceinline__ T expm1_t(T x);
template <>
__device__ __forceinline__ double expm1_t<double>(double x) { return expm1(x); }
template <>
__device__ __forceinline__ float expm1_t<float>(float x) { return expm1f(x); }
template <typename T>
__device__ __forceinline__ T sqrt_t(T x);
template <>
__device__ __forceinline__ double sqrt_t<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float sqrt_t<float>(float x) { return sqrtf(x); }

// Full-space v, w, internal moments (shared by full and half-space sets of one state).
template <typename T>
__device__ __forceinline__ void mom_common(Mom<T> &m, T V, T W, T lam, T K)
{
    const T h = T(0.5) / lam;
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
__device__ __forceinline__ void mom_full_u(Mom<T> &m, T U, T lam)
{
    m.u[0] = T(1);
    m.u[1] = U;
    recur7(m.u, U, T(0.5) / lam);
}

// sign = +1: u > 0, -1: u < 0
template <typename T>
__device__ __forceinline__ void mom_half_u(Mom<T> &m, T U, T lam, T sign)
{
    const T sl = sqrt_t(lam);
    const T e = exp_t(-lam * U * U) / (T(2) * sqrt_t(T(M_PI) * lam));
    m.u[0] = T(0.5) * erfc_t(-sign * sl * U);
    m.u[1] = U * m.u[0] + sign * e;
    recur7(m.u, U, T(0.5) / lam);
}

// <u^k v^l w^m psi>
template <int k, int l, int n, typename T>
__device__ __forceinline__ void P(const Mom<T> &M, T o[5])
{
    const T vw = M.v[l] * M.w[n];
    const T base = M.u[k] * vw;
    o[0] = base;
    o[1] = M.u[k + 1] * vw;
    o[2] = M.u[k] * M.v[l + 1] * M.w[n];
    o[3] = M.u[k] * M.v[l] * M.w[n + 1];
    o[4] = T(0.5) * (M.u[k + 2] * vw + M.u[k] * M.v[l + 2] * M.w[n] + M.u[k] * M.v[l] * M.w[n + 2] + base * M.s1);
}

// <u^k v^l w^m s^2 psi>
template <int k, int l, int n, typename T>
__device__ __forceinline__ void Ps(const Mom<T> &M, T o[5])
{
    const T vw = M.v[l] * M.w[n];
    const T base = M.u[k] * vw;
    o[0] = base * M.s1;
    o[1] = M.u[k + 1] * vw * M.s1;
    o[2] = M.u[k] * M.v[l + 1] * M.w[n] * M.s1;
    o[3] = M.u[k] * M.v[l] * M.w[n + 1] * M.s1;
    o[4] = T(0.5) * ((M.u[k + 2] * vw + M.u[k] * M.v[l + 2] * M.w[n] + M.u[k] * M.v[l] * M.w[n + 2]) * M.s1 +
                     base * M.s2);
}

// <u^k v^l w^m (a . psi) psi> for a slope a = (a1, a2, a3, a4, a5)
template <int k, int l, int n, typename T>
__device__ __forceinline__ void Pa(const Mom<T> &M, const T a[5], T o[5])
{
    T t[5];
    P<k, l, n>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = a[0] * t[j];
    P<k + 1, l, n>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += a[1] * t[j];
    P<k, l + 1, n>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += a[2] * t[j];
    P<k, l, n + 1>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += a[3] * t[j];
    T q[5];
    P<k + 2, l, n>(M, q);
    P<k, l + 2, n>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) q[j] += t[j];
    P<k, l, n + 2>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) q[j] += t[j];
    Ps<k, l, n>(M, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += T(0.5) * a[4] * (q[j] + t[j]);
}

// <u^k (a1.psi u + a2.psi v + a3.psi w) psi> for k = 0 (compatibility) or 1 (flux)
template <int k, typename T>
__device__ __forceinline__ void Padv(const Mom<T> &M, const T a[3][5], T o[5])
{
    T t[5];
    Pa<k + 1, 0, 0>(M, a[0], o);
    Pa<k, 1, 0>(M, a[1], t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += t[j];
    Pa<k, 0, 1>(M, a[2], t);
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] += t[j];
}

// Closed-form solution of <psi psi^T> a = b for a Maxwellian (U, V, W, lambda).
template <typename T>
__device__ __forceinline__ void slope_solve(const T b[5], T U, T V, T W, T lam, T K, T a[5])
{
    const T q = U * U + V * V + W * W + (K + T(3)) / (T(2) * lam);
    const T R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = b[3] - W * b[0];
    const T R5 = T(2) * b[4] - q * b[0];
    a[4] = T(4) * lam * lam / (K + T(3)) * (R5 - T(2) * (U * R2 + V * R3 + W * R4));
    a[1] = T(2) * lam * R2 - U * a[4];
    a[2] = T(2) * lam * R3 - V * a[4];
    a[3] = T(2) * lam * R4 - W * a[4];
    a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - T(0.5) * a[4] * q;
}

// primitive variables; returns false for a non-physical state
template <typename T>
__device__ __forceinline__ bool to_prim(const T q[5], T gam, T &rho, T &U, T &V, T &W, T &lam, T &p)
{
    rho = q[0];
    const T ir = T(1) / rho;
    U = q[1] * ir;
    V = q[2] * ir;
    W = q[3] * ir;
    p = (gam - T(1)) * (q[4] - T(0.5) * rho * (U * U + V * V + W * W));
    lam = rho / (T(2) * p);
    return rho > T(0) && p > T(0);
}

/*
 * out[0..4]: flux per unit area at the start of the step, out[5..9]: its time
 * derivative.  Returns false if a state (left, right or interface) is non-physical.
 */
template <typename T>
__device__ bool gp_flux(const T ql[5], const T dql[3][5], const T qr[5], const T dqr[3][5], T dt,
                        const FluxParams<T> &fp, T out[10])
{
    const T K = fp.K;
    T rl, Ul, Vl, Wl, laml, pl, rr, Ur, Vr, Wr, lamr, pr;
    bool ok = to_prim(ql, fp.gamma, rl, Ul, Vl, Wl, laml, pl);
    ok = to_prim(qr, fp.gamma, rr, Ur, Vr, Wr, lamr, pr) && ok;
    if (!ok) {
#pragma unroll
        for (int j = 0; j < 10; ++j) out[j] = T(0);
        return false;
    }
    Mom<T> Lf, Lh, Rf, Rh;
    mom_common(Lf, Vl, Wl, laml, K);
    mom_full_u(Lf, Ul, laml);
    Lh = Lf;
    mom_half_u(Lh, Ul, laml, T(1));
    mom_common(Rf, Vr, Wr, lamr, K);
    mom_full_u(Rf, Ur, lamr);
    Rh = Rf;
    mom_half_u(Rh, Ur, lamr, T(-1));

    // interface equilibrium
    T q0[5], t5[5];
    P<0, 0, 0>(Lh, q0);
    P<0, 0, 0>(Rh, t5);
#pragma unroll
    for (int j = 0; j < 5; ++j) q0[j] = rl * q0[j] + rr * t5[j];
    T r0, U0, V0, W0, lam0, p0;
    ok = to_prim(q0, fp.gamma, r0, U0, V0, W0, lam0, p0);
    Mom<T> G;
    mom_common(G, V0, W0, lam0, K);
    mom_full_u(G, U0, lam0);

    // spatial slopes on both sides
    T al[3][5], ar[3][5];
    const T irl = T(1) / rl, irr = T(1) / rr;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T b[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = dql[m][j] * irl;
        slope_solve(b, Ul, Vl, Wl, laml, K, al[m]);
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = dqr[m][j] * irr;
        slope_solve(b, Ur, Vr, Wr, lamr, K, ar[m]);
    }
    // time slopes from compatibility
    T Al[5], Ar[5];
    {
        T b[5];
        Padv<0>(Lf, al, b);
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = -b[j];
        slope_solve(b, Ul, Vl, Wl, laml, K, Al);
        Padv<0>(Rf, ar, b);
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = -b[j];
        slope_solve(b, Ur, Vr, Wr, lamr, K, Ar);
    }
    // equilibrium slopes
    T ab[3][5], Ab[5];
    const T ir0 = T(1) / r0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T b[5], c[5];
        Pa<0, 0, 0>(Lh, al[m], b);
        Pa<0, 0, 0>(Rh, ar[m], c);
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = (rl * b[j] + rr * c[j]) * ir0;
        slope_solve(b, U0, V0, W0, lam0, K, ab[m]);
    }
    {
        T b[5];
        Padv<0>(G, ab, b);
#pragma unroll
        for (int j = 0; j < 5; ++j) b[j] = -b[j];
        slope_solve(b, U0, V0, W0, lam0, K, Ab);
    }
    // collision time
    const T dp = (pl - pr) / (pl + pr);
    const T jump = (dp < T(0) ? -dp : dp) * dt;
    const T tau = fp.viscous ? fp.mu / p0 + fp.tau_C * jump : fp.tau_eps * dt + fp.tau_C * jump;

    // flux moments of every term (shared by both time integrals)
    T M0[5], Ma[5], MA[5], Mh[5], Mha[5], MhA[5];
    {
        T x[5], y[5];
        P<1, 0, 0>(G, M0);
        Padv<1>(G, ab, Ma);
        Pa<1, 0, 0>(G, Ab, MA);
        P<1, 0, 0>(Lh, x);
        P<1, 0, 0>(Rh, y);
#pragma unroll
        for (int j = 0; j < 5; ++j) Mh[j] = rl * x[j] + rr * y[j];
        Padv<1>(Lh, al, x);
        Padv<1>(Rh, ar, y);
#pragma unroll
        for (int j = 0; j < 5; ++j) Mha[j] = rl * x[j] + rr * y[j];
        Pa<1, 0, 0>(Lh, Al, x);
        Pa<1, 0, 0>(Rh, Ar, y);
#pragma unroll
        for (int j = 0; j < 5; ++j) MhA[j] = rl * x[j] + rr * y[j];
    }
    const bool prandtl = fp.viscous && fp.Pr != T(1);
    T W0m[5], Wam[5], WAm[5], Whm[5], Wham[5], WhAm[5];
    if (prandtl) {
        T x[5], y[5];
        P<0, 0, 0>(G, W0m);
        Padv<0>(G, ab, Wam);
        Pa<0, 0, 0>(G, Ab, WAm);
        P<0, 0, 0>(Lh, x);
        P<0, 0, 0>(Rh, y);
#pragma unroll
        for (int j = 0; j < 5; ++j) Whm[j] = rl * x[j] + rr * y[j];
        Padv<0>(Lh, al, x);
        Padv<0>(Rh, ar, y);
#pragma unroll
        for (int j = 0; j < 5; ++j) Wham[j] = rl * x[j] + rr * y[j];
        Pa<0, 0, 0>(Lh, Al, x);
        Pa<0, 0, 0>(Rh, Ar, y);
#pragma unroll
        for (int j = 0; j < 5; ++j) WhAm[j] = rl * x[j] + rr * y[j];
    }
    T Fd[2][5];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T d = s == 0 ? T(0.5) * dt : dt;
        const T eta = exp_t(-d / tau);
        const T om = -expm1_t(-d / tau);
        const T T1 = d - tau * om;
        const T T2 = T(2) * tau * tau * om - tau * d * (T(1) + eta);
        const T T3 = T(0.5) * d * d - tau * d + tau * tau * om;
        const T T4 = tau * om;
        const T T5 = T(2) * tau * tau * om - tau * d * eta;
#pragma unroll
        for (int j = 0; j < 5; ++j)
            Fd[s][j] = r0 * (T1 * M0[j] + T2 * Ma[j] + T3 * MA[j]) + T4 * Mh[j] - T5 * Mha[j] - tau * T4 * MhA[j];
        if (prandtl) {
            T Wv[5];
#pragma unroll
            for (int j = 0; j < 5; ++j)
                Wv[j] = r0 * (T1 * W0m[j] + T2 * Wam[j] + T3 * WAm[j]) + T4 * Whm[j] - T5 * Wham[j] -
                        tau * T4 * WhAm[j];
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

}  // namespace gks
