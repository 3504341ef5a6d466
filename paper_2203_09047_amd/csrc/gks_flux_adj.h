// Reverse mode (vector-Jacobian products) of the Gauss-point gas-kinetic flux.
//
// Each function below is the hand-written adjoint of the forward function of
// the same name in gks_flux.h: given the cotangent of the forward outputs it
// accumulates the cotangents of the forward inputs ("x_b" is the cotangent of
// x).  Forward intermediates are recomputed, never stored.  The time step is a
// constant of the step (frozen), and |x| has derivative sign(x) with sign(0) = 0.
#pragma once

#include "gks_flux.h"

namespace gks {

template <typename T>
__host__ __device__ __forceinline__ T sgn_t(T x)
{
    return x > T(0) ? T(1) : (x < T(0) ? T(-1) : T(0));
}

// cotangents of one set of normalised Maxwellian moments
template <typename T>
struct MomB {
    T u[7], v[6], w[6], s1, s2;
};

template <typename T>
__host__ __device__ __forceinline__ void momb_zero(MomB<T> &B)
{
#pragma unroll
    for (int k = 0; k < 7; ++k) B.u[k] = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) B.v[k] = B.w[k] = T(0);
    B.s1 = B.s2 = T(0);
}

// reverse of m[k+2] = U m[k+1] + (k+1) h m[k] for k = NK-3 .. 0
template <int NK, typename T>
__host__ __device__ __forceinline__ void recur_b(const T *m, T *mb, T U, T h, T &Ub, T &hb)
{
#pragma unroll
    for (int k = NK - 3; k >= 0; --k) {
        const T g = mb[k + 2];
        mb[k + 1] += U * g;
        Ub += m[k + 1] * g;
        mb[k] += T(k + 1) * h * g;
        hb += T(k + 1) * m[k] * g;
    }
}

// reverse of mom_common: v, w, s moments -> V, W, lambda (h = 1 / (2 lambda): dh/dlambda = -2 h^2)
template <typename T>
__host__ __device__ __forceinline__ void mom_common_b(const Mom<T> &M, MomB<T> &B, T V, T W, T h, T K, T &Vb, T &Wb,
                                                      T &lamb)
{
    T hb = K * B.s1 + T(2) * K * (K + T(2)) * h * B.s2;
    recur_b<6>(M.v, B.v, V, h, Vb, hb);
    Vb += B.v[1];
    recur_b<6>(M.w, B.w, W, h, Wb, hb);
    Wb += B.w[1];
    lamb += T(-2) * hb * h * h;
}

template <typename T>
__host__ __device__ __forceinline__ void mom_full_u_b(const Mom<T> &M, MomB<T> &B, T U, T h, T &Ub, T &lamb)
{
    T hb = T(0);
    recur_b<7>(M.u, B.u, U, h, Ub, hb);
    Ub += B.u[1];
    lamb += T(-2) * hb * h * h;
}

template <typename T>
__host__ __device__ __forceinline__ void mom_half_u_b(const Mom<T> &M, MomB<T> &B, T U, T lam, T h, T sign, T &Ub,
                                                      T &lamb)
{
    T hb = T(0);
    recur_b<7>(M.u, B.u, U, h, Ub, hb);
    lamb += T(-2) * hb * h * h;
    const T isl = sqrt_t(T(2) * h);  // 1 / sqrt(lambda)
    const T sl = lam * isl;
    const T g = exp_t(-lam * U * U);
    const T ip = T(0.5 * M_2_SQRTPI);  // 1 / sqrt(pi)
    const T e = g * (T(0.5) * ip * isl);
    // u1 = U u0 + sign e
    Ub += M.u[0] * B.u[1];
    const T u0b = B.u[0] + U * B.u[1];
    const T eb = sign * B.u[1];
    Ub += eb * e * (T(-2) * lam * U);
    lamb += eb * e * (-U * U - h);
    // u0 = erfc(-sign sqrt(lam) U) / 2
    Ub += u0b * sign * sl * g * ip;
    lamb += u0b * sign * U * g * ip * (T(0.5) * isl);
}

template <typename T>
__host__ __device__ __forceinline__ T dot5(const T *a, const T *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4];
}

// reverse of slope_solve: a_b -> b_b and state cotangents (a: the forward result)
template <typename T>
__host__ __device__ __forceinline__ void slope_solve_b(const T b[5], T U, T V, T W, T lam, T h, T K, const T a[5],
                                                       const T ab_in[5], T bb[5], T &Ub, T &Vb, T &Wb, T &lamb)
{
    const T iK3 = T(1) / (K + T(3));  // a constant of the launch
    const T q = U * U + V * V + W * W + (K + T(3)) * h;
    const T R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = b[3] - W * b[0];
    const T R5 = T(2) * b[4] - q * b[0];
    const T c = T(4) * lam * lam * iK3;
    const T X = R5 - T(2) * (U * R2 + V * R3 + W * R4);
    T ab[5] = {ab_in[0], ab_in[1], ab_in[2], ab_in[3], ab_in[4]};
    T qb = T(0), R2b = T(0), R3b = T(0), R4b = T(0), R5b = T(0), cb = T(0);
    // a0 = b0 - U a1 - V a2 - W a3 - a4 q / 2
    bb[0] += ab[0];
    Ub += -a[1] * ab[0];
    ab[1] += -U * ab[0];
    Vb += -a[2] * ab[0];
    ab[2] += -V * ab[0];
    Wb += -a[3] * ab[0];
    ab[3] += -W * ab[0];
    ab[4] += T(-0.5) * q * ab[0];
    qb += T(-0.5) * a[4] * ab[0];
    // a3 = 2 lam R4 - W a4 (and a2, a1)
    lamb += T(2) * R4 * ab[3];
    R4b += T(2) * lam * ab[3];
    Wb += -a[4] * ab[3];
    ab[4] += -W * ab[3];
    lamb += T(2) * R3 * ab[2];
    R3b += T(2) * lam * ab[2];
    Vb += -a[4] * ab[2];
    ab[4] += -V * ab[2];
    lamb += T(2) * R2 * ab[1];
    R2b += T(2) * lam * ab[1];
    Ub += -a[4] * ab[1];
    ab[4] += -U * ab[1];
    // a4 = c X
    cb += X * ab[4];
    const T Xb = c * ab[4];
    R5b += Xb;
    R2b += T(-2) * U * Xb;
    Ub += T(-2) * R2 * Xb;
    R3b += T(-2) * V * Xb;
    Vb += T(-2) * R3 * Xb;
    R4b += T(-2) * W * Xb;
    Wb += T(-2) * R4 * Xb;
    lamb += T(8) * lam * iK3 * cb;
    // R5 = 2 b4 - q b0
    bb[4] += T(2) * R5b;
    qb += -b[0] * R5b;
    bb[0] += -q * R5b;
    // R4 = b3 - W b0 (and R3, R2)
    bb[3] += R4b;
    Wb += -b[0] * R4b;
    bb[0] += -W * R4b;
    bb[2] += R3b;
    Vb += -b[0] * R3b;
    bb[0] += -V * R3b;
    bb[1] += R2b;
    Ub += -b[0] * R2b;
    bb[0] += -U * R2b;
    // q
    Ub += T(2) * U * qb;
    Vb += T(2) * V * qb;
    Wb += T(2) * W * qb;
    lamb += T(-2) * (K + T(3)) * h * h * qb;
}

// Reverses of the moment-matrix products.  A matrix's cotangent Qb (same symmetric layout) gathers
// the cotangents of every product that used the matrix; qmat_b then takes it to the moments once.
template <typename T>
__host__ __device__ __forceinline__ void q5_zero(Q5<T> &Q)
{
#pragma unroll
    for (int e = 0; e < 15; ++e) Q.e[e] = T(0);
}

// reverse of o = Q a (or o += Q a): Qb += cotangent of Q, ab += Q ob
template <typename T>
__host__ __device__ __forceinline__ void qmul_b(const Q5<T> &Q, const T a[5], const T ob[5], Q5<T> &Qb, T ab[5])
{
    T *g = Qb.e;
    g[0] += ob[0] * a[0];
    g[1] += ob[0] * a[1] + ob[1] * a[0];
    g[2] += ob[0] * a[2] + ob[2] * a[0];
    g[3] += ob[0] * a[3] + ob[3] * a[0];
    g[4] += ob[0] * a[4] + ob[4] * a[0];
    g[5] += ob[1] * a[1];
    g[6] += ob[1] * a[2] + ob[2] * a[1];
    g[7] += ob[1] * a[3] + ob[3] * a[1];
    g[8] += ob[1] * a[4] + ob[4] * a[1];
    g[9] += ob[2] * a[2];
    g[10] += ob[2] * a[3] + ob[3] * a[2];
    g[11] += ob[2] * a[4] + ob[4] * a[2];
    g[12] += ob[3] * a[3];
    g[13] += ob[3] * a[4] + ob[4] * a[3];
    g[14] += ob[4] * a[4];
    qmul_add(Q, ob, ab);
}

// reverse of y += s * (first column of Q) for the cotangent yb (the cotangent of s is left out)
template <typename T>
__host__ __device__ __forceinline__ void qcol0_b(T s, const T yb[5], Q5<T> &Qb)
{
#pragma unroll
    for (int j = 0; j < 5; ++j) Qb.e[j] += s * yb[j];
}

// sum over the entries of Q times Qb
template <typename T>
__host__ __device__ __forceinline__ T q5_dot(const Q5<T> &Q, const Q5<T> &Qb)
{
    T s = Q.e[0] * Qb.e[0];
#pragma unroll
    for (int e = 1; e < 15; ++e) s += Q.e[e] * Qb.e[e];
    return s;
}

// reverse of qmat<k,l,n>: matrix cotangent -> moment cotangents
template <int k, int l, int n, typename T>
__host__ __device__ __forceinline__ void qmat_b(const Mom<T> &M, const Q5<T> &Qb, MomB<T> &B)
{
    const T *u = M.u + k, *v = M.v + l, *w = M.w + n;
    const T a00 = v[0] * w[0], a10 = v[1] * w[0], a01 = v[0] * w[1], a20 = v[2] * w[0], a11 = v[1] * w[1];
    const T a02 = v[0] * w[2], a30 = v[3] * w[0], a21 = v[2] * w[1], a12 = v[1] * w[2], a03 = v[0] * w[3];
    const T a40 = v[4] * w[0], a22 = v[2] * w[2], a04 = v[0] * w[4];
    const T e0 = u[0] * a00, e1 = u[1] * a00, e2 = u[0] * a10, e3 = u[0] * a01;
    const T tr = u[2] * a00 + u[0] * a20 + u[0] * a02;
    const T *g = Qb.e;
    // the entries with psi_4 first: their parts in the other entries, s1, s2 and the raw factors
    const T h4 = T(0.5) * g[4], h8 = T(0.5) * g[8], h11 = T(0.5) * g[11], h13 = T(0.5) * g[13], q = T(0.25) * g[14];
    const T trb = h4 + T(2) * q * M.s1;
    B.s1 += h4 * e0 + h8 * e1 + h11 * e2 + h13 * e3 + T(2) * q * tr;
    B.s2 += q * e0;
    const T g0 = g[0] + h4 * M.s1 + q * M.s2, g1 = g[1] + h8 * M.s1, g2 = g[2] + h11 * M.s1, g3 = g[3] + h13 * M.s1;
    const T g5 = g[5] + trb, g9 = g[9] + trb, g12 = g[12] + trb;
    // cotangents of the u moments
    T ub[5];
    ub[0] = g0 * a00 + g2 * a10 + g3 * a01 + g9 * a20 + g[10] * a11 + g12 * a02 + h11 * (a30 + a12) +
            h13 * (a21 + a03) + q * (a40 + a04 + T(2) * a22);
    ub[1] = g1 * a00 + g[6] * a10 + g[7] * a01 + h8 * (a20 + a02);
    ub[2] = g5 * a00 + h11 * a10 + h13 * a01 + T(2) * q * (a20 + a02);
    ub[3] = h8 * a00;
    ub[4] = q * a00;
    // cotangents of the v w products
    const T b00 = g0 * u[0] + g1 * u[1] + g5 * u[2] + h8 * u[3] + q * u[4];
    const T b10 = g2 * u[0] + g[6] * u[1] + h11 * u[2];
    const T b01 = g3 * u[0] + g[7] * u[1] + h13 * u[2];
    const T b20 = g9 * u[0] + h8 * u[1] + T(2) * q * u[2];
    const T b02 = g12 * u[0] + h8 * u[1] + T(2) * q * u[2];
    const T b11 = g[10] * u[0];
    const T b30 = h11 * u[0], b12 = h11 * u[0], b21 = h13 * u[0], b03 = h13 * u[0];
    const T b40 = q * u[0], b04 = q * u[0], b22 = T(2) * q * u[0];
#pragma unroll
    for (int i = 0; i < 5; ++i) B.u[k + i] += ub[i];
    B.v[l] += b00 * w[0] + b01 * w[1] + b02 * w[2] + b03 * w[3] + b04 * w[4];
    B.v[l + 1] += b10 * w[0] + b11 * w[1] + b12 * w[2];
    B.v[l + 2] += b20 * w[0] + b21 * w[1] + b22 * w[2];
    B.v[l + 3] += b30 * w[0];
    B.v[l + 4] += b40 * w[0];
    B.w[n] += b00 * v[0] + b10 * v[1] + b20 * v[2] + b30 * v[3] + b40 * v[4];
    B.w[n + 1] += b01 * v[0] + b11 * v[1] + b21 * v[2];
    B.w[n + 2] += b02 * v[0] + b12 * v[1] + b22 * v[2];
    B.w[n + 3] += b03 * v[0];
    B.w[n + 4] += b04 * v[0];
}

// reverse of stein_add: ob (the cotangent of o) -> cotangents of Qa, P, X, h and a (accumulated);
// od += ob . (the term stein_add adds to o)
template <int DIR, typename T>
__host__ __device__ __forceinline__ void stein_add_b(const T Qa[5], const T P[5], T X, T h, const T a[5], const T ob[5],
                                                     T Qab[5], T Pb[5], T &Xb, T &hb, T ab[5], T &od)
{
    const T c = a[DIR] + a[4] * X;
    const T hc = h * c;
    const T ha4u = h * a[4] * P[0];
    T S = T(0), R = T(0);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        S += ob[j] * P[j];
        R += ob[j] * Qa[j];
        Qab[j] += X * ob[j];
        Pb[j] += hc * ob[j];
    }
    // o_j += X Qa_j + hc P_j
    Xb += R;
    T hcb = S;
    // o_DIR += h (Qa_0 + ha4u)
    hb += ob[DIR] * (Qa[0] + ha4u);
    Qab[0] += h * ob[DIR];
    T ha4ub = h * ob[DIR];
    // o_4 += h z, z = X Qa_0 + hc P_0 + ha4u X
    const T z = X * Qa[0] + hc * P[0] + ha4u * X;
    od += X * R + hc * S + h * (ob[DIR] * (Qa[0] + ha4u) + ob[4] * z);
    hb += ob[4] * z;
    const T zb = h * ob[4];
    Xb += zb * (Qa[0] + ha4u);
    Qab[0] += zb * X;
    hcb += zb * P[0];
    Pb[0] += zb * hc;
    ha4ub += zb * X;
    // ha4u = h a_4 P_0, hc = h c, c = a_DIR + a_4 X
    hb += ha4ub * a[4] * P[0] + hcb * c;
    ab[4] += ha4ub * h * P[0];
    Pb[0] += ha4ub * h * a[4];
    const T cb = hcb * h;
    ab[DIR] += cb;
    ab[4] += cb * X;
    Xb += cb * a[4];
}

// reverse of stein_u2_add: ob -> cotangents of Q1a, B, P1, P2, U, h and a (accumulated)
template <typename T>
__host__ __device__ __forceinline__ void stein_u2_add_b(const T Q1a[5], const T B[5], const T P1[5], const T P2[5], T U,
                                                        T h, const T a[5], const T ob[5], T Q1ab[5], T Bb[5],
                                                        T P1b[5], T P2b[5], T &Ub, T &hb, T ab[5])
{
    T S1 = T(0), S2 = T(0);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        Q1ab[j] += U * ob[j];
        Bb[j] += h * ob[j];
        P1b[j] += h * a[1] * ob[j];
        P2b[j] += h * a[4] * ob[j];
        Ub += ob[j] * Q1a[j];
        hb += ob[j] * (B[j] + a[1] * P1[j] + a[4] * P2[j]);
        S1 += ob[j] * P1[j];
        S2 += ob[j] * P2[j];
    }
    ab[1] += h * S1;
    ab[4] += h * S2;
    // o_1 += h Q1a_0
    hb += ob[1] * Q1a[0];
    Q1ab[0] += h * ob[1];
    // o_4 += h s2, s2 = U Q1a_0 + h c0, c0 = B_0 + a_1 P1_0 + a_4 P2_0
    const T c0 = B[0] + a[1] * P1[0] + a[4] * P2[0];
    hb += ob[4] * (U * Q1a[0] + h * c0);
    const T s2b = h * ob[4];
    Ub += s2b * Q1a[0];
    Q1ab[0] += s2b * U;
    hb += s2b * c0;
    const T c0b = s2b * h;
    Bb[0] += c0b;
    ab[1] += c0b * P1[0];
    P1b[0] += c0b * a[1];
    ab[4] += c0b * P2[0];
    P2b[0] += c0b * a[4];
}

// reverse of euler_jac_add along axis m: fb (the cotangent of f) -> cotangents of d (accumulated
// into db) and of rho, u, H, k2 and 1/rho.  The intermediates are formed again in another
// association than the forward's, so that the compiler does not keep the forward's alive until here.
template <typename T>
__host__ __device__ __forceinline__ void euler_jac_add_b(int m, T rho, T ir, const T u[3], T g1, T k2, T H,
                                                         const T d[5], const T fb[5], T db[5], T &rhob, T ub[3],
                                                         T &Hb, T &k2b, T &irb)
{
    const T d0i = d[0] * ir;
    T du[3], dub[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 3; ++k) du[k] = d[1 + k] * ir - u[k] * d0i;
    const T dp = g1 * (d[4] + k2 * d[0] - (u[0] * d[1] + u[1] * d[2] + u[2] * d[3]));
    // f4 += du_m H + u_m (d4 + dp)
    dub[m] += fb[4] * H;
    Hb += fb[4] * du[m];
    ub[m] += fb[4] * (d[4] + dp);
    db[4] += fb[4] * u[m];
    T dpb = fb[4] * u[m];
    // f_{1+m} += dp
    dpb += fb[1 + m];
    // f_{1+k} += d_{1+m} u_k + rho u_m du_k
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        db[1 + m] += fb[1 + k] * u[k];
        ub[k] += fb[1 + k] * d[1 + m];
        rhob += fb[1 + k] * u[m] * du[k];
        ub[m] += fb[1 + k] * rho * du[k];
        dub[k] += fb[1 + k] * rho * u[m];
    }
    // f0 += d_{1+m}
    db[1 + m] += fb[0];
    // dp = g1 (d4 - u . d_{1..3} + k2 d0)
    db[4] += g1 * dpb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ub[k] += -g1 * dpb * d[1 + k];
        db[1 + k] += -g1 * dpb * u[k];
    }
    k2b += g1 * dpb * d[0];
    db[0] += g1 * dpb * k2;
    // du_k = (d_{1+k} - u_k d0) / rho
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        db[1 + k] += dub[k] * ir;
        ub[k] += -dub[k] * d0i;
        db[0] += -dub[k] * u[k] * ir;
        irb += dub[k] * du[k] * rho;
    }
}

// the cotangents of u, H = E + p, k2 = |u|^2 / 2 and 1/rho to those of U, V, W, E, p and rho
template <typename T>
__host__ __device__ __forceinline__ void euler_state_b(T ir, const T u[3], const T ub[3], T Hb, T k2b, T irb, T &rhob,
                                                       T &Ub, T &Vb, T &Wb, T &pb, T &Eb)
{
    Ub += ub[0] + k2b * u[0];
    Vb += ub[1] + k2b * u[1];
    Wb += ub[2] + k2b * u[2];
    Eb += Hb;
    pb += Hb;
    rhob += -irb * ir * ir;
}

// reverse of euler_div (o: its forward result): o_b -> cotangents of rho, U, V, W, p, E and dq
// (accumulated)
template <typename T>
__host__ __device__ __forceinline__ void euler_div_b(T rho, T ir, T U, T V, T W, T p, T E, T gam, const T dq[3][5],
                                                     const T o[5], const T ob[5], T &rhob, T &Ub, T &Vb, T &Wb,
                                                     T &pb, T &Eb, T dqb[3][5])
{
    const T u[3] = {U, V, W};
    T fb[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) fb[j] = ob[j] * ir;
    // o = f / rho: the cotangent of 1 / rho is ob . f = rho (ob . o)
    T irb = rho * (ob[0] * o[0] + ob[1] * o[1] + ob[2] * o[2] + ob[3] * o[3] + ob[4] * o[4]);
    T ub[3] = {T(0), T(0), T(0)}, Hb = T(0), k2b = T(0);
#pragma unroll
    for (int m = 0; m < 3; ++m)
        euler_jac_add_b(m, rho, ir, u, gam - T(1), T(0.5) * (U * U + V * V + W * W), E + p, dq[m], fb, dqb[m], rhob,
                        ub, Hb, k2b, irb);
    euler_state_b(ir, u, ub, Hb, k2b, irb, rhob, Ub, Vb, Wb, pb, Eb);
}

// reverse of to_prim
template <typename T>
__host__ __device__ __forceinline__ void to_prim_b(const T q[5], T gam, T rhob, T Ub, T Vb, T Wb, T lamb, T pb, T qb[5])
{
    T rho, U, V, W, lam, p, h;
    to_prim(q, gam, rho, U, V, W, lam, p, h);
    const T ir = T(1) / rho;
    // lambda = rho / (2 p): d/drho = lambda / rho, d/dp = -lambda / p = -2 lambda^2 / rho
    rhob += lamb * lam * ir;
    pb += T(-2) * lamb * lam * lam * ir;
    qb[4] += (gam - T(1)) * pb;
    rhob += -(gam - T(1)) * pb * T(0.5) * (U * U + V * V + W * W);
    Ub += -(gam - T(1)) * pb * rho * U;
    Vb += -(gam - T(1)) * pb * rho * V;
    Wb += -(gam - T(1)) * pb * rho * W;
    qb[1] += Ub * ir;
    qb[2] += Vb * ir;
    qb[3] += Wb * ir;
    rhob += -(Ub * U + Vb * V + Wb * W) * ir;
    qb[0] += rhob;
}

// cotangents of the half-space accumulators
template <typename T, bool PR>
struct FluxAccB {
    T q0[5], bab[3][5], Mh[5], Mha[5], MhA[5];
    T Wha[PR ? 5 : 1], WhA[PR ? 5 : 1];
    T p[2];
};

template <typename T, bool PR>
__host__ __device__ __forceinline__ void accb_zero(FluxAccB<T, PR> &A)
{
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        A.q0[j] = A.Mh[j] = A.Mha[j] = A.MhA[j] = T(0);
        A.bab[0][j] = A.bab[1][j] = A.bab[2][j] = T(0);
        if constexpr (PR) A.Wha[j] = A.WhA[j] = T(0);
    }
    A.p[0] = A.p[1] = T(0);
}

// positions of the accumulator cotangents, in the member order of FluxAccB
enum AccSlot { kSlotQ0 = 0, kSlotBab = 5, kSlotMh = 20, kSlotMha = 25, kSlotMhA = 30, kSlotWha = 35, kSlotWhA = 40,
               kSlotP = 45 };

template <typename T, bool PR>
__host__ __device__ __forceinline__ T &accb_slot(FluxAccB<T, PR> &A, int s)
{
    if (s < kSlotBab) return A.q0[s];
    if (s < kSlotMh) return A.bab[(s - kSlotBab) / 5][(s - kSlotBab) % 5];
    if (s < kSlotMha) return A.Mh[s - kSlotMh];
    if (s < kSlotMhA) return A.Mha[s - kSlotMha];
    if (s < kSlotWha) return A.MhA[s - kSlotMhA];
    if constexpr (PR) {
        if (s < kSlotWhA) return A.Wha[s - kSlotWha];
        if (s < kSlotP) return A.WhA[s - kSlotWhA];
    }
    return A.p[s - kSlotP];
}

// reverse of side_pass: accumulator cotangents (read through get(slot), each
// once, where it is used) -> q_b, dq_b.  One moment set M holds the half-space
// u moments while the half-space accumulations are reversed, then the
// full-space ones; v, w and internal moments (and their cotangents) are shared
// by both.
template <typename T, bool PR, typename Get>
__host__ __device__ void side_pass_b(const T q[5], const T dq[3][5], T sign, const FluxParams<T> &fp, Get get, int side,
                                     T qb[5], T dqb[3][5])
{
    auto ld = [&](int slot, T o[5]) {
#pragma unroll
        for (int j = 0; j < 5; ++j) o[j] = get(slot + j);
    };
    const T K = fp.K;
    T rho, U, V, W, lam, p, h;
    to_prim(q, fp.gamma, rho, U, V, W, lam, p, h);
    const T ir = T(1) / rho;
    Mom<T> M;
    mom_common(M, V, W, h, K);
    T a[3][5], Av[5];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T bm[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) bm[j] = dq[m][j] * ir;
        slope_solve(bm, U, V, W, lam, h, K, a[m]);
    }
    {
        T bA[5];
        euler_div(rho, ir, U, V, W, p, q[4], fp.gamma, dq, bA);
#pragma unroll
        for (int j = 0; j < 5; ++j) bA[j] = -bA[j];
        slope_solve(bA, U, V, W, lam, h, K, Av);
    }
    mom_half_u(M, U, lam, h, sign);

    T rhob = T(0), Ub = T(0), Vb = T(0), Wb = T(0), lamb = T(0);
    MomB<T> B;
    momb_zero(B);
    T ab[3][5], Avb[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        Avb[j] = T(0);
        ab[0][j] = ab[1][j] = ab[2][j] = T(0);
    }
    // Every half-space accumulation is rho times a moment-matrix product; the matrix's cotangent
    // gathers the rho-scaled slot cotangents of all its products, and rho's cotangent is
    // sum(Q Qb) / rho.  (side_pass forms the v and w terms of qadv by Stein's identity; here they
    // keep their own matrices, the same function: reversed through Stein's identity this pass
    // needs more registers than the lane has.)
    T g[5], s[5], sw[5];
    auto scaled = [&](int slot, T o[5]) {
        ld(slot, g);
#pragma unroll
        for (int j = 0; j < 5; ++j) o[j] = rho * g[j];
    };
    Q5<T> Q, Qb;
    // <psi psi^T>: q0 (first column), bab[m] (a[m]), WhA (Av, PR)
    qmat<0, 0, 0>(M, Q);
    q5_zero(Qb);
    scaled(kSlotQ0, s);
    qcol0_b(T(1), s, Qb);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        scaled(kSlotBab + 5 * m, s);
        qmul_b(Q, a[m], s, Qb, ab[m]);
    }
    if constexpr (PR) {
        scaled(kSlotWhA, s);
        qmul_b(Q, Av, s, Qb, Avb);
    }
    rhob += ir * q5_dot(Q, Qb);
    qmat_b<0, 0, 0>(M, Qb, B);
    // <u psi psi^T>: Mh (first column), MhA (Av), with PR the a[0] term of Wha
    qmat<1, 0, 0>(M, Q);
    q5_zero(Qb);
    scaled(kSlotMh, s);
    qcol0_b(T(1), s, Qb);
    scaled(kSlotMhA, s);
    qmul_b(Q, Av, s, Qb, Avb);
    if constexpr (PR) {
        scaled(kSlotWha, sw);
        qmul_b(Q, a[0], sw, Qb, ab[0]);
    }
    rhob += ir * q5_dot(Q, Qb);
    qmat_b<1, 0, 0>(M, Qb, B);
    // Mha = <u^2 psi psi^T> a[0] + <u v psi psi^T> a[1] + <u w psi psi^T> a[2]
    scaled(kSlotMha, s);
    qmat<2, 0, 0>(M, Q);
    q5_zero(Qb);
    qmul_b(Q, a[0], s, Qb, ab[0]);
    rhob += ir * q5_dot(Q, Qb);
    qmat_b<2, 0, 0>(M, Qb, B);
    qmat<1, 1, 0>(M, Q);
    q5_zero(Qb);
    qmul_b(Q, a[1], s, Qb, ab[1]);
    rhob += ir * q5_dot(Q, Qb);
    qmat_b<1, 1, 0>(M, Qb, B);
    qmat<1, 0, 1>(M, Q);
    q5_zero(Qb);
    qmul_b(Q, a[2], s, Qb, ab[2]);
    rhob += ir * q5_dot(Q, Qb);
    qmat_b<1, 0, 1>(M, Qb, B);
    if constexpr (PR) {
        // the v and w terms of Wha
        qmat<0, 1, 0>(M, Q);
        q5_zero(Qb);
        qmul_b(Q, a[1], sw, Qb, ab[1]);
        rhob += ir * q5_dot(Q, Qb);
        qmat_b<0, 1, 0>(M, Qb, B);
        qmat<0, 0, 1>(M, Q);
        q5_zero(Qb);
        qmul_b(Q, a[2], sw, Qb, ab[2]);
        rhob += ir * q5_dot(Q, Qb);
        qmat_b<0, 0, 1>(M, Qb, B);
    }
    // half-space u moments done: their cotangents go to U and lambda, the v, w and internal
    // moments' to V, W and lambda (the time slope's right-hand side uses no moments)
    mom_half_u_b(M, B, U, lam, h, sign, Ub, lamb);
    mom_common_b(M, B, V, W, h, K, Vb, Wb, lamb);
    // a[m] = solve(dq[m] / rho)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T bm[5], bmb[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < 5; ++j) bm[j] = dq[m][j] * ir;
        slope_solve_b(bm, U, V, W, lam, h, K, a[m], ab[m], bmb, Ub, Vb, Wb, lamb);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            dqb[m][j] += bmb[j] * ir;
            rhob += -bmb[j] * bm[j] * ir;
        }
    }
    // Av = solve(-euler_div(q, dq))
    T pb = get(kSlotP + side), Eb = T(0);
    {
        T ed[5], bA[5];
        euler_div(rho, ir, U, V, W, p, q[4], fp.gamma, dq, ed);
#pragma unroll
        for (int j = 0; j < 5; ++j) bA[j] = -ed[j];
        T bAb[5] = {T(0), T(0), T(0), T(0), T(0)};
        slope_solve_b(bA, U, V, W, lam, h, K, Av, Avb, bAb, Ub, Vb, Wb, lamb);
#pragma unroll
        for (int j = 0; j < 5; ++j) bAb[j] = -bAb[j];
        euler_div_b(rho, ir, U, V, W, p, q[4], fp.gamma, dq, ed, bAb, rhob, Ub, Vb, Wb, pb, Eb, dqb);
    }
    to_prim_b(q, fp.gamma, rhob, Ub, Vb, Wb, lamb, pb, qb);
    qb[4] += Eb;
}

// T coefficients of the time integrals over [0, d] and their derivatives in tau
// (eta = exp(-d / tau), om = 1 - eta, itau = 1 / tau)
template <typename T>
__host__ __device__ __forceinline__ void tcoef(T d, T tau, T itau, T eta, T om, T Tc[5], T dT[5])
{
    const T deta = eta * d * itau * itau;
    const T dom = -deta;
    Tc[0] = d - tau * om;
    Tc[1] = T(2) * tau * tau * om - tau * d * (T(1) + eta);
    Tc[2] = T(0.5) * d * d - tau * d + tau * tau * om;
    Tc[3] = tau * om;
    Tc[4] = T(2) * tau * tau * om - tau * d * eta;
    dT[0] = -om - tau * dom;
    dT[1] = T(4) * tau * om + T(2) * tau * tau * dom - d * (T(1) + eta) - tau * d * deta;
    dT[2] = -d + T(2) * tau * om + tau * tau * dom;
    dT[3] = om + tau * dom;
    dT[4] = T(4) * tau * om + T(2) * tau * tau * dom - d * eta - tau * d * deta;
}

/*
 * Reverse of finish_flux: out_b -> accumulator cotangents, each handed to
 * put(slot, value) once, as soon as it is final (slots of AccSlot; the
 * Prandtl slots only when PR).
 *
 * The flux at each of the two integration lengths is a sum of coefficient x
 * vector terms (g_0 moment vectors with r_0 T_1..T_3, accumulators with
 * T_4, T_5, tau T_4; with PR the same for the heat-flux vector W), so the
 * cotangents of the coefficients are dot products of the flux cotangents
 * with one vector at a time: no vector stays live after its dot products.
 */
template <typename T, bool PR, typename Put>
__host__ __device__ void finish_flux_b(const FluxAcc<T, PR> &A, T dt, const FluxParams<T> &fp, const T outb[10],
                                       Put put)
{
    const T K = fp.K;
    T r0, U0, V0, W0, lam0, p0, h0;
    to_prim(A.q0, fp.gamma, r0, U0, V0, W0, lam0, p0, h0);
    const T ir0 = T(1) / r0;
    T ab[3][5];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T bm[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) bm[j] = A.bab[m][j] * ir0;
        slope_solve(bm, U0, V0, W0, lam0, h0, K, ab[m]);
    }
    T pv[5];  // qadv<0>(G, ab): the negated right-hand side of g_0's time slope
    euler_div(r0, ir0, U0, V0, W0, p0, A.q0[4], fp.gamma, A.bab, pv);
    const T E0 = A.q0[4], g1 = fp.gamma - T(1);
    const T u0[3] = {U0, V0, W0};
    const T dp = (A.p[0] - A.p[1]) / (A.p[0] + A.p[1]);
    const T adp = dp < T(0) ? -dp : dp;
    const T tau = fp.viscous ? fp.mu / p0 + fp.tau_C * adp * dt : fp.tau_eps * dt + fp.tau_C * adp * dt;
    // time coefficients of F(dt/2) (s = 0) and F(dt) (s = 1), their tau derivatives, and the
    // cotangents of F(dt/2), F(dt) from out = (4 F(dt/2) - F(dt)) / dt, 4 (F(dt) - 2 F(dt/2)) / dt^2
    T Tc[2][5], dT[2][5], Fb[2][5];
    {
        // the integration lengths dt / 2 and dt: exp(-dt / tau) = eta^2, 1 - exp(-dt / tau) = om (1 + eta)
        const T itau = T(1) / tau;
        const T eta = exp_t(T(-0.5) * dt * itau), om = -expm1_t(T(-0.5) * dt * itau);
        tcoef(T(0.5) * dt, tau, itau, eta, om, Tc[0], dT[0]);
        tcoef(dt, tau, itau, eta * eta, om * (T(1) + eta), Tc[1], dT[1]);
    }
    const T idt = T(1) / dt;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        Fb[0][j] = T(4) * idt * outb[j] - T(8) * idt * idt * outb[5 + j];
        Fb[1][j] = -idt * outb[j] + T(4) * idt * idt * outb[5 + j];
    }
    // Prandtl correction F_4 += kap q2, q2 = e . F - U0 e . W (uncorrected F): the cotangent of
    // the uncorrected F gains q2b e, that of W is w e with w = -U0 q2b
    const T U2 = U0 * U0 + V0 * V0 + W0 * W0;
    const T e[5] = {U2, T(-2) * U0, T(-2) * V0, T(-2) * W0, T(2)};
    T q2b[2] = {T(0), T(0)}, w[2] = {T(0), T(0)};
    if constexpr (PR) {
        const T kap = (T(1) / fp.Pr - T(1)) * T(0.5);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            q2b[s] = kap * Fb[s][4];
#pragma unroll
            for (int j = 0; j < 5; ++j) Fb[s][j] += q2b[s] * e[j];
            w[s] = -U0 * q2b[s];
        }
    }
    // accumulator cotangents that are final already
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const T mh = Tc[0][3] * Fb[0][j] + Tc[1][3] * Fb[1][j];
        put(kSlotMh + j, mh);
        put(kSlotMha + j, -(Tc[0][4] * Fb[0][j] + Tc[1][4] * Fb[1][j]));
        put(kSlotMhA + j, -tau * mh);
    }
    if constexpr (PR) {
        const T c3 = Tc[0][3] * w[0] + Tc[1][3] * w[1], c4 = Tc[0][4] * w[0] + Tc[1][4] * w[1];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            put(kSlotWha + j, -c4 * e[j]);
            put(kSlotWhA + j, -tau * c3 * e[j]);
        }
    }
    // coefficient cotangents Tb[s][k], tau, r0; with PR the parts of F and W that q2's
    // explicit velocity dependence needs
    T Tb[2][5], taub = T(0), r0b = T(0);
    T Fs[2][4], Ws[2][4], eW[2] = {T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            Tb[s][k] = T(0);
            if (k < 4) Fs[s][k] = Ws[s][k] = T(0);
        }
    // F term coef_s X with coef_s = cs * Tc[s][k]: Tb[s][k] += cs Fb_s . X
    auto fterm = [&](const T X[5], int k, T cs) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Tb[s][k] += cs * dot5(Fb[s], X);
            if constexpr (PR) {
#pragma unroll
                for (int i = 0; i < 4; ++i) Fs[s][i] += cs * Tc[s][k] * X[i];
            }
        }
    };
    // W term coef_s Y, coefficient cotangent w_s e . Y
    auto wterm = [&](const T Y[5], int k, T cs) {
        const T eY = dot5(e, Y);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            Tb[s][k] += cs * w[s] * eY;
            eW[s] += cs * Tc[s][k] * eY;
#pragma unroll
            for (int i = 0; i < 4; ++i) Ws[s][i] += cs * Tc[s][k] * Y[i];
        }
    };
    {
        // g_0's moment vectors as in finish_flux: <u psi> = (its Euler flux along n1) / r0,
        // <u (Ab . psi) psi> = that flux's Jacobian applied to -pv, <u (ab . u psi) psi> = qadv<1>;
        // with PR <psi> = q0 / r0, qadv<0> = pv and <(Ab . psi) psi> = -pv
        T X[5];
        X[0] = U0;
        X[1] = U0 * U0 + h0;
        X[2] = U0 * V0;
        X[3] = U0 * W0;
        X[4] = U0 * (E0 * ir0 + h0);
        fterm(X, 0, r0);
        r0b += Tc[0][0] * dot5(Fb[0], X) + Tc[1][0] * dot5(Fb[1], X);
        T npv[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            npv[j] = -pv[j];
            X[j] = T(0);
        }
        euler_jac_add(0, r0, ir0, u0, g1, T(0.5) * U2, E0 + p0, npv, X);
        fterm(X, 2, r0);
        r0b += Tc[0][2] * dot5(Fb[0], X) + Tc[1][2] * dot5(Fb[1], X);
        // qadv<1> of g_0 by Stein chains, as in finish_flux
        T M0v[5] = {U0, U0 * U0 + h0, U0 * V0, U0 * W0, U0 * (E0 * ir0 + h0)};
#pragma unroll
        for (int j = 0; j < 5; ++j) X[j] = T(0);
        {
            T Pw[5], P2[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) Pw[j] = A.q0[j] * ir0;
#pragma unroll
            for (int j = 0; j < 5; ++j) P2[j] = U0 * M0v[j] + h0 * Pw[j];
            P2[1] += h0 * U0;
            P2[4] += h0 * (U0 * U0 + h0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                T B[5], Q1a[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int j = 0; j < 5; ++j) B[j] = A.bab[m][j] * ir0;
                stein_add<1>(B, Pw, U0, h0, ab[m], Q1a);
                if (m == 0)
                    stein_u2_add(Q1a, B, M0v, P2, U0, h0, ab[0], X);
                else if (m == 1)
                    stein_add<2>(Q1a, M0v, V0, h0, ab[1], X);
                else
                    stein_add<3>(Q1a, M0v, W0, h0, ab[2], X);
            }
        }
        fterm(X, 1, r0);
        r0b += Tc[0][1] * dot5(Fb[0], X) + Tc[1][1] * dot5(Fb[1], X);
        if constexpr (PR) {
#pragma unroll
            for (int j = 0; j < 5; ++j) X[j] = A.q0[j] * ir0;
            wterm(X, 0, r0);
            r0b += (Tc[0][0] * w[0] + Tc[1][0] * w[1]) * dot5(e, X);
            wterm(npv, 2, r0);
            r0b += (Tc[0][2] * w[0] + Tc[1][2] * w[1]) * dot5(e, npv);
            wterm(pv, 1, r0);
            r0b += (Tc[0][1] * w[0] + Tc[1][1] * w[1]) * dot5(e, pv);
        }
    }
    fterm(A.Mh, 3, T(1));
    fterm(A.Mha, 4, T(-1));
    fterm(A.MhA, 3, -tau);
    taub += -(Tc[0][3] * dot5(Fb[0], A.MhA) + Tc[1][3] * dot5(Fb[1], A.MhA));
    if constexpr (PR) {
        wterm(A.q0, 3, T(1));
        wterm(A.Wha, 4, T(-1));
        wterm(A.WhA, 3, -tau);
        taub += -(Tc[0][3] * w[0] + Tc[1][3] * w[1]) * dot5(e, A.WhA);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int k = 0; k < 5; ++k) taub += Tb[s][k] * dT[s][k];
    T U0b = T(0), V0b = T(0), W0b = T(0), lam0b = T(0), p0b = T(0);
    if constexpr (PR) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            U0b += q2b[s] * (T(-2) * Fs[s][1] + T(2) * U0 * Fs[s][0] - eW[s] -
                             U0 * (T(-2) * Ws[s][1] + T(2) * U0 * Ws[s][0]));
            V0b += q2b[s] * (T(-2) * Fs[s][2] + T(2) * V0 * Fs[s][0] - U0 * (T(-2) * Ws[s][2] + T(2) * V0 * Ws[s][0]));
            W0b += q2b[s] * (T(-2) * Fs[s][3] + T(2) * W0 * Fs[s][0] - U0 * (T(-2) * Ws[s][3] + T(2) * W0 * Ws[s][0]));
        }
    }
    // collision time
    {
        const T sp = A.p[0] + A.p[1];
        const T dpb = fp.tau_C * dt * sgn_t(dp) * taub;
        const T isp = T(1) / sp;
        put(kSlotP + 0, dpb * T(2) * A.p[1] * isp * isp);
        put(kSlotP + 1, -dpb * T(2) * A.p[0] * isp * isp);
        if (fp.viscous) p0b += -fp.mu / p0 * (T(2) * lam0 * ir0) * taub;  // 1 / p0 = 2 lambda0 / r0
    }
    // moment vectors of g0: cotangents r0 (T_k(dt/2) Fb_0 + T_k(dt) Fb_1), and r0 c_k e for W
    T abb[3][5], babb[3][5];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int j = 0; j < 5; ++j) babb[m][j] = T(0);
#pragma unroll
    for (int j = 0; j < 5; ++j) abb[0][j] = abb[1][j] = abb[2][j] = T(0);
    T ob0[5], ob1[5], ob2[5], pvb[5], q0d[5], E0b = T(0);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        ob0[j] = r0 * (Tc[0][0] * Fb[0][j] + Tc[1][0] * Fb[1][j]);
        ob1[j] = r0 * (Tc[0][1] * Fb[0][j] + Tc[1][1] * Fb[1][j]);
        ob2[j] = r0 * (Tc[0][2] * Fb[0][j] + Tc[1][2] * Fb[1][j]);
        pvb[j] = q0d[j] = T(0);
    }
    if constexpr (PR) {
        // W's <psi> = q0 / r0 (cotangent c0 e), qadv<0> = pv (c1 e), <(Ab . psi) psi> = -pv (c2 e)
        const T c0 = r0 * (Tc[0][0] * w[0] + Tc[1][0] * w[1]);
        const T c1 = r0 * (Tc[0][1] * w[0] + Tc[1][1] * w[1]);
        const T c2 = r0 * (Tc[0][2] * w[0] + Tc[1][2] * w[1]);
        T sq = T(0);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            pvb[j] = (c1 - c2) * e[j];
            q0d[j] = c0 * e[j] * ir0;
            sq += c0 * e[j] * A.q0[j];
        }
        r0b += -sq * ir0 * ir0;
    }
    // qadv<1> of g_0 (Stein chains in u, v, w from bab / r0, W0 / r0, <u psi>, <u^2 psi>), reversed:
    // its cotangent of <u psi> joins ob0's below
    T M0b[5] = {T(0), T(0), T(0), T(0), T(0)};
    {
        const T M0v[5] = {U0, U0 * U0 + h0, U0 * V0, U0 * W0, U0 * (E0 * ir0 + h0)};
        T Pw[5], P2[5], Pwb[5] = {T(0), T(0), T(0), T(0), T(0)}, P2b[5] = {T(0), T(0), T(0), T(0), T(0)};
        T hb = T(0), od = T(0);
#pragma unroll
        for (int j = 0; j < 5; ++j) Pw[j] = A.q0[j] * ir0;
#pragma unroll
        for (int j = 0; j < 5; ++j) P2[j] = U0 * M0v[j] + h0 * Pw[j];
        P2[1] += h0 * U0;
        P2[4] += h0 * (U0 * U0 + h0);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            T B[5], Q1a[5] = {T(0), T(0), T(0), T(0), T(0)};
            T Q1ab[5] = {T(0), T(0), T(0), T(0), T(0)}, Bb[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int j = 0; j < 5; ++j) B[j] = A.bab[m][j] * ir0;
            stein_add<1>(B, Pw, U0, h0, ab[m], Q1a);
            if (m == 0)
                stein_u2_add_b(Q1a, B, M0v, P2, U0, h0, ab[0], ob1, Q1ab, Bb, M0b, P2b, U0b, hb, abb[0]);
            else if (m == 1)
                stein_add_b<2>(Q1a, M0v, V0, h0, ab[1], ob1, Q1ab, M0b, V0b, hb, abb[1], od);
            else
                stein_add_b<3>(Q1a, M0v, W0, h0, ab[2], ob1, Q1ab, M0b, W0b, hb, abb[2], od);
            stein_add_b<1>(B, Pw, U0, h0, ab[m], Q1ab, Bb, Pwb, U0b, hb, abb[m], od);
            // B = bab[m] / r0
            T sb = T(0);
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                babb[m][j] += Bb[j] * ir0;
                sb += Bb[j] * B[j];
            }
            r0b += -sb * ir0;
        }
        // P2_j = U0 M0_j + h0 Pw_j (+ h0 U0 at j = 1, + h0 (U0^2 + h0) at j = 4)
        T sp = T(0);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            U0b += P2b[j] * M0v[j];
            M0b[j] += U0 * P2b[j];
            hb += P2b[j] * Pw[j];
            Pwb[j] += h0 * P2b[j];
        }
        hb += P2b[1] * U0 + P2b[4] * (U0 * U0 + T(2) * h0);
        U0b += P2b[1] * h0 + P2b[4] * T(2) * U0 * h0;
        // Pw = q0 / r0
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            q0d[j] += Pwb[j] * ir0;
            sp += Pwb[j] * Pw[j];
        }
        r0b += -sp * ir0;
        // h0 = p0 / r0
        p0b += hb * ir0;
        r0b += -hb * h0 * ir0;
    }
    // <u psi> = (U0, U0^2 + h0, U0 V0, U0 W0, U0 (E0 / r0 + h0)), h0 = p0 / r0
    {
#pragma unroll
        for (int j = 0; j < 5; ++j) ob0[j] += M0b[j];
        U0b += ob0[0] + T(2) * U0 * ob0[1] + V0 * ob0[2] + W0 * ob0[3] + (E0 * ir0 + h0) * ob0[4];
        V0b += U0 * ob0[2];
        W0b += U0 * ob0[3];
        const T hb = ob0[1] + U0 * ob0[4];
        E0b += U0 * ir0 * ob0[4];
        r0b += -U0 * E0 * ir0 * ir0 * ob0[4];
        p0b += hb * ir0;
        r0b += -hb * h0 * ir0;
    }
    // <u (Ab . psi) psi> = F_n'(W0) (-pv)
    {
        T npv[5], npvb[5] = {T(0), T(0), T(0), T(0), T(0)}, ub[3] = {T(0), T(0), T(0)};
        T Hb = T(0), k2b = T(0), irb = T(0);
#pragma unroll
        for (int j = 0; j < 5; ++j) npv[j] = -pv[j];
        euler_jac_add_b(0, r0, ir0, u0, g1, T(0.5) * U2, E0 + p0, npv, ob2, npvb, r0b, ub, Hb, k2b, irb);
#pragma unroll
        for (int j = 0; j < 5; ++j) pvb[j] -= npvb[j];
        euler_state_b(ir0, u0, ub, Hb, k2b, irb, r0b, U0b, V0b, W0b, p0b, E0b);
    }
    // pv = euler_div(q0, bab): its cotangents of bab join the slopes' below
    euler_div_b(r0, ir0, U0, V0, W0, p0, E0, fp.gamma, A.bab, pv, pvb, r0b, U0b, V0b, W0b, p0b, E0b, babb);
    // ab[m] = solve(bab[m] / r0)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T bm[5], bmb[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < 5; ++j) bm[j] = A.bab[m][j] * ir0;
        slope_solve_b(bm, U0, V0, W0, lam0, h0, K, ab[m], abb[m], bmb, U0b, V0b, W0b, lam0b);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            put(kSlotBab + 5 * m + j, bmb[j] * ir0 + babb[m][j]);
            r0b += -bmb[j] * bm[j] * ir0;
        }
    }
    // g_0's own conserved variables, plus (PR) their appearance in W with T_4
    T q0b[5];
    {
        const T c3 = PR ? Tc[0][3] * w[0] + Tc[1][3] * w[1] : T(0);
#pragma unroll
        for (int j = 0; j < 5; ++j) q0b[j] = c3 * e[j];
    }
    to_prim_b(A.q0, fp.gamma, r0b, U0b, V0b, W0b, lam0b, p0b, q0b);
    q0b[4] += E0b;
#pragma unroll
    for (int j = 0; j < 5; ++j) q0b[j] += q0d[j];
#pragma unroll
    for (int j = 0; j < 5; ++j) put(kSlotQ0 + j, q0b[j]);
}

// reverse of gp_flux: out_b -> cotangents of both local-frame states and their derivatives
template <typename T, bool PR>
__host__ __device__ void gp_flux_b(const T ql[5], const T dql[3][5], const T qr[5], const T dqr[3][5], T dt,
                                   const FluxParams<T> &fp, const T outb[10], T qlb[5], T dqlb[3][5], T qrb[5],
                                   T dqrb[3][5])
{
    FluxAcc<T, PR> A;
    acc_zero(A);
    side_pass<T, PR>(ql, dql, T(1), fp, A, 0);
    side_pass<T, PR>(qr, dqr, T(-1), fp, A, 1);
    FluxAccB<T, PR> Ab;
    accb_zero(Ab);
    finish_flux_b<T, PR>(A, dt, fp, outb, [&](int slot, T v) { accb_slot(Ab, slot) = v; });
    auto get = [&](int slot) { return accb_slot(Ab, slot); };
    side_pass_b<T, PR>(qr, dqr, T(-1), fp, get, 1, qrb, dqrb);
    side_pass_b<T, PR>(ql, dql, T(1), fp, get, 0, qlb, dqlb);
}

// reverse of side_state: local-frame state cotangents -> coefficient cotangents cb[50] (accumulated)
template <typename T>
__host__ __device__ __forceinline__ void side_state_b(T X, T Y, T Z, const T n[3][3], const T qb[5], const T dqb[3][5],
                                                      T cb[50])
{
    // q[1+k] = v . n_k; dq[m][1+k] = (g . n_m) . n_k
    T vb[5], gb[5][3];
    vb[0] = qb[0];
    vb[4] = qb[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) vb[1 + d] = qb[1] * n[0][d] + qb[2] * n[1][d] + qb[3] * n[2][d];
#pragma unroll
    for (int c = 0; c < 5; ++c) gb[c][0] = gb[c][1] = gb[c][2] = T(0);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T dnb[5];
        dnb[0] = dqb[m][0];
        dnb[4] = dqb[m][4];
#pragma unroll
        for (int d = 0; d < 3; ++d) dnb[1 + d] = dqb[m][1] * n[0][d] + dqb[m][2] * n[1][d] + dqb[m][3] * n[2][d];
#pragma unroll
        for (int c = 0; c < 5; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) gb[c][d] += dnb[c] * n[m][d];
    }
    const T XX = X * X, XY = X * Y, XZ = X * Z, YY = Y * Y, YZ = Y * Z, ZZ = Z * Z;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        T *cc = cb + 10 * c;
        cc[0] += vb[c];
        cc[1] += vb[c] * X + gb[c][0];
        cc[2] += vb[c] * Y + gb[c][1];
        cc[3] += vb[c] * Z + gb[c][2];
        cc[4] += vb[c] * XX + T(2) * X * gb[c][0];
        cc[5] += vb[c] * XY + Y * gb[c][0] + X * gb[c][1];
        cc[6] += vb[c] * XZ + Z * gb[c][0] + X * gb[c][2];
        cc[7] += vb[c] * YY + T(2) * Y * gb[c][1];
        cc[8] += vb[c] * YZ + Z * gb[c][1] + Y * gb[c][2];
        cc[9] += vb[c] * ZZ + T(2) * Z * gb[c][2];
    }
}

/*
 * Reverse of face_gp (FP64): out_b[10] -> cotangents of the owner's and the
 * neighbour's 50 coefficients (accumulated into clb, crb).
 */
template <typename T, bool PR>
__host__ __device__ void face_gp_b(const T *__restrict__ cl, const T *__restrict__ cr, const T geo[9], T dt,
                                   const FluxParams<T> &fp, const T outb[10], T clb[50], T crb[50])
{
    T n3[3][3];
    const T area = local_frame(geo[6], geo[7], geo[8], n3);
    T ql[5], qr[5], dql[3][5], dqr[3][5];
    side_state(cl, nullptr, geo[0], geo[1], geo[2], n3, ql, dql);
    side_state(cr, nullptr, geo[3], geo[4], geo[5], n3, qr, dqr);
    T Fb[10];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        Fb[5 * s] = area * outb[5 * s];
        Fb[5 * s + 4] = area * outb[5 * s + 4];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Fb[5 * s + 1 + k] =
                area * (outb[5 * s + 1] * n3[k][0] + outb[5 * s + 2] * n3[k][1] + outb[5 * s + 3] * n3[k][2]);
    }
    T qlb[5] = {T(0), T(0), T(0), T(0), T(0)}, qrb[5] = {T(0), T(0), T(0), T(0), T(0)};
    T dqlb[3][5], dqrb[3][5];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int j = 0; j < 5; ++j) dqlb[m][j] = dqrb[m][j] = T(0);
    gp_flux_b<T, PR>(ql, dql, qr, dqr, dt, fp, Fb, qlb, dqlb, qrb, dqrb);
    side_state_b(geo[0], geo[1], geo[2], n3, qlb, dqlb, clb);
    side_state_b(geo[3], geo[4], geo[5], n3, qrb, dqrb, crb);
}

}  // namespace gks
