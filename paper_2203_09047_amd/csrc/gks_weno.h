// WENO combination of one cell and conserved component (Section 2, Eq. weno,
// Eq. indicator), after the stencil sums, and its hand-written reverse.
//
// Inputs: a[9], the least-squares quadratic's coefficients of the monomials
// x y z xx xy xz yy yz zz of (x - x_c); b[m][3], the linear polynomial of
// sub-stencil m, formed by the caller as b^m = gi[m] r[m] from the sums
// r[m] = sum_{k in S_m} D_k (Q_k - Q_0) (D_k the member's centroid offset scaled
// by h) and gi[m], the symmetric inverse of sum_{k in S_m} D_k D_k^T divided by
// h (sym3_apply).  The smoothness indicators are
// integrated over the cell with its centred second moments S (xx xy xz yy yz
// zz) and v23 = |Omega|^(2/3); the nonlinear weights use tau_w = mean |beta_0 -
// beta_m|; the nonlinear combination of Eq. weno is folded into one quadratic
// c[1..9], and c[0] = q0 - sum_n c_n (mean of monomial n over the cell).
#pragma once

#include <hip/hip_runtime.h>

namespace gks {

struct WenoParams {
    double eps, gm, p;
    int force_linear;
};

template <typename T>
__host__ __device__ __forceinline__ T wpow(T x, T p)
{
    if (p == T(1)) return x;
    if (p == T(2)) return x * x;
    return (T)pow((double)x, (double)p);
}

template <typename T>
__host__ __device__ __forceinline__ T wabs(T x)
{
    return x < T(0) ? -x : x;
}

template <typename T>
__host__ __device__ __forceinline__ T wsgn(T x)
{
    return x > T(0) ? T(1) : (x < T(0) ? T(-1) : T(0));
}

// b^m = gi[m] r[m] for a symmetric gi stored as xx xy xz yy yz zz
template <typename T>
__host__ __device__ __forceinline__ void sym3_apply(const T g[6], const T r[3], T b[3])
{
    b[0] = g[0] * r[0] + g[1] * r[1] + g[2] * r[2];
    b[1] = g[1] * r[0] + g[3] * r[1] + g[4] * r[2];
    b[2] = g[2] * r[0] + g[4] * r[1] + g[5] * r[2];
}

// forward from the linear polynomials b[m]; q0 enters only c[0] (c[0] excludes it when with_q0 is false)
template <typename T>
__host__ __device__ __forceinline__ void weno_combine(const T a[9], const T b[8][3], int M, T v23, const T S[6],
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
    T beta[8];
    T tw = T(0);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        beta[s] = v23 * (b[s][0] * b[s][0] + b[s][1] * b[s][1] + b[s][2] * b[s][2]);
        if (s < M) tw += wabs(beta0 - beta[s]);
    }
    tw /= T(M);
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
    const T corr = -(c[4] * S[0] + c[5] * S[1] + c[6] * S[2] + c[7] * S[3] + c[8] * S[4] + c[9] * S[5]);
    c[0] = with_q0 ? (T)q0 + corr : corr;
}

/*
 * Reverse of weno_combine composed with b^m = gi[m] r[m] (FP64 adjoint):
 * cb[10] -> ab[9], rb[8][3] (overwritten) and q0b (the direct dependence of
 * c[0] on the cell average).  getg(m, g) loads gi[m].  The per-sub-stencil
 * quantities are recomputed in four streaming passes over m instead of being
 * held in arrays, which keeps the live state small.
 */
template <typename T, typename GetG>
__host__ __device__ __forceinline__ void weno_combine_b(const T a[9], const T r[8][3], GetG getg, int M, T v23,
                                                        const T S[6], const WenoParams &wp, const T cb_in[10], T ab[9],
                                                        T rb[8][3], T &q0b)
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
    const bool lin = wp.force_linear != 0;
    auto slot = [&](int s, T b[3], T &beta) {
        T g[6];
        getg(s, g);
        sym3_apply(g, r[s], b);
        beta = v23 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    };
    // pass A: tau_w and the weights' sum
    T tw = T(0);
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (s < M) {
            T b[3], beta;
            slot(s, b, beta);
            tw += wabs(beta0 - beta);
        }
    tw /= T(M);
    const T x0 = lin ? T(0) : tw / (beta0 + eps);
    const T w0 = lin ? g0 : g0 * (T(1) + wpow(x0, pw));
    T sum = w0;
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (s < M) {
            T b[3], beta;
            slot(s, b, beta);
            sum += lin ? gm : gm * (T(1) + wpow(tw / (beta + eps), pw));
        }
    const T isum = T(1) / sum;
    const T f0 = w0 * isum / g0;
    const T sub0 = f0 * gm;
    auto wslot = [&](T beta, T &xs) {
        xs = lin ? T(0) : tw / (beta + eps);
        return lin ? gm : gm * (T(1) + wpow(xs, pw));
    };
    // reverse of c[0] = q0 - sum c_n S_n and of c[1 + j] = f0 a_j
    T cb[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) cb[j] = cb_in[j];
    q0b += cb[0];
#pragma unroll
    for (int q = 0; q < 6; ++q) cb[4 + q] += -S[q] * cb[0];
    T f0b = T(0);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        ab[j] = f0 * cb[1 + j];
        f0b += a[j] * cb[1 + j];
    }
    // pass B: contributions of c[1..3] += f_m b^m to f0 and to the sum
    T sumb = T(0);
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (s < M) {
            T b[3], beta, xs;
            slot(s, b, beta);
            const T ws = wslot(beta, xs);
            const T fsb = b[0] * cb[1] + b[1] * cb[2] + b[2] * cb[3];
            sumb += -fsb * ws * isum * isum;
            f0b += -fsb * gm;
            (void)xs;
        }
    sumb += -f0b * w0 * isum * isum / g0;
    const T w0b = f0b * isum / g0 + sumb;
    // pass C: tau_w cotangent
    T twb = T(0), beta0b = T(0);
    if (!lin) {
        const T dp0 = pw == T(1) ? T(1) : pw * wpow(x0, pw - T(1));
        const T x0b = w0b * g0 * dp0;
        twb += x0b / (beta0 + eps);
        beta0b += -x0b * x0 / (beta0 + eps);
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s < M) {
                T b[3], beta, xs;
                slot(s, b, beta);
                const T ws = wslot(beta, xs);
                (void)ws;
                const T fsb = b[0] * cb[1] + b[1] * cb[2] + b[2] * cb[3];
                const T wsb = fsb * isum + sumb;
                const T dps = pw == T(1) ? T(1) : pw * wpow(xs, pw - T(1));
                twb += wsb * gm * dps / (beta + eps);
            }
    }
    twb /= T(M);
    // pass D: each sub-stencil's cotangents
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        if (s < M) {
            T b[3], beta, xs;
            slot(s, b, beta);
            const T ws = wslot(beta, xs);
            const T fs = ws * isum - sub0;
            const T fsb = b[0] * cb[1] + b[1] * cb[2] + b[2] * cb[3];
            const T wsb = fsb * isum + sumb;
            T betab = T(0);
            if (!lin) {
                const T dps = pw == T(1) ? T(1) : pw * wpow(xs, pw - T(1));
                betab += -wsb * gm * dps * xs / (beta + eps);
            }
            const T sg = wsgn(beta0 - beta);
            beta0b += twb * sg;
            betab += -twb * sg;
            T bb[3], g[6];
#pragma unroll
            for (int q = 0; q < 3; ++q) bb[q] = fs * cb[1 + q] + T(2) * v23 * betab * b[q];
            getg(s, g);
            sym3_apply(g, bb, rb[s]);
        } else {
            rb[s][0] = rb[s][1] = rb[s][2] = T(0);
        }
    }
    // beta0 = v23 sum_d (a_d^2 + H_d S H_d) + v23^2 sec
    const T g1 = v23 * beta0b, g2 = v23 * v23 * beta0b;
#pragma unroll
    for (int d = 0; d < 3; ++d) ab[d] += T(2) * g1 * a[d];
    T Hb[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            T t = T(0);
#pragma unroll
            for (int q = 0; q < 3; ++q) t += Sm[p][q] * H[d][q];
            Hb[d][p] = T(2) * g1 * t;
        }
    ab[3] += T(2) * Hb[0][0] + T(8) * g2 * a[3];
    ab[4] += Hb[0][1] + Hb[1][0] + T(2) * g2 * a[4];
    ab[5] += Hb[0][2] + Hb[2][0] + T(2) * g2 * a[5];
    ab[6] += T(2) * Hb[1][1] + T(8) * g2 * a[6];
    ab[7] += Hb[1][2] + Hb[2][1] + T(2) * g2 * a[7];
    ab[8] += T(2) * Hb[2][2] + T(8) * g2 * a[8];
}

}  // namespace gks
