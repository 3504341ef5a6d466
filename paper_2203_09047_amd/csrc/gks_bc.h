// Boundary conditions of the box planes of a mesh with walls.
//
// Section 2 of Yang, Pan & Xu (arXiv 2203.09047) builds stencils across a
// boundary from ghost cells: the ghost across a boundary face is the mirror
// image of an interior cell, and its flow variables are given by the boundary
// condition from that cell's.  Here every box plane (2 axis + hi: the plane
// x_axis = 0 or L) carries one condition:
//   reflective   normal momentum negated (the Riemann problems' walls);
//   no-slip      velocity U -> 2 u_w - U with rho and p kept (adiabatic wall moving at u_w);
//   isothermal   U -> 2 u_w - U, temperature T = p / rho -> 2 T_w - T, p kept (the cavity's walls);
//   far field    Riemann invariants U_n +- 2c / (gamma - 1) against a free stream (inlet/outlet);
//   extrapolate  the ghost repeats the mirrored cell (zero-gradient, non-reflecting ends).
// A stencil member mirrored across several planes takes their conditions in axis order.  At a face
// Gauss point on a plane, the state beyond it is the ghost field there: the condition applied to the
// inner reconstructed state, and the condition's derivative applied to the inner gradient with the
// derivative across the plane negated (the mirror); the far field's ghost is uniform.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace gks {

enum { kBcSlip = 0, kBcNoSlip = 1, kBcIsothermal = 2, kBcFarField = 3, kBcExtrapolate = 4 };

// conditions of the six planes in FP64 (the ghost cell averages of the reconstruction)
struct BoundarySet {
    int type[6];
    double uw[6][3];
    double Tw[6];
    double far[6][5];  // rho, U, V, W, p
    double gamma;
    int any_general;   // a plane whose condition is not the reflective one
};

// Subsonic/supersonic far-field state in a frame whose first axis is the outward normal: the interior
// (rho, U, p) and the free stream (rf, Uf, pf) give the boundary state (rb, Ub, pb).
template <typename T>
__host__ __device__ __forceinline__ void farfield_frame(T gam, T rho, const T U[3], T p, T rf, const T Uf[3], T pf,
                                                        T &rb, T Ub[3], T &pb)
{
    const T c = sqrt(gam * p / rho);
    const T cf = sqrt(gam * pf / rf);
    if (U[0] >= c) {  // supersonic outflow: the interior state
        rb = rho;
        pb = p;
        Ub[0] = U[0];
        Ub[1] = U[1];
        Ub[2] = U[2];
        return;
    }
    if (Uf[0] <= -cf) {  // supersonic inflow: the free stream
        rb = rf;
        pb = pf;
        Ub[0] = Uf[0];
        Ub[1] = Uf[1];
        Ub[2] = Uf[2];
        return;
    }
    const T g1 = gam - T(1);
    const T Rp = U[0] + T(2) * c / g1;    // carried out by the interior
    const T Rm = Uf[0] - T(2) * cf / g1;  // carried in by the free stream
    const T un = T(0.5) * (Rp + Rm);
    const T cb = T(0.25) * g1 * (Rp - Rm);
    T s;  // entropy p / rho^gamma and tangential velocity of the upwind side
    if (un > T(0)) {
        s = p / pow(rho, gam);
        Ub[1] = U[1];
        Ub[2] = U[2];
    } else {
        s = pf / pow(rf, gam);
        Ub[1] = Uf[1];
        Ub[2] = Uf[2];
    }
    Ub[0] = un;
    rb = pow(cb * cb / (gam * s), T(1) / g1);
    pb = rb * cb * cb / gam;
}

// one plane's condition on a cell average v (global frame, in place)
__host__ __device__ inline void bc_average(const BoundarySet &b, int plane, double v[5])
{
    const int d = plane >> 1;
    const int type = b.type[plane];
    if (type == kBcSlip) {
        v[1 + d] = -v[1 + d];
        return;
    }
    if (type == kBcExtrapolate) return;
    const double g = b.gamma;
    const double rho = v[0], ir = 1.0 / rho;
    double U[3] = {v[1] * ir, v[2] * ir, v[3] * ir};
    const double p = (g - 1.0) * (v[4] - 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    double rb, Ub[3], pb = p;
    if (type == kBcFarField) {
        // the frame (outward normal, the next two axes in cyclic order)
        const double sn = (plane & 1) ? 1.0 : -1.0;
        const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        const double Ul[3] = {sn * U[d], U[a1], U[a2]};
        const double *f = b.far[plane];
        const double Uf[3] = {sn * f[1 + d], f[1 + a1], f[1 + a2]};
        double Ubl[3];
        farfield_frame<double>(g, rho, Ul, p, f[0], Uf, f[4], rb, Ubl, pb);
        Ub[d] = sn * Ubl[0];
        Ub[a1] = Ubl[1];
        Ub[a2] = Ubl[2];
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) Ub[q] = 2.0 * b.uw[plane][q] - U[q];
        rb = type == kBcIsothermal ? p / (2.0 * b.Tw[plane] - p * ir) : rho;
    }
    v[0] = rb;
#pragma unroll
    for (int q = 0; q < 3; ++q) v[1 + q] = rb * Ub[q];
    v[4] = pb / (g - 1.0) + 0.5 * rb * (Ub[0] * Ub[0] + Ub[1] * Ub[1] + Ub[2] * Ub[2]);
}

// the cell average of a stencil member mirrored across the planes coded in flip (bit d: mirrored on
// axis d; bit 3 + d: at the plane x_d = L, else at 0)
__host__ __device__ inline void ghost_average(const BoundarySet &b, unsigned flip, double v[5])
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (flip >> d & 1u) bc_average(b, 2 * d + (int)(flip >> (3 + d) & 1u), v);
}

}  // namespace gks
