// Forward-mode dual numbers for the Jacobian of the Lax-Friedrichs face flux
// (section 6.2.2) with respect to the left (own) state, shared by the
// adjoint kernels.  A Dual carries a value and its partial derivatives with
// respect to the four conserved variables of the left cell.
#pragma once

#include <hip/hip_runtime.h>

namespace fvk {
namespace dual {

struct Dual {
    double v;
    double d[4];
};

__device__ __forceinline__ Dual cst(double v)
{
    return {v, {0.0, 0.0, 0.0, 0.0}};
}
__device__ __forceinline__ Dual operator+(const Dual &a, const Dual &b)
{
    return {a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2], a.d[3] + b.d[3]}};
}
__device__ __forceinline__ Dual operator-(const Dual &a, const Dual &b)
{
    return {a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2], a.d[3] - b.d[3]}};
}
__device__ __forceinline__ Dual operator*(const Dual &a, const Dual &b)
{
    Dual r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ __forceinline__ Dual operator*(double s, const Dual &a)
{
    return {s * a.v, {s * a.d[0], s * a.d[1], s * a.d[2], s * a.d[3]}};
}
__device__ __forceinline__ Dual recip(const Dual &a)
{
    const double r = 1.0 / a.v;
    const double g = -r * r;
    return {r, {g * a.d[0], g * a.d[1], g * a.d[2], g * a.d[3]}};
}
__device__ __forceinline__ Dual dsqrt(const Dual &a)
{
    const double s = sqrt(a.v);
    const double g = 0.5 / s;
    return {s, {g * a.d[0], g * a.d[1], g * a.d[2], g * a.d[3]}};
}
__device__ __forceinline__ Dual dabs(const Dual &a)
{
    return a.v < 0.0 ? -1.0 * a : a;
}

// Lax-Friedrichs flux through a face times its length, in the frame-free
// form of the step kernel, on dual numbers for the left state.
__device__ __forceinline__ void flux_dual(const Dual UL[4], const double UR[4], double nx,
                                          double ny, double gamma, Dual F[4])
{
    const Dual irL = recip(UL[0]);
    const Dual uL = UL[1] * irL, vL = UL[2] * irL;
    const Dual pL = (gamma - 1.0) * (UL[3] - 0.5 * ((UL[1] * UL[1] + UL[2] * UL[2]) * irL));
    const Dual cL = dsqrt(gamma * (pL * irL));

    const double irR = 1.0 / UR[0];
    const double uR = UR[1] * irR, vR = UR[2] * irR;
    const double pR = (gamma - 1.0) * (UR[3] - 0.5 * (UR[1] * UR[1] + UR[2] * UR[2]) * irR);
    const double cR = sqrt(gamma * pR * irR);

    const double len = sqrt(nx * nx + ny * ny);
    const Dual VL = uL * cst(nx) + vL * cst(ny);
    const double VR = uR * nx + vR * ny;
    const Dual s = dabs(0.5 * (VL + cst(VR))) + (0.5 * len) * (cL + cst(cR));
    const Dual pp = pL + cst(pR);

    F[0] = 0.5 * (UL[0] * VL + cst(UR[0] * VR)) - 0.5 * (s * (cst(UR[0]) - UL[0]));
    F[1] = 0.5 * (UL[1] * VL + cst(UR[1] * VR) + pp * cst(nx)) - 0.5 * (s * (cst(UR[1]) - UL[1]));
    F[2] = 0.5 * (UL[2] * VL + cst(UR[2] * VR) + pp * cst(ny)) - 0.5 * (s * (cst(UR[2]) - UL[2]));
    F[3] = 0.5 * ((UL[3] + pL) * VL + cst((UR[3] + pR) * VR)) - 0.5 * (s * (cst(UR[3]) - UL[3]));
}

// acc += (dF / dU_L)^T v for the flux of the face (U_L, U_R, n).
__device__ __forceinline__ void flux_vjp(const double4 &UL, const double4 &UR, double nx, double ny,
                                         double gamma, const double v[4], double acc[4])
{
    const Dual L[4] = {{UL.x, {1, 0, 0, 0}}, {UL.y, {0, 1, 0, 0}}, {UL.z, {0, 0, 1, 0}},
                       {UL.w, {0, 0, 0, 1}}};
    const double R[4] = {UR.x, UR.y, UR.z, UR.w};
    Dual F[4];
    flux_dual(L, R, nx, ny, gamma, F);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        acc[q] += F[0].d[q] * v[0] + F[1].d[q] * v[1] + F[2].d[q] * v[2] + F[3].d[q] * v[3];
}

// c_k = dt * (1 / V_k) from the stored 1 / V_k, rounded exactly as the
// forward step forms it.
__device__ __forceinline__ double step_coef(double dt, double inv_area)
{
    return dt * inv_area;
}

}  // namespace dual
}  // namespace fvk
