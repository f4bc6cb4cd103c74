// Adjoint (vector-Jacobian product) of one explicit step (section 6.2.2).
//
// The step is U'_k = U_k - c_k sum_f G(U_k, U_j(f), n_f) with c_k = dt / V_k
// and G the Lax-Friedrichs face flux times |n_f|.  G is antisymmetric across
// a face, G(U_j, U_k, -n) = -G(U_k, U_j, n), so cell k's state enters the
// update of a neighbour j only through the face they share, with the
// opposite sign.  For a cotangent lambda' of U' the cotangent of U is
//   lambda_k = lambda'_k - sum_f (dG(U_k, U_j, n_f)/dU_k)^T (c_k lambda'_k - c_j lambda'_j)
// where the Jacobian is taken with respect to the left (own) state only.
// Each cell gathers its neighbours' lambda' and c: gather-only, no atomics.
//
// The Jacobian of G is obtained exactly in forward mode: the flux is
// evaluated on dual numbers carrying the four partial derivatives with
// respect to U_k.

#include "fv_internal.h"

namespace fvk {
namespace {

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
// form (see fv_step.hip), on dual numbers for the left state.
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

// c_k = dt * (1 / V_k), rounded exactly as the forward step forms it.
__device__ __forceinline__ double step_coef(double dt, double area)
{
    return dt * (1.0 / area);
}

__global__ __launch_bounds__(256) void adjoint_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, const double4 *__restrict__ lam_next,
    double4 *__restrict__ lam, const int32_t *__restrict__ nb, const double *__restrict__ nrm,
    const double *__restrict__ area, double dt, double gamma)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    const double4 Uk = U[k];
    const double4 lk = lam_next[k];
    const double ck = step_coef(dt, area[k]);
    Dual UL[4] = {{Uk.x, {1, 0, 0, 0}}, {Uk.y, {0, 1, 0, 0}}, {Uk.z, {0, 0, 1, 0}},
                  {Uk.w, {0, 0, 0, 1}}};
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int j = nb[f * ld + k];
        const double nx = nrm[(2 * f) * ld + k], ny = nrm[(2 * f + 1) * ld + k];
        const double4 Uj = U[j];
        const double4 lj = lam_next[j];
        const double cj = step_coef(dt, area[j]);
        const double UR[4] = {Uj.x, Uj.y, Uj.z, Uj.w};
        Dual F[4];
        flux_dual(UL, UR, nx, ny, gamma, F);
        const double v[4] = {ck * lk.x - cj * lj.x, ck * lk.y - cj * lj.y, ck * lk.z - cj * lj.z,
                             ck * lk.w - cj * lj.w};
        // acc += J^T v, J[r][q] = dF_r / dU_q
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc[q] += F[0].d[q] * v[0] + F[1].d[q] * v[1] + F[2].d[q] * v[2] + F[3].d[q] * v[3];
    }
    double4 out;
    out.x = lk.x - acc[0];
    out.y = lk.y - acc[1];
    out.z = lk.z - acc[2];
    out.w = lk.w - acc[3];
    lam[k] = out;
}

}  // namespace

hipError_t launch_adjoint(int32_t n, int32_t ld, const double4 *U, const double4 *lam_next,
                          double4 *lam, const int32_t *nb, const double *nrm, const double *area,
                          double dt, double gamma, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(adjoint_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ld, U,
                       lam_next, lam, nb, nrm, area, dt, gamma);
    return hipGetLastError();
}

}  // namespace fvk
