// K1: one explicit cell-centred finite-volume step of the 2D Euler equations
// (section 6.2.2 of the paper: semi-discrete form eqSemiDiscrete, forward
// Euler eqFWEuler, Lax-Friedrichs flux eqCompFlux).
//
// One thread per cell.  The thread reads its own state, its three face
// normals, its inverse area and the three neighbour indices, gathers the
// three neighbour states and writes the updated state into the other buffer.
// Nothing is scattered and nothing is accumulated across threads, so the
// result of a cell depends only on its own inputs, in its own face order:
// the same bits whatever the cell numbering or the launch shape.
//
// The flux is evaluated without a face frame.  With n the length-scaled
// outward normal, V = u n_x + v n_y = |n| u_n, the face-frame flux rotated
// back and multiplied by |n| equals
//   (F(U_L) + F(U_R)) . n / 2 - (|V_L + V_R| / 2 + |n| (c_L + c_R) / 2) (U_R - U_L) / 2
// where F(U) . n = (rho V, rho u V + p n_x, rho v V + p n_y, (E + p) V):
// the rotation of the momentum jump back to x-y is the identity on U, so no
// unit normal (and no division by |n|) is needed.  This is an exact
// identity; only the rounding differs from the face-frame evaluation.

#include "fv_internal.h"

namespace fvk {
namespace {

// Workgroups are dealt round-robin to the 8 XCDs of the chip (each with its
// own L2).  Remap the hardware workgroup id so that every XCD walks one
// contiguous range of cells: neighbours of a band-ordered mesh then sit in
// the XCD's own L2 instead of being fetched by all eight.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_contiguous_block(int b, int nblocks)
{
    const int q = nblocks / kXcds, r = nblocks % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

struct Prim {
    double ir;  // 1 / rho
    double p;   // pressure
    double c;   // speed of sound
};

__device__ __forceinline__ Prim primitives(const double4 &U, double gamma)
{
    Prim q;
    q.ir = 1.0 / U.x;
    // p = (gamma - 1) (E - rho |v|^2 / 2) with rho |v|^2 = (m_x^2 + m_y^2) / rho
    q.p = (gamma - 1.0) * (U.w - 0.5 * (U.y * U.y + U.z * U.z) * q.ir);
    q.c = sqrt(gamma * q.p * q.ir);
    return q;
}

__global__ __launch_bounds__(kStepBlock) void fv_step_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, double4 *__restrict__ Un,
    const int32_t *__restrict__ nb, const double *__restrict__ nrm,
    const double *__restrict__ inv_area, double dt, double gamma)
{
    const int blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int i = blk * kStepBlock + threadIdx.x;
    if (i >= n)
        return;

    const double4 Ui = U[i];
    const Prim L = primitives(Ui, gamma);
    const double uL = Ui.y * L.ir, vL = Ui.z * L.ir;

    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int j = nb[f * ld + i];
        const double nx = nrm[(2 * f) * ld + i];
        const double ny = nrm[(2 * f + 1) * ld + i];
        const double4 Uj = U[j];
        const Prim R = primitives(Uj, gamma);
        const double uR = Uj.y * R.ir, vR = Uj.z * R.ir;

        const double len = sqrt(nx * nx + ny * ny);
        const double VL = uL * nx + vL * ny;
        const double VR = uR * nx + vR * ny;
        // |n| (|u_n bar| + c bar)
        const double s = fabs(0.5 * (VL + VR)) + 0.5 * len * (L.c + R.c);
        const double pp = L.p + R.p;

        a0 += 0.5 * (Ui.x * VL + Uj.x * VR) - 0.5 * s * (Uj.x - Ui.x);
        a1 += 0.5 * (Ui.y * VL + Uj.y * VR + pp * nx) - 0.5 * s * (Uj.y - Ui.y);
        a2 += 0.5 * (Ui.z * VL + Uj.z * VR + pp * ny) - 0.5 * s * (Uj.z - Ui.z);
        a3 += 0.5 * ((Ui.w + L.p) * VL + (Uj.w + R.p) * VR) - 0.5 * s * (Uj.w - Ui.w);
    }

    const double k = dt * inv_area[i];
    double4 out;
    out.x = Ui.x - k * a0;
    out.y = Ui.y - k * a1;
    out.z = Ui.z - k * a2;
    out.w = Ui.w - k * a3;
    Un[i] = out;
}

}  // namespace

hipError_t launch_step(int32_t n, int32_t ld, const double4 *U, double4 *Un, const int32_t *nb,
                       const double *nrm, const double *inv_area, double dt, double gamma,
                       hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int blocks = (n + kStepBlock - 1) / kStepBlock;
    hipLaunchKernelGGL(fv_step_kernel, dim3(blocks), dim3(kStepBlock), 0, s, n, ld, U, Un, nb,
                       nrm, inv_area, dt, gamma);
    return hipGetLastError();
}

}  // namespace fvk
