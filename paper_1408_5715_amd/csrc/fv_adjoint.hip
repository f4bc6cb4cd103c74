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

#include "fv_dual.h"
#include "fv_internal.h"

namespace fvk {
namespace {

using namespace dual;

__global__ __launch_bounds__(256) void adjoint_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, const double4 *__restrict__ lam_next,
    double4 *__restrict__ lam, const int32_t *__restrict__ out_idx,
    const int32_t *__restrict__ nb, const double *__restrict__ nrm,
    const double *__restrict__ inv_area, double dt, double gamma)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    const double4 Uk = U[k];
    const double4 lk = lam_next[k];
    const double ck = step_coef(dt, inv_area[k]);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int j = nb[f * ld + k];
        const double nx = nrm[(2 * f) * ld + k], ny = nrm[(2 * f + 1) * ld + k];
        const double4 lj = lam_next[j];
        const double cj = step_coef(dt, inv_area[j]);
        const double v[4] = {ck * lk.x - cj * lj.x, ck * lk.y - cj * lj.y, ck * lk.z - cj * lj.z,
                             ck * lk.w - cj * lj.w};
        flux_vjp(Uk, U[j], nx, ny, gamma, v, acc);
    }
    double4 out;
    out.x = lk.x - acc[0];
    out.y = lk.y - acc[1];
    out.z = lk.z - acc[2];
    out.w = lk.w - acc[3];
    lam[out_idx[k]] = out;
}

}  // namespace

hipError_t launch_adjoint(int32_t n, int32_t ld, const double4 *U, const double4 *lam_next,
                          double4 *lam, const int32_t *out_idx, const int32_t *nb,
                          const double *nrm, const double *inv_area, double dt, double gamma,
                          hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(adjoint_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ld, U,
                       lam_next, lam, out_idx, nb, nrm, inv_area, dt, gamma);
    return hipGetLastError();
}

}  // namespace fvk
