// K3: permutation gathers and layout changes (the paper's section 3 moves
// the translation of global indices to the host, offline; here every
// per-cell array is permuted on the device instead).
//
// All kernels are gathers: thread l reads from a computed index and writes
// its own slot l, so no two threads write the same address.

#include <cmath>

#include "fv_internal.h"

namespace fvk {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t count)
{
    return (unsigned)((count + kBlock - 1) / kBlock);
}

__global__ void gather_geometry_kernel(int32_t n, int32_t ld, const int32_t *__restrict__ perm,
                                       const int32_t *__restrict__ label,
                                       const int32_t *__restrict__ nb_o,
                                       const double2 *__restrict__ nrm_o,
                                       const double *__restrict__ area_o,
                                       int32_t *__restrict__ nb_w, double *__restrict__ nrm_w,
                                       double *__restrict__ inv_area_w)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    const int v = perm[l];
    // the uploaded cell's neighbours (12 bytes) and normals (48 bytes) lie
    // together, so the scattered read touches one or two lines of each
#pragma unroll
    for (int f = 0; f < 3; ++f)
        nb_w[f * ld + l] = label[nb_o[3 * (int64_t)v + f]];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const double2 q = nrm_o[3 * (int64_t)v + f];
        nrm_w[(2 * f) * ld + l] = q.x;
        nrm_w[(2 * f + 1) * ld + l] = q.y;
    }
    inv_area_w[l] = 1.0 / area_o[v];
}

__global__ void gather_state_kernel(int32_t n, const int32_t *__restrict__ idx,
                                    const double4 *__restrict__ src, double4 *__restrict__ dst)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l < n)
        dst[l] = src[idx[l]];
}

__global__ void gather_state2_kernel(int32_t n, const int32_t *__restrict__ idx_a,
                                     const int32_t *__restrict__ idx_b,
                                     const double4 *__restrict__ src, double4 *__restrict__ dst)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l < n)
        dst[l] = src[idx_b[idx_a[l]]];
}

__global__ void check_state_kernel(int32_t n, const double4 *__restrict__ U, double gamma,
                                   int32_t *__restrict__ flag)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    const double4 u = U[l];
    const double p = (gamma - 1.0) * (u.w - 0.5 * (u.y * u.y + u.z * u.z) / u.x);
    const bool ok = isfinite(u.x) && isfinite(u.y) && isfinite(u.z) && isfinite(u.w) &&
                    u.x > 0.0 && isfinite(p) && p > 0.0;
    if (!ok)
        *flag = 1;  // every writer stores the same value
}

// Weighted gather: out[i] = sum_m w[i][m] src[idx[i][m]] (m in order); an
// index outside [0, n_src) makes out[i] NaN instead of being read.
__global__ void restrict_kernel(int64_t n, int32_t k, int64_t n_src, const double4 *__restrict__ src,
                                const int32_t *__restrict__ idx, const double *__restrict__ w,
                                double4 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    double4 a = {0.0, 0.0, 0.0, 0.0};
    bool ok = true;
    for (int32_t m = 0; m < k; ++m) {
        const int32_t j = idx[i * k + m];
        if (j < 0 || j >= n_src) {
            ok = false;
            continue;
        }
        const double wm = w[i * k + m];
        const double4 u = src[j];
        a.x += wm * u.x;
        a.y += wm * u.y;
        a.z += wm * u.z;
        a.w += wm * u.w;
    }
    if (!ok) {
        const double nan = __builtin_nan("");
        a = {nan, nan, nan, nan};
    }
    out[i] = a;
}

}  // namespace

hipError_t launch_restrict(int64_t n, int32_t k, int64_t n_src, const double4 *src,
                           const int32_t *idx, const double *w, double4 *out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(restrict_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, n, k, n_src, src, idx, w, out);
    return hipGetLastError();
}

hipError_t launch_gather_geometry(int32_t n, int32_t ld, const int32_t *perm, const int32_t *label,
                                  const int32_t *nb_o, const double *nrm_o, const double *area_o,
                                  int32_t *nb_w, double *nrm_w, double *inv_area_w, hipStream_t s)
{
    hipLaunchKernelGGL(gather_geometry_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ld, perm,
                       label, nb_o, reinterpret_cast<const double2 *>(nrm_o), area_o, nb_w, nrm_w,
                       inv_area_w);
    return hipGetLastError();
}

hipError_t launch_gather_state(int32_t n, const int32_t *idx, const double4 *src, double4 *dst,
                               hipStream_t s)
{
    hipLaunchKernelGGL(gather_state_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, idx, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_gather_state2(int32_t n, const int32_t *idx_a, const int32_t *idx_b,
                                const double4 *src, double4 *dst, hipStream_t s)
{
    hipLaunchKernelGGL(gather_state2_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, idx_a,
                       idx_b, src, dst);
    return hipGetLastError();
}

hipError_t launch_check_state(int32_t n, const double4 *U, double gamma, int32_t *flag,
                              hipStream_t s)
{
    hipLaunchKernelGGL(check_state_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, U, gamma,
                       flag);
    return hipGetLastError();
}

}  // namespace fvk
