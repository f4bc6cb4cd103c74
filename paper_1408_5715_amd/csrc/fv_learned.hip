// The step with a learned correction of the face flux (an addition to the
// paper's scheme; the Lax-Friedrichs flux and the update are those of
// section 6.2.2).
//
// Per face (left = the cell, right = the neighbour, n the length-scaled
// normal, e = n / |n|, t = (-e_y, e_x)) a small MLP y(x) = W3^T h2 + b3,
// h2 = s(W2^T h1 + b2), h1 = s(W1^T x + b1), s(z) = z / (1 + |z|), reads 12
// features x(L, R, n) = [rho_L - 1, un_L, ut_L, p_L - 1, rho_R - 1, un_R,
// ut_R, p_R - 1, e_x, e_y, l^2 (a_L + a_R) / 2, l (c_L + c_R) / 2] (a = 1/V,
// c = dt/V).  The face flux becomes
//   G = G_LF + l (R(e) y(x(L, R, n)) - R(-e) y(x(R, L, -n))),
// R(e) y = (y0, y1 e_x + y2 t_x, y1 e_y + y2 t_y, y3).  Both cells of a face
// evaluate the same two MLP rows from bit-identical inputs with the same
// code, so the correction is exactly antisymmetric and conservation holds to
// round-off.  Features, activations and weights are bfloat16, products are
// summed in float32 (MFMA), the flux and the update stay float64.
//
// MFMA mapping (v_mfma_f32_16x16x16_bf16, wave64).  Weights are the A
// operand (rows = output units, 16 per tile) and 16 MLP rows (faces) the B
// operand (columns).  The accumulator of an output tile holds, in lane l,
// units 4 (l / 16) + i of face column l % 16, which is exactly the B operand
// layout of the next layer's K-slice: layers chain in registers.  Per 16
// faces: 4 + 16 + 4 MFMAs.  A wave owns 64 cells, i.e. 6 x 64 rows; their
// features and outputs pass through LDS between the per-cell float64 code
// and the MLP.  Weight fragments stay in registers for the whole persistent
// workgroup.

#include <cstring>

#include "fv_internal.h"

namespace fvk {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;
constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kRows = 6;             // MLP rows per cell: 3 faces x 2 orientations
constexpr int kCellStride = 100;     // bf16 per cell in LDS (6 x 16, padded against bank conflicts)

__device__ __forceinline__ double recip(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ double root(double a)
{
    double r = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    r = r * fma(-h * r, r, 1.5);
    r = r * fma(-h * r, r, 1.5);
    const double s = a * r;
    const double e = fma(-s, s, a);
    const double q = fma(e, 0.5 * r, s);
    return a == 0.0 ? 0.0 : q;
}

// float -> bfloat16 bits, round to nearest even (no NaN inputs here).
__device__ __forceinline__ short bf16_bits(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float softsign(float z)
{
    return z / (1.0f + fabsf(z));
}

struct Side {
    double rho, u, v, p, c;
};

__device__ __forceinline__ Side side_of(const double4 &U, double gamma)
{
    Side s;
    const double ir = recip(U.x);
    s.rho = U.x;
    s.u = U.y * ir;
    s.v = U.z * ir;
    s.p = (gamma - 1.0) * (U.w - 0.5 * (U.y * U.y + U.z * U.z) * ir);
    s.c = root(gamma * s.p * ir);
    return s;
}

// Features of the row (L, R, unit normal e), rounded to bfloat16 and written
// as 16 shorts (12 features + 4 zeros).
__device__ __forceinline__ void write_features(short *dst, const Side &L, const Side &R, double ex,
                                               double ey, double geo_a, double geo_c)
{
    const double tx = -ey, ty = ex;
    const double f[12] = {L.rho - 1.0,           L.u * ex + L.v * ey, L.u * tx + L.v * ty,
                          L.p - 1.0,             R.rho - 1.0,         R.u * ex + R.v * ey,
                          R.u * tx + R.v * ty,   R.p - 1.0,           ex,
                          ey,                    geo_a,               geo_c};
#pragma unroll
    for (int k = 0; k < 12; ++k)
        dst[k] = bf16_bits((float)f[k]);
#pragma unroll
    for (int k = 12; k < 16; ++k)
        dst[k] = 0;
}

// R(e) y in float64
__device__ __forceinline__ void rotate(const float y[4], double ex, double ey, double out[4])
{
    const double tx = -ey, ty = ex;
    const double y1 = y[1], y2 = y[2];
    out[0] = y[0];
    out[1] = y1 * ex + y2 * tx;
    out[2] = y1 * ey + y2 * ty;
    out[3] = y[3];
}

template <bool kNarrow>
__device__ __forceinline__ int neighbour(int i, int f, int32_t ld, const int32_t *nb,
                                         const short4 *nb16)
{
    if constexpr (kNarrow) {
        const short4 o = nb16[i];
        return i + (f == 0 ? o.x : (f == 1 ? o.y : o.z));
    } else {
        return nb[f * ld + i];
    }
}

template <bool kClosed>
__device__ __forceinline__ void normal(int i, int f, int32_t ld, const double *nrm, double &nx,
                                       double &ny)
{
    if (kClosed && f == 2) {
        nx = -(nrm[i] + nrm[2 * ld + i]);
        ny = -(nrm[ld + i] + nrm[3 * ld + i]);
    } else {
        nx = nrm[2 * f * ld + i];
        ny = nrm[(2 * f + 1) * ld + i];
    }
}

template <bool kNarrow, bool kClosed>
__global__ __launch_bounds__(kBlock) void fv_step_learned_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, double4 *__restrict__ Un,
    const int32_t *__restrict__ nb, const short4 *__restrict__ nb16,
    const double *__restrict__ nrm, const double *__restrict__ coef,
    const double *__restrict__ inv_area, const s4 *__restrict__ frags,
    const float *__restrict__ bias, double gamma)
{
    __shared__ short X[kWaves][64 * kCellStride];
    __shared__ float Y[kWaves][64 * kRows * 4];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int quad = lane >> 4, col = lane & 15;

    // weight fragments (A operands) and biases of this lane, kept for all tiles
    s4 w1[4], w2[16], w3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        w1[t] = frags[t * 64 + lane];
#pragma unroll
    for (int t = 0; t < 16; ++t)
        w2[t] = frags[(4 + t) * 64 + lane];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        w3[t] = frags[(20 + t) * 64 + lane];
    float b1[16], b2[16], b3[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b1[4 * mt + i] = bias[16 * mt + 4 * quad + i];
            b2[4 * mt + i] = bias[64 + 16 * mt + 4 * quad + i];
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        b3[i] = quad == 0 ? bias[128 + i] : 0.0f;

    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = gridDim.x, b = blockIdx.x;
    const int X_ = G < kXcds ? G : kXcds;
    const int x = b % X_, k = b / X_;
    const int Px = (G - x + X_ - 1) / X_;
    const int t0 = (int)((long long)tiles * x / X_), t1 = (int)((long long)tiles * (x + 1) / X_);

    for (int tile = t0 + k; tile < t1; tile += Px) {
        const int i = tile * kBlock + threadIdx.x;
        const bool live = i < n;
        short *xs = &X[wave][lane * kCellStride];

        // 1. features of the six rows of this cell
        if (live) {
            const double4 Ui = U[i];
            const Side L = side_of(Ui, gamma);
            const double ai = inv_area[i], ci = coef[i];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const int j = neighbour<kNarrow>(i, f, ld, nb, nb16);
                double nx, ny;
                normal<kClosed>(i, f, ld, nrm, nx, ny);
                const Side R = side_of(U[j], gamma);
                const double len = root(nx * nx + ny * ny);
                const double ex = nx / len, ey = ny / len;
                const double aj = inv_area[j], cj = coef[j];
                const double geo_a = 0.5 * len * len * (ai + aj);
                const double geo_c = 0.5 * len * (ci + cj);
                const double geo_a_r = 0.5 * len * len * (aj + ai);
                const double geo_c_r = 0.5 * len * (cj + ci);
                write_features(xs + 16 * (2 * f), L, R, ex, ey, geo_a, geo_c);
                write_features(xs + 16 * (2 * f + 1), R, L, -ex, -ey, geo_a_r, geo_c_r);
            }
        } else {
#pragma unroll
            for (int q = 0; q < kRows * 16; ++q)
                xs[q] = 0;
        }
        __syncthreads();

        // 2. MLP on MFMA: 4 groups of 16 cells x 6 row kinds
        for (int g = 0; g < 4; ++g) {
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const s4 xb = *reinterpret_cast<const s4 *>(
                    &X[wave][(16 * g + col) * kCellStride + 16 * r + 4 * quad]);
                s4 h1[4];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[mt], xb, acc, 0, 0, 0);
                    s4 hb;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        hb[q] = bf16_bits(softsign(acc[q] + b1[4 * mt + q]));
                    h1[mt] = hb;
                }
                s4 h2[4];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks)
                        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w2[4 * mt + ks], h1[ks], acc,
                                                                         0, 0, 0);
                    s4 hb;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        hb[q] = bf16_bits(softsign(acc[q] + b2[4 * mt + q]));
                    h2[mt] = hb;
                }
                f4 yv = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    yv = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w3[ks], h2[ks], yv, 0, 0, 0);
                if (quad == 0) {
                    float *dst = &Y[wave][((16 * g + col) * kRows + r) * 4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        dst[q] = yv[q] + b3[q];
                }
            }
        }
        __syncthreads();

        // 3. flux, correction and update in float64
        if (live) {
            const double4 Ui = U[i];
            const Side L = side_of(Ui, gamma);
            const float *ys = &Y[wave][lane * kRows * 4];
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const int j = neighbour<kNarrow>(i, f, ld, nb, nb16);
                double nx, ny;
                normal<kClosed>(i, f, ld, nrm, nx, ny);
                const double4 Uj = U[j];
                const Side R = side_of(Uj, gamma);
                const double len = root(nx * nx + ny * ny);
                const double VL = L.u * nx + L.v * ny;
                const double VR = R.u * nx + R.v * ny;
                const double s = fabs(0.5 * (VL + VR)) + 0.5 * len * (L.c + R.c);
                const double pp = L.p + R.p;
                const double ex = nx / len, ey = ny / len;
                float yA[4], yB[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    yA[q] = ys[(2 * f) * 4 + q];
                    yB[q] = ys[(2 * f + 1) * 4 + q];
                }
                double A[4], B[4];
                rotate(yA, ex, ey, A);
                rotate(yB, -ex, -ey, B);
                const double g0 = 0.5 * (Ui.x * VL + Uj.x * VR) - 0.5 * s * (Uj.x - Ui.x);
                const double g1 = 0.5 * (Ui.y * VL + Uj.y * VR + pp * nx) - 0.5 * s * (Uj.y - Ui.y);
                const double g2 = 0.5 * (Ui.z * VL + Uj.z * VR + pp * ny) - 0.5 * s * (Uj.z - Ui.z);
                const double g3 =
                    0.5 * ((Ui.w + L.p) * VL + (Uj.w + R.p) * VR) - 0.5 * s * (Uj.w - Ui.w);
                a0 += g0 + len * (A[0] - B[0]);
                a1 += g1 + len * (A[1] - B[1]);
                a2 += g2 + len * (A[2] - B[2]);
                a3 += g3 + len * (A[3] - B[3]);
            }
            const double kk = coef[i];
            double4 out;
            out.x = Ui.x - kk * a0;
            out.y = Ui.y - kk * a1;
            out.z = Ui.z - kk * a2;
            out.w = Ui.w - kk * a3;
            Un[i] = out;
        }
        __syncthreads();
    }
}

inline unsigned short host_bf16(float x)
{
    unsigned u;
    memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

}  // namespace

void pack_correction(const float *params, short *frags, float *bias)
{
    // params: W1 [12][64], b1 [64], W2 [64][64], b2 [64], W3 [64][4], b3 [4]
    const float *W1 = params, *b1 = W1 + 12 * 64, *W2 = b1 + 64, *b2 = W2 + 64 * 64;
    const float *W3 = b2 + 64, *b3 = W3 + 64 * 4;
    auto put = [&](int frag, int lane, int j, float v) {
        frags[(frag * 64 + lane) * 4 + j] = (short)host_bf16(v);
    };
    for (int lane = 0; lane < 64; ++lane) {
        const int quad = lane >> 4, col = lane & 15;
        for (int j = 0; j < 4; ++j) {
            for (int mt = 0; mt < 4; ++mt) {
                const int kin = 4 * quad + j, m = 16 * mt + col;
                put(mt, lane, j, kin < 12 ? W1[kin * 64 + m] : 0.0f);
                for (int ks = 0; ks < 4; ++ks)
                    put(4 + 4 * mt + ks, lane, j, W2[(16 * ks + 4 * quad + j) * 64 + m]);
            }
            for (int ks = 0; ks < 4; ++ks)
                put(20 + ks, lane, j, col < 4 ? W3[(16 * ks + 4 * quad + j) * 4 + col] : 0.0f);
        }
    }
    for (int m = 0; m < 64; ++m) {
        bias[m] = b1[m];
        bias[64 + m] = b2[m];
    }
    for (int m = 0; m < 16; ++m)
        bias[128 + m] = m < 4 ? b3[m] : 0.0f;
}

hipError_t launch_step_learned(int32_t n, int32_t ld, const double4 *U, double4 *Un,
                               const int32_t *nb, const short4 *nb16, const double *nrm,
                               const double *coef, const double *inv_area, const short *frags,
                               const float *bias, double gamma, bool narrow, bool closed, int grid,
                               hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = (grid <= 0 || grid > tiles) ? (tiles < 2048 ? tiles : 2048) : grid;
    const s4 *fr = reinterpret_cast<const s4 *>(frags);
    if (narrow && closed)
        hipLaunchKernelGGL((fv_step_learned_kernel<true, true>), dim3(G), dim3(kBlock), 0, s, n, ld,
                           U, Un, nb, nb16, nrm, coef, inv_area, fr, bias, gamma);
    else if (narrow)
        hipLaunchKernelGGL((fv_step_learned_kernel<true, false>), dim3(G), dim3(kBlock), 0, s, n,
                           ld, U, Un, nb, nb16, nrm, coef, inv_area, fr, bias, gamma);
    else if (closed)
        hipLaunchKernelGGL((fv_step_learned_kernel<false, true>), dim3(G), dim3(kBlock), 0, s, n,
                           ld, U, Un, nb, nb16, nrm, coef, inv_area, fr, bias, gamma);
    else
        hipLaunchKernelGGL((fv_step_learned_kernel<false, false>), dim3(G), dim3(kBlock), 0, s, n,
                           ld, U, Un, nb, nb16, nrm, coef, inv_area, fr, bias, gamma);
    return hipGetLastError();
}

}  // namespace fvk
