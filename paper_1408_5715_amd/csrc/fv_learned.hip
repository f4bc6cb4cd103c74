// The step with a learned correction of the face flux (an addition to the
// paper's scheme; the Lax-Friedrichs flux and the update are those of
// section 6.2.2).
//
// Per face (left = the cell, right = the neighbour, n the length-scaled
// normal, e = n / |n|, t = (-e_y, e_x)) a small MLP y(x) = W3^T h2 + b3,
// h2 = relu(W2^T h1 + b2), h1 = relu(W1^T x + b1), reads 12 features
// x(L, R, n) = [rho_L - 1, un_L, ut_L, p_L - 1, rho_R - 1, un_R, ut_R,
// p_R - 1, e_x, e_y, l^2 (a_L + a_R) / 2, l (c_L + c_R) / 2] (a = 1/V,
// c = dt/V).  The face flux becomes
//   G = G_LF + l (R(e) y(x(L, R, n)) - R(-e) y(x(R, L, -n))),
// R(e) y = (y0, y1 e_x + y2 t_x, y1 e_y + y2 t_y, y3).  Both cells of a face
// evaluate the same two MLP rows from bit-identical inputs with the same
// code, so the correction is exactly antisymmetric and conservation holds to
// round-off.  Features, activations and weights are bfloat16, products are
// summed in float32 (MFMA), the flux and the update stay float64.
//
// MFMA mapping (wave64).  Weights are the A operand (rows = output units, 16
// per tile) and 16 MLP rows (faces) the B operand (columns).  The first
// layer's bias is a weight row against a constant-1 feature (so it is
// bfloat16 like the weights); the other biases are the accumulator input.
// The accumulator of an output tile holds, in lane l, units 4 (l / 16) + i of
// face column l % 16.  Two such tiles (units 32 s + 4 (l / 16) + i and
// 32 s + 16 + 4 (l / 16) + i) form lane l's eight K values of the next
// layer's v_mfma_f32_16x16x32_bf16 B operand; the weight fragments are packed
// in that K order, so layers chain in registers.  Per 16 rows: 4 (16x16x16,
// K = 12 padded to 16) + 8 + 2 (16x16x32) MFMAs.
//
// Work split: a wave owns 64 cells (lane = cell).  For each face slot f it
// computes, per cell, the Lax-Friedrichs flux and the two feature rows in
// float64, passes the 128 rows through LDS to the MLP, and adds the rotated
// outputs back.  Waves only exchange data with themselves (wave-scope
// synchronisation).  The packed weights are copied to LDS once per
// persistent workgroup and read into registers for each face slot's MLP.

#include <cstring>

#include "fv_dual.h"
#include "fv_internal.h"

namespace fvk {
namespace {

typedef short s2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kXcds = 8;
constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kXStride = 36;  // shorts per cell in LDS: 2 rows x 16 features + 4 (bank spread)
constexpr short kBf16One = 0x3f80;

// fragment offsets in shorts: W1 4 x 64 lanes x 4, W2 8 x 64 x 8, W3 2 x 64 x 8
constexpr int kFragW1 = 0;
constexpr int kFragW2 = 4 * 64 * 4;
constexpr int kFragW3 = kFragW2 + 8 * 64 * 8;
static_assert(kFragW3 + 2 * 64 * 8 == kCorrFragShorts, "fragment layout");

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

// Wave-scope ordering of LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// two floats -> two bfloat16 (round to nearest even), as 16-bit patterns
__device__ __forceinline__ s2 bf16x2(float a, float b)
{
    const f2 v = {a, b};
    return __builtin_bit_cast(s2, __builtin_convertvector(v, bf2));
}

// relu of an accumulator tile, rounded to bfloat16.  Rounding keeps the sign,
// so the max is taken on the bfloat16 patterns as 16-bit integers.
__device__ __forceinline__ s4 relu_bf16(f4 a)
{
    const s2 z = {0, 0};
    const s2 lo = __builtin_elementwise_max(bf16x2(a[0], a[1]), z);
    const s2 hi = __builtin_elementwise_max(bf16x2(a[2], a[3]), z);
    return s4{lo[0], lo[1], hi[0], hi[1]};
}

__device__ __forceinline__ bf8 join(s4 a, s4 b)
{
    const s8 v = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return __builtin_bit_cast(bf8, v);
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

// Features of the row (L, R, unit normal e) as 16 bfloat16: the 12 features
// (float64 -> float32 -> bfloat16, each rounding to nearest even), then a
// constant 1 that multiplies the first layer's bias, then zeros.  The 12 are
// returned as six packed pairs (element 0 in the low half): (rho_L, un_L),
// (ut_L, p_L), (rho_R, un_R), (ut_R, p_R), (e_x, e_y), (geo_a, geo_c).
struct FeaturePairs {
    unsigned p[6];
};

__device__ __forceinline__ unsigned pack_pair(float a, float b)
{
    const s2 v = bf16x2(a, b);
    return (unsigned)(unsigned short)v[0] | ((unsigned)(unsigned short)v[1] << 16);
}

__device__ __forceinline__ FeaturePairs features(const Side &L, const Side &R, double ex, double ey,
                                                 double geo_a, double geo_c)
{
    const double tx = -ey, ty = ex;
    FeaturePairs f;
    f.p[0] = pack_pair((float)(L.rho - 1.0), (float)(L.u * ex + L.v * ey));
    f.p[1] = pack_pair((float)(L.u * tx + L.v * ty), (float)(L.p - 1.0));
    f.p[2] = pack_pair((float)(R.rho - 1.0), (float)(R.u * ex + R.v * ey));
    f.p[3] = pack_pair((float)(R.u * tx + R.v * ty), (float)(R.p - 1.0));
    f.p[4] = pack_pair((float)ex, (float)ey);
    f.p[5] = pack_pair((float)geo_a, (float)geo_c);
    return f;
}

// One 16-value row (8-byte aligned) from six pairs: two 8-byte stores for the
// features, one for (e, geo), one for (1, 0, 0, 0).
__device__ __forceinline__ void store_row(short *dst, unsigned q0, unsigned q1, unsigned q2,
                                          unsigned q3, unsigned q4, unsigned q5)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    u2 *d = reinterpret_cast<u2 *>(dst);
    d[0] = u2{q0, q1};
    d[1] = u2{q2, q3};
    d[2] = u2{q4, q5};
    d[3] = u2{(unsigned)(unsigned short)kBf16One, 0u};
}

// The two rows of a face: x(L, R, e) at dstA and x(R, L, -e) at dstB.  The
// second is the first with the two cells' halves swapped and the signs of
// the normal and tangential velocities and of e flipped: each of those
// float64 values is the exact negation of its counterpart, and both roundings
// (to float32, then to bfloat16, nearest even) commute with negation, so
// flipping sign bits gives the patterns features(R, L, -e) would produce
// (up to the sign of an exact zero, which no sum in the MLP can observe).
__device__ __forceinline__ void write_feature_pair(short *dstA, short *dstB, const Side &L,
                                                   const Side &R, double ex, double ey,
                                                   double geo_a, double geo_c)
{
    const FeaturePairs f = features(L, R, ex, ey, geo_a, geo_c);
    store_row(dstA, f.p[0], f.p[1], f.p[2], f.p[3], f.p[4], f.p[5]);
    store_row(dstB, f.p[2] ^ 0x80000000u, f.p[3] ^ 0x00008000u, f.p[0] ^ 0x80000000u,
              f.p[1] ^ 0x00008000u, f.p[4] ^ 0x80008000u, f.p[5]);
}

// R(e) y in float64
__device__ __forceinline__ void rotate(const f4 &y, double ex, double ey, double out[4])
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
                                         const short4 *nb16, int nb16_stride)
{
    if constexpr (kNarrow) {
        const short4 o = nb16[(int64_t)nb16_stride * i];
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

// The MLP weights of one lane: A-operand fragments and accumulator-layout
// biases (the bias of output unit m sits at bias[m] of its layer).
struct Mlp {
    s4 w1[4];   // K = 12 features, the bias row, 3 zero rows
    bf8 w2[8];  // [output tile][K slice]
    bf8 w3[2];
    f4 b2[4], b3;
};

__device__ __forceinline__ void load_mlp(Mlp &W, const short *frags, const float *bias, int lane)
{
    const int quad = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        W.w1[t] = reinterpret_cast<const s4 *>(frags + kFragW1)[t * 64 + lane];
#pragma unroll
    for (int t = 0; t < 8; ++t)
        W.w2[t] = reinterpret_cast<const bf8 *>(frags + kFragW2)[t * 64 + lane];
#pragma unroll
    for (int t = 0; t < 2; ++t)
        W.w3[t] = reinterpret_cast<const bf8 *>(frags + kFragW3)[t * 64 + lane];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        W.b2[mt] = *reinterpret_cast<const f4 *>(&bias[64 + 16 * mt + 4 * quad]);
    }
    W.b3 = *reinterpret_cast<const f4 *>(&bias[128 + 4 * quad]);
}

// The MLP on the 128 rows of a wave (64 cells x 2 orientations) in X; the
// four outputs of row r of cell k go to Y[8 k + 4 r + 0..3].  The weights are
// read from the workgroup's LDS copy on every call rather than held across
// the float64 part of the step, which keeps the register count (and so the
// occupancy) at what the larger of the two phases needs.
__device__ __forceinline__ void mlp_rows(const short *Wl, const float *Bl, const short *X, float *Y,
                                         int lane)
{
    const int quad = lane >> 4, col = lane & 15;
    Mlp W;
    load_mlp(W, Wl, Bl, lane);
#pragma unroll 2
    for (int g = 0; g < 8; ++g) {
        const int cell = 16 * (g >> 1) + col, r = g & 1;
        const s4 xb = *reinterpret_cast<const s4 *>(&X[cell * kXStride + 16 * r + 4 * quad]);
        s4 h1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            h1[mt] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                W.w1[mt], xb, f4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0));
        const bf8 B0 = join(h1[0], h1[1]), B1 = join(h1[2], h1[3]);
        s4 h2[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w2[2 * mt], B0, W.b2[mt], 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w2[2 * mt + 1], B1, a, 0, 0, 0);
            h2[mt] = relu_bf16(a);
        }
        const bf8 C0 = join(h2[0], h2[1]), C1 = join(h2[2], h2[3]);
        f4 y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w3[0], C0, W.b3, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w3[1], C1, y, 0, 0, 0);
        if (quad == 0)
            *reinterpret_cast<f4 *>(&Y[cell * 8 + 4 * r]) = y;
    }
}

// Copy of the packed weights and biases into the workgroup's LDS.
__device__ __forceinline__ void stage_weights(short *Wl, float *Bl, const short *frags,
                                              const float *bias)
{
    for (int q = threadIdx.x; q < kCorrFragShorts / 8; q += blockDim.x)
        reinterpret_cast<s8 *>(Wl)[q] = reinterpret_cast<const s8 *>(frags)[q];
    for (int q = threadIdx.x; q < kCorrBias; q += blockDim.x)
        Bl[q] = bias[q];
    __syncthreads();
}

template <bool kNarrow, bool kClosed>
__global__ __launch_bounds__(kBlock, 3) void fv_step_learned_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, double4 *__restrict__ Un,
    const int32_t *__restrict__ nb, const short4 *__restrict__ nb16, int nb16_stride,
    const double *__restrict__ nrm, const double *__restrict__ coef,
    const double *__restrict__ inv_area, const short *__restrict__ frags,
    const float *__restrict__ bias, double gamma)
{
    __shared__ __attribute__((aligned(16))) short Xs[kWaves][64 * kXStride];
    __shared__ __attribute__((aligned(16))) float Ys[kWaves][64 * 8];
    __shared__ __attribute__((aligned(16))) short Wl[kCorrFragShorts];
    __shared__ __attribute__((aligned(16))) float Bl[kCorrBias];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    short *X = Xs[wave];
    float *Y = Ys[wave];
    stage_weights(Wl, Bl, frags, bias);

    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = gridDim.x, b = blockIdx.x;
    const int X_ = G < kXcds ? G : kXcds;
    const int x = b % X_, k = b / X_;
    const int Px = (G - x + X_ - 1) / X_;
    const int t0 = (int)((long long)tiles * x / X_), t1 = (int)((long long)tiles * (x + 1) / X_);

    for (int tile = t0 + k; tile < t1; tile += Px) {
        const int i = tile * kBlock + threadIdx.x;
        const bool live = i < n;
        short *xs = X + lane * kXStride;
        double4 Ui = {1.0, 0.0, 0.0, 2.5};
        double ai = 0.0, ci = 0.0;
        if (live) {
            Ui = U[i];
            ai = inv_area[i];
            ci = coef[i];
        }
        const Side L = side_of(Ui, gamma);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double len = 1.0, ex = 1.0, ey = 0.0;
            if (live) {
                const int j = neighbour<kNarrow>(i, f, ld, nb, nb16, nb16_stride);
                double nx, ny;
                normal<kClosed>(i, f, ld, nrm, nx, ny);
                const double4 Uj = U[j];
                const Side R = side_of(Uj, gamma);
                len = root(nx * nx + ny * ny);
                const double rl = recip(len);
                ex = nx * rl;
                ey = ny * rl;
                const double VL = L.u * nx + L.v * ny;
                const double VR = R.u * nx + R.v * ny;
                const double s = fabs(0.5 * (VL + VR)) + 0.5 * len * (L.c + R.c);
                const double pp = L.p + R.p;
                a0 += 0.5 * (Ui.x * VL + Uj.x * VR) - 0.5 * s * (Uj.x - Ui.x);
                a1 += 0.5 * (Ui.y * VL + Uj.y * VR + pp * nx) - 0.5 * s * (Uj.y - Ui.y);
                a2 += 0.5 * (Ui.z * VL + Uj.z * VR + pp * ny) - 0.5 * s * (Uj.z - Ui.z);
                a3 += 0.5 * ((Ui.w + L.p) * VL + (Uj.w + R.p) * VR) - 0.5 * s * (Uj.w - Ui.w);
                const double aj = inv_area[j], cj = coef[j];
                write_feature_pair(xs, xs + 16, L, R, ex, ey, 0.5 * len * len * (ai + aj),
                                   0.5 * len * (ci + cj));
            } else {
                s4 *d = reinterpret_cast<s4 *>(xs);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    d[q] = s4{0, 0, 0, 0};
            }
            wave_sync();
            mlp_rows(Wl, Bl, X, Y, lane);
            wave_sync();
            const f4 yA = *reinterpret_cast<const f4 *>(&Y[lane * 8]);
            const f4 yB = *reinterpret_cast<const f4 *>(&Y[lane * 8 + 4]);
            double A[4], B[4];
            rotate(yA, ex, ey, A);
            rotate(yB, -ex, -ey, B);
            a0 += len * (A[0] - B[0]);
            a1 += len * (A[1] - B[1]);
            a2 += len * (A[2] - B[2]);
            a3 += len * (A[3] - B[3]);
        }
        if (live) {
            double4 out;
            out.x = Ui.x - ci * a0;
            out.y = Ui.y - ci * a1;
            out.z = Ui.z - ci * a2;
            out.w = Ui.w - ci * a3;
            Un[i] = out;
        }
    }
}

// ---- adjoint of the corrected step ----------------------------------------
//
// For a cotangent lambda' of U' = U - c sum_f (G_LF + C_f) the cotangent of U
// is lambda_k = lambda'_k - sum_f (dPhi(U_k, U_j, n)/dU_k)^T v, v = c_k
// lambda'_k - c_j lambda'_j, Phi = G_LF + C (the face flux is antisymmetric,
// so cell k only needs its own faces; see fv_adjoint.hip).  With
// C = l (R(e) y_A - R(-e) y_B), y_A = y(x(k, j, n)), y_B = y(x(j, k, -n)):
//   (dC/dU_k)^T v = (dy_A/dU_k)^T w_A + (dy_B/dU_k)^T w_B,
//   w_A = l R(e)^T v = l (v0, v.e, v.t, v3),  w_B = -l R(-e)^T v = l (-v0, v.e, v.t, -v3).
// The MLP is run backwards on each row with its output cotangent w, giving
// dx; x_A depends on U_k through its features 0..3 (frame e), x_B through its
// features 4..7 (frame -e, which flips the signs of un and ut).
//
// Parameter gradient: dL/dtheta = -sum_k c_k lambda'_k . sum_f dC_f/dtheta.
// Every face appears from both of its cells with the same value of
// v . dC/dtheta (v and C both change sign), so
//   dL/dtheta = -1/2 sum_k sum_f (w_A . dy_A/dtheta + w_B . dy_B/dtheta):
// the same output cotangents as for lambda.  Rounding treats bfloat16 as the
// identity (straight through); relu' = 1 where the activation is positive.
//
// MFMA forms.  Besides the chain form of the forward kernel (units on the
// accumulator's 4-vector, rows on lanes: "C"), each pre-activation is also
// formed with the operands swapped (rows on the 4-vector, units on lanes:
// "G"), which is the operand layout of the weight-gradient products that
// contract over the 16 rows of a tile.  A lane's fragment of W as the A
// operand of W^T x equals its fragment of W as the B operand of x W, so one
// fragment set serves both forms.

// Adjoint fragment sets (shorts): W1e^T (x16), W2^T (x32) as in the forward
// kernel, then W3 as A (x16, [u][o]), W2 as A (x32, [u][o]), W1e as A (x32,
// [feature][u]); W1e = W1 with the bias row 12.
constexpr int kAF1 = 0;
constexpr int kAF2 = kAF1 + 4 * 64 * 4;
constexpr int kAF5 = kAF2 + 8 * 64 * 8;
constexpr int kAF6 = kAF5 + 4 * 64 * 4;
constexpr int kAF7 = kAF6 + 8 * 64 * 8;
static_assert(kAF7 + 2 * 64 * 8 == kCorrAdjFragShorts, "adjoint fragment layout");

constexpr int kWcStride = 8;  // bf16 cotangents per cell: row A (4), row B (4)

// Per-wave weight-gradient accumulators (float32).
struct GradAcc {
    f4 w1[4];   // [u tile]: rows = features 4 q + i, column = unit 16 t + l % 16
    f4 w2[16];  // [u tile][o tile]
    f4 w3[4];   // [u tile]: column = output l % 16 (< 4)
    float b2[4], b3;
};

__device__ __forceinline__ s4 ld_s4(const short *base, int frag, int lane)
{
    return reinterpret_cast<const s4 *>(base)[frag * 64 + lane];
}
__device__ __forceinline__ bf8 ld_bf8(const short *base, int frag, int lane)
{
    return reinterpret_cast<const bf8 *>(base)[frag * 64 + lane];
}

// keep a where the matching activation pattern is positive, then round to
// bfloat16
__device__ __forceinline__ s4 masked_bf16(f4 a, s4 h)
{
    f4 m;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        m[i] = h[i] > 0 ? a[i] : 0.0f;
    const s2 lo = bf16x2(m[0], m[1]), hi = bf16x2(m[2], m[3]);
    return s4{lo[0], lo[1], hi[0], hi[1]};
}

__device__ __forceinline__ float bf16_to_float(short b)
{
    return __uint_as_float((unsigned)(unsigned short)b << 16);
}

// The MLP backwards on the 128 rows of a wave: features in X, output
// cotangents in Wc (bfloat16), writes dx of features 0..3 of row A and 4..7
// of row B to DX[8 k + 0..7] and adds the weight gradients to acc.
__device__ __forceinline__ void mlp_adjoint_rows(const short *Af, const float *Bl, const short *X,
                                                 const short *Wc, float *DX, GradAcc &acc,
                                                 int lane)
{
    const int q = lane >> 4, col = lane & 15;
    const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int g = 0; g < 8; ++g) {
        const int cg = g >> 1, r = g & 1;
        const int cell = 16 * cg + col;
        const s4 xC = *reinterpret_cast<const s4 *>(&X[cell * kXStride + 16 * r + 4 * q]);
        s4 xG, wC = {0, 0, 0, 0}, wG = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            xG[j] = X[(16 * cg + 4 * q + j) * kXStride + 16 * r + col];
        if (q == 0)
            wC = *reinterpret_cast<const s4 *>(&Wc[cell * kWcStride + 4 * r]);
        if (col < 4) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                wG[j] = Wc[(16 * cg + 4 * q + j) * kWcStride + 4 * r + col];
        }

        // forward, both forms
        s4 h1C[4], h1G[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const s4 F1 = ld_s4(Af + kAF1, t, lane);
            h1C[t] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F1, xC, zero, 0, 0, 0));
            h1G[t] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xC, F1, zero, 0, 0, 0));
        }
        const bf8 B0 = join(h1C[0], h1C[1]), B1 = join(h1C[2], h1C[3]);
        s4 h2C[4], h2G[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf8 Fa = ld_bf8(Af + kAF2, 2 * t, lane), Fb = ld_bf8(Af + kAF2, 2 * t + 1, lane);
            const f4 bC = *reinterpret_cast<const f4 *>(&Bl[64 + 16 * t + 4 * q]);
            const float bg = Bl[64 + 16 * t + col];
            const f4 bG = {bg, bg, bg, bg};
            f4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Fa, B0, bC, 0, 0, 0);
            h2C[t] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x32_bf16(Fb, B1, a, 0, 0, 0));
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B0, Fa, bG, 0, 0, 0);
            h2G[t] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x32_bf16(B1, Fb, a, 0, 0, 0));
        }

        // dh2 = W3 w, da2 = dh2 where h2 > 0
        s4 d2C[4], d2G[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const s4 F5 = ld_s4(Af + kAF5, t, lane);
            d2C[t] = masked_bf16(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F5, wC, zero, 0, 0, 0),
                                 h2C[t]);
            const f4 dG = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wC, F5, zero, 0, 0, 0);
            float sb = 0.0f;
            f4 m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                m[i] = h2G[t][i] > 0 ? dG[i] : 0.0f;
                sb += m[i];
            }
            acc.b2[t] += sb;
            const s2 lo = bf16x2(m[0], m[1]), hi = bf16x2(m[2], m[3]);
            d2G[t] = s4{lo[0], lo[1], hi[0], hi[1]};
        }
        const bf8 D0 = join(d2C[0], d2C[1]), D1 = join(d2C[2], d2C[3]);

        // dh1 = W2 da2, da1 = dh1 where h1 > 0
        s4 d1C[4], d1G[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf8 Fa = ld_bf8(Af + kAF6, 2 * t, lane), Fb = ld_bf8(Af + kAF6, 2 * t + 1, lane);
            f4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Fa, D0, zero, 0, 0, 0);
            d1C[t] = masked_bf16(__builtin_amdgcn_mfma_f32_16x16x32_bf16(Fb, D1, a, 0, 0, 0), h1C[t]);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(D0, Fa, zero, 0, 0, 0);
            d1G[t] = masked_bf16(__builtin_amdgcn_mfma_f32_16x16x32_bf16(D1, Fb, a, 0, 0, 0), h1G[t]);
        }

        // dx = W1e da1; row A keeps features 0..3, row B features 4..7
        {
            const bf8 E0 = join(d1C[0], d1C[1]), E1 = join(d1C[2], d1C[3]);
            f4 dx = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld_bf8(Af + kAF7, 0, lane), E0, zero,
                                                            0, 0, 0);
            dx = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld_bf8(Af + kAF7, 1, lane), E1, dx, 0, 0,
                                                         0);
            if (q == r)
                *reinterpret_cast<f4 *>(&DX[cell * 8 + 4 * r]) = dx;
        }

        // weight gradients: contractions over the 16 rows of the tile
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc.w1[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xG, d1G[t], acc.w1[t], 0, 0, 0);
#pragma unroll
        for (int ut = 0; ut < 4; ++ut)
#pragma unroll
            for (int ot = 0; ot < 4; ++ot)
                acc.w2[4 * ut + ot] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                    h1G[ut], d2G[ot], acc.w2[4 * ut + ot], 0, 0, 0);
#pragma unroll
        for (int ut = 0; ut < 4; ++ut)
            acc.w3[ut] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h2G[ut], wG, acc.w3[ut], 0, 0, 0);
        acc.b3 += (bf16_to_float(wG[0]) + bf16_to_float(wG[1])) +
                  (bf16_to_float(wG[2]) + bf16_to_float(wG[3]));
    }
}

__global__ __launch_bounds__(kBlock) void fv_adjoint_learned_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, const double4 *__restrict__ lam_next,
    double4 *__restrict__ lam, const int32_t *__restrict__ out_idx,
    const int32_t *__restrict__ nb, const double *__restrict__ nrm,
    const double *__restrict__ inv_area, double dt, double gamma,
    const short *__restrict__ afrags, const float *__restrict__ bias, float *__restrict__ partial)
{
    __shared__ __attribute__((aligned(16))) short Xs[kWaves][64 * kXStride];
    __shared__ __attribute__((aligned(16))) short Ws[kWaves][64 * kWcStride];
    __shared__ __attribute__((aligned(16))) float Ds[kWaves][64 * 8];
    __shared__ __attribute__((aligned(16))) short Af[kCorrAdjFragShorts];
    __shared__ __attribute__((aligned(16))) float Bl[kCorrBias];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    short *X = Xs[wave];
    short *Wc = Ws[wave];
    float *DX = Ds[wave];
    for (int q = threadIdx.x; q < kCorrAdjFragShorts / 8; q += blockDim.x)
        reinterpret_cast<s8 *>(Af)[q] = reinterpret_cast<const s8 *>(afrags)[q];
    for (int q = threadIdx.x; q < kCorrBias; q += blockDim.x)
        Bl[q] = bias[q];
    __syncthreads();

    GradAcc acc;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc.w1[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        acc.w3[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        acc.b2[t] = 0.0f;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t)
        acc.w2[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    acc.b3 = 0.0f;

    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = gridDim.x, b = blockIdx.x;
    const int X_ = G < kXcds ? G : kXcds;
    const int x = b % X_, kx = b / X_;
    const int Px = (G - x + X_ - 1) / X_;
    const int t0 = (int)((long long)tiles * x / X_), t1 = (int)((long long)tiles * (x + 1) / X_);

    for (int tile = t0 + kx; tile < t1; tile += Px) {
        const int k = tile * kBlock + threadIdx.x;
        const bool live = k < n;
        short *xs = X + lane * kXStride;
        double4 Uk = {1.0, 0.0, 0.0, 2.5}, lk = {0.0, 0.0, 0.0, 0.0};
        double ak = 0.0, ck = 0.0;
        if (live) {
            Uk = U[k];
            lk = lam_next[k];
            ak = inv_area[k];
            ck = dual::step_coef(dt, inv_area[k]);
        }
        const Side L = side_of(Uk, gamma);
        double accU[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
        for (int f = 0; f < 3; ++f) {
            double ex = 1.0, ey = 0.0;
            if (live) {
                const int j = nb[f * ld + k];
                const double nx = nrm[(2 * f) * ld + k], ny = nrm[(2 * f + 1) * ld + k];
                const double4 Uj = U[j];
                const double4 lj = lam_next[j];
                const double aj = inv_area[j], cj = dual::step_coef(dt, inv_area[j]);
                const double v[4] = {ck * lk.x - cj * lj.x, ck * lk.y - cj * lj.y,
                                     ck * lk.z - cj * lj.z, ck * lk.w - cj * lj.w};
                dual::flux_vjp(Uk, Uj, nx, ny, gamma, v, accU);
                const Side R = side_of(Uj, gamma);
                const double len = root(nx * nx + ny * ny);
                const double rl = recip(len);
                ex = nx * rl;
                ey = ny * rl;
                write_feature_pair(xs, xs + 16, L, R, ex, ey, 0.5 * len * len * (ak + aj),
                                   0.5 * len * (ck + cj));
                const double ve = v[1] * ex + v[2] * ey, vt = -v[1] * ey + v[2] * ex;
                const s2 a01 = bf16x2((float)(len * v[0]), (float)(len * ve));
                const s2 a23 = bf16x2((float)(len * vt), (float)(len * v[3]));
                const s2 b01 = bf16x2((float)(-len * v[0]), (float)(len * ve));
                const s2 b23 = bf16x2((float)(len * vt), (float)(-len * v[3]));
                *reinterpret_cast<s8 *>(Wc + lane * kWcStride) =
                    s8{a01[0], a01[1], a23[0], a23[1], b01[0], b01[1], b23[0], b23[1]};
            } else {
                s4 *d = reinterpret_cast<s4 *>(xs);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    d[q] = s4{0, 0, 0, 0};
                *reinterpret_cast<s8 *>(Wc + lane * kWcStride) = s8{0, 0, 0, 0, 0, 0, 0, 0};
            }
            wave_sync();
            mlp_adjoint_rows(Af, Bl, X, Wc, DX, acc, lane);
            wave_sync();
            // features of U_k: (rho, un, ut, p) in frame e (row A, features
            // 0..3) and in frame -e (row B, features 4..7)
            const f4 dA = *reinterpret_cast<const f4 *>(&DX[lane * 8]);
            const f4 dB = *reinterpret_cast<const f4 *>(&DX[lane * 8 + 4]);
            const double d0 = (double)dA[0] + (double)dB[0];
            const double d1 = (double)dA[1] - (double)dB[1];
            const double d2 = (double)dA[2] - (double)dB[2];
            const double d3 = (double)dA[3] + (double)dB[3];
            const double ir = 1.0 / L.rho;
            const double tx = -ey, ty = ex;
            const double un = L.u * ex + L.v * ey, ut = L.u * tx + L.v * ty;
            const double gm = gamma - 1.0;
            accU[0] += d0 - (d1 * un + d2 * ut) * ir + d3 * gm * 0.5 * (L.u * L.u + L.v * L.v);
            accU[1] += (d1 * ex + d2 * tx) * ir - d3 * gm * L.u;
            accU[2] += (d1 * ey + d2 * ty) * ir - d3 * gm * L.v;
            accU[3] += d3 * gm;
        }
        if (live) {
            double4 out;
            out.x = lk.x - accU[0];
            out.y = lk.y - accU[1];
            out.z = lk.z - accU[2];
            out.w = lk.w - accU[3];
            lam[out_idx[k]] = out;
        }
    }

    // weight gradients of the workgroup: the waves add theirs in a fixed
    // order into LDS (reusing the fragment space), then one partial per
    // workgroup goes to global memory.
    __syncthreads();
    float *red = reinterpret_cast<float *>(Af);
    for (int p = threadIdx.x; p < kCorrParams; p += blockDim.x)
        red[p] = 0.0f;
    __syncthreads();
    const int q = lane >> 4, col = lane & 15;
    for (int w = 0; w < kWaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int fe = 4 * q + i, u = 16 * t + col;
                    if (fe < 12)
                        red[fe * 64 + u] += acc.w1[t][i];
                    else if (fe == 12)
                        red[768 + u] += acc.w1[t][i];
                }
#pragma unroll
            for (int ut = 0; ut < 4; ++ut)
#pragma unroll
                for (int ot = 0; ot < 4; ++ot)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        red[832 + (16 * ut + 4 * q + i) * 64 + 16 * ot + col] +=
                            acc.w2[4 * ut + ot][i];
#pragma unroll
            for (int ut = 0; ut < 4; ++ut)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (col < 4)
                        red[4992 + (16 * ut + 4 * q + i) * 4 + col] += acc.w3[ut][i];
            for (int qq = 0; qq < 4; ++qq) {
                wave_sync();
                if (q == qq) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        red[4928 + 16 * t + col] += acc.b2[t];
                    if (col < 4)
                        red[5248 + col] += acc.b3;
                }
            }
        }
        __syncthreads();
    }
    for (int p = threadIdx.x; p < kCorrParams; p += blockDim.x)
        partial[(size_t)blockIdx.x * kCorrParams + p] = red[p];
}

// out[p] += scale * sum_s partial[s][p], in float64 and in a fixed order.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *__restrict__ partial,
                                                          int slots, double scale,
                                                          double *__restrict__ out)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kCorrParams)
        return;
    double s = 0.0;
    int k = 0;
    // loads issued 16 at a time, sums kept in slot order
    for (; k + 16 <= slots; k += 16) {
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = partial[(size_t)(k + q) * kCorrParams + p];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            s += (double)v[q];
    }
    for (; k < slots; ++k)
        s += (double)partial[(size_t)k * kCorrParams + p];
    out[p] += scale * s;
}

inline unsigned short host_bf16(float x)
{
    unsigned u;
    memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// Input unit of K slot j of lane quad q in K slice s of a 16x16x32 operand:
// the accumulator order of the two 16-unit tiles that make up the slice.
inline int k32_unit(int s, int q, int j)
{
    return 32 * s + (j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4));
}

}  // namespace

void pack_correction(const float *params, short *frags, float *bias)
{
    // params: W1 [12][64], b1 [64], W2 [64][64], b2 [64], W3 [64][4], b3 [4]
    const float *W1 = params, *b1 = W1 + 12 * 64, *W2 = b1 + 64, *b2 = W2 + 64 * 64;
    const float *W3 = b2 + 64, *b3 = W3 + 64 * 4;
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, col = lane & 15;
        for (int mt = 0; mt < 4; ++mt)
            for (int j = 0; j < 4; ++j) {
                const int kin = 4 * q + j, m = 16 * mt + col;
                const float w = kin < 12 ? W1[kin * 64 + m] : (kin == 12 ? b1[m] : 0.0f);
                frags[kFragW1 + (mt * 64 + lane) * 4 + j] = (short)host_bf16(w);
            }
        for (int mt = 0; mt < 4; ++mt)
            for (int s = 0; s < 2; ++s)
                for (int j = 0; j < 8; ++j)
                    frags[kFragW2 + ((2 * mt + s) * 64 + lane) * 8 + j] =
                        (short)host_bf16(W2[k32_unit(s, q, j) * 64 + 16 * mt + col]);
        for (int s = 0; s < 2; ++s)
            for (int j = 0; j < 8; ++j)
                frags[kFragW3 + (s * 64 + lane) * 8 + j] =
                    (short)host_bf16(col < 4 ? W3[k32_unit(s, q, j) * 4 + col] : 0.0f);
    }
    for (int m = 0; m < 64; ++m) {
        bias[m] = b1[m];
        bias[64 + m] = b2[m];
    }
    for (int m = 0; m < 16; ++m)
        bias[128 + m] = m < 4 ? b3[m] : 0.0f;
}

void pack_correction_adjoint(const float *params, short *afrags)
{
    const float *W1 = params, *b1 = W1 + 12 * 64, *W2 = b1 + 64 * 1, *b2 = W2 + 64 * 64;
    const float *W3 = b2 + 64;
    auto W1e = [&](int f, int u) { return f < 12 ? W1[f * 64 + u] : (f == 12 ? b1[u] : 0.0f); };
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, col = lane & 15;
        for (int t = 0; t < 4; ++t)
            for (int j = 0; j < 4; ++j) {
                afrags[kAF1 + (t * 64 + lane) * 4 + j] = (short)host_bf16(W1e(4 * q + j, 16 * t + col));
                const int o = 4 * q + j;
                afrags[kAF5 + (t * 64 + lane) * 4 + j] =
                    (short)host_bf16(o < 4 ? W3[(16 * t + col) * 4 + o] : 0.0f);
            }
        for (int t = 0; t < 4; ++t)
            for (int s = 0; s < 2; ++s)
                for (int j = 0; j < 8; ++j) {
                    const int k = k32_unit(s, q, j);
                    afrags[kAF2 + ((2 * t + s) * 64 + lane) * 8 + j] =
                        (short)host_bf16(W2[k * 64 + 16 * t + col]);
                    afrags[kAF6 + ((2 * t + s) * 64 + lane) * 8 + j] =
                        (short)host_bf16(W2[(16 * t + col) * 64 + k]);
                }
        for (int s = 0; s < 2; ++s)
            for (int j = 0; j < 8; ++j)
                afrags[kAF7 + (s * 64 + lane) * 8 + j] = (short)host_bf16(W1e(col, k32_unit(s, q, j)));
    }
}

int adjoint_learned_grid(int32_t n)
{
    const int tiles = (n + kBlock - 1) / kBlock;
    return tiles < kCorrAdjMaxGrid ? tiles : kCorrAdjMaxGrid;
}

hipError_t launch_adjoint_learned(int32_t n, int32_t ld, const double4 *U, const double4 *lam_next,
                                  double4 *lam, const int32_t *out_idx, const int32_t *nb,
                                  const double *nrm, const double *inv_area, double dt,
                                  double gamma, const short *afrags, const float *bias,
                                  float *partial, double *grad, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int G = adjoint_learned_grid(n);
    hipLaunchKernelGGL(fv_adjoint_learned_kernel, dim3(G), dim3(kBlock), 0, s, n, ld, U, lam_next,
                       lam, out_idx, nb, nrm, inv_area, dt, gamma, afrags, bias, partial);
    if (grad)
        hipLaunchKernelGGL(grad_reduce_kernel, dim3((kCorrParams + 255) / 256), dim3(256), 0, s,
                           partial, G, -0.5, grad);
    return hipGetLastError();
}

hipError_t launch_step_learned(int32_t n, int32_t ld, const double4 *U, double4 *Un,
                               const int32_t *nb, const short4 *nb16, int nb16_stride,
                               const double *nrm, const double *coef, const double *inv_area,
                               const short *frags,
                               const float *bias, double gamma, bool narrow, bool closed, int grid,
                               hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = (grid <= 0 || grid > tiles) ? (tiles < 8192 ? tiles : 8192) : grid;
    if (narrow && closed)
        hipLaunchKernelGGL((fv_step_learned_kernel<true, true>), dim3(G), dim3(kBlock), 0, s, n, ld,
                           U, Un, nb, nb16, nb16_stride, nrm, coef, inv_area, frags, bias, gamma);
    else if (narrow)
        hipLaunchKernelGGL((fv_step_learned_kernel<true, false>), dim3(G), dim3(kBlock), 0, s, n,
                           ld, U, Un, nb, nb16, nb16_stride, nrm, coef, inv_area, frags, bias, gamma);
    else if (closed)
        hipLaunchKernelGGL((fv_step_learned_kernel<false, true>), dim3(G), dim3(kBlock), 0, s, n,
                           ld, U, Un, nb, nb16, nb16_stride, nrm, coef, inv_area, frags, bias, gamma);
    else
        hipLaunchKernelGGL((fv_step_learned_kernel<false, false>), dim3(G), dim3(kBlock), 0, s, n,
                           ld, U, Un, nb, nb16, nb16_stride, nrm, coef, inv_area, frags, bias, gamma);
    return hipGetLastError();
}

}  // namespace fvk
