// K1: one explicit cell-centred finite-volume step of the 2D Euler equations
// (section 6.2.2 of the paper: semi-discrete form eqSemiDiscrete, forward
// Euler eqFWEuler, Lax-Friedrichs flux eqCompFlux).
//
// One thread per cell.  The thread reads its own state, its face normals,
// its inverse area and its neighbour indices, gathers the three neighbour
// states and writes the updated state into the other buffer.  Nothing is
// scattered and nothing is accumulated across threads, so the result of a
// cell depends only on its own inputs, in its own face order: the same bits
// whatever the cell numbering or the launch shape.
//
// The flux is evaluated without a face frame.  With n the length-scaled
// outward normal, V = u n_x + v n_y = |n| u_n, the face-frame flux rotated
// back and multiplied by |n| equals
//   (F(U_L) + F(U_R)) . n / 2 - (|V_L + V_R| / 2 + |n| (c_L + c_R) / 2) (U_R - U_L) / 2
// where F(U) . n = (rho V, rho u V + p n_x, rho v V + p n_y, (E + p) V):
// the rotation of the momentum jump back to x-y is the identity on U, so no
// unit normal (and no division by |n|) is needed.  This is an exact
// identity; only the rounding differs from the face-frame evaluation.
//
// The step is bound by HBM traffic, so two exact compressions of the
// per-cell geometry are used when the mesh allows them (the paper makes the
// same two points for its memory stream: indices can be narrowed once the
// renumbering bounds the neighbour distance, section 3, and normals can be
// derived instead of stored, section 7):
//   - kNarrow: neighbour j of cell i stored as the 16-bit offset j - i
//     (four shorts, 8 bytes) instead of three 32-bit indices; used when every
//     offset fits, which the Cuthill-McKee order makes true on large meshes.
//     Beyond the Infinity Cache (kStream) the offsets are interleaved with
//     the cell's dt / V_T, so one 16-byte load brings both, and the per-cell
//     arrays are read with non-temporal loads.
//   - kClosed: the third normal read as -(n_0 + n_1) instead of from memory;
//     used when every cell's stored normals satisfy n_2 == -(n_0 + n_1)
//     exactly, so the value is bit-identical to the stored one.
//   - kFixed (with kClosed): the two stored normals as 32-bit integers k with
//     n = k 2^-32, four ints (16 bytes) instead of four doubles; used when
//     every such component is an integer multiple of 2^-32 below 2^31 in
//     size (as on meshes whose vertices are snapped to 2^-32, with faces
//     shorter than 1/2), so the decoded double is the stored one; -0.0 is
//     kept as the otherwise unused INT32_MIN.
// Bytes per cell update: 132 (general), 112 with the first two, 96 with all
// three.  The cell's
// dt / V_T comes from a per-cell array (formed as dt * (1 / V_T), the same
// single rounding whatever the batch), so meshes of a batch can step with
// their own dt in one launch.

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

// 1 / a from the hardware reciprocal estimate refined by two Newton-Raphson
// steps y <- y + y (1 - a y), each with a fused residual: the relative error
// falls from the estimate's ~2^-26 to round-off.
__device__ __forceinline__ double recip(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

// sqrt(a) for a >= 0: two Newton-Raphson steps on the hardware reciprocal
// square root estimate r <- r (3 - a r^2) / 2, then s = a r and one residual
// correction s <- s + (a - s^2) r / 2.
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

struct Prim {
    double ir;  // 1 / rho
    double p;   // pressure
    double c;   // speed of sound
};

__device__ __forceinline__ Prim primitives(const double4 &U, double gamma)
{
    Prim q;
    q.ir = recip(U.x);
    // p = (gamma - 1) (E - rho |v|^2 / 2) with rho |v|^2 = (m_x^2 + m_y^2) / rho
    q.p = (gamma - 1.0) * (U.w - 0.5 * (U.y * U.y + U.z * U.z) * q.ir);
    q.c = root(gamma * q.p * q.ir);
    return q;
}

// A normal component from its fixed-point form k (n = k 2^-32; INT32_MIN
// stands for -0.0).
__device__ __forceinline__ double from_fixed(int k)
{
    return k == INT32_MIN ? -0.0 : (double)k * 0x1p-32;
}

// Per-cell arrays read once per step (offsets, fixed-point normals, dt/V),
// with kStream as non-temporal loads: on a mesh whose working set exceeds
// the Infinity Cache they would only displace the states that the
// neighbour gathers reuse.
template <bool kStream, typename T>
__device__ __forceinline__ T read_once(const T *p)
{
    if constexpr (kStream)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Update of one cell i (the body of the step).
template <bool kNarrow, bool kClosed, bool kFixed, bool kStream>
__device__ __forceinline__ void update_cell(int i, int32_t ld, const double4 *__restrict__ U,
                                            double4 *__restrict__ Un,
                                            const int32_t *__restrict__ nb,
                                            const short4 *__restrict__ nb16,
                                            const double *__restrict__ nrm,
                                            const int4 *__restrict__ nfx,
                                            const double *__restrict__ coef, double gamma)
{
    static_assert(kNarrow || !kStream, "the streaming step reads the interleaved offsets");
    // With 16-bit offsets, in the compact layout (kFixed) and beyond the
    // Infinity Cache (kStream), a wave runs at a raised priority while it
    // issues its loads and at the base priority for its FP64 flux, so that
    // the waves about to fetch get their requests out ahead of the ones
    // computing and the memory system stays busy while others compute:
    // 4-5 % of a launch beyond the cache, where the step is bound by HBM,
    // and neutral within it.  Within the cache, with float64 normals (four
    // more loads per cell) it was 3 % slower, and with 32-bit indices on a
    // random order 0.8 % slower, so those variants keep the plain schedule.
    constexpr bool kPrio = kNarrow && (kFixed || kStream);
    if constexpr (kPrio)
        __builtin_amdgcn_s_setprio(1);
    int js[3];
    // coef = dt / V_T, formed as dt * (1 / V_T) by coef_kernel: with kStream
    // beside the offsets, else from coef after the flux
    double k;
    if constexpr (kNarrow) {
        short4 o;
        {
            // the four 16-bit offsets as one 8-byte word
            const long long *w = reinterpret_cast<const long long *>(nb16);
            const long long q = read_once<kStream>(kStream ? w + 2 * (int64_t)i : w + i);
            if constexpr (kStream)
                k = __longlong_as_double(read_once<kStream>(w + 2 * (int64_t)i + 1));
            o = *reinterpret_cast<const short4 *>(&q);
        }
        js[0] = i + o.x;
        js[1] = i + o.y;
        js[2] = i + o.z;
    } else {
        js[0] = nb[i];
        js[1] = nb[ld + i];
        js[2] = nb[2 * ld + i];
    }
    double nxs[3], nys[3];
    if constexpr (kFixed) {
        const int *qp = reinterpret_cast<const int *>(nfx) + 4 * (int64_t)i;
        const int4 q = make_int4(read_once<kStream>(qp), read_once<kStream>(qp + 1),
                                 read_once<kStream>(qp + 2), read_once<kStream>(qp + 3));
        nxs[0] = from_fixed(q.x);
        nys[0] = from_fixed(q.y);
        nxs[1] = from_fixed(q.z);
        nys[1] = from_fixed(q.w);
    } else {
        nxs[0] = read_once<kStream>(nrm + i);
        nys[0] = read_once<kStream>(nrm + ld + i);
        nxs[1] = read_once<kStream>(nrm + 2 * ld + i);
        nys[1] = read_once<kStream>(nrm + 3 * ld + i);
    }
    if constexpr (kClosed) {
        nxs[2] = -(nxs[0] + nxs[1]);
        nys[2] = -(nys[0] + nys[1]);
    } else {
        nxs[2] = read_once<kStream>(nrm + 4 * ld + i);
        nys[2] = read_once<kStream>(nrm + 5 * ld + i);
    }
    // The normals enter the flux as opaque values, so every layout runs the
    // same arithmetic: otherwise the compiler folds the derived normal's
    // negation into the products of face 2 and fuses different pairs into
    // FMAs than with a loaded normal, which changes the rounding.
#pragma unroll
    for (int f = 0; f < 3; ++f)
        asm volatile("" : "+v"(nxs[f]), "+v"(nys[f]));

    // with kPrio the cell's and its three neighbours' states are all issued
    // before the priority drops
    const double4 Ui = U[i];
    double4 Ujs[3];
    if constexpr (kPrio) {
#pragma unroll
        for (int f = 0; f < 3; ++f)
            Ujs[f] = U[js[f]];
        __builtin_amdgcn_s_setprio(0);
    }
    const Prim L = primitives(Ui, gamma);
    const double uL = Ui.y * L.ir, vL = Ui.z * L.ir;

    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const double nx = nxs[f], ny = nys[f];
        const double4 Uj = kPrio ? Ujs[f] : U[js[f]];
        const Prim R = primitives(Uj, gamma);
        const double uR = Uj.y * R.ir, vR = Uj.z * R.ir;

        const double len = root(nx * nx + ny * ny);
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

    if constexpr (!kStream)
        k = coef[i];
    double4 out;
    out.x = Ui.x - k * a0;
    out.y = Ui.y - k * a1;
    out.z = Ui.z - k * a2;
    out.w = Ui.w - k * a3;
    Un[i] = out;
}

// Tiles of kBlock cells.  With one workgroup per tile the workgroup ids are
// remapped so that each XCD takes one contiguous range of tiles; with a
// persistent grid of fewer workgroups, the tiles are split into one
// contiguous range per XCD and the workgroups of each XCD stride through it.
template <int kBlock, bool kNarrow, bool kClosed, bool kFixed, bool kStream>
__global__ __launch_bounds__(kBlock) void fv_step_kernel(
    int32_t n, int32_t ld, const double4 *__restrict__ U, double4 *__restrict__ Un,
    const int32_t *__restrict__ nb, const short4 *__restrict__ nb16,
    const double *__restrict__ nrm, const int4 *__restrict__ nfx,
    const double *__restrict__ coef, double gamma)
{
    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = gridDim.x, b = blockIdx.x;
    if (G >= tiles) {
        const int t = xcd_contiguous_block(b, G);
        const int i = t * kBlock + threadIdx.x;
        if (t < tiles && i < n)
            update_cell<kNarrow, kClosed, kFixed, kStream>(i, ld, U, Un, nb, nb16, nrm, nfx, coef,
                                                           gamma);
        return;
    }
    const int X = G < kXcds ? G : kXcds;  // XCDs that hold workgroups
    const int x = b % X, k = b / X;
    const int Px = (G - x + X - 1) / X;   // workgroups on XCD x
    const int t0 = (int)((long long)tiles * x / X), t1 = (int)((long long)tiles * (x + 1) / X);
    for (int t = t0 + k; t < t1; t += Px) {
        const int i = t * kBlock + threadIdx.x;
        if (i < n)
            update_cell<kNarrow, kClosed, kFixed, kStream>(i, ld, U, Un, nb, nb16, nrm, nfx, coef,
                                                           gamma);
    }
}

// coef[i] = dt[s] * inv_area[i] for the segment s holding i (seg: n_seg + 1
// increasing offsets); also into the dt/V slots of an interleaved offset
// array when there is one.
__global__ void coef_kernel(int32_t n, int32_t n_seg, const int64_t *__restrict__ seg,
                            const double *__restrict__ dt, const double *__restrict__ inv_area,
                            double *__restrict__ coef, short4 *__restrict__ nb16_interleaved)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    int lo = 0, hi = n_seg - 1;  // largest s with seg[s] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const double k = dt[lo] * inv_area[i];
    coef[i] = k;
    if (nb16_interleaved)
        reinterpret_cast<double *>(nb16_interleaved)[2 * (int64_t)i + 1] = k;
}

template <int kBlock, bool kNarrow, bool kClosed, bool kFixed, bool kStream = false>
void launch_variant(int G, int32_t n, int32_t ld, const double4 *U, double4 *Un,
                    const int32_t *nb, const short4 *nb16, const double *nrm, const int4 *nfx,
                    const double *coef, double gamma, hipStream_t s)
{
    hipLaunchKernelGGL((fv_step_kernel<kBlock, kNarrow, kClosed, kFixed, kStream>), dim3(G),
                       dim3(kBlock), 0, s, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma);
}

template <int kBlock>
hipError_t launch_step_block(int32_t n, int32_t ld, const double4 *U, double4 *Un,
                             const int32_t *nb, const short4 *nb16, const double *nrm,
                             const int4 *nfx, const double *coef, double gamma, bool narrow,
                             bool closed, bool fixed, int grid, hipStream_t s)
{
    const int tiles = (n + kBlock - 1) / kBlock;
    const int G = (grid <= 0 || grid > tiles) ? tiles : grid;
    fixed = fixed && closed;
    const bool stream = narrow && narrow_interleaved(n, closed, fixed);
    if (stream && fixed)
        launch_variant<kBlock, true, true, true, true>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef,
                                                        gamma, s);
    else if (stream && closed)
        launch_variant<kBlock, true, true, false, true>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef,
                                                         gamma, s);
    else if (stream)
        launch_variant<kBlock, true, false, false, true>(G, n, ld, U, Un, nb, nb16, nrm, nfx,
                                                          coef, gamma, s);
    else if (narrow && fixed)
        launch_variant<kBlock, true, true, true>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, s);
    else if (fixed)
        launch_variant<kBlock, false, true, true>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, s);
    else if (narrow && closed)
        launch_variant<kBlock, true, true, false>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, s);
    else if (narrow)
        launch_variant<kBlock, true, false, false>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, s);
    else if (closed)
        launch_variant<kBlock, false, true, false>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, s);
    else
        launch_variant<kBlock, false, false, false>(G, n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, s);
    return hipGetLastError();
}

// 16-bit neighbour offsets of the working order at nb16[stride * i];
// *too_far = 1 (every writer stores the same value) if some offset does not
// fit.
__global__ void narrow_offsets_kernel(int32_t n, int32_t ld, const int32_t *__restrict__ nb,
                                      short4 *__restrict__ nb16, int stride,
                                      int32_t *__restrict__ too_far)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const int o0 = nb[i] - i, o1 = nb[ld + i] - i, o2 = nb[2 * ld + i] - i;
    const bool fits = o0 >= -32768 && o0 <= 32767 && o1 >= -32768 && o1 <= 32767 &&
                      o2 >= -32768 && o2 <= 32767;
    nb16[(int64_t)stride * i] = make_short4((short)o0, (short)o1, (short)o2, 0);
    if (!fits)
        *too_far = 1;
}

// nfx[i] = the fixed-point form of the first two normals of working cell i
// (the mesh was checked on the host: every component converts exactly).
__global__ void fixed_normals_kernel(int32_t n, int32_t ld, const double *__restrict__ nrm,
                                     int4 *__restrict__ nfx)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    int k[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double x = nrm[c * ld + i];
        k[c] = (x == 0.0 && signbit(x)) ? INT32_MIN : (int)(x * 0x1p32);
    }
    nfx[i] = make_int4(k[0], k[1], k[2], k[3]);
}

}  // namespace

hipError_t launch_step(int32_t n, int32_t ld, const double4 *U, double4 *Un, const int32_t *nb,
                       const short4 *nb16, const double *nrm, const int4 *nfx,
                       const double *coef, double gamma, bool narrow, bool closed, bool fixed,
                       int block, int grid, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    switch (block) {
    case 128:
        return launch_step_block<128>(n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, narrow,
                                      closed, fixed, grid, s);
    case 512:
        return launch_step_block<512>(n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, narrow,
                                      closed, fixed, grid, s);
    default:
        return launch_step_block<256>(n, ld, U, Un, nb, nb16, nrm, nfx, coef, gamma, narrow,
                                      closed, fixed, grid, s);
    }
}

hipError_t launch_fixed_normals(int32_t n, int32_t ld, const double *nrm, int4 *nfx,
                                hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(fixed_normals_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ld, nrm,
                       nfx);
    return hipGetLastError();
}

hipError_t launch_coef(int32_t n, int32_t n_seg, const int64_t *seg, const double *dt,
                       const double *inv_area, double *coef, short4 *nb16_interleaved,
                       hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(coef_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, n_seg, seg, dt,
                       inv_area, coef, nb16_interleaved);
    return hipGetLastError();
}

hipError_t launch_narrow_offsets(int32_t n, int32_t ld, const int32_t *nb, short4 *nb16,
                                 int stride, int32_t *too_far, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(narrow_offsets_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ld, nb,
                       nb16, stride, too_far);
    return hipGetLastError();
}

}  // namespace fvk
