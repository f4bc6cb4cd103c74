// Internal launchers shared by the host runtime (fv_runtime.hip) and the
// kernel files.  Not part of the public ABI.
//
// Device layout of a mesh with n cells, leading dimension ld = n rounded up
// to a multiple of 64 (so every sub-array starts 256-byte aligned):
//   U       double4 [n]       (rho, rho u, rho v, E) per cell
//   nb      int32  [3][ld]    neighbour across face f (structure of arrays)
//   nrm     double [6][ld]    nx_0, ny_0, nx_1, ny_1, nx_2, ny_2
//   inv_area double [ld]      1 / V_T
//   nb16    short4 [ld]       neighbour offsets j - i, when they fit in 16 bits;
//                             interleaved with dt / V as (short4, double) [ld]
//                             on a mesh beyond the Infinity Cache
//                             (narrow_interleaved)
//   nfx     int4   [ld]       first two normals in fixed point, when exact
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fvk {

// Bytes of the working set per cell with 16-bit offsets (two states,
// offsets, dt/V, and the normals: 16 B in fixed point, 32 B with the third
// derived, 48 B all stored) and the Infinity Cache of MI355X.  A mesh whose
// working set exceeds the cache is stepped with non-temporal reads of its
// per-cell arrays and keeps its 16-bit offsets interleaved with dt/V (16
// bytes per cell: one load brings both, before the neighbour gathers).
// Within the cache the offsets are a plain short4 array and dt/V is read
// from coef after the flux (the critical first load then touches half as
// many cache lines).
constexpr int64_t kInfinityCache = int64_t(256) << 20;
inline int64_t narrow_bytes(bool closed, bool fixed)
{
    return 2 * 32 + 8 + 8 + (fixed && closed ? 16 : (closed ? 32 : 48));
}
inline bool narrow_interleaved(int64_t n, bool closed, bool fixed)
{
    return n * narrow_bytes(closed, fixed) > kInfinityCache;
}

// One forward-Euler Lax-Friedrichs step over all cells: Un = U - coef sum F
// with coef[i] = dt / V_i.
// narrow: read neighbours from nb16 (16-bit offsets) instead of nb; with
// narrow_interleaved(n, closed, fixed), nb16 is the interleaved array and
// dt/V comes from it instead of coef.
// closed: take the third normal as -(n_0 + n_1) instead of reading it.
// fixed (with closed): read the first two normals from nfx (fixed point).
// block: 128, 256 or 512 threads; grid: 0 = one workgroup per tile of
// `block` cells, else that many persistent workgroups.
hipError_t launch_step(int32_t n, int32_t ld, const double4 *U, double4 *Un, const int32_t *nb,
                       const short4 *nb16, const double *nrm, const int4 *nfx,
                       const double *coef, double gamma, bool narrow, bool closed, bool fixed,
                       int block, int grid, hipStream_t s);

// nfx[i] = (k_0x, k_0y, k_1x, k_1y), the first two normals of cell i as
// n = k 2^-32 (INT32_MIN for -0.0); every component must convert exactly.
hipError_t launch_fixed_normals(int32_t n, int32_t ld, const double *nrm, int4 *nfx,
                                hipStream_t s);

// coef[i] = dt[s] * inv_area[i], s the segment of cell i; with an
// interleaved nb16 array (else null), its dt/V slots receive the same values.
hipError_t launch_coef(int32_t n, int32_t n_seg, const int64_t *seg, const double *dt,
                       const double *inv_area, double *coef, short4 *nb16_interleaved,
                       hipStream_t s);

// nb16[stride * i] = (nb[0][i] - i, nb[1][i] - i, nb[2][i] - i, 0) as 16-bit
// offsets (stride 1: plain array, 2: interleaved with dt/V, whose slots are
// left alone); *too_far = 1 when some offset does not fit (it must be 0
// before).
hipError_t launch_narrow_offsets(int32_t n, int32_t ld, const int32_t *nb, short4 *nb16,
                                 int stride, int32_t *too_far, hipStream_t s);

// Cotangent of one step's input from the cotangent of its output, on arrays
// in any one numbering (mesh arrays nb [3][ld], nrm [6][ld], inv_area [ld]
// holding 1 / V):
// lam = lam_next - sum_f (dG(U_k, U_j, n_f)/dU_k)^T (c_k lam_next_k - c_j lam_next_j),
// c = dt * (1 / V), rounded as the step forms it.  Cell k's result goes to
// lam[out_idx[k]] (out_idx a permutation); lam and lam_next must not overlap.
hipError_t launch_adjoint(int32_t n, int32_t ld, const double4 *U, const double4 *lam_next,
                          double4 *lam, const int32_t *out_idx, const int32_t *nb,
                          const double *nrm, const double *inv_area, double dt, double gamma,
                          hipStream_t s);

// Learned correction: the packed MLP (weight fragments, kCorrFragShorts
// bfloat16, then 144 float biases: b1, b2, b3 padded to 16) and the step that
// adds it to the flux (see fv_learned.hip).
constexpr int kCorrParams = 12 * 64 + 64 + 64 * 64 + 64 + 64 * 4 + 4;  // 5252
constexpr int kCorrFragShorts = 24 * 64 * 4;
constexpr int kCorrBias = 144;
void pack_correction(const float *params, short *frags, float *bias);
// nb16_stride: 1 for the plain offset array, 2 for the interleaved one.
hipError_t launch_step_learned(int32_t n, int32_t ld, const double4 *U, double4 *Un,
                               const int32_t *nb, const short4 *nb16, int nb16_stride,
                               const double *nrm, const double *coef, const double *inv_area,
                               const short *frags,
                               const float *bias, double gamma, bool narrow, bool closed, int grid,
                               hipStream_t s);

// Adjoint of the corrected step (see fv_learned.hip): lam from lam_next as
// launch_adjoint does (same arrays, output through out_idx), plus the
// cotangent of the correction, on arrays in any one numbering; the parameter
// gradient sums the cells in that numbering.  Each workgroup leaves its part
// of the parameter gradient in partial [adjoint_learned_grid(n)][kCorrParams];
// with grad non-null, grad [kCorrParams] (float64) += the gradient.
constexpr int kCorrAdjFragShorts = (4 * 4 + 8 * 8 + 4 * 4 + 8 * 8 + 2 * 8) * 64;
constexpr int kCorrAdjMaxGrid = 512;
void pack_correction_adjoint(const float *params, short *afrags);
int adjoint_learned_grid(int32_t n);
hipError_t launch_adjoint_learned(int32_t n, int32_t ld, const double4 *U, const double4 *lam_next,
                                  double4 *lam, const int32_t *out_idx, const int32_t *nb,
                                  const double *nrm, const double *inv_area, double dt,
                                  double gamma, const short *afrags, const float *bias,
                                  float *partial, double *grad, hipStream_t s);

// ---- renumbering --------------------------------------------------------
// rec[v]: the graph nb (int32 [n][3], the uploaded order) as 16-byte
// records for the renumbering passes, no cell visited yet.
hipError_t launch_build_records(int32_t n, const int32_t *nb, int4 *rec, hipStream_t s);

// Cuthill-McKee order of every segment [seg[k], seg[k+1]) (device array of
// n_seg + 1 offsets; no face crosses a segment), one workgroup per segment:
// perm[label] = cell, label[cell] = label.  rec comes fresh from
// launch_build_records; rec2 (n records), state and probe (n_seg entries
// each), permA and ordC (n entries each) are scratch; passes[k] receives the
// number of breadth-first passes of segment k.  Not speculative: the
// confirming sweep of the pseudo-peripheral search (launch_cm_confirm) runs
// on `side` and s waits for it before the labels are final.  Speculative: the
// labels assume the search does not move, and the caller must launch the
// confirming sweep itself once s holds nothing more that touches rec, rec2,
// ordC or state, wait for `probed`, and, if some probe[k] > state[k].y
// (the eccentricity grew), renumber again without speculation.
hipError_t launch_cm_segments(int4 *rec, int4 *rec2, int4 *state, int32_t *probe, int32_t n,
                              int32_t n_seg, const int64_t *seg, int32_t *permA, int32_t *ordC,
                              int32_t *perm, int32_t *label, int32_t *passes, hipStream_t s,
                              hipStream_t side, hipEvent_t labelled, hipEvent_t probed,
                              bool speculative);

// The confirming sweep of each segment's first component on `side`, after
// everything queued on s (event `labelled`), recorded as `probed`: the graph
// renamed by the first labels into rec2 (read from rec, whose marks are the
// labels after the first pass), then the sweep from the first pass's pick,
// whose eccentricity goes to probe[k].  Until `probed`, side reads rec and
// state, and writes rec2, ordC (the sweep's frontier overflow) and probe.
hipError_t launch_cm_confirm(const int4 *rec, int4 *rec2, const int4 *state, int32_t *probe,
                             int32_t n, int32_t n_seg, const int64_t *seg, int32_t *ordC,
                             hipStream_t s, hipStream_t side, hipEvent_t labelled,
                             hipEvent_t probed);

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s);
hipError_t launch_iota(int32_t *p, int32_t count, hipStream_t s);

// ---- permutation gathers --------------------------------------------------
// Working-order geometry from the uploaded mesh (nb_o int32 [n][3] and
// nrm_o double [n][6] as uploaded, area_o double [n]): for new cell l with
// v = perm[l]: nb_w[f][l] = label[nb_o[v][f]], nrm_w[k][l] = nrm_o[v][k],
// inv_area_w[l] = 1 / area_o[v].  nrm_o must be 16-byte aligned.
hipError_t launch_gather_geometry(int32_t n, int32_t ld, const int32_t *perm, const int32_t *label,
                                  const int32_t *nb_o, const double *nrm_o, const double *area_o,
                                  int32_t *nb_w, double *nrm_w, double *inv_area_w, hipStream_t s);

// dst[l] = src[idx[l]]
hipError_t launch_gather_state(int32_t n, const int32_t *idx, const double4 *src, double4 *dst,
                               hipStream_t s);

// dst[l] = src[idx_b[idx_a[l]]]
hipError_t launch_gather_state2(int32_t n, const int32_t *idx_a, const int32_t *idx_b,
                                const double4 *src, double4 *dst, hipStream_t s);

// out[i] = sum_m w[i][m] src[idx[i][m]], m = 0..k-1 in order; NaN where an
// index is outside [0, n_src).
hipError_t launch_restrict(int64_t n, int32_t k, int64_t n_src, const double4 *src,
                           const int32_t *idx, const double *w, double4 *out, hipStream_t s);

// *flag = 1 if any cell has non-finite or non-positive rho or p (flag must be 0 before).
hipError_t launch_check_state(int32_t n, const double4 *U, double gamma, int32_t *flag,
                              hipStream_t s);

}  // namespace fvk
