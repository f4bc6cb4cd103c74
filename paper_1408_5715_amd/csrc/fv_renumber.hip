// K2: Cuthill-McKee renumbering on the GPU (section 4 of the paper: cell
// renumbering that bounds the distance between the labels of neighbours, so
// the window of states in use stays small; start vertex from a pseudo-
// diameter endpoint as in section 4.2.2).
//
// Sequential Cuthill-McKee labels the root, then visits labelled cells in
// label order and appends each one's unlabelled neighbours in (degree, id)
// order.  A cell w of level k+1 is therefore labelled by its neighbour of
// level k with the smallest label (its "owner"), and the labels of level k+1
// are the cells sorted by (owner label, degree, id).  The kernel builds the
// same labelling one level at a time: every frontier cell finds the cells it
// owns (an unlabelled neighbour w is owned by v when v has the smallest label
// among w's neighbours inside the frontier), ranks its at most three
// children, and a block-wide exclusive scan of the child counts gives every
// child its label.  The result equals the sequential order exactly.
//
// One workgroup of 1024 threads labels a whole mesh in one launch (all
// levels, the pseudo-peripheral search and every component): levels are a
// few thousand cells wide, so the work per level is small, and a grid-wide
// barrier per level (which on this chip means writing back and invalidating
// per-XCD L2 caches) would cost more than it saves.  A batch of independent
// meshes runs one such workgroup per mesh, side by side.
// Every wave leaves the level loop on the same block-uniform condition (an
// empty next level).
//
// The graph is read as 16-byte records: three neighbours and the cell's
// label (-1 while unlabelled), so one cache-line fetch answers both "is w
// labelled" and "who are w's neighbours".  Frontier cells carry their
// neighbour lists in LDS (fetched when they were discovered).  One CU runs
// the whole labelling, and its cost is set by the number of scattered lane
// requests per cell, so loads are issued only by the lanes that need them
// (about 5.6 per frontier cell: three neighbour records and the labels of
// the other neighbours of unlabelled cells).

#include <climits>

#include "fv_internal.h"

namespace fvk {
namespace {

constexpr int kCmThreads = 1024;
constexpr int kCmWaves = kCmThreads / 64;
constexpr int kFrontierCap = 4096;  // frontier entries held in LDS per buffer (2 x 64 KiB)
constexpr int kPer = 3;             // frontier cells per thread and sweep

// Block-wide exclusive scan over 1024 threads; *total receives the sum.
__device__ __forceinline__ int block_exclusive_scan(int x, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += y;
    }
    if (lane == 63)
        sh[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int w = lane < kCmWaves ? sh[lane] : 0;
        int wi = w;
#pragma unroll
        for (int d = 1; d < kCmWaves; d <<= 1) {
            const int y = __shfl_up(wi, d, 64);
            if (lane >= d)
                wi += y;
        }
        if (lane < kCmWaves)
            sh[kCmWaves + lane] = wi - w;
        if (lane == kCmWaves - 1)
            sh[2 * kCmWaves] = wi;
    }
    __syncthreads();
    const int excl = incl - x + sh[kCmWaves + wid];
    *total = sh[2 * kCmWaves];
    __syncthreads();
    return excl;
}

// Block-wide minimum of a 64-bit key over 1024 threads (all threads get it).
__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long x,
                                                            unsigned long long *sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long y = __shfl_xor(x, d, 64);
        x = y < x ? y : x;
    }
    if (lane == 0)
        sh[wid] = x;
    __syncthreads();
    unsigned long long m = sh[0];
    for (int k = 1; k < kCmWaves; ++k)
        m = sh[k] < m ? sh[k] : m;
    __syncthreads();
    return m;
}

// Distinct neighbours other than the cell itself.
__device__ __forceinline__ int degree_of(int v, int a, int b, int c)
{
    int d = 0;
    d += (a != v);
    d += (b != v && b != a);
    d += (c != v && c != a && c != b);
    return d;
}


struct PassResult {
    int count;  // cells labelled (the component of the root)
    int ecc;    // eccentricity of the root
    int pick;   // last-level cell of minimum (degree, id)
};

// LDS of one labelling pass.
struct PassLds {
    int4 frontier[2][kFrontierCap];  // (cell, nb_0, nb_1, nb_2), in label order
    int scan[2 * kCmWaves + 1];
    unsigned long long minv[kCmWaves];
};

// One breadth-first Cuthill-McKee labelling of the component of `root`,
// labels from `base`: rec[v].w = label, perm[label] = v.  rec[v].w must be
// -1 for every cell of the component.  Called by all threads of the block.
__device__ __forceinline__ PassResult cm_pass(int4 *__restrict__ rec, int32_t root, int32_t base,
                              int32_t *__restrict__ perm, PassLds &lds)
{
    int4 (&frontier)[2][kFrontierCap] = lds.frontier;
    int *scan_sh = lds.scan;
    unsigned long long *min_sh = lds.minv;

    int32_t *label = reinterpret_cast<int32_t *>(rec);  // label of cell v: label[4 v + 3]
    const int tid = threadIdx.x;

    if (tid == 0) {
        const int4 r = rec[root];
        label[4 * root + 3] = base;
        perm[base] = root;
        frontier[0][0] = make_int4(root, r.x, r.y, r.z);
    }
    __threadfence_block();
    __syncthreads();

    int a = base, b = base + 1;  // labels of the current level: [a, b)
    int cur = 0;
    int ecc = 0;
    for (;;) {
        const int F = b - a;
        int produced = 0;  // children labelled so far in this level (block-uniform)
        // One sweep covers up to kCmThreads * kPer frontier cells; thread tid
        // takes the contiguous run [tid * per, tid * per + per) of the sweep,
        // so the scan of per-thread child counts keeps the label order.
        for (int c0 = 0; c0 < F; c0 += kCmThreads * kPer) {
            const int span = min(F - c0, kCmThreads * kPer);
            const int per = (span + kCmThreads - 1) / kCmThreads;
            const int first = tid * per;

            int v[kPer], w[kPer][3];
            bool ok[kPer];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int t = first + k;
                ok[k] = k < per && t < span;
                const int ft = c0 + t;
                int4 e = frontier[cur][(ok[k] && ft < kFrontierCap) ? ft : 0];
                if (ok[k] && ft >= kFrontierCap) {
                    const int c = perm[a + ft];
                    const int4 r = rec[c];
                    e = make_int4(c, r.x, r.y, r.z);
                }
                v[k] = e.x;
                w[k][0] = e.y;
                w[k][1] = e.z;
                w[k][2] = e.w;
            }
            // records of the neighbours: their label and their neighbours
            int lw[kPer][3], x[kPer][3][3];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int4 r = ok[k] ? rec[w[k][f]] : make_int4(0, 0, 0, 0);
                    x[k][f][0] = r.x;
                    x[k][f][1] = r.y;
                    x[k][f][2] = r.z;
                    lw[k][f] = r.w;
                }
            }
            // an unlabelled neighbour ww is a child of v[k] when v[k] has the
            // smallest label among ww's neighbours inside the frontier; the
            // labels of ww's other neighbours are read for candidates only
            bool cand[kPer][3];
            int lx[kPer][3][3];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int ww = w[k][f];
                    cand[k][f] = ok[k] && ww != v[k] && !(f >= 1 && w[k][0] == ww) &&
                                 !(f == 2 && w[k][1] == ww) && lw[k][f] == -1;
#pragma unroll
                    for (int g = 0; g < 3; ++g) {
                        const int xg = x[k][f][g];
                        lx[k][f][g] = (cand[k][f] && xg != v[k]) ? label[4 * xg + 3] : -1;
                    }
                }
            }
            bool child[kPer][3];
            int kdeg[kPer][3];
            int nk[kPer];
            int total = 0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int lv = a + c0 + first + k;
                nk[k] = 0;
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    int owner = INT_MAX;
#pragma unroll
                    for (int g = 0; g < 3; ++g) {
                        const int l = x[k][f][g] == v[k] ? lv : lx[k][f][g];
                        if (l >= a && l < b && l < owner)
                            owner = l;
                    }
                    child[k][f] = cand[k][f] && owner == lv;
                    kdeg[k][f] = degree_of(w[k][f], x[k][f][0], x[k][f][1], x[k][f][2]);
                    nk[k] += child[k][f];
                }
                total += nk[k];
            }
            int sweep_total;
            int pos = produced + block_exclusive_scan(total, scan_sh, &sweep_total);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    if (child[k][f]) {
                        int rank = 0;
#pragma unroll
                        for (int g = 0; g < 3; ++g) {
                            const bool before = kdeg[k][g] < kdeg[k][f] ||
                                                (kdeg[k][g] == kdeg[k][f] && w[k][g] < w[k][f]);
                            rank += (g != f && child[k][g] && before);
                        }
                        const int p = pos + rank;
                        const int lab = b + p;
                        const int c = w[k][f];
                        label[4 * c + 3] = lab;
                        perm[lab] = c;
                        if (p < kFrontierCap)
                            frontier[cur ^ 1][p] = make_int4(c, x[k][f][0], x[k][f][1], x[k][f][2]);
                    }
                }
                pos += nk[k];
            }
            produced += sweep_total;
            // labels written by this sweep must be visible to the next one
            __threadfence_block();
            __syncthreads();
        }
        if (produced == 0)
            break;
        ++ecc;
        a = b;
        b = b + produced;
        cur ^= 1;
    }

    // last level [a, b): cell of minimum (degree, id)
    unsigned long long best = ~0ull;
    for (int t = tid; t < b - a; t += kCmThreads) {
        int4 e;
        if (t < kFrontierCap) {
            e = frontier[cur][t];
        } else {
            const int c = perm[a + t];
            const int4 r = rec[c];
            e = make_int4(c, r.x, r.y, r.z);
        }
        const int d = degree_of(e.x, e.y, e.z, e.w);
        const unsigned long long key = ((unsigned long long)d << 32) | (unsigned)e.x;
        best = key < best ? key : best;
    }
    best = block_min_u64(best, min_sh);
    PassResult r;
    r.count = b - base;
    r.ecc = ecc;
    r.pick = (int32_t)(best & 0xffffffffu);
    return r;
}

// Cuthill-McKee order of each segment [seg[s], seg[s+1]) of the graph, one
// workgroup per segment (no face may cross a segment boundary).  Within a
// segment, components are taken in order of their lowest id; each one's root
// is found by the George-Liu search from that id (label from the current
// root, take the last level's cell of minimum (degree, id), relabel from it,
// keep it while the eccentricity grows).  Output perm[label] = cell; permA
// and permB are scratch of n entries.  A cell's record label is -1 until the
// first pass reaches it, so the next component's root is the lowest cell
// still at -1.  Every loop below ends on a block-uniform condition: each
// component is labelled in full before the next starts, and the search
// moves only while the eccentricity, bounded by the segment size, strictly
// grows.
__global__ __launch_bounds__(kCmThreads) void cm_segments_kernel(
    int4 *__restrict__ rec, const int64_t *__restrict__ seg, int32_t *__restrict__ permA,
    int32_t *__restrict__ permB, int32_t *__restrict__ perm, int32_t *__restrict__ passes)
{
    __shared__ PassLds lds;
    const int tid = threadIdx.x;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    int32_t *rlabel = reinterpret_cast<int32_t *>(rec);
    int npass = 0;
    int next = s0;
    int scan_from = s0;
    while (next < s1) {
        // lowest cell of the segment no pass has reached
        int root = s1;
        for (int c0 = scan_from; c0 < s1 && root == s1; c0 += kCmThreads) {
            const int t = c0 + tid;
            const unsigned long long key =
                (t < s1 && rlabel[4 * t + 3] == -1) ? (unsigned long long)t : ~0ull;
            const unsigned long long m = block_min_u64(key, lds.minv);
            if (m != ~0ull)
                root = (int)m;
        }
        if (root >= s1)  // block-uniform; cannot happen while next < s1
            break;
        scan_from = root;

        int32_t *best = permA, *trial = permB;
        PassResult rr = cm_pass(rec, root, next, best, lds);
        ++npass;
        for (;;) {
            // Clear the component's labels before relabelling it: the first
            // component of a segment by a sweep over the whole segment (only
            // it and unreached cells live there), later ones cell by cell.
            if (next == s0) {
                for (int v = s0 + tid; v < s1; v += kCmThreads)
                    rlabel[4 * v + 3] = -1;
            } else {
                for (int l = next + tid; l < next + rr.count; l += kCmThreads)
                    rlabel[4 * best[l] + 3] = -1;
            }
            __threadfence_block();
            __syncthreads();
            const PassResult rx = cm_pass(rec, rr.pick, next, trial, lds);
            ++npass;
            if (rx.ecc > rr.ecc) {
                rr = rx;
                int32_t *t = best;
                best = trial;
                trial = t;
            } else {
                break;
            }
        }
        for (int l = next + tid; l < next + rr.count; l += kCmThreads)
            perm[l] = best[l];
        __threadfence_block();
        __syncthreads();
        next += rr.count;
    }
    if (tid == 0)
        passes[blockIdx.x] = npass;
}

__global__ void invert_kernel(int32_t n, const int32_t *__restrict__ perm,
                              int32_t *__restrict__ label)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n)
        label[perm[l]] = l;
}

// rec[v] = (nb_0[v], nb_1[v], nb_2[v], -1): no cell labelled yet.
__global__ void build_records_kernel(int32_t n, int32_t ld, const int32_t *__restrict__ nb,
                                     int4 *__restrict__ rec)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n)
        rec[v] = make_int4(nb[v], nb[ld + v], nb[2 * ld + v], -1);
}

__global__ void fill_kernel(int32_t *__restrict__ p, int32_t value, int64_t count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count)
        p[t] = value;
}

__global__ void iota_kernel(int32_t *__restrict__ p, int32_t count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count)
        p[t] = t;
}

}  // namespace

hipError_t launch_build_records(int32_t n, int32_t ld, const int32_t *nb, int4 *rec,
                                hipStream_t s)
{
    hipLaunchKernelGGL(build_records_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ld, nb,
                       rec);
    return hipGetLastError();
}

hipError_t launch_cm_segments(int4 *rec, int32_t n, int32_t n_seg, const int64_t *seg,
                              int32_t *permA, int32_t *permB, int32_t *perm, int32_t *label,
                              int32_t *passes, hipStream_t s)
{
    hipLaunchKernelGGL(cm_segments_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, seg, permA,
                       permB, perm, passes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(invert_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, perm, label);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                       value, count);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *p, int32_t count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace fvk
