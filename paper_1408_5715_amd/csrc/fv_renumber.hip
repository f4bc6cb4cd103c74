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
// among w's neighbours inside the frontier), sorts its at most three children,
// and a block-wide exclusive scan of the child counts gives every child its
// label.  The result equals the sequential order exactly.
//
// One workgroup of 1024 threads runs all levels of a component in one
// launch: levels are a few thousand cells wide, so the work per level is
// latency-bound and a grid-wide barrier per level would only add latency.
// The current and next frontier live in LDS (spilling to the global perm
// array beyond kFrontierCap cells).  Every wave leaves the level loop on the
// same block-uniform condition (an empty next level).

#include <climits>

#include "fv_internal.h"

namespace fvk {
namespace {

constexpr int kCmThreads = 1024;
constexpr int kCmWaves = kCmThreads / 64;
constexpr int kFrontierCap = 8000;  // two buffers plus scan space stay under 64 KiB of LDS

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

__global__ __launch_bounds__(kCmThreads) void cm_component_kernel(
    int32_t n, int32_t ld, const int32_t *__restrict__ nb, int32_t root, int32_t base,
    int32_t *__restrict__ label, int32_t *__restrict__ perm, CmResult *__restrict__ res)
{
    __shared__ int32_t frontier[2][kFrontierCap];
    __shared__ int scan_sh[2 * kCmWaves + 1];
    __shared__ unsigned long long min_sh[kCmWaves];

    const int32_t *nb0 = nb, *nb1 = nb + ld, *nb2 = nb + 2 * ld;
    const int tid = threadIdx.x;

    if (tid == 0) {
        label[root] = base;
        perm[base] = root;
        frontier[0][0] = root;
    }
    __syncthreads();

    int a = base, b = base + 1;  // labels of the current level: [a, b)
    int cur = 0;
    int ecc = 0;
    for (;;) {
        const int F = b - a;
        int produced = 0;  // children labelled so far in this level (block-uniform)
        for (int c0 = 0; c0 < F; c0 += kCmThreads) {
            const int t = c0 + tid;
            int kid[3];
            int kdeg[3];
            int nk = 0;
            if (t < F) {
                const int v = t < kFrontierCap ? frontier[cur][t] : perm[a + t];
                const int lv = a + t;
                const int w3[3] = {nb0[v], nb1[v], nb2[v]};
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int w = w3[f];
                    bool cand = (w != v) && !(f >= 1 && w3[0] == w) && !(f == 2 && w3[1] == w);
                    if (cand && label[w] != -1)
                        cand = false;
                    if (cand) {
                        const int x0 = nb0[w], x1 = nb1[w], x2 = nb2[w];
                        const int l0 = label[x0], l1 = label[x1], l2 = label[x2];
                        int owner = INT_MAX;
                        if (l0 >= a && l0 < b && l0 < owner)
                            owner = l0;
                        if (l1 >= a && l1 < b && l1 < owner)
                            owner = l1;
                        if (l2 >= a && l2 < b && l2 < owner)
                            owner = l2;
                        if (owner == lv) {
                            kid[nk] = w;
                            kdeg[nk] = degree_of(w, x0, x1, x2);
                            ++nk;
                        }
                    }
                }
                // order the children by (degree, id)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
#pragma unroll
                    for (int q = 0; q < 2 - p; ++q) {
                        if (q + 1 < nk) {
                            const bool swap = kdeg[q] > kdeg[q + 1] ||
                                              (kdeg[q] == kdeg[q + 1] && kid[q] > kid[q + 1]);
                            if (swap) {
                                int tk = kid[q];
                                kid[q] = kid[q + 1];
                                kid[q + 1] = tk;
                                int td = kdeg[q];
                                kdeg[q] = kdeg[q + 1];
                                kdeg[q + 1] = td;
                            }
                        }
                    }
                }
            }
            int chunk_total;
            const int off = block_exclusive_scan(nk, scan_sh, &chunk_total);
            for (int k = 0; k < nk; ++k) {
                const int pos = produced + off + k;
                const int lab = b + pos;
                label[kid[k]] = lab;
                perm[lab] = kid[k];
                if (pos < kFrontierCap)
                    frontier[cur ^ 1][pos] = kid[k];
            }
            produced += chunk_total;
            // labels written by this chunk must be visible to the next chunk
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
        const int v = t < kFrontierCap ? frontier[cur][t] : perm[a + t];
        const int d = degree_of(v, nb0[v], nb1[v], nb2[v]);
        const unsigned long long key = ((unsigned long long)d << 32) | (unsigned)v;
        best = key < best ? key : best;
    }
    best = block_min_u64(best, min_sh);
    if (tid == 0) {
        res->count = b - base;
        res->ecc = ecc;
        res->last_begin = a;
        res->pick = (int32_t)(best & 0xffffffffu);
    }
}

__global__ __launch_bounds__(kCmThreads) void find_unlabelled_kernel(
    int32_t n, const int32_t *__restrict__ label, int32_t from, int32_t *__restrict__ out)
{
    __shared__ unsigned long long min_sh[kCmWaves];
    for (int c0 = from; c0 < n; c0 += kCmThreads) {
        const int t = c0 + threadIdx.x;
        const unsigned long long key = (t < n && label[t] == -1) ? (unsigned long long)t : ~0ull;
        const unsigned long long m = block_min_u64(key, min_sh);
        if (m != ~0ull) {
            if (threadIdx.x == 0)
                *out = (int32_t)m;
            return;  // block-uniform exit
        }
    }
    if (threadIdx.x == 0)
        *out = n;
}

__global__ void commit_labels_kernel(int32_t base, int32_t count, const int32_t *__restrict__ src,
                                     int32_t *__restrict__ perm, int32_t *__restrict__ label)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) {
        const int l = base + t;
        const int v = src[l];
        perm[l] = v;
        label[v] = l;
    }
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

hipError_t launch_cm_component(int32_t n, int32_t ld, const int32_t *nb, int32_t root,
                               int32_t base, int32_t *label, int32_t *perm, CmResult *res,
                               hipStream_t s)
{
    hipLaunchKernelGGL(cm_component_kernel, dim3(1), dim3(kCmThreads), 0, s, n, ld, nb, root, base,
                       label, perm, res);
    return hipGetLastError();
}

hipError_t launch_find_unlabelled(int32_t n, const int32_t *label, int32_t from, int32_t *out,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(find_unlabelled_kernel, dim3(1), dim3(kCmThreads), 0, s, n, label, from,
                       out);
    return hipGetLastError();
}

hipError_t launch_commit_labels(int32_t base, int32_t count, const int32_t *perm_src,
                                int32_t *perm_dst, int32_t *label_dst, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(commit_labels_kernel, dim3((count + 255) / 256), dim3(256), 0, s, base,
                       count, perm_src, perm_dst, label_dst);
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
