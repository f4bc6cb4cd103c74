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
// One workgroup of 1024 threads labels a whole mesh (all levels, the
// pseudo-peripheral search and every component), in two launches around a
// grid-wide renaming of the graph: levels are a few thousand cells wide, so
// the work per level is small, and a grid-wide barrier per level (which on
// this chip means writing back and invalidating per-XCD L2 caches) would cost
// more than it saves.  A batch of independent meshes runs one such workgroup
// per mesh, side by side.  Every wave leaves the level loop on the same
// block-uniform condition (an empty next level).
//
// The graph is read as 16-byte records: three neighbours and the cell's
// label (-1 while unlabelled), so one cache-line fetch answers both "is w
// labelled" and "who are w's neighbours".  Frontier cells carry their
// neighbour lists in LDS (fetched when they were discovered), with a mask of
// the neighbours already known to be labelled then (the owner, and any whose
// label the discovery read); their records are not fetched again, since a
// labelled cell is never a child.  One CU runs the whole labelling; its cost
// is shared between the CU's path for scattered loads, its VALU and the
// synchronisation of each level, so loads are issued only by the lanes that
// need them (the records of the neighbours not known to be labelled, and the
// labels of the other neighbours of unlabelled cells), a sweep issues all its
// record loads before waiting for the first, and the sweep's code exists for
// 1, 2 and 3 frontier cells per thread so that no thread runs empty slots.

#include <climits>

#include "fv_internal.h"

namespace fvk {
namespace {

constexpr int kCmThreads = 1024;
constexpr int kCmWaves = kCmThreads / 64;
constexpr int kFrontierCap = 4096;  // frontier entries held in LDS per buffer (2 x 64 KiB + masks)
constexpr int kPer = 3;             // frontier cells per thread and sweep

typedef int i4v __attribute__((ext_vector_type(4)));  // a record as one register tuple

// Block-wide exclusive scan over 1024 threads; *total receives the sum.  One
// barrier: after it every wave scans the 16 wave totals itself.  sh must not
// be written again before every thread has returned (the callers place a
// barrier between two scans).
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
    const int t = lane < kCmWaves ? sh[lane] : 0;
    int ti = t;
#pragma unroll
    for (int d = 1; d < kCmWaves; d <<= 1) {
        const int y = __shfl_up(ti, d, 64);
        if (lane >= d)
            ti += y;
    }
    const int wave_offset = __shfl(ti - t, wid, 64);
    *total = __shfl(ti, kCmWaves - 1, 64);
    return incl - x + wave_offset;
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
    unsigned char known[2][kFrontierCap];  // bit f: nb_f was labelled at discovery
    int scan[2 * kCmWaves + 1];
    unsigned long long minv[kCmWaves];
};

// One sweep of a level [a, b) of a labelling pass: the frontier positions
// [c0, c0 + span), P per thread (thread tid takes the contiguous run
// [tid * P, tid * P + P), so the scan of per-thread child counts keeps the
// label order).  Children are labelled from b + produced on.  Waves with no
// position skip the work (P is the smallest count that covers the sweep, so
// no thread does empty slots beyond its wave's share).  Returns the number of
// children (block-uniform).  Called by all threads of the block.
template <int P>
__device__ __forceinline__ int cm_sweep(int4 *__restrict__ rec, int32_t *__restrict__ perm,
                                        PassLds &lds, int cur, int a, int b, int c0, int span,
                                        int produced)
{
    int4 (&frontier)[2][kFrontierCap] = lds.frontier;
    unsigned char (&known)[2][kFrontierCap] = lds.known;
    int32_t *label = reinterpret_cast<int32_t *>(rec);  // label of cell v: label[4 v + 3]
    const int tid = threadIdx.x;
    const int first = tid * P;
    const bool wave_busy = (tid & ~63) * P < span;  // the wave's first thread has a position

    // kept across the scan: per candidate slot, (child, rank among the cell's
    // children, mask of its neighbours known to be labelled) packed in one int
    int w[P][3], x[P][3][3], info[P][3], nk[P];
    int total = 0;
    if (wave_busy) {
        int v[P];
        unsigned kn[P];
        bool ok[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = first + k;
            ok[k] = t < span;
            const int ft = c0 + t;
            const int slot = (ok[k] && ft < kFrontierCap) ? ft : 0;
            // the LDS entry is made opaque so that the compiler keeps it an
            // LDS read instead of merging it with the global read below into
            // one generic (flat) load, whose wait would hold back every
            // global load after it
            i4v e = reinterpret_cast<const i4v *>(frontier[cur])[slot];
            unsigned kb = known[cur][slot];
            asm volatile("" : "+v"(e), "+v"(kb));
            kn[k] = kb;
            if (ok[k] && ft >= kFrontierCap) {
                const int c = perm[a + ft];
                const int4 r = rec[c];
                e = i4v{c, r.x, r.y, r.z};
                kn[k] = 0;
            }
            v[k] = e[0];
            w[k][0] = e[1];
            w[k][1] = e[2];
            w[k][2] = e[3];
        }
        // records of the neighbours not known to be labelled: their label and
        // their neighbours (a skipped one reads as labelled, w = 0).  The
        // empty asm statements after the loop make each record's value opaque
        // where it is used, so the compiler cannot move the uses into the
        // branch that loads it (which would wait for each load before issuing
        // the next): all loads are in flight together.
        const i4v *recv = reinterpret_cast<const i4v *>(rec);
        i4v rw[P][3];
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const bool fetch = ok[k] && !((kn[k] >> f) & 1u);
                rw[k][f] = i4v{0, 0, 0, 0};
                if (fetch)
                    rw[k][f] = recv[w[k][f]];
            }
        }
        int lw[P][3];
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                i4v r = rw[k][f];
                asm volatile("" : "+v"(r));
                x[k][f][0] = r[0];
                x[k][f][1] = r[1];
                x[k][f][2] = r[2];
                lw[k][f] = r[3];
            }
        }
        // an unlabelled neighbour ww is a child of v[k] when v[k] has the
        // smallest label among ww's neighbours inside the frontier; the labels
        // of ww's other neighbours are read for candidates only
        bool cand[P][3];
        int lx[P][3][3];
#pragma unroll
        for (int k = 0; k < P; ++k) {
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
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int lv = a + c0 + first + k;
            bool child[3];
            int kdeg[3];
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
                child[f] = cand[k][f] && owner == lv;
                kdeg[f] = degree_of(w[k][f], x[k][f][0], x[k][f][1], x[k][f][2]);
                nk[k] += child[f];
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                int rank = 0;
                unsigned m = 0;
#pragma unroll
                for (int g = 0; g < 3; ++g) {
                    const bool before =
                        kdeg[g] < kdeg[f] || (kdeg[g] == kdeg[f] && w[k][g] < w[k][f]);
                    rank += (g != f && child[g] && before);
                    // c's neighbours known to be labelled: its owner and those
                    // whose label was read above
                    m |= (unsigned)(x[k][f][g] == v[k] || lx[k][f][g] != -1) << g;
                }
                info[k][f] = child[f] ? (int)(1u | (unsigned)rank << 1 | m << 3) : 0;
            }
            total += nk[k];
        }
    }
    int sweep_total;
    int pos = produced + block_exclusive_scan(total, lds.scan, &sweep_total);
    if (wave_busy) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const int in = info[k][f];
                if (in & 1) {
                    const int p = pos + ((in >> 1) & 3);
                    const int lab = b + p;
                    const int c = w[k][f];
                    label[4 * c + 3] = lab;
                    perm[lab] = c;
                    if (p < kFrontierCap) {
                        frontier[cur ^ 1][p] = make_int4(c, x[k][f][0], x[k][f][1], x[k][f][2]);
                        known[cur ^ 1][p] = (unsigned char)(in >> 3);
                    }
                }
            }
            pos += nk[k];
        }
    }
    return sweep_total;
}

// One breadth-first Cuthill-McKee labelling of the component of `root`,
// labels from `base`: rec[v].w = label, perm[label] = v.  rec[v].w must be
// -1 for every cell of the component.  Called by all threads of the block.
__device__ __forceinline__ PassResult cm_pass(int4 *__restrict__ rec, int32_t root, int32_t base,
                              int32_t *__restrict__ perm, PassLds &lds)
{
    int4 (&frontier)[2][kFrontierCap] = lds.frontier;
    unsigned char (&known)[2][kFrontierCap] = lds.known;
    int *scan_sh = lds.scan;
    unsigned long long *min_sh = lds.minv;

    int32_t *label = reinterpret_cast<int32_t *>(rec);  // label of cell v: label[4 v + 3]
    const int tid = threadIdx.x;

    if (tid == 0) {
        const int4 r = rec[root];
        label[4 * root + 3] = base;
        perm[base] = root;
        frontier[0][0] = make_int4(root, r.x, r.y, r.z);
        known[0][0] = 0;
    }
    __threadfence_block();
    __syncthreads();

    int a = base, b = base + 1;  // labels of the current level: [a, b)
    int cur = 0;
    int ecc = 0;
    for (;;) {
        const int F = b - a;
        int produced = 0;  // children labelled so far in this level (block-uniform)
        // One sweep covers up to kCmThreads * kPer frontier cells, with the
        // smallest per-thread count that covers them.
        for (int c0 = 0; c0 < F; c0 += kCmThreads * kPer) {
            const int span = min(F - c0, kCmThreads * kPer);
            const int per = (span + kCmThreads - 1) / kCmThreads;
            int sweep_total;
            if (per == 1)
                sweep_total = cm_sweep<1>(rec, perm, lds, cur, a, b, c0, span, produced);
            else if (per == 2)
                sweep_total = cm_sweep<2>(rec, perm, lds, cur, a, b, c0, span, produced);
            else
                sweep_total = cm_sweep<3>(rec, perm, lds, cur, a, b, c0, span, produced);
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

// Cuthill-McKee order of each segment [seg[s], seg[s+1]), one workgroup per
// segment (no face may cross a segment boundary).  Within a segment,
// components are taken in order of their lowest id; each one's root is found
// by the George-Liu search from that id (label from the current root, take
// the last level's cell of minimum (degree, id), relabel from it, keep it
// while the eccentricity grows).  Output perm[label] = cell; permA and permB
// are scratch of n entries.  A cell's record label is -1 until the first
// pass reaches it, so the next component's root is the lowest cell still at
// -1.
//
// The search's second pass over the first component usually only confirms
// that the eccentricity does not grow, and level sets do not depend on the
// order inside a level.  So that pass runs on a copy of the component's
// graph renamed by the first pass's labels (rec2, built by
// cm_translate_kernel), whose records lie far closer together in memory than
// those of an arbitrary input order; only its eccentricity is used.  If it
// exceeds the first pass's, the search continues exactly as above on the
// original graph (where ties between children are broken by the original
// ids).
//
// cm_first_kernel: the first pass of every segment (root: the segment's
// lowest cell, into permA); state[s] = (cells labelled, eccentricity, pick).
__global__ __launch_bounds__(kCmThreads) void cm_first_kernel(int4 *__restrict__ rec,
                                                              const int64_t *__restrict__ seg,
                                                              int32_t *__restrict__ permA,
                                                              int4 *__restrict__ state)
{
    __shared__ PassLds lds;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    if (s0 >= s1) {  // block-uniform; uploads reject empty segments
        if (threadIdx.x == 0)
            state[blockIdx.x] = make_int4(0, 0, s0, 0);
        return;
    }
    const PassResult r = cm_pass(rec, s0, s0, permA, lds);
    if (threadIdx.x == 0)
        state[blockIdx.x] = make_int4(r.count, r.ecc, r.pick, 0);
}

// rec2[l] = (labels of the three neighbours of the cell labelled l, -1) for
// every label l of a segment's first component (labels from the first pass,
// which are also the positions in rec2); other positions are left alone.
__global__ void cm_translate_kernel(int32_t n, int32_t n_seg, const int64_t *__restrict__ seg,
                                    const int4 *__restrict__ state, const int4 *__restrict__ rec,
                                    const int32_t *__restrict__ permA, int4 *__restrict__ rec2)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n)
        return;
    int lo = 0, hi = n_seg - 1;  // segment of l: the last s with seg[s] <= l
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= l)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (l - (int)seg[lo] >= state[lo].x)
        return;
    const int4 r = rec[permA[l]];
    rec2[l] = make_int4(rec[r.x].w, rec[r.y].w, rec[r.z].w, -1);
}

// The rest of the search for every segment, after cm_first_kernel and
// cm_translate_kernel, as one loop with one labelling pass per iteration:
// kProbe (the first component's pick, on the renamed copy), kRoot (the root
// of the next component: its lowest unreached cell), kSearch (clear the
// component's labels, relabel it from the pick of the best pass so far).
// Every loop ends on a block-uniform condition: each component is labelled
// in full before the next starts, and the search moves only while the
// eccentricity, bounded by the segment size, strictly grows.
__global__ __launch_bounds__(kCmThreads) void cm_finish_kernel(
    int4 *__restrict__ rec, int4 *__restrict__ rec2, const int64_t *__restrict__ seg,
    const int4 *__restrict__ state, int32_t *__restrict__ permA, int32_t *__restrict__ permB,
    int32_t *__restrict__ perm, int32_t *__restrict__ passes)
{
    enum { kProbe, kRoot, kSearch };
    __shared__ PassLds lds;
    const int tid = threadIdx.x;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    int32_t *rlabel = reinterpret_cast<int32_t *>(rec);
    const int4 st = state[blockIdx.x];
    PassResult rr;  // best pass of the current component
    rr.count = st.x;
    rr.ecc = st.y;
    rr.pick = st.z;
    int32_t *best = permA, *trial = permB;
    int npass = s0 < s1 ? 1 : 0;
    int next = s0;
    int scan_from = s0;
    int mode = s0 < s1 ? kProbe : kRoot;
    for (;;) {
        int4 *graph = rec;
        int root;
        int32_t *out = trial;
        if (mode == kProbe) {
            graph = rec2;
            root = rlabel[4 * rr.pick + 3];
        } else if (mode == kRoot) {
            if (next >= s1)
                break;
            root = s1;
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
            out = best;
        } else {
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
            root = rr.pick;
        }
        const PassResult r = cm_pass(graph, root, next, out, lds);
        ++npass;
        if (mode == kRoot) {
            rr = r;
            mode = kSearch;
            continue;
        }
        if (r.ecc > rr.ecc) {
            // a probe only reports the growth: the search then relabels
            // exactly from the same pick
            if (mode == kSearch) {
                rr = r;
                int32_t *t = best;
                best = trial;
                trial = t;
            }
            mode = kSearch;
            continue;
        }
        for (int l = next + tid; l < next + rr.count; l += kCmThreads)
            perm[l] = best[l];
        __threadfence_block();
        __syncthreads();
        next += rr.count;
        mode = kRoot;
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

hipError_t launch_cm_segments(int4 *rec, int4 *rec2, int4 *state, int32_t n, int32_t n_seg,
                              const int64_t *seg, int32_t *permA, int32_t *permB, int32_t *perm,
                              int32_t *label, int32_t *passes, hipStream_t s)
{
    hipLaunchKernelGGL(cm_first_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, seg, permA,
                       state);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_translate_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, n_seg, seg,
                       state, rec, permA, rec2);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_finish_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, rec2, seg,
                       state, permA, permB, perm, passes);
    e = hipGetLastError();
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
