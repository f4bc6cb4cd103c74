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
// same labelling one level at a time: the frontier cells propose their
// unvisited neighbours, an LDS hash set keeps the smallest proposing label
// of each, every owner ranks its at most three children, and a block-wide
// exclusive scan of the child counts gives every child its label.  The
// result equals the sequential order exactly.
//
// One workgroup of 1024 threads labels a whole mesh (all levels, the
// pseudo-peripheral search and every component): levels are a few thousand
// cells wide, so the work per level is small, and a grid-wide barrier per
// level (which on this chip means writing back and invalidating per-XCD L2
// caches) would cost more than it saves.  A batch of independent meshes runs
// one such workgroup per mesh, side by side.  Every wave leaves the level
// loop on the same block-uniform condition (an empty next level).
//
// The graph is read as 16-byte records: three neighbours and the cell's
// mark (negative while unvisited), so one cache-line fetch answers both "is w
// visited" and "who are w's neighbours".  Frontier cells carry their
// neighbour lists in LDS (fetched when they were discovered), their
// discoverer marked as visited; its record is not fetched again.  One CU
// runs a pass; its cost is shared between the CU's path for scattered loads,
// its VALU and the synchronisation of each level, so loads are issued only by
// the lanes that need them, a sweep issues all its record loads before
// waiting for the first, and the sweep's code exists for 1, 2 and 3 frontier
// cells per thread so that no thread runs empty slots.

#include <climits>

#include "fv_internal.h"

namespace fvk {
namespace {

constexpr int kCmThreads = 1024;
constexpr int kCmWaves = kCmThreads / 64;
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

// A cell's record, as the passes read it: (nb_0, nb_1, nb_2, mark).  A
// neighbour equal to the cell itself or to an earlier neighbour is stored as
// its bitwise complement (negative, since ids are not), so a pass skips it
// with one sign test; the mark is the cell's label or level once visited,
// and ~degree (negative) before.  The degree counts the distinct neighbours
// other than the cell itself: the entries that are not complemented.
__device__ __forceinline__ int unvisited_mark(int4 r)
{
    return ~((r.x >= 0) + (r.y >= 0) + (r.z >= 0));
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


struct BfsResult {
    int count;  // cells reached (the component of the root)
    int ecc;    // eccentricity of the root
    int pick;   // last-level cell of minimum (degree, id)
    int width;  // largest level
};

// ---- breadth-first passes, with or without Cuthill-McKee labels ----------
//
// A pass walks the levels of the root's component one sweep at a time.  A
// frontier cell fetches the records of its neighbours not known to be
// visited; the record's fourth field marks a visited cell (negative while
// unvisited), so the same load that brings a cell's neighbour list also says
// whether it is new.  A new cell proposed by several frontier cells of one
// sweep is resolved in an LDS hash set keyed by the cell:
//   - without labels (the search's confirming sweep, which needs only the
//     eccentricity) the first proposal to insert the cell takes it (one LDS
//     compare-and-swap per proposal);
//   - with labels the set keeps, per cell, the smallest proposing frontier
//     position (a 64-bit slot: cell in the high half, position in the low
//     half; compare-and-swap into an empty slot, else an LDS minimum).  The
//     frontier is held in label order and sweeps run in that order, so after
//     one barrier each proposer knows whether it is the cell's owner, the
//     frontier neighbour of smallest label: a cell proposed in an earlier
//     sweep of the level was labelled by it, and neighbours in the cell's
//     own level or later carry larger labels.  An owner ranks its children
//     by (degree, id), and the scan of child counts in frontier order gives
//     every child its label.
// One round of scattered memory traffic per level, and no global atomics
// (which serialise where neighbouring cells share a cache line).
//
// Frontier entries are (cell, nb_0, nb_1, nb_2) from the cell's record, kept
// in LDS while they fit; the discoverer, known to be visited, is complemented
// there like the record's self and repeated neighbours, so a neighbour is
// proposed exactly when its entry is not negative.

constexpr int kHashSlots = 8192;  // > 2 * kCmThreads * kPer + 1: the set never fills
constexpr unsigned kHashEmpty = 0xffffffffu;
constexpr unsigned long long kPairEmpty = ~0ull;
static_assert(kHashSlots > 2 * kCmThreads * kPer + 1,
              "hash set must outgrow a sweep's new cells");

template <bool kLabel>
struct SetSlot {
    typedef unsigned T;  // a cell
};
template <>
struct SetSlot<true> {
    typedef unsigned long long T;  // (cell << 32) | smallest proposing position
};

template <bool kLabel>
struct BfsLds {
    // frontier entries held in LDS per buffer: what is left of the 160 KiB
    // once the set (64 KiB with labels, 32 KiB without) is placed
    static constexpr int kCap = kLabel ? 3056 : 4080;
    int4 frontier[2][kCap];
    typename SetSlot<kLabel>::T set[kHashSlots];
    int scan[2 * kCmWaves + 1];
    unsigned long long minv[kCmWaves];
};
static_assert(sizeof(BfsLds<true>) <= 160 * 1024, "labelling pass exceeds the LDS");
static_assert(sizeof(BfsLds<false>) <= 160 * 1024, "breadth-first pass exceeds the LDS");

__device__ __forceinline__ unsigned set_hash(int c)
{
    return ((unsigned)c * 0x9E3779B1u) >> 19;  // 13 bits
}

// Insert c into the set, probing from slot h on; the slot if this call
// inserted it (claims c), else -1.  At most one sweep's new cells live in the
// set, fewer than kHashSlots, so an empty slot is always reached; the loop is
// bounded by the table size.  The sweeps issue every proposal's first probe
// at once and come here only after a collision.
__device__ __forceinline__ int claim_from(unsigned *set, int c, unsigned h)
{
    for (int probe = 0; probe < kHashSlots; ++probe) {
        const unsigned old = atomicCAS(set + h, kHashEmpty, (unsigned)c);
        if (old == kHashEmpty)
            return (int)h;
        if (old == (unsigned)c)
            return -1;
        h = (h + 1) & (kHashSlots - 1);
    }
    return -1;
}

// Record the proposal of c by frontier position pos, probing from slot h on;
// returns c's slot (the smallest proposing position sits in its low half
// once every proposal of the sweep is in).  Bounded like claim_from, and like
// it reached only after a collision.
__device__ __forceinline__ int propose_from(unsigned long long *set, int c, int pos, unsigned h)
{
    const unsigned long long val = (unsigned long long)(unsigned)c << 32 | (unsigned)pos;
    for (int probe = 0; probe < kHashSlots; ++probe) {
        const unsigned long long old = atomicCAS(set + h, kPairEmpty, val);
        if (old == kPairEmpty)
            return (int)h;
        if ((unsigned)(old >> 32) == (unsigned)c) {
            if (old > val)
                atomicMin(set + h, val);
            return (int)h;
        }
        h = (h + 1) & (kHashSlots - 1);
    }
    return -1;
}

// One sweep of a level [a, b): frontier positions [c0, c0 + span), P per
// thread (thread tid takes the contiguous run [tid * P, tid * P + P), so the
// scan of per-thread counts keeps frontier order; waves with no position skip
// the work).  New cells are appended from b + produced on: ord[b + p]
// receives the p-th new cell, whose record's fourth field becomes its label
// b + p (kLabel) or `level`.  Returns the number of new cells
// (block-uniform).  The set must be empty on entry and is empty again on
// return.  Called by all threads of the block.
template <int P, bool kLabel>
__device__ __forceinline__ int bfs_sweep(int4 *__restrict__ graph, int32_t *__restrict__ ord,
                                         BfsLds<kLabel> &lds, int cur, int a, int b, int c0,
                                         int span, int produced, int level)
{
    constexpr int kCap = BfsLds<kLabel>::kCap;
    const int tid = threadIdx.x;
    const int first = tid * P;
    const bool wave_busy = (tid & ~63) * P < span;

    int v[P], w[P][3];
    i4v rw[P][3];
    int slot[P][3];  // the proposal's slot (with labels) or the claimed slot, -1 for none
    unsigned won[P];  // bit f: w[k][f] is new and joins through this thread
    if (wave_busy) {
        bool ok[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = first + k;
            ok[k] = t < span;
            const int ft = c0 + t;
            const int at = (ok[k] && ft < kCap) ? ft : 0;
            // the LDS entry is made opaque so that the compiler keeps it an
            // LDS read instead of merging it with the global reads below into
            // one generic (flat) load, whose wait would hold back every
            // global load after it
            i4v e = reinterpret_cast<const i4v *>(lds.frontier[cur])[at];
            asm volatile("" : "+v"(e));
            if (ok[k] && ft >= kCap) {
                const int c = ord[a + ft];
                const int4 r = graph[c];
                e = i4v{c, r.x, r.y, r.z};
            }
            v[k] = e[0];
#pragma unroll
            for (int f = 0; f < 3; ++f)
                w[k][f] = e[f + 1];
        }
        // records of the neighbours not known to be visited, all in flight
        // together (the empty asm statements keep the uses out of the
        // branches that load them)
        const i4v *gv = reinterpret_cast<const i4v *>(graph);
        bool cand[P][3];
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const int ww = w[k][f];
                cand[k][f] = ok[k] && ww >= 0;
                rw[k][f] = i4v{0, 0, 0, 0};
                if (cand[k][f])
                    rw[k][f] = gv[ww];
            }
        }
        // every proposal's first probe at once (one compare-and-swap each,
        // all in flight together), then the rare collisions one by one
        typedef typename SetSlot<kLabel>::T Slot;
        const Slot empty = kLabel ? (Slot)kPairEmpty : (Slot)kHashEmpty;
        bool fresh[P][3];
        unsigned h0[P][3];
        Slot old[P][3];
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                i4v r = rw[k][f];
                asm volatile("" : "+v"(r));
                rw[k][f] = r;
                fresh[k][f] = cand[k][f] && r[3] < 0;
                h0[k][f] = set_hash(w[k][f]);
                Slot val;
                if constexpr (kLabel)
                    val = (Slot)(unsigned)w[k][f] << 32 | (unsigned)(first + k);
                else
                    val = (Slot)(unsigned)w[k][f];
                old[k][f] = empty;
                if (fresh[k][f])
                    old[k][f] = atomicCAS(lds.set + h0[k][f], empty, val);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            won[k] = 0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const int c = w[k][f];
                const Slot o = old[k][f];
                if constexpr (kLabel) {
                    int sl = -1;
                    if (fresh[k][f]) {
                        const unsigned h1 = (h0[k][f] + 1) & (kHashSlots - 1);
                        if (o == empty) {
                            sl = (int)h0[k][f];
                        } else if ((unsigned)(o >> 32) == (unsigned)c) {
                            sl = (int)h0[k][f];
                            if ((unsigned)o > (unsigned)(first + k))
                                atomicMin(lds.set + sl,
                                          (Slot)(unsigned)c << 32 | (unsigned)(first + k));
                        } else {
                            sl = propose_from(lds.set, c, first + k, h1);
                        }
                    }
                    slot[k][f] = sl;
                } else {
                    int sl = -1;
                    if (fresh[k][f]) {
                        const unsigned h1 = (h0[k][f] + 1) & (kHashSlots - 1);
                        if (o == empty)
                            sl = (int)h0[k][f];
                        else if (o != (Slot)(unsigned)c)
                            sl = claim_from(lds.set, c, h1);
                    }
                    slot[k][f] = sl;
                    won[k] |= (unsigned)(sl >= 0) << f;
                }
            }
        }
    }
    // with labels: every proposal of the sweep is in; owners take their
    // children, ranked by (degree, id)
    int rank[P][3];
    int total = 0;
    if constexpr (kLabel) {
        __syncthreads();
        if (wave_busy) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                unsigned long long key[3];  // (degree, id); distinct for distinct cells
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int s = slot[k][f];
                    const bool own = s >= 0 && (unsigned)lds.set[s] == (unsigned)(first + k);
                    won[k] |= (unsigned)own << f;
                    key[f] = (unsigned long long)(unsigned)~rw[k][f][3] << 32 | (unsigned)w[k][f];
                }
                const unsigned m = won[k];
                const int c01 = key[0] < key[1], c02 = key[0] < key[2], c12 = key[1] < key[2];
                const int b0 = m & 1u, b1 = (m >> 1) & 1u, b2 = (m >> 2) & 1u;
                rank[k][0] = (b1 & (c01 ^ 1)) + (b2 & (c02 ^ 1));
                rank[k][1] = (b0 & c01) + (b2 & (c12 ^ 1));
                rank[k][2] = (b0 & c02) + (b1 & c12);
                total += __builtin_popcount(won[k]);
            }
        }
    } else {
        if (wave_busy) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
#pragma unroll
                for (int f = 0; f < 3; ++f)
                    rank[k][f] = __builtin_popcount(won[k] & ((1u << f) - 1u));
                total += __builtin_popcount(won[k]);
            }
        }
    }
    int sweep_total;
    int pos = produced + block_exclusive_scan(total, lds.scan, &sweep_total);
    // every use of the set in this sweep is done: empty it for the next sweep
    // (the caller's barrier separates this from the next sweep's inserts).
    // Every filled slot holds a cell that some thread proposed (with labels)
    // or claimed, so these threads empty exactly the filled slots.
    if (wave_busy) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (slot[k][f] >= 0)
                    lds.set[slot[k][f]] = kLabel ? kPairEmpty : kHashEmpty;
            }
        }
    }
    if (wave_busy) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if ((won[k] >> f) & 1u) {
                    const int p = pos + rank[k][f];
                    const int c = w[k][f];
                    const i4v r = rw[k][f];
                    reinterpret_cast<int32_t *>(graph)[4 * c + 3] = kLabel ? b + p : level;
                    ord[b + p] = c;
                    if (p < kCap) {
                        // the discoverer is known to be visited
                        lds.frontier[cur ^ 1][p] =
                            make_int4(c, r[0] == v[k] ? ~r[0] : r[0], r[1] == v[k] ? ~r[1] : r[1],
                                      r[2] == v[k] ? ~r[2] : r[2]);
                    }
                }
            }
            pos += __builtin_popcount(won[k]);
        }
    }
    return sweep_total;
}

// Breadth-first pass over the component of `root` in `graph` (records
// (nb_0, nb_1, nb_2, mark), the mark negative for every cell of the
// component on entry).  ord[base + p] receives the p-th cell reached (levels in order).
// With kLabel the order is the Cuthill-McKee labelling from the root, labels
// from base, and every record's mark becomes its cell's label; without, the
// marks are levels and the order within a level is arbitrary.  Called by all
// threads of the block.
template <bool kLabel>
__device__ __forceinline__ BfsResult bfs_pass(int4 *__restrict__ graph, int32_t root,
                                              int32_t base, int32_t *__restrict__ ord,
                                              BfsLds<kLabel> &lds)
{
    constexpr int kCap = BfsLds<kLabel>::kCap;
    const int tid = threadIdx.x;
    for (int t = tid; t < kHashSlots; t += kCmThreads)
        lds.set[t] = kLabel ? kPairEmpty : kHashEmpty;
    if (tid == 0) {
        const int4 r = graph[root];
        reinterpret_cast<int32_t *>(graph)[4 * root + 3] = kLabel ? base : 0;
        ord[base] = root;
        lds.frontier[0][0] = make_int4(root, r.x, r.y, r.z);
    }
    __threadfence_block();
    __syncthreads();

    int a = base, b = base + 1;  // the current level: [a, b)
    int cur = 0, ecc = 0, width = 1;
    for (;;) {
        const int F = b - a;
        int produced = 0;  // new cells so far in this level (block-uniform)
        // One sweep covers up to kCmThreads * kPer frontier cells, with the
        // smallest per-thread count that covers them.
        for (int c0 = 0; c0 < F; c0 += kCmThreads * kPer) {
            const int span = min(F - c0, kCmThreads * kPer);
            const int per = (span + kCmThreads - 1) / kCmThreads;
            int st;
            if (per == 1)
                st = bfs_sweep<1, kLabel>(graph, ord, lds, cur, a, b, c0, span, produced, ecc + 1);
            else if (per == 2)
                st = bfs_sweep<2, kLabel>(graph, ord, lds, cur, a, b, c0, span, produced, ecc + 1);
            else
                st = bfs_sweep<3, kLabel>(graph, ord, lds, cur, a, b, c0, span, produced, ecc + 1);
            // block-uniform: held in scalar registers from here on
            produced += __builtin_amdgcn_readfirstlane(st);
            // marks written by this sweep must be visible to the next one
            __threadfence_block();
            __syncthreads();
        }
        if (produced == 0)
            break;
        ++ecc;
        a = b;
        b += produced;
        width = max(width, produced);
        cur ^= 1;
    }

    // last level [a, b): cell of minimum (degree, id)
    unsigned long long best = ~0ull;
    for (int t = tid; t < b - a; t += kCmThreads) {
        int4 e;  // complemented neighbours decode to themselves
        if (t < kCap) {
            e = lds.frontier[cur][t];
        } else {
            const int c = ord[a + t];
            e = graph[c];
            e = make_int4(c, e.x, e.y, e.z);
        }
        const int c = e.x;
        const int d = degree_of(c, e.y < 0 ? ~e.y : e.y, e.z < 0 ? ~e.z : e.z, e.w < 0 ? ~e.w : e.w);
        const unsigned long long key = ((unsigned long long)d << 32) | (unsigned)c;
        best = key < best ? key : best;
    }
    best = block_min_u64(best, lds.minv);
    BfsResult res;
    res.count = b - base;
    res.ecc = ecc;
    res.pick = __builtin_amdgcn_readfirstlane((int32_t)(best & 0xffffffffu));
    res.width = width;
    return res;
}

// Cuthill-McKee order of each segment [seg[s], seg[s+1]), one workgroup per
// segment (no face may cross a segment boundary).  Within a segment,
// components are taken in order of their lowest id; each one's root is found
// by the George-Liu search from that id (level structure from the current
// root, take the last level's cell of minimum (degree, id), move to it while
// the eccentricity grows).  Output perm[label] = cell.
//
// The first component of a segment (every cell, for a connected mesh) takes
// the fast route:
//   cm_first_kernel      labelling pass from the segment's lowest id on the
//                        uploaded graph: its labels (into perm), which are
//                        the result when the search does not move (the root
//                        then stays the lowest id), eccentricity and pick;
// and, on a second stream,
//   cm_rename_kernel     the component's graph renamed by those labels (rec2:
//                        neighbours as labels), in which every level is a
//                        contiguous range and neighbours sit close;
//   cm_probe_kernel      the sweep from the pick on rec2 (the search's
//                        second step);
// then, on the first stream,
//   cm_finish_kernel     for a search that moves, and for every later
//                        component, the rest of the search with full
//                        labelling passes on the uploaded graph.  With
//                        assume_stays the finish does not wait for the
//                        probe: it keeps the first pass's labels and goes on
//                        with the later components; the caller checks the
//                        probe's eccentricities afterwards and relabels
//                        exactly if some search would have moved.
//
// cm_first_kernel: state[s] = (cells reached, eccentricity, pick, widest level).
__global__ __launch_bounds__(kCmThreads) void cm_first_kernel(int4 *__restrict__ rec,
                                                              const int64_t *__restrict__ seg,
                                                              int32_t *__restrict__ perm,
                                                              int4 *__restrict__ state)
{
    __shared__ BfsLds<true> lds;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    if (s0 >= s1) {  // block-uniform; uploads reject empty segments
        if (threadIdx.x == 0)
            state[blockIdx.x] = make_int4(0, 0, s0, 0);
        return;
    }
    const BfsResult r = bfs_pass<true>(rec, s0, s0, perm, lds);
    if (threadIdx.x == 0)
        state[blockIdx.x] = make_int4(r.count, r.ecc, r.pick, r.width);
}

// Segment of position l: the last s with seg[s] <= l.
__device__ __forceinline__ int segment_of(int l, int n_seg, const int64_t *__restrict__ seg)
{
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= l)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// rec2[L] = the record of the cell v labelled L with neighbours as labels
// (same encoding as rec), for the cells of each segment's first component,
// read from the labelled records themselves (after the first pass a cell's
// mark is its label); probe[s] = the label of the segment's pick (the probe
// sweep's root).  Labels outside the first component's range (later
// components, or cells not labelled yet) are skipped.
__global__ void cm_rename_kernel(int32_t n, int32_t n_seg, const int64_t *__restrict__ seg,
                                 const int4 *__restrict__ state, const int4 *__restrict__ rec,
                                 int4 *__restrict__ rec2, int32_t *__restrict__ root)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n)
        return;
    const int sg = segment_of(v, n_seg, seg);
    const int s0 = (int)seg[sg];
    const int4 st = state[sg];
    const int4 r = rec[v];
    const int L = r.w;
    if (L < s0 || L - s0 >= st.x)
        return;
    const int *label = reinterpret_cast<const int *>(rec) + 3;  // label of cell x: label[4 x]
    const int nbr[3] = {r.x, r.y, r.z};
    int q[3];
#pragma unroll
    for (int f = 0; f < 3; ++f)
        q[f] = nbr[f] >= 0 ? label[4 * nbr[f]] : ~label[4 * ~nbr[f]];
    rec2[L] = make_int4(q[0], q[1], q[2], ~((q[0] >= 0) + (q[1] >= 0) + (q[2] >= 0)));
    if (v == st.z)
        root[sg] = L;
}

// The sweep from the first component's pick on rec2, one workgroup per
// segment: on entry probe[s] holds the pick's label (cm_rename_kernel), on
// exit the sweep's eccentricity.  It may run beside the finish kernel, so it
// writes only rec2's marks, its own order ordC and probe, and reads nothing
// the finish kernel writes (the pick it finds is not used).
__global__ __launch_bounds__(kCmThreads) void cm_probe_kernel(
    int4 *__restrict__ rec2, const int64_t *__restrict__ seg, int32_t *__restrict__ ordC,
    int32_t *__restrict__ probe)
{
    __shared__ BfsLds<false> lds;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    if (s0 >= s1)
        return;
    const int root = probe[blockIdx.x];
    if (root < s0 || root >= s1) {  // block-uniform; cannot happen (the pick is in the component)
        __syncthreads();
        if (threadIdx.x == 0)
            probe[blockIdx.x] = INT_MAX;  // makes the finish run the exact search
        return;
    }
    const BfsResult r = bfs_pass<false>(rec2, root, s0, ordC, lds);
    __syncthreads();  // every thread has read probe[] before it is overwritten
    if (threadIdx.x == 0)
        probe[blockIdx.x] = r.ecc;
}

// The rest of the search for every segment, after cm_first_kernel, as one
// loop with one full labelling pass (on the uploaded graph) per iteration:
// kRoot (the root of the next component: its lowest cell not yet labelled),
// kSearch (clear the component's labels, relabel it from the pick of the
// best pass so far).  Every loop ends on a block-uniform condition: each
// component is labelled in full before the next starts, and the search moves
// only while the eccentricity, bounded by the segment size, strictly grows.
// The labels of the best pass of the current component are in `best`, which
// starts as perm (the first pass's labels) and trades places with permA.
__global__ __launch_bounds__(kCmThreads) void cm_finish_kernel(
    int4 *__restrict__ rec, const int64_t *__restrict__ seg, const int4 *__restrict__ state,
    const int32_t *__restrict__ probe, int32_t *__restrict__ permA, int32_t *__restrict__ perm,
    int32_t *__restrict__ passes, int32_t assume_stays)
{
    enum { kRoot, kSearch };
    __shared__ BfsLds<true> lds;
    const int tid = threadIdx.x;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    int32_t *rlabel = reinterpret_cast<int32_t *>(rec);
    const int4 st = state[blockIdx.x];
    BfsResult rr;  // best pass of the current component
    rr.count = st.x;
    rr.ecc = st.y;
    rr.pick = st.z;
    rr.width = st.w;
    int32_t *best = perm, *trial = permA;
    int npass = s0 < s1 ? 2 : 0;  // the two sweeps of the fast route
    int next = s0;
    int scan_from = s0;
    int mode = kRoot;
    if (s0 < s1) {
        if (!assume_stays && probe[blockIdx.x] > rr.ecc)
            mode = kSearch;  // relabel exactly from the same pick
        else
            next += rr.count;
    }
    for (;;) {
        int root;
        int32_t *out = trial;
        if (mode == kRoot) {
            if (next >= s1)
                break;
            root = s1;
            for (int c0 = scan_from; c0 < s1 && root == s1; c0 += kCmThreads) {
                const int t = c0 + tid;
                const unsigned long long key =
                    (t < s1 && rlabel[4 * t + 3] < 0) ? (unsigned long long)t : ~0ull;
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
                    rlabel[4 * v + 3] = unvisited_mark(rec[v]);
            } else {
                for (int l = next + tid; l < next + rr.count; l += kCmThreads)
                    rlabel[4 * best[l] + 3] = unvisited_mark(rec[best[l]]);
            }
            __threadfence_block();
            __syncthreads();
            root = rr.pick;
        }
        const BfsResult r = bfs_pass<true>(rec, root, next, out, lds);
        ++npass;
        if (mode == kRoot) {
            rr = r;
            mode = kSearch;
            continue;
        }
        if (r.ecc > rr.ecc) {
            rr = r;
            int32_t *t = best;
            best = trial;
            trial = t;
            mode = kSearch;
            continue;
        }
        if (best != perm) {
            for (int l = next + tid; l < next + rr.count; l += kCmThreads)
                perm[l] = best[l];
        }
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

// rec[v]: the records of the graph nb (int32 [n][3]), no cell visited yet.
__global__ void build_records_kernel(int32_t n, const int32_t *__restrict__ nb,
                                     int4 *__restrict__ rec)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n)
        return;
    const int a = nb[3 * v], b = nb[3 * v + 1], c = nb[3 * v + 2];
    const int4 r = make_int4(a == v ? ~a : a, (b == v || b == a) ? ~b : b,
                             (c == v || c == a || c == b) ? ~c : c, 0);
    rec[v] = make_int4(r.x, r.y, r.z, unvisited_mark(r));
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

hipError_t launch_build_records(int32_t n, const int32_t *nb, int4 *rec, hipStream_t s)
{
    hipLaunchKernelGGL(build_records_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, nb, rec);
    return hipGetLastError();
}

hipError_t launch_cm_confirm(const int4 *rec, int4 *rec2, const int4 *state, int32_t *probe,
                             int32_t n, int32_t n_seg, const int64_t *seg, int32_t *ordC,
                             hipStream_t s, hipStream_t side, hipEvent_t labelled,
                             hipEvent_t probed)
{
    // on the second stream, after everything queued on s so far
    hipError_t e = hipEventRecord(labelled, s);
    if (e != hipSuccess)
        return e;
    if ((e = hipStreamWaitEvent(side, labelled, 0)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_rename_kernel, dim3((n + 255) / 256), dim3(256), 0, side, n, n_seg, seg,
                       state, rec, rec2, probe);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_probe_kernel, dim3(n_seg), dim3(kCmThreads), 0, side, rec2, seg, ordC,
                       probe);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    return hipEventRecord(probed, side);
}

hipError_t launch_cm_segments(int4 *rec, int4 *rec2, int4 *state, int32_t *probe, int32_t n,
                              int32_t n_seg, const int64_t *seg, int32_t *permA, int32_t *ordC,
                              int32_t *perm, int32_t *label, int32_t *passes, hipStream_t s,
                              hipStream_t side, hipEvent_t labelled, hipEvent_t probed,
                              bool speculative)
{
    hipLaunchKernelGGL(cm_first_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, seg, perm,
                       state);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (!speculative) {
        if ((e = launch_cm_confirm(rec, rec2, state, probe, n, n_seg, seg, ordC, s, side,
                                   labelled, probed)) != hipSuccess)
            return e;
        if ((e = hipStreamWaitEvent(s, probed, 0)) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(cm_finish_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, seg, state,
                       probe, permA, perm, passes, (int32_t)speculative);
    if ((e = hipGetLastError()) != hipSuccess)
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
