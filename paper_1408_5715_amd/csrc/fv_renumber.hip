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

// ---- breadth-first sweeps for the pseudo-peripheral search ---------------
//
// The George-Liu search needs only level structures (eccentricity and the
// last level), which do not depend on the order inside a level, so a sweep
// does not rank children by owner label.  A frontier cell fetches the records
// of its neighbours not known to be visited; the record's fourth field marks
// a visited cell (-1 while unvisited), so the same load that brings a cell's
// neighbour list also says whether it is new.  A new cell proposed by
// several frontier cells of one sweep is claimed by exactly one of them
// through a hash set in LDS (an LDS compare-and-swap per proposal).  One
// round of scattered memory traffic per level, and no global atomics (which
// serialise where neighbouring cells share a cache line).

constexpr int kBfsCap = 3584;         // frontier entries held in LDS per buffer
constexpr int kHashSlots = 8192;      // > 2 * kCmThreads * kPer: the set never fills
constexpr unsigned kHashEmpty = 0xffffffffu;
static_assert(kHashSlots > 2 * kCmThreads * kPer, "hash set must outgrow a sweep's new cells");

struct BfsLds {
    int4 frontier[2][kBfsCap];          // (cell, nb_0, nb_1, nb_2) in breadth-first order
    unsigned char known[2][kBfsCap];    // bit f: nb_f is the cell's discoverer
    unsigned set[kHashSlots];           // cells claimed in the current sweep
    int scan[2 * kCmWaves + 1];
    unsigned long long minv[kCmWaves];
};

// Insert c into the LDS hash set; true if this call inserted it (claims c).
// At most one sweep's new cells live in the set, fewer than kHashSlots, so an
// empty slot is always reached; the loop is bounded by the table size.
__device__ __forceinline__ bool claim(unsigned *set, int c)
{
    unsigned h = ((unsigned)c * 0x9E3779B1u) >> 19;  // 13 bits
    for (int probe = 0; probe < kHashSlots; ++probe) {
        const unsigned old = atomicCAS(set + h, kHashEmpty, (unsigned)c);
        if (old == kHashEmpty)
            return true;
        if (old == (unsigned)c)
            return false;
        h = (h + 1) & (kHashSlots - 1);
    }
    return false;
}

// One sweep of a breadth-first level [a, b): frontier positions
// [c0, c0 + span), P per thread.  New cells are appended from b + produced
// on: ord[b + p] receives the p-th new cell, whose record's fourth field is
// set to `mark` (its record is kept in LDS while p < kBfsCap).  Returns the
// number of new cells (block-uniform).  The hash set must be empty on entry
// and is empty again on return.  Called by all threads of the block.
template <int P>
__device__ __forceinline__ int bfs_sweep(int4 *__restrict__ graph, int32_t *__restrict__ ord,
                                         BfsLds &lds, int cur, int a, int b, int c0, int span,
                                         int produced, int mark)
{
    const int tid = threadIdx.x;
    const int first = tid * P;
    const bool wave_busy = (tid & ~63) * P < span;

    int v[P], w[P][3];
    unsigned won[P];  // bit f: this thread claimed w[k][f]
    i4v rw[P][3];
    int total = 0;
    if (wave_busy) {
        unsigned kn[P];
        bool ok[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = first + k;
            ok[k] = t < span;
            const int ft = c0 + t;
            const int slot = (ok[k] && ft < kBfsCap) ? ft : 0;
            i4v e = reinterpret_cast<const i4v *>(lds.frontier[cur])[slot];
            unsigned kb = lds.known[cur][slot];
            asm volatile("" : "+v"(e), "+v"(kb));
            kn[k] = kb;
            if (ok[k] && ft >= kBfsCap) {
                const int c = ord[a + ft];
                const int4 r = graph[c];
                e = i4v{c, r.x, r.y, r.z};
                kn[k] = 0;
            }
            v[k] = e[0];
            w[k][0] = e[1];
            w[k][1] = e[2];
            w[k][2] = e[3];
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
                cand[k][f] = ok[k] && !((kn[k] >> f) & 1u) && ww != v[k] &&
                             !(f >= 1 && w[k][0] == ww) && !(f == 2 && w[k][1] == ww);
                rw[k][f] = i4v{0, 0, 0, 0};
                if (cand[k][f])
                    rw[k][f] = gv[ww];
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            won[k] = 0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                i4v r = rw[k][f];
                asm volatile("" : "+v"(r));
                rw[k][f] = r;
                if (cand[k][f] && r[3] == -1 && claim(lds.set, w[k][f]))
                    won[k] |= 1u << f;
            }
            total += __builtin_popcount(won[k]);
        }
    }
    int sweep_total;
    int pos = produced + block_exclusive_scan(total, lds.scan, &sweep_total);
    // every claim of this sweep is in: empty the set for the next sweep
    // (the caller's barrier separates this from the next sweep's claims)
    for (int t = tid; t < kHashSlots; t += kCmThreads)
        lds.set[t] = kHashEmpty;
    if (wave_busy) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if ((won[k] >> f) & 1u) {
                    const int c = w[k][f];
                    const i4v r = rw[k][f];
                    reinterpret_cast<int32_t *>(graph)[4 * c + 3] = mark;
                    ord[b + pos] = c;
                    if (pos < kBfsCap) {
                        lds.frontier[cur ^ 1][pos] = make_int4(c, r[0], r[1], r[2]);
                        lds.known[cur ^ 1][pos] = (unsigned char)((r[0] == v[k]) |
                                                                  (r[1] == v[k]) << 1 |
                                                                  (r[2] == v[k]) << 2);
                    }
                    ++pos;
                }
            }
        }
    }
    return sweep_total;
}

struct BfsResult {
    int count;  // cells reached (the component of the root)
    int ecc;    // eccentricity of the root
    int pick;   // last-level cell of minimum (degree, original id): its original id
    int width;  // largest level
};

// Breadth-first level structure of the component of `root` in `graph`
// (records (nb_0, nb_1, nb_2, mark), mark -1 for every cell of the
// component on entry; reached cells are marked with their level).  ord[base
// + p] receives the p-th cell reached (levels in order); lev, when not null,
// receives lev[base + k] = the first position of level k.  orig, when not
// null, gives the original id of a cell (else the cell index is its id).
// Called by all threads of the block.
__device__ __forceinline__ BfsResult bfs_pass(int4 *__restrict__ graph, int32_t root, int32_t base,
                                              int32_t *__restrict__ ord, int32_t *__restrict__ lev,
                                              const int32_t *__restrict__ orig, BfsLds &lds)
{
    const int tid = threadIdx.x;
    for (int t = tid; t < kHashSlots; t += kCmThreads)
        lds.set[t] = kHashEmpty;
    if (tid == 0) {
        const int4 r = graph[root];
        reinterpret_cast<int32_t *>(graph)[4 * root + 3] = 0;
        ord[base] = root;
        lds.frontier[0][0] = make_int4(root, r.x, r.y, r.z);
        lds.known[0][0] = 0;
        if (lev)
            lev[base] = base;
    }
    __threadfence_block();
    __syncthreads();

    int a = base, b = base + 1;
    int cur = 0, ecc = 0, width = 1;
    for (;;) {
        const int F = b - a;
        int produced = 0;
        for (int c0 = 0; c0 < F; c0 += kCmThreads * kPer) {
            const int span = min(F - c0, kCmThreads * kPer);
            const int per = (span + kCmThreads - 1) / kCmThreads;
            int st;
            if (per == 1)
                st = bfs_sweep<1>(graph, ord, lds, cur, a, b, c0, span, produced, ecc + 1);
            else if (per == 2)
                st = bfs_sweep<2>(graph, ord, lds, cur, a, b, c0, span, produced, ecc + 1);
            else
                st = bfs_sweep<3>(graph, ord, lds, cur, a, b, c0, span, produced, ecc + 1);
            produced += st;
            __threadfence_block();
            __syncthreads();
        }
        if (produced == 0)
            break;
        ++ecc;
        a = b;
        b += produced;
        width = max(width, produced);
        if (lev && tid == 0)
            lev[base + ecc] = a;
        cur ^= 1;
    }

    unsigned long long best = ~0ull;
    for (int t = tid; t < b - a; t += kCmThreads) {
        int c;
        int4 r;
        if (t < kBfsCap) {
            r = lds.frontier[cur][t];
            c = r.x;
            r = make_int4(r.y, r.z, r.w, 0);
        } else {
            c = ord[a + t];
            r = graph[c];
        }
        const int d = degree_of(c, r.x, r.y, r.z);
        const unsigned id = orig ? (unsigned)orig[c] : (unsigned)c;
        const unsigned long long key = ((unsigned long long)d << 32) | id;
        best = key < best ? key : best;
    }
    best = block_min_u64(best, lds.minv);
    BfsResult res;
    res.count = b - base;
    res.ecc = ecc;
    res.pick = (int32_t)(best & 0xffffffffu);
    res.width = width;
    return res;
}

// ---- Cuthill-McKee labels from a known level structure -------------------
//
// With the levels of the root known, level k+1 is labelled from level k
// alone: a cell's parent is its neighbour of smallest label in level k, and
// the labels of level k+1 follow (parent label, degree, original id).  The
// cells of every level are contiguous in the renamed graph (positions of
// the breadth-first order), so each level's records are one coalesced read,
// issued a level ahead; parents, sibling ranks and the scan over parents
// stay in LDS, and the barriers wait for LDS only, so the next level's
// records stay in flight across them.

constexpr int kLabelCap = 4096;  // widest level the labelling keeps in LDS

struct LabelLds {
    int lab[2][kLabelCap];        // labels of the previous / current level, by position
    int cnt[2][kLabelCap];        // children per parent of the previous level
    int first[kLabelCap];         // label offset of each parent's children
    unsigned sib[3 * kLabelCap];  // (degree, original id) keys of each parent's children
    int scan[2 * kCmWaves + 1];
};

// Barrier that orders LDS accesses only: global loads stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// block_exclusive_scan with an LDS-only barrier.
__device__ __forceinline__ int block_exclusive_scan_lds(int x, int *sh, int *total)
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
    lds_barrier();
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

// Labels of the component held at positions [base, base + count) of the
// renamed graph g (neighbours as positions; orig[p] the original id of
// position p), whose breadth-first levels from the root at position base are
// [lev[base + k], lev[base + k + 1]) for k = 0..ecc (the last ending at
// base + count), every level at most kLabelCap wide: perm[label] = original
// id for labels [base, base + count).  Called by all threads of the block.
__device__ __forceinline__ void label_levels(const int4 *__restrict__ g,
                                             const int32_t *__restrict__ orig,
                                             const int32_t *__restrict__ lev, int32_t base,
                                             int32_t count, int32_t ecc,
                                             int32_t *__restrict__ perm, LabelLds &lds)
{
    constexpr int kSlots = kLabelCap / kCmThreads;
    const int tid = threadIdx.x;
    const int end = base + count;
    for (int t = tid; t < kLabelCap; t += kCmThreads) {
        lds.cnt[0][t] = 0;
        lds.cnt[1][t] = 0;
    }
    if (tid == 0) {
        lds.lab[0][0] = base;
        perm[base] = orig[base];
    }
    // records and original ids of level 1, positions [base + 1, hi)
    int lo_prev = base, lo = base + 1;
    int hi = ecc >= 2 ? lev[base + 2] : end;
    int4 r[kSlots];
    int id[kSlots];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int q = lo + tid + j * kCmThreads;
        r[j] = q < hi ? g[q] : make_int4(0, 0, 0, 0);
        id[j] = q < hi ? orig[q] : 0;
    }
    lds_barrier();
    for (int k = 0; k < ecc; ++k) {
        // the next level's records, in flight while this level is labelled
        const int hi2 = k + 3 <= ecc ? lev[base + k + 3] : end;
        int4 rn[kSlots];
        int idn[kSlots];
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const int q = hi + tid + j * kCmThreads;
            rn[j] = q < hi2 ? g[q] : make_int4(0, 0, 0, 0);
            idn[j] = q < hi2 ? orig[q] : 0;
        }
        const int fp = lo - lo_prev;
        const int *labp = lds.lab[k & 1];
        int *labn = lds.lab[(k + 1) & 1];
        int *cnt = lds.cnt[k & 1];
        int par[kSlots];
        unsigned key[kSlots];
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const int q = lo + tid + j * kCmThreads;
            par[j] = -1;
            if (q < hi) {
                int best = INT_MAX;
                const int nb3[3] = {r[j].x, r[j].y, r[j].z};
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int x = nb3[f];
                    if (x >= lo_prev && x < lo) {
                        const int l = labp[x - lo_prev];
                        best = l < best ? l : best;
                    }
                }
                par[j] = best - lo_prev;
                key[j] = (unsigned)degree_of(q, r[j].x, r[j].y, r[j].z) << 30 | (unsigned)id[j];
                const int slot = atomicAdd(&cnt[par[j]], 1);
                lds.sib[3 * par[j] + slot] = key[j];
            }
        }
        lds_barrier();
        // exclusive scan of the children counts over the parents in label order
        int c4[kSlots], sum = 0;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const int o = tid * kSlots + j;
            c4[j] = o < fp ? cnt[o] : 0;
            sum += c4[j];
        }
        int tot;
        int off = block_exclusive_scan_lds(sum, lds.scan, &tot);
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const int o = tid * kSlots + j;
            if (o < fp)
                lds.first[o] = off;
            off += c4[j];
        }
        // the other parity's counts were last read a level ago: clear them
        // for the next level
        int *cnt_next = lds.cnt[(k + 1) & 1];
        for (int t = tid; t < hi - lo; t += kCmThreads)
            cnt_next[t] = 0;
        lds_barrier();
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const int q = lo + tid + j * kCmThreads;
            if (q < hi) {
                const int pa = par[j];
                const int nc = cnt[pa];
                int rank = 0;
                for (int u = 0; u < nc; ++u)
                    rank += lds.sib[3 * pa + u] < key[j];
                const int l = lo + lds.first[pa] + rank;
                labn[q - lo] = l;
                perm[l] = id[j];
            }
        }
        lds_barrier();
        lo_prev = lo;
        lo = hi;
        hi = hi2;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            r[j] = rn[j];
            id[j] = idn[j];
        }
    }
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
//   cm_first_kernel      breadth-first sweep from the segment's lowest id on
//                        the uploaded graph: its order (ordA), level starts
//                        (levA), eccentricity and pick; reached cells are
//                        marked in their records;
//   cm_invert_kernel,    the component's graph renamed by that order (rec2:
//   cm_rename_kernel     neighbours as positions), in which every level is a
//                        contiguous range;
//   cm_probe_kernel      the sweep from the pick on rec2 (the search's
//                        second step), on a second stream, beside
//   cm_label_kernel      the labels from the first sweep's levels
//                        (label_levels), which are the result when the
//                        eccentricity does not grow (the root then stays
//                        the lowest id);
//   cm_finish_kernel     otherwise, and for every later component, the
//                        search continues with full labelling passes on the
//                        uploaded graph (cm_pass).  With assume_stays the
//                        finish does not wait for the probe: it takes the
//                        labels of cm_label_kernel and goes on with the later
//                        components; the caller checks the probe's
//                        eccentricities afterwards and relabels exactly if
//                        some search would have moved.
//
// cm_first_kernel: state[s] = (cells reached, eccentricity, pick, widest level).
__global__ __launch_bounds__(kCmThreads) void cm_first_kernel(int4 *__restrict__ rec,
                                                              const int64_t *__restrict__ seg,
                                                              int32_t *__restrict__ ordA,
                                                              int32_t *__restrict__ levA,
                                                              int4 *__restrict__ state)
{
    __shared__ BfsLds lds;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    if (s0 >= s1) {  // block-uniform; uploads reject empty segments
        if (threadIdx.x == 0)
            state[blockIdx.x] = make_int4(0, 0, s0, 0);
        return;
    }
    const BfsResult r = bfs_pass(rec, s0, s0, ordA, levA, nullptr, lds);
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

// inv[ordA[l]] = l for the positions l of each segment's first component;
// root[s] = the position of the segment's pick (the probe sweep's root, which
// the probe kernel reads from here rather than from inv, which the final
// inverse overwrites on the other stream).
__global__ void cm_invert_kernel(int32_t n, int32_t n_seg, const int64_t *__restrict__ seg,
                                 const int4 *__restrict__ state, const int32_t *__restrict__ ordA,
                                 int32_t *__restrict__ inv, int32_t *__restrict__ root)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n)
        return;
    const int sg = segment_of(l, n_seg, seg);
    if (l - (int)seg[sg] >= state[sg].x)
        return;
    const int c = ordA[l];
    inv[c] = l;
    if (c == state[sg].z)
        root[sg] = l;
}

// rec2[l] = (positions of the three neighbours of the cell at position l, -1)
// for the positions of each segment's first component.
__global__ void cm_rename_kernel(int32_t n, int32_t n_seg, const int64_t *__restrict__ seg,
                                 const int4 *__restrict__ state, const int4 *__restrict__ rec,
                                 const int32_t *__restrict__ ordA, const int32_t *__restrict__ inv,
                                 int4 *__restrict__ rec2)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n)
        return;
    const int sg = segment_of(l, n_seg, seg);
    if (l - (int)seg[sg] >= state[sg].x)
        return;
    const int4 r = rec[ordA[l]];
    rec2[l] = make_int4(inv[r.x], inv[r.y], inv[r.z], -1);
}

// The sweep from the first component's pick on rec2, one workgroup per
// segment: on entry probe[s] holds the pick's position (cm_invert_kernel), on
// exit the sweep's eccentricity.  It may run beside the label and finish
// kernels, so it writes only rec2's marks, its own order ordC and probe, and
// reads nothing they write (the pick it finds is not used).
__global__ __launch_bounds__(kCmThreads) void cm_probe_kernel(
    int4 *__restrict__ rec2, const int64_t *__restrict__ seg, int32_t *__restrict__ ordC,
    int32_t *__restrict__ probe)
{
    __shared__ BfsLds lds;
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
    const BfsResult r = bfs_pass(rec2, root, s0, ordC, nullptr, nullptr, lds);
    __syncthreads();  // every thread has read probe[] before it is overwritten
    if (threadIdx.x == 0)
        probe[blockIdx.x] = r.ecc;
}

// The labels of each segment's first component from the first sweep's levels
// into perm, when every level fits in LDS (the finish kernel discards them if
// the search moves).  Reads only the (x, y, z) fields of rec2, which the probe
// sweep may run beside it.
__global__ __launch_bounds__(kCmThreads) void cm_label_kernel(
    const int4 *__restrict__ rec2, const int64_t *__restrict__ seg,
    const int4 *__restrict__ state, const int32_t *__restrict__ ordA,
    const int32_t *__restrict__ levA, int32_t *__restrict__ perm)
{
    __shared__ LabelLds lds;
    const int s0 = (int)seg[blockIdx.x], s1 = (int)seg[blockIdx.x + 1];
    if (s0 >= s1)
        return;
    const int4 st = state[blockIdx.x];
    if (st.w <= kLabelCap)
        label_levels(rec2, ordA, levA, s0, st.x, st.y, perm, lds);
}

// The rest of the search for every segment, after cm_probe_kernel, as one
// loop with one full labelling pass (cm_pass, on the uploaded graph) per
// iteration: kRoot (the root of the next component: its lowest cell not yet
// labelled), kSearch (clear the component's labels, relabel it from the pick
// of the best pass so far).  Every loop ends on a block-uniform condition:
// each component is labelled in full before the next starts, and the search
// moves only while the eccentricity, bounded by the segment size, strictly
// grows.  Records of cells the first sweep reached carry its marks (not -1),
// so they count as labelled when later roots are sought.
__global__ __launch_bounds__(kCmThreads) void cm_finish_kernel(
    int4 *__restrict__ rec, const int64_t *__restrict__ seg, const int4 *__restrict__ state,
    const int32_t *__restrict__ probe, int32_t *__restrict__ permA, int32_t *__restrict__ permB,
    int32_t *__restrict__ perm, int32_t *__restrict__ passes, int32_t assume_stays)
{
    enum { kRoot, kSearch };
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
    int npass = s0 < s1 ? 2 : 0;  // the two sweeps of the fast route
    int next = s0;
    int scan_from = s0;
    int mode = kRoot;
    if (s0 < s1) {
        if (!assume_stays && probe[blockIdx.x] > rr.ecc) {
            mode = kSearch;  // relabel exactly from the same pick
        } else {
            if (st.w > kLabelCap) {
                // levels too wide for the LDS labelling: a full pass from the
                // same root (the segment's lowest id) on cleared labels
                for (int v = s0 + tid; v < s1; v += kCmThreads)
                    rlabel[4 * v + 3] = -1;
                __threadfence_block();
                __syncthreads();
                (void)cm_pass(rec, s0, s0, perm, lds);
            }
            next += rr.count;
        }
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
        const PassResult r = cm_pass(rec, root, next, out, lds);
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

hipError_t launch_cm_segments(int4 *rec, int4 *rec2, int4 *state, int32_t *probe, int32_t n,
                              int32_t n_seg, const int64_t *seg, int32_t *permA, int32_t *permB,
                              int32_t *ordC, int32_t *levA, int32_t *perm, int32_t *label,
                              int32_t *passes, hipStream_t s, hipStream_t side,
                              hipEvent_t renamed, hipEvent_t probed, bool speculative)
{
    hipLaunchKernelGGL(cm_first_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, seg, permA,
                       levA, state);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // label serves as the inverse of the first order until invert_kernel
    // writes the final one
    hipLaunchKernelGGL(cm_invert_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, n_seg, seg,
                       state, permA, label, probe);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_rename_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, n_seg, seg,
                       state, rec, permA, label, rec2);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // the probe sweep on the second stream, the labels on this one
    if ((e = hipEventRecord(renamed, s)) != hipSuccess)
        return e;
    if ((e = hipStreamWaitEvent(side, renamed, 0)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_probe_kernel, dim3(n_seg), dim3(kCmThreads), 0, side, rec2, seg, ordC,
                       probe);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = hipEventRecord(probed, side)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_label_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec2, seg, state,
                       permA, levA, perm);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (!speculative && (e = hipStreamWaitEvent(s, probed, 0)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(cm_finish_kernel, dim3(n_seg), dim3(kCmThreads), 0, s, rec, seg, state,
                       probe, permA, permB, perm, passes, (int32_t)speculative);
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
