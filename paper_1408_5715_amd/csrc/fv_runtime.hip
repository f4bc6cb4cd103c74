// Host runtime behind the C ABI of include/fvgpu.h: context, arena carving,
// host-side validation, transfers on the caller's stream and orchestration
// of the kernels.  The library allocates no device memory: every device
// buffer is a slice of the caller's arena.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fv_internal.h"
#include "fvgpu.h"

namespace {

thread_local std::string g_last_error;

fv_status fail(fv_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(FV_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

constexpr size_t kAlign = 256;
// Device code forms offsets such as 6 ld + i (normals) and 4 v + 3 (the
// label field of a renumbering record) in 32-bit integers, and the labelling
// packs a degree and a cell id into 32 bits: 8 ld < 2^31 keeps all of them
// exact (about 77 GB of arena at this size).
constexpr int64_t kMaxCells = (int64_t(1) << 28) - 4096;
static_assert(kMaxCells == FV_MAX_CELLS, "FV_MAX_CELLS");
constexpr int32_t kMaxSegments = 1 << 16;

size_t align_up(size_t x)
{
    return (x + kAlign - 1) / kAlign * kAlign;
}

int64_t leading_dim(int64_t n)
{
    return (n + 63) / 64 * 64;
}

// Byte sizes of the arena regions for n cells (leading dimension ld).
struct Layout {
    size_t U, nb, nb16, nfx, nrm, area, idx, scratch, seg, corr, small, total;
    explicit Layout(int64_t n)
    {
        const size_t ld = (size_t)leading_dim(n);
        U = align_up(ld * 32);
        nb = align_up(ld * 3 * 4);
        // 16-bit offsets, interleaved with dt/V on a mesh beyond the
        // Infinity Cache
        nb16 = align_up(ld * 16);
        nfx = align_up(ld * 16);
        nrm = align_up(ld * 6 * 8);
        area = align_up(ld * 8);
        idx = align_up(ld * 4);
        // >= a staged state (32 B) and the renumbering's scratch (records,
        // a second order, renamed records, the confirming sweep's order:
        // 40 B)
        scratch = align_up(ld * 40);
        // segment offsets (int64), per-segment dt (double), per-segment pass
        // counts (int32), per-segment first-sweep results (int4) and
        // second-sweep eccentricities (int32, padded to 8 bytes)
        seg = align_up((size_t)(kMaxSegments + 1) * 8) + align_up((size_t)kMaxSegments * 8) +
              align_up((size_t)kMaxSegments * 4) + align_up((size_t)kMaxSegments * 16) +
              align_up((size_t)kMaxSegments * 8);
        corr = align_up(fvk::kCorrFragShorts * 2) + align_up(fvk::kCorrBias * 4) +
               align_up(fvk::kCorrAdjFragShorts * 2) +
               align_up((size_t)fvk::kCorrAdjMaxGrid * fvk::kCorrParams * 4);
        small = kAlign;
        total = 2 * U + 2 * nb + nb16 + nfx + 2 * nrm + 3 * area + 2 * idx + scratch + seg + corr +
                small;
    }
};

}  // namespace

struct fv_ctx {
    int32_t n = 0;
    int32_t ld = 0;
    double gamma = 1.4;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;

    double4 *U[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t *nb_o = nullptr;  // uploaded mesh as uploaded: int32 [n][3], double [n][6]
    double *nrm_o = nullptr;
    double *area_o = nullptr;
    int32_t *nb_w = nullptr;  // working (renumbered) order
    short4 *nb16_w = nullptr; // ... as 16-bit offsets, valid when `narrow` (interleaved with
                              // dt / V when `interleaved`)
    int4 *nfx_w = nullptr;    // first two normals of the working order in fixed point, when `fixed`
    double *nrm_w = nullptr;
    double *inv_area_w = nullptr;
    double *coef = nullptr;    // dt / V_T per working cell, for coef_dt
    int32_t *perm = nullptr;   // perm[new] = uploaded id
    int32_t *label = nullptr;  // label[uploaded id] = new
    char *scratch = nullptr;
    char *small = nullptr;     // flags
    int64_t *seg_dev = nullptr;   // segment offsets (n_seg + 1)
    double *dt_dev = nullptr;     // per-segment dt of `coef`
    int32_t *passes_dev = nullptr;
    int4 *cm_state = nullptr;     // per-segment first-sweep results of the renumbering
    int32_t *cm_probe = nullptr;  // per-segment eccentricity of the second sweep

    int32_t n_seg = 1;
    std::vector<int64_t> seg_host;  // segment offsets; a segment is an independent mesh
    std::vector<double> coef_dt;    // dt per segment that `coef` holds (empty: stale)

    int block = 256;  // step launch: workgroup size
    int grid = 0;     // 0 = one workgroup per tile, else persistent workgroups
    bool use_graph = false;
    bool corr_on = false;           // learned flux correction active
    short *corr_frags = nullptr;    // packed MLP weights (device)
    float *corr_bias = nullptr;
    short *corr_afrags = nullptr;   // fragments of the adjoint kernel
    float *corr_partial = nullptr;  // per-workgroup parameter gradients
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    hipStream_t side = nullptr;        // second stream of the renumbering (default priority)
    hipEvent_t ev_labelled = nullptr;  // first labelling pass done (recorded on `stream`)
    hipEvent_t ev_probed = nullptr;    // confirming sweep done (recorded on `side`)
    bool probe_pending = false;        // a speculative renumbering's confirming sweep is unchecked
    hipEvent_t ev_sync = nullptr;      // polled by wait_stream
    int32_t *host_flag = nullptr;      // pinned host word for device flags
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    long long graph_key[6] = {-1, -1, -1, -1, -1, -1};

    bool mesh_ready = false;
    bool state_ready = false;
    bool closed = false;  // every cell: n_2 == -(n_0 + n_1) exactly
    bool fixed = false;   // every n_0, n_1 component is k 2^-32, |k| < 2^31 (and `closed`)
    bool narrow = false;  // every neighbour offset of the working order fits in 16 bits
    bool interleaved = false;  // nb16 interleaves the offsets with dt / V (fvk::narrow_interleaved)
    bool cm_passes = false;  // passes_dev holds the counts of a renumbering of this mesh
};

namespace {

fv_status check_ctx(fv_ctx *c)
{
    if (!c)
        return fail(FV_EINVAL, "null context");
    return FV_OK;
}

// Host-side mesh validation: indices, closure (every face has a partner
// face with the exactly negated normal), finite non-zero normals, areas > 0.
fv_status validate_mesh(int64_t n, const int32_t *nbr, const double *nrm, const double *area)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!(std::isfinite(area[i]) && area[i] > 0.0))
            return fail(FV_EMESH, "cell %lld: area %g is not finite and positive", (long long)i,
                        area[i]);
        for (int f = 0; f < 3; ++f) {
            const int64_t j = nbr[3 * i + f];
            if (j < 0 || j >= n)
                return fail(FV_EMESH, "cell %lld face %d: neighbour %lld out of range",
                            (long long)i, f, (long long)j);
            if (j == i)
                return fail(FV_EMESH, "cell %lld face %d: cell is its own neighbour",
                            (long long)i, f);
            const double nx = nrm[6 * i + 2 * f], ny = nrm[6 * i + 2 * f + 1];
            if (!(std::isfinite(nx) && std::isfinite(ny)) || (nx == 0.0 && ny == 0.0))
                return fail(FV_EMESH, "cell %lld face %d: normal not finite and non-zero",
                            (long long)i, f);
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int f = 0; f < 3; ++f) {
            const int64_t j = nbr[3 * i + f];
            const double nx = nrm[6 * i + 2 * f], ny = nrm[6 * i + 2 * f + 1];
            bool found = false;
            for (int g = 0; g < 3 && !found; ++g)
                found = nbr[3 * j + g] == i && nrm[6 * j + 2 * g] == -nx &&
                        nrm[6 * j + 2 * g + 1] == -ny;
            if (!found)
                return fail(FV_EMESH,
                            "cell %lld face %d: neighbour %lld has no face back with the negated "
                            "normal (mesh not closed or normals not antisymmetric)",
                            (long long)i, f, (long long)j);
        }
    }
    return FV_OK;
}

fv_status validate_state(int64_t n, const double *U, double gamma)
{
    for (int64_t i = 0; i < n; ++i) {
        const double r = U[4 * i], mx = U[4 * i + 1], my = U[4 * i + 2], E = U[4 * i + 3];
        const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
        if (!(std::isfinite(r) && std::isfinite(mx) && std::isfinite(my) && std::isfinite(E) &&
              r > 0.0 && std::isfinite(p) && p > 0.0))
            return fail(FV_ESTATE, "cell %lld: rho %g p %g not finite and positive", (long long)i,
                        r, p);
    }
    return FV_OK;
}

// Every component of every cell's first two normals is an integer multiple
// k of 2^-32 with |k| < 2^31, so it converts to a 32-bit fixed-point value
// and back exactly (-0.0 is kept apart).
bool normals_fixed(int64_t n, const double *nrm)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < 4; ++c) {
            const double k = nrm[6 * i + c] * 0x1p32;  // exact: a power of two
            if (!(k == std::trunc(k) && std::fabs(k) < 0x1p31))
                return false;
        }
    }
    return true;
}

// Every cell's third normal equals -(n_0 + n_1) in binary64 (true when the
// normals are exact coordinate differences, as on snapped meshes).
bool normals_closed(int64_t n, const double *nrm)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *q = nrm + 6 * i;
        if (!(q[4] == -(q[0] + q[2]) && q[5] == -(q[1] + q[3])))
            return false;
    }
    return true;
}

// Wait for everything queued on the context's stream by polling an event.
// The host then resumes within microseconds of the device, where a blocking
// wait that follows a long renumbering can add a wake-up delay of the order
// of 100 us, during which the device has nothing queued.
fv_status wait_stream(fv_ctx *c)
{
    if (!c->ev_sync)
        HIP_TRY(hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(c->ev_sync, c->stream));
    hipError_t e;
    while ((e = hipEventQuery(c->ev_sync)) == hipErrorNotReady) {
    }
    HIP_TRY(e);
    return FV_OK;
}

// Rebuild the working geometry for the current perm/label, and its 16-bit
// neighbour offsets.  Synchronises the stream.
fv_status regather_geometry(fv_ctx *c)
{
    HIP_TRY(fvk::launch_gather_geometry(c->n, c->ld, c->perm, c->label, c->nb_o, c->nrm_o,
                                        c->area_o, c->nb_w, c->nrm_w, c->inv_area_w, c->stream));
    int32_t *dflag = reinterpret_cast<int32_t *>(c->small + 192);
    HIP_TRY(fvk::launch_fill_i32(dflag, 0, 1, c->stream));
    HIP_TRY(fvk::launch_narrow_offsets(c->n, c->ld, c->nb_w, c->nb16_w, c->interleaved ? 2 : 1,
                                       dflag, c->stream));
    if (c->fixed) {
        HIP_TRY(fvk::launch_fixed_normals(c->n, c->ld, c->nrm_w, c->nfx_w, c->stream));
    }
    if (!c->host_flag)
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&c->host_flag), sizeof(int32_t),
                              hipHostMallocDefault));
    *c->host_flag = 1;
    HIP_TRY(hipMemcpyAsync(c->host_flag, dflag, sizeof(int32_t), hipMemcpyDeviceToHost,
                           c->stream));
    if (fv_status st = wait_stream(c))
        return st;
    c->narrow = *c->host_flag == 0;
    c->coef_dt.clear();
    return FV_OK;
}

// The renumbering's second stream and its two events, created on first use.
fv_status ensure_side(fv_ctx *c)
{
    if (!c->side)
        HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (!c->ev_labelled)
        HIP_TRY(hipEventCreateWithFlags(&c->ev_labelled, hipEventDisableTiming));
    if (!c->ev_probed)
        HIP_TRY(hipEventCreateWithFlags(&c->ev_probed, hipEventDisableTiming));
    return FV_OK;
}

// The renumbering's scratch memory (bytes per cell): records 16, a second
// label order 4, renamed records 16, the confirming sweep's order 4 (ld is a
// multiple of 64, so every part stays aligned).
struct CmScratch {
    int4 *rec;
    int32_t *permA;
    int4 *rec2;
    int32_t *ordC;
    explicit CmScratch(const fv_ctx *c)
    {
        const size_t ld = (size_t)c->ld;
        rec = reinterpret_cast<int4 *>(c->scratch);
        permA = reinterpret_cast<int32_t *>(rec + ld);
        rec2 = reinterpret_cast<int4 *>(permA + ld);
        ordC = reinterpret_cast<int32_t *>(rec2 + ld);
    }
};

// Cuthill-McKee labelling of every segment of the uploaded graph into
// c->perm / c->label, one workgroup per segment, all on the device (see
// launch_cm_segments for `speculative`; the caller then launches the
// confirming sweep with cm_confirm).
fv_status cm_order(fv_ctx *c, bool speculative)
{
    const CmScratch m(c);
    if (fv_status st = ensure_side(c))
        return st;
    HIP_TRY(fvk::launch_build_records(c->n, c->nb_o, m.rec, c->stream));
    HIP_TRY(fvk::launch_cm_segments(m.rec, m.rec2, c->cm_state, c->cm_probe, c->n, c->n_seg,
                                    c->seg_dev, m.permA, m.ordC, c->perm, c->label,
                                    c->passes_dev, c->stream, c->side, c->ev_labelled,
                                    c->ev_probed, speculative));
    return FV_OK;
}

// The confirming sweep of a speculative renumbering, on the second stream
// after everything queued so far.
fv_status cm_confirm(fv_ctx *c)
{
    const CmScratch m(c);
    HIP_TRY(fvk::launch_cm_confirm(m.rec, m.rec2, c->cm_state, c->cm_probe, c->n, c->n_seg,
                                   c->seg_dev, m.ordC, c->stream, c->side, c->ev_labelled,
                                   c->ev_probed));
    return FV_OK;
}

// Make c->coef hold dt[s] / V for every cell (no work if it already does).
fv_status ensure_coef(fv_ctx *c, const double *dt)
{
    bool same = (int32_t)c->coef_dt.size() == c->n_seg;
    for (int32_t k = 0; same && k < c->n_seg; ++k)
        same = c->coef_dt[k] == dt[k];
    if (same)
        return FV_OK;
    HIP_TRY(hipMemcpyAsync(c->dt_dev, dt, (size_t)c->n_seg * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(fvk::launch_coef(c->n, c->n_seg, c->seg_dev, c->dt_dev, c->inv_area_w, c->coef,
                             c->interleaved ? c->nb16_w : nullptr, c->stream));
    // the host array of dt values is read by the copy; keep it alive until then
    if (fv_status st = wait_stream(c))
        return st;
    c->coef_dt.assign(dt, dt + c->n_seg);
    return FV_OK;
}

void drop_graph(fv_ctx *c)
{
    if (c->graph_exec)
        (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph)
        (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    for (auto &k : c->graph_key)
        k = -1;
}

// One step from buffer `from` to the other: the plain kernel, or the one
// with the learned flux correction.
hipError_t launch_one(fv_ctx *c, int from, hipStream_t st)
{
    if (c->corr_on)
        return fvk::launch_step_learned(c->n, c->ld, c->U[from], c->U[from ^ 1], c->nb_w,
                                        c->nb16_w, c->interleaved ? 2 : 1, c->nrm_w, c->coef,
                                        c->inv_area_w, c->corr_frags, c->corr_bias, c->gamma,
                                        c->narrow, c->closed, c->grid, st);
    return fvk::launch_step(c->n, c->ld, c->U[from], c->U[from ^ 1], c->nb_w, c->nb16_w,
                            c->nrm_w, c->nfx_w, c->coef, c->gamma, c->narrow, c->closed, c->fixed,
                            c->block, c->grid, st);
}

// n_steps launches of the step, ping-ponging the state buffers; through a
// captured graph (one launch of the whole sequence) when enabled.
fv_status run_steps(fv_ctx *c, int32_t n_steps)
{
    if (n_steps == 0)
        return FV_OK;
    if (!c->use_graph) {
        for (int32_t s = 0; s < n_steps; ++s) {
            HIP_TRY(launch_one(c, c->cur, c->stream));
            c->cur ^= 1;
        }
        return FV_OK;
    }
    const long long key[6] = {n_steps, c->cur, c->block, c->grid,
                              c->narrow + 2 * c->closed + 4 * c->corr_on + 8 * c->fixed, 0};
    bool hit = c->graph_exec != nullptr;
    for (int k = 0; hit && k < 6; ++k)
        hit = key[k] == c->graph_key[k];
    if (!hit) {
        drop_graph(c);
        if (!c->cap_stream)
            HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        int cur = c->cur;
        hipError_t err = hipSuccess;
        for (int32_t s = 0; s < n_steps && err == hipSuccess; ++s) {
            err = launch_one(c, cur, c->cap_stream);
            cur ^= 1;
        }
        hipGraph_t g = nullptr;
        const hipError_t end = hipStreamEndCapture(c->cap_stream, &g);
        if (err != hipSuccess)
            return fail(FV_EHIP, "step launch during capture failed: %s", hipGetErrorString(err));
        HIP_TRY(end);
        c->graph = g;
        HIP_TRY(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
        for (int k = 0; k < 6; ++k)
            c->graph_key[k] = key[k];
    }
    HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
    c->cur ^= (n_steps & 1);
    return FV_OK;
}

// A renumbering of the mesh into c->perm / c->label and the working
// geometry; the state, if any, follows into the new order in one gather
// through the old and the new order, into the spare buffer, which becomes
// the current one.  Speculative (Cuthill-McKee only): the labels assume that no
// pseudo-peripheral search moves beyond its first candidate, and the
// confirming sweep is left running on the second stream (see settle).
fv_status renumber_now(fv_ctx *c, int32_t method, bool speculative)
{
    // the old inverse order, for the state, in the coef array (which the new
    // geometry invalidates anyway)
    int32_t *old_label = reinterpret_cast<int32_t *>(c->coef);
    if (c->state_ready) {
        c->coef_dt.clear();
        HIP_TRY(hipMemcpyAsync(old_label, c->label, (size_t)c->n * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, c->stream));
    }
    c->cm_passes = false;
    if (method == FV_ORDER_IDENTITY) {
        HIP_TRY(fvk::launch_iota(c->perm, c->n, c->stream));
        HIP_TRY(fvk::launch_iota(c->label, c->n, c->stream));
    } else {
        if (fv_status st = cm_order(c, speculative))
            return st;
        c->cm_passes = true;
    }
    if (fv_status st = regather_geometry(c))
        return st;
    if (c->state_ready) {
        // new cell l is uploaded cell perm[l], which sat at old_label[perm[l]]
        HIP_TRY(fvk::launch_gather_state2(c->n, c->perm, old_label, c->U[c->cur],
                                          c->U[c->cur ^ 1], c->stream));
        c->cur ^= 1;
    }
    if (speculative && method == FV_ORDER_CM) {
        // after the gathers, so that its scattered loads do not compete with
        // theirs on the critical path
        if (fv_status st = cm_confirm(c))
            return st;
        c->probe_pending = true;
    }
    return FV_OK;
}

// Wait for the confirming sweep of a speculative renumbering (its scratch
// memory is free afterwards).  With `check`, compare its eccentricities with
// the first sweeps' and, if some search would have moved, renumber again
// without speculation: the labels then are exactly those of the sequential
// search.  The state keeps its values (a step gives the same bits in any
// cell order), so only the working order changes.
fv_status settle(fv_ctx *c, bool check)
{
    if (!c->probe_pending)
        return FV_OK;
    c->probe_pending = false;
    HIP_TRY(hipEventSynchronize(c->ev_probed));
    if (!check)
        return FV_OK;
    std::vector<int4> st((size_t)c->n_seg);
    std::vector<int32_t> pr((size_t)c->n_seg);
    HIP_TRY(hipMemcpyAsync(st.data(), c->cm_state, st.size() * sizeof(int4),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(pr.data(), c->cm_probe, pr.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    bool moved = false;
    for (int32_t k = 0; k < c->n_seg; ++k)
        moved = moved || (st[k].x > 0 && pr[k] > st[k].y);
    if (!moved)
        return FV_OK;
    drop_graph(c);
    if (fv_status s2 = renumber_now(c, FV_ORDER_CM, false))
        return s2;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FV_OK;
}

}  // namespace

extern "C" {

size_t fv_arena_bytes(int64_t n_cells)
{
    if (n_cells <= 0 || n_cells > kMaxCells)
        return 0;
    return Layout(n_cells).total;
}

fv_status fv_create(int64_t n_cells, double gamma, void *d_arena, size_t arena_bytes,
                    void *hip_stream, fv_ctx **out)
{
    g_last_error.clear();
    if (!out)
        return fail(FV_EINVAL, "out is null");
    *out = nullptr;
    if (n_cells <= 0 || n_cells > kMaxCells)
        return fail(FV_EINVAL, "n_cells %lld outside [1, %lld]", (long long)n_cells,
                    (long long)kMaxCells);
    if (!(std::isfinite(gamma) && gamma > 1.0))
        return fail(FV_EINVAL, "gamma %g must be finite and > 1", gamma);
    if (!d_arena)
        return fail(FV_EINVAL, "arena is null");
    if (reinterpret_cast<uintptr_t>(d_arena) % kAlign != 0)
        return fail(FV_EINVAL, "arena must be %zu-byte aligned", kAlign);
    const Layout lay(n_cells);
    if (arena_bytes < lay.total)
        return fail(FV_EINVAL, "arena holds %zu bytes, %zu needed", arena_bytes, lay.total);

    fv_ctx *c = new (std::nothrow) fv_ctx;
    if (!c)
        return fail(FV_ENOMEM, "context allocation failed");
    c->n = (int32_t)n_cells;
    c->ld = (int32_t)leading_dim(n_cells);
    c->gamma = gamma;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->arena = reinterpret_cast<char *>(d_arena);
    c->arena_bytes = arena_bytes;
    char *p = c->arena;
    c->U[0] = reinterpret_cast<double4 *>(p);
    p += lay.U;
    c->U[1] = reinterpret_cast<double4 *>(p);
    p += lay.U;
    c->nb_o = reinterpret_cast<int32_t *>(p);
    p += lay.nb;
    c->nb_w = reinterpret_cast<int32_t *>(p);
    p += lay.nb;
    c->nb16_w = reinterpret_cast<short4 *>(p);
    p += lay.nb16;
    c->nfx_w = reinterpret_cast<int4 *>(p);
    p += lay.nfx;
    c->nrm_o = reinterpret_cast<double *>(p);
    p += lay.nrm;
    c->nrm_w = reinterpret_cast<double *>(p);
    p += lay.nrm;
    c->area_o = reinterpret_cast<double *>(p);
    p += lay.area;
    c->inv_area_w = reinterpret_cast<double *>(p);
    p += lay.area;
    c->coef = reinterpret_cast<double *>(p);
    p += lay.area;
    c->perm = reinterpret_cast<int32_t *>(p);
    p += lay.idx;
    c->label = reinterpret_cast<int32_t *>(p);
    p += lay.idx;
    c->scratch = p;
    p += lay.scratch;
    c->seg_dev = reinterpret_cast<int64_t *>(p);
    p += align_up((size_t)(kMaxSegments + 1) * 8);
    c->dt_dev = reinterpret_cast<double *>(p);
    p += align_up((size_t)kMaxSegments * 8);
    c->passes_dev = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)kMaxSegments * 4);
    c->cm_state = reinterpret_cast<int4 *>(p);
    p += align_up((size_t)kMaxSegments * 16);
    c->cm_probe = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)kMaxSegments * 8);
    c->corr_frags = reinterpret_cast<short *>(p);
    p += align_up(fvk::kCorrFragShorts * 2);
    c->corr_bias = reinterpret_cast<float *>(p);
    p += align_up(fvk::kCorrBias * 4);
    c->corr_afrags = reinterpret_cast<short *>(p);
    p += align_up(fvk::kCorrAdjFragShorts * 2);
    c->corr_partial = reinterpret_cast<float *>(p);
    p += align_up((size_t)fvk::kCorrAdjMaxGrid * fvk::kCorrParams * 4);
    c->small = p;
    *out = c;
    return FV_OK;
}

}  // extern "C"

namespace {

// Segments: n_seg + 1 offsets from 0 to n, strictly increasing, and no face
// crossing from one segment to another.
fv_status validate_segments(int64_t n, int32_t n_seg, const int64_t *seg, const int32_t *nbr)
{
    if (n_seg < 1 || n_seg > kMaxSegments)
        return fail(FV_EINVAL, "n_seg %d outside [1, %d]", n_seg, kMaxSegments);
    if (seg[0] != 0 || seg[n_seg] != n)
        return fail(FV_EINVAL, "segment offsets must run from 0 to n_cells");
    for (int32_t k = 0; k < n_seg; ++k) {
        if (seg[k + 1] <= seg[k])
            return fail(FV_EINVAL, "segment %d is empty or offsets decrease", k);
        for (int64_t i = seg[k]; i < seg[k + 1]; ++i)
            for (int f = 0; f < 3; ++f) {
                const int64_t j = nbr[3 * i + f];
                if (j < seg[k] || j >= seg[k + 1])
                    return fail(FV_EMESH, "cell %lld face %d: neighbour %lld lies in another segment",
                                (long long)i, f, (long long)j);
            }
    }
    return FV_OK;
}

fv_status upload(fv_ctx *c, int32_t n_seg, const int64_t *seg, const int32_t *nbr,
                 const double *nrm, const double *area)
{
    if (fv_status st = validate_mesh(c->n, nbr, nrm, area))
        return st;
    if (fv_status st = validate_segments(c->n, n_seg, seg, nbr))
        return st;
    // perm and the renumbering's scratch memory change below: wait for a
    // confirming sweep that may still read them
    if (fv_status st = settle(c, false))
        return st;
    const size_t n = (size_t)c->n;
    c->mesh_ready = false;
    c->state_ready = false;
    c->cm_passes = false;
    drop_graph(c);
    c->closed = normals_closed(c->n, nrm);
    c->fixed = c->closed && normals_fixed(c->n, nrm);
    c->interleaved = fvk::narrow_interleaved(c->n, c->closed, c->fixed);
    c->n_seg = n_seg;
    c->seg_host.assign(seg, seg + n_seg + 1);
    HIP_TRY(hipMemcpyAsync(c->seg_dev, c->seg_host.data(), (n_seg + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->nb_o, nbr, n * 3 * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->nrm_o, nrm, n * 6 * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->area_o, area, n * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(fvk::launch_iota(c->perm, c->n, c->stream));
    HIP_TRY(fvk::launch_iota(c->label, c->n, c->stream));
    if (fv_status st = regather_geometry(c))
        return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->mesh_ready = true;
    return FV_OK;
}

}  // namespace

extern "C" {

fv_status fv_upload_mesh(fv_ctx *c, const int32_t *nbr, const double *nrm, const double *area)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!nbr || !nrm || !area)
        return fail(FV_EINVAL, "null mesh array");
    const int64_t seg[2] = {0, c->n};
    return upload(c, 1, seg, nbr, nrm, area);
}

fv_status fv_upload_batch(fv_ctx *c, int32_t n_meshes, const int64_t *mesh_begin,
                          const int32_t *nbr, const double *nrm, const double *area)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!mesh_begin || !nbr || !nrm || !area)
        return fail(FV_EINVAL, "null batch array");
    return upload(c, n_meshes, mesh_begin, nbr, nrm, area);
}

fv_status fv_upload_state(fv_ctx *c, const double *U)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!U)
        return fail(FV_EINVAL, "null state");
    if (!c->mesh_ready)
        return fail(FV_ESTATE, "upload the mesh before the state");
    if (fv_status st = validate_state(c->n, U, c->gamma))
        return st;
    if (fv_status st = settle(c, true))
        return st;
    HIP_TRY(hipMemcpyAsync(c->scratch, U, (size_t)c->n * 4 * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(fvk::launch_gather_state(c->n, c->perm, reinterpret_cast<const double4 *>(c->scratch),
                                     c->U[c->cur], c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->state_ready = true;
    return FV_OK;
}

fv_status fv_upload_state_device(fv_ctx *c, const double *d_U)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!d_U)
        return fail(FV_EINVAL, "null state");
    if (reinterpret_cast<uintptr_t>(d_U) % 32 != 0)
        return fail(FV_EINVAL, "device state must be 32-byte aligned");
    if (!c->mesh_ready)
        return fail(FV_ESTATE, "upload the mesh before the state");
    HIP_TRY(fvk::launch_gather_state(c->n, c->perm, reinterpret_cast<const double4 *>(d_U),
                                     c->U[c->cur], c->stream));
    c->state_ready = true;
    return FV_OK;
}

fv_status fv_renumber(fv_ctx *c, int32_t method, int32_t *perm_out)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (method != FV_ORDER_IDENTITY && method != FV_ORDER_CM)
        return fail(FV_EINVAL, "unknown renumbering method %d", method);
    if (!c->mesh_ready)
        return fail(FV_ESTATE, "upload the mesh before renumbering");
    // a pending confirming sweep is only waited for: this renumbering replaces it
    if (fv_status st = settle(c, false))
        return st;
    // without perm_out nothing waits for the confirming sweep (speculative)
    if (fv_status st = renumber_now(c, method, method == FV_ORDER_CM && !perm_out))
        return st;
    if (perm_out)
        HIP_TRY(hipMemcpyAsync(perm_out, c->perm, (size_t)c->n * sizeof(int32_t),
                               hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FV_OK;
}

fv_status fv_step(fv_ctx *c, int32_t n_steps, double dt)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (n_steps < 0)
        return fail(FV_EINVAL, "n_steps %d < 0", n_steps);
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(FV_EINVAL, "dt %g must be finite and > 0", dt);
    if (!c->mesh_ready || !c->state_ready)
        return fail(FV_ESTATE, "upload the mesh and the state before stepping");
    std::vector<double> dts((size_t)c->n_seg, dt);
    if (fv_status st = ensure_coef(c, dts.data()))
        return st;
    return run_steps(c, n_steps);
}

fv_status fv_step_batch(fv_ctx *c, int32_t n_steps, const double *dt)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (n_steps < 0)
        return fail(FV_EINVAL, "n_steps %d < 0", n_steps);
    if (!dt)
        return fail(FV_EINVAL, "null dt array");
    if (!c->mesh_ready || !c->state_ready)
        return fail(FV_ESTATE, "upload the mesh and the state before stepping");
    for (int32_t k = 0; k < c->n_seg; ++k)
        if (!(std::isfinite(dt[k]) && dt[k] > 0.0))
            return fail(FV_EINVAL, "dt[%d] = %g must be finite and > 0", k, dt[k]);
    if (fv_status st = ensure_coef(c, dt))
        return st;
    return run_steps(c, n_steps);
}

fv_status fv_step_adjoint(fv_ctx *c, const double *d_U, double *d_lambda, double dt)
{
    return fv_step_adjoint_grad(c, d_U, d_lambda, dt, nullptr);
}

fv_status fv_step_adjoint_grad(fv_ctx *c, const double *d_U, double *d_lambda, double dt,
                               double *d_grad)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!d_U || !d_lambda)
        return fail(FV_EINVAL, "null device array");
    if (reinterpret_cast<uintptr_t>(d_U) % 32 != 0 || reinterpret_cast<uintptr_t>(d_lambda) % 32 != 0)
        return fail(FV_EINVAL, "device arrays must be 32-byte aligned");
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(FV_EINVAL, "dt %g must be finite and > 0", dt);
    if (!c->mesh_ready)
        return fail(FV_ESTATE, "upload the mesh first");
    if (d_grad && reinterpret_cast<uintptr_t>(d_grad) % 8 != 0)
        return fail(FV_EINVAL, "gradient array must be 8-byte aligned");
    if (d_grad && !c->corr_on)
        return fail(FV_ESTATE, "no correction is set: there is no parameter gradient");
    if (fv_status st = settle(c, true))
        return st;
    // The adjoint runs on the working (renumbered) geometry, like the step:
    // U and lambda are gathered into the working order (the spare state
    // buffer and the scratch memory), and each cell's result is written back
    // to its place in the uploaded numbering.
    double4 *Uw = c->U[c->cur ^ 1];
    double4 *lw = reinterpret_cast<double4 *>(c->scratch);
    HIP_TRY(fvk::launch_gather_state(c->n, c->perm, reinterpret_cast<const double4 *>(d_U), Uw,
                                     c->stream));
    HIP_TRY(fvk::launch_gather_state(c->n, c->perm, reinterpret_cast<const double4 *>(d_lambda),
                                     lw, c->stream));
    double4 *out = reinterpret_cast<double4 *>(d_lambda);
    if (c->corr_on)
        HIP_TRY(fvk::launch_adjoint_learned(c->n, c->ld, Uw, lw, out, c->perm, c->nb_w, c->nrm_w,
                                            c->inv_area_w, dt, c->gamma, c->corr_afrags,
                                            c->corr_bias, c->corr_partial, d_grad, c->stream));
    else
        HIP_TRY(fvk::launch_adjoint(c->n, c->ld, Uw, lw, out, c->perm, c->nb_w, c->nrm_w,
                                    c->inv_area_w, dt, c->gamma, c->stream));
    return FV_OK;
}

fv_status fv_set_correction(fv_ctx *c, const float *params, int32_t count)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!params) {
        c->corr_on = false;
        return FV_OK;
    }
    if (count != fvk::kCorrParams)
        return fail(FV_EINVAL, "expected %d parameters, got %d", fvk::kCorrParams, count);
    for (int32_t k = 0; k < count; ++k)
        if (!std::isfinite(params[k]))
            return fail(FV_EINVAL, "parameter %d is not finite", k);
    std::vector<short> frags(fvk::kCorrFragShorts), afrags(fvk::kCorrAdjFragShorts);
    std::vector<float> bias(fvk::kCorrBias);
    fvk::pack_correction(params, frags.data(), bias.data());
    fvk::pack_correction_adjoint(params, afrags.data());
    HIP_TRY(hipMemcpyAsync(c->corr_frags, frags.data(), frags.size() * sizeof(short),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->corr_afrags, afrags.data(), afrags.size() * sizeof(short),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->corr_bias, bias.data(), bias.size() * sizeof(float),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->corr_on = true;
    return FV_OK;
}

fv_status fv_set_launch(fv_ctx *c, int32_t block, int32_t grid, int32_t use_graph)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (block != 128 && block != 256 && block != 512)
        return fail(FV_EINVAL, "block %d must be 128, 256 or 512", block);
    if (grid < 0)
        return fail(FV_EINVAL, "grid %d < 0", grid);
    if (use_graph != 0 && use_graph != 1)
        return fail(FV_EINVAL, "use_graph must be 0 or 1");
    c->block = block;
    c->grid = grid;
    c->use_graph = use_graph == 1;
    return FV_OK;
}

fv_status fv_renumber_passes(fv_ctx *c, int32_t *passes)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!passes)
        return fail(FV_EINVAL, "null passes array");
    if (!c->mesh_ready)
        return fail(FV_ESTATE, "upload the mesh first");
    if (fv_status st = settle(c, true))
        return st;
    if (!c->cm_passes)
        return fail(FV_ESTATE, "no Cuthill-McKee renumbering of this mesh yet");
    HIP_TRY(hipMemcpyAsync(passes, c->passes_dev, (size_t)c->n_seg * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FV_OK;
}

fv_status fv_working_order(fv_ctx *c, int32_t *perm_out)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!perm_out)
        return fail(FV_EINVAL, "null permutation array");
    if (!c->mesh_ready)
        return fail(FV_ESTATE, "upload the mesh first");
    if (fv_status st = settle(c, true))
        return st;
    HIP_TRY(hipMemcpyAsync(perm_out, c->perm, (size_t)c->n * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FV_OK;
}

fv_status fv_download_state(fv_ctx *c, double *U)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!U)
        return fail(FV_EINVAL, "null state");
    if (!c->state_ready)
        return fail(FV_ESTATE, "no state uploaded");
    if (fv_status st = settle(c, true))
        return st;
    double4 *stage = reinterpret_cast<double4 *>(c->scratch);
    HIP_TRY(fvk::launch_gather_state(c->n, c->label, c->U[c->cur], stage, c->stream));
    HIP_TRY(hipMemcpyAsync(U, stage, (size_t)c->n * 4 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FV_OK;
}

fv_status fv_download_state_device(fv_ctx *c, double *d_U)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!d_U)
        return fail(FV_EINVAL, "null state");
    if (reinterpret_cast<uintptr_t>(d_U) % 32 != 0)
        return fail(FV_EINVAL, "device state must be 32-byte aligned");
    if (!c->state_ready)
        return fail(FV_ESTATE, "no state uploaded");
    HIP_TRY(fvk::launch_gather_state(c->n, c->label, c->U[c->cur], reinterpret_cast<double4 *>(d_U),
                                     c->stream));
    return FV_OK;
}

int64_t fv_bytes_per_update(const fv_ctx *c)
{
    if (!c || !c->mesh_ready)
        return 0;
    return 32 + 32 + 8 + (c->narrow ? 8 : 12) + (c->fixed ? 16 : (c->closed ? 32 : 48));
}

fv_status fv_check_state(fv_ctx *c)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!c->state_ready)
        return fail(FV_ESTATE, "no state uploaded");
    int32_t *dflag = reinterpret_cast<int32_t *>(c->small + 128);
    HIP_TRY(fvk::launch_fill_i32(dflag, 0, 1, c->stream));
    HIP_TRY(fvk::launch_check_state(c->n, c->U[c->cur], c->gamma, dflag, c->stream));
    int32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, dflag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (flag)
        return fail(FV_ESTATE, "state has a cell with non-finite or non-positive rho or p");
    return FV_OK;
}

fv_status fv_restrict(const double *d_src, int64_t n_src, const int32_t *d_idx, const double *d_w,
                      int64_t n, int32_t k, double *d_out, void *hip_stream)
{
    g_last_error.clear();
    if (!d_src || !d_idx || !d_w || !d_out)
        return fail(FV_EINVAL, "null device array");
    if (n <= 0 || n_src <= 0 || k < 1 || k > 1024 || n > INT32_MAX || n_src > INT32_MAX)
        return fail(FV_EINVAL, "bad sizes n=%lld n_src=%lld k=%d", (long long)n,
                    (long long)n_src, k);
    if (reinterpret_cast<uintptr_t>(d_src) % 32 != 0 || reinterpret_cast<uintptr_t>(d_out) % 32 != 0 ||
        reinterpret_cast<uintptr_t>(d_idx) % 4 != 0 || reinterpret_cast<uintptr_t>(d_w) % 8 != 0)
        return fail(FV_EINVAL, "misaligned device array");
    HIP_TRY(fvk::launch_restrict(n, k, n_src, reinterpret_cast<const double4 *>(d_src), d_idx, d_w,
                                 reinterpret_cast<double4 *>(d_out),
                                 reinterpret_cast<hipStream_t>(hip_stream)));
    return FV_OK;
}

fv_status fv_destroy(fv_ctx *c)
{
    g_last_error.clear();
    if (!c)
        return fail(FV_EINVAL, "null context");
    (void)settle(c, false);
    drop_graph(c);
    if (c->cap_stream)
        (void)hipStreamDestroy(c->cap_stream);
    if (c->side)
        (void)hipStreamDestroy(c->side);
    if (c->ev_labelled)
        (void)hipEventDestroy(c->ev_labelled);
    if (c->ev_probed)
        (void)hipEventDestroy(c->ev_probed);
    if (c->ev_sync)
        (void)hipEventDestroy(c->ev_sync);
    if (c->host_flag)
        (void)hipHostFree(c->host_flag);
    delete c;
    return FV_OK;
}

const char *fv_last_error(void)
{
    return g_last_error.c_str();
}

}  // extern "C"

// ---- fv_step_static: the step with its scratch in a static device array ----
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, serving loops): the second state buffer of the ping-pong and the
// per-cell dt / V_T live in `scratch`, a file-scope device array of
// kStaticMaxCells cells that every device running the library holds until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address comes from hipGetSymbolAddress, once
// per device, and only that address is passed to kernels.

namespace {

constexpr int64_t kStaticMaxCells = FV_STATIC_MAX_CELLS;
constexpr int kStaticMaxDevices = 64;
// per cell: the other state buffer (32 B), then dt / V_T (8 B)
constexpr size_t kStaticStateBytes = (size_t)kStaticMaxCells * 32;
constexpr size_t kStaticBytes = kStaticStateBytes + (size_t)kStaticMaxCells * 8;

__device__ __align__(256) char scratch[kStaticBytes];

std::mutex g_static_mu;
void *g_static_ptr[kStaticMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
fv_status static_scratch(char **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices)
        return fail(FV_EHIP, "device %d outside the %d devices fv_step_static serves", dev,
                    kStaticMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr)
            return fail(FV_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_static_ptr[dev] = ptr;
    }
    *out = static_cast<char *>(g_static_ptr[dev]);
    return FV_OK;
}

// coef[i] = dt * (1 / area[i]): the same two roundings as the context path
// (1 / V_T formed at upload, times dt when dt changes).
__global__ void static_coef_kernel(int32_t n, const double *__restrict__ area, double dt,
                                   double *__restrict__ coef)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        coef[i] = dt * (1.0 / area[i]);
}

__global__ void static_copy_kernel(int32_t n, const double4 *__restrict__ src,
                                   double4 *__restrict__ dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

fv_status fv_step_static(int64_t n_cells, const int32_t *d_nbr, const double *d_nrm,
                         const double *d_area, double *d_U, int32_t n_steps, double dt,
                         double gamma, void *hip_stream)
{
    g_last_error.clear();
    if (n_cells <= 0 || n_cells > kStaticMaxCells)
        return fail(FV_EINVAL, "n_cells %lld outside [1, %lld] (the static scratch array's size)",
                    (long long)n_cells, (long long)kStaticMaxCells);
    if (!d_nbr || !d_nrm || !d_area || !d_U)
        return fail(FV_EINVAL, "null device array");
    if (reinterpret_cast<uintptr_t>(d_U) % 32 != 0 || reinterpret_cast<uintptr_t>(d_nrm) % 8 != 0 ||
        reinterpret_cast<uintptr_t>(d_area) % 8 != 0 || reinterpret_cast<uintptr_t>(d_nbr) % 4 != 0)
        return fail(FV_EINVAL, "misaligned device array (d_U needs 32 bytes)");
    if (n_steps < 0)
        return fail(FV_EINVAL, "n_steps %d < 0", n_steps);
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(FV_EINVAL, "dt %g must be finite and > 0", dt);
    if (!(std::isfinite(gamma) && gamma > 1.0))
        return fail(FV_EINVAL, "gamma %g must be finite and > 1", gamma);
    if (n_steps == 0)
        return FV_OK;
    char *base = nullptr;
    if (fv_status st = static_scratch(&base))
        return st;
    const int32_t n = (int32_t)n_cells;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    double4 *other = reinterpret_cast<double4 *>(base);
    double *coef = reinterpret_cast<double *>(base + kStaticStateBytes);
    double4 *buf[2] = {reinterpret_cast<double4 *>(d_U), other};
    hipLaunchKernelGGL(static_coef_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, d_area, dt,
                       coef);
    HIP_TRY(hipGetLastError());
    int cur = 0;
    for (int32_t k = 0; k < n_steps; ++k) {
        HIP_TRY(fvk::launch_step(n, n, buf[cur], buf[cur ^ 1], d_nbr, nullptr, d_nrm, nullptr,
                                 coef, gamma, false, false, false, 256, 0, s));
        cur ^= 1;
    }
    if (cur == 1) {
        hipLaunchKernelGGL(static_copy_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, other,
                           buf[0]);
        HIP_TRY(hipGetLastError());
    }
    return FV_OK;
}

}  // extern "C"
