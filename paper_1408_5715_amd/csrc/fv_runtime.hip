// Host runtime behind the C ABI of include/fvgpu.h: context, arena carving,
// host-side validation, transfers on the caller's stream and orchestration
// of the kernels.  The library allocates no device memory: every device
// buffer is a slice of the caller's arena.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
constexpr int64_t kMaxCells = (int64_t(1) << 31) - 4096;

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
    size_t U, nb, nb16, nrm, area, idx, scratch, small, total;
    explicit Layout(int64_t n)
    {
        const size_t ld = (size_t)leading_dim(n);
        U = align_up(ld * 32);
        nb = align_up(ld * 3 * 4);
        nb16 = align_up(ld * 8);
        nrm = align_up(ld * 6 * 8);
        area = align_up(ld * 8);
        idx = align_up(ld * 4);
        scratch = align_up(ld * 48);  // >= AoS normals (48 B), state (32 B), 4 CM arrays (16 B)
        small = kAlign;
        total = 2 * U + 2 * nb + nb16 + 2 * nrm + 2 * area + 2 * idx + scratch + small;
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
    int32_t *nb_o = nullptr;  // uploaded mesh, structure of arrays
    double *nrm_o = nullptr;
    double *area_o = nullptr;
    int32_t *nb_w = nullptr;  // working (renumbered) order
    short4 *nb16_w = nullptr; // ... as 16-bit offsets, valid when `narrow`
    double *nrm_w = nullptr;
    double *inv_area_w = nullptr;
    int32_t *perm = nullptr;   // perm[new] = uploaded id
    int32_t *label = nullptr;  // label[uploaded id] = new
    char *scratch = nullptr;
    char *small = nullptr;     // CmResult and flags

    bool mesh_ready = false;
    bool state_ready = false;
    bool closed = false;  // every cell: n_2 == -(n_0 + n_1) exactly
    bool narrow = false;  // every neighbour offset of the working order fits in 16 bits
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

// Rebuild the working geometry for the current perm/label, and its 16-bit
// neighbour offsets.  Synchronises the stream.
fv_status regather_geometry(fv_ctx *c)
{
    HIP_TRY(fvk::launch_gather_geometry(c->n, c->ld, c->perm, c->label, c->nb_o, c->nrm_o,
                                        c->area_o, c->nb_w, c->nrm_w, c->inv_area_w, c->stream));
    int32_t *dflag = reinterpret_cast<int32_t *>(c->small + 192);
    HIP_TRY(fvk::launch_fill_i32(dflag, 0, 1, c->stream));
    HIP_TRY(fvk::launch_narrow_offsets(c->n, c->ld, c->nb_w, c->nb16_w, dflag, c->stream));
    int32_t too_far = 1;
    HIP_TRY(hipMemcpyAsync(&too_far, dflag, sizeof(too_far), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->narrow = too_far == 0;
    return FV_OK;
}

// Cuthill-McKee labelling of the uploaded graph into c->perm / c->label.
// Scratch use (bytes per cell): records 16, two candidate orders 4 + 4.
fv_status cm_order(fv_ctx *c)
{
    const int32_t n = c->n;
    const size_t ld = (size_t)c->ld;
    int4 *rec = reinterpret_cast<int4 *>(c->scratch);
    int32_t *permA = reinterpret_cast<int32_t *>(rec + ld);  // best order so far
    int32_t *permB = permA + ld;                             // trial order
    fvk::CmResult *dres = reinterpret_cast<fvk::CmResult *>(c->small);
    int32_t *dfind = reinterpret_cast<int32_t *>(c->small + 64);

    // One level structure (and its labelling) from `root`.
    auto pass = [&](int32_t root, int32_t base, int32_t *perm, fvk::CmResult *out) -> fv_status {
        HIP_TRY(fvk::launch_build_records(n, c->ld, c->nb_o, rec, c->stream));
        HIP_TRY(fvk::launch_cm_component(rec, root, base, perm, dres, c->stream));
        HIP_TRY(hipMemcpyAsync(out, dres, sizeof(*out), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return FV_OK;
    };

    HIP_TRY(fvk::launch_fill_i32(c->label, -1, n, c->stream));
    int32_t next = 0;
    int32_t scan_from = 0;
    while (next < n) {
        int32_t s = 0;
        if (next > 0) {
            HIP_TRY(fvk::launch_find_unlabelled(n, c->label, scan_from, dfind, c->stream));
            HIP_TRY(hipMemcpyAsync(&s, dfind, sizeof(s), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            if (s >= n)
                return fail(FV_EHIP, "renumbering lost track of unlabelled cells");
        }
        scan_from = s;

        fvk::CmResult rr, rx;
        if (fv_status st = pass(s, next, permA, &rr))
            return st;
        // George-Liu: move the root to the far end while the eccentricity grows
        for (;;) {
            if (fv_status st = pass(rr.pick, next, permB, &rx))
                return st;
            if (rx.ecc > rr.ecc) {
                rr = rx;
                std::swap(permA, permB);
            } else {
                break;
            }
        }
        if (rr.count <= 0 || next + (int64_t)rr.count > n)
            return fail(FV_EHIP, "renumbering produced an inconsistent component size");
        HIP_TRY(fvk::launch_commit_labels(next, rr.count, permA, c->perm, c->label, c->stream));
        next += rr.count;
    }
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
    c->nrm_o = reinterpret_cast<double *>(p);
    p += lay.nrm;
    c->nrm_w = reinterpret_cast<double *>(p);
    p += lay.nrm;
    c->area_o = reinterpret_cast<double *>(p);
    p += lay.area;
    c->inv_area_w = reinterpret_cast<double *>(p);
    p += lay.area;
    c->perm = reinterpret_cast<int32_t *>(p);
    p += lay.idx;
    c->label = reinterpret_cast<int32_t *>(p);
    p += lay.idx;
    c->scratch = p;
    p += lay.scratch;
    c->small = p;
    *out = c;
    return FV_OK;
}

fv_status fv_upload_mesh(fv_ctx *c, const int32_t *nbr, const double *nrm, const double *area)
{
    g_last_error.clear();
    if (fv_status st = check_ctx(c))
        return st;
    if (!nbr || !nrm || !area)
        return fail(FV_EINVAL, "null mesh array");
    if (fv_status st = validate_mesh(c->n, nbr, nrm, area))
        return st;
    const size_t n = (size_t)c->n;
    c->mesh_ready = false;
    c->state_ready = false;
    c->closed = normals_closed(c->n, nrm);
    HIP_TRY(hipMemcpyAsync(c->scratch, nbr, n * 3 * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(fvk::launch_nb_aos_to_soa(c->n, c->ld, reinterpret_cast<int32_t *>(c->scratch),
                                      c->nb_o, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));  // scratch is reused below
    HIP_TRY(hipMemcpyAsync(c->scratch, nrm, n * 6 * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(fvk::launch_nrm_aos_to_soa(c->n, c->ld, reinterpret_cast<double *>(c->scratch),
                                       c->nrm_o, c->stream));
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
    // The state moves to the uploaded order in the spare buffer, then to the
    // new order in the current one.
    double4 *spare = c->U[c->cur ^ 1];
    if (c->state_ready)
        HIP_TRY(fvk::launch_gather_state(c->n, c->label, c->U[c->cur], spare, c->stream));
    if (method == FV_ORDER_IDENTITY) {
        HIP_TRY(fvk::launch_iota(c->perm, c->n, c->stream));
        HIP_TRY(fvk::launch_iota(c->label, c->n, c->stream));
    } else {
        if (fv_status st = cm_order(c))
            return st;
    }
    if (fv_status st = regather_geometry(c))
        return st;
    if (c->state_ready)
        HIP_TRY(fvk::launch_gather_state(c->n, c->perm, spare, c->U[c->cur], c->stream));
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
    for (int32_t s = 0; s < n_steps; ++s) {
        HIP_TRY(fvk::launch_step(c->n, c->ld, c->U[c->cur], c->U[c->cur ^ 1], c->nb_w, c->nb16_w,
                                 c->nrm_w, c->inv_area_w, dt, c->gamma, c->narrow, c->closed,
                                 c->stream));
        c->cur ^= 1;
    }
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
    return 32 + 32 + 8 + (c->narrow ? 8 : 12) + (c->closed ? 32 : 48);
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

fv_status fv_destroy(fv_ctx *c)
{
    g_last_error.clear();
    if (!c)
        return fail(FV_EINVAL, "null context");
    delete c;
    return FV_OK;
}

const char *fv_last_error(void)
{
    return g_last_error.c_str();
}

}  // extern "C"
