/*
 * fvgpu.h -- C ABI of the MI355X (gfx950) finite-volume Euler library.
 *
 * The library advances the 2D Euler equations on a closed unstructured
 * triangle mesh with the explicit cell-centred finite-volume scheme of
 * Nagy et al., "Accelerating unstructured finite volume computations on
 * field-programmable gate arrays" (arXiv:1408.5715), section 6:
 *
 *   U_T^{n+1} = U_T^n - dt / V_T * sum_{f=0..2} R_{n_f} F_f |n_f|
 *
 * with U = (rho, rho u, rho v, E), the Lax-Friedrichs numerical flux F_f
 * (eqCompFlux) evaluated between the cell and its neighbour across face f,
 * n_f the outward face normal scaled by the face length and V_T the cell
 * area (section 6.2.1).  It also renumbers cells for locality (section 4:
 * breadth-first Cuthill-McKee labelling from a pseudo-diameter endpoint) and
 * applies the permutation on the device.
 *
 * Conventions for every entry point:
 *   - All work runs on the HIP stream given to fv_create, in issue order,
 *     except the confirming sweep of a Cuthill-McKee renumbering, which runs
 *     on a second stream the context creates (default priority) and which
 *     the calls that depend on it wait for (see fv_renumber).
 *   - Host arrays are read or written during the call only; the caller owns
 *     them.  Device memory is one arena the caller allocates and owns; the
 *     library never allocates or frees device memory.
 *   - A status < 0 is an error; fv_last_error() returns a message for the
 *     calling thread.  Argument and mesh validation happens on the host
 *     before any HIP call, so a rejected call leaves the device untouched.
 *   - Results are deterministic: the step is gather-only (no atomics), so the
 *     same inputs give bitwise-equal outputs, whatever the cell numbering.
 *   - A context is not thread-safe; use one context per thread.
 */
#ifndef FVGPU_H
#define FVGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fv_ctx fv_ctx;
typedef int32_t fv_status;

#define FV_OK 0
#define FV_EINVAL (-1)  /* null or mis-sized argument, bad n, dt or step count, small arena */
#define FV_EMESH (-2)   /* mesh fails validation (see fv_upload_mesh) */
#define FV_ESTATE (-3)  /* state not positive or not finite, or not uploaded yet */
#define FV_EHIP (-4)    /* a HIP runtime call failed; the message carries hipGetErrorString */
#define FV_ENOMEM (-5)  /* host allocation failed */

#define FV_ORDER_IDENTITY 0
#define FV_ORDER_CM 1

#define FV_CORRECTION_PARAMS 5252

/* Largest mesh (cells) a context accepts: device offsets such as 6 n + i are
 * formed in 32-bit integers.  About 77 GB of arena at this size. */
#define FV_MAX_CELLS 268431360

/*
 * Device bytes the arena passed to fv_create must hold for n_cells cells
 * (about 288 bytes per cell plus 13 MB of fixed tables).  Returns 0 if
 * n_cells <= 0 or n_cells > FV_MAX_CELLS.
 */
size_t fv_arena_bytes(int64_t n_cells);

/*
 * Create a context for a mesh of n_cells triangles (section 6.2.1),
 * 1 <= n_cells <= FV_MAX_CELLS.
 *   gamma       ratio of specific heats (the paper uses 1.4; section 6.1);
 *               must be finite and > 1.
 *   d_arena     device pointer, 256-byte aligned, >= fv_arena_bytes(n_cells);
 *               owned by the caller, must outlive the context.
 *   hip_stream  hipStream_t (NULL = default stream) all work is issued on.
 *   out         receives the context.
 * FV_EINVAL on any bad argument.  Issues no HIP call.
 */
fv_status fv_create(int64_t n_cells, double gamma, void *d_arena, size_t arena_bytes,
                    void *hip_stream, fv_ctx **out);

/*
 * Upload the mesh (section 6.2.1; data structures of section 3: node array
 * plus fixed-degree connectivity and precomputed face normals, section 7).
 *   nbr   host int32 [n][3]: nbr[i][f] is the cell across face f of cell i.
 *   nrm   host double [n][3][2]: outward normal of face f of cell i, scaled
 *         by the face length.
 *   area  host double [n]: cell areas (V_T).
 * Validation (FV_EMESH): every index in [0, n) and not i itself; every face
 * (i, f) has a partner face (j, g) with nbr[j][g] == i and
 * nrm[j][g] == -nrm[i][f] exactly (the mesh is closed, e.g. periodic);
 * normals finite and non-zero; areas finite and > 0.
 * Resets the cell order to the identity and invalidates the state.
 * Synchronous with respect to the host arrays.
 */
fv_status fv_upload_mesh(fv_ctx *ctx, const int32_t *nbr, const double *nrm, const double *area);

/*
 * Upload a batch of independent closed meshes as one mesh of n_cells cells
 * (the step of section 6.2.2 applied to each mesh; every mesh keeps its own
 * time step, see fv_step_batch).
 *   n_meshes    1 .. 65536.
 *   mesh_begin  host int64 [n_meshes + 1]: mesh k owns cells
 *               [mesh_begin[k], mesh_begin[k+1]); mesh_begin[0] = 0,
 *               mesh_begin[n_meshes] = n_cells, strictly increasing.
 *   nbr, nrm, area  as for fv_upload_mesh, in batch numbering.
 * Validation as for fv_upload_mesh (FV_EMESH), plus FV_EMESH if a face joins
 * two meshes and FV_EINVAL for bad offsets.  Renumbering then keeps every
 * mesh in its own range of cells.
 */
fv_status fv_upload_batch(fv_ctx *ctx, int32_t n_meshes, const int64_t *mesh_begin,
                          const int32_t *nbr, const double *nrm, const double *area);

/*
 * Upload the conserved state U = (rho, rho u, rho v, E) (section 6.1).
 *   U  host double [n][4], in the numbering of the uploaded mesh.
 * FV_ESTATE if any rho or p = (gamma - 1)(E - rho (u^2 + v^2) / 2) is not
 * finite and > 0.  Requires an uploaded mesh.
 */
fv_status fv_upload_state(fv_ctx *ctx, const double *U);

/*
 * Same as fv_upload_state for a device array d_U [n][4] (original numbering)
 * that is already resident in device memory; it is read on the stream, so
 * it must stay valid until the stream reaches this point.  No validation of
 * the values (they are not on the host).
 */
fv_status fv_upload_state_device(fv_ctx *ctx, const double *d_U);

/*
 * Renumber the cells for memory locality (section 4; motivation in
 * sections 3 and 7.2) and permute every per-cell array on the device.
 *   method    FV_ORDER_IDENTITY: the uploaded order.
 *             FV_ORDER_CM: Cuthill-McKee.  Each connected component, taken
 *             in order of its lowest cell id, is labelled breadth-first from a
 *             pseudo-peripheral root (George-Liu search from that lowest id:
 *             move to the last-level cell of minimum (degree, id) while the
 *             eccentricity grows); the children of each labelled cell are
 *             appended in (degree, id) order.  Ids are those of the uploaded
 *             mesh, so the order depends only on the mesh.  Runs entirely on
 *             the device, one workgroup per mesh of a batch.
 *   perm_out  nullable host int32 [n]: perm_out[new] = uploaded id.
 * The state (if uploaded) is carried over.  Results of fv_step do not
 * depend on the order (bitwise).  Synchronises the stream.
 *
 * With FV_ORDER_CM and perm_out NULL the call does not wait for the search's
 * confirming sweep (the level structure from the first candidate, which only
 * decides whether the search moves on).  The labels assume that it does not,
 * the sweep runs on a second stream of the context while the caller's work
 * (typically fv_step) proceeds, and the check is made at the next call that
 * needs it: fv_renumber_passes, fv_working_order, fv_download_state,
 * fv_upload_state, fv_step_adjoint(_grad), fv_upload_mesh/batch, fv_renumber
 * and fv_destroy wait for the sweep.  If some search would have moved, the
 * first four of these relabel exactly as the sequential search does before
 * they go on.  The state keeps its values, since fv_step gives the same bits
 * in any order, so the only visible effect is the working order until then.
 */
fv_status fv_renumber(fv_ctx *ctx, int32_t method, int32_t *perm_out);

/*
 * The working (renumbered) order: perm_out[new] = uploaded id, host int32
 * [n], after any pending check of fv_renumber.  Synchronises the stream.
 */
fv_status fv_working_order(fv_ctx *ctx, int32_t *perm_out);

/*
 * Advance n_steps forward-Euler steps of size dt (section 6.2.2, eqFWEuler
 * and the update equation with the Lax-Friedrichs flux of eqCompFlux).
 * n_steps >= 0; dt finite and > 0 (no CFL check: the caller picks dt).
 * Asynchronous: returns once the kernels are queued on the stream.
 */
fv_status fv_step(fv_ctx *ctx, int32_t n_steps, double dt);

/*
 * fv_step for a batch: mesh k advances with time step dt[k].
 *   dt  host double [n_meshes], finite and > 0.
 * All meshes advance in one launch per step.  Asynchronous like fv_step.
 */
fv_status fv_step_batch(fv_ctx *ctx, int32_t n_steps, const double *dt);

/*
 * Adjoint of one step of size dt (section 6.2.2's update, differentiated):
 * given the state U^n at which the step is taken and the cotangent lambda of
 * U^{n+1}, overwrite lambda with the cotangent of U^n,
 *   lambda_k <- lambda_k - sum_f (dG(U_k, U_j, n_f)/dU_k)^T (c_k lambda_k - c_j lambda_j)
 * with G the face flux times |n_f| and c = dt / V.  When a learned
 * correction is set (fv_set_correction), G includes it and its Jacobian
 * (bfloat16 roundings are differentiated as the identity).  For a batch,
 * all meshes use this dt.
 *   d_U       device double [n][4], numbering of the uploaded mesh, 32-byte aligned.
 *   d_lambda  device double [n][4], same numbering, in/out, 32-byte aligned.
 * The adjoint runs on the working (renumbered) geometry, as fv_step does: U
 * and lambda are gathered into the working order and each cell's result is
 * written back to its place in the uploaded numbering, so each cell's result
 * does not depend on the renumbering.  Asynchronous on the stream; uses the
 * context's scratch memory and its spare state buffer (the current state is
 * kept).
 */
fv_status fv_step_adjoint(fv_ctx *ctx, const double *d_U, double *d_lambda, double dt);

/*
 * fv_step_adjoint that also accumulates the gradient of the loss with
 * respect to the correction's parameters: d_grad += (dU^{n+1}/dtheta)^T
 * lambda, in the parameter order of fv_set_correction.
 *   d_grad  device double [FV_CORRECTION_PARAMS], 8-byte aligned, in/out;
 *           NULL makes this fv_step_adjoint.
 * FV_ESTATE if d_grad is given and no correction is set.  The sum over the
 * cells is taken in a fixed order (the working order) for a given mesh and
 * renumbering, so repeated calls give the same bits.  Asynchronous on the
 * stream.
 */
fv_status fv_step_adjoint_grad(fv_ctx *ctx, const double *d_U, double *d_lambda, double dt,
                               double *d_grad);

/*
 * Learned correction of the face flux (not in the paper; added to its
 * Lax-Friedrichs flux of section 6.2.2).  Per face, with e the unit normal,
 * t = (-e_y, e_x), l the face length, a = 1/V and c = dt/V of both cells:
 *   x(L, R, n) = [rho_L - 1, u.e_L, u.t_L, p_L - 1, rho_R - 1, u.e_R, u.t_R,
 *                 p_R - 1, e_x, e_y, l^2 (a_L + a_R)/2, l (c_L + c_R)/2]
 *   y(x) = W3^T h2 + b3, h2 = relu(W2^T h1 + b2), h1 = relu(W1^T x + b1),
 *   inputs, activations, weights and b1 in bfloat16, products summed in
 *   float32;
 *   G += l (R(e) y(x(L, R, n)) - R(-e) y(x(R, L, -n))),
 *   R(e) y = (y0, y1 e_x + y2 t_x, y1 e_y + y2 t_y, y3).
 * The added flux is exactly antisymmetric across every face, so mass,
 * momentum and energy stay conserved to round-off.
 *   params  host float [FV_CORRECTION_PARAMS]: W1 [12][64], b1 [64],
 *           W2 [64][64], b2 [64], W3 [64][4], b3 [4], row-major [in][out];
 *           NULL disables the correction (the plain step).
 *   count   FV_CORRECTION_PARAMS, or 0 with NULL.
 * FV_EINVAL on a wrong count or a non-finite parameter.  Applies to every
 * later fv_step / fv_step_batch.  Synchronises the stream.
 */
fv_status fv_set_correction(fv_ctx *ctx, const float *params, int32_t count);

/*
 * Weighted gather of states from one mesh onto another, the area-weighted
 * restriction of a fine solution to a coarse mesh that nests it (the
 * training targets of the learned correction):
 *   out[i] = sum_{m<k} w[i][m] src[idx[i][m]]   (all four components, m in order)
 *   d_src  device double [n_src][4], 32-byte aligned;
 *   d_idx  device int32 [n][k]; d_w device double [n][k] (for a restriction,
 *          the fine cells' areas over the coarse cell's area);
 *   d_out  device double [n][4], 32-byte aligned, must not overlap d_src.
 * A row with an index outside [0, n_src) is written as NaN (nothing is read
 * for that index).  FV_EINVAL on null, misaligned or bad sizes (1 <= k <=
 * 1024).  Needs no context; asynchronous on hip_stream (NULL: the null
 * stream).
 */
fv_status fv_restrict(const double *d_src, int64_t n_src, const int32_t *d_idx, const double *d_w,
                      int64_t n, int32_t k, double *d_out, void *hip_stream);

/*
 * Launch shape of the step kernel (no effect on results, which are bitwise
 * independent of it).
 *   block      workgroup size: 128, 256 (default) or 512 cells.
 *   grid       0 (default): one workgroup per tile of `block` cells;
 *              g > 0: g persistent workgroups striding over the tiles.
 *   use_graph  1: fv_step / fv_step_batch capture their launches into a HIP
 *              graph (cached for the same step count and layout) and launch
 *              it as one unit on the context's stream; 0 (default): launch
 *              kernel by kernel.
 * FV_EINVAL for other values.
 */
fv_status fv_set_launch(fv_ctx *ctx, int32_t block, int32_t grid, int32_t use_graph);

/*
 * Number of breadth-first passes (level structures of section 4's
 * renumbering, including the pseudo-peripheral search) each mesh took in the
 * last fv_renumber with FV_ORDER_CM.  The search's first pass over a mesh's
 * first component labels it from the lowest id; the second sweep runs on a
 * copy of the graph renamed by those labels (same eccentricity, better
 * memory locality).  If the eccentricity does not grow, the first pass's
 * labels are the result and the mesh counts 2 passes; if it grows, the
 * search repeats that sweep as a labelling pass on the uploaded graph, so
 * such a mesh counts one pass more than the sequential search takes.
 *   passes  host int32 [n_meshes].  Synchronises the stream.
 * FV_ESTATE if no FV_ORDER_CM renumbering ran since the mesh was uploaded
 * (or the last renumbering was FV_ORDER_IDENTITY).
 */
fv_status fv_renumber_passes(fv_ctx *ctx, int32_t *passes);

/*
 * Copy the state back in the numbering of the uploaded mesh.
 *   U  host double [n][4].  Synchronises the stream.
 */
fv_status fv_download_state(fv_ctx *ctx, double *U);

/*
 * Same as fv_download_state into a device array d_U [n][4]; asynchronous on
 * the stream.
 */
fv_status fv_download_state_device(fv_ctx *ctx, double *d_U);

/*
 * Algorithmic device-memory bytes one cell update of fv_step moves with the
 * current layout: the state read and written (32 + 32), 1/V_T (8), the
 * neighbour indices (12 as 32-bit ids, or 8 as 16-bit offsets when the
 * current order keeps every neighbour within 32767 cells) and the face
 * normals (48; 32 when every cell's normals satisfy n_2 = -(n_0 + n_1)
 * exactly and the third is derived; 16 when, in addition, every component of
 * the first two is an integer multiple of 2^-32 smaller than 1/2 in size, as
 * on meshes snapped to 2^-32, and they are stored as 32-bit fixed-point
 * values that decode to the same doubles).  Neighbour states are counted as cache
 * hits (the reuse the renumbering of section 4 provides).  Returns 0 on a
 * null context or before the mesh is uploaded.
 */
int64_t fv_bytes_per_update(const fv_ctx *ctx);

/*
 * Check that every cell has finite rho > 0 and p > 0 (section 6.1 state
 * admissibility).  Returns FV_OK or FV_ESTATE.  Synchronises the stream.
 */
fv_status fv_check_state(fv_ctx *ctx);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): fv_step
 * on a mesh and state that already live in device memory, with no context
 * and no arena.  The step's scratch (the second state buffer of the
 * ping-pong and dt / V_T per cell, 40 bytes per cell) is a static device
 * array of FV_STATIC_MAX_CELLS cells that each device the library runs on
 * holds until the process ends.  Calls on one device share that array and
 * leave their values in it (each call writes it before reading it), so calls
 * that overlap on one device race: issue them on one stream, or serialise
 * them.
 *   n_cells  1 .. FV_STATIC_MAX_CELLS; FV_EINVAL beyond (nothing is
 *            allocated instead).
 *   d_nbr    device int32 [3][n_cells] (structure of arrays: neighbour
 *            across face f of cell i at d_nbr[f * n_cells + i]); every index
 *            in [0, n_cells) and the mesh closed as fv_upload_mesh requires
 *            (not checked: the arrays stay on the device).
 *   d_nrm    device double [6][n_cells]: nx_0, ny_0, nx_1, ny_1, nx_2, ny_2
 *            (outward, scaled by the face length), structure of arrays.
 *   d_area   device double [n_cells], > 0.
 *   d_U      device double [n_cells][4] (rho, rho u, rho v, E), 32-byte
 *            aligned, in/out: advanced by n_steps steps of size dt.
 *   gamma    finite and > 1.
 * The result is bitwise that of fv_step on the same mesh and state.  The
 * device is the current one; asynchronous on hip_stream (NULL: the null
 * stream).  Calls no allocating routine.
 */
#define FV_STATIC_MAX_CELLS 1048576
fv_status fv_step_static(int64_t n_cells, const int32_t *d_nbr, const double *d_nrm,
                         const double *d_area, double *d_U, int32_t n_steps, double dt,
                         double gamma, void *hip_stream);

/* Release the host-side context.  Does not touch the arena. */
fv_status fv_destroy(fv_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *fv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FVGPU_H */
