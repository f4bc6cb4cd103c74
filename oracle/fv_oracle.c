/*
 * CPU oracle for the unstructured cell-centred finite-volume Euler step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously
 * correct reference the HIP library is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may build,
 * load or call it; the product path never does.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no FMA
 * contraction, so every rounding happens where the source writes it).
 *
 * Source: Nagy et al., "Accelerating unstructured finite volume
 * computations on field-programmable gate arrays" (arXiv:1408.5715).
 *   - Section 6.1: Euler equations, state U = (rho, rho u, rho v, E),
 *     E = p/(gamma-1) + rho |v|^2 / 2, c = sqrt(gamma p / rho), gamma = 1.4.
 *   - Section 6.2.1: cell-centred triangles; n_f is the outward face normal
 *     scaled by the face length; V_T is the cell's area.
 *   - Section 6.2.2: semi-discrete form (eqSemiDiscrete), Lax-Friedrichs
 *     numerical flux (eqCompFlux), forward Euler (eqFWEuler), the update
 *     U^{n+1} = U^n - dt/V_T * sum_f R_{n_f} F_f |n_f|, and the face-frame
 *     component form (eqFi group).
 *   - Section 4.1: matrix bandwidth B_f(G), C_BW = 2 B_f(G) + 1 and the
 *     serial bandwidth S_BW.
 *   - Section 4.2.2: the pseudo-diameter start vertex used before the
 *     breadth-first labelling (Gibbs-Poole-Stockmeyer subroutine, realised
 *     here as the George-Liu pseudo-peripheral node search), and the Amoeba1
 *     (AM1) labelling of section 4.2 (bookkeeping s(i), u(i), I, imp(i) of
 *     section 4.2.1; candidate choice of section 4.2.2).
 *
 * Readings taken where the paper is silent or garbled:
 *   - Dissipation sign: F = (F_L + F_R)/2 - alpha (U_R - U_L)/2 as in
 *     eqCompFlux (the eqFi group prints "+", which is anti-diffusive).
 *   - alpha = |mean of the two face-normal velocities| + mean of the two
 *     sound speeds.
 *   - Face-frame tangent t = (-n_y, n_x) for unit normal n = (n_x, n_y).
 *   - The flux is evaluated with the unit normal and multiplied by the face
 *     length |n_f| once.
 *   - Faces are summed in stored order, ((F_0 + F_1) + F_2).
 *   - S_BW uses closed neighbourhoods (a node is a neighbour of itself).
 *   - Cuthill-McKee children are visited in order of (degree, id).
 *   - AM1: the "random element of u(I)" that starts the candidate search is
 *     the smallest id of u(I); candidates are scanned in increasing id; s(i)
 *     of a part's first node is 0; AM1 starts from the same pseudo-peripheral
 *     root as Cuthill-McKee, and a disconnected graph restarts a new part
 *     from its lowest unlabelled id.
 */

#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Primitive quantities of one state (section 6.1). */
static void primitives(const double *U, double gamma, double *rho, double *u, double *v,
                       double *p, double *c)
{
    *rho = U[0];
    *u = U[1] / U[0];
    *v = U[2] / U[0];
    /* p from E = p/(gamma-1) + rho (u^2 + v^2)/2 */
    *p = (gamma - 1.0) * (U[3] - 0.5 * (*rho) * ((*u) * (*u) + (*v) * (*v)));
    *c = sqrt(gamma * (*p) / (*rho));
}

/*
 * Lax-Friedrichs flux through one face, returned in the x-y frame and
 * multiplied by the face length: R_{n_f} F_f |n_f| of section 6.2.2.
 * UL is the cell being updated, UR the cell across the face, (nx, ny) the
 * outward normal of the face scaled by its length.
 */
void oracle_face_flux(const double *UL, const double *UR, double nx, double ny, double gamma,
                      double *Fout)
{
    double len = sqrt(nx * nx + ny * ny);
    /* face frame: x' along the unit outward normal, y' along the tangent */
    double ex = nx / len, ey = ny / len;
    double tx = -ey, ty = ex;

    double rL, uL, vL, pL, cL, rR, uR, vR, pR, cR;
    primitives(UL, gamma, &rL, &uL, &vL, &pL, &cL);
    primitives(UR, gamma, &rR, &uR, &vR, &pR, &cR);

    /* velocities in the face frame */
    double unL = uL * ex + vL * ey, vtL = uL * tx + vL * ty;
    double unR = uR * ex + vR * ey, vtR = uR * tx + vR * ty;

    /* rotated conserved states */
    double QL[4] = {rL, rL * unL, rL * vtL, UL[3]};
    double QR[4] = {rR, rR * unR, rR * vtR, UR[3]};

    /* x-component of the flux tensor (eqFlux) in the face frame */
    double GL[4] = {rL * unL, rL * unL * unL + pL, rL * unL * vtL, (UL[3] + pL) * unL};
    double GR[4] = {rR * unR, rR * unR * unR + pR, rR * unR * vtR, (UR[3] + pR) * unR};

    /* |u bar| + c bar: averages at the interface (eqCompFlux) */
    double alpha = fabs(0.5 * (unL + unR)) + 0.5 * (cL + cR);

    double Fp[4];
    for (int k = 0; k < 4; ++k)
        Fp[k] = 0.5 * (GL[k] + GR[k]) - alpha * 0.5 * (QR[k] - QL[k]);

    /* rotate back to x-y, then scale by the face length |n_f| */
    Fout[0] = len * Fp[0];
    Fout[1] = len * (Fp[1] * ex + Fp[2] * tx);
    Fout[2] = len * (Fp[1] * ey + Fp[2] * ty);
    Fout[3] = len * Fp[3];
}

/* Area-scaled sum of the three face fluxes of cell i (eqSemiDiscrete). */
void oracle_cell_residual(int64_t i, const int32_t *nbr, const double *nrm, const double *U,
                          double gamma, double *R)
{
    R[0] = R[1] = R[2] = R[3] = 0.0;
    for (int f = 0; f < 3; ++f) {
        int64_t j = nbr[3 * i + f];
        double F[4];
        oracle_face_flux(&U[4 * i], &U[4 * j], nrm[6 * i + 2 * f], nrm[6 * i + 2 * f + 1], gamma,
                         F);
        for (int k = 0; k < 4; ++k)
            R[k] += F[k];
    }
}

/*
 * n_steps forward-Euler steps (eqFWEuler and the update of section 6.2.2):
 * U_T^{n+1} = U_T^n - dt / V_T * sum_f R_{n_f} F_f |n_f|.
 * U is [n][4] (rho, rho u, rho v, E), updated in place; every step reads the
 * whole of U^n before any U^{n+1} value is used.  With n_threads > 1 the
 * cells of each step are shared among that many OpenMP threads (static
 * schedule); every cell's update reads only U^n, so the result is bitwise the
 * same.  Returns the number of threads that ran the cell loop, or -1 on a
 * bad argument or allocation failure.
 */
static int run_steps(int64_t n, const int32_t *nbr, const double *nrm, const double *area,
                     double gamma, double dt, int64_t n_steps, double *U, int n_threads)
{
    if (n <= 0 || n_steps < 0 || n_threads < 1 || !nbr || !nrm || !area || !U)
        return -1;
    double *Un = (double *)malloc((size_t)n * 4 * sizeof(double));
    if (!Un)
        return -1;
    double *cur = U, *nxt = Un;
    int used = 1;
    for (int64_t s = 0; s < n_steps; ++s) {
#pragma omp parallel for num_threads(n_threads) schedule(static) if (n_threads > 1)
        for (int64_t i = 0; i < n; ++i) {
            double R[4];
            oracle_cell_residual(i, nbr, nrm, cur, gamma, R);
            double coef = dt / area[i];
            for (int k = 0; k < 4; ++k)
                nxt[4 * i + k] = cur[4 * i + k] - coef * R[k];
            if (i == 0)
                used = omp_get_num_threads();
        }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != U)
        memcpy(U, cur, (size_t)n * 4 * sizeof(double));
    free(Un);
    return used;
}

/* The steps on the calling thread.  Returns 0, or -1 on a bad argument or
 * allocation failure. */
int oracle_step(int64_t n, const int32_t *nbr, const double *nrm, const double *area,
                double gamma, double dt, int64_t n_steps, double *U)
{
    return run_steps(n, nbr, nrm, area, gamma, dt, n_steps, U, 1) < 0 ? -1 : 0;
}

/* The steps with the cell loop on n_threads OpenMP threads (timing the
 * oracle on all the cores of a host).  Returns the number of threads used,
 * or -1. */
int oracle_step_threads(int64_t n, const int32_t *nbr, const double *nrm, const double *area,
                        double gamma, double dt, int64_t n_steps, double *U, int n_threads)
{
    return run_steps(n, nbr, nrm, area, gamma, dt, n_steps, U, n_threads);
}

/* ---------------------------------------------------------------------- */
/* Renumbering (section 4): Cuthill-McKee labelling from a pseudo-diameter */
/* endpoint, and the bandwidth metrics of section 4.1.                     */
/* ---------------------------------------------------------------------- */

/* Distinct neighbours of v other than v itself, in stored face order. */
static int distinct_neighbours(const int32_t *nbr, int64_t v, int32_t out[3])
{
    int d = 0;
    for (int f = 0; f < 3; ++f) {
        int32_t w = nbr[3 * v + f];
        if (w == v)
            continue;
        int seen = 0;
        for (int g = 0; g < d; ++g)
            if (out[g] == w)
                seen = 1;
        if (!seen)
            out[d++] = w;
    }
    return d;
}

static int degree_of(const int32_t *nbr, int64_t v)
{
    int32_t tmp[3];
    return distinct_neighbours(nbr, v, tmp);
}

/*
 * Breadth-first level structure rooted at r over the vertices with
 * mark[v] == 0 (the current component).  Returns the eccentricity of r (the
 * number of levels minus one) and the vertex of minimum (degree, id) in the
 * last level.  'queue' and 'dist' are scratch arrays of n entries; dist must
 * hold -1 for every vertex of the component on entry and is restored.
 */
static int64_t level_structure(int64_t n, const int32_t *nbr, const uint8_t *mark, int64_t r,
                               int64_t *queue, int64_t *dist, int64_t *last_pick)
{
    (void)n;
    int64_t head = 0, tail = 0;
    queue[tail++] = r;
    dist[r] = 0;
    int64_t ecc = 0;
    while (head < tail) {
        int64_t v = queue[head++];
        if (dist[v] > ecc)
            ecc = dist[v];
        int32_t nb[3];
        int d = distinct_neighbours(nbr, v, nb);
        for (int g = 0; g < d; ++g) {
            int64_t w = nb[g];
            if (!mark[w] && dist[w] < 0) {
                dist[w] = dist[v] + 1;
                queue[tail++] = w;
            }
        }
    }
    int64_t best = -1, best_deg = 0;
    for (int64_t q = 0; q < tail; ++q) {
        int64_t v = queue[q];
        if (dist[v] != ecc)
            continue;
        int64_t dg = degree_of(nbr, v);
        if (best < 0 || dg < best_deg || (dg == best_deg && v < best)) {
            best = v;
            best_deg = dg;
        }
    }
    for (int64_t q = 0; q < tail; ++q)
        dist[queue[q]] = -1;
    *last_pick = best;
    return ecc;
}

/*
 * George-Liu pseudo-peripheral root of the component of s among unmarked
 * vertices: from r = s, take the last level's vertex x of minimum
 * (degree, id); if x has a larger eccentricity than r, continue from x,
 * else return r.
 */
static int64_t pseudo_peripheral_root(int64_t n, const int32_t *nbr, const uint8_t *mark,
                                      int64_t s, int64_t *queue, int64_t *dist)
{
    int64_t r = s, x;
    int64_t ecc_r = level_structure(n, nbr, mark, r, queue, dist, &x);
    for (;;) {
        int64_t x2;
        int64_t ecc_x = level_structure(n, nbr, mark, x, queue, dist, &x2);
        if (ecc_x > ecc_r) {
            r = x;
            ecc_r = ecc_x;
            x = x2;
        } else {
            return r;
        }
    }
}

/*
 * Cuthill-McKee ordering of the dual graph given by nbr [n][3].
 * perm_out[new_label] = old id.
 * Each connected component is labelled in turn, starting with the component
 * of the lowest-id unlabelled vertex s.  Its root is a pseudo-peripheral
 * vertex found by the George-Liu search from s: take the last level of the
 * level structure rooted at r, pick its vertex of minimum (degree, id) x; if
 * x has a larger eccentricity than r, continue from x, else keep r.
 * The labelling visits labelled vertices in label order and appends each
 * one's unlabelled neighbours sorted by (degree, id).
 * Returns 0, or -1 on a bad argument or allocation failure.
 */
int oracle_cm_order(int64_t n, const int32_t *nbr, int32_t *perm_out)
{
    if (n <= 0 || !nbr || !perm_out)
        return -1;
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!mark || !queue || !dist) {
        free(mark);
        free(queue);
        free(dist);
        return -1;
    }
    for (int64_t v = 0; v < n; ++v)
        dist[v] = -1;

    int64_t next = 0;
    int64_t scan = 0;
    while (next < n) {
        while (mark[scan])
            ++scan;
        const int64_t r = pseudo_peripheral_root(n, nbr, mark, scan, queue, dist);

        /* Cuthill-McKee labelling of the component from r */
        int64_t head = next;
        perm_out[next++] = (int32_t)r;
        mark[r] = 1;
        while (head < next) {
            int64_t v = perm_out[head++];
            int32_t nb[3];
            int d = distinct_neighbours(nbr, v, nb);
            int32_t kid[3];
            int nk = 0;
            for (int g = 0; g < d; ++g)
                if (!mark[nb[g]])
                    kid[nk++] = nb[g];
            /* order children by (degree, id): insertion sort of <= 3 items */
            for (int a = 1; a < nk; ++a) {
                int32_t key = kid[a];
                int kd = degree_of(nbr, key);
                int b = a - 1;
                while (b >= 0) {
                    int bd = degree_of(nbr, kid[b]);
                    if (bd > kd || (bd == kd && kid[b] > key)) {
                        kid[b + 1] = kid[b];
                        --b;
                    } else {
                        break;
                    }
                }
                kid[b + 1] = key;
            }
            for (int a = 0; a < nk; ++a) {
                mark[kid[a]] = 1;
                perm_out[next++] = kid[a];
            }
        }
    }
    free(mark);
    free(queue);
    free(dist);
    return 0;
}

/*
 * Bandwidth metrics of section 4.1 for the labelling f(v) = label[v]
 * (0-based).  Outputs:
 *   out[0] = B_f(G) = max over edges |f(v) - f(u)|
 *   out[1] = C_BW = 2 B_f(G) + 1
 *   out[2] = S_BW = max_i (E(i) - S(i)), where for the node u labelled i,
 *            s(i) / e(i) are the min / max label over its closed
 *            neighbourhood, S(i) = min_{k >= i} s(k), E(i) = max_{k <= i} e(k).
 * Returns 0, or -1 on a bad argument or allocation failure.
 */
int oracle_bandwidth(int64_t n, const int32_t *nbr, const int32_t *label, int64_t *out)
{
    if (n <= 0 || !nbr || !label || !out)
        return -1;
    int64_t *s = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *e = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!s || !e) {
        free(s);
        free(e);
        return -1;
    }
    int64_t B = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t fu = label[u];
        int64_t lo = fu, hi = fu;
        for (int f = 0; f < 3; ++f) {
            int64_t fv = label[nbr[3 * u + f]];
            if (fv < lo)
                lo = fv;
            if (fv > hi)
                hi = fv;
            int64_t d = fv > fu ? fv - fu : fu - fv;
            if (d > B)
                B = d;
        }
        s[fu] = lo;
        e[fu] = hi;
    }
    /* S(i): suffix minimum of s; E(i): prefix maximum of e */
    for (int64_t i = n - 2; i >= 0; --i)
        if (s[i + 1] < s[i])
            s[i] = s[i + 1];
    for (int64_t i = 1; i < n; ++i)
        if (e[i - 1] > e[i])
            e[i] = e[i - 1];
    int64_t sbw = 0;
    for (int64_t i = 0; i < n; ++i)
        if (e[i] - s[i] > sbw)
            sbw = e[i] - s[i];
    out[0] = B;
    out[1] = 2 * B + 1;
    out[2] = sbw;
    free(s);
    free(e);
    return 0;
}


/*
 * Importance of the part's node at position p (section 4.2):
 * imp = (size - 1 - p) + |u(p)| + s(p) for p >= I, and 0 for p < I and for
 * ghost positions (ghost may be NULL).
 */
static int64_t am1_importance(int64_t p, int64_t I, int64_t size, const int64_t *uc,
                              const int64_t *sv, const uint8_t *ghost)
{
    if (p < I || (ghost && ghost[p]))
        return 0;
    return (size - 1 - p) + uc[p] + sv[p];
}

/*
 * AM1's next node (section 4.2): among u(I), the neighbours of node(I) not
 * yet in the part, the vertex k whose most important neighbour in the part
 * other than node(I) is most important,
 *   score(k) = max { imp(l) : l a neighbour of k in the part, l != node(I) }
 *              (0 when k has no such neighbour),
 * taken as an argmax of (score, -id): equal scores go to the smaller id
 * (the paper picks a random element of u(I) to start its search; reading
 * R13 replaces it by the smallest id).  pos[] holds part positions (-1
 * outside); uc[] and sv[] hold |u()| and s() by position.
 */
static int64_t am1_candidate(const int32_t *nbr, int64_t vI, const int64_t *pos, int64_t I,
                             int64_t size, const int64_t *uc, const int64_t *sv,
                             const uint8_t *ghost)
{
    int32_t around[3];
    const int na = distinct_neighbours(nbr, vI, around);
    int64_t best = -1, best_score = -1;
    for (int a = 0; a < na; ++a) {
        const int64_t k = around[a];
        if (pos[k] >= 0)
            continue; /* already in the part: not in u(I) */
        int32_t knb[3];
        const int kd = distinct_neighbours(nbr, k, knb);
        int64_t score = 0;
        for (int g = 0; g < kd; ++g) {
            const int64_t p = pos[knb[g]];
            if (p >= 0 && knb[g] != vI) {
                const int64_t imp = am1_importance(p, I, size, uc, sv, ghost);
                score = imp > score ? imp : score;
            }
        }
        if (best < 0 || score > best_score || (score == best_score && k < best)) {
            best = k;
            best_score = score;
        }
    }
    return best;
}

/*
 * Amoeba1 (AM1) labelling of section 4.2, perm_out[new_label] = old id.
 *
 * A part P grows one node per step.  For the node at position i of P
 * (0-based here; the paper counts from 1):
 *   s(i)  = i - (smallest position among its neighbours in P), 0 if none
 *           earlier;
 *   u(i)  = its neighbours not yet in P;
 *   I     = first position whose u() is not empty;
 *   imp(i) = (|P| - 1 - i) + |u(i)| + s(i) for i >= I, 0 for i < I.
 * Each step appends the candidate k of u(I) whose most important neighbour
 * in P other than node(I) has the largest imp(), the smaller id on ties
 * (am1_candidate).  The part starts at the George-Liu pseudo-peripheral
 * root (section 4.2.2's pseudo-diameter endpoint).
 * Returns 0, or -1 on a bad argument or allocation failure.
 */
static int am1_run(int64_t n, const int32_t *nbr, int32_t *perm_out, int64_t *exact_out)
{
    if (n <= 0 || !nbr || !perm_out)
        return -1;
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    int64_t *pos = (int64_t *)malloc((size_t)n * sizeof(int64_t));   /* position in P or -1 */
    int64_t *sv = (int64_t *)malloc((size_t)n * sizeof(int64_t));    /* s() by position */
    int64_t *uc = (int64_t *)malloc((size_t)n * sizeof(int64_t));    /* |u()| by position */
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *seen = (int64_t *)malloc((size_t)n * sizeof(int64_t)); /* union stamps */
    if (!mark || !pos || !sv || !uc || !queue || !dist || !seen) {
        free(mark);
        free(pos);
        free(sv);
        free(uc);
        free(queue);
        free(dist);
        free(seen);
        return -1;
    }
    for (int64_t v = 0; v < n; ++v) {
        pos[v] = -1;
        dist[v] = -1;
        seen[v] = -1;
        if (exact_out)
            exact_out[v] = -1;
    }
    int64_t size = 0; /* nodes labelled so far, over all parts */
    int64_t scan = 0;
    while (size < n) {
        while (mark[scan])
            ++scan;
        /* pseudo-peripheral root of this component, as for Cuthill-McKee */
        const int64_t r = pseudo_peripheral_root(n, nbr, mark, scan, queue, dist);
        const int64_t first = size; /* positions of this part start here */
        int64_t I = first;
        int64_t next = r;
        for (;;) {
            /* append `next` at position size */
            const int64_t m = size;
            perm_out[m] = (int32_t)next;
            pos[next] = m;
            mark[next] = 1;
            ++size;
            int32_t nb[3];
            const int d = distinct_neighbours(nbr, next, nb);
            int64_t lo = m, free_count = 0;
            for (int g = 0; g < d; ++g) {
                const int64_t p = pos[nb[g]];
                if (p >= 0) {
                    if (p < lo)
                        lo = p;
                    uc[p] -= 1; /* next is no longer uncovered for nb[g] */
                } else {
                    ++free_count;
                }
            }
            sv[m] = m - lo;
            uc[m] = free_count;
            while (I < size && uc[I] == 0)
                ++I;
            if (exact_out && I <= m) {
                /* Eq. exact-sbw for the node just added (i = m, part size
                 * size = m + 1): (size - 1 - i) + |union of u(k), I <= k <= i|
                 * + s(i).  The union is gathered from the stored neighbour
                 * lists of positions I..i (vertices not yet in the part). */
                int64_t un = 0;
                for (int64_t k = I; k <= m; ++k) {
                    int32_t kn[3];
                    const int kd = distinct_neighbours(nbr, perm_out[k], kn);
                    for (int g = 0; g < kd; ++g)
                        if (pos[kn[g]] < 0 && seen[kn[g]] != m) {
                            seen[kn[g]] = m;
                            ++un;
                        }
                }
                exact_out[m] = (size - 1 - m) + un + sv[m];
            }
            if (I >= size)
                break; /* component complete */

            next = am1_candidate(nbr, perm_out[I], pos, I, size, uc, sv, NULL);
        }
        (void)first;
    }
    free(mark);
    free(pos);
    free(sv);
    free(uc);
    free(queue);
    free(dist);
    free(seen);
    return 0;
}

int oracle_am1_order(int64_t n, const int32_t *nbr, int32_t *perm_out)
{
    return am1_run(n, nbr, perm_out, NULL);
}

/*
 * The serial bandwidth of each node of AM1's labelling by Eq. exact-sbw of
 * section 4.3.1: exact_out[i] = (n - i) + |union of u(k) over I <= k <= i| +
 * s(i), evaluated when node(i) joins the part (n = i + 1 then; the value
 * does not change at later steps while I <= i, since every step takes a
 * node of u(I) into the part), or -1 where I > i already then.  perm_out
 * receives the AM1 order.  Returns 0, or -1 on a bad argument or
 * allocation failure.
 */
int oracle_am1_exact_sbw(int64_t n, const int32_t *nbr, int32_t *perm_out, int64_t *exact_out)
{
    if (!exact_out)
        return -1;
    return am1_run(n, nbr, perm_out, exact_out);
}

/*
 * Access pattern with serial bandwidth at most `bound` (section 4.3): AM1
 * parts that stop growing when the largest imp() from position I on exceeds
 * the bound; a part's nodes before I are executed, the others only loaded
 * (reloaded later), and vertices executed by earlier parts that a part needs
 * again enter it as ghosts (u() empty, imp() = 0).  Each part starts at the
 * George-Liu root of the not-yet-executed vertices, searched from the lowest
 * such id.  Finalising a part: s* = min over positions k >= I of
 * (k - s(k)); nodes before s* executed by this part are perfect (all their
 * neighbours executed); nodes before I are executed.
 * Outputs: idx[m] (vertex of each load), ex[m] (1 where the load executes
 * it), part_begin[parts + 1], perfect[n]; counts[0] = m, counts[1] = parts.
 * Readings: a part that would stop before executing anything keeps growing
 * (cannot happen when bound > 3, the maximal degree); ghosts never become
 * perfect (the flag is set only for nodes executed by the part, as the
 * paper's finalisation states).
 * Returns 0; -1 on a bad argument (bound <= 3) or allocation failure; -2 if
 * the pattern or the part list exceeds its capacity.
 */
int oracle_am1_bounded(int64_t n, const int32_t *nbr, int64_t bound, int32_t *idx, uint8_t *ex,
                       int64_t cap, int64_t *part_begin, int64_t part_cap, uint8_t *perfect,
                       int64_t *counts)
{
    if (n <= 0 || !nbr || !idx || !ex || !part_begin || !perfect || !counts || bound <= 3 ||
        cap <= 0 || part_cap <= 1)
        return -1;
    uint8_t *done = (uint8_t *)calloc((size_t)n, 1);      /* executed */
    int64_t *pos = (int64_t *)malloc((size_t)n * sizeof(int64_t)); /* position in part, -1 */
    int64_t *pv = (int64_t *)malloc((size_t)n * sizeof(int64_t));  /* vertex by position */
    int64_t *sv = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *uc = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    uint8_t *ghost = (uint8_t *)malloc((size_t)n);
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int rc = 0;
    if (!done || !pos || !pv || !sv || !uc || !ghost || !queue || !dist) {
        rc = -1;
        goto out;
    }
    for (int64_t v = 0; v < n; ++v) {
        pos[v] = -1;
        dist[v] = -1;
        perfect[v] = 0;
    }
    int64_t m = 0, parts = 0, executed = 0, scan = 0;
    part_begin[0] = 0;
    while (executed < n) {
        while (done[scan])
            ++scan;
        int64_t next = pseudo_peripheral_root(n, nbr, done, scan, queue, dist);
        int64_t size = 0, I = 0;
        for (;;) {
            const int64_t p = size++;
            pv[p] = next;
            pos[next] = p;
            ghost[p] = done[next];
            int32_t nb[3];
            const int d = distinct_neighbours(nbr, next, nb);
            int64_t lo = p, free_count = 0;
            for (int g = 0; g < d; ++g) {
                const int64_t q = pos[nb[g]];
                if (q >= 0) {
                    if (q < lo)
                        lo = q;
                    if (!ghost[q])
                        uc[q] -= 1;
                } else {
                    ++free_count;
                }
            }
            sv[p] = ghost[p] ? 0 : p - lo;
            uc[p] = ghost[p] ? 0 : free_count;
            while (I < size && uc[I] == 0)
                ++I;
            if (I >= size)
                break; /* everything reachable is complete */
            int64_t max_imp = 0;
            for (int64_t k = I; k < size; ++k) {
                const int64_t imp = ghost[k] ? 0 : (size - 1 - k) + uc[k] + sv[k];
                if (imp > max_imp)
                    max_imp = imp;
            }
            if (max_imp > bound && I > 0)
                break;
            next = am1_candidate(nbr, pv[I], pos, I, size, uc, sv, ghost);
        }
        /* finalise the part */
        int64_t sstar = size;
        for (int64_t k = I; k < size; ++k)
            if (k - sv[k] < sstar)
                sstar = k - sv[k];
        if (m + size > cap || parts + 2 > part_cap) {
            rc = -2;
            goto out;
        }
        for (int64_t k = 0; k < size; ++k) {
            const int64_t v = pv[k];
            if (k < sstar && !done[v])
                perfect[v] = 1;
            const int run = k < I && !ghost[k];
            if (run) {
                done[v] = 1;
                ++executed;
            }
            idx[m] = (int32_t)v;
            ex[m] = (uint8_t)run;
            ++m;
            pos[v] = -1;
        }
        part_begin[++parts] = m;
    }
    counts[0] = m;
    counts[1] = parts;
out:
    free(done);
    free(pos);
    free(pv);
    free(sv);
    free(uc);
    free(ghost);
    free(queue);
    free(dist);
    return rc;
}
