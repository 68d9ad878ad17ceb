/*
 * orc.c -- plain double-precision CPU oracle for short-range Lennard-Jones
 * molecular dynamics (arXiv 2109.10876, "Code modernization strategies for
 * short-range non-bonded molecular dynamics simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or helper with the
 * GPU library, and the GPU library never calls it.
 *
 * Every routine is the plain definition of what the method computes, in
 * double precision, with no blocking, fusion or reordering:
 *   - Newton's equations m_i r_i'' = F_i with F = -grad U      (Sec. 2.1, Eq. newton)
 *   - Lennard-Jones pair potential, interactions only for r < r_cut
 *                                                        (Sec. 2.1.1, Eq. lj)
 *   - cell binning with cell edge >= search radius, 27-cell stencil,
 *     Verlet list = pairs within r_cut + r_skin          (Sec. 2.1.2)
 *   - velocity Verlet in two half steps (Integrate1 / Integrate2) with a
 *     skin-triggered re-binning                          (Sec. 2.1, Fig. 1)
 *   - FENE bonds and the purely repulsive LJ of the polymer melt, the
 *     cosine angle term on bonded triples of the ring melt, and a Langevin
 *     thermostat                                           (Sec. 4, setup)
 * Gradients of forces and energy with respect to positions and to the
 * (epsilon, sigma) tables are the analytic derivatives of Eq. lj.
 *
 * Conventions.  Orthorhombic periodic box L[3]; displacement
 * d = x_i - x_j reduced by the minimum-image rule d -= L*rint(d/L).
 * fr(r) = -U'(r)/r, so that the force on i from j is fr * d.  Pair sets are
 * unordered pairs i < j listed in lexicographic order.  Type tables are
 * [nt*nt] row-major and symmetric.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_OMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

#ifdef ORC_OMP
#define ORC_PAR_FOR _Pragma("omp parallel for schedule(static)")
#define ORC_PAR_FOR_SUM_K _Pragma("omp parallel for schedule(static) reduction(+ : k)")
#define ORC_PAR_FOR_MAX_DMAX _Pragma("omp parallel for schedule(static) reduction(max : dmax)")
#else
#define ORC_PAR_FOR
#define ORC_PAR_FOR_SUM_K
#define ORC_PAR_FOR_MAX_DMAX
#endif

/* ORC_OMP (a timing-only build, liborc_omp.so, used for the all-core CPU
 * baseline): the pair search runs over atoms i on all threads and the force
 * sum over pairs splits into per-thread partial force arrays.  Every pair's
 * arithmetic is the same; only the order in which per-atom forces and the
 * energy and virial are summed differs.  The checked build (liborc.so) has
 * ORC_OMP unset and runs every loop in the order written. */

/* ---------------------------------------------------------------- geometry */

EXPORT double orc_min_image(double d, double L) { return d - L * rint(d / L); }

static double dist2(const double *x, const double *y, const double *z,
                    const double *L, int32_t i, int32_t j,
                    double *dx, double *dy, double *dz)
{
    double a = orc_min_image(x[i] - x[j], L[0]);
    double b = orc_min_image(y[i] - y[j], L[1]);
    double c = orc_min_image(z[i] - z[j], L[2]);
    *dx = a; *dy = b; *dz = c;
    return a * a + b * b + c * c;
}

/* ------------------------------------------------------------- pair terms */

/* Eq. lj: U(r) = 4 eps [(sig/r)^12 - (sig/r)^6], kept only for r < rc.
 * With shift = 1 the energy is lowered by U(rc) so that it is continuous at
 * the cutoff; the force is never shifted.  Returns 1 inside the cutoff. */
EXPORT int orc_lj_pair(double r2, double eps, double sig, double rc, int32_t shift,
                       double *u, double *fr)
{
    *u = 0.0;
    *fr = 0.0;
    if (!(r2 < rc * rc)) return 0;
    double sr2 = sig * sig / r2;
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    double uu = 4.0 * eps * (sr12 - sr6);
    if (shift) {
        double sc2 = sig * sig / (rc * rc);
        double sc6 = sc2 * sc2 * sc2;
        uu -= 4.0 * eps * (sc6 * sc6 - sc6);
    }
    *u = uu;
    *fr = (48.0 * eps * sr12 - 24.0 * eps * sr6) / r2;
    return 1;
}

/* -------------------------------------------------------------- pair sets */

/* All unordered pairs i < j with minimum-image distance^2 < rcut^2, by
 * testing every pair.  Writes at most cap pairs; returns the true count. */
EXPORT int64_t orc_pairs_brute(int32_t n, const double *x, const double *y,
                               const double *z, const double *L, double rcut,
                               int32_t *pi, int32_t *pj, int64_t cap)
{
    int64_t cnt = 0;
    double dx, dy, dz;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            if (dist2(x, y, z, L, i, j, &dx, &dy, &dz) < rcut * rcut) {
                if (cnt < cap) { pi[cnt] = i; pj[cnt] = j; }
                ++cnt;
            }
    return cnt;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

static int32_t cell_coord(double w, double L, int32_t nc)
{
    int32_t c = (int32_t)floor(w * nc / L);
    if (c < 0) c = 0;
    if (c > nc - 1) c = nc - 1;
    return c;
}

/* Same pair set through a cell list (Sec. 2.1.2): cubic-ish cells of edge
 * L_d / floor(L_d / rcut) >= rcut, search of the atom's own cell and its 26
 * neighbours (each distinct cell once when a dimension has fewer than three
 * cells).  Output is sorted like orc_pairs_brute.  Returns -1 when the box is
 * too small for a unique minimum image (rcut >= L_d / 2), -2 on allocation
 * failure. */
EXPORT int64_t orc_pairs_cells(int32_t n, const double *x, const double *y,
                               const double *z, const double *L, double rcut,
                               int32_t *pi, int32_t *pj, int64_t cap)
{
    int32_t nc[3];
    for (int d = 0; d < 3; ++d) {
        if (!(rcut < 0.5 * L[d])) return -1;
        nc[d] = (int32_t)floor(L[d] / rcut);
        if (nc[d] < 1) nc[d] = 1;
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *head = malloc(sizeof(int32_t) * ncell);
    int32_t *next = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *cid = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *js = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!head || !next || !cid || !js) {
        free(head); free(next); free(cid); free(js);
        return -2;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    /* bin (insert in descending index so each chain is ascending) */
    for (int32_t i = n - 1; i >= 0; --i) {
        const double p[3] = {x[i], y[i], z[i]};
        int32_t c3[3];
        for (int d = 0; d < 3; ++d) {
            double w = p[d] - L[d] * floor(p[d] / L[d]);
            if (w >= L[d]) w -= L[d];
            c3[d] = cell_coord(w, L[d], nc[d]);
        }
        int32_t c = (c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
        cid[i] = c;
        next[i] = head[c];
        head[c] = i;
    }
    int64_t cnt = 0;
#ifdef ORC_OMP
    /* each thread searches a contiguous block of i into its own buffer; the
     * buffers are concatenated in thread order, i.e. in the serial order */
    int nth = omp_get_max_threads();
    int32_t **bufi = calloc((size_t)nth, sizeof(int32_t *));
    int32_t **bufj = calloc((size_t)nth, sizeof(int32_t *));
    int64_t *bufn = calloc((size_t)nth, sizeof(int64_t));
    int bad = !bufi || !bufj || !bufn;
#pragma omp parallel num_threads(nth) reduction(| : bad)
    {
        int th = omp_get_thread_num();
        int32_t *js_t = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
        int64_t tcap = (int64_t)n * 48 / nth + 1024, tn = 0;
        int32_t *pi_t = malloc(sizeof(int32_t) * tcap), *pj_t = malloc(sizeof(int32_t) * tcap);
        double dx, dy, dz;
        if (!js_t || !pi_t || !pj_t) bad = 1;
#pragma omp for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            if (bad) continue;
            int32_t *js = js_t;
#else
    double dx, dy, dz;
    for (int32_t i = 0; i < n; ++i) {
#endif
        int32_t c = cid[i];
        int32_t cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
        int32_t seen[27], nseen = 0, nj = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int32_t ax = ((cx + ox) % nc[0] + nc[0]) % nc[0];
                    int32_t ay = ((cy + oy) % nc[1] + nc[1]) % nc[1];
                    int32_t az = ((cz + oz) % nc[2] + nc[2]) % nc[2];
                    int32_t nb = (az * nc[1] + ay) * nc[0] + ax;
                    int dup = 0;
                    for (int s = 0; s < nseen; ++s) dup |= (seen[s] == nb);
                    if (dup) continue;
                    seen[nseen++] = nb;
                    for (int32_t j = head[nb]; j >= 0; j = next[j])
                        if (j > i && dist2(x, y, z, L, i, j, &dx, &dy, &dz) < rcut * rcut)
                            js[nj++] = j;
                }
        qsort(js, (size_t)nj, sizeof(int32_t), cmp_i32);
#ifdef ORC_OMP
            if (tn + nj > tcap) {
                tcap = 2 * (tn + nj);
                int32_t *a = realloc(pi_t, sizeof(int32_t) * tcap);
                int32_t *b = a ? realloc(pj_t, sizeof(int32_t) * tcap) : NULL;
                if (a) pi_t = a;
                if (b) pj_t = b;
                if (!a || !b) { bad = 1; continue; }
            }
            for (int32_t k = 0; k < nj; ++k) { pi_t[tn] = i; pj_t[tn] = js[k]; ++tn; }
        }
        free(js_t);
        if (bufi && bufj && bufn) { bufi[th] = pi_t; bufj[th] = pj_t; bufn[th] = tn; }
        else { free(pi_t); free(pj_t); }
    }
    for (int t = 0; !bad && t < nth; ++t) {
        for (int64_t k = 0; k < bufn[t]; ++k, ++cnt)
            if (cnt < cap) { pi[cnt] = bufi[t][k]; pj[cnt] = bufj[t][k]; }
    }
    for (int t = 0; bufi && bufj && t < nth; ++t) { free(bufi[t]); free(bufj[t]); }
    free(bufi); free(bufj); free(bufn);
    free(head); free(next); free(cid); free(js);
    return bad ? -2 : cnt;
#else
        for (int32_t k = 0; k < nj; ++k) {
            if (cnt < cap) { pi[cnt] = i; pj[cnt] = js[k]; }
            ++cnt;
        }
    }
    free(head); free(next); free(cid); free(js);
    return cnt;
#endif
}

/* ----------------------------------------------------------------- forces */

/* Forces, potential energy and pair virial from an explicit pair set.
 * F_i += fr d, F_j -= fr d for each listed pair inside rc; E = sum U;
 * W = sum fr r^2 (so that P V = N T + W / 3).  Pairs are summed in list order. */
EXPORT void orc_lj_forces_pairs(int32_t n, const double *x, const double *y,
                                const double *z, const int32_t *type, int32_t nt,
                                const double *eps, const double *sig, const double *L,
                                double rc, int32_t shift, int64_t np,
                                const int32_t *pi, const int32_t *pj,
                                double *fx, double *fy, double *fz,
                                double *energy, double *virial)
{
    for (int32_t i = 0; i < n; ++i) fx[i] = fy[i] = fz[i] = 0.0;
#ifdef ORC_OMP
    /* per-thread force arrays over contiguous blocks of pairs, summed in
     * thread order */
    int nth = omp_get_max_threads();
    double *part = calloc((size_t)nth * 3 * (size_t)n, sizeof(double));
    if (part) {
        double e = 0.0, w = 0.0;
#pragma omp parallel num_threads(nth) reduction(+ : e, w)
        {
            double *ax = part + (size_t)omp_get_thread_num() * 3 * (size_t)n;
            double *ay = ax + n, *az = ay + n, dx, dy, dz, u, fr;
#pragma omp for schedule(static)
            for (int64_t p = 0; p < np; ++p) {
                int32_t i = pi[p], j = pj[p];
                int32_t t = type ? type[i] * nt + type[j] : 0;
                double r2 = dist2(x, y, z, L, i, j, &dx, &dy, &dz);
                if (!orc_lj_pair(r2, eps[t], sig[t], rc, shift, &u, &fr)) continue;
                ax[i] += fr * dx; ay[i] += fr * dy; az[i] += fr * dz;
                ax[j] -= fr * dx; ay[j] -= fr * dy; az[j] -= fr * dz;
                e += u;
                w += fr * r2;
            }
        }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            for (int t = 0; t < nth; ++t) {
                const double *a = part + (size_t)t * 3 * (size_t)n;
                fx[i] += a[i]; fy[i] += a[n + i]; fz[i] += a[2 * (size_t)n + i];
            }
        free(part);
        *energy = e;
        *virial = w;
        return;
    }
#endif
    double e = 0.0, w = 0.0, dx, dy, dz, u, fr;
    for (int64_t p = 0; p < np; ++p) {
        int32_t i = pi[p], j = pj[p];
        int32_t t = type ? type[i] * nt + type[j] : 0;
        double r2 = dist2(x, y, z, L, i, j, &dx, &dy, &dz);
        if (!orc_lj_pair(r2, eps[t], sig[t], rc, shift, &u, &fr)) continue;
        fx[i] += fr * dx; fy[i] += fr * dy; fz[i] += fr * dz;
        fx[j] -= fr * dx; fy[j] -= fr * dy; fz[j] -= fr * dz;
        e += u;
        w += fr * r2;
    }
    *energy = e;
    *virial = w;
}

/* The plainest definition: for each i, the sum over every j != i (ascending)
 * of the pair force inside rc.  E = (1/2) sum_i sum_j U, W likewise. */
EXPORT void orc_lj_forces_brute(int32_t n, const double *x, const double *y,
                                const double *z, const int32_t *type, int32_t nt,
                                const double *eps, const double *sig, const double *L,
                                double rc, int32_t shift,
                                double *fx, double *fy, double *fz,
                                double *energy, double *virial)
{
    double e = 0.0, w = 0.0, dx, dy, dz, u, fr;
    for (int32_t i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            int32_t t = type ? type[i] * nt + type[j] : 0;
            double r2 = dist2(x, y, z, L, i, j, &dx, &dy, &dz);
            if (!orc_lj_pair(r2, eps[t], sig[t], rc, shift, &u, &fr)) continue;
            ax += fr * dx; ay += fr * dy; az += fr * dz;
            e += 0.5 * u;
            w += 0.5 * fr * r2;
        }
        fx[i] = ax; fy[i] = ay; fz[i] = az;
    }
    *energy = e;
    *virial = w;
}

/* Force on one atom i by a loop over all j (for sampled checks of large
 * systems), with i's half share of the pair energy and virial. */
EXPORT void orc_lj_force_one(int32_t i, int32_t n, const double *x, const double *y,
                             const double *z, const int32_t *type, int32_t nt,
                             const double *eps, const double *sig, const double *L,
                             double rc, int32_t shift, double *f3,
                             double *e_half, double *w_half)
{
    double ax = 0.0, ay = 0.0, az = 0.0, e = 0.0, w = 0.0, dx, dy, dz, u, fr;
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        int32_t t = type ? type[i] * nt + type[j] : 0;
        double r2 = dist2(x, y, z, L, i, j, &dx, &dy, &dz);
        if (!orc_lj_pair(r2, eps[t], sig[t], rc, shift, &u, &fr)) continue;
        ax += fr * dx; ay += fr * dy; az += fr * dz;
        e += 0.5 * u;
        w += 0.5 * fr * r2;
    }
    f3[0] = ax; f3[1] = ay; f3[2] = az;
    *e_half = e;
    *w_half = w;
}

/* Pair set within rc through the cell list, then forces from it.
 * Returns the number of pairs inside rc, or a negative error. */
EXPORT int64_t orc_lj_forces(int32_t n, const double *x, const double *y,
                             const double *z, const int32_t *type, int32_t nt,
                             const double *eps, const double *sig, const double *L,
                             double rc, int32_t shift, double *fx, double *fy,
                             double *fz, double *energy, double *virial)
{
    int64_t cap = (int64_t)n * 64 + 64;
    for (;;) {
        int32_t *pi = malloc(sizeof(int32_t) * cap);
        int32_t *pj = malloc(sizeof(int32_t) * cap);
        if (!pi || !pj) { free(pi); free(pj); return -2; }
        int64_t np = orc_pairs_cells(n, x, y, z, L, rc, pi, pj, cap);
        if (np < 0) { free(pi); free(pj); return np; }
        if (np <= cap) {
            orc_lj_forces_pairs(n, x, y, z, type, nt, eps, sig, L, rc, shift, np,
                                pi, pj, fx, fy, fz, energy, virial);
            free(pi); free(pj);
            return np;
        }
        free(pi); free(pj);
        cap = np;
    }
}

/* ------------------------------------------------------ vector-Jacobian */

/* Gradient of L(F, E) given G = dL/dF (per atom) and gE = dL/dE, with
 * respect to positions and to the (eps, sigma) tables.  From Eq. lj:
 *   fr    = 48 eps sig^12 r^-14 - 24 eps sig^6 r^-8
 *   fr'/r = -672 eps sig^12 r^-16 + 192 eps sig^6 r^-10
 *   dfr/dsig = 576 eps sig^11 r^-14 - 144 eps sig^5 r^-8
 *   dU/dsig  = 48 eps sig^11 r^-12 - 24 eps sig^5 r^-6  (minus its value at rc
 *              when the energy is shifted)
 *   fr and U (shifted or not) are linear in eps.
 * For each pair with u = G_i - G_j and d = x_i - x_j:
 *   w = fr u + (fr'/r)(d.u) d - gE fr d,  gx_i += w, gx_j -= w
 *   geps += (d.u) fr/eps + gE U/eps,  gsig += (d.u) dfr/dsig + gE dU/dsig.
 * The (eps, sigma) gradients are with respect to the shared parameter of an
 * unordered type pair: both mirrored table entries receive the full value. */
EXPORT void orc_lj_vjp_pairs(int32_t n, const double *x, const double *y,
                             const double *z, const int32_t *type, int32_t nt,
                             const double *eps, const double *sig, const double *L,
                             double rc, int32_t shift, int64_t np,
                             const int32_t *pi, const int32_t *pj,
                             const double *gfx, const double *gfy, const double *gfz,
                             double ge, double *gx, double *gy, double *gz,
                             double *geps, double *gsig)
{
    for (int32_t i = 0; i < n; ++i) gx[i] = gy[i] = gz[i] = 0.0;
    for (int32_t t = 0; t < nt * nt; ++t) geps[t] = gsig[t] = 0.0;
    double dx, dy, dz;
    for (int64_t p = 0; p < np; ++p) {
        int32_t i = pi[p], j = pj[p];
        int32_t a = type ? type[i] : 0, b = type ? type[j] : 0;
        int32_t lo = a < b ? a : b, hi = a < b ? b : a;
        int32_t t = a * nt + b;
        double r2 = dist2(x, y, z, L, i, j, &dx, &dy, &dz);
        if (!(r2 < rc * rc)) continue;
        double e = eps[t], s = sig[t];
        double sr2 = s * s / r2, sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
        double fr = (48.0 * e * sr12 - 24.0 * e * sr6) / r2;
        double dfr_r = (-672.0 * e * sr12 + 192.0 * e * sr6) / (r2 * r2);
        double u = 4.0 * e * (sr12 - sr6);
        double du_ds = (48.0 * e * sr12 - 24.0 * e * sr6) / s;
        if (shift) {
            double sc2 = s * s / (rc * rc), sc6 = sc2 * sc2 * sc2, sc12 = sc6 * sc6;
            u -= 4.0 * e * (sc12 - sc6);
            du_ds -= (48.0 * e * sc12 - 24.0 * e * sc6) / s;
        }
        double dfr_ds = (576.0 * e * sr12 - 144.0 * e * sr6) / (s * r2);
        double ux = gfx[i] - gfx[j], uy = gfy[i] - gfy[j], uz = gfz[i] - gfz[j];
        double du = dx * ux + dy * uy + dz * uz;
        double wx = fr * ux + dfr_r * du * dx - ge * fr * dx;
        double wy = fr * uy + dfr_r * du * dy - ge * fr * dy;
        double wz = fr * uz + dfr_r * du * dz - ge * fr * dz;
        gx[i] += wx; gy[i] += wy; gz[i] += wz;
        gx[j] -= wx; gy[j] -= wy; gz[j] -= wz;
        geps[lo * nt + hi] += du * fr / e + ge * u / e;
        gsig[lo * nt + hi] += du * dfr_ds + ge * du_ds;
    }
    for (int32_t a = 0; a < nt; ++a)
        for (int32_t b = a + 1; b < nt; ++b) {
            geps[b * nt + a] = geps[a * nt + b];
            gsig[b * nt + a] = gsig[a * nt + b];
        }
}

/* ------------------------------------------------------- velocity Verlet */

/* NVE velocity Verlet (Sec. 2.1, Fig. 1):
 *   Integrate1: v += dt/2 F/m; x += dt v
 *   re-binning test: rebuild when max_i |x_i - x_i(last build)| > skin/2
 *   forces from the current positions
 *   Integrate2: v += dt/2 F/m
 * Forces always come from the exact pair set inside rc (via the cell list),
 * so they do not depend on the rebuild schedule, which is only recorded:
 * rebuild[s] = 1 when the test fires at step s (x_build is then reset).
 * Positions are never wrapped.  Per step s (1..steps) records the potential
 * energy, the kinetic energy after Integrate2 and the virial; index 0 holds
 * the initial state.  Returns 0, or a negative error from the pair search. */
EXPORT int32_t orc_md_run(int32_t n, double *x, double *y, double *z,
                          double *vx, double *vy, double *vz,
                          const int32_t *type, int32_t nt, const double *mass,
                          const double *eps, const double *sig, const double *L,
                          double rc, int32_t shift, double skin, double dt,
                          int32_t steps, uint8_t *rebuild, double *epot,
                          double *ekin, double *vir,
                          double *fx, double *fy, double *fz)
{
    double *xb = malloc(sizeof(double) * n), *yb = malloc(sizeof(double) * n),
           *zb = malloc(sizeof(double) * n);
    if (!xb || !yb || !zb) { free(xb); free(yb); free(zb); return -2; }
    memcpy(xb, x, sizeof(double) * n);
    memcpy(yb, y, sizeof(double) * n);
    memcpy(zb, z, sizeof(double) * n);
    double e, w;
    int64_t rcode = orc_lj_forces(n, x, y, z, type, nt, eps, sig, L, rc, shift,
                                  fx, fy, fz, &e, &w);
    if (rcode < 0) { free(xb); free(yb); free(zb); return (int32_t)rcode; }
    double k = 0.0;
    ORC_PAR_FOR_SUM_K
    for (int32_t i = 0; i < n; ++i) {
        double m = mass[type ? type[i] : 0];
        k += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    }
    epot[0] = e; ekin[0] = k; vir[0] = w;
    const double lim2 = 0.25 * skin * skin;
    for (int32_t s = 0; s < steps; ++s) {
        ORC_PAR_FOR
        for (int32_t i = 0; i < n; ++i) {
            double im = 1.0 / mass[type ? type[i] : 0];
            vx[i] += 0.5 * dt * fx[i] * im;
            vy[i] += 0.5 * dt * fy[i] * im;
            vz[i] += 0.5 * dt * fz[i] * im;
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
        }
        double dmax = 0.0;
        ORC_PAR_FOR_MAX_DMAX
        for (int32_t i = 0; i < n; ++i) {
            double a = x[i] - xb[i], b = y[i] - yb[i], c = z[i] - zb[i];
            double d2 = a * a + b * b + c * c;
            if (d2 > dmax) dmax = d2;
        }
        rebuild[s] = (uint8_t)(dmax > lim2);
        if (rebuild[s]) {
            memcpy(xb, x, sizeof(double) * n);
            memcpy(yb, y, sizeof(double) * n);
            memcpy(zb, z, sizeof(double) * n);
        }
        rcode = orc_lj_forces(n, x, y, z, type, nt, eps, sig, L, rc, shift,
                              fx, fy, fz, &e, &w);
        if (rcode < 0) { free(xb); free(yb); free(zb); return (int32_t)rcode; }
        k = 0.0;
        ORC_PAR_FOR_SUM_K
        for (int32_t i = 0; i < n; ++i) {
            double m = mass[type ? type[i] : 0];
            double im = 1.0 / m;
            vx[i] += 0.5 * dt * fx[i] * im;
            vy[i] += 0.5 * dt * fy[i] * im;
            vz[i] += 0.5 * dt * fz[i] * im;
            k += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        }
        epot[s + 1] = e; ekin[s + 1] = k; vir[s + 1] = w;
    }
    free(xb); free(yb); free(zb);
    return 0;
}

/* ----------------------------------------------- counter-based generator */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011).  Each round multiplies words 0 and
 * 2 by the two round constants into 64-bit products and mixes the halves with
 * the other words and the key; the key is bumped by two Weyl constants
 * between rounds. */
EXPORT void orc_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in,
                              uint32_t *out)
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normal deviates for (seed, step, atom id): two Philox
 * blocks with counter (id, step_lo, step_hi, block) and key (seed_lo,
 * seed_hi); each pair of 32-bit words gives a 53-bit uniform in (0,1);
 * Box-Muller turns each pair of uniforms into two normals. */
EXPORT void orc_gauss3(uint64_t seed, uint64_t step, uint32_t id, double *g)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double z[4];
    for (uint32_t blk = 0; blk < 2; ++blk) {
        const uint32_t ctr[4] = {id, (uint32_t)step, (uint32_t)(step >> 32), blk};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        uint64_t a = ((((uint64_t)o[0]) << 32) | o[1]) >> 11;
        uint64_t b = ((((uint64_t)o[2]) << 32) | o[3]) >> 11;
        double u1 = ((double)a + 0.5) * 0x1p-53;
        double u2 = ((double)b + 0.5) * 0x1p-53;
        double rr = sqrt(-2.0 * log(u1));
        const double two_pi = 6.283185307179586476925286766559;
        z[2 * blk] = rr * cos(two_pi * u2);
        z[2 * blk + 1] = rr * sin(two_pi * u2);
    }
    g[0] = z[0]; g[1] = z[1]; g[2] = z[2];
}

/* Langevin thermostat in force form: F_i += -gamma m_i v_i +
 * sqrt(2 gamma m_i T / dt) xi_i with xi_i from orc_gauss3(seed, step, id_i). */
EXPORT void orc_langevin(int32_t n, const double *vx, const double *vy,
                         const double *vz, const int32_t *type, const double *mass,
                         const int32_t *id, double gamma, double temperature,
                         double dt, uint64_t seed, uint64_t step,
                         double *fx, double *fy, double *fz)
{
    for (int32_t i = 0; i < n; ++i) {
        double m = mass[type ? type[i] : 0];
        double amp = sqrt(2.0 * gamma * m * temperature / dt);
        double g[3];
        orc_gauss3(seed, step, (uint32_t)id[i], g);
        fx[i] += -gamma * m * vx[i] + amp * g[0];
        fy[i] += -gamma * m * vy[i] + amp * g[1];
        fz[i] += -gamma * m * vz[i] + amp * g[2];
    }
}

/* --------------------------------------------------------------- FENE bonds */

/* FENE bond U(r) = -(1/2) K R0^2 ln(1 - r^2/R0^2), fr = -K / (1 - r^2/R0^2).
 * Returns 0 when r >= R0 (bond broken; U and fr are then left at 0). */
EXPORT int orc_fene_pair(double r2, double K, double R0, double *u, double *fr)
{
    double q = 1.0 - r2 / (R0 * R0);
    *u = 0.0;
    *fr = 0.0;
    if (!(q > 0.0)) return 0;
    *u = -0.5 * K * R0 * R0 * log(q);
    *fr = -K / q;
    return 1;
}

/* Adds FENE forces for bonds (bi[b], bj[b]) given as atom indices; returns
 * the number of broken bonds; adds the bond energy and virial. */
EXPORT int64_t orc_fene_forces(int32_t n, const double *x, const double *y,
                               const double *z, const double *L, int64_t nb,
                               const int32_t *bi, const int32_t *bj, double K,
                               double R0, double *fx, double *fy, double *fz,
                               double *energy, double *virial)
{
    (void)n;
    int64_t broken = 0;
    double e = 0.0, w = 0.0, dx, dy, dz, u, fr;
    for (int64_t b = 0; b < nb; ++b) {
        int32_t i = bi[b], j = bj[b];
        double r2 = dist2(x, y, z, L, i, j, &dx, &dy, &dz);
        if (!orc_fene_pair(r2, K, R0, &u, &fr)) { ++broken; continue; }
        fx[i] += fr * dx; fy[i] += fr * dy; fz[i] += fr * dz;
        fx[j] -= fr * dx; fy[j] -= fr * dy; fz[j] -= fr * dz;
        e += u;
        w += fr * r2;
    }
    *energy += e;
    *virial += w;
    return broken;
}

/* ------------------------------------------------------ cosine angle term */

/* Angle term of the ring-polymer melt (Sec. 4, setup: a cosine potential on
 * the triples of consecutive beads).  For the triple (a, b, c) with middle
 * bead b, d1 = x_a - x_b and d2 = x_c - x_b (minimum image),
 *     cos t = d1.d2 / (|d1| |d2|),   U = K (1 + cos t),
 * so a straight triple (t = pi) costs nothing.  The forces are -grad U:
 *     dcos/dx_a = d2 / (|d1| |d2|) - cos t d1 / |d1|^2,   F_a = -K dcos/dx_a,
 *     dcos/dx_c = d1 / (|d1| |d2|) - cos t d2 / |d2|^2,   F_c = -K dcos/dx_c,
 *     F_b = -F_a - F_c.
 * Returns 0 (U and the forces left at 0) when a bond vector has zero length. */
EXPORT int orc_angle_triple(const double *d1, const double *d2, double K, double *u,
                            double *fa, double *fc)
{
    double r11 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    double r22 = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
    *u = 0.0;
    for (int k = 0; k < 3; ++k) fa[k] = fc[k] = 0.0;
    if (!(r11 > 0.0) || !(r22 > 0.0)) return 0;
    double r1 = sqrt(r11), r2 = sqrt(r22);
    double c = (d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2]) / (r1 * r2);
    *u = K * (1.0 + c);
    for (int k = 0; k < 3; ++k) {
        fa[k] = -K * (d2[k] / (r1 * r2) - c * d1[k] / r11);
        fc[k] = -K * (d1[k] / (r1 * r2) - c * d2[k] / r22);
    }
    return 1;
}

/* Adds the angle forces of the triples (ia[t], ib[t], ic[t]) (atom indices,
 * ib the middle bead); adds their energy and virial (sum over the triple of
 * x . F, i.e. d1.F_a + d2.F_c); returns the number of degenerate triples. */
EXPORT int64_t orc_angle_forces(int32_t n, const double *x, const double *y,
                                const double *z, const double *L, int64_t na,
                                const int32_t *ia, const int32_t *ib, const int32_t *ic,
                                double K, double *fx, double *fy, double *fz,
                                double *energy, double *virial)
{
    (void)n;
    int64_t bad = 0;
    double e = 0.0, w = 0.0, d1[3], d2[3], fa[3], fc[3], u;
    for (int64_t t = 0; t < na; ++t) {
        int32_t a = ia[t], b = ib[t], c = ic[t];
        dist2(x, y, z, L, a, b, &d1[0], &d1[1], &d1[2]);
        dist2(x, y, z, L, c, b, &d2[0], &d2[1], &d2[2]);
        if (!orc_angle_triple(d1, d2, K, &u, fa, fc)) { ++bad; continue; }
        fx[a] += fa[0]; fy[a] += fa[1]; fz[a] += fa[2];
        fx[c] += fc[0]; fy[c] += fc[1]; fz[c] += fc[2];
        fx[b] -= fa[0] + fc[0]; fy[b] -= fa[1] + fc[1]; fz[b] -= fa[2] + fc[2];
        e += u;
        w += d1[0] * fa[0] + d1[1] * fa[1] + d1[2] * fa[2] +
             d2[0] * fc[0] + d2[1] * fc[1] + d2[2] * fc[2];
    }
    *energy += e;
    *virial += w;
    return bad;
}

/* ------------------------------------------- MD with bonds and a thermostat */

static int64_t total_forces(int32_t n, const double *x, const double *y, const double *z,
                            const double *vx, const double *vy, const double *vz,
                            const int32_t *type, int32_t nt, const double *mass,
                            const double *eps, const double *sig, const double *L,
                            double rc, int32_t shift, int64_t nb, const int32_t *bi,
                            const int32_t *bj, double K, double R0, int64_t na,
                            const int32_t *ia, const int32_t *ib, const int32_t *ic,
                            double Ka, double gamma,
                            double temperature, double dt, uint64_t seed, uint64_t step,
                            const int32_t *ids, double *fx, double *fy, double *fz,
                            double *energy, int64_t *broken)
{
    double e, w;
    int64_t np = orc_lj_forces(n, x, y, z, type, nt, eps, sig, L, rc, shift, fx, fy, fz, &e, &w);
    if (np < 0) return np;
    if (nb > 0) *broken += orc_fene_forces(n, x, y, z, L, nb, bi, bj, K, R0, fx, fy, fz, &e, &w);
    if (na > 0) *broken += orc_angle_forces(n, x, y, z, L, na, ia, ib, ic, Ka, fx, fy, fz, &e, &w);
    if (gamma > 0.0)
        orc_langevin(n, vx, vy, vz, type, mass, ids, gamma, temperature, dt, seed, step,
                     fx, fy, fz);
    *energy = e;
    return 0;
}

/* Velocity Verlet (Sec. 2.1, Fig. 1) with LJ pair forces, optional FENE bonds
 * (pairs bi[b]-bj[b] of atom indices, the polymer melt of Sec. 4), optional
 * cosine angle terms on triples ia[t]-ib[t]-ic[t] (the ring melt) and an
 * optional Langevin thermostat (Sec. 4: equilibration to a target T).  The
 * thermostat force is evaluated with the velocity at the time of the force
 * evaluation (after Integrate1) and noise counter step0 for the initial force
 * evaluation, step0 + 1 + s for step s; atom ids are the indices.  Records the
 * rebuild test like orc_md_run, the potential energy (LJ + FENE + angle) and
 * the kinetic energy.  Returns the number of broken-bond and degenerate-angle
 * events (>= 0), or a negative error. */
EXPORT int64_t orc_md_run_ext(int32_t n, double *x, double *y, double *z, double *vx,
                              double *vy, double *vz, const int32_t *type, int32_t nt,
                              const double *mass, const double *eps, const double *sig,
                              const double *L, double rc, int32_t shift, double skin,
                              double dt, int32_t steps, int64_t nb, const int32_t *bi,
                              const int32_t *bj, double K, double R0, int64_t na,
                              const int32_t *ia, const int32_t *ib, const int32_t *ic,
                              double Ka, double gamma,
                              double temperature, uint64_t seed, uint64_t step0,
                              uint8_t *rebuild, double *epot, double *ekin,
                              double *fx, double *fy, double *fz)
{
    double *xb = malloc(sizeof(double) * n), *yb = malloc(sizeof(double) * n),
           *zb = malloc(sizeof(double) * n);
    int32_t *ids = calloc((size_t)n + 1, sizeof(int32_t));
    if (!xb || !yb || !zb || !ids) { free(xb); free(yb); free(zb); free(ids); return -2; }
    for (int32_t i = 0; i < n; ++i) ids[i] = i;
    memcpy(xb, x, sizeof(double) * n);
    memcpy(yb, y, sizeof(double) * n);
    memcpy(zb, z, sizeof(double) * n);
    int64_t broken = 0, rc_ = 0;
    double e = 0.0;
    rc_ = total_forces(n, x, y, z, vx, vy, vz, type, nt, mass, eps, sig, L, rc, shift, nb, bi,
                       bj, K, R0, na, ia, ib, ic, Ka, gamma, temperature, dt, seed, step0, ids,
                       fx, fy, fz, &e, &broken);
    double k = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double m = mass[type ? type[i] : 0];
        k += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    }
    if (rc_ < 0) goto done;
    epot[0] = e; ekin[0] = k;
    const double lim2 = 0.25 * skin * skin;
    for (int32_t s = 0; s < steps; ++s) {
        for (int32_t i = 0; i < n; ++i) {
            double im = 1.0 / mass[type ? type[i] : 0];
            vx[i] += 0.5 * dt * fx[i] * im;
            vy[i] += 0.5 * dt * fy[i] * im;
            vz[i] += 0.5 * dt * fz[i] * im;
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
        }
        double dmax = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            double a = x[i] - xb[i], b = y[i] - yb[i], c = z[i] - zb[i];
            double d2 = a * a + b * b + c * c;
            if (d2 > dmax) dmax = d2;
        }
        rebuild[s] = (uint8_t)(dmax > lim2);
        if (rebuild[s]) {
            memcpy(xb, x, sizeof(double) * n);
            memcpy(yb, y, sizeof(double) * n);
            memcpy(zb, z, sizeof(double) * n);
        }
        rc_ = total_forces(n, x, y, z, vx, vy, vz, type, nt, mass, eps, sig, L, rc, shift, nb,
                           bi, bj, K, R0, na, ia, ib, ic, Ka, gamma, temperature, dt, seed,
                           step0 + 1 + (uint64_t)s, ids, fx, fy, fz, &e, &broken);
        if (rc_ < 0) goto done;
        k = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            double m = mass[type ? type[i] : 0];
            double im = 1.0 / m;
            vx[i] += 0.5 * dt * fx[i] * im;
            vy[i] += 0.5 * dt * fy[i] * im;
            vz[i] += 0.5 * dt * fz[i] * im;
            k += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        }
        epot[s + 1] = e; ekin[s + 1] = k;
    }
done:
    free(xb); free(yb); free(zb); free(ids);
    return rc_ < 0 ? rc_ : broken;
}
