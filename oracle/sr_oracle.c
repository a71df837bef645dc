/*
 * Plain float64 CPU oracle for the short-range particle-particle force of the
 * split-force N-body method (Habib et al. 2012, "The Universe at Extreme
 * Scale", Sec. III, Eq. 7, and the cut-off paragraph that follows it).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library uses, links or
 * includes this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg call it.  It shares no code with the HIP path.
 *
 * What it computes, for every requested target particle i:
 *
 *   a_i = sum_{j != i, s_ij < r_cut^2} m_j f(s_ij) d_ij
 *   d_ij = x_j - x_i          (minimum image when the box is periodic)
 *   s_ij = d_ij . d_ij
 *   f(s) = (s + eps)^(-3/2) - sum_{k=0..5} c_k s^k
 *
 * Eq. 7 gives f_SR(s) = (s+eps)^(-3/2) - f_grid(s) with f_grid = poly[5](s);
 * the text after it applies the short-range condition inside the kernel.
 * Readings taken where the paper is silent: G = 1, attractive sign with
 * d_ij = x_j - x_i, strict s < r_cut^2 with r_cut^2 formed in float64 from
 * the float32 r_cut, and a self pair contributes nothing.
 *
 * It also computes A_i = sum_j m_j (s+eps)^(-3/2) |d_ij| (the summed
 * Newtonian pair magnitude used to floor relative errors) and the
 * vector-Jacobian product of the accelerations with respect to positions,
 *
 *   dL/dx_k = sum_j K_kj (m_k g_j - m_j g_k),   K = f(s) I + 2 f'(s) d d^T,
 *   f'(s)   = -(3/2)(s + eps)^(-5/2) - sum_k k c_k s^(k-1),
 *
 * for L = sum_i g_i . a_i, which follows from differentiating the pair term
 * m_j f(s) d of Eq. 7 with respect to both end points.
 *
 * Neighbour search is a plain linked-list cell grid with cells no smaller
 * than r_cut, so every pair inside the cut-off lies in adjacent cells.
 * Everything is float64; the polynomial is evaluated by Horner in s on the
 * float32 coefficient values.  Targets are spread over OpenMP threads; each
 * target's sum runs in one thread, so results do not depend on the thread
 * count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int periodic;
    double box;
    double lo[3];
    double side[3];
    int64_t nc[3];
    int64_t ncell;
    int64_t *head;   /* first particle of each cell, -1 if empty */
    int64_t *next;   /* next particle in the same cell */
} cellgrid;

static int64_t clamp_i64(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

static void cell_of(const cellgrid *g, const double *x, int64_t c[3]) {
    for (int a = 0; a < 3; ++a) {
        double v = x[a];
        if (g->periodic) v = v - g->box * floor(v / g->box);
        int64_t k = (int64_t)floor((v - g->lo[a]) / g->side[a]);
        c[a] = clamp_i64(k, 0, g->nc[a] - 1);
    }
}

static int build_grid(cellgrid *g, const double *pos, int64_t n, double box,
                      double rc) {
    memset(g, 0, sizeof(*g));
    g->periodic = box > 0.0;
    g->box = box;
    for (int a = 0; a < 3; ++a) {
        double lo = 0.0, hi = box;
        if (!g->periodic) {
            lo = INFINITY;
            hi = -INFINITY;
            for (int64_t i = 0; i < n; ++i) {
                if (pos[3 * i + a] < lo) lo = pos[3 * i + a];
                if (pos[3 * i + a] > hi) hi = pos[3 * i + a];
            }
            if (n == 0) { lo = 0.0; hi = 1.0; }
        }
        double ext = hi - lo;
        int64_t k = (int64_t)floor(ext / rc);
        if (k < 1) k = 1;
        if (k > 1024) k = 1024;
        g->lo[a] = lo;
        g->nc[a] = k;
        g->side[a] = ext > 0.0 ? ext / (double)k : 1.0;
        /* The cell side must not be smaller than r_cut. */
        if (g->side[a] < rc && k > 1) {
            g->nc[a] = k - 1;
            g->side[a] = ext / (double)(k - 1);
        }
    }
    g->ncell = g->nc[0] * g->nc[1] * g->nc[2];
    g->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->ncell);
    g->next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!g->head || !g->next) return -1;
    for (int64_t c = 0; c < g->ncell; ++c) g->head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t c[3];
        cell_of(g, pos + 3 * i, c);
        int64_t id = (c[0] * g->nc[1] + c[1]) * g->nc[2] + c[2];
        g->next[i] = g->head[id];
        g->head[id] = i;
    }
    return 0;
}

static void free_grid(cellgrid *g) {
    free(g->head);
    free(g->next);
}

/* The distinct neighbour cell indices along one axis (1 to 3 of them). */
static int axis_neighbours(const cellgrid *g, int a, int64_t c, int64_t out[3]) {
    int m = 0;
    for (int o = -1; o <= 1; ++o) {
        int64_t k = c + o;
        if (g->periodic) {
            k = ((k % g->nc[a]) + g->nc[a]) % g->nc[a];
        } else if (k < 0 || k >= g->nc[a]) {
            continue;
        }
        int dup = 0;
        for (int q = 0; q < m; ++q) dup |= (out[q] == k);
        if (!dup) out[m++] = k;
    }
    return m;
}

static double horner(const double c[6], double s) {
    double p = c[5];
    for (int k = 4; k >= 0; --k) p = p * s + c[k];
    return p;
}

static double horner_deriv(const double c[6], double s) {
    double p = 5.0 * c[5];
    for (int k = 4; k >= 1; --k) p = p * s + (double)k * c[k];
    return p;
}

static void min_image(double d[3], int periodic, double box) {
    if (!periodic) return;
    for (int a = 0; a < 3; ++a) d[a] -= box * nearbyint(d[a] / box);
}

/* The distinct cells adjacent to (and including) the cell of point x. */
static int neighbour_cells(const cellgrid *g, const double *x, int64_t ids[27]) {
    int64_t ci[3], nx[3], ny[3], nz[3];
    cell_of(g, x, ci);
    int mx = axis_neighbours(g, 0, ci[0], nx);
    int my = axis_neighbours(g, 1, ci[1], ny);
    int mz = axis_neighbours(g, 2, ci[2], nz);
    int m = 0;
    for (int a = 0; a < mx; ++a)
        for (int b = 0; b < my; ++b)
            for (int c = 0; c < mz; ++c)
                ids[m++] = (nx[a] * g->nc[1] + ny[b]) * g->nc[2] + nz[c];
    return m;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Accelerations for `nt` targets (all particles when targets == NULL).
 * acc: (nt,3) float64.  anewt (may be NULL): (nt,) summed Newtonian pair
 * magnitude.  npairs (may be NULL): (nt,) number of in-cut-off neighbours.
 * Returns 0, or -1 when memory runs out.
 */
int oracle_force(const double *pos, const float *mass, int64_t n, double box,
                 float r_cut, float eps, const float poly[6],
                 const int64_t *targets, int64_t nt, double *acc,
                 double *anewt, int64_t *npairs) {
    cellgrid g;
    double c[6];
    for (int k = 0; k < 6; ++k) c[k] = (double)poly[k];
    const double rc = (double)r_cut, rc2 = rc * rc, e = (double)eps;
    if (targets == NULL) nt = n;
    if (build_grid(&g, pos, n, box, rc) != 0) { free_grid(&g); return -1; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        double a[3] = {0.0, 0.0, 0.0}, an = 0.0;
        int64_t cnt = 0;
        int64_t cells[27];
        const int ncells = neighbour_cells(&g, pos + 3 * i, cells);
        for (int q = 0; q < ncells; ++q)
        for (int64_t j = g.head[cells[q]]; j >= 0; j = g.next[j]) {
            if (j == i) continue;
            double d[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1],
                           pos[3 * j + 2] - pos[3 * i + 2]};
            min_image(d, g.periodic, box);
            const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (s < rc2) {
                const double newt = 1.0 / ((s + e) * sqrt(s + e));
                const double f = newt - horner(c, s);
                const double mj = (double)mass[j];
                a[0] += mj * f * d[0];
                a[1] += mj * f * d[1];
                a[2] += mj * f * d[2];
                an += mj * newt * sqrt(s);
                ++cnt;
            }
        }
        acc[3 * t] = a[0];
        acc[3 * t + 1] = a[1];
        acc[3 * t + 2] = a[2];
        if (anewt) anewt[t] = an;
        if (npairs) npairs[t] = cnt;
    }
    free_grid(&g);
    return 0;
}

/*
 * Vector-Jacobian product dL/dx_k for L = sum_i g_i . a_i, for `nt` targets
 * k (all when targets == NULL).  g: (n,3) float64 cotangents.  out: (nt,3)
 * float64.  bnorm (may be NULL): (nt,) sum_j (N + |p| + 2 s (1.5 N / (s + eps)
 * + |p'|)) |w_kj|, N = (s + eps)^(-3/2), p the grid polynomial: the summed
 * magnitudes of the parts of f and f' before the polynomial cancels the
 * Newtonian term, the scale used to floor relative errors (the analogue for
 * the VJP of the Newtonian magnitude that floors force errors).
 *
 * pmag (may be NULL): (nt,) sum_j (|f| + 2 |f'| s) |w_kj| over the in-cut-off
 * pairs, the summed magnitudes of the pair terms' two parts f w and
 * 2 f' (d.w) d bounded through |d.w| <= |d||w| (a second, tighter floor).
 *
 * f' jumps at the cut-off (f itself is continuous there), so the VJP is
 * discontinuous wherever a pair sits on r_cut: an implementation that takes
 * the cut-off test in a lower precision may count such a pair on the other
 * side.  amb (may be NULL): (nt,) the summed magnitude (|f| + 2|f'| s)|w| of
 * the pairs with |s - r_cut^2| <= cut_band * r_cut^2, a bound on how far any
 * decision for those pairs can move the result.
 */
int oracle_force_vjp(const double *pos, const float *mass, int64_t n,
                     double box, float r_cut, float eps, const float poly[6],
                     const double *gvec, const int64_t *targets, int64_t nt,
                     double *out, double *bnorm, double *pmag,
                     double cut_band, double *amb) {
    cellgrid g;
    double c[6];
    for (int k = 0; k < 6; ++k) c[k] = (double)poly[k];
    const double rc = (double)r_cut, rc2 = rc * rc, e = (double)eps;
    if (targets == NULL) nt = n;
    if (build_grid(&g, pos, n, box, rc) != 0) { free_grid(&g); return -1; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t k = targets ? targets[t] : t;
        double o[3] = {0.0, 0.0, 0.0}, b = 0.0, pm = 0.0, am = 0.0;
        const double mk = (double)mass[k];
        const double gk[3] = {gvec[3 * k], gvec[3 * k + 1], gvec[3 * k + 2]};
        int64_t cells[27];
        const int ncells = neighbour_cells(&g, pos + 3 * k, cells);
        for (int q = 0; q < ncells; ++q)
        for (int64_t j = g.head[cells[q]]; j >= 0; j = g.next[j]) {
            if (j == k) continue;
            double d[3] = {pos[3 * j] - pos[3 * k], pos[3 * j + 1] - pos[3 * k + 1],
                           pos[3 * j + 2] - pos[3 * k + 2]};
            min_image(d, g.periodic, box);
            const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const int edge = fabs(s - rc2) <= cut_band * rc2;
            if (s < rc2 || edge) {
                const double se = s + e;
                const double newt = 1.0 / (se * sqrt(se));
                const double pv = horner(c, s), dpv = horner_deriv(c, s);
                const double f = newt - pv;
                const double fp = -1.5 * newt / se - dpv;
                const double mj = (double)mass[j];
                double w[3];
                for (int r = 0; r < 3; ++r)
                    w[r] = mk * gvec[3 * j + r] - mj * gk[r];
                const double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
                const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
                const double mag = (fabs(f) + 2.0 * fabs(fp) * s) * wn;
                if (edge) am += mag;
                if (s < rc2) {
                    for (int r = 0; r < 3; ++r) o[r] += f * w[r] + 2.0 * fp * dw * d[r];
                    b += (newt + fabs(pv) + 2.0 * s * (1.5 * newt / se + fabs(dpv))) * wn;
                    pm += mag;
                }
            }
        }
        out[3 * t] = o[0];
        out[3 * t + 1] = o[1];
        out[3 * t + 2] = o[2];
        if (bnorm) bnorm[t] = b;
        if (pmag) pmag[t] = pm;
        if (amb) amb[t] = am;
    }
    free_grid(&g);
    return 0;
}
