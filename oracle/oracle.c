/*
 * oracle.c -- plain, slow FP64 CPU oracle for the continuous ("box") Gauss
 * transform of Greengard, Jiang, Rachh and Wang, "A new version of the
 * adaptive fast Gauss transform for discrete and continuous sources".
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU path, and it includes nothing of it.
 *
 * What it computes (Section 1, Eq. (bgt); leaf model of Eq. (papprox)):
 *
 *   u(x) = sum over leaves S of  int_S G(x - y; delta) s_S(y) dy,
 *
 * where s_S is the degree-(p-1)-per-axis Legendre interpolant of the samples
 * of sigma at the tensor Gauss-Legendre nodes of leaf S, and G is the free
 * space Gaussian exp(-|x|^2/delta) (Eq. (gkernel)) or its periodization over
 * Z^d (Eq. (gper_kernel)).  Targets are the tensor Gauss-Legendre nodes of
 * requested boxes: leaves of the source tree, or any other boxes (the boxes
 * of a refined or coarsened output tree, Section 4.2).
 *
 * How (each step is the plain definition, no fast method):
 *  1. Gauss-Legendre nodes/weights on [-1,1] by Newton's method on P_p.
 *  2. Legendre coefficients of every source leaf by the quadrature formula of
 *     Lemma polycost / Eq. (val2poleq), applied axis by axis.
 *  3. For a target leaf T and source leaf S, Lemma directbox: the integral
 *     factorizes into d one-dimensional integrals
 *        g_a[i][n] = int_{S_a} exp(-(x_{a,i} - y)^2/delta) P_n(2(y-c_{S,a})/L_S) dy
 *     and u_T += (g_1 (x) ... (x) g_d) c_S, evaluated axis by axis on the
 *     tensor grid (Remark dircost).  The 1D integrals are computed by adaptive
 *     20-point Gauss-Legendre quadrature (bisection until two successive
 *     estimates agree to 1e-15 of the integral's scale).  In periodic form the
 *     kernel factorizes per axis, so g_a is summed over the per-axis images.
 *  4. Source leaves farther than r_cut = sqrt(delta*ln(1e17)) on some axis
 *     (for every image) are skipped: each skipped term is below 1e-17 of the
 *     integral of |sigma|.
 *  A 1D integral depends only on the two leaf levels and the offset of the
 *  two centers along the axis, so identical integrals are computed once and
 *  reused (memoization; the sum itself is unchanged).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXP 32
#define OR_NQ 20

/* ---------------------------------------------------------------------- */
/* step 1: Gauss-Legendre rule (ascending nodes)                           */

static void or_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double p0 = 0.0, p1 = 0.0, dp = 1.0;
        for (int it = 0; it < 100; it++) {
            p0 = 1.0;
            p1 = 0.0;
            for (int j = 1; j <= n; j++) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        /* derivative at the converged root */
        p0 = 1.0;
        p1 = 0.0;
        for (int j = 1; j <= n; j++) {
            double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

/* P_0..P_{n-1} at t by the three-term recurrence */
static void or_legendre(int n, double t, double *P)
{
    P[0] = 1.0;
    if (n > 1) P[1] = t;
    for (int k = 2; k < n; k++)
        P[k] = ((2.0 * k - 1.0) * t * P[k - 1] - (k - 1.0) * P[k - 2]) / k;
}

/* ---------------------------------------------------------------------- */
/* step 2: Legendre coefficients of one leaf (axis-by-axis, Eq. (val2poleq)) */

static int64_t or_ipow(int p, int d)
{
    int64_t r = 1;
    for (int a = 0; a < d; a++) r *= p;
    return r;
}

/* out[... n_a ...] = sum_j M[n][j] in[... j ...] along axis a (axis 0 fastest) */
static void or_apply_axis(int p, int d, int a, const double *M, const double *in, double *out)
{
    int64_t inner = or_ipow(p, a), outer = or_ipow(p, d - 1 - a);
    for (int64_t o = 0; o < outer; o++)
        for (int n = 0; n < p; n++)
            for (int64_t i = 0; i < inner; i++) {
                double s = 0.0;
                for (int j = 0; j < p; j++)
                    s += M[n * p + j] * in[(o * p + j) * inner + i];
                out[(o * p + n) * inner + i] = s;
            }
}

static void or_coefficients(int p, int d, const double *eta, const double *wgl,
                            const double *vals, double *coef, double *tmp)
{
    double Q[OR_MAXP * OR_MAXP], P[OR_MAXP];
    for (int j = 0; j < p; j++) {
        or_legendre(p, eta[j], P);
        for (int n = 0; n < p; n++) Q[n * p + j] = 0.5 * (2 * n + 1) * wgl[j] * P[n];
    }
    int64_t np = or_ipow(p, d);
    memcpy(coef, vals, sizeof(double) * np);
    for (int a = 0; a < d; a++) {
        or_apply_axis(p, d, a, Q, coef, tmp);
        memcpy(coef, tmp, sizeof(double) * np);
    }
}

/* ---------------------------------------------------------------------- */
/* step 3: adaptive Gauss-Legendre for the 1D integrals                    */

typedef struct {
    int p;
    double xi;     /* target coordinate minus source center */
    double half;   /* L_S / 2 */
    double delta;
    double tol;
    const double *xq, *wq; /* 20-point rule */
} or_integrand;

/* out[n] = int_a^b exp(-(xi - half*t)^2/delta) P_n(t) dt, one 20-point panel */
static void or_panel(const or_integrand *f, double a, double b, double *out)
{
    double P[OR_MAXP];
    double m = 0.5 * (a + b), r = 0.5 * (b - a);
    for (int n = 0; n < f->p; n++) out[n] = 0.0;
    for (int q = 0; q < OR_NQ; q++) {
        double t = m + r * f->xq[q];
        double s = f->xi - f->half * t;
        double g = exp(-s * s / f->delta) * r * f->wq[q];
        or_legendre(f->p, t, P);
        for (int n = 0; n < f->p; n++) out[n] += g * P[n];
    }
}

static void or_adapt(const or_integrand *f, double a, double b, const double *whole,
                     int depth, double *acc)
{
    double left[OR_MAXP], right[OR_MAXP];
    double m = 0.5 * (a + b);
    or_panel(f, a, m, left);
    or_panel(f, m, b, right);
    double err = 0.0;
    for (int n = 0; n < f->p; n++) {
        double e = fabs(left[n] + right[n] - whole[n]);
        if (e > err) err = e;
    }
    if (err <= f->tol || depth >= 60) {
        for (int n = 0; n < f->p; n++) acc[n] += left[n] + right[n];
        return;
    }
    or_adapt(f, a, m, left, depth + 1, acc);
    or_adapt(f, m, b, right, depth + 1, acc);
}

/* g[i][n] for the p target nodes at offsets xi[i] from the source center */
static void or_axis_matrix(int p, const double *xi, int nimg, const double *img,
                           double half, double delta, const double *xq,
                           const double *wq, double *g)
{
    or_integrand f;
    f.p = p;
    f.half = half;
    f.delta = delta;
    f.xq = xq;
    f.wq = wq;
    /* the t-space integral is bounded by min(2, sqrt(pi*delta)/half) */
    double scale = sqrt(M_PI * delta) / half;
    if (scale > 2.0) scale = 2.0;
    f.tol = 1e-15 * scale;
    for (int i = 0; i < p; i++) {
        double acc[OR_MAXP];
        for (int n = 0; n < p; n++) acc[n] = 0.0;
        for (int k = 0; k < nimg; k++) {
            double whole[OR_MAXP];
            f.xi = xi[i] + img[k];
            or_panel(&f, -1.0, 1.0, whole);
            or_adapt(&f, -1.0, 1.0, whole, 0, acc);
        }
        for (int n = 0; n < p; n++) g[i * p + n] = half * acc[n];
    }
}

/* ---------------------------------------------------------------------- */
/* memo of 1D integral matrices, keyed by (level_S, level_T, offset)       */

typedef struct {
    uint64_t *keys;
    int64_t *vals;
    int64_t cap;
    int64_t n;
} or_map;

static uint64_t or_hash(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static int or_map_init(or_map *m, int64_t cap)
{
    m->cap = 16;
    while (m->cap < 2 * cap) m->cap <<= 1;
    m->keys = (uint64_t *)malloc(sizeof(uint64_t) * m->cap);
    m->vals = (int64_t *)malloc(sizeof(int64_t) * m->cap);
    m->n = 0;
    if (!m->keys || !m->vals) return -1;
    for (int64_t i = 0; i < m->cap; i++) m->keys[i] = UINT64_MAX;
    return 0;
}

static int or_map_grow(or_map *m)
{
    or_map nm;
    if (or_map_init(&nm, m->cap) != 0) return -1;
    for (int64_t i = 0; i < m->cap; i++) {
        if (m->keys[i] == UINT64_MAX) continue;
        int64_t h = (int64_t)(or_hash(m->keys[i]) & (uint64_t)(nm.cap - 1));
        while (nm.keys[h] != UINT64_MAX) h = (h + 1) & (nm.cap - 1);
        nm.keys[h] = m->keys[i];
        nm.vals[h] = m->vals[i];
    }
    nm.n = m->n;
    free(m->keys);
    free(m->vals);
    *m = nm;
    return 0;
}

/* returns the index of key, inserting it with the next free index if new */
static int64_t or_map_get(or_map *m, uint64_t key)
{
    if (2 * (m->n + 1) > m->cap && or_map_grow(m) != 0) return -1;
    int64_t h = (int64_t)(or_hash(key) & (uint64_t)(m->cap - 1));
    while (m->keys[h] != UINT64_MAX) {
        if (m->keys[h] == key) return m->vals[h];
        h = (h + 1) & (m->cap - 1);
    }
    m->keys[h] = key;
    m->vals[h] = m->n;
    return m->n++;
}

/* ---------------------------------------------------------------------- */
/* the transform                                                            */

static int or_threads_used = 1;

int oracle_threads(void) { return or_threads_used; }

/*
 * level[nleaves], coord[nleaves*d]: leaf i is the box of side 2^-level[i]
 * with lower corner -1/2 + coord*2^-level on each axis.  sigma[nleaves][p^d]
 * holds the samples at the leaf's tensor Gauss-Legendre nodes, multi-index
 * (i_1..i_d) at i_1 + p*i_2 + p^2*i_3.
 *
 * Targets are boxes given the same way, blevel[nbox], bcoord[nbox*d]: any box
 * of [-1/2,1/2]^d, not necessarily a leaf (Section 4.2 evaluates u on the
 * tensor grids of boxes of a refined output tree).  u[nbox][p^d] receives u at
 * each box's tensor Gauss-Legendre nodes.  rcut <= 0 selects
 * sqrt(delta*ln(1e17)).  Returns the number of (target box, source leaf)
 * pairs summed, or a negative value on bad arguments.
 */
int64_t oracle_box_fgt_boxes(int d, int64_t nleaves, const int32_t *level, const int32_t *coord,
                             int p, double delta, int periodic, double rcut,
                             const double *sigma, int64_t nbox, const int32_t *blevel,
                             const int32_t *bcoord, double *u, int nthreads)
{
    if (d < 1 || d > 3 || p < 1 || p > OR_MAXP || delta <= 0.0 || nleaves < 1 || nbox < 0)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    or_threads_used = omp_get_max_threads();
#else
    (void)nthreads;
    or_threads_used = 1;
#endif
    if (rcut <= 0.0) rcut = sqrt(delta * log(1e17));
    const int64_t ntarget = nbox;
    const int64_t np = or_ipow(p, d);

    double eta[OR_MAXP], wgl[OR_MAXP], xq[OR_NQ], wq[OR_NQ];
    or_gauss_legendre(p, eta, wgl);
    or_gauss_legendre(OR_NQ, xq, wq);

    int lmax = 0;
    for (int64_t i = 0; i < nleaves; i++) {
        if (level[i] < 0 || level[i] > 40) return -1;
        if (level[i] > lmax) lmax = level[i];
    }
    for (int64_t i = 0; i < nbox; i++) {
        if (blevel[i] < 0 || blevel[i] > 40) return -1;
        if (blevel[i] > lmax) lmax = blevel[i];
    }
    /* centers in units of 2^-(lmax+1): c = (2*coord+1)*2^(lmax-level) - 2^lmax */
    const int64_t unit_per_one = (int64_t)1 << (lmax + 1);
    const double unit = 1.0 / (double)unit_per_one;
    int64_t *cint = (int64_t *)malloc(sizeof(int64_t) * nleaves * d);
    int64_t *tint = (int64_t *)malloc(sizeof(int64_t) * (nbox > 0 ? nbox : 1) * d);
    double *coef = (double *)malloc(sizeof(double) * nleaves * np);
    if (!cint || !tint || !coef) { free(cint); free(tint); free(coef); return -2; }
    for (int64_t i = 0; i < nleaves; i++)
        for (int a = 0; a < d; a++)
            cint[i * d + a] = (2 * (int64_t)coord[i * d + a] + 1) * ((int64_t)1 << (lmax - level[i]))
                              - ((int64_t)1 << lmax);
    for (int64_t i = 0; i < nbox; i++)
        for (int a = 0; a < d; a++)
            tint[i * d + a] = (2 * (int64_t)bcoord[i * d + a] + 1) * ((int64_t)1 << (lmax - blevel[i]))
                              - ((int64_t)1 << lmax);

    /* step 2 for every source leaf */
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * np);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < nleaves; s++)
            or_coefficients(p, d, eta, wgl, sigma + s * np, coef + s * np, tmp);
        free(tmp);
    }

    /* pairs (target, source) with their per-axis memo indices */
    int64_t cap = 1024, npair = 0;
    int64_t *pt = (int64_t *)malloc(sizeof(int64_t) * cap);
    int64_t *ps = (int64_t *)malloc(sizeof(int64_t) * cap);
    int64_t *pk = (int64_t *)malloc(sizeof(int64_t) * cap * 3);
    int64_t *tstart = (int64_t *)malloc(sizeof(int64_t) * (ntarget + 1));
    or_map memo;
    if (or_map_init(&memo, 1024) != 0 || !pt || !ps || !pk || !tstart) return -2;
    int64_t kcap = 1024;
    uint64_t *klist = (uint64_t *)malloc(sizeof(uint64_t) * kcap);

    for (int64_t ti = 0; ti < ntarget; ti++) {
        tstart[ti] = npair;
        for (int64_t S = 0; S < nleaves; S++) {
            int ok = 1;
            int64_t off[3];
            for (int a = 0; a < d && ok; a++) {
                int64_t o = tint[ti * d + a] - cint[S * d + a];
                if (periodic) { /* normalize to (-1/2, 1/2] in units */
                    o %= unit_per_one;
                    if (o > unit_per_one / 2) o -= unit_per_one;
                    if (o <= -unit_per_one / 2) o += unit_per_one;
                }
                off[a] = o;
                double reach = 0.5 * (ldexp(1.0, -blevel[ti]) + ldexp(1.0, -level[S])) + rcut;
                double od = fabs((double)o * unit);
                /* nearest image is j = 0 after normalization */
                if (od > reach) ok = 0;
            }
            if (!ok) continue;
            if (npair == cap) {
                cap *= 2;
                pt = (int64_t *)realloc(pt, sizeof(int64_t) * cap);
                ps = (int64_t *)realloc(ps, sizeof(int64_t) * cap);
                pk = (int64_t *)realloc(pk, sizeof(int64_t) * cap * 3);
            }
            pt[npair] = ti;
            ps[npair] = S;
            for (int a = 0; a < d; a++) {
                uint64_t key = ((uint64_t)level[S] << 56) | ((uint64_t)blevel[ti] << 48)
                               | (uint64_t)(off[a] + ((int64_t)1 << 46));
                int64_t idx = or_map_get(&memo, key);
                if (idx == memo.n - 1 && idx >= 0) {
                    if (memo.n > kcap) {
                        kcap *= 2;
                        klist = (uint64_t *)realloc(klist, sizeof(uint64_t) * kcap);
                    }
                    klist[idx] = key;
                }
                pk[npair * 3 + a] = idx;
            }
            npair++;
        }
    }
    tstart[ntarget] = npair;

    /* 1D integral matrices for every distinct (level_S, level_T, offset) */
    const int64_t nkey = memo.n;
    double *gtab = (double *)malloc(sizeof(double) * (nkey > 0 ? nkey : 1) * p * p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nkey; k++) {
        uint64_t key = klist[k];
        int ls = (int)(key >> 56), lt = (int)((key >> 48) & 0xff);
        int64_t o = (int64_t)(key & (((uint64_t)1 << 48) - 1)) - ((int64_t)1 << 46);
        double hs = ldexp(0.5, -ls), ht = ldexp(0.5, -lt);
        double xi[OR_MAXP];
        for (int i = 0; i < p; i++) xi[i] = (double)o * unit + ht * eta[i];
        double img[64];
        int nimg = 0;
        if (periodic) {
            int jr = (int)ceil(rcut + 1.0) + 1;
            for (int j = -jr; j <= jr && nimg < 64; j++) {
                double od = fabs((double)o * unit + j);
                if (od <= hs + ht + rcut) img[nimg++] = (double)j;
            }
        } else {
            img[nimg++] = 0.0;
        }
        or_axis_matrix(p, xi, nimg, img, hs, delta, xq, wq, gtab + k * p * p);
    }

    /* contraction per target leaf (Lemma directbox, axis by axis) */
    int bad = 0;
#pragma omp parallel
    {
        double *t0 = (double *)malloc(sizeof(double) * np);
        double *t1 = (double *)malloc(sizeof(double) * np);
        if (!t0 || !t1) bad = 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t ti = 0; ti < ntarget; ti++) {
            double *ut = u + ti * np;
            for (int64_t i = 0; i < np; i++) ut[i] = 0.0;
            if (!t0 || !t1) continue;
            for (int64_t q = tstart[ti]; q < tstart[ti + 1]; q++) {
                memcpy(t0, coef + ps[q] * np, sizeof(double) * np);
                for (int a = 0; a < d; a++) {
                    or_apply_axis(p, d, a, gtab + pk[q * 3 + a] * p * p, t0, t1);
                    memcpy(t0, t1, sizeof(double) * np);
                }
                for (int64_t i = 0; i < np; i++) ut[i] += t0[i];
            }
        }
        free(t0);
        free(t1);
    }

    free(cint);
    free(tint);
    free(coef);
    free(pt);
    free(ps);
    free(pk);
    free(tstart);
    free(klist);
    free(gtab);
    free(memo.keys);
    free(memo.vals);
    return bad ? -2 : npair;
}

/*
 * The same transform with the targets given as leaves of the source tree:
 * targets[ntarget] lists the leaves whose nodes receive u (NULL = all leaves
 * in order); u[ntarget][p^d].
 */
int64_t oracle_box_fgt(int d, int64_t nleaves, const int32_t *level, const int32_t *coord,
                       int p, double delta, int periodic, double rcut,
                       const double *sigma, int64_t ntarget, const int64_t *targets,
                       double *u, int nthreads)
{
    if (d < 1 || d > 3 || nleaves < 1) return -1;
    if (!targets) ntarget = nleaves;
    int32_t *bl = (int32_t *)malloc(sizeof(int32_t) * (ntarget > 0 ? ntarget : 1));
    int32_t *bc = (int32_t *)malloc(sizeof(int32_t) * (ntarget > 0 ? ntarget : 1) * d);
    if (!bl || !bc) { free(bl); free(bc); return -2; }
    for (int64_t ti = 0; ti < ntarget; ti++) {
        int64_t T = targets ? targets[ti] : ti;
        if (T < 0 || T >= nleaves) { free(bl); free(bc); return -1; }
        bl[ti] = level[T];
        for (int a = 0; a < d; a++) bc[ti * d + a] = coord[T * d + a];
    }
    int64_t r = oracle_box_fgt_boxes(d, nleaves, level, coord, p, delta, periodic, rcut, sigma,
                                     ntarget, bl, bc, u, nthreads);
    free(bl);
    free(bc);
    return r;
}

/* The Gauss-Legendre rule used above, exported so tests can pin it. */
void oracle_gauss_legendre(int n, double *x, double *w) { or_gauss_legendre(n, x, w); }

/* ---------------------------------------------------------------------- */
/* The discrete (point) Gauss transform, Section 1, Eq. (pgt):             */
/*                                                                        */
/*   u_i = sum_j exp(-|x_i - y_j|^2 / delta) q_j,                         */
/*                                                                        */
/* summed directly over the sources y_j of [-1/2,1/2]^d for every target  */
/* x_i.  With cut > 0 the sources are binned into cells of side >= cut and */
/* a target visits only the 3^d cells around its own: every source it     */
/* skips is farther than cut along some axis, so its term is below        */
/* exp(-cut^2/delta) |q_j|.  With cut = 0 every pair is summed.  Returns  */
/* the number of pairs summed.                                            */

int64_t oracle_point_fgt(int d, int64_t ns, const double *y, const double *q, int64_t nt,
                         const double *x, double delta, double cut, double *u, int nthreads)
{
    if (d < 1 || d > 3 || ns < 0 || nt < 0 || !(delta > 0)) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        or_threads_used = omp_get_num_threads();
    }
#else
    or_threads_used = 1;
#endif
    int64_t npairs = 0;
    if (cut <= 0.0) {
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : npairs)
        for (int64_t i = 0; i < nt; i++) {
            double s = 0.0;
            for (int64_t j = 0; j < ns; j++) {
                double r2 = 0.0;
                for (int a = 0; a < d; a++) {
                    const double t = x[i * d + a] - y[j * d + a];
                    r2 += t * t;
                }
                s += exp(-r2 / delta) * q[j];
            }
            u[i] = s;
            npairs += ns;
        }
        return npairs;
    }
    /* cells of side 1/nc >= cut over [-1/2, 1/2]^d */
    int nc = (int)floor(1.0 / cut);
    if (nc < 1) nc = 1;
    if (nc > 512) nc = 512;
    int64_t ncell = 1;
    for (int a = 0; a < d; a++) ncell *= nc;
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    if (!start || !order || !cellof) {
        free(start);
        free(order);
        free(cellof);
        return -2;
    }
    for (int64_t j = 0; j < ns; j++) {
        int64_t c = 0;
        for (int a = 0; a < d; a++) {
            int k = (int)floor((y[j * d + a] + 0.5) * nc);
            if (k < 0) k = 0;
            if (k >= nc) k = nc - 1;
            c = c * nc + k;
        }
        cellof[j] = c;
        start[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        if (!fill) {
            free(start);
            free(order);
            free(cellof);
            return -2;
        }
        memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
        for (int64_t j = 0; j < ns; j++) order[fill[cellof[j]]++] = j;
        free(fill);
    }
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : npairs)
    for (int64_t i = 0; i < nt; i++) {
        int k[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) {
            k[a] = (int)floor((x[i * d + a] + 0.5) * nc);
            if (k[a] < 0) k[a] = 0;
            if (k[a] >= nc) k[a] = nc - 1;
        }
        double s = 0.0;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) {
            lo[a] = k[a] > 0 ? k[a] - 1 : 0;
            hi[a] = k[a] < nc - 1 ? k[a] + 1 : nc - 1;
        }
        for (int c3 = (d > 2 ? lo[2] : 0); c3 <= (d > 2 ? hi[2] : 0); c3++)
            for (int c2 = (d > 1 ? lo[1] : 0); c2 <= (d > 1 ? hi[1] : 0); c2++)
                for (int c1 = lo[0]; c1 <= hi[0]; c1++) {
                    /* cell index with axis 1 most significant, as binned above */
                    int64_t c = c1;
                    if (d > 1) c = c * nc + c2;
                    if (d > 2) c = c * nc + c3;
                    for (int64_t t = start[c]; t < start[c + 1]; t++) {
                        const int64_t j = order[t];
                        double r2 = 0.0;
                        for (int a = 0; a < d; a++) {
                            const double e = x[i * d + a] - y[j * d + a];
                            r2 += e * e;
                        }
                        s += exp(-r2 / delta) * q[j];
                        npairs++;
                    }
                }
        u[i] = s;
    }
    free(start);
    free(order);
    free(cellof);
    return npairs;
}
