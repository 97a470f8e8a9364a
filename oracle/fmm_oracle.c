/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle for the Laplace fast multipole method of
 * Yokota & Barba, "A Tuned and Scalable Fast Multipole Method as a Preeminent
 * Algorithm for Exascale Systems" (arXiv:1106.2176).  Only the test-suite, the
 * package smoke check and the benchmark's CPU-baseline leg may call it.  It
 * shares no code, table or basis with the GPU library: the GPU path uses real
 * spherical harmonics, this file uses Cartesian Taylor series.
 *
 * What it computes (Sec. 2.1 of the paper: N sources of a 1/r potential,
 * the gravitational or electrostatic N-body problem):
 *     phi_i = sum_{j != i, x_j != x_i} q_j / |x_i - x_j|
 *     E_i   = sum_{j != i, x_j != x_i} q_j (x_i - x_j) / |x_i - x_j|^3  (= -grad phi)
 * once exactly (oracle_direct, O(N^2)) and once through the FMM
 * (oracle_fmm), step by step:
 *   S1  uniform tree: the smallest level L whose fullest box holds at most
 *       leaf_max particles (Sec. 5, future directions: for uniform particle
 *       distributions the tree is a Morton index at a fixed maximum level);
 *   S2  box index of a particle: i = min(floor(((x-lo)/size) * 2^L), 2^L-1);
 *   S3  near list: the <= 27 leaves with |di|_inf <= 1 (Sec. 2.1, near/far);
 *   S4  interaction list at level l >= 2: children of the parent's near
 *       boxes that are not near boxes themselves (Fig. 1 caption: M2L runs
 *       between same-level boxes at every level below level 1);
 *   S5  P2M, S6 M2M, S7 M2L, S8 L2L, S9 L2P (Fig. 1 and Fig. 3), with
 *       multipole and local expansions of p terms, read as total degree
 *       0..p-1 (Sec. 2.1 defines both expansions as p-term series, Taylor
 *       series being one example), centred on the geometric box centre;
 *   S10 P2P over the near list (Sec. 3.1);
 *   S11 phi = far + near, E likewise.
 *
 * Notation: multi-index a = (a0,a1,a2), |a| = a0+a1+a2, a! = a0! a1! a2!,
 * x^a = x0^a0 x1^a1 x2^a2, G(x) = 1/|x|, D^a = partial derivative.
 *   P2M  M_a   = sum_j q_j (x_j - c)^a / a!
 *   M2M  M_a(c2) = sum_{b <= a} M_b(c1) (c1 - c2)^(a-b) / (a-b)!
 *   M2L  L_b(t) += (1/b!) sum_a (-1)^|a| M_a(s) D^(a+b) G(c_t - c_s)
 *   L2L  L_b(c2) = sum_{g >= b} L_g(c1) C(g,b) (c2 - c1)^(g-b)
 *   L2P  phi(x) = sum_b L_b (x - c)^b,  E = -grad phi
 * D^k G is built from the Taylor coefficients t_k = D^k G / k! of 1/|x| by
 * the published three-term recurrence (Duan & Krasny 2001; Lindsay & Krasny
 * 2001), written here for G(x) = 1/|x|:
 *   |k| r^2 t_k + (2|k|-1) sum_i x_i t_{k-e_i} + (|k|-1) sum_i t_{k-2e_i} = 0.
 *
 * All arithmetic is IEEE FP64, no fast-math.  OpenMP parallelises only the
 * outermost loop of each step (as the paper does, Sec. 3.1); every iteration
 * writes its own outputs, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_EDOMAIN 2
#define ORACLE_ENOMEM 3

/* ------------------------------------------------------------------ */
/* multi-indices with total degree <= D, ordered by degree            */
/* ------------------------------------------------------------------ */
typedef struct {
    int D;
    int n;
    int *k;      /* [n][3] */
    int *look;   /* [(D+1)^3] -> index, -1 if |k| > D */
    int *deg;    /* [n] */
} mindex;

static void fact_init(void);

static int mindex_init(mindex *m, int D)
{
    int s = D + 1, a, b, c, d, i = 0;
    fact_init();
    m->D = D;
    m->n = (D + 1) * (D + 2) * (D + 3) / 6;
    m->k = (int *)malloc(sizeof(int) * 3 * m->n);
    m->deg = (int *)malloc(sizeof(int) * m->n);
    m->look = (int *)malloc(sizeof(int) * s * s * s);
    if (!m->k || !m->look || !m->deg) return ORACLE_ENOMEM;
    for (a = 0; a < s * s * s; ++a) m->look[a] = -1;
    for (d = 0; d <= D; ++d)
        for (a = d; a >= 0; --a)
            for (b = d - a; b >= 0; --b) {
                c = d - a - b;
                m->k[3 * i] = a;
                m->k[3 * i + 1] = b;
                m->k[3 * i + 2] = c;
                m->deg[i] = d;
                m->look[(a * s + b) * s + c] = i;
                ++i;
            }
    return ORACLE_OK;
}

static void mindex_free(mindex *m)
{
    free(m->k);
    free(m->look);
    free(m->deg);
}

static int mi(const mindex *m, int a, int b, int c)
{
    int s = m->D + 1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > m->D) return -1;
    return m->look[(a * s + b) * s + c];
}

static double FACT[171];
static int fact_ready = 0;

static void fact_init(void)
{
    int i;
    if (fact_ready) return;
    FACT[0] = 1.0;
    for (i = 1; i < 171; ++i) FACT[i] = FACT[i - 1] * (double)i;
    fact_ready = 1;
}

static double fact(int n) { return FACT[n]; }

static double ipow(double x, int e)
{
    double r = 1.0;
    int i;
    for (i = 0; i < e; ++i) r *= x;
    return r;
}

/* t_k = D^k G(x) / k!  for all |k| <= m->D (recurrence in the header). */
static void taylor_coeffs(const mindex *m, const double x[3], double *t)
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    int i, ax;
    t[0] = 1.0 / sqrt(r2);
    for (i = 1; i < m->n; ++i) {
        const int *k = m->k + 3 * i;
        int K = m->deg[i];
        double s1 = 0.0, s2 = 0.0;
        for (ax = 0; ax < 3; ++ax) {
            int km[3] = {k[0], k[1], k[2]};
            int j;
            km[ax] -= 1;
            j = mi(m, km[0], km[1], km[2]);
            if (j >= 0) s1 += x[ax] * t[j];
            km[ax] -= 1;
            j = mi(m, km[0], km[1], km[2]);
            if (j >= 0) s2 += t[j];
        }
        t[i] = -((2.0 * K - 1.0) * s1 + (K - 1.0) * s2) / (K * r2);
    }
}

/* exported for pins: t_k = D^k(1/|x|)/k!, ordered as oracle_mindex lists */
int oracle_taylor_coeffs(int D, const double *x, double *t_out)
{
    mindex m;
    if (D < 0 || D > 60) return ORACLE_EINVAL;
    if (mindex_init(&m, D)) return ORACLE_ENOMEM;
    taylor_coeffs(&m, x, t_out);
    mindex_free(&m);
    return ORACLE_OK;
}

/* exported: the multi-index list for degree <= D, [n][3] */
int oracle_mindex(int D, int *k_out)
{
    mindex m;
    if (D < 0 || D > 60) return ORACLE_EINVAL;
    if (mindex_init(&m, D)) return ORACLE_ENOMEM;
    memcpy(k_out, m.k, sizeof(int) * 3 * m.n);
    mindex_free(&m);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* single operators (S5-S9), for one box each                         */
/* ------------------------------------------------------------------ */

/* S5 P2M about c: M_a = sum_j q_j (x_j - c)^a / a!, |a| < p */
static void p2m(const mindex *mp, int64_t ns, const int64_t *idx, const double *pos,
                const double *q, const double c[3], double *M)
{
    int i;
    int64_t j;
    for (i = 0; i < mp->n; ++i) M[i] = 0.0;
    for (j = 0; j < ns; ++j) {
        int64_t s = idx ? idx[j] : j;
        double pw[3][64];
        int ax, e;
        /* pw[ax][e] = (x_ax - c_ax)^e / e! */
        for (ax = 0; ax < 3; ++ax)
            for (e = 0; e <= mp->D; ++e) pw[ax][e] = ipow(pos[3 * s + ax] - c[ax], e) / fact(e);
        for (i = 0; i < mp->n; ++i) {
            const int *a = mp->k + 3 * i;
            M[i] += q[s] * pw[0][a[0]] * pw[1][a[1]] * pw[2][a[2]];
        }
    }
}

/* S6 M2M: M_a(c2) = sum_{b <= a} M_b(c1) (c1 - c2)^(a-b) / (a-b)! (accumulates) */
static void m2m(const mindex *mp, const double *M1, const double c1[3], const double c2[3],
                double *M2)
{
    double d[3] = {c1[0] - c2[0], c1[1] - c2[1], c1[2] - c2[2]};
    int i, j;
    for (i = 0; i < mp->n; ++i) {
        const int *a = mp->k + 3 * i;
        double s = 0.0;
        for (j = 0; j < mp->n; ++j) {
            const int *b = mp->k + 3 * j;
            int e0 = a[0] - b[0], e1 = a[1] - b[1], e2 = a[2] - b[2];
            if (e0 < 0 || e1 < 0 || e2 < 0) continue;
            s += M1[j] * ipow(d[0], e0) / fact(e0) * ipow(d[1], e1) / fact(e1) *
                 ipow(d[2], e2) / fact(e2);
        }
        M2[i] += s;
    }
}

/* sumidx[j * n + i] = index (in md) of the multi-index a_i + b_j */
static int *m2l_sum_table(const mindex *mp, const mindex *md)
{
    int i, j;
    int *t = (int *)malloc(sizeof(int) * mp->n * mp->n);
    if (!t) return NULL;
    for (j = 0; j < mp->n; ++j)
        for (i = 0; i < mp->n; ++i) {
            const int *a = mp->k + 3 * i, *b = mp->k + 3 * j;
            t[j * mp->n + i] = mi(md, a[0] + b[0], a[1] + b[1], a[2] + b[2]);
        }
    return t;
}

/* S7 M2L: L_b(c_t) += (1/b!) sum_a (-1)^|a| M_a D^(a+b) G(c_t - c_s).
 * dG holds D^k G(c_t - c_s) for |k| <= 2p-2 (indexed by md); sumidx from
 * m2l_sum_table. */
static void m2l(const mindex *mp, const int *sumidx, const double *M, const double *dG, double *L)
{
    int i, j;
    for (j = 0; j < mp->n; ++j) {
        const int *b = mp->k + 3 * j;
        const int *row = sumidx + j * mp->n;
        double s = 0.0;
        for (i = 0; i < mp->n; ++i) {
            double sg = (mp->deg[i] & 1) ? -1.0 : 1.0;
            s += sg * M[i] * dG[row[i]];
        }
        L[j] += s / (fact(b[0]) * fact(b[1]) * fact(b[2]));
    }
}

/* D^k G(x) for all |k| <= md->D */
static void derivs(const mindex *md, const double x[3], double *dG)
{
    int i;
    taylor_coeffs(md, x, dG);
    for (i = 0; i < md->n; ++i) {
        const int *k = md->k + 3 * i;
        dG[i] *= fact(k[0]) * fact(k[1]) * fact(k[2]);
    }
}

static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

/* S8 L2L: L_b(c2) = sum_{g >= b} L_g(c1) C(g,b) (c2 - c1)^(g-b) (accumulates) */
static void l2l(const mindex *mp, const double *L1, const double c1[3], const double c2[3],
                double *L2)
{
    double d[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
    int i, j;
    for (i = 0; i < mp->n; ++i) {
        const int *b = mp->k + 3 * i;
        double s = 0.0;
        for (j = 0; j < mp->n; ++j) {
            const int *g = mp->k + 3 * j;
            int e0 = g[0] - b[0], e1 = g[1] - b[1], e2 = g[2] - b[2];
            if (e0 < 0 || e1 < 0 || e2 < 0) continue;
            s += L1[j] * binom(g[0], b[0]) * binom(g[1], b[1]) * binom(g[2], b[2]) *
                 ipow(d[0], e0) * ipow(d[1], e1) * ipow(d[2], e2);
        }
        L2[i] += s;
    }
}

/* S9 L2P: phi = sum_b L_b (x-c)^b ; E = -grad phi */
static void l2p(const mindex *mp, const double *L, const double c[3], const double x[3],
                double *phi, double E[3])
{
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double f = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    int i;
    for (i = 0; i < mp->n; ++i) {
        const int *b = mp->k + 3 * i;
        double p0 = ipow(d[0], b[0]), p1 = ipow(d[1], b[1]), p2 = ipow(d[2], b[2]);
        f += L[i] * p0 * p1 * p2;
        if (b[0] > 0) g0 += L[i] * b[0] * ipow(d[0], b[0] - 1) * p1 * p2;
        if (b[1] > 0) g1 += L[i] * b[1] * p0 * ipow(d[1], b[1] - 1) * p2;
        if (b[2] > 0) g2 += L[i] * b[2] * p0 * p1 * ipow(d[2], b[2] - 1);
    }
    *phi = f;
    E[0] = -g0;
    E[1] = -g1;
    E[2] = -g2;
}

/* exported single-operator entry points (all FP64, host arrays) */
int oracle_p2m(int p, int64_t ns, const double *pos, const double *q, const double *c,
               double *M_out)
{
    mindex mp;
    if (p < 1 || p > 30 || ns < 0) return ORACLE_EINVAL;
    if (mindex_init(&mp, p - 1)) return ORACLE_ENOMEM;
    p2m(&mp, ns, NULL, pos, q, c, M_out);
    mindex_free(&mp);
    return ORACLE_OK;
}

int oracle_m2m(int p, const double *M1, const double *c1, const double *c2, double *M2_out)
{
    mindex mp;
    int i;
    if (p < 1 || p > 30) return ORACLE_EINVAL;
    if (mindex_init(&mp, p - 1)) return ORACLE_ENOMEM;
    for (i = 0; i < mp.n; ++i) M2_out[i] = 0.0;
    m2m(&mp, M1, c1, c2, M2_out);
    mindex_free(&mp);
    return ORACLE_OK;
}

int oracle_m2l(int p, const double *M, const double *cs, const double *ct, double *L_out)
{
    mindex mp, md;
    double x[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
    double *dG;
    int *sumidx;
    int i;
    if (p < 1 || p > 30) return ORACLE_EINVAL;
    if (mindex_init(&mp, p - 1) || mindex_init(&md, 2 * p - 2)) return ORACLE_ENOMEM;
    dG = (double *)malloc(sizeof(double) * md.n);
    if (!dG) return ORACLE_ENOMEM;
    sumidx = m2l_sum_table(&mp, &md);
    if (!sumidx) return ORACLE_ENOMEM;
    derivs(&md, x, dG);
    for (i = 0; i < mp.n; ++i) L_out[i] = 0.0;
    m2l(&mp, sumidx, M, dG, L_out);
    free(sumidx);
    free(dG);
    mindex_free(&mp);
    mindex_free(&md);
    return ORACLE_OK;
}

int oracle_l2l(int p, const double *L1, const double *c1, const double *c2, double *L2_out)
{
    mindex mp;
    int i;
    if (p < 1 || p > 30) return ORACLE_EINVAL;
    if (mindex_init(&mp, p - 1)) return ORACLE_ENOMEM;
    for (i = 0; i < mp.n; ++i) L2_out[i] = 0.0;
    l2l(&mp, L1, c1, c2, L2_out);
    mindex_free(&mp);
    return ORACLE_OK;
}

int oracle_l2p(int p, const double *L, const double *c, int64_t nt, const double *x,
               double *phi_out, double *E_out)
{
    mindex mp;
    int64_t i;
    if (p < 1 || p > 30) return ORACLE_EINVAL;
    if (mindex_init(&mp, p - 1)) return ORACLE_ENOMEM;
    for (i = 0; i < nt; ++i) l2p(&mp, L, c, x + 3 * i, phi_out + i, E_out + 3 * i);
    mindex_free(&mp);
    return ORACLE_OK;
}

/* multipole expansion evaluated directly: phi(x) = sum_a (-1)^|a| M_a D^a G(x - c) */
int oracle_m_eval(int p, const double *M, const double *c, int64_t nt, const double *x,
                  double *phi_out)
{
    mindex mp;
    int64_t t;
    double *dG;
    int i;
    if (p < 1 || p > 30) return ORACLE_EINVAL;
    if (mindex_init(&mp, p - 1)) return ORACLE_ENOMEM;
    dG = (double *)malloc(sizeof(double) * mp.n);
    if (!dG) return ORACLE_ENOMEM;
    for (t = 0; t < nt; ++t) {
        double d[3] = {x[3 * t] - c[0], x[3 * t + 1] - c[1], x[3 * t + 2] - c[2]};
        double s = 0.0;
        derivs(&mp, d, dG);
        for (i = 0; i < mp.n; ++i) s += ((mp.deg[i] & 1) ? -1.0 : 1.0) * M[i] * dG[i];
        phi_out[t] = s;
    }
    free(dG);
    mindex_free(&mp);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* direct sum (the exact result, Sec. 2.1)                            */
/* ------------------------------------------------------------------ */

/* For each target index targets[t] (all particles when targets == NULL):
 * phi[t] = sum_{j != i, r > 0} q_j / r,  E[t] = sum q_j (x_i - x_j) / r^3. */
int oracle_direct(int64_t n, const double *pos, const double *q, int64_t nt,
                  const int64_t *targets, double *phi, double *E)
{
    int64_t t;
    if (n < 0 || nt < 0 || (!targets && nt != n)) return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < nt; ++t) {
        int64_t i = targets ? targets[t] : t, j;
        double f = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0;
        for (j = 0; j < n; ++j) {
            double d0, d1, d2, r2, r;
            if (j == i) continue;
            d0 = pos[3 * i] - pos[3 * j];
            d1 = pos[3 * i + 1] - pos[3 * j + 1];
            d2 = pos[3 * i + 2] - pos[3 * j + 2];
            r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (r2 == 0.0) continue;
            r = sqrt(r2);
            f += q[j] / r;
            e0 += q[j] * d0 / (r2 * r);
            e1 += q[j] * d1 / (r2 * r);
            e2 += q[j] * d2 / (r2 * r);
        }
        phi[t] = f;
        E[3 * t] = e0;
        E[3 * t + 1] = e1;
        E[3 * t + 2] = e2;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* tree (S1, S2) and Morton keys                                       */
/* ------------------------------------------------------------------ */

/* S2: integer box coordinate at level l of one coordinate value */
static int64_t box_coord(double x, double lo, double size, int l)
{
    double s = (x - lo) / size;
    double v = floor(s * (double)((int64_t)1 << l));
    int64_t i = (int64_t)v;
    int64_t nmax = ((int64_t)1 << l) - 1;
    if (i > nmax) i = nmax;
    if (i < 0) i = 0;
    return i;
}

static int check_domain(int64_t n, const double *pos, const double lo[3], double size)
{
    int64_t i;
    int a;
    for (i = 0; i < n; ++i)
        for (a = 0; a < 3; ++a) {
            double x = pos[3 * i + a];
            if (!(x >= lo[a] && x <= lo[a] + size)) return ORACLE_EDOMAIN;
        }
    return ORACLE_OK;
}

/* S1: smallest level l in [0, max_level] whose fullest box holds <= leaf_max
 * particles; max_level if none does. */
int oracle_select_level(int64_t n, const double *pos, int leaf_max, int max_level,
                        const double *lo, double size, int *level_out, int64_t *max_count_out)
{
    int l;
    if (n < 1 || leaf_max < 1 || max_level < 0 || max_level > 10 || !(size > 0))
        return ORACLE_EINVAL;
    if (check_domain(n, pos, lo, size)) return ORACLE_EDOMAIN;
    for (l = 0; l <= max_level; ++l) {
        int64_t side = (int64_t)1 << l, nb = side * side * side, i, mx = 0;
        int64_t *cnt = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
        if (!cnt) return ORACLE_ENOMEM;
        for (i = 0; i < n; ++i) {
            int64_t bx = box_coord(pos[3 * i], lo[0], size, l);
            int64_t by = box_coord(pos[3 * i + 1], lo[1], size, l);
            int64_t bz = box_coord(pos[3 * i + 2], lo[2], size, l);
            cnt[bx + side * (by + side * bz)] += 1;
        }
        for (i = 0; i < nb; ++i)
            if (cnt[i] > mx) mx = cnt[i];
        free(cnt);
        if (mx <= leaf_max || l == max_level) {
            *level_out = l;
            if (max_count_out) *max_count_out = mx;
            return ORACLE_OK;
        }
    }
    return ORACLE_EINVAL;
}

/* Morton key: bit 3b of the key is bit b of ix, 3b+1 of iy, 3b+2 of iz */
static uint64_t morton(int64_t ix, int64_t iy, int64_t iz, int l)
{
    uint64_t k = 0;
    int b;
    for (b = 0; b < l; ++b) {
        k |= (uint64_t)((ix >> b) & 1) << (3 * b);
        k |= (uint64_t)((iy >> b) & 1) << (3 * b + 1);
        k |= (uint64_t)((iz >> b) & 1) << (3 * b + 2);
    }
    return k;
}

/* Keys at level l, leaf ranges and the stable sort by key (ties keep the
 * input order).  leaf_start has 8^l + 1 entries; perm[k] = input index of
 * the k-th particle in sorted order. */
int oracle_tree(int64_t n, const double *pos, int l, const double *lo, double size,
                uint64_t *keys, int64_t *leaf_start, int64_t *perm)
{
    int64_t nb, i, side;
    int64_t *fill;
    if (n < 1 || l < 0 || l > 10 || !(size > 0)) return ORACLE_EINVAL;
    if (check_domain(n, pos, lo, size)) return ORACLE_EDOMAIN;
    side = (int64_t)1 << l;
    nb = side * side * side;
    for (i = 0; i <= nb; ++i) leaf_start[i] = 0;
    for (i = 0; i < n; ++i) {
        keys[i] = morton(box_coord(pos[3 * i], lo[0], size, l),
                         box_coord(pos[3 * i + 1], lo[1], size, l),
                         box_coord(pos[3 * i + 2], lo[2], size, l), l);
        leaf_start[keys[i] + 1] += 1;
    }
    for (i = 0; i < nb; ++i) leaf_start[i + 1] += leaf_start[i];
    fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    if (!fill) return ORACLE_ENOMEM;
    for (i = 0; i < nb; ++i) fill[i] = leaf_start[i];
    for (i = 0; i < n; ++i) perm[fill[keys[i]]++] = i;
    free(fill);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* the FMM (S1-S11)                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int l;          /* level */
    int64_t side;   /* 2^l */
    double w;       /* box width */
    double *M, *L;  /* [side^3][ncoef] */
    char *need;     /* boxes whose local expansion is needed */
} olevel;

static int64_t bidx(int64_t side, int64_t i, int64_t j, int64_t k) { return i + side * (j + side * k); }

static void centre(const double lo[3], double w, int64_t i, int64_t j, int64_t k, double c[3])
{
    c[0] = lo[0] + ((double)i + 0.5) * w;
    c[1] = lo[1] + ((double)j + 0.5) * w;
    c[2] = lo[2] + ((double)k + 0.5) * w;
}

/*
 * Full FMM when targets == NULL (outputs per particle), otherwise only for the
 * particles targets[0..nt) (outputs per target slot); the sampled form runs
 * S7-S9 only for the boxes that are ancestors of a target's leaf, which is
 * the same computation restricted to the outputs asked for.
 * Near (P2P) and far (L2P) parts are returned separately; phi = sum of both.
 */
int oracle_fmm(int64_t n, const double *pos, const double *q, int p, int leaf_max, int max_level,
               const double *lo, double size, int64_t nt, const int64_t *targets,
               double *phi_near, double *E_near, double *phi_far, double *E_far, int *level_out)
{
    int L, l, rc;
    int64_t side, nleaf, i, t;
    int64_t *leaf_start = NULL, *order = NULL, *leaf_of = NULL, *fill = NULL;
    mindex mp, md;
    olevel *lev = NULL;
    int *sumidx = NULL;
    double *dGtab = NULL;
    int64_t ntt = targets ? nt : n;

    if (n < 1 || p < 1 || p > 30 || (targets && nt < 0)) return ORACLE_EINVAL;
    rc = oracle_select_level(n, pos, leaf_max, max_level, lo, size, &L, NULL); /* S1 */
    if (rc) return rc;
    if (level_out) *level_out = L;

    /* S2: leaves in row-major order, particles grouped per leaf */
    side = (int64_t)1 << L;
    nleaf = side * side * side;
    leaf_start = (int64_t *)calloc((size_t)nleaf + 1, sizeof(int64_t));
    order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    leaf_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nleaf);
    if (!leaf_start || !order || !leaf_of || !fill) return ORACLE_ENOMEM;
    for (i = 0; i < n; ++i) {
        leaf_of[i] = bidx(side, box_coord(pos[3 * i], lo[0], size, L),
                          box_coord(pos[3 * i + 1], lo[1], size, L),
                          box_coord(pos[3 * i + 2], lo[2], size, L));
        leaf_start[leaf_of[i] + 1] += 1;
    }
    for (i = 0; i < nleaf; ++i) leaf_start[i + 1] += leaf_start[i];
    for (i = 0; i < nleaf; ++i) fill[i] = leaf_start[i];
    for (i = 0; i < n; ++i) order[fill[leaf_of[i]]++] = i;
    free(fill);

    if (mindex_init(&mp, p - 1) || mindex_init(&md, 2 * p - 2)) return ORACLE_ENOMEM;

    /* S10: P2P over the near list of each target's leaf */
#pragma omp parallel for schedule(dynamic, 64)
    for (t = 0; t < ntt; ++t) {
        int64_t ip = targets ? targets[t] : t;
        int64_t b = leaf_of[ip];
        int64_t bi = b % side, bj = (b / side) % side, bk = b / (side * side);
        int64_t di, dj, dk, j;
        double f = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0;
        for (dk = -1; dk <= 1; ++dk)
            for (dj = -1; dj <= 1; ++dj)
                for (di = -1; di <= 1; ++di) {
                    int64_t si = bi + di, sj = bj + dj, sk = bk + dk, s;
                    if (si < 0 || sj < 0 || sk < 0 || si >= side || sj >= side || sk >= side) continue;
                    s = bidx(side, si, sj, sk);
                    for (j = leaf_start[s]; j < leaf_start[s + 1]; ++j) {
                        int64_t jp = order[j];
                        double d0, d1, d2, r2, r;
                        if (jp == ip) continue;
                        d0 = pos[3 * ip] - pos[3 * jp];
                        d1 = pos[3 * ip + 1] - pos[3 * jp + 1];
                        d2 = pos[3 * ip + 2] - pos[3 * jp + 2];
                        r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        if (r2 == 0.0) continue;
                        r = sqrt(r2);
                        f += q[jp] / r;
                        e0 += q[jp] * d0 / (r2 * r);
                        e1 += q[jp] * d1 / (r2 * r);
                        e2 += q[jp] * d2 / (r2 * r);
                    }
                }
        phi_near[t] = f;
        E_near[3 * t] = e0;
        E_near[3 * t + 1] = e1;
        E_near[3 * t + 2] = e2;
        phi_far[t] = 0.0;
        E_far[3 * t] = E_far[3 * t + 1] = E_far[3 * t + 2] = 0.0;
    }

    if (L >= 2) {
        lev = (olevel *)calloc((size_t)L + 1, sizeof(olevel));
        if (!lev) return ORACLE_ENOMEM;
        for (l = 2; l <= L; ++l) {
            int64_t sd = (int64_t)1 << l, nb = sd * sd * sd;
            lev[l].l = l;
            lev[l].side = sd;
            lev[l].w = size / (double)sd;
            lev[l].M = (double *)calloc((size_t)(nb * mp.n), sizeof(double));
            lev[l].L = (double *)calloc((size_t)(nb * mp.n), sizeof(double));
            lev[l].need = (char *)calloc((size_t)nb, 1);
            if (!lev[l].M || !lev[l].L || !lev[l].need) return ORACLE_ENOMEM;
        }
        /* boxes whose local expansion is needed: ancestors of target leaves */
        for (t = 0; t < ntt; ++t) {
            int64_t b = leaf_of[targets ? targets[t] : t];
            int64_t bi = b % side, bj = (b / side) % side, bk = b / (side * side);
            for (l = L; l >= 2; --l) {
                int sh = L - l;
                lev[l].need[bidx(lev[l].side, bi >> sh, bj >> sh, bk >> sh)] = 1;
            }
        }

        /* S5: P2M at the leaves */
#pragma omp parallel for schedule(dynamic, 64)
        for (i = 0; i < nleaf; ++i) {
            double c[3];
            centre(lo, lev[L].w, i % side, (i / side) % side, i / (side * side), c);
            p2m(&mp, leaf_start[i + 1] - leaf_start[i], order + leaf_start[i], pos, q, c,
                lev[L].M + i * mp.n);
        }
        /* S6: M2M, level L-1 down to 2 */
        for (l = L - 1; l >= 2; --l) {
            int64_t sd = lev[l].side, nb = sd * sd * sd, b;
#pragma omp parallel for schedule(dynamic, 16)
            for (b = 0; b < nb; ++b) {
                int64_t bi = b % sd, bj = (b / sd) % sd, bk = b / (sd * sd);
                double c2[3];
                int ci;
                centre(lo, lev[l].w, bi, bj, bk, c2);
                for (ci = 0; ci < 8; ++ci) {
                    int64_t ch_i = 2 * bi + (ci & 1), ch_j = 2 * bj + ((ci >> 1) & 1),
                            ch_k = 2 * bk + ((ci >> 2) & 1);
                    double c1[3];
                    centre(lo, lev[l + 1].w, ch_i, ch_j, ch_k, c1);
                    m2m(&mp, lev[l + 1].M + bidx(2 * sd, ch_i, ch_j, ch_k) * mp.n, c1, c2,
                        lev[l].M + b * mp.n);
                }
            }
        }
        /* S7: M2L at every level >= 2 for the needed target boxes.  The
         * derivative tensor D^k G(c_t - c_s) depends only on the offset
         * c_t - c_s = w * (i_t - i_s); it is evaluated once per level for each
         * offset in {-3..3}^3 and looked up. */
        sumidx = m2l_sum_table(&mp, &md);
        dGtab = (double *)malloc(sizeof(double) * 343 * md.n);
        if (!sumidx || !dGtab) return ORACLE_ENOMEM;
        for (l = 2; l <= L; ++l) {
            int64_t sd = lev[l].side, nb = sd * sd * sd, b;
            double w = lev[l].w;
            int o;
#pragma omp parallel for schedule(static)
            for (o = 0; o < 343; ++o) {
                double x[3];
                x[0] = w * (double)(o % 7 - 3);
                x[1] = w * (double)((o / 7) % 7 - 3);
                x[2] = w * (double)(o / 49 - 3);
                if (o == 171) continue; /* zero offset, never used */
                derivs(&md, x, dGtab + (size_t)o * md.n);
            }
#pragma omp parallel for schedule(dynamic, 4)
            for (b = 0; b < nb; ++b) {
                int64_t bi = b % sd, bj = (b / sd) % sd, bk = b / (sd * sd);
                int64_t pi = bi >> 1, pj = bj >> 1, pk = bk >> 1;
                int64_t ni, nj, nk;
                if (!lev[l].need[b]) continue;
                /* S4: children of the parent's near boxes that are not near */
                for (nk = pk - 1; nk <= pk + 1; ++nk)
                    for (nj = pj - 1; nj <= pj + 1; ++nj)
                        for (ni = pi - 1; ni <= pi + 1; ++ni) {
                            int ci;
                            if (ni < 0 || nj < 0 || nk < 0 || ni >= sd / 2 || nj >= sd / 2 || nk >= sd / 2)
                                continue;
                            for (ci = 0; ci < 8; ++ci) {
                                int64_t si = 2 * ni + (ci & 1), sj = 2 * nj + ((ci >> 1) & 1),
                                        sk = 2 * nk + ((ci >> 2) & 1);
                                int64_t oi = bi - si, oj = bj - sj, ok = bk - sk;
                                if (llabs(oi) <= 1 && llabs(oj) <= 1 && llabs(ok) <= 1) continue;
                                m2l(&mp, sumidx, lev[l].M + bidx(sd, si, sj, sk) * mp.n,
                                    dGtab + (size_t)((oi + 3) + 7 * ((oj + 3) + 7 * (ok + 3))) * md.n,
                                    lev[l].L + b * mp.n);
                            }
                        }
            }
        }
        free(sumidx);
        free(dGtab);
        /* S8: L2L, level 2 down to L-1, into the needed children */
        for (l = 2; l < L; ++l) {
            int64_t sd = lev[l + 1].side, nb = sd * sd * sd, b;
#pragma omp parallel for schedule(dynamic, 16)
            for (b = 0; b < nb; ++b) {
                int64_t bi = b % sd, bj = (b / sd) % sd, bk = b / (sd * sd);
                double c1[3], c2[3];
                if (!lev[l + 1].need[b]) continue;
                centre(lo, lev[l].w, bi >> 1, bj >> 1, bk >> 1, c1);
                centre(lo, lev[l + 1].w, bi, bj, bk, c2);
                l2l(&mp, lev[l].L + bidx(sd / 2, bi >> 1, bj >> 1, bk >> 1) * mp.n, c1, c2,
                    lev[l + 1].L + b * mp.n);
            }
        }
        /* S9: L2P at the targets */
#pragma omp parallel for schedule(dynamic, 64)
        for (t = 0; t < ntt; ++t) {
            int64_t ip = targets ? targets[t] : t;
            int64_t b = leaf_of[ip];
            double c[3];
            centre(lo, lev[L].w, b % side, (b / side) % side, b / (side * side), c);
            l2p(&mp, lev[L].L + b * mp.n, c, pos + 3 * ip, phi_far + t, E_far + 3 * t);
        }
        for (l = 2; l <= L; ++l) {
            free(lev[l].M);
            free(lev[l].L);
            free(lev[l].need);
        }
        free(lev);
    }
    mindex_free(&mp);
    mindex_free(&md);
    free(leaf_start);
    free(order);
    free(leaf_of);
    return ORACLE_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* adaptive tree (the next step named in Sec. 5, future directions:   */
/* switching between uniform and adaptive tree construction)          */
/* ------------------------------------------------------------------ */
/*
 * The paper names adaptive construction but fixes no rule; this oracle takes
 * the classic one.  A box holding more than leaf_max particles is split into
 * its eight children while its level is below max_level; children with no
 * particles are not created; unsplit boxes are leaves.  Two boxes are
 * adjacent when their closed cubes intersect and neither contains the other;
 * a box's colleagues are the adjacent boxes of its own level.  Lists:
 *   U(b), b a leaf: b and every leaf adjacent to b             -> P2P
 *   V(b), any box:  children of the colleagues of b's parent
 *                   that are not adjacent to b                 -> M2L
 *   W(b), b a leaf: descendants of b's colleagues that are not
 *                   adjacent to b but whose parent is          -> M2P
 *   X(b), any box:  the boxes c with b in W(c)                 -> P2L
 * Every ordered pair of particles is then accounted for exactly once: by
 * P2P, or by one M2L between ancestors (or the leaves themselves), or by
 * one M2P / P2L between a leaf and an ancestor of the other leaf.
 *   M2P  phi(x) = sum_a (-1)^|a| M_a D^a G(x - c),  E = -grad phi (exact
 *        gradient of the truncated multipole field)
 *   P2L  L_b(c) = sum_j q_j D^b G(c - x_j) / b!
 */
typedef struct {
    int l;
    int64_t ix, iy, iz;  /* integer coordinates at level l */
    int64_t start, end;  /* particle range in the sorted order */
    int parent;
    int child[8];        /* -1: no child (empty or unsplit) */
    int leaf;
} abox;

typedef struct {
    int *v;
    int n, cap;
} ilist;

static int ilist_push(ilist *a, int x)
{
    if (a->n == a->cap) {
        int nc = a->cap ? 2 * a->cap : 8;
        int *nv = (int *)realloc(a->v, sizeof(int) * (size_t)nc);
        if (!nv) return 1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

typedef struct {
    int nbox, cap;
    abox *box;
    int depth;
    int64_t *order;  /* sorted particle order (input indices) */
    ilist *U, *V, *W, *X;
    int *lev_first, *lev_count;  /* boxes of each level, contiguous, Morton order */
} atree;

/* closed-cube intersection of boxes a and b, not nested */
static int adjacent(const abox *a, const abox *b)
{
    const abox *f = a->l >= b->l ? a : b, *c = a->l >= b->l ? b : a;
    int k = f->l - c->l, ax;
    int64_t fi[3] = {f->ix, f->iy, f->iz}, ci[3] = {c->ix, c->iy, c->iz};
    int inside = 1;
    for (ax = 0; ax < 3; ++ax) {
        int64_t lo = ci[ax] << k, hi = ((ci[ax] + 1) << k) - 1;  /* c's span at f's level */
        if (fi[ax] < lo - 1 || fi[ax] > hi + 1) return 0;
        if (fi[ax] < lo || fi[ax] > hi) inside = 0;
    }
    return !inside;
}

static int find_box(const atree *t, int l, int64_t ix, int64_t iy, int64_t iz)
{
    int64_t side = (int64_t)1 << l, key;
    int lo, hi;
    if (l > t->depth || ix < 0 || iy < 0 || iz < 0 || ix >= side || iy >= side || iz >= side) return -1;
    key = (int64_t)morton(ix, iy, iz, l);
    lo = t->lev_first[l];
    hi = lo + t->lev_count[l] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        const abox *b = t->box + mid;
        int64_t k = (int64_t)morton(b->ix, b->iy, b->iz, l);
        if (k == key) return mid;
        if (k < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static void atree_free(atree *t)
{
    int i;
    if (t->U)
        for (i = 0; i < t->nbox; ++i) {
            free(t->U[i].v);
            free(t->V[i].v);
            free(t->W[i].v);
            free(t->X[i].v);
        }
    free(t->U);
    free(t->V);
    free(t->W);
    free(t->X);
    free(t->box);
    free(t->order);
    free(t->lev_first);
    free(t->lev_count);
}

typedef struct {
    uint64_t key;
    int64_t idx;
} keyidx;

static int keyidx_cmp(const void *a, const void *b)
{
    const keyidx *x = (const keyidx *)a, *y = (const keyidx *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* descend from box d (a child of a colleague of leaf b): adjacent leaves go
 * to U(b), non-adjacent boxes to W(b), adjacent split boxes are opened */
static int descend_uw(atree *t, int b, int d)
{
    const abox *bb = t->box + b, *dd = t->box + d;
    int c;
    if (!adjacent(bb, dd)) return ilist_push(&t->W[b], d);
    if (dd->leaf) return ilist_push(&t->U[b], d);
    for (c = 0; c < 8; ++c)
        if (dd->child[c] >= 0 && descend_uw(t, b, dd->child[c])) return 1;
    return 0;
}

static int atree_build(int64_t n, const double *pos, int leaf_max, int max_level, const double lo[3],
                       double size, atree *t)
{
    keyidx *ki;
    int64_t i;
    int b, l;
    memset(t, 0, sizeof(*t));
    ki = (keyidx *)malloc(sizeof(keyidx) * (size_t)n);
    t->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!ki || !t->order) return ORACLE_ENOMEM;
    /* particles sorted by their finest-level Morton key (stable): every box
     * of every level is then one contiguous range */
    for (i = 0; i < n; ++i) {
        ki[i].key = morton(box_coord(pos[3 * i], lo[0], size, max_level),
                           box_coord(pos[3 * i + 1], lo[1], size, max_level),
                           box_coord(pos[3 * i + 2], lo[2], size, max_level), max_level);
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(keyidx), keyidx_cmp);
    for (i = 0; i < n; ++i) t->order[i] = ki[i].idx;
    /* breadth-first construction: level by level, Morton order within a level */
    t->cap = 64;
    t->box = (abox *)malloc(sizeof(abox) * (size_t)t->cap);
    t->lev_first = (int *)calloc((size_t)max_level + 2, sizeof(int));
    t->lev_count = (int *)calloc((size_t)max_level + 2, sizeof(int));
    if (!t->box || !t->lev_first || !t->lev_count) return ORACLE_ENOMEM;
    memset(t->box, 0, sizeof(abox));
    t->box[0].start = 0;
    t->box[0].end = n;
    t->box[0].parent = -1;
    t->nbox = 1;
    t->lev_first[0] = 0;
    t->lev_count[0] = 1;
    t->depth = 0;
    for (l = 0; l <= max_level; ++l) {
        int first = t->lev_first[l], cnt = t->lev_count[l];
        t->lev_first[l + 1] = t->nbox;
        for (b = first; b < first + cnt; ++b) {
            abox *bx = t->box + b;
            int c;
            for (c = 0; c < 8; ++c) bx->child[c] = -1;
            bx->leaf = !(bx->end - bx->start > leaf_max && l < max_level);
            if (bx->leaf) continue;
            {
                int64_t s = bx->start;
                int sh = 3 * (max_level - l - 1);
                for (c = 0; c < 8; ++c) {
                    uint64_t ck = ((uint64_t)morton(bx->ix, bx->iy, bx->iz, l) << 3) | (uint64_t)c;
                    int64_t e = s;
                    while (e < bx->end && (ki[e].key >> sh) == ck) ++e;
                    if (e > s) {
                        abox *nb;
                        if (t->nbox == t->cap) {
                            abox *nbx = (abox *)realloc(t->box, sizeof(abox) * (size_t)t->cap * 2);
                            if (!nbx) return ORACLE_ENOMEM;
                            t->box = nbx;
                            t->cap *= 2;
                            bx = t->box + b;
                        }
                        nb = t->box + t->nbox;
                        memset(nb, 0, sizeof(abox));
                        nb->l = l + 1;
                        nb->ix = 2 * bx->ix + (c & 1);
                        nb->iy = 2 * bx->iy + ((c >> 1) & 1);
                        nb->iz = 2 * bx->iz + (c >> 2);
                        nb->start = s;
                        nb->end = e;
                        nb->parent = b;
                        bx->child[c] = t->nbox++;
                    }
                    s = e;
                }
            }
        }
        t->lev_count[l + 1] = t->nbox - t->lev_first[l + 1];
        if (t->lev_count[l + 1] == 0) break;
        t->depth = l + 1;
    }
    free(ki);
    /* lists */
    t->U = (ilist *)calloc((size_t)t->nbox, sizeof(ilist));
    t->V = (ilist *)calloc((size_t)t->nbox, sizeof(ilist));
    t->W = (ilist *)calloc((size_t)t->nbox, sizeof(ilist));
    t->X = (ilist *)calloc((size_t)t->nbox, sizeof(ilist));
    if (!t->U || !t->V || !t->W || !t->X) return ORACLE_ENOMEM;
    for (b = 0; b < t->nbox; ++b) {
        const abox *bx = t->box + b;
        int64_t dx, dy, dz;
        /* V: children of the parent's colleagues, not adjacent to b */
        if (bx->parent >= 0) {
            const abox *pa = t->box + bx->parent;
            for (dz = -1; dz <= 1; ++dz)
                for (dy = -1; dy <= 1; ++dy)
                    for (dx = -1; dx <= 1; ++dx) {
                        int pc = find_box(t, pa->l, pa->ix + dx, pa->iy + dy, pa->iz + dz), c;
                        if (pc < 0) continue;
                        for (c = 0; c < 8; ++c) {
                            int s = t->box[pc].child[c];
                            if (s < 0 || s == b) continue;
                            if (!adjacent(bx, t->box + s) && ilist_push(&t->V[b], s)) return ORACLE_ENOMEM;
                        }
                    }
        }
        if (!bx->leaf) continue;
        /* U: b itself; coarser adjacent leaves (colleagues of ancestors);
         * same-level adjacent leaves; finer ones below the colleagues.
         * W: non-adjacent descendants of colleagues with adjacent parents. */
        if (ilist_push(&t->U[b], b)) return ORACLE_ENOMEM;
        {
            int a = bx->parent;
            while (a >= 0) {
                const abox *an = t->box + a;
                for (dz = -1; dz <= 1; ++dz)
                    for (dy = -1; dy <= 1; ++dy)
                        for (dx = -1; dx <= 1; ++dx) {
                            int c;
                            if (!dx && !dy && !dz) continue;
                            c = find_box(t, an->l, an->ix + dx, an->iy + dy, an->iz + dz);
                            if (c >= 0 && t->box[c].leaf && adjacent(bx, t->box + c) &&
                                ilist_push(&t->U[b], c))
                                return ORACLE_ENOMEM;
                        }
                a = an->parent;
            }
        }
        for (dz = -1; dz <= 1; ++dz)
            for (dy = -1; dy <= 1; ++dy)
                for (dx = -1; dx <= 1; ++dx) {
                    int c, k;
                    if (!dx && !dy && !dz) continue;
                    c = find_box(t, bx->l, bx->ix + dx, bx->iy + dy, bx->iz + dz);
                    if (c < 0) continue;
                    if (t->box[c].leaf) {
                        if (ilist_push(&t->U[b], c)) return ORACLE_ENOMEM;
                        continue;
                    }
                    for (k = 0; k < 8; ++k)
                        if (t->box[c].child[k] >= 0 && descend_uw(t, b, t->box[c].child[k])) return ORACLE_ENOMEM;
                }
    }
    /* X: the dual of W */
    for (b = 0; b < t->nbox; ++b) {
        int k;
        for (k = 0; k < t->W[b].n; ++k)
            if (ilist_push(&t->X[t->W[b].v[k]], b)) return ORACLE_ENOMEM;
    }
    return ORACLE_OK;
}

static void abox_centre(const abox *b, const double lo[3], double size, double c[3])
{
    double w = size / (double)((int64_t)1 << b->l);
    centre(lo, w, b->ix, b->iy, b->iz, c);
}

/*
 * Tree and lists of the adaptive FMM, for tests.  Boxes in breadth-first,
 * Morton order (box 0 is the root).  box_out[b*8 + 0..7] = level, ix, iy,
 * iz, start, end, parent, leaf.  Lists as CSR: *_start[nbox+1], *_items;
 * the caller sizes the outputs from oracle_adaptive_sizes.
 */
int oracle_adaptive_sizes(int64_t n, const double *pos, int leaf_max, int max_level, const double *lo,
                          double size, int64_t *sizes_out /* nbox, nU, nV, nW, nX, depth */)
{
    atree t;
    int rc, b;
    int64_t s[4] = {0, 0, 0, 0};
    if (n < 1 || leaf_max < 1 || max_level < 0 || max_level > 10 || !(size > 0)) return ORACLE_EINVAL;
    if (check_domain(n, pos, lo, size)) return ORACLE_EDOMAIN;
    rc = atree_build(n, pos, leaf_max, max_level, lo, size, &t);
    if (rc) {
        atree_free(&t);
        return rc;
    }
    for (b = 0; b < t.nbox; ++b) {
        s[0] += t.U[b].n;
        s[1] += t.V[b].n;
        s[2] += t.W[b].n;
        s[3] += t.X[b].n;
    }
    sizes_out[0] = t.nbox;
    sizes_out[1] = s[0];
    sizes_out[2] = s[1];
    sizes_out[3] = s[2];
    sizes_out[4] = s[3];
    sizes_out[5] = t.depth;
    atree_free(&t);
    return ORACLE_OK;
}

int oracle_adaptive_lists(int64_t n, const double *pos, int leaf_max, int max_level, const double *lo,
                          double size, int64_t *box_out, int64_t *order_out, int64_t *lst_start,
                          int64_t *lst_items /* U, V, W, X: each [nbox+1] starts, items concatenated */)
{
    atree t;
    int rc, b, w, k;
    int64_t at = 0;
    ilist *L[4];
    rc = atree_build(n, pos, leaf_max, max_level, lo, size, &t);
    if (rc) {
        atree_free(&t);
        return rc;
    }
    for (b = 0; b < t.nbox; ++b) {
        const abox *x = t.box + b;
        int64_t *o = box_out + 8 * (int64_t)b;
        o[0] = x->l;
        o[1] = x->ix;
        o[2] = x->iy;
        o[3] = x->iz;
        o[4] = x->start;
        o[5] = x->end;
        o[6] = x->parent;
        o[7] = x->leaf;
    }
    memcpy(order_out, t.order, sizeof(int64_t) * (size_t)n);
    L[0] = t.U;
    L[1] = t.V;
    L[2] = t.W;
    L[3] = t.X;
    for (w = 0; w < 4; ++w)
        for (b = 0; b < t.nbox; ++b) {
            lst_start[(int64_t)w * (t.nbox + 1) + b] = at;
            for (k = 0; k < L[w][b].n; ++k) lst_items[at++] = L[w][b].v[k];
            lst_start[(int64_t)w * (t.nbox + 1) + b + 1] = at;
        }
    atree_free(&t);
    return ORACLE_OK;
}

/* The adaptive FMM: P2M at the leaves, M2M upward, M2L over V and P2L over X
 * into every box, L2L downward, L2P and M2P over W at the leaves, P2P over U.
 * Outputs per particle in input order; near = P2P, far = everything else. */
int oracle_fmm_adaptive(int64_t n, const double *pos, const double *q, int p, int leaf_max,
                        int max_level, const double *lo, double size, double *phi_near,
                        double *E_near, double *phi_far, double *E_far, int64_t *info_out)
{
    atree t;
    mindex mp, md, mg;
    int rc, b, l;
    double *M = NULL, *Lc = NULL;
    int *sumidx = NULL;
    int64_t i;
    if (n < 1 || p < 1 || p > 30 || leaf_max < 1 || max_level < 0 || max_level > 10 || !(size > 0))
        return ORACLE_EINVAL;
    if (check_domain(n, pos, lo, size)) return ORACLE_EDOMAIN;
    rc = atree_build(n, pos, leaf_max, max_level, lo, size, &t);
    if (rc) {
        atree_free(&t);
        return rc;
    }
    if (mindex_init(&mp, p - 1) || mindex_init(&md, 2 * p - 2) || mindex_init(&mg, p)) return ORACLE_ENOMEM;
    M = (double *)calloc((size_t)t.nbox * mp.n, sizeof(double));
    Lc = (double *)calloc((size_t)t.nbox * mp.n, sizeof(double));
    sumidx = m2l_sum_table(&mp, &md);
    if (!M || !Lc || !sumidx) return ORACLE_ENOMEM;
    for (i = 0; i < n; ++i) {
        phi_near[i] = phi_far[i] = 0.0;
        E_near[3 * i] = E_near[3 * i + 1] = E_near[3 * i + 2] = 0.0;
        E_far[3 * i] = E_far[3 * i + 1] = E_far[3 * i + 2] = 0.0;
    }
    /* P2M at the leaves, M2M from the deepest level up */
    for (l = t.depth; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 16)
        for (b = t.lev_first[l]; b < t.lev_first[l] + t.lev_count[l]; ++b) {
            const abox *x = t.box + b;
            double c[3];
            int k;
            abox_centre(x, lo, size, c);
            if (x->leaf) {
                p2m(&mp, x->end - x->start, t.order + x->start, pos, q, c, M + (size_t)b * mp.n);
                continue;
            }
            for (k = 0; k < 8; ++k) {
                double c1[3];
                if (x->child[k] < 0) continue;
                abox_centre(t.box + x->child[k], lo, size, c1);
                m2m(&mp, M + (size_t)x->child[k] * mp.n, c1, c, M + (size_t)b * mp.n);
            }
        }
    }
    /* M2L over V and P2L over X into every box */
#pragma omp parallel for schedule(dynamic, 4)
    for (b = 0; b < t.nbox; ++b) {
        const abox *x = t.box + b;
        double ct[3], *dG = (double *)malloc(sizeof(double) * md.n);
        int k;
        int64_t j;
        abox_centre(x, lo, size, ct);
        for (k = 0; k < t.V[b].n; ++k) {
            double cs[3], d[3];
            abox_centre(t.box + t.V[b].v[k], lo, size, cs);
            d[0] = ct[0] - cs[0];
            d[1] = ct[1] - cs[1];
            d[2] = ct[2] - cs[2];
            derivs(&md, d, dG);
            m2l(&mp, sumidx, M + (size_t)t.V[b].v[k] * mp.n, dG, Lc + (size_t)b * mp.n);
        }
        for (k = 0; k < t.X[b].n; ++k) {
            const abox *s = t.box + t.X[b].v[k];
            for (j = s->start; j < s->end; ++j) {
                int64_t jp = t.order[j];
                double d[3] = {ct[0] - pos[3 * jp], ct[1] - pos[3 * jp + 1], ct[2] - pos[3 * jp + 2]};
                int a;
                derivs(&mp, d, dG);
                for (a = 0; a < mp.n; ++a) {
                    const int *bb = mp.k + 3 * a;
                    Lc[(size_t)b * mp.n + a] += q[jp] * dG[a] / (fact(bb[0]) * fact(bb[1]) * fact(bb[2]));
                }
            }
        }
        free(dG);
    }
    /* L2L from the root down */
    for (l = 1; l <= t.depth; ++l) {
#pragma omp parallel for schedule(dynamic, 16)
        for (b = t.lev_first[l]; b < t.lev_first[l] + t.lev_count[l]; ++b) {
            double c1[3], c2[3];
            abox_centre(t.box + t.box[b].parent, lo, size, c1);
            abox_centre(t.box + b, lo, size, c2);
            l2l(&mp, Lc + (size_t)t.box[b].parent * mp.n, c1, c2, Lc + (size_t)b * mp.n);
        }
    }
    /* at the leaves: L2P, M2P over W, P2P over U */
#pragma omp parallel for schedule(dynamic, 4)
    for (b = 0; b < t.nbox; ++b) {
        const abox *x = t.box + b;
        double c[3], *dG;
        int64_t ii;
        if (!x->leaf) continue;
        abox_centre(x, lo, size, c);
        dG = (double *)malloc(sizeof(double) * mg.n);
        for (ii = x->start; ii < x->end; ++ii) {
            int64_t ip = t.order[ii], j;
            double f, E[3];
            int k, a;
            l2p(&mp, Lc + (size_t)b * mp.n, c, pos + 3 * ip, &f, E);
            for (k = 0; k < t.W[b].n; ++k) {
                const double *Mw = M + (size_t)t.W[b].v[k] * mp.n;
                double cw[3], d[3];
                abox_centre(t.box + t.W[b].v[k], lo, size, cw);
                d[0] = pos[3 * ip] - cw[0];
                d[1] = pos[3 * ip + 1] - cw[1];
                d[2] = pos[3 * ip + 2] - cw[2];
                derivs(&mg, d, dG);
                for (a = 0; a < mp.n; ++a) {
                    const int *al = mp.k + 3 * a;
                    double sg = (mp.deg[a] & 1) ? -1.0 : 1.0;
                    f += sg * Mw[a] * dG[mi(&mg, al[0], al[1], al[2])];
                    E[0] -= sg * Mw[a] * dG[mi(&mg, al[0] + 1, al[1], al[2])];
                    E[1] -= sg * Mw[a] * dG[mi(&mg, al[0], al[1] + 1, al[2])];
                    E[2] -= sg * Mw[a] * dG[mi(&mg, al[0], al[1], al[2] + 1)];
                }
            }
            phi_far[ip] = f;
            E_far[3 * ip] = E[0];
            E_far[3 * ip + 1] = E[1];
            E_far[3 * ip + 2] = E[2];
            f = E[0] = E[1] = E[2] = 0.0;
            for (k = 0; k < t.U[b].n; ++k) {
                const abox *s = t.box + t.U[b].v[k];
                for (j = s->start; j < s->end; ++j) {
                    int64_t jp = t.order[j];
                    double d0, d1, d2, r2, r;
                    if (jp == ip) continue;
                    d0 = pos[3 * ip] - pos[3 * jp];
                    d1 = pos[3 * ip + 1] - pos[3 * jp + 1];
                    d2 = pos[3 * ip + 2] - pos[3 * jp + 2];
                    r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    if (r2 == 0.0) continue;
                    r = sqrt(r2);
                    f += q[jp] / r;
                    E[0] += q[jp] * d0 / (r2 * r);
                    E[1] += q[jp] * d1 / (r2 * r);
                    E[2] += q[jp] * d2 / (r2 * r);
                }
            }
            phi_near[ip] = f;
            E_near[3 * ip] = E[0];
            E_near[3 * ip + 1] = E[1];
            E_near[3 * ip + 2] = E[2];
        }
        free(dG);
    }
    if (info_out) {
        int nleaf = 0;
        for (b = 0; b < t.nbox; ++b) nleaf += t.box[b].leaf;
        info_out[0] = t.nbox;
        info_out[1] = nleaf;
        info_out[2] = t.depth;
    }
    free(M);
    free(Lc);
    free(sumidx);
    mindex_free(&mp);
    mindex_free(&md);
    mindex_free(&mg);
    atree_free(&t);
    return ORACLE_OK;
}
