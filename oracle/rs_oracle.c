/*
 * FP64 CPU oracle for ray-traced Gaussian rendering (RaySplats,
 * arXiv 2501.19196). TEST INFRASTRUCTURE ONLY: nothing in the product path
 * may link, load or call this file. Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark use it.
 *
 * It is deliberately plain and slow: every ray is tested against every
 * Gaussian, all hits are sorted, then composited. It shares no code, header
 * or constant with the HIP library.
 *
 * Paper references (sections, equations, propositions, appendices):
 *   Eq. 1-2      scene G = {(N(m_i, Sigma_i), opacity_i, c_i)}, Sigma = R S S^T R^T
 *   Eq. 3        front-to-back alpha compositing C = sum c_i a_i prod_{j<i}(1 - a_j)
 *   Sec. 3 "Intersection": confidence ellipsoid (x-m)^T Sigma^-1 (x-m) = Q; the
 *                hit point is the nearer intersection; a ray misses when the
 *                line misses the ellipsoid or that nearer root is negative
 *   Prop. 1 / App. A.1  stable nearer root t1 (Viete branch for <o',d'> < 0)
 *   Prop. 2 / App. A.2  alpha = opacity * exp(-1/2 * squared whitened distance
 *                between the line and the origin)
 *   Sec. 3 "Color Aggregation": at most K_max Gaussians per ray; rays stop
 *                once the transmittance falls below eps1
 *   App. A.3-A.6 gradients; A.6 quaternion -> rotation and dR/dq matrices
 *
 * Readings where the paper is silent or garbled (also listed in the design doc):
 *   - Prop. 1 main text drops <d',d'> under the square root; the appendix
 *     form sqrt(<d',d'> (Q - h^2)) is used.
 *   - sgn(0) = +1 in t*.
 *   - A.2 prints the exponent without the square; the squared distance h^2
 *     is used (A.2's own Mahalanobis quadratic and A.6's inner-product
 *     expansion are squared).
 *   - Sort key: nearer root t1, ties broken by Gaussian index ascending.
 *   - Composite the hit, then stop if T < eps1 (strict); at most K_max hits;
 *     the background enters as + T_final * bg.
 *   - The matrices A.6 labels dR^T/dq equal dR/dq entry for entry; they are
 *     used as dR/dq and transposed where d(R^T x)/dq is formed.
 *   - A.6 writes the scale derivative with e_y e_y^T for the x component and
 *     for a sigmoid-activated scale; here the scale is the activated world
 *     scale, so d(1/s_x)/ds_x = -1/s_x^2 and the projector is e_x e_x^T.
 *   - The adjoint is the exact derivative of the truncated forward (the hits
 *     actually composited); A.4/A.5's front-to-back recursion gives the same
 *     value and is used by the tests as a pin. Here the division-free
 *     back-to-front form is used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double Q;              /* chi^2(3) quantile of the confidence ellipsoid */
    double eps1;           /* transmittance threshold */
    double t_min;          /* a hit needs t1 >= t_min */
    int64_t max_hits;      /* K_max; 0 = unbounded */
    double bg[3];          /* background colour */
    int32_t zero_colour;   /* 1: every Gaussian colour is taken as 0 (transmittance rays) */
} orc_params;

typedef struct {
    int64_t n;
    const float *mean, *scale, *quat, *opacity, *rgb;
} orc_scene;

typedef struct {
    int64_t n;
    const float *origin, *dir;
    const double *t_max;   /* optional [n]: hits need t1 < t_max; NULL = +inf */
    const double *bg;      /* optional [n][3]: per-ray background; NULL = params bg */
} orc_rays;

typedef struct {
    double t1, h2, alpha;
    int64_t idx;
} orc_hit;

/* ---------------------------------------------------------------------- */
/* Rotation of a (not necessarily unit) quaternion q = (r, i, j, k) as
 * written in App. A.6 (s = 2 / |q|^2). */
static void rotation(const double q[4], double R[3][3])
{
    double a = q[0], b = q[1], c = q[2], d = q[3];
    double s = 2.0 / (a * a + b * b + c * c + d * d);
    double bs = b * s, cs = c * s, ds = d * s;
    double ab = a * bs, ac = a * cs, ad = a * ds;
    double bb = b * bs, bc = b * cs, bd = b * ds;
    double cc = c * cs, cd = c * ds, dd = d * ds;
    R[0][0] = 1.0 - cc - dd; R[0][1] = bc - ad;       R[0][2] = bd + ac;
    R[1][0] = bc + ad;       R[1][1] = 1.0 - bb - dd; R[1][2] = cd - ab;
    R[2][0] = bd - ac;       R[2][1] = cd + ab;       R[2][2] = 1.0 - bb - cc;
}

/* The four matrices of App. A.6 (printed there under the label dR^T/dq;
 * they are dR/dq). D[k] is the derivative with respect to q[k]. */
static void rotation_derivs(const double q[4], double D[4][3][3])
{
    double a = q[0], b = q[1], c = q[2], d = q[3];
    double s = 2.0 / (a * a + b * b + c * c + d * d);
    double aa = a * a * s, bb = b * b * s, cc = c * c * s, dd = d * d * s;
    double ab = a * b * s, cd = c * d * s;
    /* d/dq_r */
    D[0][0][0] = s * a * ((1 - aa) + (1 - bb));
    D[0][0][1] = s * (-d * (1 - aa) - ab * c);
    D[0][0][2] = s * (c * (1 - aa) - ab * d);
    D[0][1][0] = s * (d * (1 - aa) - ab * c);
    D[0][1][1] = s * a * ((1 - aa) + (1 - cc));
    D[0][1][2] = s * (-b * (1 - aa) - a * cd);
    D[0][2][0] = s * (-c * (1 - aa) - ab * d);
    D[0][2][1] = s * (b * (1 - aa) - a * cd);
    D[0][2][2] = s * a * ((1 - aa) + (1 - dd));
    /* d/dq_i */
    D[1][0][0] = s * b * ((1 - bb) + (1 - aa));
    D[1][0][1] = s * (c * (1 - bb) - (-ab * d));
    D[1][0][2] = s * (d * (1 - bb) - ab * c);
    D[1][1][0] = s * (c * (1 - bb) - ab * d);
    D[1][1][1] = -s * b * ((1 - bb) + (1 - dd));
    D[1][1][2] = s * (-a * (1 - bb) - b * cd);
    D[1][2][0] = s * (d * (1 - bb) - (-ab * c));
    D[1][2][1] = s * (a * (1 - bb) - b * cd);
    D[1][2][2] = -s * b * ((1 - bb) + (1 - cc));
    /* d/dq_j */
    D[2][0][0] = -s * c * ((1 - cc) + (1 - dd));
    D[2][0][1] = s * (b * (1 - cc) - (-a * cd));
    D[2][0][2] = s * (a * (1 - cc) - b * cd);
    D[2][1][0] = s * (b * (1 - cc) - a * cd);
    D[2][1][1] = s * c * ((1 - cc) + (1 - aa));
    D[2][1][2] = s * (d * (1 - cc) - (-ab * c));
    D[2][2][0] = s * (-a * (1 - cc) - b * cd);
    D[2][2][1] = s * (d * (1 - cc) - ab * c);
    D[2][2][2] = -s * c * ((1 - cc) + (1 - bb));
    /* d/dq_k */
    D[3][0][0] = -s * d * ((1 - dd) + (1 - cc));
    D[3][0][1] = s * (-a * (1 - dd) - b * cd);
    D[3][0][2] = s * (b * (1 - dd) - a * cd);
    D[3][1][0] = s * (a * (1 - dd) - b * cd);
    D[3][1][1] = -s * d * ((1 - dd) + (1 - bb));
    D[3][1][2] = s * (c * (1 - dd) - (-ab * d));
    D[3][2][0] = s * (b * (1 - dd) - (-a * cd));
    D[3][2][1] = s * (c * (1 - dd) - ab * d);
    D[3][2][2] = s * d * ((1 - dd) + (1 - aa));
}

/* Whitened ray of Prop. 1: o' = S^-1 R^T (o - m), d' = S^-1 R^T d. */
typedef struct {
    double R[3][3];
    double x[3];      /* o - m */
    double op[3], dp[3];
    double a, b;      /* <d',d'>, <o',d'> */
    double h2;        /* squared whitened distance between the line and the origin */
    double t1;        /* nearer root (valid when h2 <= Q) */
} orc_geom;

static void whiten(const orc_scene *sc, int64_t i, const double o[3], const double d[3], orc_geom *g)
{
    double q[4], m[3], s[3];
    for (int k = 0; k < 4; ++k) q[k] = sc->quat[4 * i + k];
    for (int k = 0; k < 3; ++k) { m[k] = sc->mean[3 * i + k]; s[k] = sc->scale[3 * i + k]; }
    rotation(q, g->R);
    for (int k = 0; k < 3; ++k) g->x[k] = o[k] - m[k];
    for (int k = 0; k < 3; ++k) {
        /* row k of R^T is column k of R */
        double rx = g->R[0][k] * g->x[0] + g->R[1][k] * g->x[1] + g->R[2][k] * g->x[2];
        double rd = g->R[0][k] * d[0] + g->R[1][k] * d[1] + g->R[2][k] * d[2];
        g->op[k] = rx / s[k];
        g->dp[k] = rd / s[k];
    }
    g->a = g->dp[0] * g->dp[0] + g->dp[1] * g->dp[1] + g->dp[2] * g->dp[2];
    g->b = g->op[0] * g->dp[0] + g->op[1] * g->dp[1] + g->op[2] * g->dp[2];
    /* Prop. 2 / App. A.2: || o' - d^ <o', d^> ||^2 with d^ = d'/||d'|| */
    double nd = sqrt(g->a);
    double dh[3] = {g->dp[0] / nd, g->dp[1] / nd, g->dp[2] / nd};
    double pr = g->op[0] * dh[0] + g->op[1] * dh[1] + g->op[2] * dh[2];
    double h2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = g->op[k] - dh[k] * pr;
        h2 += e * e;
    }
    g->h2 = h2;
}

/* Prop. 1 (appendix form): nearer root of <o'+t d', o'+t d'> = Q. */
static double nearer_root(const orc_geom *g, double Q)
{
    double root = sqrt(g->a * (Q - g->h2));
    if (g->b >= 0.0) /* sgn(0) read as +1 */
        return (-g->b - root) / g->a;
    double tstar = (-g->b + root) / g->a;
    double oo = g->op[0] * g->op[0] + g->op[1] * g->op[1] + g->op[2] * g->op[2];
    return (oo - Q) / (g->a * tstar);
}

/* Ray / Gaussian test (Sec. 3, Prop. 1, Prop. 2). Returns 1 on a hit. */
static int intersect(const orc_scene *sc, int64_t i, const double o[3], const double d[3],
                     double Q, double t_min, double t_max, orc_geom *g)
{
    whiten(sc, i, o, d, g);
    if (!(g->h2 <= Q)) return 0;
    g->t1 = nearer_root(g, Q);
    return g->t1 >= t_min && g->t1 < t_max;
}

static int cmp_hit(const void *pa, const void *pb)
{
    const orc_hit *a = (const orc_hit *)pa, *b = (const orc_hit *)pb;
    if (a->t1 < b->t1) return -1;
    if (a->t1 > b->t1) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Every Gaussian hit by one ray, sorted by (t1, index). Caller frees. */
static int64_t collect(const orc_scene *sc, const double o[3], const double d[3], const orc_params *p,
                       double t_max, orc_hit **out)
{
    int64_t cap = 64, n = 0;
    orc_hit *h = (orc_hit *)malloc(sizeof(orc_hit) * cap);
    for (int64_t i = 0; i < sc->n; ++i) {
        orc_geom g;
        if (!intersect(sc, i, o, d, p->Q, p->t_min, t_max, &g)) continue;
        if (n == cap) {
            cap *= 2;
            h = (orc_hit *)realloc(h, sizeof(orc_hit) * cap);
        }
        h[n].t1 = g.t1;
        h[n].h2 = g.h2;
        h[n].alpha = (double)sc->opacity[i] * exp(-0.5 * g.h2);
        h[n].idx = i;
        ++n;
    }
    qsort(h, (size_t)n, sizeof(orc_hit), cmp_hit);
    *out = h;
    return n;
}

static void colour_of(const orc_scene *sc, const orc_params *p, int64_t i, double c[3])
{
    for (int k = 0; k < 3; ++k) c[k] = p->zero_colour ? 0.0 : (double)sc->rgb[3 * i + k];
}

/* Eq. 3 with the K_max and eps1 rules: returns the number L of composited hits. */
static int64_t composite(const orc_scene *sc, const orc_params *p, const orc_hit *h, int64_t n,
                         const double bg[3], double out[3], double *T_out)
{
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t L = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (p->max_hits > 0 && L >= p->max_hits) break;
        double c[3];
        colour_of(sc, p, h[k].idx, c);
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * h[k].alpha * c[ch];
        T *= (1.0 - h[k].alpha);
        ++L;
        if (T < p->eps1) break;
    }
    for (int ch = 0; ch < 3; ++ch) out[ch] = C[ch] + T * bg[ch];
    *T_out = T;
    return L;
}

static void ray_of(const orc_rays *r, int64_t k, double o[3], double d[3])
{
    for (int c = 0; c < 3; ++c) {
        o[c] = r->origin[3 * k + c];
        d[c] = r->dir[3 * k + c];
    }
}

static const double *bg_of(const orc_rays *r, const orc_params *p, int64_t k)
{
    return r->bg ? r->bg + 3 * k : p->bg;
}

static double tmax_of(const orc_rays *r, int64_t k)
{
    return r->t_max ? r->t_max[k] : INFINITY;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ---------------------------------------------------------------------- */
/* Public entry points (ctypes). */

int orc_version(void) { return 3; }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_rotation(const double q[4], double R[9])
{
    double M[3][3];
    rotation(q, M);
    memcpy(R, M, sizeof(M));
}

void orc_rotation_derivs(const double q[4], double D[36])
{
    double M[4][3][3];
    rotation_derivs(q, M);
    memcpy(D, M, sizeof(M));
}

/* One ray against one Gaussian (arrays of length 1 scene index i). Writes
 * t1, h2 (t1 = NAN when the line misses the ellipsoid). Returns 1 on a hit. */
int orc_intersect(const orc_scene *sc, int64_t i, const float o32[3], const float d32[3],
                  double Q, double t_min, double *t1, double *h2)
{
    double o[3] = {o32[0], o32[1], o32[2]}, d[3] = {d32[0], d32[1], d32[2]};
    orc_geom g;
    whiten(sc, i, o, d, &g);
    *h2 = g.h2;
    if (!(g.h2 <= Q)) {
        *t1 = NAN;
        return 0;
    }
    g.t1 = nearer_root(&g, Q);
    *t1 = g.t1;
    return g.t1 >= t_min;
}

/* Sorted hits of ray k: writes up to cap entries; returns the total count. */
int64_t orc_ray_hits(const orc_scene *sc, const orc_rays *r, int64_t k, const orc_params *p,
                     int64_t cap, int64_t *idx, double *t1, double *h2, double *alpha)
{
    double o[3], d[3];
    ray_of(r, k, o, d);
    orc_hit *h;
    int64_t n = collect(sc, o, d, p, tmax_of(r, k), &h);
    for (int64_t j = 0; j < n && j < cap; ++j) {
        idx[j] = h[j].idx;
        t1[j] = h[j].t1;
        h2[j] = h[j].h2;
        alpha[j] = h[j].alpha;
    }
    free(h);
    return n;
}

/* Forward render: colour, final transmittance and composited count per ray. */
int orc_render_fwd(const orc_scene *sc, const orc_rays *r, const orc_params *p,
                   double *out_rgb, double *out_T, int64_t *out_L, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < r->n; ++k) {
        double o[3], d[3], T;
        ray_of(r, k, o, d);
        orc_hit *h;
        int64_t n = collect(sc, o, d, p, tmax_of(r, k), &h);
        int64_t L = composite(sc, p, h, n, bg_of(r, p, k), out_rgb + 3 * k, &T);
        if (out_T) out_T[k] = T;
        if (out_L) out_L[k] = L;
        free(h);
    }
    return 0;
}

/* The composited hits of every ray in compositing order (Eq. 3 with the K_max
 * and eps1 rules): ids[k][0..cap) holds the first min(L, cap) Gaussian indices,
 * then -1; L_out[k] = L. */
int orc_render_lists(const orc_scene *sc, const orc_rays *r, const orc_params *p, int64_t cap, int64_t *ids,
                     int64_t *L_out, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < r->n; ++k) {
        double o[3], d[3], T, C[3];
        ray_of(r, k, o, d);
        orc_hit *h;
        int64_t n = collect(sc, o, d, p, tmax_of(r, k), &h);
        int64_t L = composite(sc, p, h, n, bg_of(r, p, k), C, &T);
        for (int64_t j = 0; j < cap; ++j) ids[k * cap + j] = j < L ? h[j].idx : -1;
        L_out[k] = L;
        free(h);
    }
    return 0;
}

/* dC/dalpha_k and dC/dc_k weights for one composited list (division-free,
 * back to front). grad: upstream dL/dC (3). Writes g_alpha[k] = <grad, dC/dalpha_k>
 * and w[k] = alpha_k T_k (so dL/dc_k = grad * w[k]). Returns L. */
static int64_t adjoint_list(const orc_scene *sc, const orc_params *p, const orc_hit *h, int64_t n,
                            const double bg[3], const double grad[3], double *g_alpha, double *w)
{
    double T = 1.0, Tfinal;
    int64_t L = 0;
    /* forward sweep for T_k */
    double *Tk = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t k = 0; k < n; ++k) {
        if (p->max_hits > 0 && L >= p->max_hits) break;
        Tk[k] = T;
        T *= (1.0 - h[k].alpha);
        ++L;
        if (T < p->eps1) break;
    }
    Tfinal = T;
    (void)Tfinal;
    /* back to front with the suffix S (colour seen behind hit k) */
    double S[3] = {bg[0], bg[1], bg[2]};
    for (int64_t k = L - 1; k >= 0; --k) {
        double c[3];
        colour_of(sc, p, h[k].idx, c);
        double ga = 0.0;
        for (int ch = 0; ch < 3; ++ch) ga += grad[ch] * Tk[k] * (c[ch] - S[ch]);
        g_alpha[k] = ga;
        w[k] = h[k].alpha * Tk[k];
        for (int ch = 0; ch < 3; ++ch) S[ch] = c[ch] * h[k].alpha + (1.0 - h[k].alpha) * S[ch];
    }
    free(Tk);
    return L;
}

/* Per-hit dC/dalpha (one channel vector form) for ray k, for pinning the
 * adjoint against the paper's A.4/A.5 recursion. Writes up to cap entries of
 * dC/dalpha_k for each channel ([cap][3]). Returns L. */
int64_t orc_ray_dC_dalpha(const orc_scene *sc, const orc_rays *r, int64_t k, const orc_params *p,
                          int64_t cap, double *dCda)
{
    double o[3], d[3];
    ray_of(r, k, o, d);
    orc_hit *h;
    int64_t n = collect(sc, o, d, p, tmax_of(r, k), &h);
    double *ga = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    int64_t L = 0;
    for (int ch = 0; ch < 3; ++ch) {
        double g[3] = {0, 0, 0};
        g[ch] = 1.0;
        L = adjoint_list(sc, p, h, n, bg_of(r, p, k), g, ga, w);
        for (int64_t j = 0; j < L && j < cap; ++j) dCda[3 * j + ch] = ga[j];
    }
    free(ga);
    free(w);
    free(h);
    return L;
}

/* dh^2/dtheta for one (ray, Gaussian) pair following App. A.6:
 *   dh2 = 2 <p, do'> - 2 (<d',o'>/<d',d'>) <p, dd'>,  p = o' - d' <d',o'>/<d',d'>.
 * Outputs d h^2 / d mean (3), d scale (3), d quat (4). */
static void dh2_dparams(const orc_scene *sc, int64_t i, const orc_geom *g, const double d[3],
                        double dm[3], double ds[3], double dq[4])
{
    double s[3], q[4];
    for (int k = 0; k < 3; ++k) s[k] = sc->scale[3 * i + k];
    for (int k = 0; k < 4; ++k) q[k] = sc->quat[4 * i + k];
    double ba = g->b / g->a;
    double pv[3];
    for (int k = 0; k < 3; ++k) pv[k] = g->op[k] - g->dp[k] * ba;
    /* mean: do'/dm_x = -S^-1 R^T e_x, dd'/dm = 0 */
    for (int x = 0; x < 3; ++x) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += pv[k] * (-g->R[x][k] / s[k]);
        dm[x] = 2.0 * acc;
    }
    /* scale (activated): do'/ds_x = -(1/s_x^2) e_x e_x^T R^T (o - m), likewise d' */
    for (int x = 0; x < 3; ++x) {
        double rx = g->R[0][x] * g->x[0] + g->R[1][x] * g->x[1] + g->R[2][x] * g->x[2];
        double rd = g->R[0][x] * d[0] + g->R[1][x] * d[1] + g->R[2][x] * d[2];
        double dop = -rx / (s[x] * s[x]);
        double ddp = -rd / (s[x] * s[x]);
        ds[x] = 2.0 * pv[x] * dop - 2.0 * ba * pv[x] * ddp;
    }
    /* quaternion: do'/dq = S^-1 (dR/dq)^T (o - m), dd'/dq = S^-1 (dR/dq)^T d */
    double D[4][3][3];
    rotation_derivs(q, D);
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) {
            double rx = D[c][0][k] * g->x[0] + D[c][1][k] * g->x[1] + D[c][2][k] * g->x[2];
            double rd = D[c][0][k] * d[0] + D[c][1][k] * d[1] + D[c][2][k] * d[2];
            acc += 2.0 * pv[k] * (rx / s[k]) - 2.0 * ba * pv[k] * (rd / s[k]);
        }
        dq[c] = acc;
    }
}

static void atomic_add(double *p, double v)
{
#pragma omp atomic
    *p += v;
}

/* Backward render: gradients of sum_k <grad_rgb[k], C_k> with respect to the
 * activated parameters. Outputs are overwritten. d_bg (optional, [n][3])
 * receives dL/d(per-ray background) = grad * T_final. */
int orc_render_bwd(const orc_scene *sc, const orc_rays *r, const orc_params *p, const double *grad_rgb,
                   double *d_mean, double *d_scale, double *d_quat, double *d_opacity, double *d_rgb,
                   double *d_bg, int nthreads)
{
    set_threads(nthreads);
    memset(d_mean, 0, sizeof(double) * 3 * sc->n);
    memset(d_scale, 0, sizeof(double) * 3 * sc->n);
    memset(d_quat, 0, sizeof(double) * 4 * sc->n);
    memset(d_opacity, 0, sizeof(double) * sc->n);
    memset(d_rgb, 0, sizeof(double) * 3 * sc->n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < r->n; ++k) {
        double o[3], d[3];
        ray_of(r, k, o, d);
        const double *g = grad_rgb + 3 * k;
        orc_hit *h;
        int64_t n = collect(sc, o, d, p, tmax_of(r, k), &h);
        double *ga = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
        double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
        int64_t L = adjoint_list(sc, p, h, n, bg_of(r, p, k), g, ga, w);
        double T = 1.0;
        for (int64_t j = 0; j < L; ++j) T *= (1.0 - h[j].alpha);
        if (d_bg)
            for (int ch = 0; ch < 3; ++ch) d_bg[3 * k + ch] = g[ch] * T;
        for (int64_t j = 0; j < L; ++j) {
            int64_t i = h[j].idx;
            if (!p->zero_colour)
                for (int ch = 0; ch < 3; ++ch) atomic_add(&d_rgb[3 * i + ch], g[ch] * w[j]);
            /* alpha = opacity * exp(-h2/2) */
            double e = exp(-0.5 * h[j].h2);
            atomic_add(&d_opacity[i], ga[j] * e);
            double g_h2 = ga[j] * (-0.5 * h[j].alpha);
            orc_geom geo;
            whiten(sc, i, o, d, &geo);
            double dm[3], ds[3], dq[4];
            dh2_dparams(sc, i, &geo, d, dm, ds, dq);
            for (int c = 0; c < 3; ++c) atomic_add(&d_mean[3 * i + c], g_h2 * dm[c]);
            for (int c = 0; c < 3; ++c) atomic_add(&d_scale[3 * i + c], g_h2 * ds[c]);
            for (int c = 0; c < 4; ++c) atomic_add(&d_quat[4 * i + c], g_h2 * dq[c]);
        }
        free(ga);
        free(w);
        free(h);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* The paper's backward variant (Sec. 3 and Sec. 5, second threshold): when a
 * ray stops because its transmittance fell below eps1 after L hits, the
 * forward keeps collecting the next hits j = L+1, L+2, ... (without changing
 * the image) while the transmittance of the collected ones,
 * prod_{k=L+1}^{j-1} (1 - alpha_k), is not below eps2 and the buffer holds
 * fewer than K_max entries. The gradient of the last "meaningful" Gaussian L
 * then sees those hits instead of only the background. Reading: the
 * gradients are those of
 *   E = C_<=L + T_{L+1} R2,  R2 = sum_{j>L} c_j alpha_j prod_{L<k<j} (1 - alpha_k)
 *                              + prod_{L<k<=J} (1 - alpha_k) bg,
 * with the collected set frozen, for the composited Gaussians only; that is
 * the exact adjoint with bg replaced by R2. extra[k] receives J - L and
 * near[k] = 1 when some eps2 decision on a rounded T2 (after at least one
 * collected hit) had |T2 - eps2| <= 1e-3 eps2. */
static int64_t phase2(const orc_scene *sc, const orc_params *p, double eps2, const orc_hit *h, int64_t n,
                      const double bg[3], double R2[3], int *near)
{
    double T = 1.0;
    int64_t L = 0;
    int by_eps = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (p->max_hits > 0 && L >= p->max_hits) break;
        T *= (1.0 - h[k].alpha);
        ++L;
        if (T < p->eps1) {
            by_eps = 1;
            break;
        }
    }
    for (int ch = 0; ch < 3; ++ch) R2[ch] = 0.0;
    double T2 = 1.0;
    int64_t x = 0;
    *near = 0;
    if (by_eps) {
        for (int64_t j = L; j < n; ++j) {
            if (p->max_hits > 0 && L + x >= p->max_hits) break;
            /* before the first collected hit T2 is the exact empty product 1: no rounding */
            if (x > 0 && fabs(T2 - eps2) <= 1e-3 * eps2) *near = 1;
            if (T2 < eps2) break;
            double c[3];
            colour_of(sc, p, h[j].idx, c);
            for (int ch = 0; ch < 3; ++ch) R2[ch] += T2 * h[j].alpha * c[ch];
            T2 *= (1.0 - h[j].alpha);
            ++x;
        }
    }
    for (int ch = 0; ch < 3; ++ch) R2[ch] += T2 * bg[ch];
    return x;
}

int orc_render_bwd_paper(const orc_scene *sc, const orc_rays *r, const orc_params *p, double eps2,
                         const double *grad_rgb, double *d_mean, double *d_scale, double *d_quat, double *d_opacity,
                         double *d_rgb, int32_t *extra, int32_t *near, int nthreads)
{
    set_threads(nthreads);
    memset(d_mean, 0, sizeof(double) * 3 * sc->n);
    memset(d_scale, 0, sizeof(double) * 3 * sc->n);
    memset(d_quat, 0, sizeof(double) * 4 * sc->n);
    memset(d_opacity, 0, sizeof(double) * sc->n);
    memset(d_rgb, 0, sizeof(double) * 3 * sc->n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < r->n; ++k) {
        double o[3], d[3];
        ray_of(r, k, o, d);
        const double *g = grad_rgb + 3 * k;
        orc_hit *h;
        int64_t n = collect(sc, o, d, p, tmax_of(r, k), &h);
        double R2[3];
        int nr = 0;
        int64_t x = phase2(sc, p, eps2, h, n, bg_of(r, p, k), R2, &nr);
        if (extra) extra[k] = (int32_t)x;
        if (near) near[k] = nr;
        double *ga = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
        double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
        int64_t L = adjoint_list(sc, p, h, n, R2, g, ga, w);
        for (int64_t j = 0; j < L; ++j) {
            int64_t i = h[j].idx;
            if (!p->zero_colour)
                for (int ch = 0; ch < 3; ++ch) atomic_add(&d_rgb[3 * i + ch], g[ch] * w[j]);
            double e = exp(-0.5 * h[j].h2);
            atomic_add(&d_opacity[i], ga[j] * e);
            double g_h2 = ga[j] * (-0.5 * h[j].alpha);
            orc_geom geo;
            whiten(sc, i, o, d, &geo);
            double dm[3], ds[3], dq[4];
            dh2_dparams(sc, i, &geo, d, dm, ds, dq);
            for (int c = 0; c < 3; ++c) atomic_add(&d_mean[3 * i + c], g_h2 * dm[c]);
            for (int c = 0; c < 3; ++c) atomic_add(&d_scale[3 * i + c], g_h2 * ds[c]);
            for (int c = 0; c < 4; ++c) atomic_add(&d_quat[4 * i + c], g_h2 * dq[c]);
        }
        free(ga);
        free(w);
        free(h);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Acceptance alternatives. A float32 renderer may legitimately differ from
 * this oracle where the decision depends on a quantity within its rounding
 * error: (i) membership when |h2 - Q| <= dh * Q, (ii) membership when
 * |t1 - t_min| <= dt * max(|t1|, 1), (iii) the order of two neighbouring hits
 * with |t1_a - t1_b| <= dt * max(|t1|, 1), (iv) the eps1 stop when
 * |T - eps1| <= dT * eps1. For one ray, enumerate every combination of these
 * events among the hits that matter and return the resulting colours.
 * Returns the number of alternatives written (<= cap), or -1 when more than
 * max_events events occur (the pixel is then reported as unresolved). */

typedef struct {
    const orc_scene *sc;
    const orc_params *p;
    const double *bg;
    double dT;
    double *out;
    int64_t cap, nout;
    int events;
    int max_events;
} alt_ctx;

static void alt_composite(alt_ctx *ctx, const orc_hit *h, int64_t n, int64_t k0, double T0, const double C0[3],
                          int64_t L0, int events)
{
    double T = T0, C[3] = {C0[0], C0[1], C0[2]};
    int64_t L = L0;
    for (int64_t k = k0; k < n; ++k) {
        if (ctx->p->max_hits > 0 && L >= ctx->p->max_hits) break;
        double c[3];
        colour_of(ctx->sc, ctx->p, h[k].idx, c);
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * h[k].alpha * c[ch];
        T *= (1.0 - h[k].alpha);
        ++L;
        int stop = T < ctx->p->eps1;
        if (fabs(T - ctx->p->eps1) <= ctx->dT * ctx->p->eps1 && events < ctx->max_events) {
            /* branch: take the other decision too */
            if (stop)
                alt_composite(ctx, h, n, k + 1, T, C, L, events + 1);
            else {
                if (ctx->nout < ctx->cap)
                    for (int ch = 0; ch < 3; ++ch) ctx->out[3 * ctx->nout + ch] = C[ch] + T * ctx->bg[ch];
                ctx->nout++;
            }
            if (events + 1 > ctx->events) ctx->events = events + 1;
        }
        if (stop) break;
    }
    if (ctx->nout < ctx->cap)
        for (int ch = 0; ch < 3; ++ch) ctx->out[3 * ctx->nout + ch] = C[ch] + T * ctx->bg[ch];
    ctx->nout++;
}

int64_t orc_ray_alternatives(const orc_scene *sc, const orc_rays *r, int64_t k, const orc_params *p,
                             double dh, double dt, double dT, int max_events, int64_t cap, double *out_rgb)
{
    double o[3], d[3];
    ray_of(r, k, o, d);
    double tmax = tmax_of(r, k);
    /* all candidates, including near misses within the membership window */
    int64_t capn = 64, n = 0;
    orc_hit *h = (orc_hit *)malloc(sizeof(orc_hit) * capn);
    int64_t *amb = (int64_t *)malloc(sizeof(int64_t) * capn);
    for (int64_t i = 0; i < sc->n; ++i) {
        orc_geom g;
        whiten(sc, i, o, d, &g);
        if (!(g.h2 <= p->Q * (1.0 + dh))) continue;
        double t1 = g.h2 <= p->Q ? nearer_root(&g, p->Q) : -g.b / g.a;
        int inside = g.h2 <= p->Q && t1 >= p->t_min && t1 < tmax;
        double tol = dt * fmax(fabs(t1), 1.0);
        int near_q = fabs(g.h2 - p->Q) <= dh * p->Q;
        int near_t = fabs(t1 - p->t_min) <= tol || (isfinite(tmax) && fabs(t1 - tmax) <= tol);
        if (!inside && !near_q && !near_t) continue;
        if (!inside && t1 < p->t_min - tol) continue;
        if (n == capn) {
            capn *= 2;
            h = (orc_hit *)realloc(h, sizeof(orc_hit) * capn);
            amb = (int64_t *)realloc(amb, sizeof(int64_t) * capn);
        }
        h[n].t1 = t1;
        h[n].h2 = g.h2;
        h[n].alpha = (double)sc->opacity[i] * exp(-0.5 * fmin(g.h2, p->Q * (1.0 + dh)));
        h[n].idx = i;
        /* amb: 0 certain member, 1 uncertain membership; sign: nominal in/out */
        amb[n] = (near_q || near_t) ? (inside ? 1 : 2) : 0;
        ++n;
    }
    /* sort hits together with their flags */
    orc_hit *tmp = (orc_hit *)malloc(sizeof(orc_hit) * (n > 0 ? n : 1));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    memcpy(tmp, h, sizeof(orc_hit) * n);
    for (int64_t j = 0; j < n; ++j) tmp[j].idx = j; /* sort positions */
    for (int64_t j = 0; j < n; ++j) tmp[j].h2 = (double)h[j].idx;
    /* sort by (t1, original idx) */
    for (int64_t j = 1; j < n; ++j) {
        orc_hit v = tmp[j];
        int64_t z = j - 1;
        while (z >= 0 && (tmp[z].t1 > v.t1 || (tmp[z].t1 == v.t1 && tmp[z].h2 > v.h2))) {
            tmp[z + 1] = tmp[z];
            --z;
        }
        tmp[z + 1] = v;
    }
    for (int64_t j = 0; j < n; ++j) order[j] = tmp[j].idx;
    orc_hit *hs = (orc_hit *)malloc(sizeof(orc_hit) * (n > 0 ? n : 1));
    int64_t *as = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) {
        hs[j] = h[order[j]];
        as[j] = amb[order[j]];
    }
    /* events among the hits: membership flags and near-tied neighbours;
     * only the ones before the nominal stop (plus one) matter */
    int64_t ev_pos[16];
    int ev_kind[16];
    int n_ev = 0;
    int too_many = 0;
    {
        /* nominal stop position */
        double T = 1.0;
        int64_t L = 0, lim = n;
        for (int64_t j = 0; j < n; ++j) {
            if (as[j] == 2) continue;
            if (p->max_hits > 0 && L >= p->max_hits) { lim = j; break; }
            T *= (1.0 - hs[j].alpha);
            ++L;
            if (T < p->eps1 * (1.0 - dT)) { lim = j + 1; break; }
        }
        for (int64_t j = 0; j < n && j <= lim + 1; ++j) {
            if (as[j] != 0) {
                if (n_ev < 16) { ev_pos[n_ev] = j; ev_kind[n_ev] = 0; }
                ++n_ev;
            }
            if (j + 1 < n) {
                double tol = dt * fmax(fabs(hs[j].t1), 1.0);
                if (fabs(hs[j + 1].t1 - hs[j].t1) <= tol) {
                    if (n_ev < 16) { ev_pos[n_ev] = j; ev_kind[n_ev] = 1; }
                    ++n_ev;
                }
            }
        }
    }
    if (n_ev > max_events) too_many = 1;
    int64_t result = -1;
    if (!too_many) {
        alt_ctx ctx = {sc, p, bg_of(r, p, k), dT, out_rgb, cap, 0, 0, max_events};
        orc_hit *lst = (orc_hit *)malloc(sizeof(orc_hit) * (n > 0 ? n : 1));
        for (int mask = 0; mask < (1 << n_ev); ++mask) {
            /* apply swaps first, then memberships */
            int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
            orc_hit *work = (orc_hit *)malloc(sizeof(orc_hit) * (n > 0 ? n : 1));
            memcpy(work, hs, sizeof(orc_hit) * n);
            for (int64_t j = 0; j < n; ++j) inc[j] = as[j] != 2;
            for (int e = 0; e < n_ev; ++e) {
                if (!(mask & (1 << e))) continue;
                int64_t j = ev_pos[e];
                if (ev_kind[e] == 0) {
                    inc[j] = !inc[j];
                } else {
                    orc_hit t = work[j];
                    work[j] = work[j + 1];
                    work[j + 1] = t;
                    int64_t ti = inc[j];
                    inc[j] = inc[j + 1];
                    inc[j + 1] = ti;
                }
            }
            int64_t m = 0;
            for (int64_t j = 0; j < n; ++j)
                if (inc[j]) lst[m++] = work[j];
            double C0[3] = {0, 0, 0};
            alt_composite(&ctx, lst, m, 0, 1.0, C0, 0, n_ev);
            free(inc);
            free(work);
        }
        free(lst);
        result = ctx.nout;
    }
    free(h);
    free(amb);
    free(tmp);
    free(order);
    free(hs);
    free(as);
    return result;
}

/* orc_ray_alternatives for many rays at once (OpenMP over rays). out_n[k] is
 * the count for ray k (or -1); out_rgb is [n][cap][3]. */
void orc_alternatives_batch(const orc_scene *sc, const orc_rays *r, const orc_params *p, double dh, double dt,
                            double dT, int max_events, int64_t cap, int64_t *out_n, double *out_rgb, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < r->n; ++k)
        out_n[k] = orc_ray_alternatives(sc, r, k, p, dh, dt, dT, max_events, cap, out_rgb + 3 * cap * k);
}
