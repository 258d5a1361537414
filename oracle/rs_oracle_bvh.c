/*
 * CPU reference for the BVH build (TEST INFRASTRUCTURE ONLY; the product path
 * never links it). The paper traverses with a vendor ray-tracing API (Sec. 5)
 * and specifies no acceleration structure; the structure checked here is the
 * linear BVH of Karras (HPG 2012) over 30-bit Morton codes of the Gaussian
 * means, defined bit-exactly as follows.
 *
 *   lo, hi   float32 min / max of the means per axis
 *   scale_k  = 1024 / (hi_k - lo_k) (float32, correctly rounded), 0 if hi_k == lo_k
 *   q_k      = min(uint32((c_k - lo_k) * scale_k), 1023), float32 operations
 *              without contraction, truncation toward zero
 *   code     = bit interleave of (q_x, q_y, q_z), x in the highest position
 *
 * The sort is a stable sort of the codes (ties keep the input order). The
 * topology is the unique binary radix tree over the augmented keys
 * (code, sorted position): this file builds it top down, serially; internal
 * node i covers a key range with i at one end, its children are the split
 * position g and g + 1 (a leaf when the child range is a single key).
 *
 * The default builder of the library is PLOC (at the end of this file); the
 * linear BVH above is its alternative. Must be compiled with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint32_t spread10(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

void orc_morton_codes(int64_t n, const float *mean, uint32_t *codes, float lo_out[3], float hi_out[3])
{
    float lo[3], hi[3], sc[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = n > 0 ? mean[k] : 0.0f;
        hi[k] = lo[k];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            float c = mean[3 * i + k];
            if (c < lo[k]) lo[k] = c;
            if (c > hi[k]) hi[k] = c;
        }
    for (int k = 0; k < 3; ++k) {
        volatile float ext = hi[k] - lo[k];
        sc[k] = (hi[k] == lo[k]) ? 0.0f : 1024.0f / ext;
        lo_out[k] = lo[k];
        hi_out[k] = hi[k];
    }
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            volatile float off = mean[3 * i + k] - lo[k];
            volatile float v = off * sc[k];
            uint32_t u = (uint32_t)v;
            q[k] = u > 1023u ? 1023u : u;
        }
        codes[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    }
}

typedef struct { uint32_t code; int64_t idx; } kv;

static int cmp_kv(const void *a, const void *b)
{
    const kv *x = (const kv *)a, *y = (const kv *)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

void orc_sort_codes(int64_t n, const uint32_t *codes, uint32_t *sorted, int32_t *perm)
{
    kv *a = (kv *)malloc(sizeof(kv) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { a[i].code = codes[i]; a[i].idx = i; }
    qsort(a, (size_t)n, sizeof(kv), cmp_kv);
    for (int64_t i = 0; i < n; ++i) { sorted[i] = a[i].code; perm[i] = (int32_t)a[i].idx; }
    free(a);
}

/* Length of the common prefix of augmented keys i and j (64-bit: code, index). */
static int prefix(const uint32_t *k, int64_t i, int64_t j)
{
    uint64_t a = ((uint64_t)k[i] << 32) | (uint64_t)(uint32_t)i;
    uint64_t b = ((uint64_t)k[j] << 32) | (uint64_t)(uint32_t)j;
    uint64_t x = a ^ b;
    if (x == 0) return 64;
    return __builtin_clzll(x);
}

/* Children of every internal node: child[2*i+0] (left), child[2*i+1] (right),
 * leaf[2*i+c] = 1 when that child is a leaf (child value = sorted position). */
void orc_radix_tree(int64_t n, const uint32_t *sorted, int32_t *child, int32_t *leaf)
{
    if (n < 2) return;
    /* explicit stack of ranges [f, l] with their node index */
    int64_t cap = 128;
    int64_t *st = (int64_t *)malloc(sizeof(int64_t) * 3 * cap);
    int64_t sp = 0;
    st[0] = 0; st[1] = n - 1; st[2] = 0;
    sp = 1;
    while (sp > 0) {
        --sp;
        int64_t f = st[3 * sp], l = st[3 * sp + 1], node = st[3 * sp + 2];
        int common = prefix(sorted, f, l);
        /* split: last position g in [f, l-1] whose key shares more than `common`
         * leading bits with key f */
        int64_t g = f;
        for (int64_t t = f; t < l; ++t)
            if (prefix(sorted, f, t) > common) g = t;
        int64_t lf = f, ll = g, rf = g + 1, rl = l;
        int32_t lnode = (int32_t)g, rnode = (int32_t)(g + 1);
        child[2 * node] = lnode;
        leaf[2 * node] = (lf == ll);
        child[2 * node + 1] = rnode;
        leaf[2 * node + 1] = (rf == rl);
        if (sp + 2 > cap) {
            cap *= 2;
            st = (int64_t *)realloc(st, sizeof(int64_t) * 3 * cap);
        }
        if (lf != ll) { st[3 * sp] = lf; st[3 * sp + 1] = ll; st[3 * sp + 2] = lnode; ++sp; }
        if (rf != rl) { st[3 * sp] = rf; st[3 * sp + 1] = rl; st[3 * sp + 2] = rnode; ++sp; }
    }
    free(st);
}

/* ------------------------------------------------------------ leaf boxes
 *
 * Axis-aligned box of Gaussian i's confidence ellipsoid (x-m)^T Sigma^-1
 * (x-m) = Q, Sigma = R S S^T R^T (Eq. 2), R from the quaternion (App. A.6),
 * bit-exact spec. The float32 inputs are widened to FP64 and every step below
 * is one correctly rounded FP64 operation, in the order written:
 *   nq = ((a a + b b) + c c) + d d for q = (a, b, c, d); q = (1, 0, 0, 0), nq = 1 when !(nq > 0)
 *   s = 2 / nq
 *   R = [[1 - s (c c + d d), s (b c - a d),     s (b d + a c)],
 *        [s (b c + a d),     1 - s (b b + d d), s (c d - a b)],
 *        [s (b d - a c),     s (c d + a b),     1 - s (b b + c c)]]
 *   e2_k = ((R_k0 s_0)^2 + (R_k1 s_1)^2) + (R_k2 s_2)^2   (half extent^2 / Q along axis k)
 *   e_k = sqrt(Q e2_k) (1 + 1e-5) + 1e-7 (1 + |m_k|)        (relative and absolute padding)
 *   box_k = [m_k - e_k rounded down to float32, m_k + e_k rounded up to float32]
 * Q is the float32 knob of the render parameters, widened to FP64. Boxes are
 * written in sorted order: row j is Gaussian perm[j].
 */
static float f32_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}

static float f32_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

void orc_leaf_boxes(int64_t n, const float *mean, const float *scale, const float *quat, float Q,
                    const int32_t *perm, float *boxes)
{
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i = perm[j];
        double a = quat[4 * i], b = quat[4 * i + 1], c = quat[4 * i + 2], d = quat[4 * i + 3];
        double aa = a * a, bb = b * b, cc = c * c, dd = d * d;
        double nq = aa + bb;
        nq = nq + cc;
        nq = nq + dd;
        if (!(nq > 0.0)) {
            a = 1.0; b = c = d = 0.0;
            aa = 1.0; bb = cc = dd = 0.0;
            nq = 1.0;
        }
        const double s = 2.0 / nq;
        const double ab = a * b, ac = a * c, ad = a * d, bc = b * c, bd = b * d, cd = c * d;
        double R[3][3];
        double t;
        t = cc + dd; t = s * t; R[0][0] = 1.0 - t;
        t = bc - ad; R[0][1] = s * t;
        t = bd + ac; R[0][2] = s * t;
        t = bc + ad; R[1][0] = s * t;
        t = bb + dd; t = s * t; R[1][1] = 1.0 - t;
        t = cd - ab; R[1][2] = s * t;
        t = bd - ac; R[2][0] = s * t;
        t = cd + ab; R[2][1] = s * t;
        t = bb + cc; t = s * t; R[2][2] = 1.0 - t;
        for (int k = 0; k < 3; ++k) {
            double e2 = 0.0;
            for (int q = 0; q < 3; ++q) {
                const double v = R[k][q] * (double)scale[3 * i + q];
                const double v2 = v * v;
                e2 = e2 + v2;
            }
            const double m = mean[3 * i + k];
            double e = (double)Q * e2;
            e = sqrt(e);
            e = e * (1.0 + 1e-5);
            const double pad = 1e-7 * (1.0 + fabs(m));
            e = e + pad;
            boxes[6 * j + k] = f32_down(m - e);
            boxes[6 * j + 3 + k] = f32_up(m + e);
        }
    }
}

/* ------------------------------------------------------------------ PLOC
 *
 * Locally-ordered agglomerative clustering (Meister and Bittner, 2018) over
 * the leaf boxes in sorted (Morton) order, bit-exact spec. Clusters start as
 * the N leaves. Each iteration t (while n > 1 clusters remain):
 *   d(i, j) = (ex ey + ey ez) + ez ex, ex = max(hi_i.x, hi_j.x) - min(lo_i.x, lo_j.x)
 *             etc.: half the surface area of the union box, float32 operations
 *             without contraction, NaN taken as +inf
 *   t <  T_cap: nn(i) = the j != i, |i - j| <= 8, 0 <= j < n, that minimises
 *               (d(i, j), |i - j|, min(i, j) mod 2, min(i, j)) lexicographically
 *               (a symmetric total order on pairs: the best pair overall is
 *               mutual, so every iteration merges; equal boxes pair up as
 *               (0, 1), (2, 3), ...)
 *   t >= T_cap: nn(i) = i xor 1 when that is < n, else none
 *   i merges with j = nn(i) when nn(j) = i; the merged cluster (box = union)
 *   takes position min(i, j), the other position is dropped and the survivors
 *   keep their order. The k-th merge of the build (counted over iterations,
 *   then positions) is internal node N - 2 - k with children (lower position,
 *   upper position) and their boxes, so the last merge is the root, node 0.
 *   T_cap = 256 + (N <= 4096 ? 0 : 10 ceil(log2(ceil(N / 4096)))).
 * Child references: >= 0 internal node, < 0 leaf ~(sorted position).
 * Returns the number of iterations.
 */
static float ploc_dist(const float *a, const float *b)
{
    float e[3];
    for (int k = 0; k < 3; ++k) {
        const float hi = fmaxf(a[3 + k], b[3 + k]);
        const float lo = fminf(a[k], b[k]);
        e[k] = hi - lo;
    }
    const float xy = e[0] * e[1], yz = e[1] * e[2], zx = e[2] * e[0];
    float d = xy + yz;
    d = d + zx;
    return d == d ? d : INFINITY;
}

int64_t orc_ploc_cap(int64_t n)
{
    int64_t g = 0;
    if (n > 4096) {
        int64_t c = (n + 4095) / 4096, l = 0;
        while (((int64_t)1 << l) < c) ++l;
        g = 10 * l;
    }
    return 256 + g;
}

int64_t orc_ploc(int64_t N, const float *leaf_boxes, int32_t *child, float *cbox)
{
    if (N < 2) return 0;
    const int64_t cap = orc_ploc_cap(N);
    int64_t n = N, made = 0, t = 0;
    int32_t *ref = (int32_t *)malloc(sizeof(int32_t) * N);
    int64_t *nn = (int64_t *)malloc(sizeof(int64_t) * N);
    float *box = (float *)malloc(sizeof(float) * 6 * N);
    for (int64_t i = 0; i < N; ++i) {
        ref[i] = ~(int32_t)i;
        memcpy(box + 6 * i, leaf_boxes + 6 * i, 6 * sizeof(float));
    }
    while (n > 1) {
        for (int64_t i = 0; i < n; ++i) {
            if (t >= cap) {
                nn[i] = (i ^ 1) < n ? (i ^ 1) : -1;
                continue;
            }
            int64_t best = -1;
            float bd = 0.0f;
            for (int64_t j = i - 8; j <= i + 8; ++j) {
                if (j < 0 || j >= n || j == i) continue;
                const float dd = ploc_dist(box + 6 * i, box + 6 * j);
                if (best < 0 || dd < bd) { best = j; bd = dd; continue; }
                if (dd > bd) continue;
                /* equal distance: smaller offset, then even lower end, then lower end */
                const int64_t oj = j > i ? j - i : i - j, ob = best > i ? best - i : i - best;
                const int64_t mj = j < i ? j : i, mb = best < i ? best : i;
                if (oj != ob) { if (oj < ob) best = j; continue; }
                if ((mj & 1) != (mb & 1)) { if ((mj & 1) == 0) best = j; continue; }
                if (mj < mb) best = j;
            }
            nn[i] = best;
        }
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t j = nn[i];
            const int mutual = j >= 0 && nn[j] == i;
            if (mutual && j < i) continue; /* merged into position j */
            if (mutual) {
                const int64_t id = N - 2 - made;
                ++made;
                child[2 * id] = ref[i];
                child[2 * id + 1] = ref[j];
                memcpy(cbox + 12 * id, box + 6 * i, 6 * sizeof(float));
                memcpy(cbox + 12 * id + 6, box + 6 * j, 6 * sizeof(float));
                float u[6];
                for (int k = 0; k < 3; ++k) {
                    u[k] = fminf(box[6 * i + k], box[6 * j + k]);
                    u[3 + k] = fmaxf(box[6 * i + 3 + k], box[6 * j + 3 + k]);
                }
                ref[m] = (int32_t)id;
                memcpy(box + 6 * m, u, sizeof(u));
            } else {
                ref[m] = ref[i];
                memmove(box + 6 * m, box + 6 * i, 6 * sizeof(float));
            }
            ++m;
        }
        n = m;
        ++t;
    }
    free(ref);
    free(nn);
    free(box);
    return t;
}
