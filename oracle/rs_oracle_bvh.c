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
 * Must be compiled with -ffp-contract=off.
 */
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
