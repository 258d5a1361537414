// BVH build for gfx950: preprocessing of the Gaussians into 64-byte records,
// 30-bit Morton codes, an LDS-tiled stable LSD radix sort, Karras radix-tree
// linking and a bottom-up box refit.
//
// The paper finds the ellipsoids hit by a ray with a vendor ray-tracing API
// (Sec. 3 "Intersection", Sec. 5); this linear BVH (Karras, HPG 2012) takes
// its place. Leaf boxes bound the confidence ellipsoid (x-m)^T Sigma^-1 (x-m)
// = Q with Sigma = R S S^T R^T (Eq. 2); R comes from the quaternion as in
// App. A.6.
#include <math.h>

#include "rs_internal.h"

namespace rs {

// ------------------------------------------------------------- header init

__global__ void k_init_header(WsHeader *h)
{
    if (threadIdx.x == 0) {
        h->status = 0;
        h->queue = 0;
        for (int k = 0; k < 16; ++k) h->counters[k] = 0;
        for (int k = 0; k < 3; ++k) {
            h->bounds[k] = 0xffffffffu;
            h->bounds[3 + k] = 0u;
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------- scene bounds

__global__ __launch_bounds__(256) void k_bounds(const float *__restrict__ mean, int64_t n, WsHeader *h)
{
    __shared__ uint32_t lo[3], hi[3];
    if (threadIdx.x < 3) {
        lo[threadIdx.x] = 0xffffffffu;
        hi[threadIdx.x] = 0u;
    }
    __syncthreads();
    uint32_t l[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, u[3] = {0u, 0u, 0u};
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int k = 0; k < 3; ++k) {
            uint32_t o = float_to_ordered(mean[3 * i + k]);
            l[k] = min(l[k], o);
            u[k] = max(u[k], o);
        }
    }
    for (int k = 0; k < 3; ++k) {
        atomicMin(&lo[k], l[k]);
        atomicMax(&hi[k], u[k]);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        atomicMin(&h->bounds[threadIdx.x], lo[threadIdx.x]);
        atomicMax(&h->bounds[3 + threadIdx.x], hi[threadIdx.x]);
    }
}

// ------------------------------------------------------------------ Morton

__device__ inline uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline bool finite3(float a, float b, float c) { return isfinite(a) && isfinite(b) && isfinite(c); }

// Codes of the bit-exact spec: lo/hi the float32 min/max of the means,
// scale = 1024 / (hi - lo) correctly rounded (0 on a flat axis),
// q = min(uint((c - lo) * scale), 1023) without contraction, x in the top bit.
__global__ __launch_bounds__(256) void k_morton(const float *__restrict__ mean, const float *__restrict__ scale,
                                                const float *__restrict__ quat, const float *__restrict__ opacity,
                                                const float *__restrict__ rgb, int64_t n, WsHeader *h,
                                                uint32_t *__restrict__ codes, uint32_t *__restrict__ vals)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float lo[3], sc[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = ordered_to_float(h->bounds[k]);
        float hi = ordered_to_float(h->bounds[3 + k]);
        float ext = __fsub_rn(hi, lo[k]);
        sc[k] = (hi == lo[k]) ? 0.0f : __fdiv_rn(1024.0f, ext);
    }
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        float v = __fmul_rn(__fsub_rn(mean[3 * i + k], lo[k]), sc[k]);
        v = fminf(fmaxf(v, 0.0f), 1023.0f);  // also maps NaN to 0 (fmaxf returns the number)
        uint32_t u = uint32_t(v);
        q[k] = u > 1023u ? 1023u : u;
    }
    codes[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[i] = uint32_t(i);
    if (!scale) return;  // triangle centroids: validated elsewhere
    // input validation (sticky device status)
    float s0 = scale[3 * i], s1 = scale[3 * i + 1], s2 = scale[3 * i + 2];
    float q0 = quat[4 * i], q1 = quat[4 * i + 1], q2 = quat[4 * i + 2], q3 = quat[4 * i + 3];
    float op = opacity[i];
    bool ok = finite3(mean[3 * i], mean[3 * i + 1], mean[3 * i + 2]) && finite3(s0, s1, s2) && s0 > 0.0f &&
              s1 > 0.0f && s2 > 0.0f && finite3(q0, q1, q2) && isfinite(q3) &&
              (q0 != 0.0f || q1 != 0.0f || q2 != 0.0f || q3 != 0.0f) && op >= 0.0f && op <= 1.0f &&
              finite3(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2]);
    if (!ok) atomicOr(&h->status, kStatusNonfinite);
}

// -------------------------------------------------------------- radix sort

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                          uint32_t *__restrict__ hist, int64_t nblocks)
{
    __shared__ uint32_t hs[256];
    hs[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int c = 0; c < kSortItems; ++c) {
        int64_t i = base + c * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&hs[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nblocks + blockIdx.x] = hs[threadIdx.x];
}

// Exclusive scan of the digit-major histogram in two steps: each workgroup
// scans one digit's row over the tiles and records the row total, then one
// workgroup scans the 256 totals into digit bases.
__global__ __launch_bounds__(256) void k_sort_scan_rows(uint32_t *__restrict__ hist, int64_t nblocks,
                                                        uint32_t *__restrict__ totals)
{
    __shared__ uint32_t s[256];
    const int t = threadIdx.x;
    uint32_t *row = hist + int64_t(blockIdx.x) * nblocks;
    const int64_t per = (nblocks + 255) / 256;
    const int64_t b = t * per, e = min(b + per, nblocks);
    uint32_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += row[i];
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    uint32_t run = s[t] - sum;
    for (int64_t i = b; i < e; ++i) {
        uint32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (t == 255) totals[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(256) void k_sort_scan_bases(uint32_t *__restrict__ totals)
{
    __shared__ uint32_t s[256];
    const int t = threadIdx.x;
    const uint32_t mine = totals[t];
    s[t] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    totals[256 + t] = s[t] - mine;  // exclusive base of digit t
}

// Stable scatter: within a tile, keys are ranked among equal digits in input
// order (wavefront match on the 8 digit bits, then a prefix over the four
// wavefronts of the workgroup and over the chunks already placed).
__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(const uint32_t *__restrict__ kin,
                                                             const uint32_t *__restrict__ vin,
                                                             uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                             int64_t n, int shift, const uint32_t *__restrict__ hist,
                                                             int64_t nblocks, const uint32_t *__restrict__ bases)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcount[kSortBlock / kWave][256];
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    run[t] = bases[t] + hist[int64_t(t) * nblocks + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int c = 0; c < kSortItems; ++c) {
        for (int ww = 0; ww < kSortBlock / kWave; ++ww) wcount[ww][t] = 0;
        __syncthreads();
        int64_t i = base + c * kSortBlock + t;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u, val = valid ? vin[i] : 0u;
        uint32_t digit = (key >> shift) & 255u;
        uint64_t peers = wave_ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            bool on = (digit >> bit) & 1u;
            uint64_t bal = wave_ballot(valid && on);
            peers &= on ? bal : ~bal;
        }
        if (!valid) peers = 0;
        uint32_t rank = __popcll(peers & lt_mask);
        bool last = valid && ((peers >> lane) == 1ull);
        if (last) wcount[w][digit] = __popcll(peers);
        __syncthreads();
        {
            uint32_t acc = run[t];
            for (int ww = 0; ww < kSortBlock / kWave; ++ww) {
                uint32_t v = wcount[ww][t];
                wcount[ww][t] = acc;
                acc += v;
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = wcount[w][digit] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- records

// Records and leaf boxes in sorted order; computed in FP64 from the float32
// inputs and stored rounded (boxes rounded outward).
__global__ __launch_bounds__(256) void k_records(const uint32_t *__restrict__ perm, const float *__restrict__ mean,
                                                 const float *__restrict__ scale, const float *__restrict__ quat,
                                                 const float *__restrict__ opacity, int64_t n, float Q,
                                                 float4 *__restrict__ records, float *__restrict__ leaf_boxes,
                                                 int32_t *__restrict__ inv)
{
    int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    uint32_t i = perm[j];
    // Every FP64 step is one correctly rounded operation in the order written
    // (explicit intrinsics, no contraction): the leaf boxes are bit-exact.
    double a = quat[4 * i], b = quat[4 * i + 1], c = quat[4 * i + 2], d = quat[4 * i + 3];
    double aa = __dmul_rn(a, a), bb = __dmul_rn(b, b), cc = __dmul_rn(c, c), dd = __dmul_rn(d, d);
    double nq = __dadd_rn(__dadd_rn(__dadd_rn(aa, bb), cc), dd);
    if (!(nq > 0.0)) {
        a = 1.0;
        b = c = d = 0.0;
        aa = 1.0;
        bb = cc = dd = 0.0;
        nq = 1.0;
    }
    const double s = __ddiv_rn(2.0, nq);
    const double ab = __dmul_rn(a, b), ac = __dmul_rn(a, c), ad = __dmul_rn(a, d), bc = __dmul_rn(b, c),
                 bd = __dmul_rn(b, d), cd = __dmul_rn(c, d);
    double R[3][3];
    R[0][0] = __dadd_rn(1.0, -__dmul_rn(s, __dadd_rn(cc, dd)));
    R[0][1] = __dmul_rn(s, __dadd_rn(bc, -ad));
    R[0][2] = __dmul_rn(s, __dadd_rn(bd, ac));
    R[1][0] = __dmul_rn(s, __dadd_rn(bc, ad));
    R[1][1] = __dadd_rn(1.0, -__dmul_rn(s, __dadd_rn(bb, dd)));
    R[1][2] = __dmul_rn(s, __dadd_rn(cd, -ab));
    R[2][0] = __dmul_rn(s, __dadd_rn(bd, -ac));
    R[2][1] = __dmul_rn(s, __dadd_rn(cd, ab));
    R[2][2] = __dadd_rn(1.0, -__dmul_rn(s, __dadd_rn(bb, cc)));
    double sc[3], m[3];
    for (int k = 0; k < 3; ++k) {
        sc[k] = scale[3 * i + k];
        m[k] = mean[3 * i + k];
    }
    float4 r0, r1, r2, r3;
    // row k of R^T is column k of R
    r0 = make_float4(float(R[0][0]), float(R[1][0]), float(R[2][0]), float(R[0][1]));
    r1 = make_float4(float(R[1][1]), float(R[2][1]), float(R[0][2]), float(R[1][2]));
    r2 = make_float4(float(R[2][2]), float(1.0 / sc[0]), float(1.0 / sc[1]), float(1.0 / sc[2]));
    r3 = make_float4(float(m[0]), float(m[1]), float(m[2]), opacity[i]);
    records[4 * j + 0] = r0;
    records[4 * j + 1] = r1;
    records[4 * j + 2] = r2;
    records[4 * j + 3] = r3;
    // half extent along world axis k: sqrt(Q * sum_c (R_kc s_c)^2), padded by
    // 1e-5 relative and 1e-7 (1 + |m_k|) absolute, rounded outward
    for (int k = 0; k < 3; ++k) {
        double e2 = 0.0;
        for (int q = 0; q < 3; ++q) {
            const double v = __dmul_rn(R[k][q], sc[q]);
            e2 = __dadd_rn(e2, __dmul_rn(v, v));
        }
        double e = __dsqrt_rn(__dmul_rn(double(Q), e2));
        e = __dmul_rn(e, 1.0 + 1e-5);
        e = __dadd_rn(e, __dmul_rn(1e-7, __dadd_rn(1.0, fabs(m[k]))));
        leaf_boxes[6 * j + k] = __double2float_rd(__dadd_rn(m[k], -e));
        leaf_boxes[6 * j + 3 + k] = __double2float_ru(__dadd_rn(m[k], e));
    }
    inv[i] = int32_t(j);
}

// ------------------------------------------------------------ Karras link

__device__ inline int delta(const uint32_t *__restrict__ codes, int64_t n, int64_t i, int64_t j)
{
    if (j < 0 || j >= n) return -1;
    uint32_t a = codes[i], b = codes[j];
    if (a == b) return 32 + __clz(uint32_t(i) ^ uint32_t(j));
    return __clz(a ^ b);
}

__global__ __launch_bounds__(256) void k_karras(const uint32_t *__restrict__ codes, int64_t n,
                                                float4 *__restrict__ nodes, int32_t *__restrict__ parent)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int dir = (delta(codes, n, i, i + 1) - delta(codes, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(codes, n, i, i - dir);
    int64_t lmax = 2;
    while (delta(codes, n, i, i + lmax * dir) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (delta(codes, n, i, i + (l + t) * dir) > dmin) l += t;
    int64_t j = i + l * dir;
    int dnode = delta(codes, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) / 2;
        if (delta(codes, n, i, i + (s + t) * dir) > dnode) s += t;
    } while (t > 1);
    int64_t gamma = i + s * dir + (dir < 0 ? -1 : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t left = (lo == gamma) ? ~int32_t(gamma) : int32_t(gamma);
    int32_t right = (hi == gamma + 1) ? ~int32_t(gamma + 1) : int32_t(gamma + 1);
    float4 n3;
    n3.x = __int_as_float(left);
    n3.y = __int_as_float(right);
    n3.z = 0.0f;
    n3.w = 0.0f;
    nodes[4 * i + 3] = n3;
    // parent links: leaves at [0, n), internal nodes at [n, 2n - 1)
    parent[left < 0 ? ~left : n + left] = int32_t(i);
    parent[right < 0 ? ~right : n + right] = int32_t(i);
    if (i == 0) parent[n] = -1;
}

// --------------------------------------------------------------- box refit

__device__ inline float ld_agent(const float *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bottom-up box of every internal node: one thread per leaf climbs while it
// is the second child to arrive at a node (atomic visit counter), computing
// that node's box from its two children (leaf boxes, written by an earlier
// kernel, or boxes of internal nodes finished by other threads). No box is
// carried across iterations: each node's box goes to ibox[node] and
// k_fill_nodes copies the child boxes into the traversal nodes afterwards.
//
// Hand-off without cache write-backs: ibox is written with agent-scope
// (write-through) stores and read with agent-scope loads, and a thread waits
// for its stores to complete before its next visit atomic, so a thread that
// sees the counter at 1 finds the sibling's box at the coherence point.
__device__ inline void st_agent(float *p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void child_box(int32_t ref, const float *__restrict__ leaf_boxes, const float *ibox, float *b)
{
    if (ref < 0) {
        const float *src = leaf_boxes + 6 * int64_t(~ref);
        for (int k = 0; k < 6; ++k) b[k] = src[k];
    } else {
        const float *src = ibox + 6 * int64_t(ref);
        for (int k = 0; k < 6; ++k) b[k] = ld_agent(src + k);
    }
}

__global__ __launch_bounds__(256) void k_refit(const float *__restrict__ leaf_boxes, const int32_t *__restrict__ parent,
                                               const float4 *__restrict__ nodes, float *ibox, uint32_t *visit,
                                               int64_t n)
{
    int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t node = parent[j];
    while (node >= 0) {
        const uint32_t old = __hip_atomic_fetch_add(&visit[node], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0) return;
        const float4 n3 = nodes[4 * int64_t(node) + 3];
        float bl[6], br[6];
        child_box(__float_as_int(n3.x), leaf_boxes, ibox, bl);
        child_box(__float_as_int(n3.y), leaf_boxes, ibox, br);
        float *dst = ibox + 6 * int64_t(node);
        for (int k = 0; k < 3; ++k) {
            st_agent(dst + k, fminf(bl[k], br[k]));
            st_agent(dst + 3 + k, fmaxf(bl[3 + k], br[3 + k]));
        }
        __builtin_amdgcn_s_waitcnt(0);  // the box is at the coherence point before the next visit atomic
        node = parent[n + node];
    }
}

// Child boxes into the traversal nodes (floats [0, 6) left, [6, 12) right).
__global__ __launch_bounds__(256) void k_fill_nodes(const float *__restrict__ leaf_boxes, const float *__restrict__ ibox,
                                                    float *__restrict__ nodes_f, int64_t n_int, WsHeader *h)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    float *nf = nodes_f + 16 * i;
    for (int c = 0; c < 2; ++c) {
        const int32_t ref = __float_as_int(nf[12 + c]);
        const float *src = ref < 0 ? leaf_boxes + 6 * int64_t(~ref) : ibox + 6 * int64_t(ref);
        for (int k = 0; k < 6; ++k) nf[6 * c + k] = src[k];
    }
    if (i == 0)
        for (int k = 0; k < 6; ++k) h->root_box[k] = ibox[k];
}

// ----------------------------------------------------------- triangle mesh

__device__ inline int32_t clamp_index(int32_t v, int64_t n_verts, WsHeader *h)
{
    if (v < 0 || v >= n_verts) {
        atomicOr(&h->status, kStatusNonfinite);
        return 0;
    }
    return v;
}

// Triangle centroids (into the record area, before the sort); indices out of
// range set the status and read vertex 0 instead.
__global__ __launch_bounds__(256) void k_tri_centroids(const float *__restrict__ verts, const int32_t *__restrict__ tris,
                                                       int64_t n_tris, int64_t n_verts, float *__restrict__ cent,
                                                       WsHeader *h)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_tris) return;
    float c[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k) {
        const int32_t v = clamp_index(tris[3 * i + k], n_verts, h);
        for (int a = 0; a < 3; ++a) c[a] += verts[3 * v + a];
    }
    for (int a = 0; a < 3; ++a) cent[3 * i + a] = c[a] * (1.0f / 3.0f);
}

// Triangle records in sorted order: r0 = (v0, e1.x), r1 = (e1.yz, e2.xy),
// r2 = (e2.z, material bits, triangle index bits, 0), r3 unused; leaf boxes
// are the vertex bounds rounded outward.
__global__ __launch_bounds__(256) void k_tri_records(const uint32_t *__restrict__ perm, const float *__restrict__ verts,
                                                     const int32_t *__restrict__ tris,
                                                     const int32_t *__restrict__ material, int64_t n_tris,
                                                     int64_t n_verts, float4 *__restrict__ records,
                                                     float *__restrict__ leaf_boxes, int32_t *__restrict__ inv,
                                                     WsHeader *h)
{
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n_tris) return;
    const uint32_t i = perm[j];
    float v[3][3];
    for (int k = 0; k < 3; ++k) {
        const int32_t vi = clamp_index(tris[3 * i + k], n_verts, h);
        for (int a = 0; a < 3; ++a) v[k][a] = verts[3 * vi + a];
    }
    const float e1x = v[1][0] - v[0][0], e1y = v[1][1] - v[0][1], e1z = v[1][2] - v[0][2];
    const float e2x = v[2][0] - v[0][0], e2y = v[2][1] - v[0][1], e2z = v[2][2] - v[0][2];
    const int32_t mat = material ? material[i] : 0;
    records[4 * j + 0] = make_float4(v[0][0], v[0][1], v[0][2], e1x);
    records[4 * j + 1] = make_float4(e1y, e1z, e2x, e2y);
    records[4 * j + 2] = make_float4(e2z, __int_as_float(mat), __int_as_float(int32_t(i)), 0.0f);
    records[4 * j + 3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int a = 0; a < 3; ++a) {
        const float lo = fminf(fminf(v[0][a], v[1][a]), v[2][a]);
        const float hi = fmaxf(fmaxf(v[0][a], v[1][a]), v[2][a]);
        const float pad = 1e-6f * (1.0f + fmaxf(fabsf(lo), fabsf(hi)));
        leaf_boxes[6 * j + a] = lo - pad;
        leaf_boxes[6 * j + 3 + a] = hi + pad;
    }
    inv[i] = int32_t(j);
}

// -------------------------------------------------------------------- PLOC
//
// Locally-ordered agglomerative clustering (Meister and Bittner, 2018) over
// the leaves in Morton order. Each iteration every cluster finds its nearest
// neighbour within kPlocR positions (distance: half the surface area of the
// union box); mutual nearest neighbours merge into a new internal node, which
// takes the lower position, and the survivors are compacted in order. The
// k-th merge of the build becomes node n - 2 - k, so the root is node 0 and
// the top of the tree sits at the front of the node array.
//
// Large cluster counts run as grid-wide iterations (nearest neighbours +
// merge codes + per-chunk counts, then prefix + scatter), each kernel reading
// its cluster count from the control array so the launch sequence is fixed
// (graph-capturable); the last few thousand clusters are finished by one
// workgroup in LDS. Ties follow a symmetric total order on pairs (distance,
// offset, parity of the lower end, lower end), so the best pair is always
// mutual and every iteration merges; from iteration ploc_cap(n) clusters are
// paired by position, which bounds the iteration count.

struct PlocCtrl {
    int32_t n, created, buf, pad;
};

__device__ inline float ploc_dist(float alx, float aly, float alz, float ahx, float ahy, float ahz, float blx,
                                  float bly, float blz, float bhx, float bhy, float bhz)
{
    const float ex = __fsub_rn(fmaxf(ahx, bhx), fminf(alx, blx));
    const float ey = __fsub_rn(fmaxf(ahy, bhy), fminf(aly, bly));
    const float ez = __fsub_rn(fmaxf(ahz, bhz), fminf(alz, blz));
    const float d = __fadd_rn(__fadd_rn(__fmul_rn(ex, ey), __fmul_rn(ey, ez)), __fmul_rn(ez, ex));
    return d == d ? d : __builtin_huge_valf();
}

// Nearest neighbour of position i among [i - R, i + R] of n clusters; boxes
// are read through `at(j)` (a 6-float box of position j). The pair order
// (distance, offset, parity of the lower end, lower end) is one 64-bit key:
// order-preserving distance bits, then offset, parity and side (for a given
// offset the left candidate is the lower end).
__device__ inline uint32_t ordered_bits(float d)
{
    const uint32_t u = __float_as_uint(d + 0.0f);  // -0 -> +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

template <typename BoxAt>
__device__ inline int32_t ploc_nearest(int64_t i, int64_t n, BoxAt at)
{
    float a[6];
    at(i, a);
    int32_t best = -1;
    uint64_t bk = ~0ull;
#pragma unroll
    for (int off = 1; off <= kPlocR; ++off) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int64_t j = side ? i + off : i - off;
            if (j < 0 || j >= n) continue;
            float b[6];
            at(j, b);
            const float d = ploc_dist(a[0], a[1], a[2], a[3], a[4], a[5], b[0], b[1], b[2], b[3], b[4], b[5]);
            const uint32_t par = uint32_t(side ? i : j) & 1u;
            const uint64_t key = (uint64_t(ordered_bits(d)) << 32) | (uint32_t(off) << 2) | (par << 1) | uint32_t(side);
            if (key < bk) {
                bk = key;
                best = int32_t(j);
            }
        }
    }
    return best;
}

// The same order from the pair side: the distance of pair (p, p + off) is
// computed once and offered to both ends as a 64-bit key (side bit 1: the
// candidate lies to the right); the smallest key a position receives names
// its nearest neighbour.
__device__ inline uint64_t pair_key(float d, int off, int64_t lower, uint32_t right)
{
    return (uint64_t(ordered_bits(d)) << 32) | (uint32_t(off) << 2) | ((uint32_t(lower) & 1u) << 1) | right;
}

__device__ inline int32_t key_neighbour(uint64_t key, int64_t i)
{
    if (key == ~0ull) return -1;
    const int off = int(key >> 2) & 15;
    return int32_t((key & 1ull) ? i + off : i - off);
}

// Exclusive scan of two counts over a workgroup of THREADS; ws holds 2 ints
// per wave. Returns the workgroup totals. Ends with a barrier (ws reusable).
template <int THREADS>
__device__ inline void block_scan2(int a, int b, int &ea, int &eb, int &ta, int &tb, int *ws)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int ia = a, ib = b;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int xa = __shfl_up(ia, d), xb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += xa;
            ib += xb;
        }
    }
    if (lane == kWave - 1) {
        ws[2 * wave] = ia;
        ws[2 * wave + 1] = ib;
    }
    __syncthreads();
    int pa = 0, pb = 0;
    ta = 0;
    tb = 0;
#pragma unroll
    for (int w = 0; w < THREADS / kWave; ++w) {
        const int va = ws[2 * w], vb = ws[2 * w + 1];
        if (w < wave) {
            pa += va;
            pb += vb;
        }
        ta += va;
        tb += vb;
    }
    ea = pa + ia - a;
    eb = pb + ib - b;
    __syncthreads();
}

__device__ inline void write_node(float4 *__restrict__ nodes, int64_t id, const float *bl, const float *br, int32_t rl,
                                  int32_t rr)
{
    float4 *nd = nodes + 4 * id;
    nd[0] = make_float4(bl[0], bl[1], bl[2], bl[3]);
    nd[1] = make_float4(bl[4], bl[5], br[0], br[1]);
    nd[2] = make_float4(br[2], br[3], br[4], br[5]);
    nd[3] = make_float4(__int_as_float(rl), __int_as_float(rr), 0.0f, 0.0f);
}

// Clusters of iteration 0: the leaves (buffer 0), and the control entry.
__global__ __launch_bounds__(256) void k_ploc_init(const float *__restrict__ leaf_boxes, int64_t n,
                                                   float *__restrict__ box, int32_t *__restrict__ ref,
                                                   PlocCtrl *ctrl)
{
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j == 0) ctrl[0] = PlocCtrl{int32_t(n), 0, 0, 0};
    if (j >= n) return;
    for (int k = 0; k < 6; ++k) box[k * n + j] = leaf_boxes[6 * j + k];
    ref[j] = ~int32_t(j);
}

// Grid iteration, step 1: nearest neighbours of a chunk and of kPlocR
// positions either side (from boxes staged in LDS with 2 kPlocR margin),
// then the merge code of each position (-1 keep, -2 merged into a lower
// position, m > i: merges with m into a new node) and the chunk's counts.
__global__ __launch_bounds__(kPlocThreads) void k_ploc_nn(const float *__restrict__ box_all, const PlocCtrl *ctrl,
                                                          int it, int64_t N, int32_t *__restrict__ pm,
                                                          int32_t *__restrict__ blk)
{
    constexpr int W = kPlocChunk + 4 * kPlocR;
    __shared__ float sb[6][W];
    __shared__ unsigned long long skey[W];
    __shared__ int ws[2 * kPlocThreads / kWave];
    const PlocCtrl c = ctrl[it];
    const int64_t n = c.n;
    if (n <= kPlocLocal) return;
    const int64_t base = int64_t(blockIdx.x) * kPlocChunk;
    if (base >= n) return;
    const float *box = box_all + size_t(c.buf) * 6 * N;
    const int64_t w0 = base - 2 * kPlocR;
    for (int t = threadIdx.x; t < W; t += kPlocThreads) {
        const int64_t i = w0 + t;
        const bool in = i >= 0 && i < n;
        for (int k = 0; k < 6; ++k) sb[k][t] = in ? box[k * N + i] : 0.0f;
        skey[t] = ~0ull;
    }
    __syncthreads();
    // every pair inside the window: positions [base - R, base + chunk + R) see all their candidates
    for (int t = threadIdx.x; t < W; t += kPlocThreads) {
        const int64_t p = w0 + t;
        if (p < 0 || p >= n) continue;
        const float a0 = sb[0][t], a1 = sb[1][t], a2 = sb[2][t], a3 = sb[3][t], a4 = sb[4][t], a5 = sb[5][t];
        uint64_t kp = ~0ull;
#pragma unroll
        for (int off = 1; off <= kPlocR; ++off) {
            const int tq = t + off;
            if (tq >= W || p + off >= n) break;
            const float d = ploc_dist(a0, a1, a2, a3, a4, a5, sb[0][tq], sb[1][tq], sb[2][tq], sb[3][tq], sb[4][tq],
                                      sb[5][tq]);
            const uint64_t kr = pair_key(d, off, p, 1u);
            kp = kr < kp ? kr : kp;
            atomicMin(&skey[tq], (unsigned long long)(kr ^ 1ull));
        }
        atomicMin(&skey[t], (unsigned long long)kp);
    }
    __syncthreads();
    int keep = 0, make = 0;
    for (int t = threadIdx.x; t < kPlocChunk; t += kPlocThreads) {
        const int64_t i = base + t;
        if (i >= n) break;
        const int32_t m = key_neighbour(skey[t + 2 * kPlocR], i);
        int32_t code = -1;
        if (m >= 0 && key_neighbour(skey[m - w0], m) == int32_t(i)) code = m > i ? m : -2;
        pm[i] = code;
        keep += code != -2;
        make += code >= 0;
    }
    int ek, em, tk, tm;
    block_scan2<kPlocThreads>(keep, make, ek, em, tk, tm, ws);
    if (threadIdx.x == 0) {
        blk[2 * blockIdx.x] = tk;
        blk[2 * blockIdx.x + 1] = tm;
    }
}

// Grid iteration, step 2: each chunk sums the counts of the chunks before it,
// scans its own positions (four consecutive per thread), writes the survivors
// to the other buffer and the new nodes; the last chunk writes the next
// control entry.
__global__ __launch_bounds__(kPlocThreads) void k_ploc_scatter(float *__restrict__ box_all, int32_t *__restrict__ ref_all,
                                                               PlocCtrl *ctrl, int it, int64_t N,
                                                               const int32_t *__restrict__ pm,
                                                               const int32_t *__restrict__ blk,
                                                               float4 *__restrict__ nodes)
{
    __shared__ int ws[2 * kPlocThreads / kWave];
    const PlocCtrl c = ctrl[it];
    const int64_t n = c.n;
    if (n <= kPlocLocal) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[it + 1] = c;
        return;
    }
    const int64_t nb = (n + kPlocChunk - 1) / kPlocChunk;
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    int kp = 0, mp = 0;
    for (int64_t q = threadIdx.x; q < b; q += kPlocThreads) {
        kp += blk[2 * q];
        mp += blk[2 * q + 1];
    }
    int e0, e1;
    block_scan2<kPlocThreads>(kp, mp, e0, e1, kp, mp, ws);
    constexpr int E = kPlocChunk / kPlocThreads;
    const int64_t i0 = b * kPlocChunk + int64_t(threadIdx.x) * E;
    int32_t code[E];
    int lk = 0, lm = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        code[e] = i0 + e < n ? pm[i0 + e] : -2;
        lk += code[e] != -2;
        lm += code[e] >= 0;
    }
    int ok, om, tk, tm;
    block_scan2<kPlocThreads>(lk, lm, ok, om, tk, tm, ws);
    const float *sbx = box_all + size_t(c.buf) * 6 * N;
    float *dbx = box_all + size_t(1 - c.buf) * 6 * N;
    const int32_t *sref = ref_all + size_t(c.buf) * N;
    int32_t *dref = ref_all + size_t(1 - c.buf) * N;
    int64_t pos = int64_t(kp) + ok;
    int64_t made = int64_t(c.created) + mp + om;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t i = i0 + e;
        if (code[e] == -2) continue;
        float bi[6];
        for (int k = 0; k < 6; ++k) bi[k] = sbx[k * N + i];
        int32_t ri = sref[i];
        if (code[e] >= 0) {
            const int64_t m = code[e];
            float bm[6];
            for (int k = 0; k < 6; ++k) bm[k] = sbx[k * N + m];
            const int64_t id = N - 2 - made;
            ++made;
            if (id >= 0) write_node(nodes, id, bi, bm, ri, sref[m]);
            for (int k = 0; k < 3; ++k) {
                bi[k] = fminf(bi[k], bm[k]);
                bi[3 + k] = fmaxf(bi[3 + k], bm[3 + k]);
            }
            ri = int32_t(id);
        }
        for (int k = 0; k < 6; ++k) dbx[k * N + pos] = bi[k];
        dref[pos] = ri;
        ++pos;
    }
    if (b == nb - 1 && threadIdx.x == 0)
        ctrl[it + 1] = PlocCtrl{kp + tk, int32_t(c.created + mp + tm), 1 - c.buf, 0};
}

// The remaining iterations in one workgroup. Positions are compacted in
// place, a chunk of kPlocFinishThreads * 2 at a time: every position of a
// chunk (and its merge partner, which lies above it) is read before any is
// written, and a survivor's new position never exceeds its old one, so no
// unread position is overwritten.
template <typename Arr>
__device__ inline void ploc_finish_loop(Arr A, int64_t n, int64_t made, int t, int cap, int64_t N,
                                        float4 *__restrict__ nodes, int *ws)
{
    constexpr int E = 2;
    constexpr int CH = kPlocFinishThreads * E;
    while (n > 1) {
        A.nearest_all(n, t >= cap);
        __syncthreads();
        int64_t kc = 0, mc = 0;
        for (int64_t base = 0; base < n; base += CH) {
            const int64_t i0 = base + int64_t(threadIdx.x) * E;
            int32_t code[E], ri[E], rm[E];
            float bi[E][6], bm[E][6];
            int lk = 0, lm = 0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t i = i0 + e;
                code[e] = -2;
                if (i < n) {
                    const int32_t m = A.nn(i);
                    code[e] = (m >= 0 && A.nn(m) == int32_t(i)) ? (m > i ? m : -2) : -1;
                }
                if (code[e] != -2) {
                    for (int k = 0; k < 6; ++k) bi[e][k] = A.box(k, i);
                    ri[e] = A.ref(i);
                }
                if (code[e] >= 0) {
                    for (int k = 0; k < 6; ++k) bm[e][k] = A.box(k, code[e]);
                    rm[e] = A.ref(code[e]);
                }
                lk += code[e] != -2;
                lm += code[e] >= 0;
            }
            int ok, om, tk, tm;
            block_scan2<kPlocFinishThreads>(lk, lm, ok, om, tk, tm, ws);
            int64_t pos = kc + ok, id_n = made + mc + om;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (code[e] == -2) continue;
                int32_t r = ri[e];
                if (code[e] >= 0) {
                    const int64_t id = N - 2 - id_n;
                    ++id_n;
                    if (id >= 0) write_node(nodes, id, bi[e], bm[e], ri[e], rm[e]);
                    for (int k = 0; k < 3; ++k) {
                        bi[e][k] = fminf(bi[e][k], bm[e][k]);
                        bi[e][3 + k] = fmaxf(bi[e][3 + k], bm[e][3 + k]);
                    }
                    r = int32_t(id);
                }
                for (int k = 0; k < 6; ++k) A.box(k, pos) = bi[e][k];
                A.ref(pos) = r;
                ++pos;
            }
            kc += tk;
            mc += tm;
            __syncthreads();
        }
        n = kc;
        made += mc;
        ++t;
    }
}

// Cluster storage of the finish loop. nearest_all(n, forced) fills the
// nearest neighbours of positions [0, n) (ends without a barrier), nn(i)
// reads one back (-1: none). Forced: i pairs with i xor 1.
struct PlocLds {
    float (*b)[kPlocLocal];
    int32_t *r;
    unsigned long long *key;
    __device__ float &box(int k, int64_t j) const { return b[k][j]; }
    __device__ int32_t &ref(int64_t j) const { return r[j]; }
    __device__ int32_t nn(int64_t i) const { return key_neighbour(key[i], i); }
    __device__ void nearest_all(int64_t n, bool forced) const
    {
        for (int64_t i = threadIdx.x; i < n; i += kPlocFinishThreads)
            key[i] = forced ? ((i ^ 1) < n ? ((1ull << 2) | ((i & 1) ? 0ull : 1ull)) : ~0ull) : ~0ull;
        if (forced) return;
        __syncthreads();
        for (int64_t p = threadIdx.x; p < n; p += kPlocFinishThreads) {
            const float a0 = b[0][p], a1 = b[1][p], a2 = b[2][p], a3 = b[3][p], a4 = b[4][p], a5 = b[5][p];
            uint64_t kp = ~0ull;
#pragma unroll
            for (int off = 1; off <= kPlocR; ++off) {
                const int64_t q = p + off;
                if (q >= n) break;
                const float d = ploc_dist(a0, a1, a2, a3, a4, a5, b[0][q], b[1][q], b[2][q], b[3][q], b[4][q], b[5][q]);
                const uint64_t kr = pair_key(d, off, p, 1u);
                kp = kr < kp ? kr : kp;
                atomicMin(&key[q], (unsigned long long)(kr ^ 1ull));
            }
            atomicMin(&key[p], (unsigned long long)kp);
        }
    }
};

struct PlocGlobal {
    float *b;
    int32_t *r, *q;
    int64_t N;
    __device__ float &box(int k, int64_t j) const { return b[k * N + j]; }
    __device__ int32_t &ref(int64_t j) const { return r[j]; }
    __device__ int32_t nn(int64_t i) const { return q[i]; }
    __device__ void nearest_all(int64_t n, bool forced) const
    {
        auto at = [&](int64_t j, float *bx) {
            for (int k = 0; k < 6; ++k) bx[k] = b[k * N + j];
        };
        for (int64_t i = threadIdx.x; i < n; i += kPlocFinishThreads)
            q[i] = forced ? ((i ^ 1) < n ? int32_t(i ^ 1) : -1) : ploc_nearest(i, n, at);
    }
};

// Finish of the clustering when at most kPlocLocal clusters remain (the usual
// case): clusters staged in LDS. Writes the root box.
__global__ __launch_bounds__(kPlocFinishThreads) void k_ploc_finish_lds(const float *__restrict__ box_all,
                                                                        const int32_t *__restrict__ ref_all,
                                                                        const PlocCtrl *ctrl, int G, int cap, int64_t N,
                                                                        float4 *__restrict__ nodes, WsHeader *h)
{
    __shared__ float sb[6][kPlocLocal];
    __shared__ int32_t sref[kPlocLocal];
    __shared__ unsigned long long skey[kPlocLocal];
    __shared__ int ws[2 * kPlocFinishThreads / kWave];
    const PlocCtrl c = ctrl[G];
    const int64_t n = c.n;
    if (n > kPlocLocal) return;
    const float *gbox = box_all + size_t(c.buf) * 6 * N;
    const int32_t *gref = ref_all + size_t(c.buf) * N;
    for (int64_t i = threadIdx.x; i < n; i += kPlocFinishThreads) {
        for (int k = 0; k < 6; ++k) sb[k][i] = gbox[k * N + i];
        sref[i] = gref[i];
    }
    __syncthreads();
    ploc_finish_loop(PlocLds{sb, sref, skey}, n, c.created, G, cap, N, nodes, ws);
    if (threadIdx.x < 6) h->root_box[threadIdx.x] = sb[threadIdx.x][0];
}

// The same from global memory, in place, for more than kPlocLocal clusters
// (only when the grid iterations left that many: slow, but bounded by the
// pairing cap).
__global__ __launch_bounds__(kPlocFinishThreads) void k_ploc_finish_global(float *__restrict__ box_all,
                                                                           int32_t *__restrict__ ref_all,
                                                                           int32_t *__restrict__ pm,
                                                                           const PlocCtrl *ctrl, int G, int cap,
                                                                           int64_t N, float4 *__restrict__ nodes,
                                                                           WsHeader *h)
{
    __shared__ int ws[2 * kPlocFinishThreads / kWave];
    const PlocCtrl c = ctrl[G];
    const int64_t n = c.n;
    if (n <= kPlocLocal) return;
    float *gbox = box_all + size_t(c.buf) * 6 * N;
    int32_t *gref = ref_all + size_t(c.buf) * N;
    ploc_finish_loop(PlocGlobal{gbox, gref, pm, N}, n, c.created, G, cap, N, nodes, ws);
    if (threadIdx.x < 6) h->root_box[threadIdx.x] = gbox[threadIdx.x * N];
}

// ------------------------------------------------------------------- host

static inline int blocks_for(int64_t n, int threads) { return int((n + threads - 1) / threads); }

// Sort + link + refit shared by the Gaussian and the triangle BVH: `points`
// are the Morton sites; `records_fn` writes records and leaf boxes in sorted
// order once the permutation is known.
template <typename RecordsFn>
static int build_core(int64_t n, const float *points, const float *scale, const float *quat, const float *opacity,
                      const float *rgb, char *ws, hipStream_t st, RecordsFn records_fn, bool init_header, bool lbvh)
{
    Layout L = make_layout(n);
    WsHeader *h = reinterpret_cast<WsHeader *>(ws + L.header);
    if (init_header) k_init_header<<<1, 64, 0, st>>>(h);
    if (n == 0) return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
    uint32_t *codes = reinterpret_cast<uint32_t *>(ws + L.codes);
    uint32_t *vals = reinterpret_cast<uint32_t *>(ws + L.gidx);
    uint32_t *kalt = reinterpret_cast<uint32_t *>(ws + L.keys_alt);
    uint32_t *valt = reinterpret_cast<uint32_t *>(ws + L.vals_alt);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *totals = reinterpret_cast<uint32_t *>(ws + L.totals);
    float4 *records = reinterpret_cast<float4 *>(ws + L.records);
    float4 *nodes = reinterpret_cast<float4 *>(ws + L.nodes);
    float *leaf_boxes = reinterpret_cast<float *>(ws + L.leaf_boxes);
    int32_t *inv = reinterpret_cast<int32_t *>(ws + L.inv);
    int32_t *parent = reinterpret_cast<int32_t *>(ws + L.parent);
    uint32_t *visit = reinterpret_cast<uint32_t *>(ws + L.visit);

    int bgrid = blocks_for(n, 256);
    k_bounds<<<bgrid < 1024 ? bgrid : 1024, 256, 0, st>>>(points, n, h);
    k_morton<<<bgrid, 256, 0, st>>>(points, scale, quat, opacity, rgb, n, h, codes, vals);
    // 4 passes of 8 bits: A -> B -> A -> B -> A
    uint32_t *ka = codes, *va = vals, *kb = kalt, *vb = valt;
    int64_t nb = L.sort_blocks;
    for (int pass = 0; pass < 4; ++pass) {
        int shift = 8 * pass;
        k_sort_hist<<<int(nb), kSortBlock, 0, st>>>(ka, n, shift, hist, nb);
        k_sort_scan_rows<<<256, 256, 0, st>>>(hist, nb, totals);
        k_sort_scan_bases<<<1, 256, 0, st>>>(totals);
        k_sort_scatter<<<int(nb), kSortBlock, 0, st>>>(ka, va, kb, vb, n, shift, hist, nb, totals + 256);
        uint32_t *t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    records_fn(vals, records, leaf_boxes, inv, h);
    if (n >= 2 && !lbvh) {
        float *pbox = reinterpret_cast<float *>(ws + L.ploc_box);
        int32_t *pref = reinterpret_cast<int32_t *>(ws + L.ploc_ref);
        int32_t *pm = reinterpret_cast<int32_t *>(ws + L.ploc_pm);
        int32_t *blk = reinterpret_cast<int32_t *>(ws + L.ploc_blk);
        PlocCtrl *ctrl = reinterpret_cast<PlocCtrl *>(ws + L.ploc_ctrl);
        k_ploc_init<<<bgrid, 256, 0, st>>>(leaf_boxes, n, pbox, pref, ctrl);
        const int G = ploc_global_iters(n);
        const int nchunks = int(L.ploc_chunks);
        for (int it = 0; it < G; ++it) {
            k_ploc_nn<<<nchunks, kPlocThreads, 0, st>>>(pbox, ctrl, it, n, pm, blk);
            k_ploc_scatter<<<nchunks, kPlocThreads, 0, st>>>(pbox, pref, ctrl, it, n, pm, blk, nodes);
        }
        k_ploc_finish_lds<<<1, kPlocFinishThreads, 0, st>>>(pbox, pref, ctrl, G, ploc_cap(n), n, nodes, h);
        if (G > 0)
            k_ploc_finish_global<<<1, kPlocFinishThreads, 0, st>>>(pbox, pref, pm, ctrl, G, ploc_cap(n), n, nodes, h);
    } else if (n >= 2) {
        k_fill_u32<<<blocks_for(L.n_int, 256) < 2048 ? blocks_for(L.n_int, 256) : 2048, 256, 0, st>>>(visit, L.n_int,
                                                                                                       0u);
        k_karras<<<blocks_for(n - 1, 256), 256, 0, st>>>(codes, n, nodes, parent);
        float *ibox = reinterpret_cast<float *>(ws + L.ibox);
        k_refit<<<bgrid, 256, 0, st>>>(leaf_boxes, parent, nodes, ibox, visit, n);
        k_fill_nodes<<<blocks_for(L.n_int, 256), 256, 0, st>>>(leaf_boxes, ibox, reinterpret_cast<float *>(nodes),
                                                                L.n_int, h);
    } else {
        (void)hipMemcpyAsync(h->root_box, leaf_boxes, 6 * sizeof(float), hipMemcpyDeviceToDevice, st);
    }
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

int launch_build(const rs_gaussians *g, float Q, bool lbvh, char *ws, hipStream_t st)
{
    const int64_t n = g->n;
    const int bgrid = blocks_for(n, 256);
    auto rec = [&](const uint32_t *perm, float4 *records, float *leaf_boxes, int32_t *inv, WsHeader *) {
        k_records<<<bgrid, 256, 0, st>>>(perm, g->mean, g->scale, g->quat, g->opacity, n, Q, records, leaf_boxes, inv);
    };
    return build_core(n, g->mean, g->scale, g->quat, g->opacity, g->rgb, ws, st, rec, true, lbvh);
}

int launch_build_mesh(const rs_mesh *m, char *ws, hipStream_t st)
{
    const int64_t n = m->n_tris;
    Layout L = make_layout(n);
    WsHeader *h = reinterpret_cast<WsHeader *>(ws + L.header);
    k_init_header<<<1, 64, 0, st>>>(h);
    if (n == 0) return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
    const int bgrid = blocks_for(n, 256);
    float *cent = reinterpret_cast<float *>(ws + L.records);  // overwritten by the records afterwards
    k_tri_centroids<<<bgrid, 256, 0, st>>>(m->verts, m->tris, n, m->n_verts, cent, h);
    auto rec = [&](const uint32_t *perm, float4 *records, float *leaf_boxes, int32_t *inv, WsHeader *hh) {
        k_tri_records<<<bgrid, 256, 0, st>>>(perm, m->verts, m->tris, m->material, n, m->n_verts, records, leaf_boxes,
                                             inv, hh);
    };
    return build_core(n, cent, nullptr, nullptr, nullptr, nullptr, ws, st, rec, false, false);
}

}  // namespace rs
