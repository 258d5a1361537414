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
        for (int k = 0; k < 12; ++k) h->counters[k] = 0;
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
    double a = quat[4 * i], b = quat[4 * i + 1], c = quat[4 * i + 2], d = quat[4 * i + 3];
    double nq = a * a + b * b + c * c + d * d;
    if (!(nq > 0.0)) {
        a = 1.0;
        b = c = d = 0.0;
        nq = 1.0;
    }
    double s = 2.0 / nq;
    double R[3][3];
    R[0][0] = 1.0 - s * (c * c + d * d);
    R[0][1] = s * (b * c - a * d);
    R[0][2] = s * (b * d + a * c);
    R[1][0] = s * (b * c + a * d);
    R[1][1] = 1.0 - s * (b * b + d * d);
    R[1][2] = s * (c * d - a * b);
    R[2][0] = s * (b * d - a * c);
    R[2][1] = s * (c * d + a * b);
    R[2][2] = 1.0 - s * (b * b + c * c);
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
    // half extent along world axis k: sqrt(Q * sum_c (R_kc s_c)^2), padded
    for (int k = 0; k < 3; ++k) {
        double e2 = 0.0;
        for (int cc = 0; cc < 3; ++cc) {
            double v = R[k][cc] * sc[cc];
            e2 += v * v;
        }
        double e = sqrt(double(Q) * e2) * (1.0 + 1e-5) + 1e-7 * (1.0 + fabs(m[k]));
        leaf_boxes[6 * j + k] = __double2float_rd(m[k] - e);
        leaf_boxes[6 * j + 3 + k] = __double2float_ru(m[k] + e);
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

// ------------------------------------------------------------------- host

static inline int blocks_for(int64_t n, int threads) { return int((n + threads - 1) / threads); }

// Sort + link + refit shared by the Gaussian and the triangle BVH: `points`
// are the Morton sites; `records_fn` writes records and leaf boxes in sorted
// order once the permutation is known.
template <typename RecordsFn>
static int build_core(int64_t n, const float *points, const float *scale, const float *quat, const float *opacity,
                      const float *rgb, char *ws, hipStream_t st, RecordsFn records_fn, bool init_header)
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
    if (n >= 2) {
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

int launch_build(const rs_gaussians *g, float Q, char *ws, hipStream_t st)
{
    const int64_t n = g->n;
    const int bgrid = blocks_for(n, 256);
    auto rec = [&](const uint32_t *perm, float4 *records, float *leaf_boxes, int32_t *inv, WsHeader *) {
        k_records<<<bgrid, 256, 0, st>>>(perm, g->mean, g->scale, g->quat, g->opacity, n, Q, records, leaf_boxes, inv);
    };
    return build_core(n, g->mean, g->scale, g->quat, g->opacity, g->rgb, ws, st, rec, true);
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
    return build_core(n, cent, nullptr, nullptr, nullptr, nullptr, ws, st, rec, false);
}

}  // namespace rs
