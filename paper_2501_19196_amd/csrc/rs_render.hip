// Ray-packet traversal, ellipsoid intersection, depth-ordered compositing and
// its adjoint, for gfx950 (wave64).
//
// One wavefront traces one packet of 64 rays (an 8x8 pixel tile). The whole
// wave walks the BVH together: node and Gaussian records are fetched once per
// wave (uniform addresses, scalar loads) and every lane tests them against its
// own ray; a child is entered when any lane's ray overlaps it (ballot). The
// traversal stack is wave-uniform and lives in one VGPR (entry k in lane k).
//
// Each lane keeps its K nearest not-yet-composited hits, ordered by the key
// (t1, Gaussian index), in registers. A round traverses the BVH collecting
// the K smallest keys above the previous round's last key (nodes are culled
// against [last t, K-th t]), then composites them front to back (Eq. 3) with
// the K_max and eps1 stops (Sec. 3, "Color Aggregation"). Rounds repeat
// until every lane has stopped or run out of hits.
//
// The adjoint (App. A.3-A.6) walks each ray's composited hits back to front,
// either from the forward's stored lists or by traversing the BVH again in
// rounds that collect the K largest keys below the previous round's first
// one. The colour seen behind hit k, S_{k+1}, is built back to front
// (S <- alpha c + (1 - alpha) S from the background), so dL/dalpha_k =
// T_k <g, c_k - S_{k+1}> needs no division by 1 - alpha_k. T_k comes from the
// final T as T_{k+1} / (1 - alpha_k) (a relative error of about 2 ulp per
// hit), restarted from the T the forward saved where T left the normal floats
// (reached 0 when alpha = 1, or underflowed). The
// gradients of alpha with respect to the Gaussian parameters follow App. A.6
// in a cancellation-free form (see grad_hit). Per-Gaussian gradient
// contributions of a wave are summed across lanes before one set of float32
// atomics per Gaussian.
#include <math.h>

#include "rs_device.h"

#pragma clang fp contract(on)

namespace rs {

struct RenderParams {
    int64_t n_packets;         // all sets
    int64_t packets_per_set;   // every set has the same ray layout (views / packets)
    int64_t n_rays;            // rays per set
    int64_t n_gauss;
    int32_t root;
    int32_t stack_depth;
    float Q, eps1, t_min;
    int32_t max_hits;
    uint32_t flags;
    int32_t persistent;
    int32_t brute;
    int32_t count;
    int32_t n_views;
    int32_t tile_shift;
    int32_t strip_tiles;   // persistent: tile strip width of the packet order (0 = row-major)
    int32_t lists;         // stored hit lists: the forward appends rows, the adjoint replays them
    int32_t overflow_only; // traversal adjoint next to stored lists: only rays whose list is incomplete
    int32_t paper;         // RS_PAPER_GRADIENT: second phase after an eps1 stop
    float eps2;
    int64_t chunk;         // persistent: packets per XCD queue
    ViewEntry views[RS_MAX_VIEWS];
};

// ------------------------------------------------------------ intersection

// Ray / confidence-ellipsoid test (Sec. 3, Prop. 1, Prop. 2) for the record
// r0..r3 (R^T, 1/s, mean, opacity). With x = o - m, the whitened ray is
// o' = D R^T x, d' = D R^T d (D = diag(1/s)); its squared distance to the
// origin is h^2 = |o' x d'|^2 / |d'|^2 and o' x d' = cof(D) R^T (x cross d)
// with cof(D) = (D1 D2, D0 D2, D0 D1): every term is a sum of squares, so flat
// Gaussians (one scale -> 0) lose no precision to cancellation. The nearer
// root is t1 = -b/a - sqrt((Q - h^2)/a) for b = <o',d'> >= 0 and the Viete
// form (|o'|^2 - Q) / (a t*) otherwise (Prop. 1, App. A.1).
// Intermediates of the test that the adjoint of a hit reuses (the body-frame
// offset y = R^T (o - m) and direction e = R^T d, the scaled cross product u,
// b = <o',d'>, 1/a).
struct HitGeom {
    float y0, y1, y2, e0, e1, e2, u0, u1, u2, b, ia;
};

// The test in two parts, so a wave can skip the second when no lane's ray meets the ellipsoid.
// First part: the whitened geometry and h^2.
__device__ inline float ellipsoid_h2(const Ray &ray, const float4 r0, const float4 r1, const float4 r2, const float4 r3,
                                     HitGeom &G)
{
    const float xx = ray.ox - r3.x, xy = ray.oy - r3.y, xz = ray.oz - r3.z;
    // rows of R^T
    const float a00 = r0.x, a01 = r0.y, a02 = r0.z, a10 = r0.w, a11 = r1.x, a12 = r1.y, a20 = r1.z, a21 = r1.w,
                a22 = r2.x;
    const float D0 = r2.y, D1 = r2.z, D2 = r2.w;
    const float y0 = a00 * xx + a01 * xy + a02 * xz;
    const float y1 = a10 * xx + a11 * xy + a12 * xz;
    const float y2 = a20 * xx + a21 * xy + a22 * xz;
    const float e0 = a00 * ray.dx + a01 * ray.dy + a02 * ray.dz;
    const float e1 = a10 * ray.dx + a11 * ray.dy + a12 * ray.dz;
    const float e2 = a20 * ray.dx + a21 * ray.dy + a22 * ray.dz;
    // R^T ((o - m) x d) = y x e: a rotation preserves cross products
    const float v0 = y1 * e2 - y2 * e1;
    const float v1 = y2 * e0 - y0 * e2;
    const float v2 = y0 * e1 - y1 * e0;
    const float o0 = D0 * y0, o1 = D1 * y1, o2 = D2 * y2;
    const float d0 = D0 * e0, d1 = D1 * e1, d2 = D2 * e2;
    const float u0 = (D1 * D2) * v0, u1 = (D0 * D2) * v1, u2 = (D0 * D1) * v2;
    const float a = d0 * d0 + d1 * d1 + d2 * d2;
    const float b = o0 * d0 + o1 * d1 + o2 * d2;
    const float uu = u0 * u0 + u1 * u1 + u2 * u2;
    const float ia = __builtin_amdgcn_rcpf(a);
    G = HitGeom{y0, y1, y2, e0, e1, e2, u0, u1, u2, b, ia};
    return uu * ia;
}

// Second part: the nearer root t1 (meaningful where h2 <= Q). Both root forms are computed for
// every lane and one is selected, no divergent branch (where the ray hits the chosen form is
// the same arithmetic).
__device__ inline float ellipsoid_t1(const HitGeom &G, const float4 r2, float h2, float Q)
{
    const float D0 = r2.y, D1 = r2.z, D2 = r2.w;
    const float o0 = D0 * G.y0, o1 = D1 * G.y1, o2 = D2 * G.y2;
    const float sq = __builtin_amdgcn_sqrtf((Q - h2) * G.ia);  // hardware square root (1 ulp)
    const float tc = -G.b * G.ia;
    const float oo = o0 * o0 + o1 * o1 + o2 * o2;
    const float t_viete = ((oo - Q) * G.ia) * __builtin_amdgcn_rcpf(tc + sq);
    float t1 = G.b >= 0.0f ? tc - sq : t_viete;
    if (t1 == 0.0f) t1 = 0.0f;  // -0 -> +0 so the key order matches float order
    return t1;
}

__device__ inline bool ellipsoid_hit(const Ray &ray, const float4 r0, const float4 r1, const float4 r2, const float4 r3,
                                     float Q, float &t1, float &h2, HitGeom &G)
{
    h2 = ellipsoid_h2(ray, r0, r1, r2, r3, G);
    t1 = ellipsoid_t1(G, r2, h2, Q);
    return h2 <= Q;
}

// ------------------------------------------------------------- hit buffer

// A hit's sort key (t1, Gaussian index) packed into the bit pattern of a
// positive normal double: ((float bits of t1) + 2^20) << 32 | index. For
// t1 >= 0 the double order is the (t1, index) order, so a sorted insert is a
// chain of v_min_f64 / v_max_f64 (no compares, selects or hazards).
constexpr uint32_t kKeyBias = 0x00100000u;  // keeps every key a normal double
constexpr double kNoHit = __builtin_huge_val();  // empty slot, above every key

__device__ inline double hit_key(float t1, uint32_t gid)
{
    const uint64_t hi = uint64_t(__float_as_uint(t1) + kKeyBias);
    return __longlong_as_double((long long)((hi << 32) | gid));
}
__device__ inline float hit_key_t(double k)
{
    return __uint_as_float(uint32_t(uint64_t(__double_as_longlong(k)) >> 32) - kKeyBias);
}
__device__ inline uint32_t hit_key_gid(double k) { return uint32_t(uint64_t(__double_as_longlong(k))); }

// Sorted insert of k into the ascending keys key[0..N): slot s becomes max(key[s-1],
// min(key[s], k)) and slot 0 min(key[0], k), each from the old keys, so the 2N operations do
// not form a chain through a carried key. They are issued from the back, each max three slots
// behind its min, so a min's result is read five instructions later (f64 results need wait
// states before they are read; two slots behind left some). The keys are never NaN, so the
// min/max are the bare instructions (the generic fmin/fmax would first quiet every key in IEEE
// mode). OUT: returns max(key[N-1], k), the key pushed out (else kNoHit).
template <int N, bool OUT>
__device__ inline double sorted_insert(double (&key)[N], double k)
{
    double out = kNoHit;
    if (OUT) asm volatile("v_max_f64 %0, %1, %2" : "=v"(out) : "v"(key[N - 1]), "v"(k));
    double t[N];
#pragma unroll
    for (int s = N - 1; s >= -2; --s) {
        if (s >= 0) asm volatile("v_min_f64 %0, %1, %2" : "=v"(t[s]) : "v"(key[s]), "v"(k));
        const int m = s + 3;  // the slot whose max is due
        if (m >= 1 && m <= N - 1) asm volatile("v_max_f64 %0, %1, %2" : "=v"(key[m]) : "v"(key[m - 1]), "v"(t[m]));
    }
    key[0] = t[0];
    return out;
}

template <int K>
struct HitBuf {
    static constexpr int size = K;
    double key[K];  // sorted ascending; kNoHit marks an empty slot

    __device__ inline void clear()
    {
#pragma unroll
        for (int s = 0; s < K; ++s) key[s] = kNoHit;
    }
    __device__ inline double front() const { return key[0]; }
    __device__ inline double last() const { return key[K - 1]; }

    // drop the front entry (static register moves: no dynamic indexing)
    __device__ inline void pop_front()
    {
#pragma unroll
        for (int s = 0; s + 1 < K; ++s) key[s] = key[s + 1];
        key[K - 1] = kNoHit;
    }

    // sorted insert of k; the last entry falls off (inserting kNoHit changes nothing). The keys
    // are never NaN, so the min/max are the bare instructions: the generic fmin/fmax would first
    // quiet every loop-carried key (one more v_max_f64 per entry in IEEE mode).
    __device__ inline void insert(double k) { sorted_insert<K, false>(key, k); }
};

// The same sorted buffer of KR + KT keys with its last KT entries in LDS: a per-wave ring of KT
// slots of 64 lanes (slot-major, so one slot of the wave is one contiguous 512-byte row) whose
// wave-uniform head is the tail's first entry. The registers hold the KR smallest keys. An
// insertion runs the register chain, then carries its key on through the tail when some lane
// carries one; a pop shifts the registers and takes the tail's first entry into the last one.
// `kmax` mirrors the buffer's last entry, so the candidate test and the culling bound need no
// LDS read. The workgroup is one wave.
#ifndef RS_RING_GROUP
#define RS_RING_GROUP 8
#endif
template <int KR, int KT>
struct HitBufTail {
    static constexpr int size = KR + KT;
    double key[KR];
    double kmax;
    int32_t head;
    double *ring;  // this wave's LDS ring, KT x 64 doubles
    int lane;

    __device__ inline void clear()
    {
#pragma unroll
        for (int s = 0; s < KR; ++s) key[s] = kNoHit;
        kmax = kNoHit;
        head = 0;
#pragma unroll
        for (int i = 0; i < KT; ++i) ring[i * kWave + lane] = kNoHit;
    }
    __device__ inline double front() const { return key[0]; }
    __device__ inline double last() const { return kmax; }

    __device__ inline void pop_front()
    {
#pragma unroll
        for (int s = 0; s + 1 < KR; ++s) key[s] = key[s + 1];
        double *e = ring + head * kWave + lane;
        key[KR - 1] = *e;
        *e = kNoHit;
        head = head + 1 == KT ? 0 : head + 1;
        kmax = kNoHit;
    }

    __device__ inline void insert(double k)
    {
        k = sorted_insert<KR, true>(key, k);
        if (!wave_ballot(k != kNoHit)) return;  // every carried key fell into an empty register slot
        // the ring's entries are read RG at a time (their LDS reads in flight together), then
        // passed through the min/max chain and written back
        constexpr int RG = RS_RING_GROUP;
        static_assert(KT % RG == 0, "ring group");
        int32_t p = head;
#pragma unroll
        for (int g = 0; g < KT; g += RG) {
            double t[RG];
            double *e[RG];
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                e[i] = ring + p * kWave + lane;
                p = p + 1 == KT ? 0 : p + 1;
            }
#pragma unroll
            for (int i = 0; i < RG; ++i) t[i] = *e[i];
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                double hi = 0.0;
                if (g + i + 1 < KT) asm volatile("v_max_f64 %0, %1, %2" : "=v"(hi) : "v"(t[i]), "v"(k));
                asm volatile("v_min_f64 %0, %0, %1" : "+v"(t[i]) : "v"(k));
                if (g + i + 1 == KT) kmax = t[i];
                k = hi;
            }
#pragma unroll
            for (int i = 0; i < RG; ++i) *e[i] = t[i];
        }
    }
};

// The forward's buffer for a hit-buffer size K. At K = 48 the last 16 keys live in LDS (8 KB
// per wave): 32 keys in registers let the kernel run four waves per SIMD instead of three,
// which hides more of the node and record fetch latency than the LDS traffic of the tail costs
// (measured: 9.6 against 10.5 ms at the scene-scale workload; 28 + 20 keys 9.7, 36 + 12 9.6,
// 40 + 8 10.3). At K = 32 the same split loses (16 + 16 keys at five waves: 10.5 against 10.3).
constexpr int kTailKeys = 16;
template <int K>
struct FwdBuf {
    using type = HitBuf<K>;
};
template <>
struct FwdBuf<48> {
    using type = HitBufTail<48 - kTailKeys, kTailKeys>;
};

// ------------------------------------------------------------- compositing

// One front-to-back step (Eq. 3): shared by the forward and adjoint kernels so
// both see bit-identical T and C sequences.
struct Accum {
    float T, Cr, Cg, Cb;
    int n;
};

__device__ inline void composite_step(Accum &A, float a, float cr, float cg, float cb)
{
    const float w = A.T * a;
    A.Cr = __builtin_fmaf(w, cr, A.Cr);
    A.Cg = __builtin_fmaf(w, cg, A.Cg);
    A.Cb = __builtin_fmaf(w, cb, A.Cb);
    const float om = 1.0f - a;
    A.T = A.T * om;
    A.n += 1;
}

__device__ inline bool stop_after(const Accum &A, const RenderParams &P)
{
    return A.T < P.eps1 || (P.max_hits > 0 && A.n >= P.max_hits);
}

// --------------------------------------------------------------- adjoint

// Gradient of h^2 (and so of alpha = opacity exp(-h^2/2)) for one hit, in the
// Gaussian's body frame. With p = o' - (b/a) d' (the whitened closest point,
// obtained without cancellation as p = (d' x u) / a, u = o' x d'), D = diag(1/s)
// and y_w = y - (b/a) e the body-frame closest-approach offset, App. A.6 gives
//   dh2/dm = -2 R D p,   dh2/ds_k = -2 D_k p_k^2,   dh2/dR = 2 R y_w (D p)^T.
// The rotation enters only through R^T dh2/dR, whose antisymmetric part is the
// angular vector w = 2 (D p) x y_w: a change dR = R [dtheta]x changes h2 by
// <w, dtheta>. So a hit contributes, per Gaussian,
//   acc_m = gh D p,  acc_s = -2 gh D_k p_k^2,  acc_w = 2 gh (D p) x y_w,
// (gh = dL/dh2), and k_scatter_grads applies R and the quaternion map once per
// Gaussian: dL/dm = -2 R acc_m, dL/dq = (2/|q|) E(q/|q|)^T acc_w, where
// dtheta = (2/|q|) E(n) dq, E(n) = [-v | w I - [v]x] for n = (w, v).
struct GradOut {
    float v[13];  // mean (body frame) 3, scale 3, angular 3, opacity 1, rgb 3
};

__device__ inline void grad_hit(const float4 r2, const HitGeom &g, float h2, float dLda, float alpha, GradOut &G)
{
    const float D0 = r2.y, D1 = r2.z, D2 = r2.w;
    const float d0 = D0 * g.e0, d1 = D1 * g.e1, d2 = D2 * g.e2;
    // p = (d' x u) / a
    const float p0 = (d1 * g.u2 - d2 * g.u1) * g.ia;
    const float p1 = (d2 * g.u0 - d0 * g.u2) * g.ia;
    const float p2 = (d0 * g.u1 - d1 * g.u0) * g.ia;
    const float Dp0 = D0 * p0, Dp1 = D1 * p1, Dp2 = D2 * p2;
    const float ba = g.b * g.ia;
    const float w0 = g.y0 - ba * g.e0, w1 = g.y1 - ba * g.e1, w2 = g.y2 - ba * g.e2;
    const float gh = dLda * (-0.5f * alpha);  // dL/dh2
    G.v[0] = gh * Dp0;
    G.v[1] = gh * Dp1;
    G.v[2] = gh * Dp2;
    G.v[3] = gh * (-2.0f * Dp0 * p0);
    G.v[4] = gh * (-2.0f * Dp1 * p1);
    G.v[5] = gh * (-2.0f * Dp2 * p2);
    const float c = 2.0f * gh;
    G.v[6] = c * (Dp1 * w2 - Dp2 * w1);
    G.v[7] = c * (Dp2 * w0 - Dp0 * w2);
    G.v[8] = c * (Dp0 * w1 - Dp1 * w0);
    // opacity: alpha = opacity * exp(-h2/2)
    G.v[9] = dLda * __expf(-0.5f * h2);
}

// ----------------------------------------------------------------- kernel

// One set of rays traced by a launch: its rays, optional per-ray limit and
// background, outputs (forward) or upstream gradient (adjoint), and its state.
struct RaySet {
    const float *origin, *dir, *tmax, *bgray, *grad;
    float *out_rgb;
    float4 *fin;  // final colour and T
    uint4 *last;  // last composited key, restart point of the T recursion
    int4 *list;   // stored-list bookkeeping (hit lists only)
    float bg[3];
    int32_t zero_colour;
};

struct Ptrs {
    const float *rgb;
    RaySet set[kMaxSets];
    int32_t *status;
    uint32_t *queue;  // XCD queue counters (kXcdQueues)
    unsigned long long *counters;
    float *gacc;  // adjoint accumulator, 16 floats per Gaussian (see k_scatter_grads)
    ListPool pool;
};

// ------------------------------------------------------- shared kernel steps

// Next packet of a wave (wave-uniform; n_packets when there is none). Plain
// grids take one packet per workgroup; persistent ones first drain the queue
// of their own XCD's chunk (a compact image region, so that XCD's L2 holds
// its working set), then take from the other chunks.
#ifndef RS_XCD_RUN
#define RS_XCD_RUN 32
#endif
constexpr int64_t kXcdRun = RS_XCD_RUN;

template <typename PT>
__device__ inline int64_t next_packet(const PT &P, uint32_t *queue, int lane, int xcd, int &qi, int64_t &iter)
{
    if (!P.persistent) {
        // plain grid: workgroups are dealt to the XCDs in turn, so workgroup b runs on XCD
        // b mod 8. Packets are dealt in runs of kXcdRun consecutive ones (a compact strip of
        // tiles), so the waves an XCD runs at a time share fewer Gaussians in its L2, while
        // every XCD still samples the whole image (the grid is rounded up to whole deals; the
        // few packets beyond n_packets exit)
        if (iter++ > 0) return P.n_packets;
        const int64_t b = blockIdx.x, i = b / kXcdQueues;
        return (i / kXcdRun * kXcdQueues + b % kXcdQueues) * kXcdRun + i % kXcdRun;
    }
    while (qi < kXcdQueues) {
        const int q = (xcd + qi) & (kXcdQueues - 1);
        uint32_t p = 0;
        if (lane == 0) p = atomicAdd(queue + q, 1u);
        p = __builtin_amdgcn_readfirstlane(p);
        const int64_t g = q * P.chunk + p;
        if (g < P.n_packets && p < P.chunk) return g;
        ++qi;
    }
    return P.n_packets;
}

__device__ inline int xcd_id() { return int(__builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11))) & (kXcdQueues - 1); }

// A lane's ray of packet `pkt`: its set, index, geometry, t_max and background.
struct LaneRay {
    int si;
    bool valid;
    int64_t id;
    Ray ray;
    float tmax, bgr, bgg, bgb;
};

template <typename PT>
__device__ inline LaneRay lane_ray(const PT &P, const Ptrs &ptr, int64_t pkt, int lane)
{
    LaneRay L;
    L.si = 0;
    while (L.si + 1 < kMaxSets && pkt >= int64_t(L.si + 1) * P.packets_per_set) ++L.si;
    const RaySet &S = ptr.set[L.si];
    const int64_t local = pkt - L.si * P.packets_per_set;
    L.id = packet_ray(P, P.persistent ? strip_major_packet(P, local, P.strip_tiles) : local, lane, L.valid);
    L.tmax = kInf;
    L.bgr = S.bg[0];
    L.bgg = S.bg[1];
    L.bgb = S.bg[2];
    if (L.valid) {
        L.ray.ox = S.origin[3 * L.id];
        L.ray.oy = S.origin[3 * L.id + 1];
        L.ray.oz = S.origin[3 * L.id + 2];
        L.ray.dx = S.dir[3 * L.id];
        L.ray.dy = S.dir[3 * L.id + 1];
        L.ray.dz = S.dir[3 * L.id + 2];
        if (S.tmax) L.tmax = S.tmax[L.id];
        if (S.bgray) {
            L.bgr = S.bgray[3 * L.id];
            L.bgg = S.bgray[3 * L.id + 1];
            L.bgb = S.bgray[3 * L.id + 2];
        }
    } else {
        L.ray.ox = L.ray.oy = L.ray.oz = 0.0f;
        L.ray.dx = L.ray.dy = 0.0f;
        L.ray.dz = 1.0f;
    }
    return L;
}

// One composited hit (Eq. 3): the record of Gaussian gid is fetched, alpha is
// recomputed with the leaf test's own arithmetic (so every kernel sees the
// same alpha bit for bit) and the front-to-back step is applied.
struct HitData {
    float4 r0, r1, r2, r3;
    float al, cr, cg, cb, Tk;
    float t1, h2;  // entry distance (the hit key's t) and squared whitened distance
    HitGeom g;
};

// alpha of the Gaussian at sorted position js along the ray, with the leaf test's own arithmetic
__device__ inline float hit_alpha_at(int32_t js, const Ray &ray, const float4 *__restrict__ records, float Q,
                                     float4 &r0, float4 &r1, float4 &r2, float4 &r3, float &t1, float &h2,
                                     HitGeom &G)
{
    r0 = records[4 * js + 0];
    r1 = records[4 * js + 1];
    r2 = records[4 * js + 2];
    r3 = records[4 * js + 3];
    ellipsoid_hit(ray, r0, r1, r2, r3, Q, t1, h2, G);
    return r3.w * __expf(-0.5f * h2);
}

// the same for Gaussian gid
__device__ inline float hit_alpha(uint32_t gid, const Ray &ray, const float4 *__restrict__ records,
                                  const int32_t *__restrict__ inv, float Q, float4 &r0, float4 &r1, float4 &r2,
                                  float4 &r3, float &t1, float &h2, HitGeom &G)
{
    return hit_alpha_at(inv[gid], ray, records, Q, r0, r1, r2, r3, t1, h2, G);
}

// alpha, colour and test intermediates of a hit (no compositing). EVERY: every lane
// computes, the caller giving idle lanes a valid Gaussian index whose values it never
// uses, so no lane is masked off and nothing is zeroed first.
template <bool EVERY = false>
__device__ inline void recompute_hit(bool act, uint32_t gid, const Ray &ray, const float4 *__restrict__ records,
                                     const int32_t *__restrict__ inv, const float *__restrict__ rgb, bool zc, float Q,
                                     HitData &H)
{
    H.Tk = 0.0f;
    if (!EVERY) {
        H.al = H.cr = H.cg = H.cb = H.t1 = H.h2 = 0.0f;
        H.g = HitGeom{};
    }
    if (EVERY || act) {
        H.al = hit_alpha(gid, ray, records, inv, Q, H.r0, H.r1, H.r2, H.r3, H.t1, H.h2, H.g);
        H.cr = H.cg = H.cb = 0.0f;
        if (!zc) {
            H.cr = rgb[3 * gid];
            H.cg = rgb[3 * gid + 1];
            H.cb = rgb[3 * gid + 2];
        }
    }
}

// (js: the hit's sorted position, looked up by the caller ahead of time)
__device__ inline void composite_hit(bool act, uint32_t gid, int32_t js, const Ray &ray,
                                     const float4 *__restrict__ records, const float *__restrict__ rgb, bool zc,
                                     const RenderParams &P, Accum &A, HitData &H)
{
    H.al = H.cr = H.cg = H.cb = H.t1 = H.h2 = 0.0f;
    H.g = HitGeom{};
    if (act) {
        H.al = hit_alpha_at(js, ray, records, P.Q, H.r0, H.r1, H.r2, H.r3, H.t1, H.h2, H.g);
        if (!zc) {
            H.cr = rgb[3 * gid];
            H.cg = rgb[3 * gid + 1];
            H.cb = rgb[3 * gid + 2];
        }
    }
    H.Tk = A.T;
    if (act) composite_step(A, H.al, H.cr, H.cg, H.cb);
}

// ------------------------------------------------------- back-to-front adjoint

// Smallest normal float: below it T loses relative precision, so the adjoint does not
// divide back from there (the forward saves the T before the hit that crossed it).
constexpr float kMinNormal = 1.17549435e-38f;

// Upstream gradient of a lane's pixel.
struct LaneGrad {
    float gr, gg, gb;
};

// Back-to-front state of a lane's adjoint: T_{k+1} (the transmittance behind
// the hit being processed), the colour S_{k+1} seen behind it (background
// first), the hits done so far, and where the forward's T fell below the normal
// floats: the T just before that hit (Tz) and how many composited hits followed
// it (mz, -1 when T stayed normal). Behind that hit T is taken as 0 (it is below
// 1.2e-38 there).
struct Back {
    float T, Sr, Sg, Sb, Tz;
    int32_t done, mz;
};

__device__ inline Back back_init(const float4 fin, const uint4 last, float bgr, float bgg, float bgb)
{
    Back B;
    B.T = fin.w;
    B.Sr = bgr;
    B.Sg = bgg;
    B.Sb = bgb;
    B.Tz = __uint_as_float(last.z);
    B.mz = int32_t(last.w);
    B.done = 0;
    return B;
}

// T_k of the next hit (back to front) with opacity al: T_{k+1} / (1 - al), except
// 0 behind the hit that took T below the normal floats and the saved T at that hit
// (a select, so a quotient 0/0 there is never used).
__device__ inline float back_T(const Back &B, float al)
{
    const float Td = B.T * __builtin_amdgcn_rcpf(1.0f - al);
    return B.done < B.mz ? 0.0f : (B.done == B.mz ? B.Tz : Td);
}

// hit k (alpha al, colour c) now lies behind the next hit: S <- al c + (1 - al) S
__device__ inline void back_over(Back &B, float al, float cr, float cg, float cb)
{
    B.Sr = __builtin_fmaf(al, cr - B.Sr, B.Sr);
    B.Sg = __builtin_fmaf(al, cg - B.Sg, B.Sg);
    B.Sb = __builtin_fmaf(al, cb - B.Sb, B.Sb);
}

// Per-wave gradient accumulation in LDS (the traversal adjoint): a table of Gaussian slots,
// each holding the 13 partial sums of one Gaussian, found by hashing its index with linear
// probing over kAccProbes slots. Every hit adds its values into its Gaussian's slot with LDS
// atomics; a slot's sums reach the global accumulators (one 64-byte line per Gaussian) only
// when the table is flushed: when some lane finds no slot in its probe window, and at the end
// of the kernel. The hits of one Gaussian on the rays of a packet, over every compositing
// step, so cost one line of global atomics per flush instead of one per step. The workgroup
// is one wave.
constexpr int kAccSlots = 128;
constexpr int kAccProbes = 8;
constexpr int kAccVals = 13;
struct AccTable {
    int32_t tag[kAccSlots];           // Gaussian index, -1: free
    int32_t list[kAccSlots];          // occupied slots, compacted by a flush
    float acc[kAccSlots * kAccVals];  // partial sums (odd stride: distinct slots, distinct banks)
};

__device__ inline AccTable &acc_table()
{
    __shared__ AccTable T;
    return T;
}

__device__ inline void acc_clear(AccTable &T, int lane)
{
    for (int s = lane; s < kAccSlots; s += kWave) T.tag[s] = -1;
    for (int s = lane; s < kAccSlots * kAccVals; s += kWave) T.acc[s] = 0.0f;
    __syncthreads();
}

__device__ inline uint32_t acc_home(uint32_t gid)
{
    return uint32_t((uint64_t(gid * 2654435761u) * uint64_t(kAccSlots)) >> 32);
}

// Adds every occupied slot's sums to the global accumulators (16-lane segments, one slot
// each, lane v of a segment adding value v) and frees the table.
template <bool COUNT>
__device__ inline void acc_flush(AccTable &T, float *gacc, int lane, uint64_t &c_group)
{
    __syncthreads();
    int32_t cnt = 0;
    for (int base = 0; base < kAccSlots; base += kWave) {
        const int s = base + lane;
        const bool occ = s < kAccSlots && T.tag[s] != -1;
        const uint64_t m = wave_ballot(occ);
        if (occ) T.list[cnt + int32_t(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)))] = s;
        cnt += __popcll(m);
    }
    __syncthreads();
    const int v = lane & 15, q = lane >> 4;
    for (int i = 0; i < cnt; i += 4) {
        const int k = i + q;
        if (k < cnt && v < kAccVals) {
            const int s = T.list[k];
            const uint32_t g = uint32_t(T.tag[s]);
            float *a = T.acc + s * kAccVals + v;
            unsafeAtomicAdd(gacc + 16 * int64_t(g) + v, *a);
            *a = 0.0f;
        }
    }
    if (COUNT) c_group += uint64_t(cnt);
    __syncthreads();
    for (int s = lane; s < kAccSlots; s += kWave) T.tag[s] = -1;
    __syncthreads();
}

// One step of the pairwise sum: lanes paired by the DPP pattern CTRL (an involution) that
// hold the same Gaussian are merged into the `keep` lane of the pair. Called with every lane
// of the wave active.
template <int CTRL>
__device__ inline void acc_pair(bool &act, uint32_t gid, GradOut &G, bool keep)
{
    const int32_t pg = __builtin_amdgcn_mov_dpp(int32_t(gid), CTRL, 0xF, 0xF, false);
    const int32_t pa = __builtin_amdgcn_mov_dpp(act ? 1 : 0, CTRL, 0xF, 0xF, false);
    const bool m = act && pa != 0 && pg == int32_t(gid);
#pragma unroll
    for (int v = 0; v < kAccVals; ++v) {
        const float pv = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(G.v[v]), CTRL, 0xF, 0xF, false));
        G.v[v] = (m && keep) ? G.v[v] + pv : G.v[v];
    }
    act = act && !(m && !keep);
}

// Adjoint of one composited hit (App. A.3-A.6) and its wave aggregation.
//   dL/dalpha_k = T_k <g, c_k - S_{k+1}>,  dL/dc_k = alpha_k T_k g,
// then alpha's chain rule (grad_hit). TABLE: the contributions go into the wave's LDS table
// (the traversal adjoint, whose long traversal hides the LDS atomics). Otherwise (the stored-
// list adjoint, where the table's same-address LDS atomics would be the bottleneck) the active
// lanes' contributions are summed per distinct Gaussian of this step through LDS, and one
// 13-lane segment of an atomic instruction adds each Gaussian's totals to its 64-byte
// accumulator line (four Gaussians per instruction).
template <bool COUNT, bool TABLE>
__device__ inline void adjoint_hit(bool act, uint64_t act_mask, uint32_t gid, const HitData &H, float Tk,
                                   const Back &B, const LaneGrad &Gd, bool zc, float *gacc, int lane, uint64_t &c_group)
{
    GradOut G;
    // the table path sums neighbouring lanes' values, so idle lanes contribute zeros; the
    // stored-list path stores active lanes' values only and computes on every lane
    if (TABLE) {
#pragma unroll
        for (int v = 0; v < 13; ++v) G.v[v] = 0.0f;
    }
    if (!TABLE || act) {
        const float dLda = Tk * (Gd.gr * (H.cr - B.Sr) + Gd.gg * (H.cg - B.Sg) + Gd.gb * (H.cb - B.Sb));
        grad_hit(H.r2, H.g, H.h2, dLda, H.al, G);
        const float wgt = H.al * Tk;
        G.v[10] = zc ? 0.0f : Gd.gr * wgt;
        G.v[11] = zc ? 0.0f : Gd.gg * wgt;
        G.v[12] = zc ? 0.0f : Gd.gb * wgt;
    }
    if constexpr (TABLE) {
        (void)act_mask;
        // Lanes of one 16-lane row holding the same Gaussian are first summed pairwise (lane^1,
        // lane^2, then mirrored halves and rows: neighbouring pixels of the packet tile), so
        // fewer LDS atomics meet at one address.
        acc_pair<0xB1>(act, gid, G, (lane & 1) == 0);   // quad_perm [1,0,3,2]
        acc_pair<0x4E>(act, gid, G, (lane & 2) == 0);   // quad_perm [2,3,0,1]
        acc_pair<0x141>(act, gid, G, (lane & 7) < 4);   // row_half_mirror
        acc_pair<0x140>(act, gid, G, (lane & 15) < 8);  // row_mirror
        AccTable &T = acc_table();
        const uint32_t home = acc_home(gid);
        bool pend = act;
        for (;;) {
            int32_t slot = -1;
            if (pend) {
                uint32_t h = home;
                for (int p = 0; p < kAccProbes; ++p) {
                    const int32_t old = atomicCAS(&T.tag[h], -1, int32_t(gid));
                    if (old == -1 || old == int32_t(gid)) {
                        slot = int32_t(h);
                        break;
                    }
                    h = h + 1 == uint32_t(kAccSlots) ? 0u : h + 1;
                }
            }
            if (slot >= 0) {
                float *a = T.acc + slot * kAccVals;
#pragma unroll
                for (int v = 0; v < kAccVals; ++v)
                    __hip_atomic_fetch_add(a + v, G.v[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                pend = false;
            }
            // lanes left without a slot: flush the table and probe again from their home slots
            if (!wave_ballot(pend)) break;
            acc_flush<COUNT>(T, gacc, lane, c_group);
        }
    } else {
        // Lanes holding the same Gaussian form a group; groups are numbered in order of their
        // lowest lane and each group's lanes store their 13 values in consecutive LDS rows. The
        // scalar loop keeps only masks and counts in scalar registers; a lane records its row,
        // and after the loop each group's lowest lane writes the group's (Gaussian, first row),
        // the next group's first row closing it. Then 16-lane segments sum one
        // group's rows each, so one atomic instruction adds the totals of four Gaussians (one
        // 64-byte accumulator line per segment). The wave is the whole workgroup, and its LDS
        // operations complete in order.
        __shared__ float rows[kWave * 16];
        __shared__ int2 groups[kWave + 1];  // Gaussian index, first row
        uint64_t todo = act_mask, leaders = 0;
        int32_t pos = 0, mypos = 0;
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const uint32_t lg = __builtin_amdgcn_readlane(gid, leader);
            const uint64_t same = wave_ballot(gid == lg) & todo;
            const bool mine = __builtin_amdgcn_inverse_ballot_w64(same);  // this lane is in the group
            todo &= ~same;
            leaders |= 1ull << leader;
            if (COUNT) ++c_group;
            const int32_t at = int32_t(
                __builtin_amdgcn_mbcnt_hi(uint32_t(same >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(same), uint32_t(pos))));
            mypos = mine ? at : mypos;
            pos += __popcll(same);
        }
        const int32_t ng = __popcll(leaders);
        // a group's number is the number of leaders below its leader (groups open in lane order)
        const int32_t mygrp = int32_t(
            __builtin_amdgcn_mbcnt_hi(uint32_t(leaders >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(leaders), 0u)));
        if (__builtin_amdgcn_inverse_ballot_w64(leaders)) groups[mygrp] = make_int2(int32_t(gid), mypos);
        if (lane == 0) groups[ng] = make_int2(0, pos);
        if (act) {
            float *r = rows + 16 * mypos;
#pragma unroll
            for (int v = 0; v < 13; ++v) r[v] = G.v[v];
        }
        // the segments read other lanes' rows and descriptors: a (one-wave) barrier keeps the
        // compiler from reusing a lane's own earlier stores in their place
        __syncthreads();
        const int v = lane & 15;
        for (int b = 0; b < ng; b += 4) {
            const int gi = b + (lane >> 4);
            if (gi < ng && v < 13) {
                const int2 gd = groups[gi];
                const int32_t end = groups[gi + 1].y;
                float t = rows[16 * gd.y + v];
                for (int j = gd.y + 1; j < end; ++j) t += rows[16 * j + v];
                unsafeAtomicAdd(gacc + 16 * int64_t(uint32_t(gd.x)) + v, t);
            }
        }
    }
}

// ------------------------------------------------------------ stored lists

// Row cursor of a packet's stored list (wave-uniform).
struct ListCursor {
    int32_t rows;   // rows stored
    int32_t chunk;  // current chunk (-1: none yet)
    int32_t fill;   // slots used in the current chunk
    int32_t slots;  // slots stored (rows and masks)
    bool ok;        // false once the pool was found exhausted
};

// Appends one row (called from wave-uniform control flow): the entries of the lanes
// whose `entry` is not kListIdle, in lane order, then their lane mask as two words.
// A row that does not fit the current chunk starts a new one, taken from the pool
// and linked to the packet's previous chunk. Once the pool is exhausted the packet
// stores nothing more (the adjoint then traverses for its rays, or, for the paper
// variant, the sticky status reports it).
__device__ inline void list_append(const ListPool &pool, ListCursor &L, uint32_t entry, int lane, int32_t &stored,
                                   bool paper, int32_t *status)
{
    if (!L.ok) return;
    const uint64_t m = wave_ballot(entry != kListIdle);
    if (m == 0) return;
    const int32_t need = __popcll(m) + 2;
    if (L.chunk < 0 || L.fill + need > kChunkSlots) {
        int32_t c = 0;
        if (lane == 0) {
            if (L.chunk >= 0) pool.fill[L.chunk] = L.fill;
            const unsigned long long k = atomicAdd(pool.hdr, 1ull);
            c = k < (unsigned long long)pool.chunks ? int32_t(k) : -1;
        }
        c = __builtin_amdgcn_readfirstlane(c);
        if (c < 0) {
            L.ok = false;
            if (lane == 0) {
                atomicOr(pool.hdr + 1, 1ull);
                if (paper) atomicOr(status, kStatusListPool);
            }
            return;
        }
        if (lane == 0) pool.prev[c] = L.chunk;
        L.chunk = c;
        L.fill = 0;
    }
    // The rows are streamed out with nontemporal stores: they are read back only by the adjoint,
    // after this launch, and the forward's own fetches wait less behind them.
    uint32_t *row = pool.slots + int64_t(L.chunk) * kChunkSlots + L.fill;
    if (entry != kListIdle) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
        __builtin_nontemporal_store(entry, row + below);
        if (entry < kListSecond) ++stored;
    }
    if (lane == 0) {
        __builtin_nontemporal_store(uint32_t(m), row + need - 2);
        __builtin_nontemporal_store(uint32_t(m >> 32), row + need - 1);
    }
    L.fill += need;
    L.slots += need;
    ++L.rows;
}

// Records the fill of the packet's last chunk (after its last row).
__device__ inline void list_close(const ListPool &pool, const ListCursor &L, int lane)
{
    if (L.ok && L.chunk >= 0 && lane == 0) pool.fill[L.chunk] = L.fill;
}

// min of two floats that are never NaN-signalling, as the bare instruction
__device__ inline float fmin_bare(float a, float b)
{
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

constexpr int32_t kDone = INT32_MIN;

// Wave-uniform descent from `node` through internal nodes to the next leaf
// (returned as ~leaf) or to the end of the walk (kDone). A child is entered
// when some live lane's ray overlaps its box within [t_lo, t_hi]; when both
// are, the one the leader lane reaches first (REV: leaves last) is taken and the
// other pushed (stack entry k lives in lane k of `stackv`). Ordering by the leader
// lane costs one compare instead of a vote and, in simulation at the scene-scale
// workload, visits within 0.5 % as many nodes as a majority vote. The loop has one exit (a
// full stack ends the walk through the same path as an empty one) and decides the
// two-children case with one scalar compare, which keeps the scalar control flow short.
template <int OCT, bool COUNT, bool REV>
__device__ inline int32_t descend(int32_t node, const float4 *__restrict__ nodes, const Slab &sl, uint64_t lead_bit,
                                  float t_lo, float t_hi_w, int lane, int32_t stack_depth, int32_t &sp,
                                  int32_t &stackv, bool &overflow, uint64_t &c_node, uint64_t &c_lchild)
{
    while (node >= 0) {
        const uint32_t ns = __builtin_amdgcn_readfirstlane(node);
        const float4 *nd = nodes + 4 * uint64_t(ns);
        const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2];
        const int2 lr = *reinterpret_cast<const int2 *>(nd + 3);
        float ln, lf, rn, rf;
        child_slabs<OCT>(n0, n1, n2, sl, ln, lf, rn, rf);
        // [max(near, t_lo), min(widened exit, t_hi)] non-empty as two compares against
        // x = min(widened exit, t_hi): t_lo <= t_hi holds on every live lane, and t_lo is NaN on
        // the others, so no compare passes there. The min is the bare instruction (t_hi is
        // loop-carried; the generic fminf would quiet it first).
        const float lx = fmin_bare(widen_exit(lf, sl.pad), t_hi_w), rx = fmin_bare(widen_exit(rf, sl.pad), t_hi_w);
        const uint64_t bl = wave_ballot(ln <= lx) & wave_ballot(t_lo <= lx);
        const uint64_t br = wave_ballot(rn <= rx) & wave_ballot(t_lo <= rx);
        const int32_t left = lr.x, right = lr.y;
        if (COUNT) {
            ++c_node;
            c_lchild += __popcll(bl) + __popcll(br);
        }
        // nonzero iff both children are entered (one scalar compare for the branch)
        const uint32_t both = min(uint32_t(__popcll(bl)), uint32_t(__popcll(br)));
        int32_t next;
        if (both != 0) {
            // both entered: the child the leader lane (lowest live lane) reaches first (REV: leaves
            // last) goes first
            const bool lfirst = (wave_ballot(REV ? lf >= rf : ln <= rn) & lead_bit) != 0;
            if (sp >= stack_depth) {
                overflow = true;
                next = kDone;
            } else {
                stackv = (lane == sp) ? (lfirst ? right : left) : stackv;
                ++sp;
                next = lfirst ? left : right;
            }
        } else if ((bl | br) != 0) {
            next = bl != 0 ? left : right;
        } else if (sp == 0) {
            next = kDone;
        } else {
            --sp;
            next = __builtin_amdgcn_readlane(stackv, sp);
        }
        node = next;
    }
    return node;
}

// The wave-uniform walk of the whole BVH for one round: descend to a leaf, test it
// (leaf(j), which may move t_lo / t_hi_w), resume from the stack. The walk is specialised on the
// wave's direction octant as a whole, so the octant is dispatched once per walk.
#define RS_WALK_OCT(O)                                                                                        \
    {                                                                                                         \
        int32_t node = P.root;                                                                                \
        int32_t sp = 0;                                                                                       \
        int32_t stackv = 0;                                                                                   \
        const uint64_t live_mask = wave_ballot(live);                                                         \
        const uint64_t lead_bit = live_mask & (~live_mask + 1);                                               \
        for (;;) {                                                                                            \
            node = descend<O, COUNT, kRev>(node, nodes, sl, lead_bit, t_lo, t_hi_w, lane, P.stack_depth, sp,  \
                                           stackv, overflow, c_node, c_lchild);                               \
            if (node == kDone) break;                                                                         \
            leaf(~node);                                                                                      \
            if (sp == 0) break;                                                                               \
            --sp;                                                                                             \
            node = __builtin_amdgcn_readlane(stackv, sp);                                                     \
        }                                                                                                     \
    }

#define RS_WALK_BVH()                                                                                         \
    switch (oct) {                                                                                            \
    case 0: RS_WALK_OCT(0) break;                                                                             \
    case 1: RS_WALK_OCT(1) break;                                                                             \
    case 2: RS_WALK_OCT(2) break;                                                                             \
    case 3: RS_WALK_OCT(3) break;                                                                             \
    case 4: RS_WALK_OCT(4) break;                                                                             \
    case 5: RS_WALK_OCT(5) break;                                                                             \
    case 6: RS_WALK_OCT(6) break;                                                                             \
    case 7: RS_WALK_OCT(7) break;                                                                             \
    default: RS_WALK_OCT(kMixedOctant) break;                                                                 \
    }

// Occupancy target (waves per SIMD) of each variant, i.e. its VGPR budget
// (512 / waves): the adjoint carries the gradient temporaries as well. The
// forward targets are measured optima: a few dozen bytes of scratch spills
// (kbuf 24 at five waves, 48 at four with its LDS tail) cost less than the
// node-fetch latency the extra wave hides, while larger spills (kbuf 24 at six,
// 32 at five) lose.
// The adjoint's are measured the same way: kbuf 24 and 32 at four waves and
// 48 at three beat one wave fewer by 10-20 %, while one wave more (five, and
// four for 48) spills heavily and doubles the time.
#ifndef RS_FWD16_WAVES
#define RS_FWD16_WAVES 5
#endif
#ifndef RS_BWD16_WAVES
#define RS_BWD16_WAVES 4
#endif
#ifndef RS_FWD24_WAVES
#define RS_FWD24_WAVES 5
#endif
#ifndef RS_BWD24_WAVES
#define RS_BWD24_WAVES 4
#endif
#ifndef RS_BWD32_WAVES
#define RS_BWD32_WAVES 4
#endif
#ifndef RS_BWD48_WAVES
#define RS_BWD48_WAVES 3
#endif
#ifndef RS_FWD32_WAVES
#define RS_FWD32_WAVES 4
#endif
#ifndef RS_FWD48_WAVES
#define RS_FWD48_WAVES 4
#endif
constexpr int waves_for(int K, bool bwd)
{
    return bwd ? (K <= 8 ? 4 : (K <= 16 ? RS_BWD16_WAVES : (K <= 24 ? RS_BWD24_WAVES : (K <= 32 ? RS_BWD32_WAVES : RS_BWD48_WAVES))))
               : (K <= 8 ? 6 : (K <= 16 ? RS_FWD16_WAVES : (K <= 24 ? RS_FWD24_WAVES : (K <= 32 ? RS_FWD32_WAVES : RS_FWD48_WAVES))));
}

// ------------------------------------------------------------ forward render

template <int K, bool BRUTE, bool COUNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_for(K, false)))) void k_render(
    const float4 *__restrict__ records, const float4 *__restrict__ nodes, const int32_t *__restrict__ gidx,
    const int32_t *__restrict__ inv, const Ptrs ptr, const RenderParams P)
{
    constexpr bool kRev = false;
    const int lane = threadIdx.x;
    int64_t iter_pkt = 0;
    const int xcd = xcd_id();
    int qi = 0;
    // work counters (wave-uniform, scalar registers; only in the COUNT variants)
    uint64_t c_pkt = 0, c_node = 0, c_leaf = 0, c_round = 0, c_lleaf = 0, c_lbuf = 0, c_lcomp = 0, c_lchild = 0,
             c_rows = 0, c_slots = 0;
    for (;;) {
        const int64_t pkt = next_packet(P, ptr.queue, lane, xcd, qi, iter_pkt);
        if (pkt >= P.n_packets) break;
        if (COUNT) ++c_pkt;

        const LaneRay LR = lane_ray(P, ptr, pkt, lane);
        const RaySet &S = ptr.set[LR.si];
        const bool zc = S.zero_colour != 0;
        const bool valid = LR.valid;
        const int64_t ray_id = LR.id;
        const Ray ray = LR.ray;
        const float tmax = LR.tmax, bgr = LR.bgr, bgg = LR.bgg, bgb = LR.bgb;
        const Slab sl = make_slab(ray);
        const int oct = wave_octant(sl, valid);

        Accum A{1.0f, 0.0f, 0.0f, 0.0f, 0};
        bool live = valid && P.n_gauss > 0 && tmax > P.t_min;
        double last = -kNoHit;  // the last consumed key; keys of the next round must exceed it
        // T just before the composited hit that took T below the normal floats (to 0, or into the
        // subnormals, where T_{k+1} / (1 - alpha_k) would lose its digits), and that hit's index
        float Tz = 0.0f;
        int32_t z = -1;
        // stored hit lists: the packet's row cursor; per lane the composited ids stored
        const bool lists = P.lists && S.list != nullptr;
        ListCursor LC{0, -1, 0, 0, true};
        int32_t stored = 0;
        // RS_PAPER_GRADIENT forward: after an eps1 stop the lane keeps consuming hits without
        // compositing them, recording their ids while T2 (their transmittance) stays >= eps2
        const bool paper = P.paper && lists;
        bool phase2 = false;
        float T2 = 1.0f;
        int32_t extra = 0;
        bool overflow = false;

        while (wave_ballot(live)) {
            typename FwdBuf<K>::type hb;
            if constexpr (!std::is_same<typename FwdBuf<K>::type, HitBuf<K>>::value) {
                __shared__ double ring[kTailKeys * kWave];
                hb.ring = ring;
                hb.lane = lane;
            }
            hb.clear();
            if (COUNT) ++c_round;
            // NaN on lanes that are not live: no box test passes for them
            const float t_lo =
                !live ? __builtin_nanf("") : (last == -kNoHit ? P.t_min : fmaxf(P.t_min, hit_key_t(last)));
            float t_hi_w = widen(tmax, sl.pad);

            // the round's live lanes as a mask: the leaf step combines per-compare masks with it
            // (a ballot of a compound condition would first turn it into a vector value)
            const uint64_t live_now = wave_ballot(live);
            auto leaf = [&](int64_t j) {
                const int64_t js = __builtin_amdgcn_readfirstlane(int32_t(j));
                const float4 r0 = records[4 * js + 0], r1 = records[4 * js + 1], r2 = records[4 * js + 2],
                             r3 = records[4 * js + 3];
                const uint32_t gid = uint32_t(gidx[js]);
                // every lane evaluates the test and the key (no divergent branch); only lanes
                // whose ray hits take part, and the entry distance and key only when one does
                HitGeom hg;
                const float h2 = ellipsoid_h2(ray, r0, r1, r2, r3, hg);
                // the index load is issued with the record's (its latency hides behind theirs)
                asm volatile("" ::"s"(gid));
                if (COUNT) {
                    ++c_leaf;
                    c_lleaf += __popcll(live_now);
                }
                const uint64_t hmask = wave_ballot(h2 <= P.Q) & live_now;
                if (!hmask) return;
                const float t1 = ellipsoid_t1(hg, r2, h2, P.Q);
                const double k = hit_key(t1, gid);
                const uint64_t cmask = hmask & wave_ballot(t1 >= P.t_min) & wave_ballot(t1 < tmax) &
                                       wave_ballot(k > last) & wave_ballot(k < hb.last());
                const bool cand = __builtin_amdgcn_inverse_ballot_w64(cmask);
                if (COUNT) c_lbuf += __popcll(cmask);
                if (cmask) {
                    // every lane runs the insertion network; lanes without a candidate insert
                    // the empty key, which moves nothing
                    hb.insert(cand ? k : kNoHit);
                    if (hb.last() != kNoHit) t_hi_w = widen(fminf(tmax, hit_key_t(hb.last())), sl.pad);
                }
            };

            if (BRUTE) {
                for (int64_t j = 0; j < P.n_gauss; ++j) leaf(j);
            } else {
                // While-while traversal: descend internal nodes until a leaf is reached (or the
                // stack runs dry), then test that leaf; the hit buffer changes only in the leaf step.
                // The walk is specialised on the wave's direction octant.
                RS_WALK_BVH()
            }
            if (overflow) {
                if (lane == 0) atomicOr(ptr.status, kStatusStack);
                live = false;
                break;
            }

            // composite this round's hits front to back; alpha is recomputed from the record
            // with the leaf test's own arithmetic. The buffer is consumed from its front.
            const double round_last = hb.last();
            bool more = true;
            // the sorted position of the buffer's front key is looked up one step ahead, so its
            // latency overlaps the previous step (an empty key reads position 0, unused)
            int32_t js_next = inv[hb.front() != kNoHit ? hit_key_gid(hb.front()) : 0u];
            for (int s = 0; s < hb.size; ++s) {
                const double key_s = hb.front();
                const int32_t js_s = js_next;
                hb.pop_front();
                js_next = inv[hb.front() != kNoHit ? hit_key_gid(hb.front()) : 0u];
                const bool act = more && live && key_s != kNoHit;
                const uint64_t act_mask = wave_ballot(act);
                more = act_mask != 0;
                if (!more) break;
                if (COUNT) c_lcomp += __popcll(act_mask);
                const uint32_t gid = hit_key_gid(key_s);
                uint32_t entry = kListIdle;
                if (paper && phase2) {
                    if (act) {
                        if (T2 < P.eps2 || A.n + extra >= P.max_hits) {
                            live = false;  // the second phase ends before this hit
                        } else {
                            float4 r0, r1, r2, r3;
                            float t1, h2;
                            HitGeom hg;
                            const float al = hit_alpha_at(js_s, ray, records, P.Q, r0, r1, r2, r3, t1, h2, hg);
                            entry = gid | kListSecond;
                            T2 *= 1.0f - al;
                            ++extra;
                            last = key_s;
                        }
                    }
                } else {
                    HitData H;
                    composite_hit(act, gid, js_s, ray, records, ptr.rgb, zc, P, A, H);
                    if (act) {
                        entry = gid;
                        last = key_s;
                        if (A.T < kMinNormal && H.Tk >= kMinNormal) {
                            Tz = H.Tk;
                            z = A.n - 1;
                        }
                    }
                    const bool stopped = act && stop_after(A, P);
                    if (stopped) {
                        if (paper && A.T < P.eps1)
                            phase2 = true;  // stays live for the second phase
                        else
                            live = false;
                    }
                }
                if (lists) list_append(ptr.pool, LC, entry, lane, stored, paper, ptr.status);
            }
            // a lane whose buffer did not fill has consumed all its hits
            if (live && round_last == kNoHit) live = false;
        }

        if (lists) {
            list_close(ptr.pool, LC, lane);
            if (COUNT) {
                c_rows += uint64_t(LC.rows);
                c_slots += uint64_t(LC.slots);
            }
        }
        if (valid) {
            const float orr = __builtin_fmaf(A.T, bgr, A.Cr), og = __builtin_fmaf(A.T, bgg, A.Cg),
                        ob = __builtin_fmaf(A.T, bgb, A.Cb);
            S.out_rgb[3 * ray_id] = orr;
            S.out_rgb[3 * ray_id + 1] = og;
            S.out_rgb[3 * ray_id + 2] = ob;
            if (S.fin) {
                S.fin[ray_id] = make_float4(orr, og, ob, A.T);
                const uint64_t kb = A.n > 0 ? uint64_t(__double_as_longlong(last)) : 0ull;
                S.last[ray_id] = make_uint4(uint32_t(kb), uint32_t(kb >> 32), __float_as_uint(Tz),
                                            z >= 0 ? uint32_t(A.n - 1 - z) : 0xffffffffu);
            }
            if (lists) S.list[ray_id] = make_int4(A.n, stored, LC.chunk, LC.rows);
        }
    }
    if (COUNT && lane == 0 && c_pkt > 0) {
        atomicAdd(ptr.counters + 0, (unsigned long long)c_pkt);
        atomicAdd(ptr.counters + 1, (unsigned long long)c_node);
        atomicAdd(ptr.counters + 2, (unsigned long long)c_leaf);
        atomicAdd(ptr.counters + 3, (unsigned long long)c_round);
        atomicAdd(ptr.counters + 4, (unsigned long long)c_lleaf);
        atomicAdd(ptr.counters + 5, (unsigned long long)c_lbuf);
        atomicAdd(ptr.counters + 6, (unsigned long long)c_lcomp);
        atomicAdd(ptr.counters + 7, (unsigned long long)c_lchild);
        atomicAdd(ptr.counters + 12, (unsigned long long)c_rows);
        atomicAdd(ptr.counters + 14, (unsigned long long)c_slots);
    }
}

// ------------------------------------------------- adjoint by re-traversal

// The adjoint re-traverses each ray back to front: a round collects the K largest
// keys below the previous round's smallest (the first round: up to and including the
// last composited key the forward saved), keeping them in the hit buffer as negated
// keys so the same min/max network serves; nodes are culled against [K-th largest t,
// upper t] and the leader lane takes the child it leaves last first. The round's hits
// are then processed largest key first. Next to stored lists it serves the rays whose
// list is incomplete (the pool ran out).
template <int K, bool BRUTE, bool COUNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_for(K, true)))) void k_adjoint_trav(
    const float4 *__restrict__ records, const float4 *__restrict__ nodes, const int32_t *__restrict__ gidx,
    const int32_t *__restrict__ inv, const Ptrs ptr, const RenderParams P)
{
    constexpr bool kRev = true;
    if (P.overflow_only && ptr.pool.hdr[1] == 0ull) return;  // every list is complete
    const int lane = threadIdx.x;
    int64_t iter_pkt = 0;
    const int xcd = xcd_id();
    int qi = 0;
    uint64_t c_pkt = 0, c_node = 0, c_leaf = 0, c_round = 0, c_lleaf = 0, c_lbuf = 0, c_lcomp = 0, c_lchild = 0,
             c_group = 0;
    acc_clear(acc_table(), lane);
    for (;;) {
        const int64_t pkt = next_packet(P, ptr.queue, lane, xcd, qi, iter_pkt);
        if (pkt >= P.n_packets) break;
        if (COUNT) ++c_pkt;

        const LaneRay LR = lane_ray(P, ptr, pkt, lane);
        const RaySet &S = ptr.set[LR.si];
        const bool zc = S.zero_colour != 0;
        const bool valid = LR.valid;
        const int64_t ray_id = LR.id;
        const Ray ray = LR.ray;
        const float tmax = LR.tmax;
        const Slab sl = make_slab(ray);
        const int oct = wave_octant(sl, valid);

        LaneGrad Gd{0.0f, 0.0f, 0.0f};
        Back B{1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0, -1};
        bool live = false;
        double hi = 0.0;  // keys of a round lie below it
        if (valid) {
            Gd.gr = S.grad[3 * ray_id];
            Gd.gg = S.grad[3 * ray_id + 1];
            Gd.gb = S.grad[3 * ray_id + 2];
            const uint4 ls = S.last[ray_id];
            B = back_init(S.fin[ray_id], ls, LR.bgr, LR.bgg, LR.bgb);
            live = ls.y != 0u && P.n_gauss > 0 && !(Gd.gr == 0.0f && Gd.gg == 0.0f && Gd.gb == 0.0f);
            if (P.overflow_only) {
                const int4 li = S.list[ray_id];
                live = live && li.y < li.x;
            }
            // the successor of the last composited key (next Gaussian index, same t)
            hi = __longlong_as_double((long long)(((uint64_t(ls.y) << 32) | ls.x) + 1ull));
        }
        bool overflow = false;

        while (wave_ballot(live)) {
            HitBuf<K> hb;  // negated keys, ascending: the largest key first
            hb.clear();
            if (COUNT) ++c_round;
            float t_lo = !live ? __builtin_nanf("") : P.t_min;  // rises to the K-th largest t
            const float t_hi_w = widen(hit_key_t(hi), sl.pad);

            const uint64_t live_now = wave_ballot(live);  // as in the forward's leaf step
            auto leaf = [&](int64_t j) {
                const int64_t js = __builtin_amdgcn_readfirstlane(int32_t(j));
                const float4 r0 = records[4 * js + 0], r1 = records[4 * js + 1], r2 = records[4 * js + 2],
                             r3 = records[4 * js + 3];
                const uint32_t gid = uint32_t(gidx[js]);
                HitGeom hg;
                const float h2 = ellipsoid_h2(ray, r0, r1, r2, r3, hg);
                // the index load is issued with the record's (its latency hides behind theirs)
                asm volatile("" ::"s"(gid));
                if (COUNT) {
                    ++c_leaf;
                    c_lleaf += __popcll(live_now);
                }
                const uint64_t hmask = wave_ballot(h2 <= P.Q) & live_now;
                if (!hmask) return;
                const float t1 = ellipsoid_t1(hg, r2, h2, P.Q);
                const double k = hit_key(t1, gid);
                const uint64_t cmask = hmask & wave_ballot(t1 >= P.t_min) & wave_ballot(t1 < tmax) & wave_ballot(k < hi) &
                                       wave_ballot(-k < hb.key[K - 1]);
                const bool cand = __builtin_amdgcn_inverse_ballot_w64(cmask);
                if (COUNT) c_lbuf += __popcll(cmask);
                if (cmask) {
                    hb.insert(cand ? -k : kNoHit);
                    if (hb.key[K - 1] != kNoHit) t_lo = fmaxf(P.t_min, hit_key_t(-hb.key[K - 1]));
                }
            };

            if (BRUTE) {
                for (int64_t j = 0; j < P.n_gauss; ++j) leaf(j);
            } else {
                RS_WALK_BVH()
            }
            if (overflow) {
                if (lane == 0) atomicOr(ptr.status, kStatusStack);
                live = false;
                break;
            }

            const double round_first = hb.key[K - 1];  // minus the round's smallest key (kNoHit: not full)
            bool more = true;
            for (int s = 0; s < K; ++s) {
                const double nk = hb.key[0];
                hb.pop_front();
                const bool act = more && live && nk != kNoHit;
                const uint64_t act_mask = wave_ballot(act);
                more = act_mask != 0;
                if (!more) break;
                if (COUNT) c_lcomp += __popcll(act_mask);
                const uint32_t gid = hit_key_gid(nk);
                HitData H;
                recompute_hit(act, gid, ray, records, inv, ptr.rgb, zc, P.Q, H);
                const float Tk = back_T(B, H.al);
                adjoint_hit<COUNT, true>(act, act_mask, gid, H, Tk, B, Gd, zc, ptr.gacc, lane, c_group);
                if (act) {
                    back_over(B, H.al, H.cr, H.cg, H.cb);
                    B.T = Tk;
                    ++B.done;
                }
            }
            // a lane whose buffer did not fill has reached its first hit
            if (live) {
                if (round_first == kNoHit)
                    live = false;
                else
                    hi = -round_first;
            }
        }
    }
    acc_flush<COUNT>(acc_table(), ptr.gacc, lane, c_group);
    if (COUNT && lane == 0 && c_pkt > 0) {
        atomicAdd(ptr.counters + 1, (unsigned long long)c_node);
        atomicAdd(ptr.counters + 2, (unsigned long long)c_leaf);
        atomicAdd(ptr.counters + 3, (unsigned long long)c_round);
        atomicAdd(ptr.counters + 4, (unsigned long long)c_lleaf);
        atomicAdd(ptr.counters + 5, (unsigned long long)c_lbuf);
        atomicAdd(ptr.counters + 6, (unsigned long long)c_lcomp);
        atomicAdd(ptr.counters + 7, (unsigned long long)c_lchild);
        atomicAdd(ptr.counters + 8, (unsigned long long)c_group);
        atomicAdd(ptr.counters + 13, (unsigned long long)c_pkt);
    }
}

// ------------------------------------------------- adjoint from stored lists

// The forward appended one row per compositing step of each packet; the adjoint
// walks the packet's rows from the last to the first, so every lane meets its
// own hits back to front (rows where it was idle hold kListIdle), and recomputes
// each hit with the forward's own per-hit arithmetic: no traversal and no hit
// buffer. The paper variant's second-phase hits (flagged, after the composited
// ones) only build the colour behind the last composited hit. Rays whose list is
// incomplete are left to the traversal adjoint.
// Six waves per SIMD hide the gathers better than five; seven and eight spill.
#ifndef RS_LIST_WAVES
#define RS_LIST_WAVES 6
#endif
// Row cursor of the list adjoint (wave-uniform): `start` is where the row read last began,
// so the next row (back to front) ends there, or at the fill of an earlier chunk.
__device__ inline void row_seek(const int32_t *__restrict__ prev, const int32_t *__restrict__ fill, int32_t &chunk,
                                int32_t &start)
{
    // wave-uniform addresses, read through the constant address space (scalar loads)
    typedef const __attribute__((address_space(4))) int32_t *const_i32;
    while (start == 0 && chunk >= 0) {
        chunk = ((const_i32)prev)[chunk];
        start = chunk >= 0 ? ((const_i32)fill)[chunk] : 0;
    }
}

// Reads the row ending at `start` of `chunk` (its lane mask), moves `start` to the row's first
// slot, and returns this lane's entry (kListIdle for a lane without one, or not live).
__device__ inline uint32_t row_entry(const uint32_t *__restrict__ slots, int32_t chunk, int32_t &start, bool live,
                                     int lane)
{
    const uint32_t *row_end = slots + int64_t(chunk) * kChunkSlots + start;
    // the mask's address is wave-uniform: read it through the constant address space, so it is
    // a scalar load (the pool is only read by this kernel)
    typedef const __attribute__((address_space(4))) uint32_t *const_u32;
    const const_u32 mend = (const_u32)(row_end - 2);
    const uint64_t m = uint64_t(mend[0]) | (uint64_t(mend[1]) << 32);
    const int32_t k = __popcll(m);
    start -= k + 2;
    const bool mine = ((m >> lane) & 1ull) != 0;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    const uint32_t *row = row_end - 2 - k;
    return live && mine ? row[below] : kListIdle;
}

template <bool COUNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RS_LIST_WAVES))) void k_adjoint_list(
    const float4 *__restrict__ records, const int32_t *__restrict__ inv, const Ptrs ptr, const RenderParams P)
{
    const int lane = threadIdx.x;
    int64_t iter_pkt = 0;
    const int xcd = xcd_id();
    int qi = 0;
    uint64_t c_pkt = 0, c_lcomp = 0, c_group = 0;
    // the pool is only read here
    const uint32_t *__restrict__ slots = ptr.pool.slots;
    const int32_t *__restrict__ prev = ptr.pool.prev;
    const int32_t *__restrict__ fill = ptr.pool.fill;
    for (;;) {
        const int64_t pkt = next_packet(P, ptr.queue, lane, xcd, qi, iter_pkt);
        if (pkt >= P.n_packets) break;
        if (COUNT) ++c_pkt;
        const LaneRay LR = lane_ray(P, ptr, pkt, lane);
        const RaySet &S = ptr.set[LR.si];
        const bool zc = S.zero_colour != 0;
        LaneGrad Gd{0.0f, 0.0f, 0.0f};
        Back B{1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0, -1};
        int4 li = make_int4(0, 0, -1, 0);
        bool live = false;
        if (LR.valid) {
            li = S.list[LR.id];
            Gd.gr = S.grad[3 * LR.id];
            Gd.gg = S.grad[3 * LR.id + 1];
            Gd.gb = S.grad[3 * LR.id + 2];
            B = back_init(S.fin[LR.id], S.last[LR.id], LR.bgr, LR.bgg, LR.bgb);
            live = li.x > 0 && li.y == li.x && P.n_gauss > 0 && !(Gd.gr == 0.0f && Gd.gg == 0.0f && Gd.gb == 0.0f);
        }
        // the packet's last chunk (lane 0 always holds one of the packet's rays)
        int32_t chunk = __builtin_amdgcn_readfirstlane(li.z);
        if (!wave_ballot(live) || chunk < 0) continue;
        // Rows are walked from the last to the first: a row ends with its lane mask, so the
        // mask at the row's end gives its start, which is the previous row's end. The next
        // row's mask and this lane's entry in it are loaded while a row is processed.
        int32_t start = fill[chunk];
        row_seek(prev, fill, chunk, start);
        uint32_t e = kListIdle;
        if (chunk >= 0) e = row_entry(slots, chunk, start, live, lane);
        while (chunk >= 0) {
            int32_t nchunk = chunk, nstart = start;
            row_seek(prev, fill, nchunk, nstart);
            uint32_t ne = kListIdle;
            if (nchunk >= 0) ne = row_entry(slots, nchunk, nstart, live, lane);
            chunk = nchunk;
            start = nstart;
            const uint32_t cur = e;
            e = ne;
            const bool act = cur != kListIdle;
            if (!wave_ballot(act)) continue;
            const bool comp = act && cur < kListSecond;
            const uint32_t gid = act ? cur & ~kListSecond : 0u;  // idle lanes read Gaussian 0 (unused)
            HitData H;
            recompute_hit<true>(act, gid, LR.ray, records, inv, ptr.rgb, zc, P.Q, H);
            const float Tk = back_T(B, H.al);
            const uint64_t comp_mask = wave_ballot(comp);
            if (COUNT) c_lcomp += __popcll(comp_mask);
            if (comp_mask)
                adjoint_hit<COUNT, false>(comp, comp_mask, gid, H, Tk, B, Gd, zc, ptr.gacc, lane, c_group);
            if (act) back_over(B, H.al, H.cr, H.cg, H.cb);
            if (comp) {
                B.T = Tk;
                ++B.done;
            }
        }
    }
    if (COUNT && lane == 0 && c_pkt > 0) {
        atomicAdd(ptr.counters + 9, (unsigned long long)c_pkt);
        atomicAdd(ptr.counters + 10, (unsigned long long)c_lcomp);
        atomicAdd(ptr.counters + 11, (unsigned long long)c_group);
    }
}

// ------------------------------------------------------------------- host

__global__ void k_zero_f32(float *p, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

// Accumulator (16 floats per Gaussian: body-frame mean 3, scale 3, angular 3,
// opacity 1, rgb 3, 3 unused) -> the caller's gradient arrays: dL/dm = -2 R acc_m
// and dL/dq = (2/|q|) E(q/|q|)^T acc_w (see grad_hit), with R^T from the
// Gaussian's record (the rotation the renders used).
__global__ __launch_bounds__(256) void k_scatter_grads(const float4 *__restrict__ gacc, const float4 *__restrict__ records,
                                                       const int32_t *__restrict__ inv, const float *__restrict__ quat,
                                                       int64_t n, float *d_mean, float *d_scale, float *d_quat,
                                                       float *d_opacity, float *d_rgb)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 a = gacc[4 * i], b = gacc[4 * i + 1], c = gacc[4 * i + 2], d = gacc[4 * i + 3];
    const float am0 = a.x, am1 = a.y, am2 = a.z, w0 = b.z, w1 = b.w, w2 = c.x;
    if (d_mean) {
        // R = (R^T)^T: dm_k = -2 sum_j RT_jk am_j
        const int32_t js = inv[i];
        const float4 r0 = records[4 * js], r1 = records[4 * js + 1], r2 = records[4 * js + 2];
        const float t00 = r0.x, t01 = r0.y, t02 = r0.z, t10 = r0.w, t11 = r1.x, t12 = r1.y, t20 = r1.z, t21 = r1.w,
                    t22 = r2.x;
        d_mean[3 * i] = -2.0f * (t00 * am0 + t10 * am1 + t20 * am2);
        d_mean[3 * i + 1] = -2.0f * (t01 * am0 + t11 * am1 + t21 * am2);
        d_mean[3 * i + 2] = -2.0f * (t02 * am0 + t12 * am1 + t22 * am2);
    }
    if (d_scale) {
        d_scale[3 * i] = a.w;
        d_scale[3 * i + 1] = b.x;
        d_scale[3 * i + 2] = b.y;
    }
    if (d_quat) {
        const float4 q = reinterpret_cast<const float4 *>(quat)[i];
        const float nq = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
        const float in = 1.0f / nq, k = 2.0f * in;
        const float qw = q.x * in, vx = q.y * in, vy = q.z * in, vz = q.w * in;
        reinterpret_cast<float4 *>(d_quat)[i] =
            make_float4(-k * (vx * w0 + vy * w1 + vz * w2), k * (qw * w0 + (vy * w2 - vz * w1)),
                        k * (qw * w1 + (vz * w0 - vx * w2)), k * (qw * w2 + (vx * w1 - vy * w0)));
    }
    if (d_opacity) d_opacity[i] = c.y;
    if (d_rgb) {
        d_rgb[3 * i] = c.z;
        d_rgb[3 * i + 1] = c.w;
        d_rgb[3 * i + 2] = d.x;
    }
}

__global__ void k_zero_queue(uint32_t *q)
{
    if (threadIdx.x < kXcdQueues) q[threadIdx.x] = 0u;
}

__global__ void k_zero_pool_header(unsigned long long *h)
{
    if (threadIdx.x < 2) h[threadIdx.x] = 0ull;
}

void reset_pool(const ListPool &pool, hipStream_t st)
{
    if (pool.hdr) k_zero_pool_header<<<1, 64, 0, st>>>(pool.hdr);
}

static void zero(float *p, int64_t n, hipStream_t st)
{
    if (!p || n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_zero_f32<<<int(blocks), 256, 0, st>>>(p, n);
}

struct KernArgs {
    int grid;
    const float4 *records, *nodes;
    const int32_t *gidx, *inv;
};

template <int K>
static void launch_k(Pass pass, const KernArgs &a, const Ptrs &ptr, const RenderParams &P, hipStream_t st)
{
    if (pass == Pass::Forward) {
        if (P.brute)
            k_render<K, true, false><<<a.grid, kWave, 0, st>>>(a.records, a.nodes, a.gidx, a.inv, ptr, P);
        else if (P.count)
            k_render<K, false, true><<<a.grid, kWave, 0, st>>>(a.records, a.nodes, a.gidx, a.inv, ptr, P);
        else
            k_render<K, false, false><<<a.grid, kWave, 0, st>>>(a.records, a.nodes, a.gidx, a.inv, ptr, P);
    } else {
        if (P.brute)
            k_adjoint_trav<K, true, false><<<a.grid, kWave, 0, st>>>(a.records, a.nodes, a.gidx, a.inv, ptr, P);
        else if (P.count)
            k_adjoint_trav<K, false, true><<<a.grid, kWave, 0, st>>>(a.records, a.nodes, a.gidx, a.inv, ptr, P);
        else
            k_adjoint_trav<K, false, false><<<a.grid, kWave, 0, st>>>(a.records, a.nodes, a.gidx, a.inv, ptr, P);
    }
}

void zero_gacc(const BvhDesc &D, hipStream_t st)
{
    Layout L = make_layout(D.n);
    zero(reinterpret_cast<float *>(D.ws + L.gacc), 16 * D.n, st);
}

void scatter_gacc(const BvhDesc &D, const float *quat, const rs_grads *grads, hipStream_t st)
{
    if (D.n <= 0) return;
    Layout L = make_layout(D.n);
    k_scatter_grads<<<int((D.n + 255) / 256), 256, 0, st>>>(
        reinterpret_cast<const float4 *>(D.ws + L.gacc), reinterpret_cast<const float4 *>(D.ws + L.records),
        reinterpret_cast<const int32_t *>(D.ws + L.inv), quat, D.n, grads->d_mean, grads->d_scale, grads->d_quat,
        grads->d_opacity, grads->d_rgb);
}

// One launch over up to kMaxSets ray sets sharing a layout (same count, same views).
int launch_sets(const BvhDesc &D, const rs_gaussians *g, const rs_params *p, int nsets, const SetDesc *sets,
                const ListPool &pool, Pass pass, hipStream_t st)
{
    Layout L = make_layout(D.n);
    char *ws = D.ws;
    WsHeader *h = reinterpret_cast<WsHeader *>(ws + L.header);
    const rs_rays *rays = sets[0].rays;

    RenderParams P{};
    P.n_rays = rays->n;
    P.n_gauss = D.n;
    P.root = D.root;
    P.stack_depth = p->stack_depth > 0 ? p->stack_depth : 64;
    P.Q = p->Q;
    P.eps1 = p->eps1;
    P.t_min = p->t_min;
    P.max_hits = p->max_hits;
    P.flags = p->flags;
    P.persistent = (p->flags & RS_PERSISTENT) ? 1 : 0;
    P.brute = (p->flags & RS_BRUTE_FORCE) ? 1 : 0;
    P.count = (p->flags & RS_COUNTERS) ? 1 : 0;
    const int64_t packets = plan_packets(P, rays, tile_shift_of(p));
    P.packets_per_set = packets;
    P.n_packets = packets * nsets;
    P.strip_tiles = kStripTiles;
    P.lists = pool.chunks > 0 ? 1 : 0;
    P.overflow_only = (pass == Pass::AdjointTraverse && P.lists) ? 1 : 0;
    P.paper = (p->flags & RS_PAPER_GRADIENT) && P.lists ? 1 : 0;
    P.eps2 = p->eps2;
    P.chunk = (P.n_packets + kXcdQueues - 1) / kXcdQueues;

    Ptrs ptr{};
    ptr.rgb = g->rgb;
    for (int k = 0; k < kMaxSets; ++k) {
        const SetDesc &E = sets[k < nsets ? k : 0];
        RaySet &R = ptr.set[k];
        R.origin = E.rays->origin;
        R.dir = E.rays->dir;
        R.tmax = E.rays->t_max;
        R.bgray = E.rays->bg;
        R.grad = E.grad;
        R.out_rgb = E.out_rgb;
        R.fin = E.state.fin;
        R.last = E.state.last;
        R.list = E.state.list;
        for (int c = 0; c < 3; ++c) R.bg[c] = E.bg[c];
        R.zero_colour = E.zero_colour;
    }
    ptr.status = &h->status;
    ptr.queue = h->xq;
    ptr.counters = reinterpret_cast<unsigned long long *>(h->counters);
    ptr.gacc = reinterpret_cast<float *>(ws + L.gacc);
    ptr.pool = pool;

    if (pass == Pass::Forward && P.lists) reset_pool(pool, st);
    if (P.n_packets > 0) {
        KernArgs a;
        if (P.persistent) {
            k_zero_queue<<<1, 64, 0, st>>>(h->xq);
            int dev = 0, cus = 256;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            const int64_t waves = int64_t(cus) * 24;  // up to 6 waves per SIMD (the most any variant fits)
            a.grid = int(waves < P.n_packets ? waves : P.n_packets);
        } else {
            const int64_t deal = int64_t(kXcdQueues) * kXcdRun;
            a.grid = int((P.n_packets + deal - 1) / deal * deal);
        }
        a.records = reinterpret_cast<const float4 *>(ws + L.records);
        a.nodes = reinterpret_cast<const float4 *>(ws + L.nodes);
        a.gidx = reinterpret_cast<const int32_t *>(ws + L.gidx);
        a.inv = reinterpret_cast<const int32_t *>(ws + L.inv);
        // the hit-buffer size never changes the result (same hits, same order, same arithmetic);
        // the default is the fastest measured size on MI355X
        if (pass == Pass::AdjointList) {
            if (P.count)
                k_adjoint_list<true><<<a.grid, kWave, 0, st>>>(a.records, a.inv, ptr, P);
            else
                k_adjoint_list<false><<<a.grid, kWave, 0, st>>>(a.records, a.inv, ptr, P);
        } else {
            const int K = p->kbuf > 0 ? p->kbuf : 48;
            switch (K) {
            case 8: launch_k<8>(pass, a, ptr, P, st); break;
            case 16: launch_k<16>(pass, a, ptr, P, st); break;
            case 24: launch_k<24>(pass, a, ptr, P, st); break;
            case 32: launch_k<32>(pass, a, ptr, P, st); break;
            case 48: launch_k<48>(pass, a, ptr, P, st); break;
            default: return RS_ERR_INVALID_ARG;
            }
        }
    }
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

int launch_render(const BvhDesc &D, const rs_gaussians *g, const rs_rays *rays, const rs_params *p,
                  float *out_rgb, void *state, const float *grad, const rs_grads *grads, hipStream_t st)
{
    const bool bwd = grad != nullptr;
    SetDesc S{};
    S.rays = rays;
    S.out_rgb = out_rgb;
    S.grad = grad;
    for (int c = 0; c < 3; ++c) S.bg[c] = p->bg[c];
    S.zero_colour = (p->flags & RS_ZERO_COLOUR) ? 1 : 0;
    const int32_t cap = p->hit_list;
    S.state = state_at(state, rays->n, cap);
    ListPool pool{nullptr, nullptr, nullptr, 0};
    if (state && cap > 0 && rays->n > 0) {
        const StateLayout sl = state_layout(rays->n, cap);
        pool = list_pool_at(static_cast<char *>(state) + sl.pool, sl.chunks);
    }
    if (!bwd) return launch_sets(D, g, p, 1, &S, pool, Pass::Forward, st);
    int e;
    zero_gacc(D, st);
    if (pool.chunks > 0) {
        // stored lists first; the traversal adjoint then takes the rays whose list is
        // incomplete (it exits at once when the forward found the pool large enough).
        // The paper variant has no traversal form: its pool running out is an error.
        if ((e = launch_sets(D, g, p, 1, &S, pool, Pass::AdjointList, st))) return e;
        if (!(p->flags & RS_PAPER_GRADIENT))
            if ((e = launch_sets(D, g, p, 1, &S, pool, Pass::AdjointTraverse, st))) return e;
    } else {
        if ((e = launch_sets(D, g, p, 1, &S, pool, Pass::AdjointTraverse, st))) return e;
    }
    scatter_gacc(D, g->quat, grads, st);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

}  // namespace rs
