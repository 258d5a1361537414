// Triangle mesh + Gaussians: triangle BVH traversal (closest or any hit,
// Moller-Trumbore), spawning of the path and shadow rays of every level, and
// the forward / adjoint orchestration of the diffuse + mirror + glass shading
// model declared in raysplats.h. The paper shows meshes with reflections,
// shadows and glass in a Gaussian scene (Sec. 1, Figs. 1 and 3-6) but
// specifies no shading model; the one implemented here is stated in the
// header.
#include <math.h>
#include <string.h>

#include "rs_device.h"

namespace rs {

struct MeshParams {
    int64_t n_rays;
    int64_t n_packets;
    int64_t n_tris;
    int32_t root;
    int32_t any_hit;
    int32_t n_views;
    int32_t tile_shift;
    ViewEntry views[RS_MAX_VIEWS];
};

// Moller-Trumbore for record r0..r2 (v0, e1, e2), both faces: t > 0 or +inf.
__device__ inline float tri_hit(const Ray &ray, const float4 r0, const float4 r1, const float4 r2)
{
    const float e1x = r0.w, e1y = r1.x, e1z = r1.y;
    const float e2x = r1.z, e2y = r1.w, e2z = r2.x;
    const float px = ray.dy * e2z - ray.dz * e2y;
    const float py = ray.dz * e2x - ray.dx * e2z;
    const float pz = ray.dx * e2y - ray.dy * e2x;
    const float det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0f) return kInf;
    const float inv = 1.0f / det;
    const float sx = ray.ox - r0.x, sy = ray.oy - r0.y, sz = ray.oz - r0.z;
    const float u = (sx * px + sy * py + sz * pz) * inv;
    if (u < 0.0f || u > 1.0f) return kInf;
    const float qx = sy * e1z - sz * e1y;
    const float qy = sz * e1x - sx * e1z;
    const float qz = sx * e1y - sy * e1x;
    const float v = (ray.dx * qx + ray.dy * qy + ray.dz * qz) * inv;
    if (v < 0.0f || u + v > 1.0f) return kInf;
    const float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
    return t > 0.0f ? t : kInf;
}

// One wavefront per 64-ray tile, wave-uniform BVH walk (as the Gaussian
// traversal); each lane keeps its closest hit below its limit. With any_hit a
// lane stops at its first hit.
__global__ __launch_bounds__(64) void k_mesh_trace(const float4 *__restrict__ records, const float4 *__restrict__ nodes,
                                                   const float *__restrict__ origin, const float *__restrict__ dir,
                                                   const float *__restrict__ t_limit, float *__restrict__ t_out,
                                                   int32_t *__restrict__ tri_out, int32_t *status, const MeshParams P)
{
    const int lane = threadIdx.x;
    const int64_t pkt = blockIdx.x;
    if (pkt >= P.n_packets) return;
    bool valid;
    const int64_t rid = packet_ray(P, pkt, lane, valid);
    Ray ray;
    float limit = kInf;
    if (valid) {
        ray.ox = origin[3 * rid];
        ray.oy = origin[3 * rid + 1];
        ray.oz = origin[3 * rid + 2];
        ray.dx = dir[3 * rid];
        ray.dy = dir[3 * rid + 1];
        ray.dz = dir[3 * rid + 2];
        if (t_limit) limit = t_limit[rid];
    } else {
        ray.ox = ray.oy = ray.oz = 0.0f;
        ray.dx = ray.dy = 0.0f;
        ray.dz = 1.0f;
    }
    const Slab sl = make_slab(ray);
    bool live = valid && limit > 0.0f && P.n_tris > 0;
    float best = limit;  // hits need t < best
    int32_t best_tri = -1;
    float t_hi_w = widen(best, sl.pad);
    constexpr int32_t kDone = INT32_MIN;
    int32_t node = P.root;
    int32_t sp = 0, stackv = 0;
    bool overflow = false;
    if (wave_ballot(live)) {
        for (;;) {
            while (node >= 0) {
                const int64_t ns = __builtin_amdgcn_readfirstlane(node);
                const float4 n0 = nodes[4 * ns], n1 = nodes[4 * ns + 1], n2 = nodes[4 * ns + 2], n3 = nodes[4 * ns + 3];
                float ln, lf, rn, rf;
                child_slabs<kMixedOctant>(n0, n1, n2, sl, ln, lf, rn, rf);
                const bool hl = live && overlaps(ln, widen_exit(lf, sl.pad), 0.0f, t_hi_w);
                const bool hr = live && overlaps(rn, widen_exit(rf, sl.pad), 0.0f, t_hi_w);
                const uint64_t bl = wave_ballot(hl), br = wave_ballot(hr);
                const int32_t left = __float_as_int(n3.x), right = __float_as_int(n3.y);
                if (bl && br) {
                    const uint64_t pref = wave_ballot(hl && (!hr || ln <= rn));
                    const bool lfirst = 2 * __popcll(pref) >= __popcll(bl | br);
                    if (sp >= 64) {
                        overflow = true;
                        node = kDone;
                        break;
                    }
                    stackv = (lane == sp) ? (lfirst ? right : left) : stackv;
                    ++sp;
                    node = lfirst ? left : right;
                } else if (bl) {
                    node = left;
                } else if (br) {
                    node = right;
                } else if (sp == 0) {
                    node = kDone;
                } else {
                    --sp;
                    node = __builtin_amdgcn_readlane(stackv, sp);
                }
            }
            if (node == kDone) break;
            {
                const int64_t js = __builtin_amdgcn_readfirstlane(~node);
                const float4 r0 = records[4 * js], r1 = records[4 * js + 1], r2 = records[4 * js + 2];
                const float t = live ? tri_hit(ray, r0, r1, r2) : kInf;
                if (t < best) {
                    best = t;
                    best_tri = __float_as_int(r2.z);
                    t_hi_w = widen(best, sl.pad);
                    if (P.any_hit) live = false;
                }
            }
            if (!wave_ballot(live)) break;
            if (sp == 0) break;
            --sp;
            node = __builtin_amdgcn_readlane(stackv, sp);
        }
    }
    if (overflow && lane == 0) atomicOr(status, kStatusStack);
    if (valid) {
        t_out[rid] = best_tri >= 0 ? best : kInf;
        tri_out[rid] = best_tri;
    }
}

// Frame scratch: per level k, the path rays (level 0: the caller's rays) and
// the shadow rays of their hits. Inactive rays carry t_max = -inf.
struct PathLevel {
    float *o, *d;        // [n][3] rays (level >= 1)
    float *tmax, *bg;    // [n] Gaussian range, [n][3] background of the forward render
    float *out;          // [n][3] C_k (+ T_k bg when the ray leaves the mesh)
    SetState st;         // forward state (final colour and T, last key, list bookkeeping)
    float *t;            // [n] closest triangle distance
    int32_t *tri;        // [n] closest triangle (-1 none)
    float *w;            // [n] continuation weight (0: none)
    float *shade;        // [n][3] background of the adjoint: D_k + w R_{k+1} at a hit, bg_k otherwise
    float *g;            // [n][3] upstream gradient (level >= 1)
    float *W;            // [n] path weight
};

struct ShadowLevel {
    float *o, *d, *tmax;  // rays to the light (t_max = distance)
    float *out;           // [n][3] transmittance in channel 0
    SetState st;
    float *wd;            // [n] diffuse weight * albedo * (n.l) * intensity (0 when blocked or absent)
    float *tb;            // [n] blocker distance (any hit)
    int32_t *trib;        // [n] blocker (-1 none)
    float *g;             // [n][3] upstream gradient of the transmittance (channel 0)
};

// The stored hit lists of all 2B + 1 ray sets share one pool of C slots per ray
// and set on average.
struct Frame {
    PathLevel P[RS_MAX_BOUNCES + 1];
    ShadowLevel S[RS_MAX_BOUNCES];
    ListPool pool;
    int32_t bounces;
    size_t total;
};

static Frame frame_layout(char *base, int64_t n, int32_t cap, int bounces)
{
    Frame F{};
    F.bounces = bounces;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align256(off + bytes);
        return p;
    };
    const size_t f = size_t(n > 0 ? n : 1) * 4;
    auto fl = [&](size_t k) { return reinterpret_cast<float *>(take(k * f)); };
    auto state = [&]() {
        SetState S;
        S.fin = reinterpret_cast<float4 *>(fl(4));
        S.last = reinterpret_cast<uint4 *>(fl(4));
        S.list = cap > 0 ? reinterpret_cast<int4 *>(fl(4)) : nullptr;
        return S;
    };
    for (int k = 0; k <= bounces; ++k) {
        PathLevel &L = F.P[k];
        if (k > 0) {
            L.o = fl(3);
            L.d = fl(3);
            L.g = fl(3);
        }
        L.tmax = fl(1);
        L.bg = fl(3);
        L.out = fl(3);
        L.st = state();
        L.t = fl(1);
        L.tri = reinterpret_cast<int32_t *>(fl(1));
        L.w = fl(1);
        L.shade = fl(3);
        L.W = fl(1);
    }
    for (int k = 0; k < bounces; ++k) {
        ShadowLevel &S = F.S[k];
        S.o = fl(3);
        S.d = fl(3);
        S.tmax = fl(1);
        S.out = fl(3);
        S.st = state();
        S.wd = fl(1);
        S.tb = fl(1);
        S.trib = reinterpret_cast<int32_t *>(fl(1));
        S.g = fl(3);
    }
    if (cap > 0 && n > 0) {
        const int64_t chunks = list_chunks(n * int64_t(cap) * (2 * bounces + 1));
        F.pool = list_pool_at(take(list_pool_bytes(chunks)), chunks);
        if (!base) F.pool.chunks = chunks;
    }
    F.total = off;
    return F;
}

struct ShadeConst {
    float lx, ly, lz, intensity, albedo, wm, wd, offset, ior;
    float bg[3];
};

constexpr int32_t kMatMirror = 1, kMatGlass = 2;

// Level 0: every camera ray is active.
__global__ void k_path_init(const PathLevel L, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    L.tmax[i] = kInf;
}

// After a level's closest-hit trace: the Gaussians of an active ray stop at
// its triangle (over black) or run to infinity (over bg).
__global__ void k_path_prep(const PathLevel L, int64_t n, ShadeConst C)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool active = L.tmax[i] > 0.0f;
    const bool hit = active && L.tri[i] >= 0;
    if (active) L.tmax[i] = hit ? L.t[i] : kInf;
    for (int c = 0; c < 3; ++c) L.bg[3 * i + c] = active && !hit ? C.bg[c] : 0.0f;
    L.w[i] = 0.0f;
}

// From the hits of path level k (rays o, d): the continuation rays of level
// k + 1 (mirror reflection, glass refraction or total internal reflection)
// with their weights, and the shadow rays of level k.
__global__ void k_path_spawn(const float *__restrict__ origin, const float *__restrict__ dir, const PathLevel L,
                             const PathLevel N, const ShadowLevel S, const float4 *__restrict__ trecords,
                             const int32_t *__restrict__ tinv, int64_t n, ShadeConst C)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    N.tmax[i] = -kInf;
    S.tmax[i] = -kInf;
    S.wd[i] = 0.0f;
    for (int c = 0; c < 3; ++c) {
        N.o[3 * i + c] = 0.0f;
        S.o[3 * i + c] = 0.0f;
        N.d[3 * i + c] = c == 2 ? 1.0f : 0.0f;
        S.d[3 * i + c] = c == 2 ? 1.0f : 0.0f;
    }
    if (!(L.tmax[i] > 0.0f) || L.tri[i] < 0) return;
    const int32_t j = tinv[L.tri[i]];
    const float4 r0 = trecords[4 * j], r1 = trecords[4 * j + 1], r2 = trecords[4 * j + 2];
    const float e1x = r0.w, e1y = r1.x, e1z = r1.y, e2x = r1.z, e2y = r1.w, e2z = r2.x;
    float gx = e1y * e2z - e1z * e2y, gy = e1z * e2x - e1x * e2z, gz = e1x * e2y - e1y * e2x;
    const float gn = 1.0f / sqrtf(gx * gx + gy * gy + gz * gz);
    gx *= gn;
    gy *= gn;
    gz *= gn;
    const float dx = dir[3 * i], dy = dir[3 * i + 1], dz = dir[3 * i + 2];
    const float dg = dx * gx + dy * gy + dz * gz;
    const bool entering = !(dg > 0.0f);  // the facing normal n = -n_g when the ray runs along n_g
    const float nx = entering ? gx : -gx, ny = entering ? gy : -gy, nz = entering ? gz : -gz;
    const float dn = entering ? dg : -dg;  // d.n <= 0
    const float t = L.t[i];
    const float Px = origin[3 * i] + t * dx, Py = origin[3 * i + 1] + t * dy, Pz = origin[3 * i + 2] + t * dz;
    const int32_t mat = __float_as_int(r2.y);
    const float rho_d = mat == kMatMirror ? C.wd : (mat == kMatGlass ? 0.0f : 1.0f);
    const float ox = Px + C.offset * nx, oy = Py + C.offset * ny, oz = Pz + C.offset * nz;
    // continuation
    float w = 0.0f, cx = 0.0f, cy = 0.0f, cz = 1.0f, side = 1.0f;
    if (mat == kMatMirror && C.wm > 0.0f) {
        w = C.wm;
        cx = dx - 2.0f * dn * nx;
        cy = dy - 2.0f * dn * ny;
        cz = dz - 2.0f * dn * nz;
    } else if (mat == kMatGlass) {
        const float eta = entering ? 1.0f / C.ior : C.ior;
        const float cos_i = -dn;
        const float k = 1.0f - eta * eta * (1.0f - cos_i * cos_i);
        if (k < 0.0f) {
            w = 1.0f;
            cx = dx + 2.0f * cos_i * nx;
            cy = dy + 2.0f * cos_i * ny;
            cz = dz + 2.0f * cos_i * nz;
        } else {
            const float ks = sqrtf(k);
            const float a = eta * cos_i - ks;
            cx = eta * dx + a * nx;
            cy = eta * dy + a * ny;
            cz = eta * dz + a * nz;
            const float q = (1.0f - C.ior) / (1.0f + C.ior);
            const float r0f = q * q;
            const float c = 1.0f - (entering ? cos_i : ks);
            const float c2 = c * c;
            const float F = r0f + (1.0f - r0f) * (c2 * c2 * c);
            w = 1.0f - F;
            side = -1.0f;
        }
    }
    if (w > 0.0f) {
        N.o[3 * i] = Px + side * C.offset * nx;
        N.o[3 * i + 1] = Py + side * C.offset * ny;
        N.o[3 * i + 2] = Pz + side * C.offset * nz;
        N.d[3 * i] = cx;
        N.d[3 * i + 1] = cy;
        N.d[3 * i + 2] = cz;
        N.tmax[i] = kInf;
        L.w[i] = w;
    }
    // shadow ray
    const float lx = C.lx - Px, ly = C.ly - Py, lz = C.lz - Pz;
    const float nl = (nx * lx + ny * ly + nz * lz) / sqrtf(lx * lx + ly * ly + lz * lz);
    if (rho_d > 0.0f && nl > 0.0f) {
        const float sx = C.lx - ox, sy = C.ly - oy, sz = C.lz - oz;
        const float dist = sqrtf(sx * sx + sy * sy + sz * sz);
        S.o[3 * i] = ox;
        S.o[3 * i + 1] = oy;
        S.o[3 * i + 2] = oz;
        S.d[3 * i] = sx / dist;
        S.d[3 * i + 1] = sy / dist;
        S.d[3 * i + 2] = sz / dist;
        S.tmax[i] = dist;
        S.wd[i] = rho_d * C.albedo * nl * C.intensity;
    }
}

// A blocked shadow ray does no work and contributes nothing.
__global__ void k_shadow_prep(const ShadowLevel S, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (S.tmax[i] > 0.0f && S.trib[i] >= 0) {
        S.tmax[i] = -kInf;
        S.wd[i] = 0.0f;
    }
}

// Radiance bottom-up: R_B = C_B; R_k = C_k + T_k (D_k + w_k R_{k+1}) at a hit
// with k < B; pixel = R_0. The shade D_k + w_k R_{k+1} is the background of
// path ray k's adjoint.
__global__ void k_path_combine(const Frame F, int64_t n, ShadeConst C, float *__restrict__ out_rgb)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float R[3] = {0.0f, 0.0f, 0.0f};
    bool next = false;  // R holds an active R_{k+1}
    for (int k = F.bounces; k >= 0; --k) {
        const PathLevel &L = F.P[k];
        if (!(L.tmax[i] > -kInf)) {  // not spawned
            next = false;
            continue;
        }
        const float T = L.st.fin[i].w;
        const bool hit = k < F.bounces && L.tri[i] >= 0;
        float sh[3];
        for (int c = 0; c < 3; ++c) sh[c] = L.bg[3 * i + c];
        if (hit) {
            const float D = F.S[k].tmax[i] > 0.0f ? F.S[k].wd[i] * F.S[k].out[3 * i] : 0.0f;
            const float w = next ? L.w[i] : 0.0f;
            for (int c = 0; c < 3; ++c) sh[c] = __builtin_fmaf(w, R[c], D);
        }
        for (int c = 0; c < 3; ++c) {
            R[c] = hit ? __builtin_fmaf(T, sh[c], L.out[3 * i + c]) : L.out[3 * i + c];
            L.shade[3 * i + c] = sh[c];
        }
        next = true;
    }
    for (int c = 0; c < 3; ++c) out_rgb[3 * i + c] = R[c];
}

// Upstream gradients top-down: W_0 = 1, W_{k+1} = W_k T_k w_k; path ray k
// gets W_k g, shadow ray k gets W_k T_k D-weight sum(g) on its transmittance.
__global__ void k_path_bwd_prep(const Frame F, int64_t n, const float *__restrict__ grad)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g0 = grad[3 * i], g1 = grad[3 * i + 1], g2 = grad[3 * i + 2];
    float W = 1.0f;
    for (int k = 0; k <= F.bounces; ++k) {
        const PathLevel &L = F.P[k];
        const bool active = L.tmax[i] > -kInf;
        if (!active) W = 0.0f;
        if (k > 0) {
            L.g[3 * i] = g0 * W;
            L.g[3 * i + 1] = g1 * W;
            L.g[3 * i + 2] = g2 * W;
        }
        const float T = active ? L.st.fin[i].w : 0.0f;
        if (k < F.bounces) {
            const ShadowLevel &S = F.S[k];
            const float ws = S.tmax[i] > 0.0f ? W * T * S.wd[i] : 0.0f;
            S.g[3 * i] = (g0 + g1 + g2) * ws;
            S.g[3 * i + 1] = 0.0f;
            S.g[3 * i + 2] = 0.0f;
            W = W * T * L.w[i];
        }
    }
}

// ------------------------------------------------------------------- host

static inline int grid_for(int64_t n) { return int((n + 255) / 256); }

static MeshParams mesh_params(const BvhDesc &M, const rs_rays *rays, int any_hit, int tile_shift)
{
    MeshParams P{};
    P.n_rays = rays->n;
    P.root = M.root;
    P.n_tris = M.n;
    P.any_hit = any_hit;
    P.n_packets = plan_packets(P, rays, tile_shift);
    return P;
}

int launch_trace_mesh(const BvhDesc &M, const rs_rays *rays, const float *t_limit, int any_hit, int tile_shift,
                      float *t_hit, int32_t *tri, hipStream_t st)
{
    Layout L = make_layout(M.n);
    WsHeader *h = reinterpret_cast<WsHeader *>(M.ws + L.header);
    MeshParams P = mesh_params(M, rays, any_hit, tile_shift);
    if (rays->n == 0) return RS_OK;
    k_mesh_trace<<<int(P.n_packets > 0 ? P.n_packets : 1), kWave, 0, st>>>(
        reinterpret_cast<const float4 *>(M.ws + L.records), reinterpret_cast<const float4 *>(M.ws + L.nodes),
        rays->origin, rays->dir, t_limit, t_hit, tri, &h->status, P);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

size_t mesh_frame_bytes(int64_t n, int32_t cap, int bounces) { return frame_layout(nullptr, n, cap, bounces).total; }

// The state and list pool of ray set `set` of a frame (0..B: path levels, B+1..2B: shadow levels).
int mesh_frame_set(char *frame, int64_t n, int32_t cap, int bounces, int set, SetState *st, ListPool *pool)
{
    if (set < 0 || set > 2 * bounces) return RS_ERR_INVALID_ARG;
    const Frame F = frame_layout(frame, n, cap, bounces);
    *st = set <= bounces ? F.P[set].st : F.S[set - bounces - 1].st;
    *pool = F.pool;
    return RS_OK;
}

static ShadeConst shade_const(const rs_shading *sh, const rs_params *p)
{
    ShadeConst C;
    C.lx = sh->light[0];
    C.ly = sh->light[1];
    C.lz = sh->light[2];
    C.intensity = sh->intensity;
    C.albedo = sh->albedo;
    C.wm = sh->mirror_reflectance;
    C.wd = sh->mirror_diffuse;
    C.offset = sh->offset;
    C.ior = sh->ior;
    for (int c = 0; c < 3; ++c) C.bg[c] = p->bg[c];
    return C;
}

// rays of the frame with the primary's layout (same count and views)
static rs_rays frame_rays(const rs_rays *prim, const float *o, const float *d, const float *tmax, const float *bg)
{
    rs_rays r = *prim;
    r.origin = o;
    r.dir = d;
    r.t_max = tmax;
    r.bg = bg;
    return r;
}

// The 2B + 1 ray sets of a pixel: path rays of levels 0..B (Gaussians up to
// their triangle) and the shadow rays of levels 0..B-1. Spawning depends only
// on the triangle traces, so all of them render in one persistent launch.
static int mesh_sets(const Frame &F, const rs_rays *rays, rs_rays *sr, SetDesc *S, bool bwd, const float *grad)
{
    int m = 0;
    for (int k = 0; k <= F.bounces; ++k) {
        const PathLevel &L = F.P[k];
        sr[m] = frame_rays(rays, k ? L.o : rays->origin, k ? L.d : rays->dir, L.tmax, bwd ? L.shade : L.bg);
        S[m] = SetDesc{};
        S[m].rays = &sr[m];
        S[m].state = L.st;
        if (bwd)
            S[m].grad = k ? L.g : grad;  // the shade is the background behind the ray's last hit
        else
            S[m].out_rgb = L.out;
        ++m;
    }
    for (int k = 0; k < F.bounces; ++k) {
        const ShadowLevel &H = F.S[k];
        sr[m] = frame_rays(rays, H.o, H.d, H.tmax, nullptr);
        S[m] = SetDesc{};
        S[m].rays = &sr[m];
        S[m].state = H.st;
        if (bwd)
            S[m].grad = H.g;
        else
            S[m].out_rgb = H.out;
        S[m].bg[0] = S[m].bg[1] = S[m].bg[2] = 1.0f;  // transmittance: zero colours, white background
        S[m].zero_colour = 1;
        ++m;
    }
    return m;
}

int launch_mesh_fwd(const BvhDesc &G, const BvhDesc &M, const rs_gaussians *g, const rs_shading *sh,
                    const rs_rays *rays, const rs_params *p, float *out_rgb, void *frame, hipStream_t st)
{
    const int64_t n = rays->n;
    if (n == 0) return RS_OK;
    Frame F = frame_layout(static_cast<char *>(frame), n, p->hit_list, sh->max_bounces);
    const ShadeConst C = shade_const(sh, p);
    Layout LM = make_layout(M.n);
    const int ts = tile_shift_of(p);
    const float4 *trec = reinterpret_cast<const float4 *>(M.ws + LM.records);
    const int32_t *tinv = reinterpret_cast<const int32_t *>(M.ws + LM.inv);
    rs_rays sr[kMaxSets];
    SetDesc S[kMaxSets];
    const int nsets = mesh_sets(F, rays, sr, S, false, nullptr);
    int e;
    // 1. triangle traces level by level: closest hits of the path rays, spawning, shadow blockers
    k_path_init<<<grid_for(n), 256, 0, st>>>(F.P[0], n);
    for (int k = 0; k <= F.bounces; ++k) {
        const PathLevel &L = F.P[k];
        if ((e = launch_trace_mesh(M, &sr[k], L.tmax, 0, ts, L.t, L.tri, st))) return e;
        k_path_prep<<<grid_for(n), 256, 0, st>>>(L, n, C);
        if (k == F.bounces) break;
        const ShadowLevel &H = F.S[k];
        k_path_spawn<<<grid_for(n), 256, 0, st>>>(k ? L.o : rays->origin, k ? L.d : rays->dir, L, F.P[k + 1], H,
                                                   trec, tinv, n, C);
        // blockers: any triangle strictly before the light
        if ((e = launch_trace_mesh(M, &sr[F.bounces + 1 + k], H.tmax, 1, ts, H.tb, H.trib, st))) return e;
        k_shadow_prep<<<grid_for(n), 256, 0, st>>>(H, n);
    }
    // 2. Gaussians along all ray sets in one persistent launch
    rs_params ps = *p;
    ps.flags |= RS_PERSISTENT;
    if ((e = launch_sets(G, g, &ps, nsets, S, F.pool, Pass::Forward, st))) return e;
    // 3. combine bottom-up
    k_path_combine<<<grid_for(n), 256, 0, st>>>(F, n, C, out_rgb);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

int launch_mesh_bwd(const BvhDesc &G, const rs_gaussians *g, const rs_shading *sh, const rs_rays *rays,
                    const rs_params *p, const float *grad, void *frame, const rs_grads *grads, hipStream_t st)
{
    const int64_t n = rays->n;
    zero_gacc(G, st);
    if (n > 0) {
        Frame F = frame_layout(static_cast<char *>(frame), n, p->hit_list, sh->max_bounces);
        k_path_bwd_prep<<<grid_for(n), 256, 0, st>>>(F, n, grad);
        rs_rays sr[kMaxSets];
        SetDesc S[kMaxSets];
        const int nsets = mesh_sets(F, rays, sr, S, true, grad);
        rs_params ps = *p;
        ps.flags |= RS_PERSISTENT;
        int e;
        if (F.pool.chunks > 0) {
            // stored lists of all sets, then traversal for the rays whose list is incomplete
            if ((e = launch_sets(G, g, &ps, nsets, S, F.pool, Pass::AdjointList, st))) return e;
        }
        if ((e = launch_sets(G, g, &ps, nsets, S, F.pool, Pass::AdjointTraverse, st))) return e;
    }
    scatter_gacc(G, g->quat, grads, st);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

}  // namespace rs
