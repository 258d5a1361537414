// Triangle mesh + Gaussians: triangle BVH traversal (closest or any hit,
// Moller-Trumbore), secondary-ray spawning, and the forward / adjoint
// orchestration of the mirror + shadow shading model declared in
// raysplats.h. The paper shows meshes with reflections and shadows in a
// Gaussian scene (Sec. 1, Figs. 1 and 3-6) but specifies no shading model;
// the one implemented here is stated in the header.
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

// Frame scratch layout (per ray): see frame_layout.
struct Frame {
    float *t_mesh;   // [n]
    int32_t *tri;    // [n]
    int32_t *tri2;   // [n] secondary trace results
    float *tmax_p;   // [n]
    float *bg_p;     // [n][3]
    float *out_p;    // [n][3]
    float4 *st_p;    // [n]
    float *r_o, *r_d, *r_tmax, *r_bg, *out_r;  // reflection rays
    float4 *st_r;
    float *s_o, *s_d, *s_tmax, *out_s;  // shadow rays
    float4 *st_s;
    float *t2;       // [n] secondary trace distances
    float *w_m;      // [n] reflection weight of the hit triangle
    float *w_s;      // [n] diffuse weight * albedo * (n.l) * intensity (0 when blocked)
    float *shade;    // [n][3] background of the primary adjoint
    float4 *st_pb;   // [n] primary state with the final colour
    float *g_r, *g_s;  // [n][3] upstream gradients of the secondary rays
    int32_t *cnt[3];   // stored hit lists of the three ray sets (hit_list > 0)
    int32_t *ids[3];   // [cap][n] each
    size_t total;
};

static Frame frame_layout(char *base, int64_t n, int32_t cap)
{
    Frame F{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align256(off + bytes);
        return p;
    };
    const size_t f = size_t(n > 0 ? n : 1) * 4;
    F.t_mesh = reinterpret_cast<float *>(take(f));
    F.tri = reinterpret_cast<int32_t *>(take(f));
    F.tri2 = reinterpret_cast<int32_t *>(take(f));
    F.tmax_p = reinterpret_cast<float *>(take(f));
    F.bg_p = reinterpret_cast<float *>(take(3 * f));
    F.out_p = reinterpret_cast<float *>(take(3 * f));
    F.st_p = reinterpret_cast<float4 *>(take(4 * f));
    F.r_o = reinterpret_cast<float *>(take(3 * f));
    F.r_d = reinterpret_cast<float *>(take(3 * f));
    F.r_tmax = reinterpret_cast<float *>(take(f));
    F.r_bg = reinterpret_cast<float *>(take(3 * f));
    F.out_r = reinterpret_cast<float *>(take(3 * f));
    F.st_r = reinterpret_cast<float4 *>(take(4 * f));
    F.s_o = reinterpret_cast<float *>(take(3 * f));
    F.s_d = reinterpret_cast<float *>(take(3 * f));
    F.s_tmax = reinterpret_cast<float *>(take(f));
    F.out_s = reinterpret_cast<float *>(take(3 * f));
    F.st_s = reinterpret_cast<float4 *>(take(4 * f));
    F.t2 = reinterpret_cast<float *>(take(f));
    F.w_m = reinterpret_cast<float *>(take(f));
    F.w_s = reinterpret_cast<float *>(take(f));
    F.shade = reinterpret_cast<float *>(take(3 * f));
    F.st_pb = reinterpret_cast<float4 *>(take(4 * f));
    F.g_r = reinterpret_cast<float *>(take(3 * f));
    F.g_s = reinterpret_cast<float *>(take(3 * f));
    for (int k = 0; k < 3; ++k) {
        F.cnt[k] = cap > 0 ? reinterpret_cast<int32_t *>(take(f)) : nullptr;
        F.ids[k] = cap > 0 ? reinterpret_cast<int32_t *>(take(f * size_t(cap))) : nullptr;
    }
    F.total = off;
    return F;
}

struct ShadeConst {
    float lx, ly, lz, intensity, albedo, wm, wd, offset;
    float bg[3];
};

// Primary rays: Gaussians are bounded by the closest triangle; a ray that hits a
// triangle composites over a black background (its shade is added later).
__global__ void k_mesh_primary_prep(const Frame F, int64_t n, ShadeConst C)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool hit = F.tri[i] >= 0;
    F.tmax_p[i] = hit ? F.t_mesh[i] : kInf;
    for (int c = 0; c < 3; ++c) F.bg_p[3 * i + c] = hit ? 0.0f : C.bg[c];
}

// Reflection and shadow rays of every primary ray that hit a triangle; the
// others get t_max = -inf (no work).
__global__ void k_mesh_spawn(const float *__restrict__ origin, const float *__restrict__ dir,
                             const float4 *__restrict__ trecords, const int32_t *__restrict__ tinv, const Frame F,
                             int64_t n, ShadeConst C)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t tri = F.tri[i];
    F.r_tmax[i] = -kInf;
    F.s_tmax[i] = -kInf;
    F.w_m[i] = 0.0f;
    F.w_s[i] = 0.0f;
    for (int c = 0; c < 3; ++c) {
        F.r_o[3 * i + c] = 0.0f;
        F.s_o[3 * i + c] = 0.0f;
        F.r_d[3 * i + c] = c == 2 ? 1.0f : 0.0f;
        F.s_d[3 * i + c] = c == 2 ? 1.0f : 0.0f;
    }
    if (tri < 0) return;
    const int32_t j = tinv[tri];
    const float4 r0 = trecords[4 * j], r1 = trecords[4 * j + 1], r2 = trecords[4 * j + 2];
    const float e1x = r0.w, e1y = r1.x, e1z = r1.y, e2x = r1.z, e2y = r1.w, e2z = r2.x;
    float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const float nn = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
    nx *= nn;
    ny *= nn;
    nz *= nn;
    const float dx = dir[3 * i], dy = dir[3 * i + 1], dz = dir[3 * i + 2];
    float dn = dx * nx + dy * ny + dz * nz;
    if (dn > 0.0f) {
        nx = -nx;
        ny = -ny;
        nz = -nz;
        dn = -dn;
    }
    const float t = F.t_mesh[i];
    const float Px = origin[3 * i] + t * dx, Py = origin[3 * i + 1] + t * dy, Pz = origin[3 * i + 2] + t * dz;
    const bool mirror = __float_as_int(r2.y) == 1;
    const float rho_m = mirror ? C.wm : 0.0f, rho_d = mirror ? C.wd : 1.0f;
    const float ox = Px + C.offset * nx, oy = Py + C.offset * ny, oz = Pz + C.offset * nz;
    if (rho_m > 0.0f) {
        F.r_o[3 * i] = ox;
        F.r_o[3 * i + 1] = oy;
        F.r_o[3 * i + 2] = oz;
        F.r_d[3 * i] = dx - 2.0f * dn * nx;
        F.r_d[3 * i + 1] = dy - 2.0f * dn * ny;
        F.r_d[3 * i + 2] = dz - 2.0f * dn * nz;
        F.r_tmax[i] = kInf;
        F.w_m[i] = rho_m;
    }
    const float lx = C.lx - Px, ly = C.ly - Py, lz = C.lz - Pz;
    const float nl = (nx * lx + ny * ly + nz * lz) / sqrtf(lx * lx + ly * ly + lz * lz);
    if (rho_d > 0.0f && nl > 0.0f) {
        const float sx = C.lx - ox, sy = C.ly - oy, sz = C.lz - oz;
        const float dist = sqrtf(sx * sx + sy * sy + sz * sz);
        F.s_o[3 * i] = ox;
        F.s_o[3 * i + 1] = oy;
        F.s_o[3 * i + 2] = oz;
        F.s_d[3 * i] = sx / dist;
        F.s_d[3 * i + 1] = sy / dist;
        F.s_d[3 * i + 2] = sz / dist;
        F.s_tmax[i] = dist;
        F.w_s[i] = rho_d * C.albedo * nl * C.intensity;
    }
}

// After the secondary triangle traces: a reflection ray stops at its triangle
// (black beyond it, bg when it hits none); a blocked shadow ray does no work.
__global__ void k_mesh_secondary_prep(const Frame F, int64_t n, ShadeConst C, const float *__restrict__ t_shadow,
                                      const int32_t *__restrict__ tri_shadow)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (F.r_tmax[i] > 0.0f) {
        const bool hit = F.tri2[i] >= 0;
        F.r_tmax[i] = hit ? F.t2[i] : kInf;
        for (int c = 0; c < 3; ++c) F.r_bg[3 * i + c] = hit ? 0.0f : C.bg[c];
    } else {
        for (int c = 0; c < 3; ++c) F.r_bg[3 * i + c] = 0.0f;
    }
    if (F.s_tmax[i] > 0.0f && tri_shadow[i] >= 0) {
        F.s_tmax[i] = -kInf;
        F.w_s[i] = 0.0f;
    }
}

// pixel = C_p + T_p * shade, shade = w_m C_r + w_d albedo (n.l) I T_s; the shade
// is also the background of the primary ray's adjoint.
__global__ void k_mesh_combine(const Frame F, int64_t n, ShadeConst C, float *__restrict__ out_rgb)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 sp = F.st_p[i];
    const float Tp = sp.w;
    const bool hit = F.tri[i] >= 0;
    float o[3], sh[3];
    for (int c = 0; c < 3; ++c) {
        sh[c] = hit ? F.w_m[i] * F.out_r[3 * i + c] + F.w_s[i] * F.out_s[3 * i] : C.bg[c];
        o[c] = hit ? __builtin_fmaf(Tp, sh[c], F.out_p[3 * i + c]) : F.out_p[3 * i + c];
        out_rgb[3 * i + c] = o[c];
        F.shade[3 * i + c] = sh[c];
    }
    F.st_pb[i] = make_float4(o[0], o[1], o[2], Tp);
}

// Upstream gradients of the secondary rays: g * T_p * w_m per channel for the
// reflection, sum(g) * T_p * w_s in channel 0 for the shadow transmittance.
__global__ void k_mesh_bwd_prep(const Frame F, int64_t n, const float *__restrict__ grad)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g0 = grad[3 * i], g1 = grad[3 * i + 1], g2 = grad[3 * i + 2];
    const float Tp = F.st_p[i].w;
    const float wm = Tp * F.w_m[i], ws = Tp * F.w_s[i];
    F.g_r[3 * i] = g0 * wm;
    F.g_r[3 * i + 1] = g1 * wm;
    F.g_r[3 * i + 2] = g2 * wm;
    F.g_s[3 * i] = (g0 + g1 + g2) * ws;
    F.g_s[3 * i + 1] = 0.0f;
    F.g_s[3 * i + 2] = 0.0f;
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

size_t mesh_frame_bytes(int64_t n, int32_t cap) { return frame_layout(nullptr, n, cap).total; }

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

// The three ray sets of a pixel: the primary ray (Gaussians in front of the
// mesh), its mirror reflection and its shadow ray. Spawning depends only on
// the triangle traces, so all three render in one persistent launch.
static void mesh_sets(const Frame &F, const rs_rays *rays, rs_rays sets_rays[3], SetDesc S[3], bool bwd,
                      const float *grad)
{
    sets_rays[0] = frame_rays(rays, rays->origin, rays->dir, F.tmax_p, bwd ? F.shade : F.bg_p);
    sets_rays[1] = frame_rays(rays, F.r_o, F.r_d, F.r_tmax, F.r_bg);
    sets_rays[2] = frame_rays(rays, F.s_o, F.s_d, F.s_tmax, nullptr);
    for (int k = 0; k < 3; ++k) {
        S[k] = SetDesc{};
        S[k].rays = &sets_rays[k];
        S[k].count = F.cnt[k];
        S[k].ids = F.ids[k];
    }
    if (bwd) {
        S[0].state = F.st_pb;  // final colour of the pixel, with the shade as background
        S[0].grad = grad;
        S[1].grad = F.g_r;
        S[2].grad = F.g_s;
    } else {
        S[0].out_rgb = F.out_p;
        S[1].out_rgb = F.out_r;
        S[2].out_rgb = F.out_s;
        S[0].state = F.st_p;
    }
    S[1].state = F.st_r;
    S[2].state = F.st_s;
    S[2].bg[0] = S[2].bg[1] = S[2].bg[2] = 1.0f;  // transmittance: zero colours, white background
    S[2].zero_colour = 1;
}

int launch_mesh_fwd(const BvhDesc &G, const BvhDesc &M, const rs_gaussians *g, const rs_shading *sh,
                    const rs_rays *rays, const rs_params *p, float *out_rgb, void *frame, hipStream_t st)
{
    const int64_t n = rays->n;
    if (n == 0) return RS_OK;
    Frame F = frame_layout(static_cast<char *>(frame), n, p->hit_list);
    const ShadeConst C = shade_const(sh, p);
    Layout LM = make_layout(M.n);
    const int ts = tile_shift_of(p);
    int e;
    // 1. triangle traces: primary closest hits, then the secondary rays they spawn
    if ((e = launch_trace_mesh(M, rays, nullptr, 0, ts, F.t_mesh, F.tri, st))) return e;
    k_mesh_primary_prep<<<grid_for(n), 256, 0, st>>>(F, n, C);
    k_mesh_spawn<<<grid_for(n), 256, 0, st>>>(rays->origin, rays->dir,
                                               reinterpret_cast<const float4 *>(M.ws + LM.records),
                                               reinterpret_cast<const int32_t *>(M.ws + LM.inv), F, n, C);
    rs_rays rr[3];
    SetDesc S[3];
    mesh_sets(F, rays, rr, S, false, nullptr);
    if ((e = launch_trace_mesh(M, &rr[1], F.r_tmax, 0, ts, F.t2, F.tri2, st))) return e;
    // shadow blockers: any triangle strictly before the light (results parked in out_s / g_s)
    if ((e = launch_trace_mesh(M, &rr[2], F.s_tmax, 1, ts, F.out_s, reinterpret_cast<int32_t *>(F.g_s), st)))
        return e;
    k_mesh_secondary_prep<<<grid_for(n), 256, 0, st>>>(F, n, C, F.out_s, reinterpret_cast<const int32_t *>(F.g_s));
    // 2. Gaussians along all three ray sets in one persistent launch
    rs_params ps = *p;
    ps.flags |= RS_PERSISTENT;
    if ((e = launch_sets(G, g, &ps, 3, S, false, st))) return e;
    // 3. combine
    k_mesh_combine<<<grid_for(n), 256, 0, st>>>(F, n, C, out_rgb);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

int launch_mesh_bwd(const BvhDesc &G, const rs_gaussians *g, const rs_rays *rays, const rs_params *p,
                    const float *grad, void *frame, const rs_grads *grads, hipStream_t st)
{
    const int64_t n = rays->n;
    zero_gacc(G, st);
    if (n > 0) {
        Frame F = frame_layout(static_cast<char *>(frame), n, p->hit_list);
        k_mesh_bwd_prep<<<grid_for(n), 256, 0, st>>>(F, n, grad);
        rs_rays rr[3];
        SetDesc S[3];
        mesh_sets(F, rays, rr, S, true, grad);
        rs_params ps = *p;
        ps.flags |= RS_PERSISTENT;
        int e;
        if (p->hit_list > 0) {
            // stored lists of all three sets, then traversal for the rays whose list overflowed
            if ((e = launch_sets(G, g, &ps, 3, S, true, st, true))) return e;
            if (p->max_hits == 0 || p->max_hits > p->hit_list)
                if ((e = launch_sets(G, g, &ps, 3, S, true, st))) return e;
        } else {
            if ((e = launch_sets(G, g, &ps, 3, S, true, st))) return e;
        }
    }
    scatter_gacc(G, grads, st);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

}  // namespace rs
