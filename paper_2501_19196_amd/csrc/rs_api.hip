// C ABI entry points: argument validation, workspace sizing and dispatch to
// the build and render launchers.
#include <string.h>

#include <algorithm>
#include <unordered_map>
#include <vector>

#include "rs_internal.h"

using namespace rs;

static bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static int check_gaussians(const rs_gaussians *g)
{
    if (!g || g->n < 0 || g->n > 0x7ffffffeLL) return RS_ERR_INVALID_ARG;
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->rgb)) return RS_ERR_INVALID_ARG;
    if (g->n > 0 && !aligned(g->quat, 16)) return RS_ERR_INVALID_ARG;
    return RS_OK;
}

static int check_params(const rs_params *p)
{
    if (!p) return RS_ERR_INVALID_ARG;
    if (!(p->Q > 0.0f) || !(p->eps1 >= 0.0f) || p->max_hits < 0 || !(p->t_min >= 0.0f) || !(p->t_min < 3.0e38f))
        return RS_ERR_INVALID_ARG;
    if (p->kbuf != 0 && p->kbuf != 8 && p->kbuf != 16 && p->kbuf != 24 && p->kbuf != 32 && p->kbuf != 48)
        return RS_ERR_INVALID_ARG;
    if (p->stack_depth < 0 || p->stack_depth > 64) return RS_ERR_INVALID_ARG;
    if (p->tile_width != 0 && p->tile_width != 4 && p->tile_width != 8 && p->tile_width != 16 && p->tile_width != 32)
        return RS_ERR_INVALID_ARG;
    if (p->flags & ~(RS_BRUTE_FORCE | RS_PERSISTENT | RS_ZERO_COLOUR | RS_COUNTERS | RS_PAPER_GRADIENT | RS_BUILD_LBVH))
        return RS_ERR_INVALID_ARG;
    if (p->hit_list < 0 || p->hit_list > 4096) return RS_ERR_INVALID_ARG;
    if (p->flags & RS_PAPER_GRADIENT) {
        // the second phase lives in the stored lists: K_max bounds a ray's entries
        if (!(p->eps2 >= 0.0f && p->eps2 <= 1.0f)) return RS_ERR_INVALID_ARG;
        if (p->max_hits <= 0 || p->hit_list <= 0) return RS_ERR_INVALID_ARG;
    }
    return RS_OK;
}

// the list pool's chunk counter and chunk indices are 31-bit
static int check_pool(int64_t n_rays, const rs_params *p, int64_t sets)
{
    if (p->hit_list > 0 && list_chunks(n_rays * int64_t(p->hit_list) * sets) >= (int64_t(1) << 31))
        return RS_ERR_UNSUPPORTED;
    return RS_OK;
}

static int check_rays(const rs_rays *r)
{
    if (!r || r->n < 0) return RS_ERR_INVALID_ARG;
    if (r->n > 0 && (!r->origin || !r->dir)) return RS_ERR_INVALID_ARG;
    if (r->n_views < 0) return RS_ERR_INVALID_ARG;
    if (r->n_views > RS_MAX_VIEWS) return RS_ERR_UNSUPPORTED;
    if (r->n_views > 0) {
        if (!r->views) return RS_ERR_INVALID_ARG;
        int64_t expect = 0;
        for (int v = 0; v < r->n_views; ++v) {
            const rs_view &V = r->views[v];
            if (V.width <= 0 || V.height <= 0 || V.ray_offset != expect) return RS_ERR_INVALID_ARG;
            expect += int64_t(V.width) * V.height;
        }
        if (expect != r->n) return RS_ERR_INVALID_ARG;
    }
    return RS_OK;
}

static int check_bvh(const rs_bvh *b, const rs_gaussians *g, const rs_params *p, BvhDesc &D)
{
    if (!b) return RS_ERR_INVALID_ARG;
    memcpy(&D, b, sizeof(D));
    if (D.magic != kMagic || !D.ws || D.kind != kKindGaussians) return RS_ERR_INVALID_ARG;
    if (D.n != g->n || D.Q != p->Q) return RS_ERR_BVH_MISMATCH;
    return RS_OK;
}

extern "C" {

void rs_default_params(rs_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->Q = 11.3449f;
    p->eps1 = 1e-4f;
    p->t_min = 0.0f;
    p->max_hits = 512;
    p->eps2 = 1e-4f;
}

size_t rs_bvh_workspace_bytes(int64_t n_gaussians)
{
    if (n_gaussians < 0) return 0;
    return make_layout(n_gaussians).total;
}

size_t rs_ray_state_bytes(int64_t n_rays, const rs_params *p)
{
    return n_rays > 0 ? state_layout(n_rays, p ? p->hit_list : 0).total : 0;
}

int rs_build_bvh(const rs_gaussians *g, const rs_params *p, void *ws, size_t ws_bytes, rs_bvh *out, void *stream)
{
    int e = check_gaussians(g);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if (!ws || !out || !aligned(ws, 256)) return RS_ERR_INVALID_ARG;
    if (ws_bytes < make_layout(g->n).total) return RS_ERR_WORKSPACE;
    e = launch_build(g, p->Q, (p->flags & RS_BUILD_LBVH) != 0, static_cast<char *>(ws), static_cast<hipStream_t>(stream));
    if (e) return e;
    BvhDesc D{};
    D.magic = kMagic;
    D.n = g->n;
    D.Q = p->Q;
    D.root = g->n >= 2 ? 0 : ~0;
    D.ws = static_cast<char *>(ws);
    D.ws_bytes = ws_bytes;
    D.kind = kKindGaussians;
    memset(out, 0, sizeof(*out));
    memcpy(out, &D, sizeof(D));
    return RS_OK;
}

int rs_render_fwd(const rs_bvh *bvh, const rs_gaussians *g, const rs_rays *rays, const rs_params *p, float *out_rgb,
                  void *ray_state, void *stream)
{
    int e = check_gaussians(g);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if ((e = check_rays(rays))) return e;
    BvhDesc D;
    if ((e = check_bvh(bvh, g, p, D))) return e;
    if (rays->n > 0 && !out_rgb) return RS_ERR_INVALID_ARG;
    if (ray_state && !aligned(ray_state, 16)) return RS_ERR_INVALID_ARG;
    if ((e = check_pool(rays->n, p, 1))) return e;
    return launch_render(D, g, rays, p, out_rgb, ray_state, nullptr, nullptr, static_cast<hipStream_t>(stream));
}

int rs_render_bwd(const rs_bvh *bvh, const rs_gaussians *g, const rs_rays *rays, const rs_params *p,
                  const float *grad_rgb, const void *ray_state, rs_grads *out, void *stream)
{
    int e = check_gaussians(g);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if ((e = check_rays(rays))) return e;
    BvhDesc D;
    if ((e = check_bvh(bvh, g, p, D))) return e;
    if (!out) return RS_ERR_INVALID_ARG;
    if (rays->n > 0 && (!grad_rgb || !ray_state || !aligned(ray_state, 16))) return RS_ERR_INVALID_ARG;
    if ((e = check_pool(rays->n, p, 1))) return e;
    return launch_render(D, g, rays, p, nullptr, const_cast<void *>(ray_state), grad_rgb, out,
                         static_cast<hipStream_t>(stream));
}

static int check_mesh(const rs_mesh *m)
{
    if (!m || m->n_tris < 0 || m->n_tris > 0x7ffffffeLL || m->n_verts < 0) return RS_ERR_INVALID_ARG;
    if (m->n_tris > 0 && (!m->verts || !m->tris || m->n_verts == 0)) return RS_ERR_INVALID_ARG;
    return RS_OK;
}

static int check_mesh_bvh(const rs_bvh *b, const rs_mesh *m, BvhDesc &D)
{
    if (!b) return RS_ERR_INVALID_ARG;
    memcpy(&D, b, sizeof(D));
    if (D.magic != kMagic || !D.ws || D.kind != kKindMesh) return RS_ERR_INVALID_ARG;
    if (m && D.n != m->n_tris) return RS_ERR_BVH_MISMATCH;
    return RS_OK;
}

static int check_shading(const rs_shading *sh)
{
    if (!sh) return RS_ERR_INVALID_ARG;
    const float v[9] = {sh->light[0], sh->light[1], sh->light[2], sh->intensity, sh->albedo, sh->mirror_reflectance,
                        sh->mirror_diffuse, sh->offset, sh->ior};
    for (float x : v)
        if (!(x == x) || x == __builtin_huge_valf() || x == -__builtin_huge_valf()) return RS_ERR_INVALID_ARG;
    if (sh->offset < 0.0f || sh->mirror_reflectance < 0.0f || sh->mirror_diffuse < 0.0f) return RS_ERR_INVALID_ARG;
    if (sh->max_bounces < 1 || sh->max_bounces > RS_MAX_BOUNCES || !(sh->ior > 0.0f)) return RS_ERR_INVALID_ARG;
    return RS_OK;
}

void rs_default_shading(rs_shading *s)
{
    if (!s) return;
    s->light[0] = 2.0f;
    s->light[1] = -2.0f;
    s->light[2] = 5.0f;
    s->intensity = 1.0f;
    s->albedo = 0.8f;
    s->mirror_reflectance = 0.8f;
    s->mirror_diffuse = 0.2f;
    s->offset = 1e-4f;
    s->max_bounces = 1;
    s->ior = 1.5f;
}

int rs_build_mesh_bvh(const rs_mesh *m, void *ws, size_t ws_bytes, rs_bvh *out, void *stream)
{
    int e = check_mesh(m);
    if (e) return e;
    if (!ws || !out || !aligned(ws, 256)) return RS_ERR_INVALID_ARG;
    if (ws_bytes < make_layout(m->n_tris).total) return RS_ERR_WORKSPACE;
    e = launch_build_mesh(m, static_cast<char *>(ws), static_cast<hipStream_t>(stream));
    if (e) return e;
    BvhDesc D{};
    D.magic = kMagic;
    D.n = m->n_tris;
    D.Q = 0.0f;
    D.root = m->n_tris >= 2 ? 0 : ~0;
    D.ws = static_cast<char *>(ws);
    D.ws_bytes = ws_bytes;
    D.kind = kKindMesh;
    memset(out, 0, sizeof(*out));
    memcpy(out, &D, sizeof(D));
    return RS_OK;
}

int rs_trace_mesh(const rs_bvh *mesh_bvh, const rs_rays *rays, const float *t_limit, int any_hit, float *t_hit,
                  int32_t *tri, void *stream)
{
    int e = check_rays(rays);
    if (e) return e;
    BvhDesc M;
    if ((e = check_mesh_bvh(mesh_bvh, nullptr, M))) return e;
    if (rays->n > 0 && (!t_hit || !tri)) return RS_ERR_INVALID_ARG;
    return launch_trace_mesh(M, rays, t_limit, any_hit ? 1 : 0, tile_shift_of(nullptr), t_hit, tri,
                             static_cast<hipStream_t>(stream));
}

size_t rs_mesh_frame_bytes(int64_t n_rays, const rs_params *p, const rs_shading *sh)
{
    const int b = sh && sh->max_bounces >= 1 && sh->max_bounces <= RS_MAX_BOUNCES ? sh->max_bounces : 1;
    return n_rays >= 0 ? mesh_frame_bytes(n_rays, p && p->hit_list > 0 ? p->hit_list : 0, b) : 0;
}

int rs_render_mesh_fwd(const rs_bvh *gauss_bvh, const rs_bvh *mesh_bvh, const rs_gaussians *g, const rs_mesh *m,
                       const rs_shading *sh, const rs_rays *rays, const rs_params *p, float *out_rgb, void *frame,
                       void *stream)
{
    int e = check_gaussians(g);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if ((e = check_rays(rays))) return e;
    if ((e = check_mesh(m))) return e;
    if ((e = check_shading(sh))) return e;
    if (rays->t_max || rays->bg || (p->flags & RS_PAPER_GRADIENT)) return RS_ERR_UNSUPPORTED;
    BvhDesc G, M;
    if ((e = check_bvh(gauss_bvh, g, p, G))) return e;
    if ((e = check_mesh_bvh(mesh_bvh, m, M))) return e;
    if (rays->n > 0 && (!out_rgb || !frame || !aligned(frame, 256))) return RS_ERR_INVALID_ARG;
    if ((e = check_pool(rays->n, p, 2 * sh->max_bounces + 1))) return e;
    return launch_mesh_fwd(G, M, g, sh, rays, p, out_rgb, frame, static_cast<hipStream_t>(stream));
}

int rs_render_mesh_bwd(const rs_bvh *gauss_bvh, const rs_bvh *mesh_bvh, const rs_gaussians *g, const rs_mesh *m,
                       const rs_shading *sh, const rs_rays *rays, const rs_params *p, const float *grad_rgb,
                       void *frame, rs_grads *out, void *stream)
{
    int e = check_gaussians(g);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if ((e = check_rays(rays))) return e;
    if ((e = check_mesh(m))) return e;
    if ((e = check_shading(sh))) return e;
    if (rays->t_max || rays->bg || (p->flags & RS_PAPER_GRADIENT)) return RS_ERR_UNSUPPORTED;
    BvhDesc G, M;
    if ((e = check_bvh(gauss_bvh, g, p, G))) return e;
    if ((e = check_mesh_bvh(mesh_bvh, m, M))) return e;
    if (!out) return RS_ERR_INVALID_ARG;
    if (rays->n > 0 && (!grad_rgb || !frame || !aligned(frame, 256))) return RS_ERR_INVALID_ARG;
    if ((e = check_pool(rays->n, p, 2 * sh->max_bounces + 1))) return e;
    return launch_mesh_bwd(G, g, sh, rays, p, grad_rgb, frame, out, static_cast<hipStream_t>(stream));
}

int rs_read_status(const rs_bvh *bvh, void *stream)
{
    if (!bvh) return RS_ERR_INVALID_ARG;
    BvhDesc D;
    memcpy(&D, bvh, sizeof(D));
    if (D.magic != kMagic || !D.ws) return RS_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(st) != hipSuccess) return RS_ERR_HIP;
    int32_t s = 0;
    Layout L = make_layout(D.n);
    if (hipMemcpy(&s, D.ws + L.header, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return RS_ERR_HIP;
    if (s & kStatusStack) return RS_ERR_STACK_OVERFLOW;
    if (s & kStatusNonfinite) return RS_ERR_NONFINITE;
    if (s & kStatusListPool) return RS_ERR_LIST_POOL;
    return RS_OK;
}

int rs_read_counters(const rs_bvh *bvh, uint64_t *out, void *stream)
{
    if (!bvh || !out) return RS_ERR_INVALID_ARG;
    BvhDesc D;
    memcpy(&D, bvh, sizeof(D));
    if (D.magic != kMagic || !D.ws) return RS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RS_ERR_HIP;
    WsHeader h;
    Layout L = make_layout(D.n);
    if (hipMemcpy(&h, D.ws + L.header, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return RS_ERR_HIP;
    for (int k = 0; k < 16; ++k) out[k] = h.counters[k];
    return RS_OK;
}

int rs_autotune(const rs_bvh *bvh, const rs_gaussians *g, const rs_rays *rays, const rs_params *base,
                const float *grad_rgb, float *out_rgb, void *ray_state, rs_grads *grads, int reps, rs_tune *result,
                void *stream)
{
    int e = check_gaussians(g);
    if (e) return e;
    if ((e = check_params(base))) return e;
    if ((e = check_rays(rays))) return e;
    BvhDesc D;
    if ((e = check_bvh(bvh, g, base, D))) return e;
    if (!result || reps < 1 || reps > 100) return RS_ERR_INVALID_ARG;
    if (rays->n > 0 && !out_rgb) return RS_ERR_INVALID_ARG;
    if (grad_rgb && (!ray_state || !grads)) return RS_ERR_INVALID_ARG;
    if (ray_state && !aligned(ray_state, 16)) return RS_ERR_INVALID_ARG;
    if ((e = check_pool(rays->n, base, 1))) return e;
    memset(result, 0, sizeof(*result));
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return RS_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return RS_ERR_HIP;
    }
    // mean ms of `reps` launches of f (after one untimed launch)
    auto timed = [&](auto &&f, float &ms) -> int {
        int r = f();
        if (r) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return RS_ERR_HIP;
        for (int k = 0; k < reps; ++k)
            if ((r = f())) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return RS_ERR_HIP;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return RS_ERR_HIP;
        ms /= float(reps);
        return RS_OK;
    };
    static const int kbufs[5] = {8, 16, 24, 32, 48};
    const int n_tiles = rays->n_views > 0 ? 2 : 1;
    int best_f = -1, best_b = -1;
    for (int ki = 0; ki < 5 && !e; ++ki) {
        for (int pers = 0; pers < 2 && !e; ++pers) {
            for (int ti = 0; ti < n_tiles && !e; ++ti) {
                const int c = result->n;
                rs_params p = *base;
                p.kbuf = kbufs[ki];
                p.flags = (base->flags & ~(RS_PERSISTENT | RS_COUNTERS)) | (pers ? RS_PERSISTENT : 0u);
                p.tile_width = ti == 0 ? 8 : 16;
                result->kbuf[c] = p.kbuf;
                result->persistent[c] = pers;
                result->tile_width[c] = p.tile_width;
                e = timed([&] { return launch_render(D, g, rays, &p, out_rgb, ray_state, nullptr, nullptr, st); },
                          result->ms_fwd[c]);
                if (!e && grad_rgb)
                    e = timed([&] { return launch_render(D, g, rays, &p, nullptr, ray_state, grad_rgb, grads, st); },
                              result->ms_bwd[c]);
                if (e) break;
                if (best_f < 0 || result->ms_fwd[c] < result->ms_fwd[best_f]) {
                    best_f = c;
                    result->fwd = p;
                }
                if (grad_rgb && (best_b < 0 || result->ms_bwd[c] < result->ms_bwd[best_b])) {
                    best_b = c;
                    result->bwd = p;
                }
                result->n = c + 1;
            }
        }
    }
    if (!grad_rgb) result->bwd = result->fwd;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

void rs_default_loss_params(rs_loss_params *lp)
{
    if (!lp) return;
    lp->lambda = 0.2f;
    lp->radius = 5;
    lp->sigma = 1.5f;
}

size_t rs_loss_workspace_bytes(int32_t width, int32_t height)
{
    return (width > 0 && height > 0) ? loss_workspace_bytes(width, height) : 0;
}

int rs_loss(const float *img, const float *target, int32_t width, int32_t height, const rs_loss_params *lp,
            float *loss, float *grad, void *ws, void *stream)
{
    if (!img || !target || !lp || !loss || !ws || width <= 0 || height <= 0) return RS_ERR_INVALID_ARG;
    if (!(lp->lambda >= 0.0f && lp->lambda <= 1.0f) || lp->radius < 1 || lp->radius > 7 || !(lp->sigma > 0.0f))
        return RS_ERR_INVALID_ARG;
    if (int64_t(width) * height > (int64_t(1) << 30)) return RS_ERR_UNSUPPORTED;
    if (!aligned(ws, 256)) return RS_ERR_INVALID_ARG;
    return launch_loss(img, target, width, height, lp, loss, grad, ws, static_cast<hipStream_t>(stream));
}

int rs_loss_noalloc(const float *img, const float *target, int32_t width, int32_t height, const rs_loss_params *lp,
                    float *loss, float *grad, void *stream)
{
    if (!img || !target || !lp || !loss || width <= 0 || height <= 0) return RS_ERR_INVALID_ARG;
    if (!(lp->lambda >= 0.0f && lp->lambda <= 1.0f) || lp->radius < 1 || lp->radius > 7 || !(lp->sigma > 0.0f))
        return RS_ERR_INVALID_ARG;
    if (int64_t(width) * height > (int64_t(1) << 30)) return RS_ERR_UNSUPPORTED;
    if (loss_workspace_bytes(width, height) > loss_scratch_bytes()) return RS_ERR_UNSUPPORTED;
    void *ws = nullptr;
    const int e = loss_scratch(&ws);
    if (e) return e;
    return launch_loss(img, target, width, height, lp, loss, grad, ws, static_cast<hipStream_t>(stream));
}

size_t rs_loss_noalloc_max_bytes(void) { return loss_scratch_bytes(); }

const char *rs_status_string(int code)
{
    switch (code) {
    case RS_OK: return "ok";
    case RS_ERR_INVALID_ARG: return "invalid argument";
    case RS_ERR_WORKSPACE: return "workspace too small";
    case RS_ERR_HIP: return "HIP runtime error";
    case RS_ERR_BVH_MISMATCH: return "BVH built for a different scene size or Q";
    case RS_ERR_STACK_OVERFLOW: return "traversal stack overflow";
    case RS_ERR_NONFINITE: return "non-finite or out-of-range Gaussian parameter";
    case RS_ERR_UNSUPPORTED: return "unsupported configuration";
    case RS_ERR_LIST_POOL: return "stored hit-list pool exhausted (paper gradient variant)";
    default: return "unknown status";
    }
}

int rs_bvh_download(const rs_bvh *bvh, uint32_t *codes, int32_t *perm, int32_t *child, float *boxes,
                    float *leaf_boxes, float *bounds, void *stream)
{
    if (!bvh) return RS_ERR_INVALID_ARG;
    BvhDesc D;
    memcpy(&D, bvh, sizeof(D));
    if (D.magic != kMagic || !D.ws) return RS_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(st) != hipSuccess) return RS_ERR_HIP;
    Layout L = make_layout(D.n);
    const int64_t n = D.n, ni = L.n_int;
    auto cp = [&](void *dst, size_t off, size_t bytes) {
        return (!dst || bytes == 0) ? hipSuccess : hipMemcpy(dst, D.ws + off, bytes, hipMemcpyDeviceToHost);
    };
    if (cp(codes, L.codes, size_t(n) * 4) != hipSuccess) return RS_ERR_HIP;
    if (cp(perm, L.gidx, size_t(n) * 4) != hipSuccess) return RS_ERR_HIP;
    if (cp(leaf_boxes, L.leaf_boxes, size_t(n) * 24) != hipSuccess) return RS_ERR_HIP;
    if (bounds) {
        WsHeader h;
        if (hipMemcpy(&h, D.ws + L.header, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return RS_ERR_HIP;
        for (int k = 0; k < 6; ++k) {
            uint32_t u = h.bounds[k];
            uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
            memcpy(&bounds[k], &b, 4);
        }
    }
    if ((child || boxes) && ni > 0) {
        float *tmp = new float[size_t(ni) * 16];
        if (hipMemcpy(tmp, D.ws + L.nodes, size_t(ni) * 64, hipMemcpyDeviceToHost) != hipSuccess) {
            delete[] tmp;
            return RS_ERR_HIP;
        }
        for (int64_t i = 0; i < ni; ++i) {
            if (child) {
                memcpy(&child[2 * i], &tmp[16 * i + 12], 4);
                memcpy(&child[2 * i + 1], &tmp[16 * i + 13], 4);
            }
            if (boxes)
                for (int k = 0; k < 12; ++k) boxes[12 * i + k] = tmp[16 * i + k];
        }
        delete[] tmp;
    }
    return RS_OK;
}

// Lane of ray r inside its 64-ray packet (the tile layout of rs_render_fwd).
static int ray_lane(const rs_rays *rays, int tile_shift, int64_t r)
{
    if (rays->n_views == 0) return int(r % kWave);
    for (int v = 0; v < rays->n_views; ++v) {
        const rs_view &V = rays->views[v];
        const int64_t local = r - V.ray_offset;
        if (local < 0 || local >= int64_t(V.width) * V.height) continue;
        const int64_t y = local / V.width, x = local - y * V.width;
        const int tw = 1 << tile_shift, th = kWave >> tile_shift;
        return int((y % th) * tw + (x % tw));
    }
    return 0;
}

// Host copies of stored lists (the list bookkeeping of a ray set and its pool).
static int lists_download(const rs_rays *rays, int tile_shift, const int4 *dev_list, const ListPool &P,
                          const int64_t *sel, int64_t n_sel, int32_t *count, int32_t *stored, int32_t *extra,
                          int32_t *ids, int32_t cap)
{
    const int64_t n = rays->n;
    const int64_t m = sel ? n_sel : n;
    if (m <= 0 || n == 0) return RS_OK;
    if (sel)
        for (int64_t i = 0; i < m; ++i)
            if (sel[i] < 0 || sel[i] >= n) return RS_ERR_INVALID_ARG;
    std::vector<int4> li(static_cast<size_t>(n));
    if (hipMemcpy(li.data(), dev_list, size_t(n) * 16, hipMemcpyDeviceToHost) != hipSuccess) return RS_ERR_HIP;
    unsigned long long taken = 0;
    if (hipMemcpy(&taken, P.hdr, 8, hipMemcpyDeviceToHost) != hipSuccess) return RS_ERR_HIP;
    const int64_t used = int64_t(taken < (unsigned long long)P.chunks ? taken : (unsigned long long)P.chunks);
    std::vector<int32_t> prev(size_t(used > 0 ? used : 1)), fill(size_t(used > 0 ? used : 1));
    std::vector<uint32_t> slots(size_t(used > 0 ? used : 1) * kChunkSlots);
    if (used > 0) {
        if (hipMemcpy(prev.data(), P.prev, size_t(used) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(fill.data(), P.fill, size_t(used) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(slots.data(), P.slots, size_t(used) * kChunkSlots * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return RS_ERR_HIP;
    }
    // a packet's rows, first to last: (first slot, lane mask); a chunk's rows are found
    // from its fill backwards, each row ending with its mask
    std::unordered_map<int32_t, std::vector<std::pair<int64_t, uint64_t>>> chains;
    for (int64_t i = 0; i < m; ++i) {
        const int64_t r = sel ? sel[i] : i;
        const int4 L = li[size_t(r)];
        if (count) count[i] = L.x;
        if (stored) stored[i] = L.y;
        int32_t x = 0, w = 0;
        if (L.w > 0 && L.z >= 0 && L.z < used) {
            auto it = chains.find(L.z);
            if (it == chains.end()) {
                std::vector<std::pair<int64_t, uint64_t>> rows;  // last to first
                int64_t hops = 0;
                for (int32_t c = L.z; c >= 0 && c < used && hops <= used; c = prev[size_t(c)], ++hops) {
                    int32_t end = fill[size_t(c)];
                    if (end < 0 || end > kChunkSlots) break;
                    while (end >= 2) {
                        const size_t at = size_t(c) * kChunkSlots + size_t(end);
                        const uint64_t mask = uint64_t(slots[at - 2]) | (uint64_t(slots[at - 1]) << 32);
                        const int32_t k = __builtin_popcountll(mask);
                        if (k + 2 > end) break;
                        end -= k + 2;
                        rows.emplace_back(int64_t(c) * kChunkSlots + end, mask);
                    }
                }
                std::reverse(rows.begin(), rows.end());
                it = chains.emplace(L.z, std::move(rows)).first;
            }
            const int lane = ray_lane(rays, tile_shift, r);
            for (const auto &row : it->second) {
                if (!((row.second >> lane) & 1ull)) continue;
                const uint64_t below = lane ? row.second & ((1ull << lane) - 1ull) : 0ull;
                const uint32_t v = slots[size_t(row.first) + size_t(__builtin_popcountll(below))];
                if (v & kListSecond) ++x;
                if (ids && w < cap) ids[i * int64_t(cap) + w] = int32_t(v & ~kListSecond);
                ++w;
            }
        }
        if (ids)
            for (int32_t k = w; k < cap; ++k) ids[i * int64_t(cap) + k] = -1;
        if (extra) extra[i] = x;
    }
    return RS_OK;
}

int rs_hit_lists_download(const rs_rays *rays, const rs_params *p, const void *ray_state, const int64_t *rays_sel,
                          int64_t n_sel, int32_t *count, int32_t *stored, int32_t *extra, int32_t *ids, int32_t cap,
                          void *stream)
{
    int e = check_rays(rays);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if (!ray_state || p->hit_list <= 0 || cap < 0 || (ids && cap == 0) || (rays_sel && n_sel < 0))
        return RS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RS_ERR_HIP;
    if (rays->n == 0) return RS_OK;
    const StateLayout SL = state_layout(rays->n, p->hit_list);
    char *base = const_cast<char *>(static_cast<const char *>(ray_state));
    return lists_download(rays, tile_shift_of(p), reinterpret_cast<const int4 *>(base + SL.list),
                          list_pool_at(base + SL.pool, SL.chunks), rays_sel, n_sel, count, stored, extra, ids, cap);
}

int rs_mesh_hit_lists_download(const rs_rays *rays, const rs_params *p, const rs_shading *sh, const void *frame,
                               int32_t set, const int64_t *rays_sel, int64_t n_sel, int32_t *count, int32_t *stored,
                               int32_t *ids, int32_t cap, void *stream)
{
    int e = check_rays(rays);
    if (e) return e;
    if ((e = check_params(p))) return e;
    if ((e = check_shading(sh))) return e;
    if (!frame || p->hit_list <= 0 || cap < 0 || (ids && cap == 0) || (rays_sel && n_sel < 0))
        return RS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RS_ERR_HIP;
    if (rays->n == 0) return RS_OK;
    SetState st;
    ListPool pool;
    if ((e = mesh_frame_set(const_cast<char *>(static_cast<const char *>(frame)), rays->n, p->hit_list,
                            sh->max_bounces, set, &st, &pool)))
        return e;
    return lists_download(rays, tile_shift_of(p), st.list, pool, rays_sel, n_sel, count, stored, nullptr, ids, cap);
}

}  // extern "C"
