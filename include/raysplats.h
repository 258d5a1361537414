/*
 * raysplats.h -- C ABI of the MI355X ray-traced Gaussian renderer.
 *
 * The library renders a scene of 3D (or flat) Gaussians by ray tracing, as in
 * RaySplats (arXiv 2501.19196), and computes the adjoint of that rendering:
 *
 *   scene (Eq. 1-2)  G = {(N(m_i, Sigma_i), opacity_i, c_i)}, Sigma = R S S^T R^T,
 *                    R from the quaternion q_i (App. A.6), S = diag(s_i)
 *   hit (Sec. 3, Prop. 1)  ray r(t) = o + t d meets the confidence ellipsoid
 *                    (x-m)^T Sigma^-1 (x-m) = Q; the hit depth is the nearer
 *                    root t1; a ray misses when the line misses or t1 < t_min
 *   alpha (Prop. 2)  alpha_i = opacity_i * exp(-h_i^2 / 2), h_i^2 the squared
 *                    whitened distance between the line and the Gaussian centre
 *   colour (Eq. 3)   hits sorted by (t1, Gaussian index) are composited front to
 *                    back, C += T alpha c, T *= (1 - alpha); a ray stops after
 *                    K_max hits or once T < eps1 (Sec. 3, "Color Aggregation");
 *                    the output is C + T * background
 *   adjoint (App. A.3-A.6)  gradients of sum_k <grad_rgb_k, C_k> with respect
 *                    to every Gaussian parameter
 *
 * Conventions
 *  - Plain C, no HIP or torch types. Every pointer documented as "device" is a
 *    device (HBM) address; "host" pointers are read synchronously during the
 *    call. `stream` is a hipStream_t passed as void* (NULL = default stream).
 *  - The caller owns every buffer, including the BVH workspace and the ray
 *    state. The library keeps no per-call global state and never allocates
 *    device memory.
 *  - All calls are asynchronous on `stream`; argument validation is
 *    synchronous and returns a negative status before anything is enqueued.
 *  - Device-side faults (traversal stack overflow, non-finite inputs) are
 *    recorded in a sticky status word inside the BVH workspace; read it with
 *    rs_read_status.
 *  - Parameters are the activated values: world-space scales (> 0), opacity
 *    in [0, 1], raw quaternions (r, i, j, k), nonzero, not necessarily unit.
 *    Gradients are with respect to these same values.
 */
#ifndef RAYSPLATS_H
#define RAYSPLATS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
    RS_OK = 0,
    RS_ERR_INVALID_ARG = -1,     /* a null pointer, negative size, bad flag or knob */
    RS_ERR_WORKSPACE = -2,       /* workspace smaller than rs_bvh_workspace_bytes */
    RS_ERR_HIP = -3,             /* a HIP runtime call failed (launch, copy) */
    RS_ERR_BVH_MISMATCH = -4,    /* BVH built for another scene size or Q */
    RS_ERR_STACK_OVERFLOW = -5,  /* device: traversal stack deeper than stack_depth */
    RS_ERR_NONFINITE = -6,       /* device: a non-finite or out-of-range Gaussian parameter */
    RS_ERR_UNSUPPORTED = -7,     /* valid but unsupported combination (e.g. too many views) */
    RS_ERR_LIST_POOL = -8        /* device: the paper variant's stored-list pool ran out */
};

/* ------------------------------------------------------------------- flags */
#define RS_BRUTE_FORCE  (1u << 0)  /* test every Gaussian against every ray (no BVH pruning) */
#define RS_PERSISTENT   (1u << 1)  /* persistent launch: waves pop ray packets from a queue */
#define RS_ZERO_COLOUR  (1u << 2)  /* take every Gaussian colour as 0: output = T * background
                                      (transmittance / shadow rays) */
#define RS_COUNTERS     (1u << 3)  /* count traversal work (see rs_read_counters; not with
                                      RS_BRUTE_FORCE); an instrumented kernel variant */
#define RS_PAPER_GRADIENT (1u << 4) /* the paper's backward variant (Sec. 3, Sec. 5): after an
                                      eps1 stop the forward keeps the ids of the next hits
                                      while their transmittance stays >= eps2 (image unchanged),
                                      and the last composited Gaussian's gradient sees them
                                      instead of the background. Needs 0 < max_hits and
                                      hit_list > 0; with full 64-ray packets a pool of
                                      5/4 max_hits + 8 slots per ray never runs out
                                      (RS_ERR_LIST_POOL otherwise; a packet of r rays
                                      stores at most (r + 2) max_hits slots).
                                      Not for the mesh renders. */

#define RS_BUILD_LBVH   (1u << 5)  /* rs_build_bvh: link the Morton-sorted leaves as a binary radix
                                      tree (Karras) instead of clustering them (PLOC, the default);
                                      faster to build, about 1.6x the traversal work */

#define RS_MAX_VIEWS 64

/* Gaussian scene, structure of arrays, all device pointers, float32,
 * row-major: mean[n][3], scale[n][3] (> 0), quat[n][4] (r, i, j, k),
 * opacity[n] (in [0, 1]), rgb[n][3]. n <= 2^31 - 2. Read only. */
typedef struct {
    int64_t n;
    const float *mean, *scale, *quat, *opacity, *rgb;
} rs_gaussians;

/* One camera's rays inside the ray array: rays [ray_offset, ray_offset + width*height)
 * are an image of `width` x `height` pixels in row-major order. The renderer
 * groups rays into 64-pixel tiles (one wavefront each; 8x8 unless
 * rs_params.tile_width says otherwise) for coherence. */
typedef struct {
    int64_t ray_offset;
    int32_t width, height;
} rs_view;

/* Rays r(t) = o + t d (device pointers, float32 [n][3]; d nonzero, need not be unit).
 *  t_max  optional device [n]: a hit needs t1 < t_max[k] (NULL = +inf)
 *  bg     optional device [n][3]: per-ray background (NULL = params->bg)
 *  views  optional host table of n_views <= RS_MAX_VIEWS images tiling the rays
 *         in order; n_views = 0 groups consecutive rays 64 at a time. */
typedef struct {
    int64_t n;
    const float *origin, *dir;
    const float *t_max;
    const float *bg;
    int32_t n_views;
    const rs_view *views;
} rs_rays;

/* Renderer knobs. Q: ellipsoid quantile (Sec. 3; > 0). eps1: transmittance
 * threshold (>= 0). t_min: minimum hit depth (finite, >= 0). max_hits: K_max (0 = unbounded).
 * kbuf: hits gathered per ray per traversal round (8, 16, 24, 32 or 48; 0 = 48,
 * the size rs_autotune picks for the forward on every measured workload; the
 * result does not depend on it).
 * stack_depth: traversal stack entries (1..64; 0 = 64). tile_width: width in
 * pixels of the 64-ray packet tile of a view (4, 8, 16 or 32, i.e. 4x16, 8x8,
 * 16x4 or 32x2 pixels; 0 = 8); like kbuf it changes the time, not the result.
 * hit_list: store-or-recompute choice of the adjoint (0..4096; 0 = recompute):
 * with C > 0 the forward also records the ids of the Gaussians each ray
 * composites, in a pool of C 4-byte slots per ray on average inside the ray
 * state (per compositing step of its wavefront a packet of 64 rays stores one
 * row: the ids of the lanes that took a hit at that step and their 64-bit lane
 * mask, in chunks of 512 slots), and the adjoint replays those lists
 * instead of traversing the BVH again. The rays of a packet that finds the pool
 * exhausted are traversed again by the adjoint. The gradients are the same (up to
 * float atomic order). The mesh renders keep one pool for all their ray sets in
 * the frame. */
typedef struct {
    float Q, eps1, t_min;
    int32_t max_hits;
    float bg[3];
    uint32_t flags;
    int32_t kbuf;
    int32_t stack_depth;
    int32_t tile_width;
    int32_t hit_list;
    float eps2;  /* second threshold of RS_PAPER_GRADIENT, in [0, 1] */
} rs_params;

/* Gradient outputs (device, float32, same shapes as the inputs). Any pointer
 * may be NULL to skip that group. Overwritten (the library zeroes them first). */
typedef struct {
    float *d_mean, *d_scale, *d_quat, *d_opacity, *d_rgb;
} rs_grads;

/* BVH descriptor: plain data naming sections of the caller's workspace. */
typedef struct {
    uint64_t opaque[16];
} rs_bvh;

/* Fill *p with the defaults: Q = 11.3449 (chi^2(3) 0.99 quantile), eps1 = 1e-4,
 * t_min = 0, max_hits = 512, black background, no flags, automatic kbuf,
 * stack depth and packet size, no hit lists, eps2 = 1e-4. */
void rs_default_params(rs_params *p);

/* Device workspace needed to build and keep a BVH over n Gaussians. */
size_t rs_bvh_workspace_bytes(int64_t n_gaussians);

/* Per-ray state written by rs_render_fwd and read by rs_render_bwd (p may be
 * NULL: C = 0). Its first 16 n bytes are float32 [n][4]: the final colour
 * (composite + T background) and the final transmittance T of each ray. Then
 * 16 bytes per ray that the adjoint starts from (the last composited hit and
 * where T reached 0) and, when p->hit_list = C > 0, 16 bytes of list
 * bookkeeping per ray plus the stored-list pool (C slots of 4 bytes per ray on
 * average, in whole chunks of 2 KiB, after a 256-byte header). */
size_t rs_ray_state_bytes(int64_t n_rays, const rs_params *p);

/* Build the BVH: 30-bit Morton codes of the means, LDS radix sort, leaf boxes
 * of the confidence ellipsoids, then PLOC (locally-ordered agglomerative
 * clustering of the sorted leaves by the surface area of merged boxes,
 * neighbourhood radius 8; deterministic) or, with RS_BUILD_LBVH in p->flags,
 * Karras radix-tree linking plus a bottom-up box refit. The paper traverses
 * with a vendor ray-tracing API (Sec. 5); this structure replaces it. Both
 * trees give identical renders; PLOC trees cut traversal work.
 *  g        scene (device arrays)
 *  p        knobs; Q fixes the ellipsoid size the boxes bound
 *  ws       device workspace of ws_bytes >= rs_bvh_workspace_bytes(g->n),
 *           256-byte aligned; owned by the caller, must outlive every render
 *           that uses *out
 *  out      descriptor (host) to pass to the render calls
 * Also resets the sticky status word. Returns RS_OK or a negative status. */
int rs_build_bvh(const rs_gaussians *g, const rs_params *p, void *ws, size_t ws_bytes, rs_bvh *out,
                 void *stream);

/* Forward render (Sec. 3 "Color Aggregation", Eq. 3, Props. 1-2).
 *  bvh        from rs_build_bvh over the same scene size and Q
 *  out_rgb    device float32 [rays->n][3], written
 *  ray_state  device buffer of rs_ray_state_bytes(rays->n, p) bytes, 16-byte
 *             aligned, written; needed by rs_render_bwd (may be NULL when no
 *             backward pass follows). The caller must pass a buffer of that
 *             size: the call takes no size. */
int rs_render_fwd(const rs_bvh *bvh, const rs_gaussians *g, const rs_rays *rays, const rs_params *p,
                  float *out_rgb, void *ray_state, void *stream);

/* Adjoint render (App. A.3-A.6): walks each ray's composited hits back to
 * front, from its stored hit list (p->hit_list > 0) or by traversing the BVH
 * again from the last composited hit, builds the colour S_{k+1} seen behind
 * each hit from the background forward (dL/dalpha_k = T_k <g, c_k - S_{k+1}>,
 * no division by 1 - alpha_k), and accumulates d/dtheta sum_k <grad_rgb[k], C_k>
 * into `out` with float32 atomics, aggregated per wave by Gaussian. Must use the
 * same bvh, scene, rays and params (hit_list included) as the forward call that
 * wrote ray_state. grad_rgb: device float32 [rays->n][3]. */
int rs_render_bwd(const rs_bvh *bvh, const rs_gaussians *g, const rs_rays *rays, const rs_params *p,
                  const float *grad_rgb, const void *ray_state, rs_grads *out, void *stream);

/* Synchronise `stream` and return the sticky device status of this BVH's
 * workspace (RS_OK, RS_ERR_STACK_OVERFLOW, RS_ERR_NONFINITE or
 * RS_ERR_LIST_POOL): what the last rs_build_bvh found in the inputs and what
 * every render and adjoint call since then found (a build clears it). */
int rs_read_status(const rs_bvh *bvh, void *stream);

/* Synchronise `stream` and copy the work counters accumulated by render calls
 * made with RS_COUNTERS since the last rs_build_bvh (host uint64 out[16]):
 * [0] forward ray packets, [1] inner-node visits, [2] leaf visits, [3]
 * traversal rounds (all per wavefront), [4] lane leaf tests on live rays, [5]
 * hits entering a lane's buffer, [6] forward: hits consumed (composited, or
 * collected by the paper variant), traversal adjoint: hits differentiated, [7]
 * lane child-box overlaps, [8] traversal adjoint: accumulator lines flushed
 * from its LDS tables, stored-list adjoint: [9] ray packets, [10]
 * differentiated hits, [11] gradient groups (distinct Gaussians per step);
 * [12] stored-list rows the forward stored, [13] traversal adjoint packets,
 * [14] stored-list slots the forward stored (ids and lane masks), [15] unused.
 * Instrumentation for tuning and roofline accounting; not part of the method. */
int rs_read_counters(const rs_bvh *bvh, uint64_t *out, void *stream);

/* ------------------------------------------------------------- autotuning */
/* Tuning helper, not part of the method: the launch shape (hit-buffer size
 * kbuf, plain or persistent grid, packet tile width) changes the time of a
 * render, never a rendered value (nor a gradient beyond float atomic order). */
#define RS_TUNE_MAX 32
typedef struct {
    rs_params fwd;  /* fastest forward configuration (a copy of *base with the knobs set) */
    rs_params bwd;  /* fastest adjoint configuration (= fwd when grad_rgb is NULL) */
    int32_t n;      /* candidates timed */
    int32_t kbuf[RS_TUNE_MAX], persistent[RS_TUNE_MAX], tile_width[RS_TUNE_MAX];
    float ms_fwd[RS_TUNE_MAX], ms_bwd[RS_TUNE_MAX]; /* mean ms per launch (bwd 0 without grad_rgb) */
} rs_tune;

/* Times every candidate on the caller's own BVH, Gaussians and rays: kbuf in
 * {8, 16, 24, 32, 48} x {one workgroup per packet, persistent queue} x tile width
 * {8, 16} (8x8 / 16x4 pixels; only 8 when the rays carry no views). Each runs
 * once untimed, then `reps` (1..100) times between hipEvents on `stream`.
 * grad_rgb (device [n][3], optional) also times the adjoint, which then
 * needs ray_state and grads; out_rgb, ray_state and grads receive the
 * results of the last candidate run. Host-synchronous (waits for `stream`).
 * Returns the first error of any launch. */
int rs_autotune(const rs_bvh *bvh, const rs_gaussians *g, const rs_rays *rays, const rs_params *base,
                const float *grad_rgb, float *out_rgb, void *ray_state, rs_grads *grads, int reps,
                rs_tune *result, void *stream);

/* ------------------------------------------------------ mesh + Gaussians */
/* The paper combines triangle meshes with Gaussians for mirror reflections,
 * shadows and glass (Sec. 1, Figs. 1 and 3-6) without giving a shading model.
 * This library implements the following one. A pixel follows a chain of up
 * to B + 1 path rays, B = max_bounces (1..RS_MAX_BOUNCES); path ray 0 is the
 * camera ray. Path ray k (origin o, unit direction d):
 *   closest triangle hit t_k (Moller-Trumbore, both faces, t > 0); the
 *     Gaussians with t1 < t_k composite to (C_k, T_k) over black when it hits
 *     a triangle, over bg when it hits none.
 *   at a hit P with k < B, unit geometric normal n_g (e1 x e2 of the vertex
 *   order), n = n_g turned to face the ray, unit light direction l:
 *     diffuse (material 0): diffuse weight 1, no continuation;
 *     mirror (1): diffuse weight mirror_diffuse; continuation from
 *       P + offset*n along d - 2 (d.n) n with weight mirror_reflectance;
 *     glass (2): no diffuse term; eta = 1/ior entering (d.n_g < 0), ior
 *       leaving; cos_i = -d.n, k = 1 - eta^2 (1 - cos_i^2); k < 0: total
 *       internal reflection (from P + offset*n, weight 1), else refraction
 *       from P - offset*n along eta d + (eta cos_i - sqrt(k)) n with weight
 *       1 - F, F = R0 + (1 - R0)(1 - c)^5 (Schlick), R0 = ((1-ior)/(1+ior))^2,
 *       c = cos_i entering, sqrt(k) leaving; the reflected part is not traced.
 *   shadow ray from P + offset*n to the light (diffuse weight > 0, n.l > 0):
 *     0 if a triangle blocks it, else the Gaussians' transmittance T_s.
 *   R_k = C_k + T_k (w_d albedo max(0, n.l) intensity T_s + w R_{k+1}) at a
 *   hit with k < B, R_k = C_k otherwise (a hit of path ray B is black);
 *   pixel = R_0. B = 1 gives primary, mirror reflection and shadow rays.
 * Material codes outside 0..2 shade as diffuse. Spawned rays are float32.
 * The K_max / eps1 rules apply to every ray. Gradients flow through the
 * Gaussian hits of every ray. */
#define RS_MAX_BOUNCES 3
typedef struct {
    int64_t n_verts, n_tris;
    const float *verts;      /* device [n_verts][3] */
    const int32_t *tris;     /* device [n_tris][3] vertex indices (out-of-range indices
                                set RS_ERR_NONFINITE and read vertex 0) */
    const int32_t *material; /* device [n_tris]: 0 diffuse, 1 mirror, 2 glass; NULL = all diffuse */
} rs_mesh;

typedef struct {
    float light[3];           /* point light position */
    float intensity, albedo;  /* light intensity, grey diffuse albedo */
    float mirror_reflectance; /* reflection weight of mirror triangles */
    float mirror_diffuse;     /* diffuse weight of mirror triangles */
    float offset;             /* secondary-ray origin offset along the normal */
    int32_t max_bounces;      /* B: specular continuations along a pixel's chain, 1..RS_MAX_BOUNCES */
    float ior;                /* index of refraction of glass triangles, > 0 */
} rs_shading;

/* light (2,-2,5), intensity 1, albedo 0.8, mirror weights 0.8 / 0.2, offset
 * 1e-4, one bounce, ior 1.5 */
void rs_default_shading(rs_shading *s);

/* Build a triangle BVH (the PLOC builder over triangle centroids) in a
 * caller workspace of rs_bvh_workspace_bytes(m->n_tris) bytes. */
int rs_build_mesh_bvh(const rs_mesh *m, void *ws, size_t ws_bytes, rs_bvh *out, void *stream);

/* Closest (any_hit = 0) or any (any_hit = 1) triangle hit per ray with
 * 0 < t < t_limit[k] (t_limit NULL = +inf; rays with t_limit <= 0 are
 * skipped). Writes t_hit[k] (+inf when none) and tri[k] (-1 when none),
 * device arrays of rays->n entries. */
int rs_trace_mesh(const rs_bvh *mesh_bvh, const rs_rays *rays, const float *t_limit, int any_hit, float *t_hit,
                  int32_t *tri, void *stream);

/* Per-frame device scratch of the mesh render for n rays (the path and shadow
 * rays of every level, their states, the terms the adjoint needs and, with
 * p->hit_list = C > 0, one stored-list pool for the 2B + 1 ray sets of
 * (2B + 1) C slots of 4 bytes per ray), 256-byte aligned. p may be NULL
 * (C = 0); sh may be NULL (B = 1). */
size_t rs_mesh_frame_bytes(int64_t n_rays, const rs_params *p, const rs_shading *sh);

/* Forward render of Gaussians + mesh with path and shadow rays. After the
 * triangle traces of every level, the Gaussians along all path and shadow
 * rays of all pixels are rendered in one persistent launch (2B + 1 ray sets,
 * one packet queue). `frame` (rs_mesh_frame_bytes(n, p, sh)) must be kept for
 * rs_render_mesh_bwd. */
int rs_render_mesh_fwd(const rs_bvh *gauss_bvh, const rs_bvh *mesh_bvh, const rs_gaussians *g, const rs_mesh *m,
                       const rs_shading *sh, const rs_rays *rays, const rs_params *p, float *out_rgb, void *frame,
                       void *stream);

/* Adjoint of rs_render_mesh_fwd with respect to the Gaussian parameters
 * (the mesh and the light carry no gradient). Overwrites `out`. Needs the
 * frame of the forward call, made with the same params (hit_list included). */
int rs_render_mesh_bwd(const rs_bvh *gauss_bvh, const rs_bvh *mesh_bvh, const rs_gaussians *g, const rs_mesh *m,
                       const rs_shading *sh, const rs_rays *rays, const rs_params *p, const float *grad_rgb,
                       void *frame, rs_grads *out, void *stream);

/* --------------------------------------------------------- training loss */
/* The paper's training loss (Sec. 3, loss function) of one image against its
 * target, and its gradient (App. A.7). Per colour channel
 *   L_ch = (1 - lambda) mean (I - I^)^2 + lambda (1 - mean SSIM) / 2,
 * and L is the mean over the three channels. SSIM uses the moments of a
 * normalised Gaussian window (zero outside the image) with c1 = 0.01^2,
 * c2 = 0.03^2 for intensities in [0, 1]; the gradient of mean SSIM is
 * App. A.7's (1/hw) ((E * w) + I^ (F * w) - I (G * w)). The paper gives no
 * window or lambda: the defaults are the usual 11 x 11 window (radius 5,
 * sigma 1.5) and lambda = 0.2. */
typedef struct {
    float lambda;   /* D-SSIM weight in [0, 1] */
    int32_t radius; /* window radius, 1..7 */
    float sigma;    /* window standard deviation, > 0 */
} rs_loss_params;

void rs_default_loss_params(rs_loss_params *lp);

/* Device workspace of rs_loss for a width x height image (E, F, G maps and
 * per-tile partial sums), 256-byte aligned. */
size_t rs_loss_workspace_bytes(int32_t width, int32_t height);

/* img, target: device float32 [height][width][3] (row-major pixels, the
 * order of a view's rays). loss: device float32 [1], written. grad: device
 * float32 [height][width][3], written with dL/dimg (NULL: loss only).
 * ws: rs_loss_workspace_bytes(width, height) bytes, 256-byte aligned.
 * Asynchronous on `stream`; errors for null pointers, empty images or bad
 * knobs are returned before anything is enqueued. */
int rs_loss(const float *img, const float *target, int32_t width, int32_t height, const rs_loss_params *lp,
            float *loss, float *grad, void *ws, void *stream);

/* rs_loss without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). The E, F, G maps and partial sums live in a
 * library-owned device array of rs_loss_noalloc_max_bytes() bytes (96 MiB),
 * which every GPU the library runs on holds until the process ends; images
 * whose rs_loss_workspace_bytes exceeds it return RS_ERR_UNSUPPORTED before
 * anything is enqueued. Allocates nothing. All calls on one GPU share that
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race. Results equal rs_loss's. */
int rs_loss_noalloc(const float *img, const float *target, int32_t width, int32_t height, const rs_loss_params *lp,
                    float *loss, float *grad, void *stream);
size_t rs_loss_noalloc_max_bytes(void);

/* Human-readable text of a status code (static string). */
const char *rs_status_string(int code);

/* Copy the stored hit lists of a ray state written by rs_render_fwd (with the
 * same rays and params, p->hit_list > 0) to host memory; synchronises
 * `stream`. Inspection helper for tests and tools, not part of the method.
 *  rays_sel   host int64 [n_sel] ray indices to copy (NULL: every ray, n_sel ignored)
 *  count      [m] hits each ray composited (m = n_sel, or rays->n)
 *  stored     [m] how many of them its list holds (fewer when the pool ran out)
 *  extra      [m] ids the paper variant collected after the eps1 stop, else 0
 *  ids        [m][cap]: per ray its stored ids in compositing order, then the
 *             collected ones; -1 after the last (entries beyond cap dropped)
 * Any output pointer may be NULL (ids needs cap > 0). */
int rs_hit_lists_download(const rs_rays *rays, const rs_params *p, const void *ray_state, const int64_t *rays_sel,
                          int64_t n_sel, int32_t *count, int32_t *stored, int32_t *extra, int32_t *ids, int32_t cap,
                          void *stream);

/* The same for ray set `set` of a mesh frame written by rs_render_mesh_fwd
 * (same rays, params and shading, p->hit_list > 0): sets 0..B are the path
 * rays of levels 0..B (0: the camera rays), sets B+1..2B the shadow rays of
 * levels 0..B-1, B = sh->max_bounces. Rays of a set that were not spawned
 * composite nothing. */
int rs_mesh_hit_lists_download(const rs_rays *rays, const rs_params *p, const rs_shading *sh, const void *frame,
                               int32_t set, const int64_t *rays_sel, int64_t n_sel, int32_t *count, int32_t *stored,
                               int32_t *ids, int32_t cap, void *stream);

/* Copy the built BVH to host memory for inspection (synchronises `stream`).
 * Any pointer may be NULL. codes[n] (uint32, sorted Morton codes),
 * perm[n] (int32, sorted position -> Gaussian index),
 * child[n-1][2] (int32; >= 0 internal node, < 0 leaf ~position),
 * boxes[n-1][2][6] (float32 child boxes lo.xyz, hi.xyz),
 * leaf_boxes[n][6], bounds[6] (scene box of the means). */
int rs_bvh_download(const rs_bvh *bvh, uint32_t *codes, int32_t *perm, int32_t *child, float *boxes,
                    float *leaf_boxes, float *bounds, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAYSPLATS_H */
