// Internal declarations of the MI355X renderer: workspace layout, the BVH
// descriptor, record layouts and small device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raysplats.h"

namespace rs {

constexpr uint64_t kMagic = 0x5253425648495031ull;  // "RSBVHIP1"
constexpr int kWave = 64;
constexpr int kMaxSets = 2 * RS_MAX_BOUNCES + 1;  // ray sets one render launch can carry (mesh path + shadow rays)
constexpr int kXcdQueues = 8;  // persistent packet queues (one per XCD of MI355X)
constexpr int kStripTiles = 16;  // persistent packet order: strips 16 tiles wide

// log2 of the packet tile width of a launch (tile_width 0 = 8x8 tiles)
inline int tile_shift_of(const rs_params *p)
{
    switch (p ? p->tile_width : 0) {
    case 4: return 2;
    case 16: return 4;
    case 32: return 5;
    default: return 3;
    }
}
constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;  // keys per thread per sort tile
constexpr int kSortTile = kSortBlock * kSortItems;

// PLOC build: neighbourhood radius, clusters per workgroup of the grid-wide
// iterations (small chunks keep every workgroup short once few clusters are
// left), the finish kernel's LDS capacity, workgroup sizes.
constexpr int kPlocR = 8;
constexpr int kPlocChunk = 512;
constexpr int kPlocThreads = 256;
constexpr int kPlocLocal = 4096;
constexpr int kPlocFinishThreads = 1024;
constexpr int kPlocMaxIters = 512;  // size of the per-iteration control array

// ceil(log2(ceil(n / kPlocLocal))) for n > kPlocLocal, else 0
inline int ploc_halvings(int64_t n)
{
    if (n <= kPlocLocal) return 0;
    const int64_t c = (n + kPlocLocal - 1) / kPlocLocal;
    int l = 0;
    while ((int64_t(1) << l) < c) ++l;
    return l;
}
// Grid-wide iterations launched for n clusters (the clustering removes about
// a tenth of the clusters per iteration; whatever is left above kPlocLocal
// afterwards is finished from global memory).
inline int ploc_global_iters(int64_t n) { return 7 * ploc_halvings(n); }
// Iteration from which clusters are paired by position instead of by
// distance, so every build ends after a bounded number of iterations.
inline int ploc_cap(int64_t n) { return 256 + 10 * ploc_halvings(n); }

// Device status bits (sticky, OR-ed by kernels).
constexpr int kStatusStack = 1;
constexpr int kStatusNonfinite = 2;
constexpr int kStatusListPool = 4;  // RS_PAPER_GRADIENT: the stored-list pool ran out

// Gaussian record, one per sorted position (64 bytes, four float4):
//   r0 = (RT00, RT01, RT02, RT10), r1 = (RT11, RT12, RT20, RT21),
//   r2 = (RT22, 1/sx, 1/sy, 1/sz), r3 = (mx, my, mz, opacity)
// RT = R^T, R the rotation of the normalised quaternion.
// BVH node, one per internal node (64 bytes, four float4):
//   n0 = (L.lo.x, L.lo.y, L.lo.z, L.hi.x), n1 = (L.hi.y, L.hi.z, R.lo.x, R.lo.y),
//   n2 = (R.lo.z, R.hi.x, R.hi.y, R.hi.z), n3 = (left ref, right ref, -, -) as int bits
// A child ref >= 0 names an internal node; ref < 0 names leaf ~ref.

// Header block at the start of the workspace (256 bytes).
struct WsHeader {
    int32_t status;
    uint32_t queue;        // persistent packet counter
    uint32_t bounds[6];    // ordered-uint min xyz, max xyz of the means
    float root_box[6];
    uint64_t counters[16];  // instrumentation (RS_COUNTERS)
    uint32_t xq[8];         // persistent packet counters, one per XCD chunk
    uint32_t pad[10];
};
static_assert(sizeof(WsHeader) == 256, "header size");

struct Layout {
    size_t header, records, nodes, gidx, inv, codes, leaf_boxes, parent, visit, ibox, keys_alt, vals_alt, hist, totals, gacc;
    size_t ploc_box, ploc_ref, ploc_pm, ploc_blk, ploc_ctrl, total;
    int64_t n, n_int, sort_blocks, ploc_chunks;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout make_layout(int64_t n)
{
    Layout L{};
    L.n = n;
    L.n_int = n > 1 ? n - 1 : 0;
    int64_t nn = n > 0 ? n : 1;
    int64_t ni = L.n_int > 0 ? L.n_int : 1;
    L.sort_blocks = (nn + kSortTile - 1) / kSortTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.header = take(sizeof(WsHeader));
    L.records = take(size_t(nn) * 64);
    L.nodes = take(size_t(ni) * 64);
    L.gidx = take(size_t(nn) * 4);
    L.inv = take(size_t(nn) * 4);
    L.codes = take(size_t(nn) * 4);
    L.leaf_boxes = take(size_t(nn) * 24);
    L.parent = take(size_t(2 * nn) * 4);
    L.visit = take(size_t(ni) * 4);
    L.ibox = take(size_t(ni) * 24);
    L.keys_alt = take(size_t(nn) * 4);
    L.vals_alt = take(size_t(nn) * 4);
    L.hist = take(size_t(256) * L.sort_blocks * 4);
    L.totals = take(size_t(512) * 4);
    L.gacc = take(size_t(nn) * 64);
    // PLOC clusters: two buffers of boxes (6 float arrays of n each) and refs,
    // the merge code per position, per-chunk counts, per-iteration control
    L.ploc_chunks = (nn + kPlocChunk - 1) / kPlocChunk;
    L.ploc_box = take(size_t(nn) * 48);
    L.ploc_ref = take(size_t(nn) * 8);
    L.ploc_pm = take(size_t(nn) * 4);
    L.ploc_blk = take(size_t(L.ploc_chunks) * 8);
    L.ploc_ctrl = take(size_t(kPlocMaxIters) * 16);
    L.total = off;
    return L;
}

// Descriptor stored in rs_bvh.opaque.
struct BvhDesc {
    uint64_t magic;
    int64_t n;
    float Q;
    int32_t root;       // root ref (0: internal node 0; ~0: single leaf; unused when n == 0)
    char *ws;
    uint64_t ws_bytes;
    int32_t kind;       // kKindGaussians or kKindMesh
    int32_t pad0;
    uint64_t pad[9];
};
constexpr int32_t kKindGaussians = 1;
constexpr int32_t kKindMesh = 2;
static_assert(sizeof(BvhDesc) <= sizeof(rs_bvh), "descriptor size");

// ---------------------------------------------------------------- helpers

// Wave-wide vote as a plain 64-bit lane mask (no int materialisation of the
// predicate, unlike the generic ballot).
__device__ inline uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ inline uint32_t float_to_ordered(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float ordered_to_float(uint32_t u)
{
    uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    return __uint_as_float(b);
}

// Ray state of one ray set (caller-owned), 256-byte aligned sections:
//   fin[n]   float4: final colour (composite + T bg) and final transmittance T
//   last[n]  uint4: the last composited hit's key (low word: Gaussian index,
//            high word: float bits of t1 + bias; both 0 when nothing was
//            composited), then T just before the hit that took T below the
//            smallest normal float (to 0 when alpha = 1) and the number of
//            composited hits after that one (0xffffffff when T stayed normal).
//            The adjoint walks the hits back to front from that key and
//            recovers T_k = T_{k+1} / (1 - alpha_k) from the final T; the saved
//            T restarts the recursion where it would divide 0 by 0 or lose its
//            digits in the subnormals.
//   list[n]  int4 (only with stored hit lists): composited hits, how many of
//            them the pool holds, the ray's packet's last pool chunk and the
//            packet's stored row count.
struct SetState {
    float4 *fin;
    uint4 *last;
    int4 *list;
};

// Stored hit lists: one pool shared by every packet of a launch. A packet's
// wavefront appends one row per compositing step: the entries of the lanes that
// consumed a hit at that step, in lane order (the Gaussian index it composited,
// or the index | kListSecond for a hit it only collected in the paper variant's
// second phase), then the 64-bit mask of those lanes as two words. Rows are
// packed into chunks of kChunkSlots 4-byte slots (a row never straddles two
// chunks), linked backwards per packet; fill[c] is the number of slots chunk c
// holds. The pool header holds the chunk counter (64-bit) and a flag set when a
// packet found the pool exhausted (its later rows are not stored).
constexpr int kChunkSlots = 512;
constexpr uint32_t kListIdle = 0xffffffffu;
constexpr uint32_t kListSecond = 0x80000000u;
struct ListPool {
    unsigned long long *hdr;  // [0] chunks taken, [1] exhausted flag
    int32_t *prev;            // [chunks] previous chunk of the same packet (-1: first)
    int32_t *fill;            // [chunks] slots used
    uint32_t *slots;          // [chunks][kChunkSlots]
    int64_t chunks;
};
inline int64_t list_chunks(int64_t slots_wanted)
{
    return (slots_wanted + kChunkSlots - 1) / kChunkSlots;
}
// bytes of a pool of `chunks` chunks (header, links, fills, slots), 256-byte aligned
inline size_t list_pool_bytes(int64_t chunks)
{
    if (chunks <= 0) return 0;
    return 256 + 2 * align256(size_t(chunks) * 4) + size_t(chunks) * kChunkSlots * 4;
}
inline ListPool list_pool_at(char *base, int64_t chunks)
{
    ListPool P{nullptr, nullptr, nullptr, nullptr, 0};
    if (!base || chunks <= 0) return P;
    P.hdr = reinterpret_cast<unsigned long long *>(base);
    P.prev = reinterpret_cast<int32_t *>(base + 256);
    P.fill = reinterpret_cast<int32_t *>(base + 256 + align256(size_t(chunks) * 4));
    P.slots = reinterpret_cast<uint32_t *>(base + 256 + 2 * align256(size_t(chunks) * 4));
    P.chunks = chunks;
    return P;
}

// Host description of one ray set of a render launch.
struct SetDesc {
    const rs_rays *rays;
    float *out_rgb;   // forward output (may be null in the adjoint)
    SetState state;   // fin may be null: no state written (forward without adjoint)
    const float *grad;
    float bg[3];
    int32_t zero_colour;
};

// Layout of the caller's ray state for n rays and hit-list capacity C
// (pool of C slots per ray on average).
struct StateLayout {
    size_t fin, last, list, pool, total;
    int64_t chunks;
};
inline StateLayout state_layout(int64_t n, int32_t cap)
{
    StateLayout L{0, 0, 0, 0, 0, 0};
    const size_t nn = size_t(n > 0 ? n : 0);
    L.fin = 0;
    L.last = align256(nn * 16);
    L.total = L.last + nn * 16;
    if (cap <= 0 || nn == 0) return L;
    L.list = align256(L.total);
    L.pool = align256(L.list + nn * 16);
    L.chunks = list_chunks(int64_t(nn) * cap);
    L.total = L.pool + list_pool_bytes(L.chunks);
    return L;
}
inline SetState state_at(void *base, int64_t n, int32_t cap)
{
    SetState S{nullptr, nullptr, nullptr};
    if (!base || n <= 0) return S;
    const StateLayout L = state_layout(n, cap);
    char *b = static_cast<char *>(base);
    S.fin = reinterpret_cast<float4 *>(b + L.fin);
    S.last = reinterpret_cast<uint4 *>(b + L.last);
    if (L.chunks > 0) S.list = reinterpret_cast<int4 *>(b + L.list);
    return S;
}

// What a render launch does.
enum class Pass { Forward, AdjointList, AdjointTraverse };

int launch_build(const rs_gaussians *g, float Q, bool lbvh, char *ws, hipStream_t st);
int launch_sets(const BvhDesc &D, const rs_gaussians *g, const rs_params *p, int nsets, const SetDesc *sets,
                const ListPool &pool, Pass pass, hipStream_t st);
// zero a pool's header (before a forward that stores lists)
void reset_pool(const ListPool &pool, hipStream_t st);
int launch_render(const BvhDesc &D, const rs_gaussians *g, const rs_rays *rays, const rs_params *p, float *out_rgb,
                  void *state, const float *grad, const rs_grads *grads, hipStream_t st);
void zero_gacc(const BvhDesc &D, hipStream_t st);
int launch_build_mesh(const rs_mesh *m, char *ws, hipStream_t st);
int launch_trace_mesh(const BvhDesc &M, const rs_rays *rays, const float *t_limit, int any_hit, int tile_shift, float *t_hit,
                      int32_t *tri, hipStream_t st);
size_t mesh_frame_bytes(int64_t n, int32_t cap, int bounces);
int mesh_frame_set(char *frame, int64_t n, int32_t cap, int bounces, int set, SetState *st, ListPool *pool);
size_t loss_workspace_bytes(int32_t w, int32_t h);
int launch_loss(const float *img, const float *tgt, int32_t w, int32_t h, const rs_loss_params *lp, float *loss,
                float *grad, void *ws, hipStream_t st);
size_t loss_scratch_bytes();
int loss_scratch(void **out);
int launch_mesh_fwd(const BvhDesc &G, const BvhDesc &M, const rs_gaussians *g, const rs_shading *sh,
                    const rs_rays *rays, const rs_params *p, float *out_rgb, void *frame, hipStream_t st);
int launch_mesh_bwd(const BvhDesc &G, const rs_gaussians *g, const rs_shading *sh, const rs_rays *rays, const rs_params *p,
                    const float *grad, void *frame, const rs_grads *grads, hipStream_t st);
void scatter_gacc(const BvhDesc &D, const float *quat, const rs_grads *grads, hipStream_t st);

}  // namespace rs
