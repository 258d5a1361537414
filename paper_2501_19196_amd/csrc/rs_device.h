// Device helpers shared by the Gaussian and triangle traversals: packets of
// 64-pixel tiles (8x8 by default), rays and conservative slab tests.
#pragma once

#include "rs_internal.h"

namespace rs {

struct ViewEntry {
    int64_t ray_offset;
    int64_t first_packet;
    int32_t width, height, tiles_x, tiles_y;
};

struct Ray {
    float ox, oy, oz, dx, dy, dz;
};

constexpr float kInf = __builtin_huge_valf();

// --------------------------------------------------------------- packets

// Host: fill the view table of a launch (tiles of 2^tile_shift x 64 / 2^tile_shift
// pixels) and return its packet count.
template <typename PT>
inline int64_t plan_packets(PT &P, const rs_rays *rays, int tile_shift)
{
    P.n_views = rays->n_views;
    P.tile_shift = tile_shift;
    if (rays->n_views == 0) return (rays->n + kWave - 1) / kWave;
    const int tw = 1 << tile_shift, th = kWave >> tile_shift;
    int64_t packets = 0;
    for (int v = 0; v < rays->n_views; ++v) {
        const rs_view &V = rays->views[v];
        ViewEntry &E = P.views[v];
        E.ray_offset = V.ray_offset;
        E.width = V.width;
        E.height = V.height;
        E.tiles_x = (V.width + tw - 1) / tw;
        E.tiles_y = (V.height + th - 1) / th;
        E.first_packet = packets;
        packets += int64_t(E.tiles_x) * E.tiles_y;
    }
    return packets;
}

// Strip-major order of a view's tiles: the view is cut into vertical strips
// of `strip` tiles and each strip is walked row by row, so that a contiguous
// range of this order covers a compact image region. Maps an index of that
// order to the row-major tile index (both counted over all views).
template <typename PT>
__device__ inline int64_t strip_major_packet(const PT &P, int64_t pkt, int strip)
{
    if (P.n_views == 0 || strip <= 0) return pkt;
    int v = 0;
    for (int k = 1; k < P.n_views; ++k)
        if (pkt >= P.views[k].first_packet) v = k;
    const ViewEntry &V = P.views[v];
    const uint32_t l = uint32_t(pkt - V.first_packet);
    const uint32_t tx_n = uint32_t(V.tiles_x), ty_n = uint32_t(V.tiles_y), sw = uint32_t(strip);
    const uint32_t s = l / (sw * ty_n);
    const uint32_t rem = l - s * sw * ty_n;
    const uint32_t w = tx_n - s * sw < sw ? tx_n - s * sw : sw;
    const uint32_t ty = rem / w, tx = s * sw + (rem - ty * w);
    return V.first_packet + int64_t(ty) * tx_n + tx;
}

// Packet index -> ray index of this lane (row-major tiles within each view).
template <typename PT>
__device__ inline int64_t packet_ray(const PT &P, int64_t pkt, int lane, bool &valid)
{
    if (P.n_views == 0) {
        int64_t r = pkt * kWave + lane;
        valid = r < P.n_rays;
        return r;
    }
    int v = 0;
    for (int k = 1; k < P.n_views; ++k)
        if (pkt >= P.views[k].first_packet) v = k;
    const ViewEntry &V = P.views[v];
    const int sh = P.tile_shift;
    int64_t local = pkt - V.first_packet;
    int64_t ty = local / V.tiles_x, tx = local - ty * V.tiles_x;
    int64_t x = (tx << sh) + (lane & ((1 << sh) - 1));
    int64_t y = ty * (kWave >> sh) + (lane >> sh);
    valid = x < V.width && y < V.height;
    return V.ray_offset + y * V.width + x;
}

// Slab-test constants: a box [lo, hi] is entered at max_k (near_k - o_k) / d_k and
// left at min_k (far_k - o_k) / d_k, evaluated as fma(plane, 1/d, -o/d). The far
// distance and the round's upper bound are widened by a relative 2^-19 plus the
// rounding scale of o/d, so rounding never culls a box the exact test keeps.
constexpr float kWiden = 1.9073486328125e-6f;  // 2^-19

struct Slab {
    float ix, iy, iz, nx, ny, nz, pad;
};

__device__ inline float widen(float t, float pad) { return __builtin_fmaf(fabsf(t), kWiden, t) + pad; }

// A child box's exit distance widened for the overlap test: t (1 + 2^-19) + pad.
// Equal to widen(t, pad) for t >= 0; for t < 0 (box behind the origin up to
// rounding) it still exceeds the exact exit distance, since the rounding error
// of a slab distance near 0 is below 2^-22 |o/d|, less than pad.
constexpr float kWidenUp = 1.0000019073486328125f;  // 1 + 2^-19
__device__ inline float widen_exit(float t, float pad) { return __builtin_fmaf(t, kWidenUp, pad); }

// Whether [near, exit] meets [t_lo, t_hi] (written as compares so that no
// min/max of loop-carried values needs NaN canonicalisation).
__device__ inline bool overlaps(float near, float exit_w, float t_lo, float t_hi_w)
{
    return near <= exit_w && near <= t_hi_w && t_lo <= exit_w;
}

// Slab constants of a ray (zero direction components replaced by a tiny value of the same sign).
__device__ inline Slab make_slab(const Ray &ray)
{
    Slab sl;
    const float sx = fabsf(ray.dx) > 1e-20f ? ray.dx : copysignf(1e-20f, ray.dx);
    const float sy = fabsf(ray.dy) > 1e-20f ? ray.dy : copysignf(1e-20f, ray.dy);
    const float sz = fabsf(ray.dz) > 1e-20f ? ray.dz : copysignf(1e-20f, ray.dz);
    sl.ix = 1.0f / sx;
    sl.iy = 1.0f / sy;
    sl.iz = 1.0f / sz;
    sl.nx = -ray.ox * sl.ix;
    sl.ny = -ray.oy * sl.iy;
    sl.nz = -ray.oz * sl.iz;
    sl.pad = kWiden * fmaxf(fmaxf(fabsf(sl.nx), fabsf(sl.ny)), fabsf(sl.nz));
    return sl;
}

// Direction octant shared by every valid lane of the wave (bit 0: +x, bit 1:
// +y, bit 2: +z), or kMixedOctant when the lanes' direction signs differ.
constexpr int kMixedOctant = 8;

__device__ inline int wave_octant(const Slab &sl, bool valid)
{
    const uint64_t vmask = wave_ballot(valid);
    const uint64_t bx = wave_ballot(valid && sl.ix >= 0.0f), by = wave_ballot(valid && sl.iy >= 0.0f),
                   bz = wave_ballot(valid && sl.iz >= 0.0f);
    const bool uni = (bx == 0 || bx == vmask) && (by == 0 || by == vmask) && (bz == 0 || bz == vmask);
    const int oct = (bx != 0 ? 1 : 0) | (by != 0 ? 2 : 0) | (bz != 0 ? 4 : 0);
    return __builtin_amdgcn_readfirstlane(uni ? oct : kMixedOctant);
}

// Entry and exit distances of both child boxes of a node
// (L = (n0.xyz, n0.w n1.xy), R = (n1.zw n2.x, n2.yzw)). For a known octant the
// near and far planes are fixed at compile time (12 FMAs and 4 min3/max3);
// the mixed form orders each plane pair per lane.
template <int OCT>
__device__ inline void child_slabs(const float4 n0, const float4 n1, const float4 n2, const Slab &sl, float &ln,
                                   float &lf, float &rn, float &rf)
{
    if constexpr (OCT != kMixedOctant) {
        constexpr bool px = (OCT & 1) != 0, py = (OCT & 2) != 0, pz = (OCT & 4) != 0;
        ln = fmaxf(fmaxf(__builtin_fmaf(px ? n0.x : n0.w, sl.ix, sl.nx), __builtin_fmaf(py ? n0.y : n1.x, sl.iy, sl.ny)),
                   __builtin_fmaf(pz ? n0.z : n1.y, sl.iz, sl.nz));
        lf = fminf(fminf(__builtin_fmaf(px ? n0.w : n0.x, sl.ix, sl.nx), __builtin_fmaf(py ? n1.x : n0.y, sl.iy, sl.ny)),
                   __builtin_fmaf(pz ? n1.y : n0.z, sl.iz, sl.nz));
        rn = fmaxf(fmaxf(__builtin_fmaf(px ? n1.z : n2.y, sl.ix, sl.nx), __builtin_fmaf(py ? n1.w : n2.z, sl.iy, sl.ny)),
                   __builtin_fmaf(pz ? n2.x : n2.w, sl.iz, sl.nz));
        rf = fminf(fminf(__builtin_fmaf(px ? n2.y : n1.z, sl.ix, sl.nx), __builtin_fmaf(py ? n2.z : n1.w, sl.iy, sl.ny)),
                   __builtin_fmaf(pz ? n2.w : n2.x, sl.iz, sl.nz));
    } else {
        const float lx0 = __builtin_fmaf(n0.x, sl.ix, sl.nx), lx1 = __builtin_fmaf(n0.w, sl.ix, sl.nx);
        const float ly0 = __builtin_fmaf(n0.y, sl.iy, sl.ny), ly1 = __builtin_fmaf(n1.x, sl.iy, sl.ny);
        const float lz0 = __builtin_fmaf(n0.z, sl.iz, sl.nz), lz1 = __builtin_fmaf(n1.y, sl.iz, sl.nz);
        const float rx0 = __builtin_fmaf(n1.z, sl.ix, sl.nx), rx1 = __builtin_fmaf(n2.y, sl.ix, sl.nx);
        const float ry0 = __builtin_fmaf(n1.w, sl.iy, sl.ny), ry1 = __builtin_fmaf(n2.z, sl.iy, sl.ny);
        const float rz0 = __builtin_fmaf(n2.x, sl.iz, sl.nz), rz1 = __builtin_fmaf(n2.w, sl.iz, sl.nz);
        ln = fmaxf(fmaxf(fminf(lx0, lx1), fminf(ly0, ly1)), fminf(lz0, lz1));
        lf = fminf(fminf(fmaxf(lx0, lx1), fmaxf(ly0, ly1)), fmaxf(lz0, lz1));
        rn = fmaxf(fmaxf(fminf(rx0, rx1), fminf(ry0, ry1)), fminf(rz0, rz1));
        rf = fminf(fminf(fmaxf(rx0, rx1), fmaxf(ry0, ry1)), fmaxf(rz0, rz1));
    }
}

}  // namespace rs
