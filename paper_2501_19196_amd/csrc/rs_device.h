// Device helpers shared by the Gaussian and triangle traversals: packets of
// 64-pixel tiles (8x8 by default), rays and conservative slab tests.
#pragma once

#include "rs_internal.h"

namespace rs {

struct ViewEntry {
    int64_t ray_offset;
    int64_t first_packet;
    int32_t width, height, tiles_x, pad;
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
        E.first_packet = packets;
        packets += int64_t(E.tiles_x) * ((V.height + th - 1) / th);
    }
    return packets;
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

// Direction signs shared by every valid lane of the wave: when they agree per
// axis (uni), the near and far planes of a box are chosen once per wave.
struct WaveSigns {
    bool uni, px, py, pz;
};

__device__ inline WaveSigns wave_signs(const Slab &sl, bool valid)
{
    const uint64_t vmask = __ballot(valid);
    const uint64_t bx = __ballot(valid && sl.ix >= 0.0f), by = __ballot(valid && sl.iy >= 0.0f),
                   bz = __ballot(valid && sl.iz >= 0.0f);
    WaveSigns w;
    w.uni = (bx == 0 || bx == vmask) && (by == 0 || by == vmask) && (bz == 0 || bz == vmask);
    w.px = bx != 0;
    w.py = by != 0;
    w.pz = bz != 0;
    return w;
}

// Entry and exit distances of both child boxes of a node
// (L = (n0.xyz, n0.w n1.xy), R = (n1.zw n2.x, n2.yzw)).
__device__ inline void child_slabs(const float4 n0, const float4 n1, const float4 n2, const Slab &sl,
                                   const WaveSigns &ws, float &ln, float &lf, float &rn, float &rf)
{
    if (ws.uni) {
        const bool px = ws.px, py = ws.py, pz = ws.pz;
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
