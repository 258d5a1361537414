// Training loss of one image against its target and its gradient
// (Sec. 3, loss function; App. A.7): per colour channel
//   L_ch = (1 - lambda) mean (I - I^)^2 + lambda (1 - mean SSIM) / 2,
// averaged over the three channels. SSIM uses window moments of a normalised
// Gaussian window (zero outside the image); the gradient of mean SSIM is
// App. A.7's (1/hw) ((E * w) + I^ (F * w) - I (G * w)).
//
// Three launches: k_ssim_maps (moments by separable LDS-tiled window sums,
// the SSIM map reduced per tile, the E, F, G maps written), k_ssim_grad
// (window sums of E, F, G, then the per-pixel gradient) and k_loss_total.
#include <math.h>

#include <mutex>

#include "rs_internal.h"

namespace rs {

constexpr int kLossTw = 32, kLossTh = 8;  // output tile (256 threads)
constexpr int kMaxRadius = 7;

struct LossConst {
    int32_t w, h, r, tiles_x;
    float lambda;
    float g[2 * kMaxRadius + 1];  // normalised 1-D window (the 2-D window is its outer product)
};

// LDS patch of the tile plus a halo of r on every side; values outside the image are 0.
__device__ inline float ld_px(const float *__restrict__ img, int x, int y, int ch, const LossConst &L)
{
    return (x >= 0 && x < L.w && y >= 0 && y < L.h) ? img[(int64_t(y) * L.w + x) * 3 + ch] : 0.0f;
}

__global__ __launch_bounds__(256) void k_ssim_maps(const float *__restrict__ img, const float *__restrict__ tgt,
                                                   float *__restrict__ efg, float *__restrict__ partial,
                                                   const LossConst L)
{
    constexpr int PW = kLossTw + 2 * kMaxRadius, PH = kLossTh + 2 * kMaxRadius;
    __shared__ float pi[PH][PW], pt[PH][PW];
    __shared__ float hs[5][PH][kLossTw];  // horizontal window sums of I, I^, I^2, I^^2, I I^
    __shared__ float red[2][256];
    const int tid = threadIdx.x;
    const int tx0 = (blockIdx.x % L.tiles_x) * kLossTw, ty0 = (blockIdx.x / L.tiles_x) * kLossTh;
    const int r = L.r;
    const int pw = kLossTw + 2 * r, ph = kLossTh + 2 * r;
    const int ox = tid % kLossTw, oy = tid / kLossTw;
    const int gx = tx0 + ox, gy = ty0 + oy;
    const bool inside = gx < L.w && gy < L.h;
    float ssim_sum[3], sq_sum[3];
    for (int ch = 0; ch < 3; ++ch) {
        __syncthreads();
        for (int k = tid; k < pw * ph; k += 256) {
            const int px = k % pw, py = k / pw;
            pi[py][px] = ld_px(img, tx0 - r + px, ty0 - r + py, ch, L);
            pt[py][px] = ld_px(tgt, tx0 - r + px, ty0 - r + py, ch, L);
        }
        __syncthreads();
        for (int k = tid; k < ph * kLossTw; k += 256) {
            const int py = k / kLossTw, px = k % kLossTw;
            float a = 0.0f, b = 0.0f, aa = 0.0f, bb = 0.0f, ab = 0.0f;
            for (int m = 0; m <= 2 * r; ++m) {
                const float wv = L.g[m], x = pi[py][px + m], y = pt[py][px + m];
                a = __builtin_fmaf(wv, x, a);
                b = __builtin_fmaf(wv, y, b);
                aa = __builtin_fmaf(wv, x * x, aa);
                bb = __builtin_fmaf(wv, y * y, bb);
                ab = __builtin_fmaf(wv, x * y, ab);
            }
            hs[0][py][px] = a;
            hs[1][py][px] = b;
            hs[2][py][px] = aa;
            hs[3][py][px] = bb;
            hs[4][py][px] = ab;
        }
        __syncthreads();
        float s = 0.0f, q = 0.0f;
        if (inside) {
            float mu = 0.0f, mh = 0.0f, eaa = 0.0f, ebb = 0.0f, eab = 0.0f;
            for (int m = 0; m <= 2 * r; ++m) {
                const float wv = L.g[m];
                mu = __builtin_fmaf(wv, hs[0][oy + m][ox], mu);
                mh = __builtin_fmaf(wv, hs[1][oy + m][ox], mh);
                eaa = __builtin_fmaf(wv, hs[2][oy + m][ox], eaa);
                ebb = __builtin_fmaf(wv, hs[3][oy + m][ox], ebb);
                eab = __builtin_fmaf(wv, hs[4][oy + m][ox], eab);
            }
            const float c1 = 1e-4f, c2 = 9e-4f;
            const float A = 2.0f * mu * mh + c1;
            const float B = 2.0f * (eab - mu * mh) + c2;
            const float C = mu * mu + mh * mh + c1;
            const float D = (eaa - mu * mu) + (ebb - mh * mh) + c2;
            const float inv = 1.0f / (C * D);
            const float S = A * B * inv;
            s = S;
            const float d = pi[oy + r][ox + r] - pt[oy + r][ox + r];
            q = d * d;
            // App. A.7: E, F, G (factored through 1 / (C D) to stay in range)
            const float E = 2.0f * inv * (mh * (B - A) - S * mu * (D - C));
            const float F = 2.0f * A * inv;
            const float G = 2.0f * S / D;
            const int64_t plane = int64_t(L.w) * L.h, pix = int64_t(gy) * L.w + gx;
            efg[(3 * ch + 0) * plane + pix] = E;
            efg[(3 * ch + 1) * plane + pix] = F;
            efg[(3 * ch + 2) * plane + pix] = G;
        }
        ssim_sum[ch] = s;
        sq_sum[ch] = q;
    }
    // per-tile sums of the SSIM map and the squared error, per channel
    for (int ch = 0; ch < 3; ++ch) {
        __syncthreads();
        red[0][tid] = ssim_sum[ch];
        red[1][tid] = sq_sum[ch];
        __syncthreads();
        for (int step = 128; step > 0; step >>= 1) {
            if (tid < step) {
                red[0][tid] += red[0][tid + step];
                red[1][tid] += red[1][tid + step];
            }
            __syncthreads();
        }
        if (tid == 0) {
            partial[6 * int64_t(blockIdx.x) + ch] = red[0][0];
            partial[6 * int64_t(blockIdx.x) + 3 + ch] = red[1][0];
        }
    }
}

__global__ __launch_bounds__(256) void k_ssim_grad(const float *__restrict__ img, const float *__restrict__ tgt,
                                                   const float *__restrict__ efg, float *__restrict__ grad,
                                                   const LossConst L)
{
    constexpr int PW = kLossTw + 2 * kMaxRadius, PH = kLossTh + 2 * kMaxRadius;
    __shared__ float pm[3][PH][PW];
    __shared__ float hs[3][PH][kLossTw];
    const int tid = threadIdx.x;
    const int tx0 = (blockIdx.x % L.tiles_x) * kLossTw, ty0 = (blockIdx.x / L.tiles_x) * kLossTh;
    const int r = L.r;
    const int pw = kLossTw + 2 * r, ph = kLossTh + 2 * r;
    const int ox = tid % kLossTw, oy = tid / kLossTw;
    const int gx = tx0 + ox, gy = ty0 + oy;
    const bool inside = gx < L.w && gy < L.h;
    const int64_t plane = int64_t(L.w) * L.h;
    const float inv_n = 1.0f / float(plane);
    for (int ch = 0; ch < 3; ++ch) {
        __syncthreads();
        for (int k = tid; k < pw * ph; k += 256) {
            const int px = k % pw, py = k / pw;
            const int x = tx0 - r + px, y = ty0 - r + py;
            const bool in = x >= 0 && x < L.w && y >= 0 && y < L.h;
            const int64_t pix = int64_t(y) * L.w + x;
            for (int q = 0; q < 3; ++q) pm[q][py][px] = in ? efg[(3 * ch + q) * plane + pix] : 0.0f;
        }
        __syncthreads();
        for (int k = tid; k < ph * kLossTw; k += 256) {
            const int py = k / kLossTw, px = k % kLossTw;
            float e = 0.0f, f = 0.0f, g = 0.0f;
            for (int m = 0; m <= 2 * r; ++m) {
                const float wv = L.g[m];
                e = __builtin_fmaf(wv, pm[0][py][px + m], e);
                f = __builtin_fmaf(wv, pm[1][py][px + m], f);
                g = __builtin_fmaf(wv, pm[2][py][px + m], g);
            }
            hs[0][py][px] = e;
            hs[1][py][px] = f;
            hs[2][py][px] = g;
        }
        __syncthreads();
        if (inside) {
            float e = 0.0f, f = 0.0f, g = 0.0f;
            for (int m = 0; m <= 2 * r; ++m) {
                const float wv = L.g[m];
                e = __builtin_fmaf(wv, hs[0][oy + m][ox], e);
                f = __builtin_fmaf(wv, hs[1][oy + m][ox], f);
                g = __builtin_fmaf(wv, hs[2][oy + m][ox], g);
            }
            const int64_t at = (int64_t(gy) * L.w + gx) * 3 + ch;
            const float I = img[at], T = tgt[at];
            const float dssim = (e + T * f - I * g) * inv_n;
            grad[at] = (2.0f * (1.0f - L.lambda) * inv_n * (I - T) - 0.5f * L.lambda * dssim) * (1.0f / 3.0f);
        }
    }
}

__global__ __launch_bounds__(256) void k_loss_total(const float *__restrict__ partial, int64_t n_tiles,
                                                    float *__restrict__ loss, const LossConst L)
{
    __shared__ double red[6][256];
    const int tid = threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = tid; b < n_tiles; b += 256)
        for (int k = 0; k < 6; ++k) acc[k] += double(partial[6 * b + k]);
    for (int k = 0; k < 6; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int step = 128; step > 0; step >>= 1) {
        if (tid < step)
            for (int k = 0; k < 6; ++k) red[k][tid] += red[k][tid + step];
        __syncthreads();
    }
    if (tid == 0) {
        const double n = double(L.w) * double(L.h), lam = L.lambda;
        double tot = 0.0;
        for (int ch = 0; ch < 3; ++ch)
            tot += (1.0 - lam) * red[3 + ch][0] / n + lam * (1.0 - red[ch][0] / n) * 0.5;
        loss[0] = float(tot / 3.0);
    }
}

// ------------------------------------------------------------------- host

static LossConst loss_const(int32_t w, int32_t h, const rs_loss_params *lp)
{
    LossConst L{};
    L.w = w;
    L.h = h;
    L.r = lp->radius;
    L.tiles_x = (w + kLossTw - 1) / kLossTw;
    L.lambda = lp->lambda;
    double g[2 * kMaxRadius + 1], sum = 0.0;
    for (int m = -L.r; m <= L.r; ++m) {
        g[m + L.r] = exp(-double(m) * m / (2.0 * double(lp->sigma) * lp->sigma));
        sum += g[m + L.r];
    }
    for (int m = 0; m <= 2 * L.r; ++m) L.g[m] = float(g[m] / sum);
    return L;
}

static int64_t loss_tiles(int32_t w, int32_t h)
{
    return int64_t((w + kLossTw - 1) / kLossTw) * ((h + kLossTh - 1) / kLossTh);
}

size_t loss_workspace_bytes(int32_t w, int32_t h)
{
    const size_t maps = align256(size_t(9) * size_t(w) * size_t(h) * 4);
    return maps + align256(size_t(loss_tiles(w, h)) * 6 * 4);
}

int launch_loss(const float *img, const float *tgt, int32_t w, int32_t h, const rs_loss_params *lp, float *loss,
                float *grad, void *ws, hipStream_t st)
{
    const LossConst L = loss_const(w, h, lp);
    const int64_t tiles = loss_tiles(w, h);
    float *efg = static_cast<float *>(ws);
    float *partial = reinterpret_cast<float *>(static_cast<char *>(ws) +
                                               align256(size_t(9) * size_t(w) * size_t(h) * 4));
    k_ssim_maps<<<int(tiles), 256, 0, st>>>(img, tgt, efg, partial, L);
    if (grad) k_ssim_grad<<<int(tiles), 256, 0, st>>>(img, tgt, efg, grad, L);
    k_loss_total<<<1, 256, 0, st>>>(partial, tiles, loss, L);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

// ------------------------------------------------ allocation-free variant

// Device scratch of rs_loss_noalloc: a file-scope array each GPU holds for the
// life of the process (its E, F, G maps and per-tile partial sums). Host code
// never passes the array's name to a kernel: it takes the array's device
// address on each device once, with hipGetSymbolAddress, and uses that.
constexpr size_t kLossScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices];

size_t loss_scratch_bytes() { return kLossScratchBytes; }

// The scratch array's device address on the current device (taken on the first
// call made with that device current).
int loss_scratch(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RS_ERR_HIP;
    if (dev < 0 || dev >= kMaxScratchDevices) return RS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RS_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RS_OK;
}

}  // namespace rs
