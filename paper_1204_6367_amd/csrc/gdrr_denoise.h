// Scatter denoising (Sec. 2.5, Eq. 5) and noise assembly (Sec. 2.6).
//
// Eq. 5 is a Jacobi-type sweep: every pixel's new value needs its four
// neighbours' previous values.  A pass loads a region of 64 columns x 80 rows
// (a 48 x 64 tile with a halo of kDnHalo = 8 pixels) and runs up to kDnHalo
// sweeps on it without touching global memory: a wrong value at the region's
// outer edge (its missing neighbours are taken as itself) moves inward one
// pixel per sweep, so the tile stays exact.  Each wavefront holds a band of
// kDnRows rows of the region in registers, one column per lane: vertical
// neighbours are registers (the band's edge rows go through LDS), horizontal
// ones come from the neighbouring lanes.  At the detector's own edges the
// missing neighbour is the pixel itself, as in the definition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gdrr {

constexpr int kDnHalo = 8;
constexpr int kDnCols = 64;                          // region width = wavefront width
constexpr int kDnWaves = 4;
constexpr int kDnRows = 20;                          // rows per wavefront
constexpr int kDnTileU = kDnCols - 2 * kDnHalo;      // 48
constexpr int kDnTileV = kDnWaves * kDnRows - 2 * kDnHalo;   // 64
constexpr int kDnBlock = 64 * kDnWaves;

struct DnParams {
    const double* shat;       // image k at shat + k * shat_stride, [nv][nu]
    long long shat_stride;
    const float* s_in;        // previous pass [n][nv][nu], or null: start from max(shat, floor)
    float* s_out;             // next pass (float), or null
    double* out;              // final pass [n][nv][nu] (double), or null
    int n_img, nv, nu, tiles_u, tiles_v;
    int iters;                // sweeps in this pass (<= kDnHalo)
    float omega, inv_beta, s_floor;
};

__global__ __launch_bounds__(kDnBlock) void denoise_kernel(DnParams D) {
    __shared__ float edge[2][kDnWaves][64];              // first / last row of each band
    const int per_img = D.tiles_u * D.tiles_v;
    const int img = blockIdx.x / per_img, t = blockIdx.x % per_img;
    const int y0 = (t / D.tiles_u) * kDnTileV - kDnHalo, x0 = (t % D.tiles_u) * kDnTileU - kDnHalo;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the part of the region inside the image
    const int rlo = max(0, -y0), rhi = min(kDnWaves * kDnRows - 1, D.nv - 1 - y0);
    const int clo = max(0, -x0), chi = min(kDnCols - 1, D.nu - 1 - x0);
    const bool col_in = lane >= clo && lane <= chi;
    const int band = wave * kDnRows;                     // first region row of this wave
    const size_t npix = (size_t)D.nv * D.nu;
    const double* H = D.shat + (size_t)img * D.shat_stride;
    float s[kDnRows], h[kDnRows];
#pragma unroll
    for (int k = 0; k < kDnRows; ++k) {
        const int r = band + k;
        h[k] = 0.0f;
        s[k] = 0.0f;
        if (col_in && r >= rlo && r <= rhi) {
            const size_t p = (size_t)(y0 + r) * D.nu + (x0 + lane);
            h[k] = (float)H[p];
            s[k] = D.s_in ? D.s_in[(size_t)img * npix + p] : fmaxf(h[k], D.s_floor);
        }
    }
    const float w1 = 1.0f - D.omega, qw = 0.25f * D.omega;
    for (int it = 0; it < D.iters; ++it) {
        edge[0][wave][lane] = s[0];
        edge[1][wave][lane] = s[kDnRows - 1];
        __syncthreads();
        const float above = wave > 0 ? edge[1][wave - 1][lane] : s[0];
        const float below = wave < kDnWaves - 1 ? edge[0][wave + 1][lane] : s[kDnRows - 1];
        __syncthreads();
        float prev = above;                              // old value of the row above
#pragma unroll
        for (int k = 0; k < kDnRows; ++k) {
            const int r = band + k;
            const float sk = s[k];
            const float up = r > rlo ? prev : sk;
            const float dn = r < rhi ? (k + 1 < kDnRows ? s[k + 1] : below) : sk;
            const float left = __shfl_up(sk, 1);         // lane - 1 (lane 0 keeps its own)
            const float right = __shfl_down(sk, 1);      // lane + 1 (lane 63 keeps its own)
            const float lf = lane > clo ? left : sk;
            const float rt = lane < chi ? right : sk;
            const float hk = h[k];
            // 1 - h/s with the hardware reciprocal (about 1 ulp)
            const float data = hk == 0.0f ? 1.0f : 1.0f - hk * __builtin_amdgcn_rcpf(sk);
            const float v = fmaxf(w1 * sk + qw * ((up + dn + lf + rt) - data * D.inv_beta), D.s_floor);
            prev = sk;
            s[k] = (col_in && r >= rlo && r <= rhi) ? v : sk;
        }
    }
    if (lane < kDnHalo || lane >= kDnHalo + kDnTileU || lane > chi) return;
#pragma unroll
    for (int k = 0; k < kDnRows; ++k) {
        const int r = band + k;
        if (r < kDnHalo || r >= kDnHalo + kDnTileV || r > rhi) continue;
        const size_t p = (size_t)img * npix + (size_t)(y0 + r) * D.nu + (x0 + lane);
        if (D.out) D.out[p] = (double)s[k];
        else D.s_out[p] = s[k];
    }
}

// N = alpha ((Phat - P) + (Shat - S)) and the projection P + S + N, per pixel.
struct NoiseParams {
    const double* phat;       // image k at phat + k * phat_stride
    long long phat_stride;
    const double* p;          // [n][npix]
    const double* shat;       // image k at shat + k * shat_stride
    long long shat_stride;
    const double* s;          // [n][npix]
    double alpha;
    double* noise;            // [n][npix] or null
    double* image;            // [n][npix] or null
    long long npix, n;        // pixels per image, images
};

__global__ __launch_bounds__(256) void noise_kernel(NoiseParams Q) {
    const long long total = Q.npix * Q.n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long k = i / Q.npix, q = i - k * Q.npix;
        const double ph = Q.phat[k * Q.phat_stride + q], sh = Q.shat[k * Q.shat_stride + q];
        const double pp = Q.p[i], ss = Q.s[i];
        const double nn = Q.alpha * ((ph - pp) + (sh - ss));
        if (Q.noise) Q.noise[i] = nn;
        if (Q.image) Q.image[i] = (pp + ss) + nn;
    }
}

}  // namespace gdrr
