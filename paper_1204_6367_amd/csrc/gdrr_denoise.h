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

// Neighbours in the row from the lanes on either side (DPP whole-wavefront
// shifts: lane i reads lane i - 1, resp. i + 1); lane 0, resp. 63, keeps its
// own value, the missing neighbour at the region's edge.
__device__ __forceinline__ float dn_left(float x) {
    const int v = __float_as_int(x);
    return __int_as_float(__builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false));   // wave_shr:1
}
__device__ __forceinline__ float dn_right(float x) {
    const int v = __float_as_int(x);
    return __int_as_float(__builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false));   // wave_shl:1
}

// Images of at least kDnWaves * kDnRows rows and kDnCols columns: the region
// of each tile is shifted to lie inside the image (toward the interior at
// the borders).  Where a region edge then falls on the image's edge the
// missing neighbour is the pixel itself, as the definition wants there; every
// other region edge is at least kDnHalo pixels from the tile's own pixels.
// No pixel of the region needs a bounds test.
__global__ __launch_bounds__(kDnBlock) void denoise_inside_kernel(DnParams D) {
    __shared__ float edge[2][kDnWaves][64];
    const int per_img = D.tiles_u * D.tiles_v;
    const int img = blockIdx.x / per_img, t = blockIdx.x % per_img;
    const int ty = (t / D.tiles_u) * kDnTileV, tx = (t % D.tiles_u) * kDnTileU;   // the tile's first row, column
    const int y0 = min(max(ty - kDnHalo, 0), D.nv - kDnWaves * kDnRows);
    const int x0 = min(max(tx - kDnHalo, 0), D.nu - kDnCols);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int band = wave * kDnRows;
    const size_t npix = (size_t)D.nv * D.nu;
    const double* H = D.shat + (size_t)img * D.shat_stride + (size_t)(y0 + band) * D.nu + (x0 + lane);
    const float* Sin = D.s_in ? D.s_in + (size_t)img * npix + (size_t)(y0 + band) * D.nu + (x0 + lane) : nullptr;
    float s[kDnRows], h[kDnRows];
#pragma unroll
    for (int k = 0; k < kDnRows; ++k) {
        h[k] = (float)H[(size_t)k * D.nu];
        s[k] = Sin ? Sin[(size_t)k * D.nu] : fmaxf(h[k], D.s_floor);
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
            const float sk = s[k];
            const float dn = k + 1 < kDnRows ? s[k + 1] : below;
            const float hk = h[k];
            // 1 - h/s with the hardware reciprocal (about 1 ulp)
            const float data = hk == 0.0f ? 1.0f : 1.0f - hk * __builtin_amdgcn_rcpf(sk);
            const float v = w1 * sk + qw * ((prev + dn + dn_left(sk) + dn_right(sk)) - data * D.inv_beta);
            prev = sk;
            s[k] = fmaxf(v, D.s_floor);
        }
    }
    // the tile's own pixels
    const int col = x0 + lane;
    if (col < tx || col >= tx + kDnTileU) return;
#pragma unroll
    for (int k = 0; k < kDnRows; ++k) {
        const int row = y0 + band + k;
        if (row < ty || row >= ty + kDnTileV || row >= D.nv) continue;
        const size_t p = (size_t)img * npix + (size_t)row * D.nu + col;
        if (D.out) D.out[p] = (double)s[k];
        else D.s_out[p] = s[k];
    }
}

// Whole images that fit one workgroup's registers (nu = 64 C, nv = R x the
// number of wavefronts, at most 16): lane l of wavefront w holds the C x R
// block of columns [l C, l C + C) and rows [w R, w R + R), and all the sweeps
// run in one launch, with no halo and no pass through memory between sweeps.
// Neighbours inside the block are registers; across lanes the first/last
// column comes from the neighbouring lane by a DPP whole-wavefront shift (at
// the image's left/right edge a lane keeps its own pixel); across wavefronts
// the first/last row goes through LDS (at the top/bottom edge the pixel
// itself).  One workgroup per image.  The data Shat of the block's first R/2
// rows waits in LDS (96 KiB a workgroup), the rest in registers: with all of
// it in registers the 128 a lane has at 16 wavefronts per compute unit spilled.
// With the edge rows' two buffers a workgroup takes up to the whole 160 KiB.
template <int C, int R>
__global__ __launch_bounds__(1024) void denoise_image_kernel(DnParams D) {
    constexpr int RL = R / 2;                              // rows of Shat kept in LDS
    // first and last row of each wavefront's band, in two buffers used by turns: the writes
    // of sweep i + 2 come after the barrier of sweep i + 1, which every read of sweep i
    // precedes, so one barrier a sweep suffices
    __shared__ float edge[2][2][16][64 * C];
    __shared__ float4 h_lds[RL][16][64 * C / 4];          // [row][wavefront][lane's C values]
    static_assert(C == 4 || C == 2 || C == 1, "block width");
    const int img = blockIdx.x;
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t npix = (size_t)D.nv * D.nu;
    const int r0 = wave * R, c0 = lane * C;
    const double* H = D.shat + (size_t)img * D.shat_stride + (size_t)r0 * D.nu + c0;
    float s[R][C], h[R - RL][C];
    float* const hl = reinterpret_cast<float*>(&h_lds[0][wave][0]) + c0;   // row k at hl[k * 16 * 64 C]
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float hv = (float)H[(size_t)k * D.nu + c];
            if (k < RL) hl[(size_t)k * 16 * 64 * C + c] = hv;
            else h[k - RL][c] = hv;
            s[k][c] = fmaxf(hv, D.s_floor);
        }
    const float w1 = 1.0f - D.omega, qw = 0.25f * D.omega;
    for (int it = 0; it < D.iters; ++it) {
        const int e = it & 1;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            edge[e][0][wave][c0 + c] = s[0][c];
            edge[e][1][wave][c0 + c] = s[R - 1][c];
        }
        __syncthreads();
        float above[C], below[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            above[c] = wave > 0 ? edge[e][1][wave - 1][c0 + c] : s[0][c];
            below[c] = wave < waves - 1 ? edge[e][0][wave + 1][c0 + c] : s[R - 1][c];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            // the row's old values and its neighbours outside this lane's block
            float row[C], hrow[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                row[c] = s[k][c];
                hrow[c] = k < RL ? hl[(size_t)k * 16 * 64 * C + c] : h[k < RL ? 0 : k - RL][c];
            }
            const float left = __int_as_float(__builtin_amdgcn_update_dpp(
                __float_as_int(row[0]), __float_as_int(row[C - 1]), 0x138, 0xf, 0xf, false));   // wave_shr:1
            const float right = __int_as_float(__builtin_amdgcn_update_dpp(
                __float_as_int(row[C - 1]), __float_as_int(row[0]), 0x130, 0xf, 0xf, false));  // wave_shl:1
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float sk = row[c];
                const float up = above[c];
                const float dn = k + 1 < R ? s[k + 1][c] : below[c];
                const float lf = c > 0 ? row[c - 1] : left;
                const float rt = c + 1 < C ? row[c + 1] : right;
                const float hk = hrow[c];
                const float data = hk == 0.0f ? 1.0f : 1.0f - hk * __builtin_amdgcn_rcpf(sk);
                const float v = w1 * sk + qw * ((up + dn + lf + rt) - data * D.inv_beta);
                s[k][c] = fmaxf(v, D.s_floor);
                above[c] = sk;                            // old value, the next row's upper neighbour
            }
        }
    }
    double* out = D.out + (size_t)img * npix + (size_t)r0 * D.nu + c0;
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int c = 0; c < C; ++c) out[(size_t)k * D.nu + c] = (double)s[k][c];
}

// Any image size: the region may stick out of the image; rows and columns
// outside it are masked.
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
