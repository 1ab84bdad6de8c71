// Device-side building blocks of the gfx950 Monte Carlo projection step:
// counter-based random numbers, the per-job geometry, table lookups,
// interaction samplers and the direction update.  Everything here is
// float32 except the inverse-CDF comparisons of source sampling (float64,
// once per history).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gdrr {

constexpr float kMeC2 = 510.99895f;       // electron rest energy, keV
constexpr float kHc = 12.398419843f;      // h c, keV Angstrom
constexpr int kMaxTries = 256;            // rejection-sampler cap (never reached in practice)
constexpr uint32_t kMaxSteps = 1u << 20;  // free flights per history before it is declared lost
constexpr double kQ1 = 1048576.0;         // tally fixed point: 2^20 units per keV
constexpr double kQ2 = 1024.0;            // squared tally: 2^10 units per keV^2
constexpr float kMaxResponse = 1024.0f;   // r(E) clamp (keeps the fixed-point sums inside 64 bits)

enum : int { kPrimary = 0, kScatter = 1, kAbsorbed = 2, kCut = 3, kMissed = 4, kLost = 5 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Counter (c0, c1, c2, c3) =
// (photon index, job id, step, sub), key = 64-bit seed.
// ---------------------------------------------------------------------------
struct Block {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Block philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // (three-way xors in one gfx950 v_bitop3_b32 each; truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block{c0, c1, c2, c3};
}

// 23 random bits -> odd multiple of 2^-24 in (0, 1); exact in float32.
__device__ __forceinline__ float u24(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 0x1p-23f; }

// 53 random bits of two words -> [0, 1), exact in float64.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return (double)(((uint64_t)a << 21) | (uint64_t)(b >> 11)) * 0x1p-53;
}

__device__ __forceinline__ float fast_log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
// -expm1(e) = 1 - exp(e) for e <= 0.  For e in [-0.47, 0] (photon energies up
// to 150 keV in the Compton sampler) by its Taylor series to e^7 (relative
// error below 3e-7 there), without the cancellation of 1 - exp(e); below
// -0.47, 1 - exp(e) > 0.37 has no cancellation and is evaluated directly.
__device__ __forceinline__ float one_minus_exp(float e) {
    if (e < -0.47f) return 1.0f - fast_exp(e);
    float t = 1.0f + e * (1.0f / 7.0f);
    t = 1.0f + e * (1.0f / 6.0f) * t;
    t = 1.0f + e * (1.0f / 5.0f) * t;
    t = 1.0f + e * (1.0f / 4.0f) * t;
    t = 1.0f + e * (1.0f / 3.0f) * t;
    t = 1.0f + e * 0.5f * t;
    return -e * t;
}

// A voxel density as the kernels use it: negative, NaN and infinite values
// count as 0 (the kernels that read them also set the input-error bit).
__device__ __forceinline__ bool density_ok(float r) { return r >= 0.0f && r <= 3.402823466e38f; }
__device__ __forceinline__ float clean_density(float r) { return density_ok(r) ? r : 0.0f; }

// Input-error bits, or-ed into a call's status word.
enum : unsigned int { kErrDensity = 1u, kErrMaterial = 2u, kErrWeights = 4u };

// sin / cos of 2 pi r (the hardware unit takes revolutions)
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// ---------------------------------------------------------------------------
// Launch-time descriptors (built on the host).
// ---------------------------------------------------------------------------
// One record per cell of the lattice of voxel centres: cell (i, j, k),
// i in [-1, nx-1], has the voxel centres i and i+1 (clamped into the volume)
// as corners along x, likewise along y and z; corner c = bx + 2 by + 4 bz.
// The record holds the eight corner densities in 32 bytes; their sign bits
// (densities are >= 0) carry the materials: d[0]'s sign set means the
// corners' materials differ (they are then read from the voxel array),
// otherwise the signs of d[1..4] hold the corners' common material, clamped
// to n_mat - 1 (n_mat <= 16).  The stencil of a free flight is one pair of
// 16-byte loads.
struct alignas(32) CellRec {
    float d[8];
};

struct DVolume {
    const float* density;
    const uint8_t* material;
    const CellRec* cells;     // [(nz+1)][(ny+1)][(nx+1)]
    int nx, ny, nz, nxy;
    int cx, cxy;              // cells per row (nx+1) and per slab ((nx+1)(ny+1))
    float lox, loy, loz;      // box corner (-n d / 2)
    float hix, hiy, hiz;
    float idx, idy, idz;      // 1 / voxel size
    int lds_majorant;         // offset (float2 units) of this volume's majorant table in LDS
    // local majorants (null: one majorant per energy interval for the whole volume)
    const uint2* macro;       // per cube: (1 + margin) rho_max (float bits), material bit mask
    int mnx, mny, mnz, mcube; // cubes per axis; voxels per cube edge
    float mex, mey, mez;      // cube edge, mm
    float imx, imy, imz;      // 1 / cube edge
};

struct DSource {
    const float* spec_e;      // [n_spec]
    const double* spec_cdf;   // [rows][n_spec]
    const uint32_t* spec_guide;  // [rows][spec_k]
    const double* flu_cdf;    // [npix]
    const uint32_t* flu_guide;   // [flu_k]
    int n_spec, spec_k, npix, flu_k;
    int spec_rows;            // 1, or nu: the spectrum of detector column iu is row iu
};

// One job, as the kernels read it (global memory, 112 bytes).
struct alignas(16) DJob {
    float Sx, Sy, Sz;
    uint32_t first;           // first photon index of the job
    float Px, Py, Pz, pad1;
    float nx, ny, nz, pad2;   // detector normal
    float ux, uy, uz, pad3;   // u axis; v axis is +z
    float du, dv, idu, idv;
    int nu, nv, src, vol;
    uint32_t job_id, n_lo, n_hi, index;   // photons of the job; index into the caller's job array
    long long tally_off;      // u64 element offset of the job's fixed-point block
    long long adj_off;        // double element offset of the job's adjoint weights
};

// Inverse CDF with a guide table: the smallest i with u < cdf[i].
// guide[g] = smallest i with cdf[i] > g / K, so the search starts there.
__device__ __forceinline__ int sample_cdf(const double* __restrict__ cdf, const uint32_t* __restrict__ guide,
                                          int n, int k, double u) {
    int g = (int)(u * (double)k);
    g = g < k - 1 ? g : k - 1;
    int i = (int)guide[g];
    while (i < n - 1 && !(u < cdf[i])) ++i;
    return i;
}

// New direction after a deflection by theta (cosine ct) at azimuth 2 pi r
// about d: d' = ct d + st (cos e1 + sin e2) with (e1, e2, d) orthonormal;
// e2 = (z x d)/|z x d| away from the z axis, (x x d)/|x x d| within 0.1 of it.
__device__ __forceinline__ void rotate(float& dx, float& dy, float& dz, float ct, float r) {
    const float st = sqrtf(fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
    const float cp = cos_rev(r), sp = sin_rev(r);
    const float rxy2 = dx * dx + dy * dy;
    float e1x, e1y, e1z, e2x, e2y, e2z;
    if (rxy2 > 0.01f) {
        const float ir = __builtin_amdgcn_rsqf(rxy2);
        const float rr = rxy2 * ir;
        e2x = -dy * ir; e2y = dx * ir; e2z = 0.0f;
        e1x = dx * dz * ir; e1y = dy * dz * ir; e1z = -rr;
    } else {
        const float q2 = dy * dy + dz * dz;
        const float iq = __builtin_amdgcn_rsqf(q2);
        e2x = 0.0f; e2y = -dz * iq; e2z = dy * iq;
        e1x = -q2 * iq; e1y = dx * dy * iq; e1z = dx * dz * iq;
    }
    const float a = st * cp, b = st * sp;
    float ox = ct * dx + a * e1x + b * e2x;
    float oy = ct * dy + a * e1y + b * e2y;
    float oz = ct * dz + a * e1z + b * e2z;
    const float inv = __builtin_amdgcn_rsqf(ox * ox + oy * oy + oz * oz);
    dx = ox * inv; dy = oy * inv; dz = oz * inv;
}

// Distance from a point inside the box to its boundary along d.
__device__ __forceinline__ float box_exit(const DVolume& V, float px, float py, float pz,
                                          float dx, float dy, float dz) {
    float t = INFINITY;
    if (dx != 0.0f) t = fminf(t, ((dx > 0.0f ? V.hix : V.lox) - px) * fast_rcp(dx));
    if (dy != 0.0f) t = fminf(t, ((dy > 0.0f ? V.hiy : V.loy) - py) * fast_rcp(dy));
    if (dz != 0.0f) t = fminf(t, ((dz > 0.0f ? V.hiz : V.loz) - pz) * fast_rcp(dz));
    return fmaxf(t, 0.0f);
}

// Slab-method entry of the ray S + t d (t >= 0) into the box; false on a miss.
__device__ __forceinline__ bool box_entry(const DVolume& V, float sx, float sy, float sz,
                                          float dx, float dy, float dz, float& tin, float& tout) {
    float t0 = 0.0f, t1 = INFINITY;
    const float s[3] = {sx, sy, sz}, d[3] = {dx, dy, dz};
    const float lo[3] = {V.lox, V.loy, V.loz}, hi[3] = {V.hix, V.hiy, V.hiz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (s[a] < lo[a] || s[a] > hi[a]) return false;
            continue;
        }
        const float inv = fast_rcp(d[a]);
        float ta = (lo[a] - s[a]) * inv, tb = (hi[a] - s[a]) * inv;
        if (ta > tb) { const float t = ta; ta = tb; tb = t; }
        t0 = fmaxf(t0, ta);
        t1 = fminf(t1, tb);
    }
    tin = t0;
    tout = t1;
    return t0 < t1;
}

// Scattering angle of a Compton or a Rayleigh event, both by rejection with
// one Philox block (photon, job, step, 1 + try) per try; the try's fourth word
// is the azimuth (in revolutions).  Returns cos(theta) (1 if every try is
// rejected).  The two samplers share the loop and its Philox block, so that a
// wavefront holding both kinds of event generates each try's block once.
//
// Compton, free-electron Klein-Nishina: tau = E'/E drawn from the mixture of
// densities ~1/tau (weight ln(1+2k)) and ~tau (weight (1-tau0^2)/2) on
// [tau0, 1], kept with probability 1 - tau sin^2/(1+tau^2); E *= tau.
//
// Rayleigh with F(x) = Z exp(-x/x0), x = sin(theta/2)/lambda in [0, 1/lambda]:
// x from Gamma(2, x0/2) truncated at 1/lambda when 1/lambda >= x0, else from
// the density ~x on [0, 1/lambda] kept with probability exp(-2x/x0); then kept
// with probability (1 + cos^2)/2.
__device__ __forceinline__ float scatter_angle(bool is_rayleigh, uint32_t pid, uint32_t job, uint32_t step,
                                               uint32_t k0, uint32_t k1, float& E, float x0, float& az) {
    // Compton constants
    const float k = E * (1.0f / kMeC2);
    const float tau0 = fast_rcp(1.0f + 2.0f * k);
    const float a1 = fast_log(1.0f + 2.0f * k);
    const float ik = fast_rcp(k);
    const float omt02 = 1.0f - tau0 * tau0;
    const float a2 = 0.5f * omt02;
    // Rayleigh constants
    const float xmax = E * (1.0f / kHc);
    const float ixmax = kHc * fast_rcp(E);
    const float m2ix0 = -2.0f * fast_rcp(x0);
    for (int t = 0; t < kMaxTries; ++t) {
        const Block b = philox(pid, job, step, 1u + (uint32_t)t, k0, k1);
        const float b0 = u24(b.x), b1 = u24(b.y), b2 = u24(b.z);
        az = u24(b.w);
        if (is_rayleigh) {
            float xx;
            bool ok;
            if (xmax >= x0) {
                xx = -0.5f * x0 * (fast_log(b0) + fast_log(b1));
                ok = xx <= xmax;
            } else {
                xx = xmax * sqrtf(b0);
                ok = b1 <= fast_exp(m2ix0 * xx);
            }
            const float r = xx * ixmax;
            const float ct = 1.0f - 2.0f * r * r;
            if (ok && b2 <= 0.5f * (1.0f + ct * ct)) return ct;
        } else {
            float tau, omt;   // tau and 1 - tau, the latter without cancellation
            if (b0 * (a1 + a2) < a1) {
                const float e = -a1 * b1;               // in [-ln(1 + 2k), 0]; |e| <= 0.47 for E <= 150 keV
                omt = one_minus_exp(e);
                tau = 1.0f - omt;
            } else {
                const float t2 = tau0 * tau0 + omt02 * b1;
                tau = sqrtf(t2);
                omt = omt02 * (1.0f - b1) * fast_rcp(1.0f + tau);
            }
            const float itau = fast_rcp(tau);
            const float omc = omt * ik * itau;          // 1 - cos(theta)
            const float ct = 1.0f - omc;
            const float sin2 = omc * (2.0f - omc);
            const float g = 1.0f - tau * sin2 * fast_rcp(1.0f + tau * tau);
            if (b2 <= g) {
                E *= tau;
                return ct;
            }
        }
    }
    return 1.0f;
}

}  // namespace gdrr
