// Primary signal by ray tracing (Sec. 2.3, Eq. 1): one lane per detector
// pixel, every energy channel of the spectrum.
//
//   P(u) = sum_k phi_k w(u) r(E_k) exp(-sum_j dl_j mu(x_j, E_k))
//
// The ray from the source to the pixel centre is cut into intervals
// [j dl, (j+1) dl) of its length from the source; the part of an interval
// inside the phantom box is one term, evaluated at that part's midpoint.
// mu(x, E) is the trilinear interpolation of the voxel attenuation
// coefficients rho_v mu_tot(m_v, E) (the corners of the lattice cell around
// x, clamped at the edges), or the containing voxel's value with the
// interpolation off.
//
// mu is linear in the per-voxel products, so the energy channels share one
// march: the lane accumulates, per material m, the line integral of the
// density carried by m's corners (L_m), and the channel sums come out as
// sum_m mu_tot(m, E_k) L_m after it.  Almost every lattice cell has a single
// material; those steps add the interpolated density into one register
// accumulator that is written to the lane's LDS slot of its material only when
// the material changes.  Mixed cells add each corner's share to its
// material's slot.
#pragma once

#include "gdrr_device.h"

namespace gdrr {

constexpr int kRtBlock = 256;     // 16 x 16 pixels; each wavefront an 8 x 8 quadrant
constexpr int kXcds = 8;          // workgroup i runs on XCD i mod 8

struct RtSource {
    const float* fluence;         // [nv][nu] weights w(u) (unnormalised)
    const float* coef;            // [rows][n_spec] phi_k r(E_k) / sum phi (row iu: detector column iu)
    const float* tab;             // [n_spec][n_mat] 0.1 mu_tot(m, E_k): mm of density-length -> optical depth
    const double* inv_wsum;       // 1 / sum_u w(u)
    int n_spec, rows;
};

struct RtParams {
    DVolume vol[GDRR_MAX_VOLUMES];
    RtSource src[GDRR_MAX_SOURCES];
    float dl[GDRR_MAX_VOLUMES];   // interval length per volume, mm
    const DJob* jobs;
    // Work units (runs of consecutive tiles within one tile row of one job),
    // listed XCD by XCD:
    // XCD x owns units [xcd_start[x], xcd_start[x+1]); unit_pref is the
    // running tile count within its XCD's list.
    const int* unit_job;
    const unsigned int* unit_first;    // first tile of the unit within its job
    const unsigned int* unit_pref;
    unsigned int xcd_start[kXcds + 1];
    unsigned int xcd_tiles[kXcds];
    const long long* out_off;     // [n_jobs] element offset of each job's image in out
    double* out;
    int n_mat, interp, accumulate;
};

// Slab clip of t in [t0, t1] to lo <= s + t d <= hi.
__device__ __forceinline__ void rt_slab(float s, float d, float lo, float hi, float& t0, float& t1) {
    if (d != 0.0f) {
        const float ta = (lo - s) / d, tb = (hi - s) / d;
        t0 = fmaxf(t0, fminf(ta, tb));
        t1 = fminf(t1, fmaxf(ta, tb));
    } else if (s < lo || s > hi) {
        t1 = -1.0f;
    }
}

__global__ __launch_bounds__(kRtBlock) void raytrace_kernel(RtParams P) {
    extern __shared__ float rt_lds[];          // [n_mat][kRtBlock]: the lanes' L_m
    // Workgroups are dealt to the XCDs in turn; each XCD walks its own list of
    // units in order.  The host orders the units by phantom, then tile row,
    // then job, and deals them round the XCDs, so at any time the whole chip
    // traces one band of detector rows -- one slab of the phantom -- over all
    // that phantom's projections.
    const unsigned int x = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
    if (slot >= P.xcd_tiles[x]) return;         // whole workgroup; no barrier in this kernel
    int lo = (int)P.xcd_start[x], hi = (int)P.xcd_start[x + 1] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.unit_pref[mid] <= slot) lo = mid; else hi = mid - 1;
    }
    const DJob& J = P.jobs[P.unit_job[lo]];
    const unsigned int local = P.unit_first[lo] + (slot - P.unit_pref[lo]);
    const int tiles_u = (J.nu + 15) >> 4;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int iu = (int)(local % tiles_u) * 16 + (w & 1) * 8 + (l & 7);
    const int iv = (int)(local / tiles_u) * 16 + (w >> 1) * 8 + (l >> 3);
    if (iu >= J.nu || iv >= J.nv) return;

    float* Lm = rt_lds + threadIdx.x;
    for (int m = 0; m < P.n_mat; ++m) Lm[m * kRtBlock] = 0.0f;

    const DVolume& V = P.vol[J.vol];
    const float uc = ((float)iu + 0.5f - 0.5f * (float)J.nu) * J.du;
    const float vc = ((float)iv + 0.5f - 0.5f * (float)J.nv) * J.dv;
    float dx = J.Px + uc * J.ux - J.Sx;
    float dy = J.Py + uc * J.uy - J.Sy;
    float dz = J.Pz + vc - J.Sz;                       // v axis = +z
    const float len = sqrtf(dx * dx + dy * dy + dz * dz);
    dx /= len; dy /= len; dz /= len;
    float t0 = 0.0f, t1 = len;
    rt_slab(J.Sx, dx, V.lox, V.hix, t0, t1);
    rt_slab(J.Sy, dy, V.loy, V.hiy, t0, t1);
    rt_slab(J.Sz, dz, V.loz, V.hiz, t0, t1);

    if (t0 < t1) {
        const float dl = P.dl[J.vol];
        // the volume's fields in registers for the march
        const CellRec* __restrict__ cells = V.cells;       // 32-byte records, materials in the sign bits
        const float* __restrict__ dens = V.density;
        const uint8_t* __restrict__ mats = V.material;
        const int nx = V.nx, ny = V.ny, nz = V.nz, nxy = V.nxy, cx = V.cx, cxy = V.cxy;
        // the ray in lattice coordinates (voxel units, cell corners at integers):
        // g(t) = g0 + t gd per axis, one FMA per axis and interval
        const float g0x = (J.Sx - V.lox) * V.idx - 0.5f, g0y = (J.Sy - V.loy) * V.idy - 0.5f,
                    g0z = (J.Sz - V.loz) * V.idz - 0.5f;
        const float gdx = dx * V.idx, gdy = dy * V.idy, gdz = dz * V.idz;
        const int n_mat = P.n_mat;
        const bool interp = P.interp != 0;
        float acc = 0.0f;
        int cur = -1;
        // Interval j: its length inside the box h (<= 0 outside the ray's part
        // in the box), the lattice cell (ix, iy, iz) of its midpoint (clamped)
        // and the fractions there.
        auto interval = [&](int j, float& h, float& fx, float& fy, float& fz, int& ix, int& iy, int& iz) {
            const float a = fmaxf((float)j * dl, t0), e = fminf((float)(j + 1) * dl, t1);
            h = e - a;
            const float t = 0.5f * (a + e);
            const float gx = g0x + t * gdx, gy = g0y + t * gdy, gz = g0z + t * gdz;
            const float fx0 = floorf(gx), fy0 = floorf(gy), fz0 = floorf(gz);
            ix = min(max((int)fx0, -1), nx - 1);
            iy = min(max((int)fy0, -1), ny - 1);
            iz = min(max((int)fz0, -1), nz - 1);
            fx = fminf(fmaxf(gx - fx0, 0.0f), 1.0f);
            fy = fminf(fmaxf(gy - fy0, 0.0f), 1.0f);
            fz = fminf(fmaxf(gz - fz0, 0.0f), 1.0f);
        };
        // one interval of slack on both sides (rounding of t / dl); empty ones have h <= 0
        const int jb = (int)floorf(t0 / dl) - 1, je = (int)ceilf(t1 / dl) + 1;
        if (!interp) {
            for (int j = jb; j < je; ++j) {
                float h, fx, fy, fz;
                int ix, iy, iz;
                interval(j, h, fx, fy, fz, ix, iy, iz);
                if (!(h > 0.0f)) continue;
                // containing voxel: the cell corner nearest to the point
                const int vx = min(max(ix + (fx >= 0.5f ? 1 : 0), 0), nx - 1);
                const int vy = min(max(iy + (fy >= 0.5f ? 1 : 0), 0), ny - 1);
                const int vz = min(max(iz + (fz >= 0.5f ? 1 : 0), 0), nz - 1);
                const long long v = (long long)vz * nxy + (long long)vy * nx + vx;
                const int m = min((int)mats[v], n_mat - 1);
                if (m != cur) {
                    if (cur >= 0) Lm[cur * kRtBlock] += acc;
                    cur = m;
                    acc = 0.0f;
                }
                acc += h * clean_density(dens[v]);
            }
        } else {
            // software-pipelined: the next interval's cell record is read while
            // this one is summed
            float h, fx, fy, fz;
            int ix, iy, iz;
            interval(jb, h, fx, fy, fz, ix, iy, iz);
            const int cell = (iz + 1) * cxy + (iy + 1) * cx + (ix + 1);
            float4 d0 = *reinterpret_cast<const float4*>(&cells[cell].d[0]);
            float4 d1 = *reinterpret_cast<const float4*>(&cells[cell].d[4]);
            for (int j = jb; j < je; ++j) {
                float hn, fxn, fyn, fzn;
                int jx, jy, jz;
                interval(j + 1, hn, fxn, fyn, fzn, jx, jy, jz);
                const int celln = (jz + 1) * cxy + (jy + 1) * cx + (jx + 1);
                const float4 n0 = *reinterpret_cast<const float4*>(&cells[celln].d[0]);
                const float4 n1 = *reinterpret_cast<const float4*>(&cells[celln].d[4]);
                if (h > 0.0f) {
                    const uint32_t s0 = __float_as_uint(d0.x), s1 = __float_as_uint(d0.y), s2 = __float_as_uint(d0.z),
                                   s3 = __float_as_uint(d0.w), s4 = __float_as_uint(d1.x);
                    // the densities without their flag bits
                    const float c0 = fabsf(d0.x), c1 = fabsf(d0.y), c2 = fabsf(d0.z), c3 = fabsf(d0.w);
                    const float c4 = fabsf(d1.x), c5 = d1.y, c6 = d1.z, c7 = d1.w;
                    if (!(s0 >> 31)) {
                        const float a00 = c0 + fx * (c1 - c0), a01 = c2 + fx * (c3 - c2);
                        const float a10 = c4 + fx * (c5 - c4), a11 = c6 + fx * (c7 - c6);
                        const float b0 = a00 + fy * (a01 - a00), b1 = a10 + fy * (a11 - a10);
                        const int m = (int)((s1 >> 31) | ((s2 >> 30) & 2u) | ((s3 >> 29) & 4u) | ((s4 >> 28) & 8u));
                        if (m != cur) {
                            if (cur >= 0) Lm[cur * kRtBlock] += acc;
                            cur = m;
                            acc = 0.0f;
                        }
                        acc += h * (b0 + fz * (b1 - b0));
                    } else {
                        const float gx0 = 1.0f - fx, gy0 = 1.0f - fy, gz0 = 1.0f - fz;
                        const float wz0 = h * gz0, wz1 = h * fz;
                        const float cd[8] = {c0, c1, c2, c3, c4, c5, c6, c7};
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const int x = min(max(ix + (c & 1), 0), nx - 1);
                            const int y = min(max(iy + ((c >> 1) & 1), 0), ny - 1);
                            const int z = min(max(iz + (c >> 2), 0), nz - 1);
                            const int m = min((int)mats[(long long)z * nxy + (long long)y * nx + x], n_mat - 1);
                            const float wc = (c & 1 ? fx : gx0) * (c & 2 ? fy : gy0) * (c & 4 ? wz1 : wz0);
                            Lm[m * kRtBlock] += wc * cd[c];
                        }
                    }
                }
                h = hn; fx = fxn; fy = fyn; fz = fzn;
                ix = jx; iy = jy; iz = jz;
                d0 = n0; d1 = n1;
            }
        }
        if (cur >= 0) Lm[cur * kRtBlock] += acc;
    }

    float Lr[GDRR_MAX_MATERIALS];
#pragma unroll
    for (int m = 0; m < GDRR_MAX_MATERIALS; ++m) Lr[m] = m < P.n_mat ? Lm[m * kRtBlock] : 0.0f;
    const RtSource& S = P.src[J.src];
    const float* coef = S.coef + (S.rows > 1 ? iu * S.n_spec : 0);
    float sum = 0.0f;
    for (int k = 0; k < S.n_spec; ++k) {
        const float* row = S.tab + k * P.n_mat;
        float tau = 0.0f;
#pragma unroll
        for (int m = 0; m < GDRR_MAX_MATERIALS; ++m)
            if (m < P.n_mat) tau += row[m] * Lr[m];
        sum += coef[k] * expf(-tau);
    }
    const int pix = iv * J.nu + iu;
    const double val = (double)S.fluence[pix] * S.inv_wsum[0] * (double)sum;
    double* o = P.out + P.out_off[J.index] + pix;
    *o = P.accumulate ? *o + val : val;
}

// Input check of a volume the ray tracer reads without cell records (no
// interpolation): the status bits of invalid densities and materials.
struct VolCheckParams {
    const float* density;
    const uint8_t* material;
    long long n;
    int n_mat;
    unsigned int* error;
};

__global__ __launch_bounds__(256) void volume_check_kernel(VolCheckParams C) {
    unsigned int err = 0u;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < C.n; v += (long long)gridDim.x * blockDim.x) {
        if (!density_ok(C.density[v])) err |= kErrDensity;
        if (C.material[v] >= C.n_mat) err |= kErrMaterial;
    }
    if (err) atomicOr(C.error, err);
}

// Per source: the channel weights phi_k r(E_k) / sum phi (workgroup r: row r
// of a joint source), the table 0.1 mu_tot(m, E_k) (linear in E between grid
// points) and 1 / sum w (workgroup 0).
struct RtPrepParams {
    const float* spec_e;
    const float* spec_p;          // [rows][n_spec]
    const float* fluence;
    int n_spec, npix;
    const float* mu_mass;         // [n_mat][n_e][3]
    const float* response;        // [n_e] or null
    int n_mat, n_e;
    double e0, de;
    float* coef;
    float* tab;
    double* inv_wsum;
    unsigned int* error;          // input-error bits (invalid spectrum or fluence weights)
};

__global__ __launch_bounds__(256) void raytrace_prep_kernel(RtPrepParams R) {
    __shared__ double red[2][256];
    const int row = blockIdx.x;
    const float* phi = R.spec_p + (size_t)row * R.n_spec;
    float* coef = R.coef + (size_t)row * R.n_spec;
    double sp = 0.0, sw = 0.0;
    bool bad = false;
    for (int k = threadIdx.x; k < R.n_spec; k += 256) {
        const double x = (double)phi[k];
        bad = bad || !(x >= 0.0) || isinf(x);
        sp += x;
    }
    if (row == 0)
        for (int k = threadIdx.x; k < R.npix; k += 256) {
            const double x = (double)R.fluence[k];
            bad = bad || !(x >= 0.0) || isinf(x);
            sw += x;
        }
    if (bad) atomicOr(R.error, kErrWeights);
    red[0][threadIdx.x] = sp;
    red[1][threadIdx.x] = sw;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    const double psum = red[0][0], wsum = red[1][0];
    if (row == 0 && threadIdx.x == 0) R.inv_wsum[0] = wsum > 0.0 ? 1.0 / wsum : 0.0;
    if (threadIdx.x == 0 && (!(psum > 0.0) || (row == 0 && !(wsum > 0.0)))) atomicOr(R.error, kErrWeights);
    for (int k = threadIdx.x; k < R.n_spec; k += 256) {
        const double E = (double)R.spec_e[k];
        const double g = (E - R.e0) / R.de;
        int j = (int)floor(g);
        j = j < 0 ? 0 : (j > R.n_e - 2 ? R.n_e - 2 : j);
        const double f = g - (double)j;
        double r = E;
        if (R.response) r = (double)R.response[j] + f * ((double)R.response[j + 1] - (double)R.response[j]);
        coef[k] = psum > 0.0 ? (float)((double)phi[k] / psum * r) : 0.0f;
        if (row != 0) continue;
        for (int m = 0; m < R.n_mat; ++m) {
            const float* a = R.mu_mass + ((size_t)m * R.n_e + j) * 3;
            const double ta = (double)a[0] + (double)a[1] + (double)a[2];
            const double tb = (double)a[3] + (double)a[4] + (double)a[5];
            R.tab[k * R.n_mat + m] = (float)(0.1 * (ta + f * (tb - ta)));
        }
    }
}

}  // namespace gdrr
