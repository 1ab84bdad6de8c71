// Kernels of the gfx950 Monte Carlo projection step (Step 2 of gDRR,
// Sec. 2.4 of arXiv:1204.6367) and their launch parameters.
//
// One wavefront lane carries one photon history at a time.  Lanes live for
// the whole launch (a persistent grid): a lane whose history ends takes the
// next photon index of its wavefront's chunk, and wavefronts take chunks of
// (job, photon range) from one atomic dispenser, so all the angles and
// phantoms of a batch run in the same launch.  Each loop iteration has three
// phases -- refill (start new histories), flight (one Woodcock step of every
// flying lane) and collision (interaction sampling) -- and the two rare ones
// run only when enough lanes wait for them (`defer` for refills, `cdefer` for
// collisions), so that the wavefront's SIMD lanes mostly execute the same
// free-flight code.
#pragma once

#include "gdrr_device.h"

namespace gdrr {

enum : int { kDead = 0, kFly = 1, kColl = 2 };
enum : int { kModeForward = 0, kModeTrace = 1, kModeBackward = 2 };

constexpr int kMaxVol = 8;
constexpr int kMaxSrc = 8;

struct KParams {
    DVolume vol[kMaxVol];
    DSource src[kMaxSrc];
    const DJob* jobs;
    const unsigned long long* chunk_prefix;   // [n_jobs + 1]: first chunk of each job
    unsigned long long* counter;              // [0] chunk dispenser
    unsigned long long* tally;                // fixed-point tallies
    const float* mu_mass;                     // [n_mat][n_e][3]
    const float* response;                    // [n_e] or null
    const float* majorants;                   // [n_vols][n_e - 1], 1/cm
    unsigned long long total_chunks;
    int n_jobs, n_vols, n_mat, n_e;
    int n_maj;                                // volumes whose single-majorant table is staged in LDS (0 or n_vols)
    int tot_rows;                             // rows per energy of the LDS attenuation table (>= n_mat)
    int mask_rows;                            // rows after the materials' kept for material sets of cubes
    float e0, inv_de, e_max, e_cut, x0;
    uint32_t k0, k1;
    uint32_t flags;
    int chunk, defer, cdefer;
    // diagnostics (trace mode)
    int8_t* t_cls;
    int32_t* t_pixel;
    float* t_e;
    int32_t* t_steps;
    int32_t* t_nc;
    int32_t* t_nr;
    // adjoint (backward mode)
    const double* adj;
    double* grad;
    // local majorants staged in LDS after the tables: per volume the offset (records) or -1
    int macro_lds[kMaxVol];
    int macro_lds_n;          // records staged in total
};

// LDS holds what every free flight reads: the total attenuation per
// (grid point, row) and the majorants; interaction-type splits are read from
// the global table at the (rarer) real collisions.  Rows 0 .. n_mat-1 are the
// materials; with local majorants the rows after them hold, for the material
// sets of several materials that cubes have, the chord between the largest
// mu_tot of the set at the interval's two grid energies (the set's bound).
__host__ __device__ inline size_t table_floats2(int tot_rows, int n_e, int n_maj) {
    return (size_t)tot_rows * n_e + (size_t)n_maj * (n_e - 1);
}

// Bytes of cube records per cube in LDS: the all-local instantiation keeps one
// word (the density bound, whose low 5 bits are zero, with a table row there),
// the others the record as built.
__host__ __device__ inline size_t lds_record_bytes(int local_kind) { return local_kind == 3 ? 4 : 8; }

// Per wavefront, after the tables and cube records: 64 slots of source draws
// (16 bytes each), starting at a 16-byte boundary.
__host__ __device__ inline size_t draw_slots_offset_bytes(size_t tables_and_records_bytes) {
    return (tables_and_records_bytes + 15) & ~(size_t)15;
}

// The row field of an all-local LDS record: 31 = no row (the bound then comes
// from the cube's material mask in its global record).
constexpr uint32_t kNoRow = 31u;

struct Tables {
    const float2* tot;    // [j][row] (tot_j, tot_j+1 - tot_j): the rows of one interval side by side
    const float2* maj;    // [v][j] (mbar, mean free path per unit of -ln u, mm)
};

// Energy-interval cache of a photon: interval index, fraction, majorant, mfp.
struct ECache {
    int j;
    float f, mbar, mfp;
};

// vol_off < 0: the volume tracks with local majorants and has no staged table.
__device__ __forceinline__ ECache energy_cache(const KParams& P, const Tables& T, int vol_off, float E) {
    const float g = (E - P.e0) * P.inv_de;
    int j = (int)floorf(g);
    j = j < 0 ? 0 : (j > P.n_e - 2 ? P.n_e - 2 : j);
    const float2 m = vol_off >= 0 ? T.maj[vol_off + j] : make_float2(0.0f, 0.0f);
    return ECache{j, g - (float)j, m.x, m.y};
}

// Density at x (tri-linear on the voxel-centre lattice, clamped to the edge
// voxels; or the containing voxel's) and the containing voxel's material, from
// the cell records (one 32-byte record; the voxel array only for the material
// of a cell whose corners differ).
// The containing voxel is corner (f >= 1/2) of the cell along each axis.
__device__ __forceinline__ float cell_density(const DVolume& V, bool interp, float px, float py, float pz,
                                              int& mat) {
    const float hx = (px - V.lox) * V.idx - 0.5f, hy = (py - V.loy) * V.idy - 0.5f, hz = (pz - V.loz) * V.idz - 0.5f;
    const float fx0 = floorf(hx), fy0 = floorf(hy), fz0 = floorf(hz);
    const int ix = min(max((int)fx0, -1), V.nx - 1);
    const int iy = min(max((int)fy0, -1), V.ny - 1);
    const int iz = min(max((int)fz0, -1), V.nz - 1);
    const float fx = fminf(fmaxf(hx - fx0, 0.0f), 1.0f);
    const float fy = fminf(fmaxf(hy - fy0, 0.0f), 1.0f);
    const float fz = fminf(fmaxf(hz - fz0, 0.0f), 1.0f);
    const CellRec* r = V.cells + ((iz + 1) * V.cxy + (iy + 1) * V.cx + (ix + 1));
    const float4 lo4 = *reinterpret_cast<const float4*>(&r->d[0]);
    const float4 hi4 = *reinterpret_cast<const float4*>(&r->d[4]);
    const int bits = (fx >= 0.5f ? 1 : 0) | (fy >= 0.5f ? 2 : 0) | (fz >= 0.5f ? 4 : 0);
    const uint32_t s0 = __float_as_uint(lo4.x);
    if (!(s0 >> 31)) {
        mat = (int)((__float_as_uint(lo4.y) >> 31) | ((__float_as_uint(lo4.z) >> 30) & 2u) |
                    ((__float_as_uint(lo4.w) >> 29) & 4u) | ((__float_as_uint(hi4.x) >> 28) & 8u));
    } else {
        const int vx = min(max(ix + (bits & 1), 0), V.nx - 1);
        const int vy = min(max(iy + ((bits >> 1) & 1), 0), V.ny - 1);
        const int vz = min(max(iz + (bits >> 2), 0), V.nz - 1);
        mat = V.material[vz * V.nxy + vy * V.nx + vx];
    }
    const float c0 = fabsf(lo4.x), c1 = fabsf(lo4.y), c2 = fabsf(lo4.z), c3 = fabsf(lo4.w);
    const float c4 = fabsf(hi4.x), c5 = hi4.y, c6 = hi4.z, c7 = hi4.w;
    if (!interp) {
        const int b2 = bits & 3;
        return bits & 4 ? (b2 == 0 ? c4 : (b2 == 1 ? c5 : (b2 == 2 ? c6 : c7)))
                        : (b2 == 0 ? c0 : (b2 == 1 ? c1 : (b2 == 2 ? c2 : c3)));
    }
    const float a00 = c0 + fx * (c1 - c0), a01 = c2 + fx * (c3 - c2);
    const float a10 = c4 + fx * (c5 - c4), a11 = c6 + fx * (c7 - c6);
    const float b0 = a00 + fy * (a01 - a00), b1 = a10 + fy * (a11 - a10);
    return b0 + fz * (b1 - b0);
}

// (read from global memory: one lookup per scored photon; j <= n_e - 2)
__device__ __forceinline__ float response_at(const KParams& P, const Tables& T, const ECache& ec, float E) {
    if (!P.response) return E;
    const float r0 = P.response[ec.j], r1 = P.response[ec.j + 1];
    return r0 + ec.f * (r1 - r0);
}

// Per-lane photon state.
struct Photon {
    float px, py, pz, dx, dy, dz, E, trem;
    uint32_t pid, step, jid;   // photon index, free flights so far, Philox job word
    int job;                   // index into the job table
    int pix0;                  // sampled aim pixel (the pixel of a primary)
    uint32_t nsc;              // Compton count | Rayleigh count << 16
    int st;
    bool passb;                // adjoint: second (visiting) pass
    ECache ec;
    uint32_t pair;             // flight pairs opened so far (Philox step of the flight block)
    float sel;                 // pending collision: ladder / rho, compared with mu_R and mu_R + mu_C
    int pm;                    // pending collision: material
    double w;                  // adjoint weight of the history
};

// Source photon (Sec. 2.1/2.4), in two parts.  The draw: aim pixel and energy
// channel by inverse CDF (the energy from the row of the pixel's column for a
// joint source) and the two jitter words, from photon `pid`'s step-0 blocks
// alone, so that a wavefront can draw for the next photons of its chunk all at
// once.  Returns (pixel, channel, jitter word u, jitter word v).
__device__ __forceinline__ uint4 draw_source(const KParams& P, int job, uint32_t pid) {
    const DJob& J = P.jobs[job];
    const DSource& S = P.src[J.src];
    const Block b0 = philox(pid, J.job_id, 0u, 0u, P.k0, P.k1);
    const Block b1 = philox(pid, J.job_id, 0u, 1u, P.k0, P.k1);
    const int kf = sample_cdf(S.flu_cdf, S.flu_guide, S.npix, S.flu_k, u53(b0.z, b0.w));
    const int iu = kf - (kf / J.nu) * J.nu;
    const int row = S.spec_rows > 1 ? iu : 0;
    const int ke = sample_cdf(S.spec_cdf + (size_t)row * S.n_spec, S.spec_guide + (size_t)row * S.spec_k, S.n_spec,
                              S.spec_k, u53(b0.x, b0.y));
    return make_uint4((uint32_t)kf, (uint32_t)ke, b1.x, b1.y);
}

// The rest of the start: aim point uniform inside the pixel, straight line from
// S to the phantom.  Returns true if the photon enters the phantom; otherwise
// it reaches its aim pixel unscattered.
__device__ __forceinline__ bool start_from_draw(const KParams& P, const Tables& T, const DVolume& V, int vol_off,
                                                Photon& ph, uint4 d) {
    const DJob& J = P.jobs[ph.job];
    const DSource& S = P.src[J.src];
    const int kf = (int)d.x, ke = (int)d.y;
    const int iv = kf / J.nu, iu = kf - iv * J.nu;
    const float uc = ((float)iu + u24(d.z) - 0.5f * (float)J.nu) * J.du;
    const float vc = ((float)iv + u24(d.w) - 0.5f * (float)J.nv) * J.dv;
    float dx = J.Px + uc * J.ux - J.Sx;
    float dy = J.Py + uc * J.uy - J.Sy;
    float dz = J.Pz + uc * J.uz + vc - J.Sz;
    const float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
    dx *= inv; dy *= inv; dz *= inv;
    ph.dx = dx; ph.dy = dy; ph.dz = dz;
    ph.E = fminf(fmaxf(S.spec_e[ke], P.e0), P.e_max);
    ph.ec = energy_cache(P, T, vol_off, ph.E);
    ph.step = 0;
    ph.pair = 0;
    ph.nsc = 0;
    ph.pix0 = kf;
    float tin, tout;
    if (box_entry(V, J.Sx, J.Sy, J.Sz, dx, dy, dz, tin, tout)) {
        ph.px = J.Sx + tin * dx;
        ph.py = J.Sy + tin * dy;
        ph.pz = J.Sz + tin * dz;
        ph.trem = tout - tin;
        return true;
    }
    return false;
}

__device__ __forceinline__ bool start_photon(const KParams& P, const Tables& T, const DVolume& V, int vol_off,
                                             Photon& ph) {
    return start_from_draw(P, T, V, vol_off, ph, draw_source(P, ph.job, ph.pid));
}

// Detector hit of a photon leaving the phantom: the primary pixel for an
// unscattered photon, else the intersection of its line with the detector
// plane (half-open pixels).  Returns the class (primary / scatter / missed).
__device__ __forceinline__ int detector_pixel(const DJob& J, const Photon& ph, int& pixel) {
    if (ph.nsc == 0) { pixel = ph.pix0; return kPrimary; }
    const float dn = ph.dx * J.nx + ph.dy * J.ny + ph.dz * J.nz;
    pixel = -1;
    if (!(dn > 0.0f)) return kMissed;
    const float t = ((J.Px - ph.px) * J.nx + (J.Py - ph.py) * J.ny + (J.Pz - ph.pz) * J.nz) * fast_rcp(dn);
    if (!(t >= 0.0f)) return kMissed;
    const float hx = ph.px + t * ph.dx - J.Px, hy = ph.py + t * ph.dy - J.Py, hz = ph.pz + t * ph.dz - J.Pz;
    const float fu = (hx * J.ux + hy * J.uy + hz * J.uz) * J.idu + 0.5f * (float)J.nu;
    const float fv = hz * J.idv + 0.5f * (float)J.nv;
    const float ku = floorf(fu), kv = floorf(fv);
    if (ku >= 0.0f && ku < (float)J.nu && kv >= 0.0f && kv < (float)J.nv) {
        pixel = (int)kv * J.nu + (int)ku;
        return kScatter;
    }
    return kMissed;
}

__device__ __forceinline__ bool counts_as_scatter(uint32_t flags, uint32_t nsc) {
    const uint32_t nc = nsc & 0xFFFFu, nr = nsc >> 16;
    if (flags & 16u) return nc == 1 && nr == 0;
    if (flags & 8u) return nc + nr == 1;
    return true;
}

__device__ __forceinline__ void tally_add(const KParams& P, const DJob& J, int cls, int pixel, float r) {
    const int npix = J.nu * J.nv;
    unsigned long long* t = P.tally + J.tally_off + (cls == kPrimary ? 0 : 2 * npix) + pixel;
    const double rd = (double)r;
    atomicAdd(t, (unsigned long long)__double2ll_rn(rd * kQ1));
    if (P.flags & 2u) atomicAdd(t + npix, (unsigned long long)__double2ll_rn(rd * rd * kQ2));
}

template <int MODE>
__device__ __forceinline__ void trace_out(const KParams& P, const Photon& ph, int cls, int pixel) {
    if (MODE != kModeTrace) return;
    const uint32_t i = ph.pid - P.jobs[ph.job].first;
    if (P.t_cls) P.t_cls[i] = (int8_t)cls;
    if (P.t_pixel) P.t_pixel[i] = pixel;
    if (P.t_e) P.t_e[i] = ph.E;
    if (P.t_steps) P.t_steps[i] = (int32_t)ph.step;
    if (P.t_nc) P.t_nc[i] = (int32_t)(ph.nsc & 0xFFFFu);
    if (P.t_nr) P.t_nr[i] = (int32_t)(ph.nsc >> 16);
}

// The end of a history: score it (forward), record it (trace) or turn it
// into the adjoint's visiting pass (backward).
template <int MODE>
__device__ __forceinline__ void finish(const KParams& P, const Tables& T, const DVolume& V, int vol_off,
                                      Photon& ph, int cls, int pixel) {
    const DJob& J = P.jobs[ph.job];
    const bool counted = cls == kPrimary || (cls == kScatter && counts_as_scatter(P.flags, ph.nsc));
    if (MODE == kModeTrace) trace_out<MODE>(P, ph, cls, pixel);
    if (MODE == kModeForward) {
        if (counted) tally_add(P, J, cls, pixel, fminf(fmaxf(response_at(P, T, ph.ec, ph.E), 0.0f), kMaxResponse));
        ph.st = kDead;
        return;
    }
    if (MODE == kModeBackward && !ph.passb && counted) {
        const double n = (double)J.n_lo + 4294967296.0 * (double)J.n_hi;
        const int npix = J.nu * J.nv;
        const double a = P.adj[J.adj_off + (cls == kPrimary ? 0 : npix) + pixel];
        const float r = fminf(fmaxf(response_at(P, T, ph.ec, ph.E), 0.0f), kMaxResponse);
        const double w = a * (double)r / n;
        if (w != 0.0) {
            ph.w = w;
            ph.passb = true;
            ph.st = start_photon(P, T, V, vol_off, ph) ? kFly : kDead;
            return;
        }
    }
    ph.st = kDead;
}

// Score-function terms of one tentative collision (adjoint, second pass):
// base w_v / rho (real) or -mu_tot w_v / (mbar - rho mu_tot) (null) times the
// history's weight, added to every stencil voxel v.  The stencil -- the eight
// lattice corners of the interpolation (clamped to the edge voxels, so a
// clamped corner repeats a voxel) and their weights, or the containing voxel --
// comes from the position alone: rho is the density the collision test has
// just computed, so no voxel is read again.
__device__ __forceinline__ void visit(const KParams& P, const DVolume& V, bool interp, const Photon& ph,
                                      bool real, float rho, float tot, float mbar) {
    const float base = real ? 1.0f / rho : -tot / (mbar - rho * tot);
    const float gx = (ph.px - V.lox) * V.idx, gy = (ph.py - V.loy) * V.idy, gz = (ph.pz - V.loz) * V.idz;
    if (!interp) {
        const int cx = min(max((int)floorf(gx), 0), V.nx - 1);
        const int cy = min(max((int)floorf(gy), 0), V.ny - 1);
        const int cz = min(max((int)floorf(gz), 0), V.nz - 1);
        if (base != 0.0f) unsafeAtomicAdd(P.grad + (cz * V.nxy + cy * V.nx + cx), ph.w * (double)base);
        return;
    }
    const float hx = gx - 0.5f, hy = gy - 0.5f, hz = gz - 0.5f;
    const float fx0 = floorf(hx), fy0 = floorf(hy), fz0 = floorf(hz);
    const float fx = hx - fx0, fy = hy - fy0, fz = hz - fz0;
    const int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
    const int x0 = min(max(ix, 0), V.nx - 1), x1 = min(max(ix + 1, 0), V.nx - 1);
    const int y0 = min(max(iy, 0), V.ny - 1) * V.nx, y1 = min(max(iy + 1, 0), V.ny - 1) * V.nx;
    const int z0 = min(max(iz, 0), V.nz - 1) * V.nxy, z1 = min(max(iz + 1, 0), V.nz - 1) * V.nxy;
    const float gx0 = 1.0f - fx, gy0 = 1.0f - fy, gz0 = 1.0f - fz;
    const int vox[8] = {z0 + y0 + x0, z0 + y0 + x1, z0 + y1 + x0, z0 + y1 + x1,
                        z1 + y0 + x0, z1 + y0 + x1, z1 + y1 + x0, z1 + y1 + x1};
    const float wt[8] = {gx0 * gy0 * gz0, fx * gy0 * gz0, gx0 * fy * gz0, fx * fy * gz0,
                         gx0 * gy0 * fz, fx * gy0 * fz, gx0 * fy * fz, fx * fy * fz};
    const double wb = ph.w * (double)base;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (wt[k] != 0.0f) unsafeAtomicAdd(P.grad + vox[k], wb * (double)wt[k]);
}

// One Woodcock free flight with uniforms (ra, rb): flight length -ln(u)/mbar,
// then the collision ladder.  Returns true after a null collision (the photon
// flies on); escape, a real collision or the step limit return false.
template <int MODE>
__device__ __forceinline__ bool flight(const KParams& P, const Tables& T, const DVolume& V, int vo, bool interp,
                                       Photon& ph, uint32_t ra, uint32_t rb) {
    if (ph.step >= kMaxSteps) {                          // step limit: the history is lost
        if (MODE == kModeTrace) trace_out<MODE>(P, ph, kLost, -1);
        ph.st = kDead;
        return false;
    }
    ph.step += 1;
    const float s = -fast_log(u24(ra)) * ph.ec.mfp;
    if (!(s < ph.trem)) {
        int pixel;
        const int cls = detector_pixel(P.jobs[ph.job], ph, pixel);
        finish<MODE>(P, T, V, vo, ph, cls, pixel);
        return false;
    }
    ph.px += s * ph.dx;
    ph.py += s * ph.dy;
    ph.pz += s * ph.dz;
    ph.trem -= s;
    int m;
    const float rho = cell_density(V, interp, ph.px, ph.py, ph.pz, m);
    m = m < P.n_mat ? m : P.n_mat - 1;
    const float2 tt = T.tot[ph.ec.j * P.tot_rows + m];
    const float tot = tt.x + ph.ec.f * tt.y;
    // one uniform on [0, mbar): real below mu = rho tot, then the type ladder
    const float ladder = u24(rb) * ph.ec.mbar;
    const bool real = ladder < rho * tot;
    if (MODE == kModeBackward && ph.passb) visit(P, V, interp, ph, real, rho, tot, ph.ec.mbar);
    if (real) {
        ph.st = kColl;
        ph.sel = ladder * fast_rcp(rho);
        ph.pm = m;
        return false;
    }
    return true;
}

// Material factor of a cube's bound from its material mask, tot pointing at the
// row of the photon's energy interval j: the chord between the largest mu_tot
// of the cube's materials at E_j and at E_j+1 (the next interval's rows; j <=
// n_e - 2), the same float operations as a row of the set's (stage_records_rows),
// so that a cube's bound does not depend on where it is read from.
__device__ __forceinline__ float set_bound(const float2* tot, int rows, uint32_t mask, float f) {
    float t0 = 0.0f, t1 = 0.0f;
    for (; mask; mask &= mask - 1u) {
        const int m = __builtin_ctz(mask);
        const float a = tot[m].x, b = tot[rows + m].x;
        t0 = a > t0 ? a : t0;
        t1 = b > t1 ? b : t1;
    }
    return t0 + f * (t1 - t0);
}

// One free flight under local majorants (uniforms ra, rb): an optical depth
// tau = -ln(u) is spent cube by cube along the line, each cube at its own
// bound mbar_B = (1 + margin) rho_max(B) max_{m in B} mu_tot(m, E); where tau
// runs out the collision ladder runs against that cube's bound; leaving the
// last cube is an escape.  Returns true after a null collision.  REC: where
// the cube records are read: 0 = global memory; 1 = their LDS copy lds_rec
// (a separate instantiation, so that the load is an LDS read, not a generic
// one); 2 = the all-local LDS words (density bound and table row; a cube
// without a row takes its material mask from the global record).
template <int MODE, int REC>
__device__ __forceinline__ bool flight_local(const KParams& P, const Tables& T, const DVolume& V, int vo,
                                             bool interp, Photon& ph, uint32_t ra, uint32_t rb,
                                             const void* lds_rec) {
    if (ph.step >= kMaxSteps) {
        if (MODE == kModeTrace) trace_out<MODE>(P, ph, kLost, -1);
        ph.st = kDead;
        return false;
    }
    ph.step += 1;
    float tau = -fast_log(u24(ra));
    int bx = min(max((int)floorf((ph.px - V.lox) * V.imx), 0), V.mnx - 1);
    int by = min(max((int)floorf((ph.py - V.loy) * V.imy), 0), V.mny - 1);
    int bz = min(max((int)floorf((ph.pz - V.loz) * V.imz), 0), V.mnz - 1);
    // Distances along the line (from the flight's start) to the next cube face
    // on each axis, advanced by one cube edge per crossing (Amanatides-Woo).
    const float rx = ph.dx != 0.0f ? fast_rcp(ph.dx) : 0.0f;
    const float ry = ph.dy != 0.0f ? fast_rcp(ph.dy) : 0.0f;
    const float rz = ph.dz != 0.0f ? fast_rcp(ph.dz) : 0.0f;
    const int sx = ph.dx > 0.0f ? 1 : (ph.dx < 0.0f ? -1 : 0);
    const int sy = ph.dy > 0.0f ? 1 : (ph.dy < 0.0f ? -1 : 0);
    const int sz = ph.dz > 0.0f ? 1 : (ph.dz < 0.0f ? -1 : 0);
    // where the line leaves the box through a face on the positive side of an axis (the last
    // cube there may reach past the face); leaving through a negative side is the cube index
    // leaving the grid
    const float tex = fminf(sx > 0 ? (V.hix - ph.px) * rx : INFINITY,
                            fminf(sy > 0 ? (V.hiy - ph.py) * ry : INFINITY, sz > 0 ? (V.hiz - ph.pz) * rz : INFINITY));
    float tmx = sx > 0 ? (V.lox + (float)(bx + 1) * V.mex - ph.px) * rx
              : (sx < 0 ? (V.lox + (float)bx * V.mex - ph.px) * rx : INFINITY);
    float tmy = sy > 0 ? (V.loy + (float)(by + 1) * V.mey - ph.py) * ry
              : (sy < 0 ? (V.loy + (float)by * V.mey - ph.py) * ry : INFINITY);
    float tmz = sz > 0 ? (V.loz + (float)(bz + 1) * V.mez - ph.pz) * rz
              : (sz < 0 ? (V.loz + (float)bz * V.mez - ph.pz) * rz : INFINITY);
    const float dtx = V.mex * fabsf(rx), dty = V.mey * fabsf(ry), dtz = V.mez * fabsf(rz);
    const float2* tot = T.tot + ph.ec.j * P.tot_rows;
    // the cube index moves by one of these per crossing
    const int cix = sx, ciy = sy * V.mnx, ciz = sz * V.mnx * V.mny;
    int ci = (bz * V.mny + by) * V.mnx + bx;
    // REC 2 (at most 512 cubes per axis): crossings left per axis, as in flight_pair_all_local
    uint32_t left = 0u;
    if constexpr (REC == 2)
        left = ((512u + (uint32_t)(sx > 0 ? V.mnx - 1 - bx : (sx < 0 ? bx : 511)))) |
               ((512u + (uint32_t)(sy > 0 ? V.mny - 1 - by : (sy < 0 ? by : 511))) << 10) |
               ((512u + (uint32_t)(sz > 0 ? V.mnz - 1 - bz : (sz < 0 ? bz : 511))) << 20);
    float mb = 0.0f, t = 0.0f;
    bool hit = false;
    // (selects instead of fminf/fmaxf below: no NaN can occur, and these need
    // no canonicalisation of their operands)
    for (;;) {
        float tmax;
        uint32_t rho_bits;
        if constexpr (REC == 2) {
            const uint32_t w = reinterpret_cast<const uint32_t*>(lds_rec)[ci];
            const uint32_t row = w & 31u;
            rho_bits = w & ~31u;
            if (row != kNoRow) {
                const float2 tt = tot[row];
                tmax = tt.x + ph.ec.f * tt.y;
            } else {
                tmax = set_bound(tot, P.tot_rows, V.macro[ci].y, ph.ec.f);
            }
        } else {
            const uint2 rec = REC == 1 ? reinterpret_cast<const uint2*>(lds_rec)[ci] : V.macro[ci];
            rho_bits = rec.x;
            tmax = set_bound(tot, P.tot_rows, rec.y, ph.ec.f);
        }
        mb = __uint_as_float(rho_bits) * tmax;
        const float tnext = fminf(tmx, fminf(tmy, tmz));
        const float tn = tnext < tex ? tnext : tex;                    // the cube's exit, within the box
        const float span = tn - t;
        const float need = 0.1f * mb * (span > 0.0f ? span : 0.0f);   // mbar in 1/cm, lengths in mm
        if (tau < need) {                                                // (need = 0 when mb = 0: tau > 0)
            t += tau * fast_rcp(0.1f * mb);
            hit = true;
            break;
        }
        tau -= need;
        t = tn > t ? tn : t;
        if (!(tn < tex)) break;                                        // left the box
        // the axis of the nearest face (ties to x, then y)
        const bool ax = tmx == tnext, ay = !ax && tmy == tnext, az = !ax && !ay;
        ci += ax ? cix : (ay ? ciy : ciz);
        tmx = ax ? tmx + dtx : tmx;
        tmy = ay ? tmy + dty : tmy;
        tmz = az ? tmz + dtz : tmz;
        if constexpr (REC == 2) {
            constexpr uint32_t kGuards = (1u << 9) | (1u << 19) | (1u << 29);
            left -= ax ? 1u : (ay ? 1u << 10 : 1u << 20);
            if ((left & kGuards) != kGuards) break;                   // left the grid
        } else {
            bx += ax ? sx : 0;
            by += ay ? sy : 0;
            bz += az ? sz : 0;
            if ((unsigned)bx >= (unsigned)V.mnx || (unsigned)by >= (unsigned)V.mny || (unsigned)bz >= (unsigned)V.mnz)
                break;
        }
    }
    ph.px += t * ph.dx;
    ph.py += t * ph.dy;
    ph.pz += t * ph.dz;
    if (!hit) {
        int pixel;
        const int cls = detector_pixel(P.jobs[ph.job], ph, pixel);
        finish<MODE>(P, T, V, vo, ph, cls, pixel);
        return false;
    }
    int m;
    const float rho = cell_density(V, interp, ph.px, ph.py, ph.pz, m);
    m = m < P.n_mat ? m : P.n_mat - 1;
    const float2 tt = T.tot[ph.ec.j * P.tot_rows + m];
    const float tot_m = tt.x + ph.ec.f * tt.y;
    const float ladder = u24(rb) * mb;
    const bool real = ladder < rho * tot_m;
    if (MODE == kModeBackward && ph.passb) visit(P, V, interp, ph, real, rho, tot_m, mb);
    if (real) {
        ph.st = kColl;
        ph.sel = ladder * fast_rcp(rho);
        ph.pm = m;
        return false;
    }
    return true;
}

// Both free flights of a pair (words x, y for the first, z, w for the second)
// in the all-local instantiation.  The same flights as two calls of
// flight_local, but the walk is set up once: after a null collision the
// second flight goes on along the same line from the same cube, whose face
// distances and crossings left stay valid (the distances re-based to the
// null collision).  Cube records are the LDS words (density bound and table
// row; a cube without a row takes its material mask from the global record).
template <int MODE>
__device__ __forceinline__ void flight_pair_all_local(const KParams& P, const Tables& T, const DVolume& V, int vo,
                                                      Photon& ph, const Block& b, const uint32_t* lds_rec) {
    const float p0x = ph.px, p0y = ph.py, p0z = ph.pz;     // (for the set-up only)
    int bx = min(max((int)floorf((p0x - V.lox) * V.imx), 0), V.mnx - 1);
    int by = min(max((int)floorf((p0y - V.loy) * V.imy), 0), V.mny - 1);
    int bz = min(max((int)floorf((p0z - V.loz) * V.imz), 0), V.mnz - 1);
    const float rx = ph.dx != 0.0f ? fast_rcp(ph.dx) : 0.0f;
    const float ry = ph.dy != 0.0f ? fast_rcp(ph.dy) : 0.0f;
    const float rz = ph.dz != 0.0f ? fast_rcp(ph.dz) : 0.0f;
    const int sx = ph.dx > 0.0f ? 1 : (ph.dx < 0.0f ? -1 : 0);
    const int sy = ph.dy > 0.0f ? 1 : (ph.dy < 0.0f ? -1 : 0);
    const int sz = ph.dz > 0.0f ? 1 : (ph.dz < 0.0f ? -1 : 0);
    // where the line leaves the box through a face on the positive side of an axis (the last
    // cube there may reach past the face); leaving through a negative side is leaving the grid
    float tex = fminf(sx > 0 ? (V.hix - p0x) * rx : INFINITY,
                      fminf(sy > 0 ? (V.hiy - p0y) * ry : INFINITY, sz > 0 ? (V.hiz - p0z) * rz : INFINITY));
    float tmx = sx > 0 ? (V.lox + (float)(bx + 1) * V.mex - p0x) * rx
              : (sx < 0 ? (V.lox + (float)bx * V.mex - p0x) * rx : INFINITY);
    float tmy = sy > 0 ? (V.loy + (float)(by + 1) * V.mey - p0y) * ry
              : (sy < 0 ? (V.loy + (float)by * V.mey - p0y) * ry : INFINITY);
    float tmz = sz > 0 ? (V.loz + (float)(bz + 1) * V.mez - p0z) * rz
              : (sz < 0 ? (V.loz + (float)bz * V.mez - p0z) * rz : INFINITY);
    const float dtx = V.mex * fabsf(rx), dty = V.mey * fabsf(ry), dtz = V.mez * fabsf(rz);
    const float2* tot = T.tot + ph.ec.j * P.tot_rows;
    const int cix = sx, ciy = sy * V.mnx, ciz = sz * V.mnx * V.mny;
    int ci = (bz * V.mny + by) * V.mnx + bx;
    // the crossings left along each axis's direction of travel before the line leaves the
    // grid (at most 512 cubes per axis), in 10-bit fields whose top bit is a guard that the
    // crossing past the last cube clears
    uint32_t left = ((512u + (uint32_t)(sx > 0 ? V.mnx - 1 - bx : (sx < 0 ? bx : 511)))) |
                    ((512u + (uint32_t)(sy > 0 ? V.mny - 1 - by : (sy < 0 ? by : 511))) << 10) |
                    ((512u + (uint32_t)(sz > 0 ? V.mnz - 1 - bz : (sz < 0 ? bz : 511))) << 20);
    constexpr uint32_t kGuards = (1u << 9) | (1u << 19) | (1u << 29);
    float t = 0.0f;
    for (int f = 0; f < 2; ++f) {
        if (ph.step >= kMaxSteps) {
            if (MODE == kModeTrace) trace_out<MODE>(P, ph, kLost, -1);
            ph.st = kDead;
            return;
        }
        ph.step += 1;
        float tau = -fast_log(u24(f == 0 ? b.x : b.z));
        float mb = 0.0f;
        bool hit = false;
        // (selects instead of fminf/fmaxf below: no NaN can occur, and these need
        // no canonicalisation of their operands)
        for (;;) {
            const uint32_t w = lds_rec[ci];
            const uint32_t row = w & 31u;
            float tmax;
            if (row != kNoRow) {
                const float2 tt = tot[row];
                tmax = tt.x + ph.ec.f * tt.y;
            } else {
                tmax = set_bound(tot, P.tot_rows, V.macro[ci].y, ph.ec.f);
            }
            mb = __uint_as_float(w & ~31u) * tmax;
            const float tnext = fminf(tmx, fminf(tmy, tmz));
            const float tn = tnext < tex ? tnext : tex;                    // the cube's exit, within the box
            const float span = tn - t;
            const float need = 0.1f * mb * (span > 0.0f ? span : 0.0f);   // mbar in 1/cm, lengths in mm
            if (tau < need) {                                            // (need = 0 when mb = 0: tau > 0)
                t += tau * fast_rcp(0.1f * mb);
                hit = true;
                break;
            }
            tau -= need;
            t = tn > t ? tn : t;
            if (!(tn < tex)) break;                                        // left the box
            // the axis of the nearest face (ties to x, then y)
            const bool ax = tmx == tnext, ay = !ax && tmy == tnext, az = !ax && !ay;
            ci += ax ? cix : (ay ? ciy : ciz);
            tmx = ax ? tmx + dtx : tmx;
            tmy = ay ? tmy + dty : tmy;
            tmz = az ? tmz + dtz : tmz;
            left -= ax ? 1u : (ay ? 1u << 10 : 1u << 20);
            if ((left & kGuards) != kGuards) break;                       // left the grid
        }
        ph.px += t * ph.dx;
        ph.py += t * ph.dy;
        ph.pz += t * ph.dz;
        if (!hit) {
            int pixel;
            const int cls = detector_pixel(P.jobs[ph.job], ph, pixel);
            finish<MODE>(P, T, V, vo, ph, cls, pixel);
            return;
        }
        int m;
        const float rho = cell_density(V, true, ph.px, ph.py, ph.pz, m);
        m = m < P.n_mat ? m : P.n_mat - 1;
        const float2 tt = T.tot[ph.ec.j * P.tot_rows + m];
        const float tot_m = tt.x + ph.ec.f * tt.y;
        const float ladder = u24(f == 0 ? b.y : b.w) * mb;
        const bool real = ladder < rho * tot_m;
        if (MODE == kModeBackward && ph.passb) visit(P, V, true, ph, real, rho, tot_m, mb);
        if (real) {
            ph.st = kColl;
            ph.sel = ladder * fast_rcp(rho);
            ph.pm = m;
            return;
        }
        // a null collision: the second flight starts here, the distances re-based to it
        tmx -= t;
        tmy -= t;
        tmz -= t;
        tex -= t;
        t = 0.0f;
    }
}

// A real collision (Sec. 2.4): the ladder value picks Rayleigh, Compton or
// photoelectric absorption; scattering samples the angle, updates energy and
// direction and the distance to the phantom's boundary.
template <int MODE, bool ALL_LOCAL>
__device__ __forceinline__ void collide(const KParams& P, const Tables& T, const DVolume& V, int vo, Photon& ph) {
    const int m = ph.pm;
    const float* a = P.mu_mass + ((size_t)m * P.n_e + ph.ec.j) * 3;   // j <= n_e - 2
    const float R = a[0] + ph.ec.f * (a[3] - a[0]);
    const float C = a[1] + ph.ec.f * (a[4] - a[1]);
    const float sel = ph.sel;
    if (!(sel < R + C)) {
        if (MODE == kModeTrace) trace_out<MODE>(P, ph, kAbsorbed, -1);
        ph.st = kDead;
        return;
    }
    const bool is_rayleigh = sel < R;
    float az = 0.0f;
    const float ct = scatter_angle(is_rayleigh, ph.pid, ph.jid, ph.step, P.k0, P.k1, ph.E, P.x0, az);
    if (is_rayleigh) {
        ph.nsc += 1u << 16;
    } else {
        ph.nsc += 1u;
        ph.ec = energy_cache(P, T, vo, ph.E);
    }
    rotate(ph.dx, ph.dy, ph.dz, ct, az);
    if (ph.E < P.e_cut) {
        if (MODE == kModeTrace) trace_out<MODE>(P, ph, kCut, -1);
        ph.st = kDead;
        return;
    }
    if (!ALL_LOCAL && !V.macro) ph.trem = box_exit(V, ph.px, ph.py, ph.pz, ph.dx, ph.dy, ph.dz);   // local majorants walk cubes instead
    ph.st = kFly;
}

// Copies the per-launch tables into LDS (all threads of the workgroup).
// mu_tot of material m at grid point j (float32, summed as everywhere)
__device__ __forceinline__ float tot_at(const KParams& P, int m, int j) {
    const float* a = P.mu_mass + ((size_t)m * P.n_e + j) * 3;
    return a[0] + a[1] + a[2];
}

__device__ __forceinline__ Tables stage_tables(const KParams& P, float2* lds) {
    float2* s_tot = lds;
    float2* s_maj = s_tot + P.tot_rows * P.n_e;
    for (int i = threadIdx.x; i < P.n_mat * P.n_e; i += blockDim.x) {
        const int j = i / P.n_mat, m = i - j * P.n_mat;
        const float t0 = tot_at(P, m, j), t1 = tot_at(P, m, j + 1 < P.n_e ? j + 1 : j);
        s_tot[j * P.tot_rows + m] = make_float2(t0, t1 - t0);
    }
    for (int i = threadIdx.x; i < P.n_maj * (P.n_e - 1); i += blockDim.x) {
        const float mb = P.majorants[i];
        s_maj[i] = make_float2(mb, mb > 0.0f ? 1.0f / (0.1f * mb) : INFINITY);
    }
    return Tables{s_tot, s_maj};
}

// Rank of bit b among the set bits of the 256-bit set bm.
__device__ __forceinline__ int set_rank(const uint32_t* bm, uint32_t b) {
    int r = __popc(bm[b >> 5] & ((1u << (b & 31u)) - 1u));
    for (uint32_t w = 0; w < (b >> 5); ++w) r += __popc(bm[w]);
    return r;
}

// All-local launches: one LDS word per cube, its density bound with the row of
// the LDS table that holds its material factor: the material's own for a cube
// of one material; for several, a row of their set, if the set is among the
// first mask_rows distinct sets (by mask value) of the staged volumes (n_mat
// <= 8, masks < 256); kNoRow otherwise.  bm: 8 + 32 words of LDS scratch.
__device__ __forceinline__ void stage_records_rows(const KParams& P, float2* s_tot, uint32_t* rec_lds,
                                                   uint32_t* bm) {
    if (P.mask_rows > 0) {
        if (threadIdx.x < 8) bm[threadIdx.x] = 0u;
        __syncthreads();
        for (int v = 0; v < P.n_vols; ++v) {
            if (P.macro_lds[v] < 0 || !P.vol[v].macro) continue;
            const int n = P.vol[v].mnx * P.vol[v].mny * P.vol[v].mnz;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const uint32_t mask = P.vol[v].macro[i].y;
                if (mask & (mask - 1u)) atomicOr(&bm[(mask >> 5) & 7u], 1u << (mask & 31u));
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < 256; t += blockDim.x)
            if ((bm[t >> 5] >> (t & 31)) & 1u) {
                const int r = set_rank(bm, (uint32_t)t);
                if (r < P.mask_rows) bm[8 + r] = (uint32_t)t;
            }
        __syncthreads();
        int n_sets = 0;
        for (int w = 0; w < 8; ++w) n_sets += __popc(bm[w]);
        for (int i = threadIdx.x; i < P.mask_rows * P.n_e; i += blockDim.x) {
            const int j = i / P.mask_rows, k = i - j * P.mask_rows;
            const int j1 = j + 1 < P.n_e ? j + 1 : j;
            float t0 = 0.0f, t1 = 0.0f;
            if (k < n_sets)
                for (uint32_t mask = bm[8 + k]; mask; mask &= mask - 1u) {
                    const int m = __builtin_ctz(mask);
                    const float a = tot_at(P, m, j), b = tot_at(P, m, j1);
                    t0 = a > t0 ? a : t0;
                    t1 = b > t1 ? b : t1;
                }
            s_tot[j * P.tot_rows + P.n_mat + k] = make_float2(t0, t1 - t0);
        }
    }
    for (int v = 0; v < P.n_vols; ++v) {
        if (P.macro_lds[v] < 0 || !P.vol[v].macro) continue;
        const int n = P.vol[v].mnx * P.vol[v].mny * P.vol[v].mnz;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const uint2 rec = P.vol[v].macro[i];
            uint32_t row = kNoRow;
            if (!(rec.y & (rec.y - 1u))) {
                const uint32_t m = rec.y ? (uint32_t)__builtin_ctz(rec.y) : kNoRow;
                row = m < kNoRow ? m : kNoRow;
            } else if (P.mask_rows > 0) {
                const int r = set_rank(bm, rec.y & 255u);
                row = r < P.mask_rows ? (uint32_t)(P.n_mat + r) : kNoRow;
            }
            rec_lds[P.macro_lds[v] + i] = (rec.x & ~31u) | row;
        }
    }
}

// LOCAL: 0 = every volume has one majorant per energy interval; 1 = some
// volume tracks with local majorants, cube records read from global memory;
// 2 = the same with every such volume's records staged in LDS; 3 = every
// traced volume tracks with local majorants, records in LDS, at most 512 cubes
// per axis, and density is interpolated (no single-majorant flight and no
// nearest-voxel lookup in the code at all).  Separate instantiations, so that each loop keeps its
// register budget.
template <int MODE, int LOCAL>
__device__ __forceinline__ void mc_body(const KParams& P) {
    extern __shared__ float2 lds[];
    const Tables T = stage_tables(P, lds);
    // local majorants small enough to stage: every volume's cube records after the tables
    float2* const lds_rec = lds + table_floats2(P.tot_rows, P.n_e, P.n_maj);
    // the source-draw slots (offset in bytes from the LDS base of the first wavefront's)
    const uint32_t slots_off = (uint32_t)draw_slots_offset_bytes(
        table_floats2(P.tot_rows, P.n_e, P.n_maj) * 8 + (size_t)P.macro_lds_n * lds_record_bytes(LOCAL));
    // this wavefront's slots (wavefront-uniform)
    const uint32_t draws_off = __builtin_amdgcn_readfirstlane((int)(slots_off + (threadIdx.x & ~63u) * 16u));
    if (LOCAL == 3) {
        // (the slots serve as scratch until the transport starts)
        stage_records_rows(P, lds, reinterpret_cast<uint32_t*>(lds_rec),
                           reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(lds) + slots_off));
    } else if (LOCAL == 2) {
        uint2* r = reinterpret_cast<uint2*>(lds_rec);
        for (int v = 0; v < P.n_vols; ++v) {
            if (P.macro_lds[v] < 0 || !P.vol[v].macro) continue;
            const int n = P.vol[v].mnx * P.vol[v].mny * P.vol[v].mnz;
            for (int i = threadIdx.x; i < n; i += blockDim.x) r[P.macro_lds[v] + i] = P.vol[v].macro[i];
        }
    }
    __syncthreads();
    const bool interp = LOCAL == 3 || (P.flags & 1u) != 0;
    const int lane = __lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;

    Photon ph;
    ph.st = kDead;
    ph.passb = false;
    ph.w = 0.0;
    ph.job = 0;
    ph.pid = 0;
    ph.jid = 0;
    ph.nsc = 0;
    ph.sel = 0.0f;
    ph.pair = 0u;
    ph.pm = 0;

    // wavefront-uniform dispenser state; the draw slots hold photons [d_first, d_end) of the chunk
    int w_vol = -1, w_job = 0, w_hold = 0, w_done = 0;
    uint32_t w_next = 0, w_end = 0, d_first = 0, d_end = 0;

    for (;;) {
        const uint64_t dead = __ballot(ph.st == kDead);
        const int n_dead = __popcll(dead);
        const int n_coll = __popcll(__ballot(ph.st == kColl));
        const int n_fly = 64 - n_dead - n_coll;

        // ---- refill ----
        if (w_hold && n_dead == 64) {       // drained: switch to the held chunk's phantom
            w_vol = __builtin_amdgcn_readfirstlane(P.jobs[w_job].vol);
            w_hold = 0;
        }
        if (!w_done && !w_hold && n_dead > 0 && (n_dead >= P.defer || n_fly == 0)) {
            if (w_next >= w_end) {
                unsigned long long c = 0;
                if (lane == 0) c = atomicAdd(P.counter, 1ull);
                // lane 0's value in scalar registers (every lane is active here): the branches on
                // it, and so the wavefront's volume and job, stay wavefront-uniform to the compiler,
                // which then reads the volume's fields with scalar loads
                c = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(c >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)c);
                if (c >= P.total_chunks) {
                    w_done = 1;
                } else {
                    int lo = 0, hi = P.n_jobs - 1;          // last job whose first chunk <= c
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (P.chunk_prefix[mid] <= c) lo = mid; else hi = mid - 1;
                    }
                    w_job = __builtin_amdgcn_readfirstlane(lo);
                    const DJob& J = P.jobs[w_job];
                    const unsigned long long nph = (unsigned long long)J.n_lo | ((unsigned long long)J.n_hi << 32);
                    const unsigned long long first = (c - P.chunk_prefix[w_job]) * (unsigned long long)P.chunk;
                    const unsigned long long last = first + (unsigned long long)P.chunk < nph ? first + P.chunk : nph;
                    // photon indices J.first + [first, last); J.first + nph < 2^32
                    w_next = (uint32_t)__builtin_amdgcn_readfirstlane((int)(J.first + (uint32_t)first));
                    w_end = (uint32_t)__builtin_amdgcn_readfirstlane((int)(J.first + (uint32_t)last));
                    d_first = d_end = w_next;                  // no draws of this chunk yet
                    const int v = __builtin_amdgcn_readfirstlane(J.vol);
                    if (v != w_vol) {
                        if (n_dead == 64) w_vol = v; else w_hold = 1;
                    }
                }
            }
            if (!w_done && !w_hold) {
                // Not enough drawn photons left for the waiting lanes: every lane draws one of the
                // chunk's next 64 photons (the draws of a photon depend on its index alone).
                if (w_next + (uint32_t)n_dead > d_end && d_end < w_end) {
                    const uint32_t nd = w_end - w_next < 64u ? w_end - w_next : 64u;
                    uint4* draws = reinterpret_cast<uint4*>(reinterpret_cast<char*>(lds) + draws_off);
                    if ((uint32_t)lane < nd) draws[lane] = draw_source(P, w_job, w_next + (uint32_t)lane);
                    d_first = w_next;
                    d_end = w_next + nd;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the slots are read by other lanes
                }
                const uint32_t avail = d_end - w_next;
                const uint32_t rank = (uint32_t)__popcll(dead & lt);
                if (ph.st == kDead && rank < avail) {
                    ph.pid = w_next + rank;
                    ph.job = w_job;
                    ph.jid = P.jobs[w_job].job_id;
                    ph.passb = false;
                    const DVolume& V = P.vol[w_vol];
                    const int vo = V.lds_majorant;
                    const uint4* draws = reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(lds) + draws_off);
                    if (start_from_draw(P, T, V, vo, ph, draws[ph.pid - d_first])) ph.st = kFly;
                    else finish<MODE>(P, T, V, vo, ph, kPrimary, ph.pix0);
                }
                w_next += (uint32_t)n_dead < avail ? (uint32_t)n_dead : avail;
            }
        }
        if (w_done && n_dead == 64) break;
        if (w_vol < 0) continue;
        const DVolume& V = P.vol[w_vol];
        const int vo = V.lds_majorant;

        // ---- flight: one Woodcock step (Sec. 2.4) ----
        // Free flights in pairs (Sec. 2.4): one Philox block per pair, two words per
        // flight; a null collision continues the pair, a real one ends it.
        if (ph.st == kFly) {
            ph.pair += 1u;
            const Block b = philox(ph.pid, ph.jid, ph.pair, 0u, P.k0, P.k1);
            if constexpr (LOCAL == 3) {
                const uint32_t* lr = reinterpret_cast<const uint32_t*>(lds_rec) + P.macro_lds[w_vol];
                // the adjoint keeps two walks a pair: the one walk's state across the
                // collision test and its gradient visit would spill its registers
                if constexpr (MODE == kModeBackward) {
                    if (flight_local<MODE, 2>(P, T, V, vo, interp, ph, b.x, b.y, lr))
                        flight_local<MODE, 2>(P, T, V, vo, interp, ph, b.z, b.w, lr);
                } else {
                    flight_pair_all_local<MODE>(P, T, V, vo, ph, b, lr);
                }
            } else if (LOCAL == 2 && V.macro) {
                const uint2* lr = reinterpret_cast<const uint2*>(lds_rec) + P.macro_lds[w_vol];
                if (flight_local<MODE, 1>(P, T, V, vo, interp, ph, b.x, b.y, lr))
                    flight_local<MODE, 1>(P, T, V, vo, interp, ph, b.z, b.w, lr);
            } else {
                if (LOCAL == 1 && V.macro) {
                    if (flight_local<MODE, 0>(P, T, V, vo, interp, ph, b.x, b.y, nullptr))
                        flight_local<MODE, 0>(P, T, V, vo, interp, ph, b.z, b.w, nullptr);
                } else if (flight<MODE>(P, T, V, vo, interp, ph, b.x, b.y)) {
                    flight<MODE>(P, T, V, vo, interp, ph, b.z, b.w);
                }
            }
        }

        // ---- collision: interaction type and sampling ----
        const int n_coll2 = __popcll(__ballot(ph.st == kColl));
        const int n_fly2 = __popcll(__ballot(ph.st == kFly));
        if (n_coll2 > 0 && (n_coll2 >= P.cdefer || n_fly2 == 0 || w_done || w_hold)) {
            if (ph.st == kColl) collide<MODE, LOCAL == 3>(P, T, V, vo, ph);
        }
    }
}

// The forward and trace transport: at most 80 VGPRs (6 wavefronts per SIMD);
// the all-local forward at most 64 (8 wavefronts per SIMD, without spills),
// which the 1024-thread workgroups, two per compute unit, then use.
template <int MODE, int LOCAL>
__global__ __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(MODE == kModeForward && LOCAL == 3 ? 8 : 6))) void mc_kernel(KParams P) {
    mc_body<MODE, LOCAL>(P);
}

// The adjoint: at most 96 VGPRs (5 wavefronts per SIMD), where it would
// otherwise take 97 and drop to 4; the all-local instantiation at most 64 (8
// wavefronts per SIMD; it would take 70, and the 44 bytes it spills cost less
// than the occupancy: 5.38e9 against 5.11e9 histories/s at 6).
template <int LOCAL>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(LOCAL == 3 ? 8 : 5))) void mc_adjoint_kernel(
    KParams P) {
    mc_body<kModeBackward, LOCAL>(P);
}

// ---------------------------------------------------------------------------
// Majorant: per-material maximum density (over the 3x3x3 neighbourhood with
// interpolation), then per energy interval the maximum over materials.
// ---------------------------------------------------------------------------
struct MajParams {
    const float* density;
    const uint8_t* material;
    int nx, ny, nz;
    int interp, n_mat;
    unsigned int* rho_max;       // [256] float bits, zeroed
    unsigned int* present;       // [256], zeroed
    unsigned int* error;         // error word
};

__global__ __launch_bounds__(256) void rho_max_kernel(MajParams M) {
    __shared__ unsigned int s_max[256];
    __shared__ unsigned int s_pres[256];
    s_max[threadIdx.x] = 0u;
    s_pres[threadIdx.x] = 0u;
    __syncthreads();
    const long long n = (long long)M.nx * M.ny * M.nz;
    const long long nxy = (long long)M.nx * M.ny;
    unsigned int err = 0u;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < n;
         v += (long long)gridDim.x * blockDim.x) {
        // invalid inputs as the transport reads them: density 0, material n_mat - 1
        const int mr = M.material[v];
        const int m = min(mr, M.n_mat - 1);
        if (mr != m) err |= kErrMaterial;
        float r = M.density[v];
        if (!density_ok(r)) { err |= kErrDensity; r = 0.0f; }
        if (M.interp) {
            const int z = (int)(v / nxy), y = (int)((v / M.nx) % M.ny), x = (int)(v % M.nx);
            for (int dz = -1; dz <= 1; ++dz) {
                const int zz = min(max(z + dz, 0), M.nz - 1);
                for (int dy = -1; dy <= 1; ++dy) {
                    const int yy = min(max(y + dy, 0), M.ny - 1);
                    const float* row = M.density + (long long)zz * nxy + (long long)yy * M.nx;
                    for (int dx = -1; dx <= 1; ++dx) {
                        const float q = clean_density(row[min(max(x + dx, 0), M.nx - 1)]);
                        r = q > r ? q : r;
                    }
                }
            }
        }
        atomicMax(&s_max[m], __float_as_uint(r));
        s_pres[m] = 1u;
    }
    if (err) atomicOr(M.error, err);
    __syncthreads();
    if (s_pres[threadIdx.x]) {
        atomicMax(&M.rho_max[threadIdx.x], s_max[threadIdx.x]);
        atomicOr(&M.present[threadIdx.x], 1u);
    }
}

struct MajFinParams {
    const unsigned int* rho_max;
    const unsigned int* present;
    const float* mu_mass;
    int n_mat, n_e;
    double scale;              // 1 + margin
    float* out;                // [n_e - 1]
    unsigned int* error;
};

__global__ __launch_bounds__(256) void majorant_kernel(MajFinParams F) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < F.n_e - 1; j += gridDim.x * blockDim.x) {
        double best = 0.0;
        for (int m = 0; m < F.n_mat; ++m) {
            if (!F.present[m]) continue;
            const float* a = F.mu_mass + ((size_t)m * F.n_e + j) * 3;
            const double t0 = (double)a[0] + (double)a[1] + (double)a[2];
            const double t1 = (double)a[3] + (double)a[4] + (double)a[5];
            const double t = (double)__uint_as_float(F.rho_max[m]) * (t0 > t1 ? t0 : t1);
            best = t > best ? t : best;
        }
        F.out[j] = __double2float_ru(best * F.scale);
    }
}

// ---------------------------------------------------------------------------
// Local majorants: per cube of mcube^3 voxels, the largest density (at least
// rho_min) and the materials over the cube grown by one voxel (the
// interpolation corners of every point in the cube, with a voxel to spare at
// its faces).
// ---------------------------------------------------------------------------
struct MacroParams {
    const float* density;
    const uint8_t* material;
    int nx, ny, nz, mcube, mnx, mny, mnz, n_mat;
    double scale;              // 1 + margin
    float rho_min;             // least density a cube's bound assumes
    uint2* out;
};

// One workgroup per cube (grid-stride over the cubes): the lanes stride over
// the voxels of the cube grown by one voxel, x fastest (coalesced), then the
// largest density and the union of the materials are reduced over the
// workgroup.  Max and or are exact in any order, so the records are those of
// a plain loop over the voxels.
__global__ __launch_bounds__(256) void macro_kernel(MacroParams M) {
    __shared__ float s_r[4];
    __shared__ uint32_t s_m[4];
    const long long n = (long long)M.mnx * M.mny * M.mnz;
    for (long long c = blockIdx.x; c < n; c += gridDim.x) {
        const int bx = (int)(c % M.mnx), by = (int)((c / M.mnx) % M.mny), bz = (int)(c / ((long long)M.mnx * M.mny));
        const int x0 = max(bx * M.mcube - 1, 0), x1 = min((bx + 1) * M.mcube, M.nx - 1);
        const int y0 = max(by * M.mcube - 1, 0), y1 = min((by + 1) * M.mcube, M.ny - 1);
        const int z0 = max(bz * M.mcube - 1, 0), z1 = min((bz + 1) * M.mcube, M.nz - 1);
        const int nxc = x1 - x0 + 1, nyc = y1 - y0 + 1;
        const int nv = nxc * nyc * (z1 - z0 + 1);
        float r = M.rho_min;
        uint32_t mask = 0u;
        for (int i = threadIdx.x; i < nv; i += blockDim.x) {
            const int x = x0 + i % nxc, rest = i / nxc;
            const int y = y0 + rest % nyc, z = z0 + rest / nyc;
            const long long v = ((long long)z * M.ny + y) * M.nx + x;
            r = fmaxf(r, clean_density(M.density[v]));
            mask |= 1u << min((int)M.material[v], M.n_mat - 1);
        }
        for (int o = 32; o > 0; o >>= 1) {
            r = fmaxf(r, __shfl_xor(r, o));
            mask |= __shfl_xor(mask, o);
        }
        if ((threadIdx.x & 63) == 0) {
            s_r[threadIdx.x >> 6] = r;
            s_m[threadIdx.x >> 6] = mask;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
                r = fmaxf(r, s_r[w]);
                mask |= s_m[w];
            }
            // the density factor rounded up to 19 significant bits: the low 5 bits stay free
            const uint32_t rb = __float_as_uint(__double2float_ru((double)r * M.scale));
            M.out[c] = make_uint2((rb + 31u) & ~31u, mask);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Cell records of a volume (the per-flight data layout).
// ---------------------------------------------------------------------------
struct CellParams {
    const float* density;
    const uint8_t* material;
    int nx, ny, nz, n_mat;
    CellRec* cells;
    unsigned int* error;       // input-error bits (invalid densities or materials)
};

__global__ __launch_bounds__(256) void cells_kernel(CellParams C) {
    const long long cx = C.nx + 1, cy = C.ny + 1, n = cx * cy * (long long)(C.nz + 1);
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(t % cx) - 1, j = (int)((t / cx) % cy) - 1, k = (int)(t / (cx * cy)) - 1;
        uint32_t d[8];
        uint32_t m0 = 0u, err = 0u;
        bool same = true;
        for (int c = 0; c < 8; ++c) {
            const int x = min(max(i + (c & 1), 0), C.nx - 1);
            const int y = min(max(j + ((c >> 1) & 1), 0), C.ny - 1);
            const int z = min(max(k + (c >> 2), 0), C.nz - 1);
            const long long v = ((long long)z * C.ny + y) * C.nx + x;
            const float rho = C.density[v];
            if (!density_ok(rho)) err |= kErrDensity;
            d[c] = __float_as_uint(clean_density(rho)) & 0x7FFFFFFFu;   // (-0 loses its sign too)
            // a material beyond the table reads as the last one, here as everywhere
            const uint32_t mr = C.material[v];
            if (mr >= (uint32_t)C.n_mat) err |= kErrMaterial;
            const uint32_t m = min(mr, (uint32_t)(C.n_mat - 1));
            if (c == 0) m0 = m;
            same = same && m == m0;
        }
        if (err) atomicOr(C.error, err);
        if (!same) {
            d[0] |= 0x80000000u;
        } else {
            for (int b = 0; b < 4; ++b) d[1 + b] |= ((m0 >> b) & 1u) << 31;
        }
        float4* out = reinterpret_cast<float4*>(C.cells + t);
        out[0] = make_float4(__uint_as_float(d[0]), __uint_as_float(d[1]), __uint_as_float(d[2]), __uint_as_float(d[3]));
        out[1] = make_float4(__uint_as_float(d[4]), __uint_as_float(d[5]), __uint_as_float(d[6]), __uint_as_float(d[7]));
    }
}

// ---------------------------------------------------------------------------
// Source preparation: normalised CDFs (running float64 sum in index order,
// divided by the total) and guide tables, for `rows` tables of n weights.
// ---------------------------------------------------------------------------
struct SrcPrepParams {
    const float* w;           // [rows][n]
    int n, rows;
    double* cdf;              // [rows][n]
    uint32_t* guide;          // [rows][k]
    int k;
    unsigned int* error;
};

// One workgroup of 1024 threads per row: each thread sums a contiguous segment in
// index order, the segment totals are scanned, and each thread writes its
// segment's running sums divided by the total.  The sums are those of the
// definition, accumulated in a different association (float64 rounding only).
__global__ __launch_bounds__(1024) void cdf_kernel(SrcPrepParams S) {
    __shared__ double part[1024];
    __shared__ int bad;
    const int t = threadIdx.x, nt = blockDim.x;
    const float* w = S.w + (size_t)blockIdx.x * S.n;
    double* cdf = S.cdf + (size_t)blockIdx.x * S.n;
    if (t == 0) bad = 0;
    const int per = (S.n + nt - 1) / nt;
    const int a = min(S.n, t * per), b = min(S.n, a + per);
    double s = 0.0;
    int mybad = 0;
    for (int i = a; i < b; ++i) {
        const double x = (double)w[i];
        if (!(x >= 0.0) || isinf(x)) mybad = 1;
        s += x;
    }
    part[t] = s;
    __syncthreads();
    if (mybad) bad = 1;
    for (int off = 1; off < nt; off <<= 1) {     // inclusive Hillis-Steele scan of the totals
        const double v = t >= off ? part[t - off] : 0.0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const double total = part[nt - 1];
    double run = t > 0 ? part[t - 1] : 0.0;
    for (int i = a; i < b; ++i) {
        run += (double)w[i];
        cdf[i] = run / total;
    }
    if (t == 0 && (bad || !(total > 0.0))) atomicOr(S.error, kErrWeights);
}

__global__ __launch_bounds__(256) void guide_kernel(SrcPrepParams S) {
    const long long total = (long long)S.rows * S.k;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / S.k;
        const int g = (int)(e - r * S.k);
        const double* cdf = S.cdf + r * S.n;
        const double t = (double)g / (double)S.k;
        int lo = 0, hi = S.n - 1;                 // smallest i with cdf[i] > t
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cdf[mid] > t) hi = mid; else lo = mid + 1;
        }
        S.guide[e] = (uint32_t)lo;
    }
}

// ---------------------------------------------------------------------------
// Clear and finalize.
// ---------------------------------------------------------------------------
struct FillParams {
    unsigned long long* p;
    long long n;
};

__global__ __launch_bounds__(256) void fill_zero_kernel(FillParams F) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < F.n; i += (long long)gridDim.x * blockDim.x)
        F.p[i] = 0ull;
}

// The dispenser prefix, job record and output offset of a one-job launch,
// written from the kernel's arguments instead of copied from the host.
struct JobTableParams {
    unsigned long long* prefix;     // [2]
    DJob* jobs;                     // [1]
    long long* out_off;             // [1]
    unsigned long long p0, p1;
    long long off;
    DJob job;
};

__global__ __launch_bounds__(64) void job_table_kernel(JobTableParams T) {
    if (threadIdx.x != 0) return;
    T.prefix[0] = T.p0;
    T.prefix[1] = T.p1;
    T.out_off[0] = T.off;
    T.jobs[0] = T.job;
}

struct FinParams {
    const DJob* jobs;
    int n_jobs;
    const unsigned long long* tally;
    double* out;
    const long long* out_off;   // [n_jobs] double element offsets in `out`
    uint32_t flags;             // GDRR_TALLY_SUMSQ 2, GDRR_ACCUMULATE 4, GDRR_RESUME 32
};

__global__ __launch_bounds__(256) void finalize_kernel(FinParams F) {
    const int k = blockIdx.y;
    const DJob& J = F.jobs[k];
    const int npix = J.nu * J.nv;
    // per source photon of the run: a resumed run's sums cover [0, first + n)
    const double n = (double)J.n_lo + 4294967296.0 * (double)J.n_hi + ((F.flags & 32u) ? (double)J.first : 0.0);
    const double inv = n > 0.0 ? 1.0 / n : 0.0;
    const bool sumsq = (F.flags & 2u) != 0, acc = (F.flags & 4u) != 0;
    double* out = F.out + F.out_off[k];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 4 * npix; i += gridDim.x * blockDim.x) {
        const int plane = i / npix;
        if ((plane & 1) && !sumsq) continue;
        const double q = (plane & 1) ? kQ2 : kQ1;
        const double v = (double)F.tally[J.tally_off + i] / q * inv;
        out[i] = acc ? out[i] + v : v;
    }
}

struct GradClearParams {
    double* p;
    long long n;
};

__global__ __launch_bounds__(256) void grad_zero_kernel(GradClearParams G) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < G.n; i += (long long)gridDim.x * blockDim.x)
        G.p[i] = 0.0;
}

}  // namespace gdrr
