/*
 * gdrr.h -- C ABI of libgdrr, the MI355X (gfx950) Monte Carlo projection step
 * of gDRR (Jia, Yan, Cervino, Folkerts, Jiang: "A GPU tool for efficient,
 * accurate, and realistic simulation of cone beam CT projections",
 * arXiv:1204.6367).
 *
 * The library computes Step 2 of the paper (Sec. 2.4): photon histories are
 * generated from a spectrum and a fluence map (Sec. 2.1), tracked through a
 * voxel phantom by Woodcock (delta) tracking with tri-linearly interpolated
 * density, undergo photoelectric absorption, Compton (Klein-Nishina) and
 * Rayleigh scattering, and, when they leave the phantom towards the detector,
 * add r(E) to a primary or a scatter tally per pixel depending on whether they
 * scattered.  Tallies are per source photon (Sec. 2.6).  It also offers the
 * gradient of a loss of the tallies with respect to voxel densities (path
 * replay of the same random numbers; not in the paper), Step 1, the
 * primary signal by tri-linear ray tracing (Sec. 2.3, Eq. 1), and Steps 3
 * and 4, the Poisson denoising of the scatter (Sec. 2.5) and the noise of a
 * scan at a given mAs (Sec. 2.6).
 *
 * Conventions (the paper leaves them open; these are the library's reading):
 *  - lengths in mm, energies in keV, mass attenuation in cm^2/g, density in
 *    g/cm^3;
 *  - the phantom is centred on the isocentre O, x fastest: voxel (i,j,k) has
 *    its centre at ((i + 1/2 - nx/2) dx, (j + 1/2 - ny/2) dy, (k + 1/2 - nz/2) dz)
 *    and element k*ny*nx + j*nx + i;
 *  - source S = -SAD (cos phi, sin phi, 0); detector normal
 *    n = (cos(phi+theta), sin(phi+theta), 0); detector centre P = AID n;
 *    u axis = z x n, v axis = z; pixel (iu, iv) covers
 *    u in [(iu - nu/2) du, (iu + 1 - nu/2) du), likewise v; tallies are
 *    [plane][nv][nu];
 *  - the fluence map w(u) is given per detector pixel (an air-scan image);
 *    the aim point is uniform inside the sampled pixel;
 *  - the random numbers of photon i of job `job_id` under `seed` come from
 *    Philox4x32-10 blocks with counter (i, job_id, step, sub) and key seed,
 *    so results depend only on (seed, job_id, photon index) and the inputs.
 *
 * Memory: every array pointer inside the structs below, and every output
 * array, is a DEVICE pointer owned by the caller; the struct pointers
 * themselves are host pointers read during the call.  All calls are
 * asynchronous on `stream` (a hipStream_t passed as void*; NULL = the null
 * stream) and may be recorded into a HIP graph.  The library allocates no
 * device memory and keeps none between calls, apart from the fixed array in
 * its code object behind gdrr_mc_project_static: scratch lives in the
 * caller's workspace, which also
 * holds a per-call copy of each phantom laid out for the transport kernel
 * (32 bytes per cell of the lattice of voxel centres, (nx+1)(ny+1)(nz+1)
 * cells: the eight interpolation corners of the cell, the materials in their
 * sign bits).  Each call that takes a workspace reports the bytes it needs
 * through its own query (gdrr_*_workspace), sized for that call's arguments.
 *
 * Errors: functions return GDRR_OK (0) or a negative code; no exception
 * crosses the ABI; gdrr_last_error() gives a message for the calling thread.
 * Arguments the host can see are checked before anything is launched.  Array
 * contents live on the device and are checked by the kernels while they run:
 * a density that is negative, NaN or infinite is transported as 0, a
 * material index >= n_mat as n_mat - 1, and the call still returns GDRR_OK;
 * gdrr_input_status() on the call's workspace afterwards says whether that
 * happened (GDRR_EINVAL and a message) -- or whether spectrum or fluence
 * weights were negative, non-finite or all zero.
 */
#ifndef GDRR_H
#define GDRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GDRR_OK 0
#define GDRR_EINVAL (-1)   /* invalid argument (message via gdrr_last_error) */
#define GDRR_EHIP (-2)     /* HIP runtime / launch error */
#define GDRR_ENOTSUP (-3)  /* valid but unsupported configuration */

/* flags */
#define GDRR_INTERP_DENSITY 1u     /* tri-linear density at the photon position (Sec. 2.4); else voxel-constant */
#define GDRR_TALLY_SUMSQ 2u        /* also tally r(E)^2 (planes 1 and 3), for per-pixel variances */
#define GDRR_ACCUMULATE 4u         /* add to the output tallies / gradient instead of overwriting them */
#define GDRR_SCATTER_FIRST 8u      /* scatter tally counts only photons scattered exactly once (Sec. 2.4, type-specific tally) */
#define GDRR_SCATTER_FIRST_COMPTON 16u /* ... only photons scattered exactly once, by Compton */
#define GDRR_RESUME 32u            /* forward: keep the fixed-point sums an earlier call left in the same workspace
                                      and add to them; see gdrr_job.first_photon */

#define GDRR_MAX_MATERIALS 16
#define GDRR_MAX_VOLUMES 8
#define GDRR_MAX_SOURCES 8

/* Voxel phantom (Sec. 2.1): material index and density per voxel. */
typedef struct gdrr_volume {
    int32_t nx, ny, nz;
    float dx_mm, dy_mm, dz_mm;
    const float* density;      /* [nz][ny][nx] g/cm^3, finite and >= 0 (others are transported as 0 and
                                  reported by gdrr_input_status) */
    const uint8_t* material;   /* [nz][ny][nx] indices < gdrr_physics.n_mat (others: n_mat - 1, reported) */
    /* (nx+1)(ny+1)(nz+1) < 2^31 */
    /* Local majorants (not in the paper; 0 = off): the volume is cut into cubes of
     * `macro`^3 voxels (the last ones along an axis shorter), each with the bound
     * (1 + macro_margin) max(rho_max, macro_rho_min) max_m mu_tot(m, E), rho_max and
     * the materials taken over the cube grown by one voxel;
     * a free flight spends an optical depth -ln(u) cube by cube and the collision
     * ladder runs against the bound of the cube it ends in.  Unbiased like the
     * single majorant, with far fewer null collisions in air and soft tissue; it uses
     * the random numbers differently, so results differ history by history.  When on,
     * the `majorants` argument is not used for this volume.  1 <= macro <= 256. */
    int32_t macro;
    float macro_margin;        /* >= 0; 2^-20 for projections, 0.1-0.2 for the adjoint */
    /* >= 0, g/cm^3: the least density a cube's bound assumes (0 for projections).  A
     * cube of air alone gets a bound so small that one unit of optical depth spans
     * metres; float32 rounding of the optical depth left after denser cubes then
     * moves its collisions by a visible fraction of a voxel, and the adjoint's
     * 1/rho terms of real collisions in air magnify that.  A floor of about 0.05
     * keeps a free path in such cubes near a metre at a few more null collisions. */
    float macro_rho_min;
} gdrr_volume;

/* Mass attenuation tables mu_k(i, E) of Sec. 2.1 on the grid
 * E_j = e0 + j de, j < n_e, linear in E between grid points; the detector
 * response r(E) on the same grid. */
typedef struct gdrr_physics {
    int32_t n_mat, n_e;        /* 1 <= n_mat <= GDRR_MAX_MATERIALS, 2 <= n_e <= 1024 */
    float e0_kev, de_kev;
    const float* mu_mass;      /* [n_mat][n_e][3] cm^2/g: Rayleigh, Compton, photoelectric */
    const float* response;     /* [n_e] keV deposited per photon of energy E_j, or NULL for r(E) = E;
                                  values are clamped to [0, 1024] keV */
    float rayleigh_x0_invA;    /* form factor F(x) = Z exp(-x/x0), x = sin(theta/2)/lambda, 1/Angstrom */
    float e_cut_kev;           /* photons below this energy are absorbed locally; >= e0 */
} gdrr_physics;

/* Source of Sec. 2.1, defined after the bowtie: spectrum phi(E) and fluence
 * map w(u); both are normalised by the library (weights need only be >= 0).
 *
 * Joint source (spec_rows = fu): spec_prob holds one spectrum per detector
 * column, row iu being phi(E | column iu), the fuller description of a beam
 * that a bowtie hardens more toward the edges of the fan.  A photon's aim
 * pixel is drawn from w first and its energy from the row of that pixel's
 * column, with the random numbers of the factorised source, so equal rows
 * reproduce it history for history.  Every row needs a positive sum.
 * rows * n_spec <= 2^24. */
typedef struct gdrr_source {
    int32_t n_spec;            /* 1 <= n_spec <= 4096 energy channels */
    const float* spec_e_kev;   /* [n_spec] channel energies within the physics grid (shared by all rows) */
    const float* spec_prob;    /* [n_spec] weights, or [fu][n_spec] when spec_rows = fu */
    int32_t fu, fv;            /* fluence grid = the detector's pixel grid (fu = nu, fv = nv) */
    const float* fluence;      /* [fv][fu] weights */
    int32_t spec_rows;         /* 0 or 1: one spectrum for every direction; fu: one per detector column */
} gdrr_source;

/* Geometry of Sec. 2.1 (Fig. 1). */
typedef struct gdrr_geometry {
    float sad_mm, aid_mm;      /* source-axis and axis-imager distances */
    float phi_rad, theta_rad;  /* gantry angle; imager angle from SO to OP */
    int32_t nu, nv;            /* detector pixels */
    float du_mm, dv_mm;
} gdrr_geometry;

/* One projection of a batch: the histories of photon indices
 * first_photon .. first_photon + n_photons - 1 of job `job_id`.  Their tally
 * is per source photon of that range (divided by n_photons).  A run can be
 * split and resumed (a checkpoint being the workspace): a call over
 * [0, m) and then, on the same workspace with the same arguments, a call with
 * first_photon = m, n_photons = N - m and GDRR_RESUME give bit for bit the
 * tallies of one call over [0, N), since the fixed-point sums continue and
 * the output is then divided by first_photon + n_photons. */
typedef struct gdrr_job {
    int32_t volume;            /* index into the batch's volumes */
    int32_t source;            /* index into the batch's sources */
    gdrr_geometry geom;
    uint64_t n_photons;        /* first_photon + n_photons < 2^32 */
    uint32_t job_id;           /* Philox counter word 1 */
    uint32_t first_photon;     /* first photon index (Philox counter word 0) */
    int64_t tally_offset;      /* element offset of this job's [4][nv][nu] block in `tallies` */
} gdrr_job;

/* Launch shape of the persistent kernel (0 = library default). */
typedef struct gdrr_tuning {
    int32_t block;             /* threads per workgroup: a multiple of 64 up to 1024 */
    int32_t blocks_per_cu;     /* workgroups per compute unit */
    int32_t chunk;             /* photons handed out at a time (multiple of 64) */
    int32_t defer;             /* refills run when >= defer lanes of a wavefront wait (1..64) */
    int32_t coll_defer;        /* interactions run when >= coll_defer lanes wait (1..64; 0: defer) */
} gdrr_tuning;

/*
 * Woodcock majorant (the bound delta tracking needs, Sec. 2.4 [Woodcock]):
 * out[j], j < n_e - 1, is the largest linear attenuation (1/cm) any position
 * of `vol` can show for E in [E_j, E_j+1), times (1 + margin).  With
 * GDRR_INTERP_DENSITY the density at a position mixes the voxel centres of
 * the 3x3x3 neighbourhood of its containing voxel, whose material it takes,
 * so each material's bound uses that neighbourhood's maximum density.
 * margin >= 2^-20 keeps the bound valid under float32 rounding; the adjoint
 * needs a larger one (0.05 - 0.2) for a bounded variance.
 * Workspace: gdrr_majorant_workspace() bytes.
 */
int gdrr_majorant(const gdrr_volume* vol, const gdrr_physics* phys, uint32_t flags, float margin,
                  float* out, void* workspace, size_t ws_bytes, void* stream);
size_t gdrr_majorant_workspace(void);

/*
 * One projection (Sec. 2.4): n_photons histories, photon indices
 * 0..n_photons-1 of job `job_id`.  `majorant` (device, [n_e-1], 1/cm) may be
 * NULL: the library then computes it with margin 2^-20 into the workspace.
 * tally [4][nv][nu] (double, per source photon): primary sum of r(E), its
 * sum of squares, scatter sum of r(E), its sum of squares (the squares only
 * with GDRR_TALLY_SUMSQ, else those planes are left untouched).
 * Workspace: gdrr_mc_project_workspace() bytes.
 */
int gdrr_mc_project(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                    const gdrr_geometry* geom, const float* majorant, uint64_t seed,
                    uint64_t n_photons, uint32_t job_id, uint32_t flags, double* tally,
                    void* workspace, size_t ws_bytes, void* stream);
size_t gdrr_mc_project_workspace(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                                 const gdrr_geometry* geom);

/* Bytes of the per-device scratch array behind gdrr_mc_project_static. */
#define GDRR_STATIC_SCRATCH_BYTES (128u << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * gdrr_mc_project without a workspace argument.  Its scratch is one array of
 * GDRR_STATIC_SCRATCH_BYTES per device, part of the library's code object, so
 * each device the library runs on holds it until the process ends; its device
 * address is looked up once per device, by gdrr_init() or by the first call of
 * this function there.  Arguments and results are those of gdrr_mc_project,
 * bit for bit, with these differences:
 *  - a call whose gdrr_mc_project_workspace() exceeds GDRR_STATIC_SCRATCH_BYTES
 *    (about 4 million interpolation cells, e.g. 128x128x96 fits, 256x256x160
 *    does not), or that sets GDRR_RESUME, returns GDRR_EINVAL before any
 *    device work;
 *  - the device-side input checks are not reported (gdrr_input_status needs a
 *    caller's workspace) and the timing hook is not applied.
 * Allocates no device memory and issues no host-to-device copy (the job's
 * tables travel as kernel arguments); host bookkeeping uses the C++ heap.
 * Every call on a device uses that device's one array, which keeps the last
 * call's contents (the call clears what must start at zero): calls that
 * overlap on one device -- other streams, other threads -- race and give wrong
 * results, so the caller orders them.
 */
int gdrr_mc_project_static(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                           const gdrr_geometry* geom, const float* majorant, uint64_t seed,
                           uint64_t n_photons, uint32_t job_id, uint32_t flags, double* tally, void* stream);

/*
 * Batch: every job of `jobs` (host array) in one persistent launch, replayed
 * from a cached HIP graph when called again with the same arguments.  Job k
 * gives exactly the tallies gdrr_mc_project gives for its volume, source,
 * geometry, photon count and job_id (bitwise).  All volumes share `phys`.
 * `majorants` (device, [n_vols][n_e-1]) may be NULL (computed, margin 2^-20).
 * `tallies` receives each job's [4][nv][nu] block at its tally_offset.
 * `tune` may be NULL for the defaults.
 */
int gdrr_mc_project_batch(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                          const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs,
                          int32_t n_jobs, const float* majorants, uint64_t seed, uint32_t flags,
                          const gdrr_tuning* tune, double* tallies, void* workspace,
                          size_t ws_bytes, void* stream);
size_t gdrr_mc_project_batch_workspace(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                                       const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs,
                                       int32_t n_jobs);

/*
 * Gradient of a loss of the tallies with respect to voxel density (not in the
 * paper): with adj[k] = dL/dT for job k ([2][nv][nu] double: primary,
 * scatter; device, at element offset 2*npix*k), adds to grad_density
 * ([nz][ny][nx] double, device) of every job's volume the path-replay,
 * score-function estimate
 *   dL/drho_v = sum_jobs (1/N) sum_i adj[c_i][p_i] r(E_i) sum_{collisions e of i} s_e(v),
 * s_e = w_v/rho for a real collision and -mu_tot w_v/(mbar - mu) for a null
 * one (w_v the interpolation weight of voxel v), holding the majorant fixed.
 * Each history is regenerated twice from its Philox counters (outcome, then
 * collisions); nothing is stored per history.  `majorants` is required and
 * must be the one the forward used; only jobs of volume `volume` are run.
 * Workspace: gdrr_mc_project_batch_workspace() bytes.
 */
int gdrr_mc_backward(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                     const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs,
                     int32_t volume, const float* majorants, uint64_t seed, uint32_t flags,
                     const gdrr_tuning* tune, const double* adj, double* grad_density,
                     void* workspace, size_t ws_bytes, void* stream);

/*
 * Per-history outcomes of one projection (a diagnostic of the same transport
 * code): class (0 primary hit, 1 scatter hit, 2 photoelectric, 3 energy cut,
 * 4 missed the detector, 5 step limit), pixel (iv*nu+iu or -1), final energy,
 * number of free flights, Compton and Rayleigh events.  Arrays are device
 * arrays of n_photons elements; any may be NULL.
 */
int gdrr_mc_trace(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                  const gdrr_geometry* geom, const float* majorant, uint64_t seed,
                  uint64_t n_photons, uint32_t job_id, uint32_t flags, int8_t* cls, int32_t* pixel,
                  float* e_final, int32_t* steps, int32_t* n_compton, int32_t* n_rayleigh,
                  void* workspace, size_t ws_bytes, void* stream);

/*
 * Primary signal by ray tracing (Sec. 2.3, Eq. 1), the deterministic
 * counterpart of the MC's primary tally, per source photon:
 *   P(u) = sum_k phi_k w(u) r(E_k) exp(-sum_j dl_j mu(x_j, E_k)),
 * phi and w normalised to sum 1, over the spectrum's channels (E_k, phi_k).
 * The ray runs from S to the centre of pixel u; its length from S is cut
 * into intervals [j dl, (j+1) dl), and the part of each interval inside the
 * phantom box is one term with mu at its midpoint.  With GDRR_INTERP_DENSITY
 * mu(x, E) interpolates the voxel attenuation coefficients
 * rho_v mu_tot(m_v, E) trilinearly over the lattice of voxel centres
 * (clamped at the edges); without it mu is the containing voxel's value.
 * step_mm is dl (<= 0: half the smallest voxel edge of the job's volume);
 * a ray may take at most 2^20 intervals.  Job k's image [nv][nu] (double)
 * goes to out + jobs[k].tally_offset; n_photons and job_id are ignored.
 * Flags: GDRR_INTERP_DENSITY, GDRR_ACCUMULATE (add to out); others are
 * rejected.  Workspace: gdrr_primary_workspace() bytes (it holds the cell
 * records of each volume when interpolating).  The timing hook brackets the
 * ray-tracing kernel.
 */
int gdrr_primary(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys, const gdrr_source* srcs,
                 int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs, float step_mm, uint32_t flags,
                 double* out, void* workspace, size_t ws_bytes, void* stream);
size_t gdrr_primary_workspace(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                              const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs);

/*
 * Scatter denoising (Sec. 2.5): n_img iterations of Eq. 5,
 *   S'(i,j) = (1 - omega) S(i,j) + (omega/4) [S(i-1,j) + S(i+1,j) + S(i,j-1)
 *             + S(i,j+1) - (1/beta) (1 - Shat(i,j) / S(i,j))],
 * every value on the right from the previous iterate, S^(0) = Shat (the
 * paper uses omega = 0.8).  A neighbour beyond the detector edge is the pixel
 * itself; the data term is 1 where Shat = 0; iterates are held >= s_floor > 0.
 * Arithmetic is float32 (images of up to 2^24 counts keep 7 digits).
 * shat: image k is [nv][nu] doubles at shat + k * shat_stride (0 = nv*nu), so
 * plane 2 of a batch's tallies can be passed in place (stride 4 nv nu);
 * out: [n_img][nv][nu] doubles, not overlapping shat.  iters <= 2^20 (0 copies
 * max(Shat, s_floor)).  Workspace: gdrr_denoise_workspace() bytes.  The timing
 * hook brackets all passes.
 */
int gdrr_denoise(const double* shat, int64_t shat_stride, int32_t n_img, int32_t nv, int32_t nu, float beta,
                 float omega, int32_t iters, float s_floor, double* out, void* workspace, size_t ws_bytes,
                 void* stream);
size_t gdrr_denoise_workspace(int32_t n_img, int32_t nv, int32_t nu);

/*
 * Noise of a simulated scan (Sec. 2.6): per pixel
 *   noise = alpha ((Phat - P) + (Shat - S)),   image = P + S + noise,
 * Phat, Shat the MC primary and scatter tallies, P the ray-traced primary, S
 * the denoised scatter, alpha = sqrt(n_sim / (zeta I)) for n_sim simulated
 * source photons, zeta source photons per mAs and I mAs.  Phat and Shat may
 * be strided like gdrr_denoise's input (image k at + k * stride, 0 = npix);
 * P, S, noise and image are [n_img][npix] doubles; noise or image may be NULL.
 */
int gdrr_noise(int32_t n_img, int64_t npix, const double* phat, int64_t phat_stride, const double* p,
               const double* shat, int64_t shat_stride, const double* s, double alpha, double* noise,
               double* image, void* stream);

/*
 * The noise scale of Sec. 2.6, second equation: *alpha = sqrt(n_sim / (zeta I))
 * for n_sim simulated source photons, zeta source photons per mAs and I mAs
 * (host arithmetic in float64; all three must be finite and > 0, else
 * GDRR_EINVAL).
 */
int gdrr_noise_scale(double n_sim, double zeta, double mas, double* alpha);

/*
 * Status of the device-side input checks of the last call that used
 * `workspace` (gdrr_majorant, gdrr_mc_project, gdrr_mc_project_batch,
 * gdrr_mc_backward, gdrr_mc_trace, gdrr_primary): waits for `stream`, then
 * returns GDRR_OK, or GDRR_EINVAL with a message naming what the kernels
 * found -- densities that are negative, NaN or infinite (transported as 0),
 * material indices >= n_mat (transported as n_mat - 1), spectrum or fluence
 * weights that are negative, non-finite or sum to zero (the source is then
 * undefined).  Does not launch or allocate; not for use under graph capture.
 */
int gdrr_input_status(const void* workspace, void* stream);

/*
 * Timing hook (autotuner, benchmarks): while enabled, the transport kernel of
 * every call is bracketed by HIP events recorded on the call's stream (also
 * inside a batch's cached graph); gdrr_last_kernel_ms waits for the most
 * recent bracket of the current device and returns its duration in ms.
 * Concurrent calls on one device share the bracket.
 */
int gdrr_enable_timing(int enable);
int gdrr_last_kernel_ms(float* ms);

/* Default launch shape for this device (after gdrr_init). */
int gdrr_default_tuning(gdrr_tuning* out);

/* Optional: binds the library to the current device and reads its properties. */
int gdrr_init(void);

/* Message of the last error of the calling thread ("" if none). */
const char* gdrr_last_error(void);

/* Library version string. */
const char* gdrr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GDRR_H */
