/*
 * CPU oracle for the Monte Carlo projection step of gDRR (Jia et al., "A GPU
 * tool for efficient, accurate, and realistic simulation of cone beam CT
 * projections", arXiv:1204.6367).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, double-precision
 * restatement of what the method computes, used by the tests, by the smoke
 * check and by the benchmark's CPU-baseline leg to check the GPU library.  The
 * product path never links, loads or calls it, and it shares no code, header
 * or table with the GPU library: the two meet only in the seeded input arrays.
 *
 * What it follows:
 *   Sec. 2.1  geometry (source S at SAD, angle phi; detector normal to OP at
 *             AID, angle theta; (u,v) frame at P with v parallel to z), the
 *             voxel phantom (material index + density), the mass attenuation
 *             tables mu_k(i,E) (k = Rayleigh, Compton, photoelectric), the
 *             spectrum phi(E) and fluence map w(u) as normalised pdfs, and the
 *             detector response r(E).  Optionally the spectrum varies with
 *             the detector column the photon is aimed at (a joint pdf
 *             w(u) phi(E|u), the fuller form of a source after a bowtie); the
 *             aim pixel is drawn first, then the energy from its column's row.
 *   Sec. 2.3  Eq. 1 (Beer-Lambert primary): the ray-tracing sum over
 *             intervals of length dl with trilinearly interpolated attenuation
 *             at their midpoints, and, as a check of the MC, the same
 *             integral evaluated exactly for the MC's density model.
 *   Sec. 2.4  the MC: one history at a time -- source photon from spectrum and
 *             fluence map, Woodcock (delta) tracking, photoelectric absorption
 *             terminates, Compton and Rayleigh angles from their differential
 *             cross sections, escape -> geometric detector hit -> r(E) added
 *             to the primary or the scatter counter by the scatter indicator;
 *             density tri-linearly interpolated at the photon's position.
 *   Sec. 2.6  tallies normalised per source photon.
 * Readings where the paper is silent (conventions, the random-number layout,
 * the samplers, the majorant) are the ones listed in the design notes and are
 * restated beside the code that implements them.
 *
 * Everything is double precision.  Inputs arrive as float32 / uint8 arrays
 * and are widened on read.  OpenMP splits the photon-index range into fixed
 * chunks; per-thread tallies are reduced in thread order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_ME_C2_KEV 510.99895
#define OR_HC_KEV_A 12.398419843
#define OR_MAX_TRIES 256
#define OR_MAX_STEPS (1 << 20)

enum { OR_PRIMARY = 0, OR_SCATTER = 1, OR_ABSORBED = 2, OR_CUT = 3, OR_MISSED = 4, OR_LOST = 5 };

/* Problem description (the oracle's own layout; plain host arrays). */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;                 /* mm */
    const float* density;              /* [nz][ny][nx] g/cm^3 */
    const uint8_t* material;           /* [nz][ny][nx] */
    int32_t n_mat, n_e;
    double e0, de;                     /* energy grid E_j = e0 + j de, keV */
    const float* mu;                   /* [n_mat][n_e][3] cm^2/g: Rayleigh, Compton, photo */
    const float* response;             /* [n_e] keV, or NULL for r(E) = E */
    double x0_rayleigh;                /* form-factor scale, 1/Angstrom */
    double e_cut;                      /* keV */
    int32_t n_spec;
    const float* spec_e;               /* [n_spec] keV */
    const float* spec_p;               /* [n_spec], or [nu][n_spec] when spec_rows = nu */
    int32_t spec_rows;                 /* 0 or 1: one spectrum phi(E) for every direction; nu: row iu is
                                          the spectrum of photons aimed at detector column iu (joint E|u) */
    const float* fluence;              /* [nv][nu] */
    double sad, aid, phi, theta;       /* mm, rad */
    int32_t nu, nv;
    double du, dv;                     /* mm */
    int32_t macro;                     /* local majorants on cubes of macro^3 voxels; 0 = one global majorant */
    double macro_margin;               /* their relative margin */
    double macro_rho_min;              /* the least density (g/cm^3) a cube's bound assumes */
} or_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the */
/* round keys advanced by the Weyl constants between rounds.                 */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1) from 23 random bits: odd multiples of 2^-24, exact in
 * both float32 and float64. */
static double u24(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Uniform in [0,1) from 53 random bits of two words, exact in float64. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t k = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)k * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Sampling from a tabulated pdf: inverse CDF.  C_k = S_k / S_{n-1} with     */
/* S_k the running sum (in index order) of the non-negative weights; the     */
/* sampled index is the smallest k with u < C_k.                             */
/* ------------------------------------------------------------------------ */
static int build_cdf(const float* w, int n, double* cdf)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        double x = (double)w[k];
        if (!(x >= 0.0) || isinf(x)) return -1;
        s += x;
        cdf[k] = s;
    }
    if (!(s > 0.0)) return -1;
    for (int k = 0; k < n; ++k) cdf[k] = cdf[k] / s;
    return 0;
}

static int cdf_search(const double* cdf, int n, double u)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (u < cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Tests: sample indices for given uniforms. */
int or_sample_cdf(const float* w, int32_t n, const double* u, int64_t m, int32_t* out)
{
    double* cdf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!cdf) return -1;
    if (build_cdf(w, n, cdf)) { free(cdf); return -1; }
    for (int64_t i = 0; i < m; ++i) out[i] = cdf_search(cdf, n, u[i]);
    free(cdf);
    return 0;
}

/* Spectrum of the photons aimed at detector column iu: the only one, or its
 * row of the joint table phi(E|u) (a bowtie hardens the beam differently
 * along u; the fluence map stays the marginal w(u) of the aim pixel). */
static int spec_rows(const or_problem* p) { return p->spec_rows > 1 ? p->spec_rows : 1; }
static const float* spec_row(const or_problem* p, int iu)
{
    return p->spec_p + (p->spec_rows > 1 ? (size_t)iu * p->n_spec : 0);
}

/* ------------------------------------------------------------------------ */
/* Geometry, Sec. 2.1: the source S rotates in the xOy plane at distance SAD */
/* with phi the angle from +x to SO; the detector is perpendicular to xOy    */
/* and to OP, at distance AID, with theta the angle from SO to OP (counter-  */
/* clockwise); (u, v) has its origin at P and v along +z; u = z x n.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    double S[3], P[3], n[3], eu[3], ev[3];
    double lo[3], hi[3], vs[3];
    int nvox[3];
    double* cdf_e;                     /* [rows][n_spec] */
    double* cdf_f;
    const double* mbar;                /* [n_e - 1], 1/cm */
    int nb[3];                         /* macro cells per axis (local majorants) */
    double* mac_rho;                   /* [nbz][nby][nbx] (1 + margin) x the largest density the cube's
                                          positions can show, 19 significant bits rounded up */
    uint64_t* mac_mask;                /* materials its positions can take, one bit each */
    uint32_t key[2];
    uint32_t job;
    int interp;
} or_ctx;

static void setup_geometry(const or_problem* p, or_ctx* c)
{
    double cp = cos(p->phi), sp = sin(p->phi);
    double cq = cos(p->phi + p->theta), sq = sin(p->phi + p->theta);
    c->S[0] = -p->sad * cp; c->S[1] = -p->sad * sp; c->S[2] = 0.0;
    c->n[0] = cq; c->n[1] = sq; c->n[2] = 0.0;
    c->P[0] = p->aid * cq; c->P[1] = p->aid * sq; c->P[2] = 0.0;
    c->eu[0] = -sq; c->eu[1] = cq; c->eu[2] = 0.0;
    c->ev[0] = 0.0; c->ev[1] = 0.0; c->ev[2] = 1.0;
    c->nvox[0] = p->nx; c->nvox[1] = p->ny; c->nvox[2] = p->nz;
    c->vs[0] = p->dx; c->vs[1] = p->dy; c->vs[2] = p->dz;
    for (int a = 0; a < 3; ++a) {
        c->lo[a] = -0.5 * c->nvox[a] * c->vs[a];
        c->hi[a] = 0.5 * c->nvox[a] * c->vs[a];
    }
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Slab-method intersection of the ray x + t d (t >= 0) with the phantom box. */
static int box_entry(const or_ctx* c, const double* x, const double* d, double* tin, double* tout)
{
    double t0 = 0.0, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (x[a] < c->lo[a] || x[a] > c->hi[a]) return 0;
            continue;
        }
        double ta = (c->lo[a] - x[a]) / d[a];
        double tb = (c->hi[a] - x[a]) / d[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (!(t0 < t1)) return 0;
    *tin = t0; *tout = t1;
    return 1;
}

/* Distance from a point inside the box to its boundary along d. */
static double box_exit(const or_ctx* c, const double* x, const double* d)
{
    double t = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double ta = INFINITY;
        if (d[a] > 0.0) ta = (c->hi[a] - x[a]) / d[a];
        else if (d[a] < 0.0) ta = (c->lo[a] - x[a]) / d[a];
        if (ta < t) t = ta;
    }
    return t < 0.0 ? 0.0 : t;
}

/* ------------------------------------------------------------------------ */
/* Material tables, Sec. 2.1/2.3: mu(x,E) = rho(x) * sum_k mu_k(i(x), E).     */
/* The tables are linear in E between grid points.                           */
/* ------------------------------------------------------------------------ */
static int e_interval(const or_problem* p, double E, double* f)
{
    double g = (E - p->e0) / p->de;
    int j = (int)floor(g);
    if (j < 0) j = 0;
    if (j > p->n_e - 2) j = p->n_e - 2;
    *f = g - (double)j;
    return j;
}

static void xs_at(const or_problem* p, int m, double E, double mu3[3])
{
    double f;
    int j = e_interval(p, E, &f);
    const float* a = p->mu + ((size_t)m * p->n_e + j) * 3;
    const float* b = a + 3;
    for (int k = 0; k < 3; ++k) mu3[k] = (double)a[k] + f * ((double)b[k] - (double)a[k]);
}

static double response_at(const or_problem* p, double E)
{
    if (!p->response) return E;
    double f;
    int j = e_interval(p, E, &f);
    return (double)p->response[j] + f * ((double)p->response[j + 1] - (double)p->response[j]);
}

static int clampi(int i, int lo, int hi) { return i < lo ? lo : (i > hi ? hi : i); }

static size_t vidx(const or_problem* p, int ix, int iy, int iz)
{
    return ((size_t)iz * p->ny + iy) * p->nx + ix;
}

/* Containing voxel (clamped so rounding at the faces stays inside). */
static size_t containing_voxel(const or_problem* p, const or_ctx* c, const double* x)
{
    int i[3];
    for (int a = 0; a < 3; ++a)
        i[a] = clampi((int)floor((x[a] - c->lo[a]) / c->vs[a]), 0, c->nvox[a] - 1);
    return vidx(p, i[0], i[1], i[2]);
}

/* Trilinear stencil of Sec. 2.4: density on the lattice of voxel centres,
 * clamped to the edge voxels outside the outermost centres.  Fills the eight
 * corner voxel indices and weights; returns rho(x). */
static double trilinear(const or_problem* p, const or_ctx* c, const double* x,
                        size_t vox[8], double wt[8])
{
    int i0[3], i1[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double g = (x[a] - c->lo[a]) / c->vs[a] - 0.5;
        int k = (int)floor(g);
        f[a] = g - (double)k;
        i0[a] = clampi(k, 0, c->nvox[a] - 1);
        i1[a] = clampi(k + 1, 0, c->nvox[a] - 1);
    }
    double rho = 0.0;
    int n = 0;
    for (int bz = 0; bz < 2; ++bz)
        for (int by = 0; by < 2; ++by)
            for (int bx = 0; bx < 2; ++bx) {
                double w = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
                size_t v = vidx(p, bx ? i1[0] : i0[0], by ? i1[1] : i0[1], bz ? i1[2] : i0[2]);
                vox[n] = v; wt[n] = w; ++n;
                rho += w * (double)p->density[v];
            }
    return rho;
}

/* ------------------------------------------------------------------------ */
/* Woodcock majorant: for each energy interval [E_j, E_j+1), the largest     */
/* attenuation any position can show, times (1 + 2^-20).  With interpolation */
/* on, a position's density mixes the 2x2x2 centres around it, all inside    */
/* the 3x3x3 neighbourhood of its containing voxel (whose material it takes),*/
/* so rho_max(m) is the 3x3x3-neighbourhood maximum over voxels of m.        */
/* ------------------------------------------------------------------------ */
int or_majorant_margin(const or_problem* p, int32_t interp, double margin, double* out);

int or_majorant(const or_problem* p, int32_t interp, double* out)
{
    return or_majorant_margin(p, interp, 1.0 / 1048576.0, out);
}

/* The same bound times (1 + margin) instead of (1 + 2^-20): any margin keeps
 * delta tracking unbiased; the adjoint's null-collision terms need a
 * margin well above zero for a finite variance. */
int or_majorant_margin(const or_problem* p, int32_t interp, double margin, double* out)
{
    double rmax[256];
    int present[256];
    if (p->n_mat < 1 || p->n_mat > 256 || p->n_e < 2) return -1;
    for (int m = 0; m < 256; ++m) { rmax[m] = 0.0; present[m] = 0; }
    for (int iz = 0; iz < p->nz; ++iz)
        for (int iy = 0; iy < p->ny; ++iy)
            for (int ix = 0; ix < p->nx; ++ix) {
                size_t v = vidx(p, ix, iy, iz);
                int m = p->material[v];
                if (m >= p->n_mat) return -1;
                double r = (double)p->density[v];
                if (!(r >= 0.0) || isinf(r)) return -1;
                if (interp) {
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                size_t w = vidx(p, clampi(ix + dx, 0, p->nx - 1),
                                                clampi(iy + dy, 0, p->ny - 1),
                                                clampi(iz + dz, 0, p->nz - 1));
                                double q = (double)p->density[w];
                                if (q > r) r = q;
                            }
                }
                if (r > rmax[m]) rmax[m] = r;
                present[m] = 1;
            }
    for (int j = 0; j < p->n_e - 1; ++j) {
        double best = 0.0;
        for (int m = 0; m < p->n_mat; ++m) {
            if (!present[m]) continue;
            const float* a = p->mu + ((size_t)m * p->n_e + j) * 3;
            double t0 = (double)a[0] + (double)a[1] + (double)a[2];
            double t1 = (double)a[3] + (double)a[4] + (double)a[5];
            double t = rmax[m] * (t0 > t1 ? t0 : t1);
            if (t > best) best = t;
        }
        out[j] = best * (1.0 + margin);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Random-number layout: block (photon i, job, step, sub) under key = seed.  */
/* step 0 = source (sub 0: energy and pixel, sub 1: position in the pixel).  */
/* Free flights come in pairs: pair p takes block (i, job, p, 0), words 0-1 */
/* for its first flight and words 2-3 for its second -- each time one word   */
/* for the flight length and one for the collision "ladder".  A real         */
/* collision ends the pair (its unused words are discarded), so the next     */
/* flight opens pair p + 1.  The t-th try of the angular sampler at the k-th */
/* flight of the history uses block (i, job, k, 1 + t); its word 3 is the    */
/* azimuth if that try is accepted.                                          */
/* ------------------------------------------------------------------------ */
static void rblock(const or_ctx* c, uint32_t i, uint32_t step, uint32_t sub, uint32_t x[4])
{
    uint32_t ctr[4] = { i, c->job, step, sub };
    or_philox(ctr, c->key, x);
}

/* Compton scattering, free-electron Klein-Nishina.  With kappa = E/mc^2 and
 * tau = E'/E in [tau0, 1], tau0 = 1/(1+2 kappa), the KN density in tau is
 * proportional to (1/tau + tau)(1 - tau sin^2/(1+tau^2)).  It is sampled as a
 * mixture of the densities 1/tau (weight ln(1/tau0)) and tau (weight
 * (1-tau0^2)/2), then accepted with probability 1 - tau sin^2/(1+tau^2). */
static void compton(const or_ctx* c, uint32_t i, uint32_t step, double E, double* tau_out, double* cos_out,
                    double* az_out, int* tries)
{
    double k = E / OR_ME_C2_KEV;
    double tau0 = 1.0 / (1.0 + 2.0 * k);
    double a1 = log(1.0 + 2.0 * k);
    double a2 = 0.5 * (1.0 - tau0 * tau0);
    for (uint32_t t = 0; t < OR_MAX_TRIES; ++t) {
        uint32_t x[4];
        rblock(c, i, step, 1 + t, x);
        double b0 = u24(x[0]), b1 = u24(x[1]), b2 = u24(x[2]);
        double tau;
        if (b0 * (a1 + a2) < a1) tau = exp(-a1 * b1);
        else tau = sqrt(tau0 * tau0 + (1.0 - tau0 * tau0) * b1);
        double cost = 1.0 - (1.0 - tau) / (k * tau);
        double sin2 = (1.0 - cost) * (1.0 + cost);
        double g = 1.0 - tau * sin2 / (1.0 + tau * tau);
        ++*tries;
        *az_out = u24(x[3]);
        if (b2 <= g) { *tau_out = tau; *cos_out = cost; return; }
    }
    *tau_out = 1.0; *cos_out = 1.0;
}

/* Rayleigh scattering with form factor F(x) = Z exp(-x/x0), x = sin(theta/2)/
 * lambda in [0, 1/lambda]: the density in x is proportional to
 * (1 + cos^2) x exp(-2x/x0) with cos = 1 - 2 (lambda x)^2.  Above
 * 1/lambda >= x0, x is drawn from Gamma(2, x0/2) and rejected beyond
 * 1/lambda; below, x is drawn with density ~ x on [0, 1/lambda] and kept with
 * probability exp(-2x/x0).  Either way it is then kept with probability
 * (1 + cos^2)/2. */
static double rayleigh(const or_ctx* c, uint32_t i, uint32_t step, double E, double x0, double* az_out,
                       int* tries)
{
    double xmax = E / OR_HC_KEV_A;
    for (uint32_t t = 0; t < OR_MAX_TRIES; ++t) {
        uint32_t x[4];
        rblock(c, i, step, 1 + t, x);
        double b0 = u24(x[0]), b1 = u24(x[1]), b2 = u24(x[2]);
        double xx;
        ++*tries;
        *az_out = u24(x[3]);
        if (xmax >= x0) {
            xx = -0.5 * x0 * log(b0 * b1);
            if (xx > xmax) continue;
        } else {
            xx = xmax * sqrt(b0);
            if (b1 > exp(-2.0 * xx / x0)) continue;
        }
        double r = xx / xmax;
        double cost = 1.0 - 2.0 * r * r;
        if (b2 <= 0.5 * (1.0 + cost * cost)) return cost;
    }
    return 1.0;
}

/* New direction at polar angle theta (cosine `cost`) and azimuth `ph` about
 * d: d' = cos(theta) d + sin(theta) (cos(ph) e1 + sin(ph) e2) with (e1, e2, d)
 * an orthonormal frame.  Away from the z axis e2 = (z x d)/|z x d| =
 * (-dy, dx, 0)/r and e1 = e2 x d = (dx dz, dy dz, -r^2)/r, r = |(dx, dy)|;
 * within 0.1 rad of it the frame is built on x instead: e2 = (x x d)/q =
 * (0, -dz, dy)/q and e1 = e2 x d = (-q^2, dx dy, dx dz)/q, q = |(dy, dz)|.
 * The result is renormalised. */
void or_rotate(const double d[3], double cost, double ph, double out[3])
{
    double sint = sqrt(fmax(0.0, 1.0 - cost * cost));
    double cph = cos(ph), sph = sin(ph);
    double e1[3], e2[3];
    double r = sqrt(d[0] * d[0] + d[1] * d[1]);
    if (r > 0.1) {
        e2[0] = -d[1] / r; e2[1] = d[0] / r; e2[2] = 0.0;
        e1[0] = d[0] * d[2] / r; e1[1] = d[1] * d[2] / r; e1[2] = -r;
    } else {
        double q = sqrt(d[1] * d[1] + d[2] * d[2]);
        e2[0] = 0.0; e2[1] = -d[2] / q; e2[2] = d[1] / q;
        e1[0] = -q; e1[1] = d[0] * d[1] / q; e1[2] = d[0] * d[2] / q;
    }
    double o[3];
    for (int a = 0; a < 3; ++a) o[a] = cost * d[a] + sint * (cph * e1[a] + sph * e2[a]);
    double nrm = sqrt(dot3(o, o));
    out[0] = o[0] / nrm; out[1] = o[1] / nrm; out[2] = o[2] / nrm;
}

/* ------------------------------------------------------------------------ */
/* Local majorants (not in the paper: Woodcock tracking only needs a bound   */
/* at every point, which may vary in space).  The phantom is cut into cubes  */
/* of M^3 voxels (the last ones along an axis shorter).  Positions in a cube */
/* take their density from voxel centres, and their material from the       */
/* containing voxel, within one voxel of the cube (the interpolation corners */
/* of any point in the cube, with one voxel to spare for rounding at its     */
/* faces), so mbar_B(E) = (1 + margin) rho_max(B) max_{m in B} mu_tot(m, E)  */
/* bounds mu there, with rho_max and the material set taken over the cube    */
/* grown by one voxel.  A flight draws an optical depth tau = -ln u and      */
/* spends it cube by cube along its line (each cube costs mbar_B times the   */
/* length inside it); the collision point is where tau runs out, tested      */
/* against that cube's mbar_B; running out of cubes is an escape.  rho_max   */
/* may be raised to a floor macro_rho_min: any larger bound is still a bound. */
/* Two more liberties a bound allows fix its exact values:                   */
/*  - the density factor (1 + margin) max(rho_max, floor) is kept with 19    */
/*    significant bits, rounded up;                                          */
/*  - within an energy interval [E_j, E_j+1] the material factor is the      */
/*    chord from max_{m in B} mu_tot(m, E_j) to max_{m in B} mu_tot(m,       */
/*    E_j+1).  Each mu_tot(m, .) is linear on the interval, so their maximum */
/*    is convex there and never above that chord; the two agree wherever one */
/*    material is the largest at both ends, and always for one material.     */
/* ------------------------------------------------------------------------ */

/* The least number with 19 significant bits that is >= v (v >= 0). */
static double round_up_19_bits(double v)
{
    if (!(v > 0.0)) return v;
    int e;
    const double m = frexp(v, &e);                 /* v = m 2^e, m in [1/2, 1) */
    return ldexp(ceil(ldexp(m, 19)), e - 19);
}
static int build_macro(const or_problem* p, or_ctx* c)
{
    const int M = p->macro;
    const int n[3] = { p->nx, p->ny, p->nz };
    if (p->n_mat > 64) return -1;
    for (int a = 0; a < 3; ++a) c->nb[a] = (n[a] + M - 1) / M;
    const size_t nb = (size_t)c->nb[0] * c->nb[1] * c->nb[2];
    c->mac_rho = (double*)calloc(nb, sizeof(double));
    c->mac_mask = (uint64_t*)calloc(nb, sizeof(uint64_t));
    if (!c->mac_rho || !c->mac_mask) return -1;
    for (int bz = 0; bz < c->nb[2]; ++bz)
        for (int by = 0; by < c->nb[1]; ++by)
            for (int bx = 0; bx < c->nb[0]; ++bx) {
                const int b[3] = { bx, by, bz };
                int lo[3], hi[3];
                for (int a = 0; a < 3; ++a) {
                    lo[a] = clampi(b[a] * M - 1, 0, n[a] - 1);
                    hi[a] = clampi((b[a] + 1) * M, 0, n[a] - 1);     /* inclusive: one voxel beyond the cube */
                }
                double r = p->macro_rho_min;
                uint64_t mask = 0;
                for (int z = lo[2]; z <= hi[2]; ++z)
                    for (int y = lo[1]; y <= hi[1]; ++y)
                        for (int x = lo[0]; x <= hi[0]; ++x) {
                            size_t v = vidx(p, x, y, z);
                            if ((double)p->density[v] > r) r = (double)p->density[v];
                            mask |= (uint64_t)1 << p->material[v];
                        }
                size_t bi = ((size_t)bz * c->nb[1] + by) * c->nb[0] + bx;
                c->mac_rho[bi] = round_up_19_bits((1.0 + p->macro_margin) * r);
                c->mac_mask[bi] = mask;
            }
    return 0;
}

static double macro_mbar(const or_problem* p, const or_ctx* c, size_t bi, double E)
{
    double f;
    const int j = e_interval(p, E, &f);
    double t0 = 0.0, t1 = 0.0;                     /* max mu_tot of the cube's materials at E_j, E_j+1 */
    for (int m = 0; m < p->n_mat; ++m) {
        if (!((c->mac_mask[bi] >> m) & 1u)) continue;
        const float* a = p->mu + ((size_t)m * p->n_e + j) * 3;
        const float* b = a + 3;
        const double s0 = (double)a[0] + (double)a[1] + (double)a[2];
        const double s1 = (double)b[0] + (double)b[1] + (double)b[2];
        if (s0 > t0) t0 = s0;
        if (s1 > t1) t1 = s1;
    }
    return c->mac_rho[bi] * (t0 + f * (t1 - t0));
}

/* Spends optical depth tau from pos along dir; on a collision moves pos there,
 * sets *mbar_out to the cube's bound and returns 1; returns 0 on leaving the
 * phantom (pos then on its boundary).  *crossings counts cube faces crossed. */
static int macro_flight(const or_problem* p, const or_ctx* c, double pos[3], const double dir[3], double E,
                        double tau, double* mbar_out, int* crossings)
{
    const int M = p->macro;
    const int n[3] = { p->nx, p->ny, p->nz };
    int b[3];
    for (int a = 0; a < 3; ++a)
        b[a] = clampi((int)floor((pos[a] - c->lo[a]) / (M * c->vs[a])), 0, c->nb[a] - 1);
    for (;;) {
        const size_t bi = ((size_t)b[2] * c->nb[1] + b[1]) * c->nb[0] + b[0];
        const double mb = macro_mbar(p, c, bi, E);
        double texit = INFINITY;
        int axis = 0;
        for (int a = 0; a < 3; ++a) {
            double t;
            if (dir[a] > 0.0) {
                int f = (b[a] + 1) * M < n[a] ? (b[a] + 1) * M : n[a];
                t = (c->lo[a] + f * c->vs[a] - pos[a]) / dir[a];
            } else if (dir[a] < 0.0) {
                t = (c->lo[a] + b[a] * M * c->vs[a] - pos[a]) / dir[a];
            } else {
                continue;
            }
            if (t < texit) { texit = t; axis = a; }
        }
        if (texit < 0.0) texit = 0.0;
        if (mb > 0.0 && tau < 0.1 * mb * texit) {            /* mbar in 1/cm, lengths in mm */
            const double s = tau / (0.1 * mb);
            for (int a = 0; a < 3; ++a) pos[a] += s * dir[a];
            *mbar_out = mb;
            return 1;
        }
        tau -= 0.1 * mb * texit;
        for (int a = 0; a < 3; ++a) pos[a] += texit * dir[a];
        b[axis] += dir[axis] > 0.0 ? 1 : -1;
        ++*crossings;
        if (b[axis] < 0 || b[axis] >= c->nb[axis]) return 0;
    }
}

/* ------------------------------------------------------------------------ */
/* One history, Sec. 2.4.                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int cls;
    int pixel;
    double e_src, e_final, recoil;
    int steps, n_real, n_compton, n_rayleigh, tries, crossings;
} or_outcome;

/* Visitor for tentative collisions inside the phantom (for the adjoint). */
typedef struct {
    double weight;          /* W of the history; 0 => no visit */
    double* grad;           /* [nz][ny][nx] */
} or_visit;

static void visit(const or_problem* p, const or_ctx* c, or_visit* vis, const double* x,
                  int real, double rho, double tot, double mbar)
{
    /* Score-function terms of delta tracking, the majorant held fixed:
     * real:  d log(rho mu_k / mbar)       / d rho_v = w_v / rho
     * null:  d log(1 - rho mu_tot / mbar) / d rho_v = -mu_tot w_v / (mbar - rho mu_tot) */
    size_t vox[8];
    double wt[8];
    if (c->interp) {
        trilinear(p, c, x, vox, wt);
        for (int n = 0; n < 8; ++n) {
            double s = real ? wt[n] / rho : -tot * wt[n] / (mbar - rho * tot);
            vis->grad[vox[n]] += vis->weight * s;
        }
    } else {
        size_t v = containing_voxel(p, c, x);
        double s = real ? 1.0 / rho : -tot / (mbar - rho * tot);
        vis->grad[v] += vis->weight * s;
    }
}

static void history(const or_problem* p, const or_ctx* c, uint32_t i, or_outcome* o, or_visit* vis)
{
    uint32_t x[4];
    rblock(c, i, 0, 0, x);
    int kf = cdf_search(c->cdf_f, p->nu * p->nv, u53(x[2], x[3]));
    int iu = kf % p->nu, iv = kf / p->nu;
    int row = p->spec_rows > 1 ? iu : 0;
    int ke = cdf_search(c->cdf_e + (size_t)row * p->n_spec, p->n_spec, u53(x[0], x[1]));
    rblock(c, i, 0, 1, x);
    double ju = u24(x[0]), jv = u24(x[1]);
    double E = (double)p->spec_e[ke];
    o->e_src = E; o->recoil = 0.0;
    o->steps = 0; o->n_real = 0; o->n_compton = 0; o->n_rayleigh = 0; o->tries = 0; o->crossings = 0;

    /* aim point D on the detector, uniform within the sampled pixel */
    double uc = ((double)iu + ju - 0.5 * p->nu) * p->du;
    double vc = ((double)iv + jv - 0.5 * p->nv) * p->dv;
    double pos[3], dir[3];
    for (int a = 0; a < 3; ++a) dir[a] = c->P[a] + uc * c->eu[a] + vc * c->ev[a] - c->S[a];
    double nd = sqrt(dot3(dir, dir));
    for (int a = 0; a < 3; ++a) { dir[a] /= nd; pos[a] = c->S[a]; }

    int scattered = 0;
    double tin, tout;
    if (box_entry(c, pos, dir, &tin, &tout)) {
        for (int a = 0; a < 3; ++a) pos[a] += tin * dir[a];
        double trem = tout - tin;
        uint32_t fb[4] = {0, 0, 0, 0};
        uint32_t pair = 0;
        int half = 2;                                         /* 2: the next flight opens a pair */
        for (uint32_t step = 1;; ++step) {
            if (step > OR_MAX_STEPS) { o->cls = OR_LOST; o->pixel = -1; o->e_final = E; return; }
            o->steps = (int)step;
            if (half == 2) { ++pair; rblock(c, i, pair, 0, fb); half = 0; }
            double r0 = u24(fb[2 * half]), r1 = u24(fb[2 * half + 1]);
            ++half;
            double mbar;
            if (p->macro > 0) {
                if (!macro_flight(p, c, pos, dir, E, -log(r0), &mbar, &o->crossings)) break;   /* escaped */
            } else {
                double f;
                int j = e_interval(p, E, &f);
                mbar = c->mbar[j];
                double s = -log(r0) / (0.1 * mbar);          /* mm; mbar in 1/cm */
                if (s >= trem) break;                         /* leaves the phantom */
                for (int a = 0; a < 3; ++a) pos[a] += s * dir[a];
                trem -= s;
            }
            size_t v = containing_voxel(p, c, pos);
            int m = p->material[v];
            double rho;
            if (c->interp) { size_t vv[8]; double ww[8]; rho = trilinear(p, c, pos, vv, ww); }
            else rho = (double)p->density[v];
            double mu3[3];
            xs_at(p, m, E, mu3);
            double tot = mu3[0] + mu3[1] + mu3[2];
            double mu = rho * tot;
            /* One uniform on [0, mbar) decides the event: Rayleigh below rho
             * mu_R, Compton below rho (mu_R + mu_C), photoelectric below mu,
             * null collision above -- probabilities rho mu_k / mbar and
             * 1 - mu / mbar, as delta tracking requires. */
            double ladder = r1 * mbar;
            int real = ladder < mu;
            if (vis) visit(p, c, vis, pos, real, rho, tot, mbar);
            if (!real) continue;                              /* null collision */
            o->n_real++;
            half = 2;                                         /* a real collision ends the pair */
            double cost, az = 0.0;
            if (ladder < rho * mu3[0]) {                      /* Rayleigh: E unchanged */
                cost = rayleigh(c, i, step, E, p->x0_rayleigh, &az, &o->tries);
                o->n_rayleigh++;
            } else if (ladder < rho * (mu3[0] + mu3[1])) {    /* Compton */
                double tau;
                compton(c, i, step, E, &tau, &cost, &az, &o->tries);
                o->recoil += E - tau * E;
                E = tau * E;
                o->n_compton++;
            } else {                                          /* photoelectric: history ends */
                o->cls = OR_ABSORBED; o->pixel = -1; o->e_final = E;
                return;
            }
            double nd2[3];
            or_rotate(dir, cost, 2.0 * M_PI * az, nd2);
            dir[0] = nd2[0]; dir[1] = nd2[1]; dir[2] = nd2[2];
            scattered = 1;
            if (E < p->e_cut) { o->cls = OR_CUT; o->pixel = -1; o->e_final = E; return; }
            if (p->macro <= 0) trem = box_exit(c, pos, dir);
        }
    }
    o->e_final = E;
    if (!scattered) {                   /* straight line to the sampled aim point */
        o->cls = OR_PRIMARY;
        o->pixel = iv * p->nu + iu;
        return;
    }
    /* vacuum outside the phantom: straight line to the detector plane */
    double dn = dot3(dir, c->n);
    if (dn > 0.0) {
        double w[3];
        for (int a = 0; a < 3; ++a) w[a] = c->P[a] - pos[a];
        double t = dot3(w, c->n) / dn;
        if (t >= 0.0) {
            double h[3];
            for (int a = 0; a < 3; ++a) h[a] = pos[a] + t * dir[a] - c->P[a];
            double fu = dot3(h, c->eu) / p->du + 0.5 * p->nu;
            double fv = dot3(h, c->ev) / p->dv + 0.5 * p->nv;
            double ku = floor(fu), kv = floor(fv);
            if (ku >= 0.0 && ku < p->nu && kv >= 0.0 && kv < p->nv) {
                o->cls = OR_SCATTER;
                o->pixel = (int)kv * p->nu + (int)ku;
                return;
            }
        }
    }
    o->cls = OR_MISSED;
    o->pixel = -1;
}

/* ------------------------------------------------------------------------ */
static int validate(const or_problem* p)
{
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (!(p->dx > 0 && p->dy > 0 && p->dz > 0)) return -1;
    if (!p->density || !p->material || !p->mu || !p->spec_e || !p->spec_p || !p->fluence) return -1;
    if (p->n_mat < 1 || p->n_mat > 256 || p->n_e < 2 || !(p->de > 0)) return -1;
    if (p->n_spec < 1 || p->nu < 1 || p->nv < 1 || !(p->du > 0 && p->dv > 0)) return -1;
    if (p->spec_rows < 0 || (p->spec_rows > 1 && p->spec_rows != p->nu)) return -1;
    double emax = p->e0 + p->de * (p->n_e - 1);
    for (int k = 0; k < p->n_spec; ++k)
        if (!(p->spec_e[k] >= p->e0 && p->spec_e[k] <= emax)) return -1;
    if (!(p->e_cut >= p->e0)) return -1;
    if (p->macro < 0 || (p->macro > 0 && (p->n_mat > 64 || !(p->macro_margin >= 0.0) ||
                                          !(p->macro_rho_min >= 0.0) || isinf(p->macro_rho_min)))) return -1;
    /* every voxel: a material of the table, a finite density >= 0 */
    size_t nvox = (size_t)p->nx * p->ny * p->nz;
    for (size_t v = 0; v < nvox; ++v)
        if (p->material[v] >= p->n_mat || !(p->density[v] >= 0.0f) || isinf(p->density[v])) return -1;
    /* the phantom must lie on the source side of the detector plane */
    double rxy = sqrt(0.25 * (p->nx * p->dx) * (p->nx * p->dx) + 0.25 * (p->ny * p->dy) * (p->ny * p->dy));
    if (!(rxy < p->aid) || !(rxy < p->sad)) return -1;
    return 0;
}

static int make_ctx(const or_problem* p, uint64_t seed, uint32_t job, int interp,
                    const double* mbar, or_ctx* c)
{
    memset(c, 0, sizeof(*c));
    setup_geometry(p, c);
    c->cdf_e = (double*)malloc(sizeof(double) * (size_t)spec_rows(p) * p->n_spec);
    c->cdf_f = (double*)malloc(sizeof(double) * (size_t)p->nu * p->nv);
    if (!c->cdf_e || !c->cdf_f) return -1;
    for (int r = 0; r < spec_rows(p); ++r)
        if (build_cdf(spec_row(p, r), p->n_spec, c->cdf_e + (size_t)r * p->n_spec)) return -1;
    if (build_cdf(p->fluence, p->nu * p->nv, c->cdf_f)) return -1;
    c->mbar = mbar;
    if (p->macro > 0 && build_macro(p, c)) return -1;
    c->key[0] = (uint32_t)seed;
    c->key[1] = (uint32_t)(seed >> 32);
    c->job = job;
    c->interp = interp;
    return 0;
}

static void free_ctx(or_ctx* c) { free(c->cdf_e); free(c->cdf_f); free(c->mac_rho); free(c->mac_mask); }

#define OR_CHUNK 4096

/* Type-specific scatter tally (Sec. 2.4 offers e.g. first-order Compton):
 * mode 0 counts every scattered photon, mode 1 only photons scattered exactly
 * once (Compton or Rayleigh), mode 2 only photons scattered exactly once by
 * Compton.  The primary tally is the same in every mode. */
static int counts_as_scatter(const or_outcome* o, int mode)
{
    if (mode == 1) return o->n_compton + o->n_rayleigh == 1;
    if (mode == 2) return o->n_compton == 1 && o->n_rayleigh == 0;
    return 1;
}

/*
 * The MC projection: n photons with ids 0..n-1 of job `job` under `seed`.
 * tally [4][nv][nu]: sum r(E), sum r(E)^2 over primary hits, then the same
 * over scatter hits, each divided by n (per source photon).  Optional
 * per-history outputs (any may be NULL): cls, pixel, e_final, steps,
 * n_compton, n_rayleigh.  `mode` selects the scatter tally (above).  stats[14] (optional): totals of steps, real events,
 * Compton, Rayleigh, histories per class [6], source energy, final energy plus
 * recoil energy, angular-sampler tries, cube faces crossed (local majorants).
 * `mbar` NULL => the majorant is computed here.
 */
int or_mc_project(const or_problem* p, uint64_t seed, uint64_t n, uint32_t job, int32_t interp,
                  int32_t mode, const double* mbar_in, double* tally, int8_t* cls, int32_t* pixel, double* e_final,
                  int32_t* steps, int32_t* n_compton, int32_t* n_rayleigh, double* stats, int32_t nthreads)
{
    if (validate(p) || !tally || n > 0xFFFFFFFFull) return -1;
    double* mb = NULL;
    if (!mbar_in && p->macro <= 0) {
        mb = (double*)malloc(sizeof(double) * (size_t)(p->n_e - 1));
        if (!mb || or_majorant(p, interp, mb)) { free(mb); return -1; }
    }
    or_ctx c;
    if (make_ctx(p, seed, job, interp, mbar_in ? mbar_in : mb, &c)) { free_ctx(&c); free(mb); return -1; }
    size_t npix = (size_t)p->nu * p->nv;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    double* part = (double*)calloc((size_t)nt * 4 * npix, sizeof(double));
    double* st = (double*)calloc((size_t)nt * 16, sizeof(double));
    if (!part || !st) { free(part); free(st); free_ctx(&c); free(mb); return -1; }
    uint64_t nchunks = (n + OR_CHUNK - 1) / OR_CHUNK;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double* my = part + (size_t)t * 4 * npix;
        double* ms = st + (size_t)t * 16;
        for (uint64_t ch = (uint64_t)t; ch < nchunks; ch += (uint64_t)nt) {
            uint64_t a = ch * OR_CHUNK, b = a + OR_CHUNK < n ? a + OR_CHUNK : n;
            for (uint64_t i = a; i < b; ++i) {
                or_outcome o;
                history(p, &c, (uint32_t)i, &o, NULL);
                if (o.cls == OR_PRIMARY || (o.cls == OR_SCATTER && counts_as_scatter(&o, mode))) {
                    double r = response_at(p, o.e_final);
                    size_t base = (o.cls == OR_PRIMARY ? 0 : 2) * npix + (size_t)o.pixel;
                    my[base] += r;
                    my[base + npix] += r * r;
                }
                if (cls) cls[i] = (int8_t)o.cls;
                if (pixel) pixel[i] = o.pixel;
                if (e_final) e_final[i] = o.e_final;
                if (steps) steps[i] = o.steps;
                if (n_compton) n_compton[i] = o.n_compton;
                if (n_rayleigh) n_rayleigh[i] = o.n_rayleigh;
                ms[0] += o.steps; ms[1] += o.n_real; ms[2] += o.n_compton; ms[3] += o.n_rayleigh;
                ms[4 + o.cls] += 1.0;
                ms[10] += o.e_src; ms[11] += o.e_final + o.recoil;
                ms[12] += o.tries;
                ms[13] += o.crossings;
            }
        }
    }
    double inv = n ? 1.0 / (double)n : 0.0;
    for (size_t k = 0; k < 4 * npix; ++k) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * 4 * npix + k];
        tally[k] = s * inv;
    }
    if (stats)
        for (int k = 0; k < 14; ++k) {
            double s = 0.0;
            for (int t = 0; t < nt; ++t) s += st[t * 16 + k];
            stats[k] = s;
        }
    free(part); free(st); free_ctx(&c); free(mb);
    return 0;
}

/*
 * Selected histories: the outcome of photons ids[k] (k < m) of job `job`,
 * exactly as or_mc_project computes them (for comparing sampled histories of
 * runs too large to repeat on the CPU).
 */
int or_mc_histories(const or_problem* p, uint64_t seed, uint32_t job, int32_t interp, const double* mbar,
                    const uint32_t* ids, int64_t m, int8_t* cls, int32_t* pixel, double* e_final,
                    int32_t* steps, int32_t* n_compton, int32_t* n_rayleigh, int32_t nthreads)
{
    if (validate(p) || (!mbar && p->macro <= 0) || !ids) return -1;
    or_ctx c;
    if (make_ctx(p, seed, job, interp, mbar, &c)) { free_ctx(&c); return -1; }
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#endif
    for (int64_t k = 0; k < m; ++k) {
        or_outcome o;
        history(p, &c, ids[k], &o, NULL);
        if (cls) cls[k] = (int8_t)o.cls;
        if (pixel) pixel[k] = o.pixel;
        if (e_final) e_final[k] = o.e_final;
        if (steps) steps[k] = o.steps;
        if (n_compton) n_compton[k] = o.n_compton;
        if (n_rayleigh) n_rayleigh[k] = o.n_rayleigh;
    }
    (void)nt;
    free_ctx(&c);
    return 0;
}

/*
 * Adjoint by path replay.  For a loss L(T) with adj = dL/dT over the primary
 * and scatter tallies ([2][nv][nu]), adds to grad[nz][ny][nx] the estimate
 *   dL/drho_v = (1/n) sum_i adj[c_i][p_i] r(E_i) sum_{events e of i} s_e(v)
 * with the score-function terms s_e of the visitor above.  Each history is run
 * once to find its outcome and, when its weight is non-zero, once more with
 * the same random numbers to visit its collisions.  `mbar` must be the
 * majorant of the forward run (it is held fixed under differentiation).
 */
int or_mc_backward(const or_problem* p, uint64_t seed, uint64_t n, uint32_t job, int32_t interp,
                   int32_t mode, const double* mbar, const double* adj, double* grad, int32_t nthreads)
{
    if (validate(p) || (!mbar && p->macro <= 0) || !adj || !grad || n > 0xFFFFFFFFull) return -1;
    or_ctx c;
    if (make_ctx(p, seed, job, interp, mbar, &c)) { free_ctx(&c); return -1; }
    size_t npix = (size_t)p->nu * p->nv;
    size_t nvox = (size_t)p->nx * p->ny * p->nz;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    double* part = (double*)calloc((size_t)nt * nvox, sizeof(double));
    if (!part) { free_ctx(&c); return -1; }
    uint64_t nchunks = (n + OR_CHUNK - 1) / OR_CHUNK;
    double inv = n ? 1.0 / (double)n : 0.0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        or_visit vis;
        vis.grad = part + (size_t)t * nvox;
        for (uint64_t ch = (uint64_t)t; ch < nchunks; ch += (uint64_t)nt) {
            uint64_t a = ch * OR_CHUNK, b = a + OR_CHUNK < n ? a + OR_CHUNK : n;
            for (uint64_t i = a; i < b; ++i) {
                or_outcome o;
                history(p, &c, (uint32_t)i, &o, NULL);
                if (o.cls != OR_PRIMARY && !(o.cls == OR_SCATTER && counts_as_scatter(&o, mode))) continue;
                double w = adj[(o.cls == OR_PRIMARY ? 0 : 1) * npix + (size_t)o.pixel]
                           * response_at(p, o.e_final) * inv;
                if (w == 0.0) continue;
                vis.weight = w;
                history(p, &c, (uint32_t)i, &o, &vis);
            }
        }
    }
    for (size_t k = 0; k < nvox; ++k) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * nvox + k];
        grad[k] += s;
    }
    free(part); free_ctx(&c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1, evaluated exactly for the density model the MC samples.  Along a  */
/* line, the containing voxel (hence the material) changes only at voxel     */
/* faces and the trilinear cell (and the clamping) only at the planes of     */
/* voxel centres; between consecutive such planes rho is a polynomial of     */
/* degree <= 3 in the arc length, so two-point Gauss-Legendre integrates it  */
/* exactly.  rho_int[m] receives the integral of rho over the pieces of      */
/* material m (mm * g/cm^3), so that int mu dl = 0.1 sum_m mu_tot(m,E)       */
/* rho_int[m] in dimensionless units.                                        */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int or_rho_integrals(const or_problem* p, int32_t interp, const double* a, const double* b, double* rho_int)
{
    or_ctx c;
    memset(&c, 0, sizeof(c));
    setup_geometry(p, &c);
    c.interp = interp;
    for (int m = 0; m < p->n_mat; ++m) rho_int[m] = 0.0;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = b[k] - a[k];
    double len = sqrt(dot3(d, d));
    if (!(len > 0.0)) return 0;
    for (int k = 0; k < 3; ++k) d[k] /= len;
    double tin, tout;
    if (!box_entry(&c, a, d, &tin, &tout)) return 0;
    if (tout > len) tout = len;
    if (!(tin < tout)) return 0;
    int cap = 2 * (2 * (p->nx + p->ny + p->nz) + 3) + 2;
    double* br = (double*)malloc(sizeof(double) * (size_t)cap);
    if (!br) return -1;
    int nb = 0;
    br[nb++] = tin;
    br[nb++] = tout;
    for (int ax = 0; ax < 3; ++ax) {
        if (d[ax] == 0.0) continue;
        for (int h = 0; h <= 2 * c.nvox[ax]; ++h) {          /* faces and centres */
            double plane = c.lo[ax] + 0.5 * h * c.vs[ax];
            double t = (plane - a[ax]) / d[ax];
            if (t > tin && t < tout) br[nb++] = t;
        }
    }
    qsort(br, (size_t)nb, sizeof(double), cmp_double);
    const double gq = 0.5 / sqrt(3.0);
    for (int k = 0; k + 1 < nb; ++k) {
        double t0 = br[k], t1 = br[k + 1];
        if (!(t1 > t0)) continue;
        double mid[3], x[3];
        for (int q = 0; q < 3; ++q) mid[q] = a[q] + 0.5 * (t0 + t1) * d[q];
        int m = p->material[containing_voxel(p, &c, mid)];
        double acc = 0.0;
        for (int g = -1; g <= 1; g += 2) {
            double t = 0.5 * (t0 + t1) + g * gq * (t1 - t0);
            for (int q = 0; q < 3; ++q) x[q] = a[q] + t * d[q];
            if (interp) { size_t vv[8]; double ww[8]; acc += trilinear(p, &c, x, vv, ww); }
            else acc += (double)p->density[containing_voxel(p, &c, x)];
        }
        rho_int[m] += 0.5 * (t1 - t0) * acc;
    }
    free(br);
    return 0;
}

/*
 * Expected primary tally E[P_hat] per pixel ([nv][nu], per source photon):
 *   sum_j phi_j W_p r(E_j) <exp(-int mu dl)>_p
 * where phi_j, W_p are the normalised spectrum (the row of the pixel's column
 * for a joint source) and fluence weights and <.>_p
 * averages over the pixel (the aim point is uniform inside it) with an
 * nq x nq Gauss-Legendre rule.
 */
int or_primary_exact(const or_problem* p, int32_t interp, int32_t nq, double* out)
{
    if (validate(p) || nq < 1 || nq > 64) return -1;
    or_ctx c;
    memset(&c, 0, sizeof(c));
    setup_geometry(p, &c);
    /* Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_nq */
    double gx[64], gw[64];
    for (int k = 0; k < nq; ++k) {
        double z = cos(M_PI * (k + 0.75) / (nq + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int l = 1; l <= nq; ++l) { double p2 = p1; p1 = p0; p0 = ((2 * l - 1) * z * p1 - (l - 1) * p2) / l; }
            double dp = nq * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-15) break;
        }
        double p0 = 1.0, p1 = 0.0;
        for (int l = 1; l <= nq; ++l) { double p2 = p1; p1 = p0; p0 = ((2 * l - 1) * z * p1 - (l - 1) * p2) / l; }
        double dp = nq * (z * p0 - p1) / (z * z - 1.0);
        gx[k] = 0.5 * (1.0 - z);
        gw[k] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    double sf = 0.0;
    for (int k = 0; k < p->nu * p->nv; ++k) sf += p->fluence[k];
    double* ri = (double*)malloc(sizeof(double) * (size_t)p->n_mat);
    double* muj = (double*)malloc(sizeof(double) * (size_t)p->n_spec * p->n_mat);
    if (!ri || !muj) { free(ri); free(muj); return -1; }
    for (int k = 0; k < p->n_spec; ++k)
        for (int m = 0; m < p->n_mat; ++m) {
            double mu3[3];
            xs_at(p, m, p->spec_e[k], mu3);
            muj[(size_t)k * p->n_mat + m] = mu3[0] + mu3[1] + mu3[2];
        }
    for (int iv = 0; iv < p->nv; ++iv)
        for (int iu = 0; iu < p->nu; ++iu) {
            const float* phi = spec_row(p, iu);
            double sp = 0.0;
            for (int k = 0; k < p->n_spec; ++k) sp += phi[k];
            double acc = 0.0;
            for (int qa = 0; qa < nq; ++qa)
                for (int qb = 0; qb < nq; ++qb) {
                    double uc = ((double)iu + gx[qa] - 0.5 * p->nu) * p->du;
                    double vc = ((double)iv + gx[qb] - 0.5 * p->nv) * p->dv;
                    double D[3];
                    for (int q = 0; q < 3; ++q) D[q] = c.P[q] + uc * c.eu[q] + vc * c.ev[q];
                    if (or_rho_integrals(p, interp, c.S, D, ri)) { free(ri); free(muj); return -1; }
                    double e_sum = 0.0;
                    for (int k = 0; k < p->n_spec; ++k) {
                        double li = 0.0;
                        for (int m = 0; m < p->n_mat; ++m) li += muj[(size_t)k * p->n_mat + m] * ri[m];
                        e_sum += (phi[k] / sp) * response_at(p, p->spec_e[k]) * exp(-0.1 * li);
                    }
                    acc += gw[qa] * gw[qb] * e_sum;
                }
            out[iv * p->nu + iu] = (p->fluence[iv * p->nu + iu] / sf) * acc;
        }
    free(ri); free(muj);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sampler access for the tests: n draws at energy E, photon ids 0..n-1,     */
/* step 1, the same try layout as in transport.                              */
/* ------------------------------------------------------------------------ */
int or_sample_compton(double E, uint64_t seed, uint64_t n, double* cost, double* tau)
{
    or_ctx c;
    memset(&c, 0, sizeof(c));
    c.key[0] = (uint32_t)seed; c.key[1] = (uint32_t)(seed >> 32);
    int tries = 0;
    double az;
    for (uint64_t i = 0; i < n; ++i) compton(&c, (uint32_t)i, 1, E, &tau[i], &cost[i], &az, &tries);
    return 0;
}

int or_sample_rayleigh(double E, double x0, uint64_t seed, uint64_t n, double* cost)
{
    or_ctx c;
    memset(&c, 0, sizeof(c));
    c.key[0] = (uint32_t)seed; c.key[1] = (uint32_t)(seed >> 32);
    int tries = 0;
    double az;
    for (uint64_t i = 0; i < n; ++i) cost[i] = rayleigh(&c, (uint32_t)i, 1, E, x0, &az, &tries);
    return 0;
}

/* Geometry frame for the tests: S, P, n, eu, ev (15 doubles). */
void or_geometry(const or_problem* p, double* out15)
{
    or_ctx c;
    memset(&c, 0, sizeof(c));
    setup_geometry(p, &c);
    for (int k = 0; k < 3; ++k) {
        out15[k] = c.S[k]; out15[3 + k] = c.P[k]; out15[6 + k] = c.n[k];
        out15[9 + k] = c.eu[k]; out15[12 + k] = c.ev[k];
    }
}

/* Trilinear density at points (tests). */
int or_density_at(const or_problem* p, int32_t interp, const double* xyz, int64_t m, double* out)
{
    or_ctx c;
    memset(&c, 0, sizeof(c));
    setup_geometry(p, &c);
    for (int64_t k = 0; k < m; ++k) {
        const double* x = xyz + 3 * k;
        if (interp) { size_t vv[8]; double ww[8]; out[k] = trilinear(p, &c, x, vv, ww); }
        else out[k] = (double)p->density[containing_voxel(p, &c, x)];
    }
    return 0;
}

/* Batched form of or_rho_integrals: segments a -> b[k], k < m; out [m][n_mat]. */
int or_rho_integrals_many(const or_problem* p, int32_t interp, const double* a, const double* b,
                          int64_t m, double* out)
{
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(|:bad)
#endif
    for (int64_t k = 0; k < m; ++k)
        bad |= or_rho_integrals(p, interp, a, b + 3 * k, out + (size_t)k * p->n_mat) != 0;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Primary signal by ray tracing, Sec. 2.3, Eq. 1:                           */
/*   P(u) = sum_k phi_k w(u) r(E_k) exp(-sum_j dl_j mu(x_j, E_k))            */
/* over the spectrum's energy channels.  The ray runs from the source to the */
/* centre of pixel u.  Its length from the source is cut into intervals     */
/* [j dl, (j+1) dl); the part of each interval inside the phantom box is     */
/* one term, with mu taken at that part's midpoint (all terms have length dl */
/* except the two cut by the box faces).  mu(x, E) is the trilinear          */
/* interpolation of the voxel attenuation coefficients rho_v mu_tot(m_v, E)  */
/* on the lattice of voxel centres (clamped at the edges); with the          */
/* interpolation off it is the containing voxel's value.  dl <= 0 selects    */
/* half of the smallest voxel edge.  phi and w are normalised to sum 1; for */
/* a joint source phi is the row of the pixel's column.                      */
/* Pixels: the m indices iv * nu + iu in pix, or all pixels when pix is      */
/* NULL (out is then [nv][nu]).                                              */
/* ------------------------------------------------------------------------ */
int or_primary_raytrace(const or_problem* p, int32_t interp, double dl, const int32_t* pix, int64_t m,
                        double* out)
{
    if (validate(p)) return -1;
    const int64_t npx = pix ? m : (int64_t)p->nu * p->nv;
    if (pix)
        for (int64_t q = 0; q < m; ++q)
            if (pix[q] < 0 || pix[q] >= p->nu * p->nv) return -1;
    for (size_t v = 0; v < (size_t)p->nx * p->ny * p->nz; ++v)
        if (p->material[v] >= p->n_mat) return -1;
    if (!(dl > 0.0)) {
        dl = p->dx;
        if (p->dy < dl) dl = p->dy;
        if (p->dz < dl) dl = p->dz;
        dl *= 0.5;
    }
    or_ctx c;
    memset(&c, 0, sizeof(c));
    setup_geometry(p, &c);
    double sf = 0.0;
    for (int k = 0; k < p->nu * p->nv; ++k) sf += p->fluence[k];
    if (!(sf > 0.0)) return -1;
    for (int r = 0; r < spec_rows(p); ++r) {
        double sp = 0.0;
        for (int k = 0; k < p->n_spec; ++k) sp += spec_row(p, r)[k];
        if (!(sp > 0.0)) return -1;
    }
    /* total mass attenuation of every material at every channel energy */
    double* mut = (double*)malloc(sizeof(double) * (size_t)p->n_spec * p->n_mat);
    if (!mut) return -1;
    for (int k = 0; k < p->n_spec; ++k)
        for (int mm = 0; mm < p->n_mat; ++mm) {
            double mu3[3];
            xs_at(p, mm, p->spec_e[k], mu3);
            mut[(size_t)k * p->n_mat + mm] = mu3[0] + mu3[1] + mu3[2];
        }
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel reduction(|:bad)
#endif
    {
        double* L = (double*)malloc(sizeof(double) * (size_t)p->n_spec);
        if (!L) bad = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t q = 0; q < npx; ++q) {
            if (!L) continue;
            const int id = pix ? pix[q] : (int)q;
            const int iu = id % p->nu, iv = id / p->nu;
            const double uc = ((double)iu + 0.5 - 0.5 * p->nu) * p->du;
            const double vc = ((double)iv + 0.5 - 0.5 * p->nv) * p->dv;
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = c.P[a] + uc * c.eu[a] + vc * c.ev[a] - c.S[a];
            const double len = sqrt(dot3(d, d));
            for (int a = 0; a < 3; ++a) d[a] /= len;
            for (int k = 0; k < p->n_spec; ++k) L[k] = 0.0;
            double tin, tout;
            if (box_entry(&c, c.S, d, &tin, &tout)) {
                if (tout > len) tout = len;
                const int64_t j0 = (int64_t)floor(tin / dl), j1 = (int64_t)ceil(tout / dl);
                for (int64_t j = j0; j < j1; ++j) {
                    double a = (double)j * dl, b = (double)(j + 1) * dl;
                    if (a < tin) a = tin;
                    if (b > tout) b = tout;
                    if (!(b > a)) continue;
                    double x[3];
                    for (int r = 0; r < 3; ++r) x[r] = c.S[r] + 0.5 * (a + b) * d[r];
                    if (interp) {
                        size_t vox[8];
                        double wt[8];
                        trilinear(p, &c, x, vox, wt);
                        for (int k = 0; k < p->n_spec; ++k) {
                            double mu = 0.0;
                            for (int s = 0; s < 8; ++s)
                                mu += wt[s] * (double)p->density[vox[s]] *
                                      mut[(size_t)k * p->n_mat + p->material[vox[s]]];
                            L[k] += (b - a) * mu;
                        }
                    } else {
                        const size_t v = containing_voxel(p, &c, x);
                        for (int k = 0; k < p->n_spec; ++k)
                            L[k] += (b - a) * (double)p->density[v] * mut[(size_t)k * p->n_mat + p->material[v]];
                    }
                }
            }
            const float* phi = spec_row(p, iu);
            double sp = 0.0, acc = 0.0;
            for (int k = 0; k < p->n_spec; ++k) sp += phi[k];
            for (int k = 0; k < p->n_spec; ++k)       /* mm * 1/cm -> 0.1 */
                acc += (phi[k] / sp) * response_at(p, p->spec_e[k]) * exp(-0.1 * L[k]);
            out[q] = ((double)p->fluence[id] / sf) * acc;
        }
        free(L);
    }
    free(mut);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Scatter denoising, Sec. 2.5: the iteration of Eq. 5,                      */
/*   S'(i,j) = (1 - w) S(i,j) + (w/4) [sum of the 4 neighbours of S(i,j)     */
/*             - (1/beta) (1 - Shat(i,j) / S(i,j))],                         */
/* with every value on the right taken from the previous iterate and         */
/* S^(0) = Shat.  At the detector edge a missing neighbour takes the pixel's */
/* own value (no flux through the edge, the boundary condition under which   */
/* Eq. 4 is the optimality condition of the discretised Eq. 2).  The data    */
/* term is 1 where Shat = 0; iterates are kept at or above s_floor > 0 so    */
/* that Shat / S stays defined.  images: [n_img][nv][nu]; s0 may be NULL     */
/* (then S^(0) = Shat).                                                      */
/* ------------------------------------------------------------------------ */
int or_denoise(const double* shat, const double* s0, int32_t n_img, int32_t nv, int32_t nu, double beta,
               double omega, int32_t iters, double s_floor, double* out)
{
    if (!shat || !out || n_img < 1 || nv < 1 || nu < 1 || !(beta > 0.0) || !(s_floor > 0.0) || iters < 0)
        return -1;
    const size_t npx = (size_t)nv * nu;
    double* a = (double*)malloc(sizeof(double) * npx);
    double* b = (double*)malloc(sizeof(double) * npx);
    if (!a || !b) { free(a); free(b); return -1; }
    for (int32_t m = 0; m < n_img; ++m) {
        const double* h = shat + (size_t)m * npx;
        const double* g = s0 ? s0 + (size_t)m * npx : h;
        for (size_t k = 0; k < npx; ++k) a[k] = g[k] > s_floor ? g[k] : s_floor;
        for (int32_t it = 0; it < iters; ++it) {
            for (int32_t i = 0; i < nv; ++i)
                for (int32_t j = 0; j < nu; ++j) {
                    const double s = a[(size_t)i * nu + j];
                    const double up = i > 0 ? a[(size_t)(i - 1) * nu + j] : s;
                    const double dn = i + 1 < nv ? a[(size_t)(i + 1) * nu + j] : s;
                    const double lf = j > 0 ? a[(size_t)i * nu + j - 1] : s;
                    const double rt = j + 1 < nu ? a[(size_t)i * nu + j + 1] : s;
                    const double hk = h[(size_t)i * nu + j];
                    const double data = hk == 0.0 ? 1.0 : 1.0 - hk / s;
                    double v = (1.0 - omega) * s + 0.25 * omega * ((up + dn + lf + rt) - data / beta);
                    b[(size_t)i * nu + j] = v > s_floor ? v : s_floor;
                }
            double* t = a; a = b; b = t;
        }
        memcpy(out + (size_t)m * npx, a, sizeof(double) * npx);
    }
    free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Noise assembly, Sec. 2.6: the MC noise Nhat = (Phat - P) + (Shat - S)     */
/* (the second Eq. 4), scaled by alpha = sqrt(n_sim / (zeta I)) (the second  */
/* Eq. 5) to the noise of a scan at I mAs: N = alpha Nhat; the simulated     */
/* projection is P + S + N.  Either output may be NULL.                      */
/* ------------------------------------------------------------------------ */
int or_noise(int64_t n, const double* phat, const double* p, const double* shat, const double* s, double alpha,
             double* noise, double* image)
{
    if (n < 0 || !phat || !p || !shat || !s) return -1;
    for (int64_t k = 0; k < n; ++k) {
        const double nn = alpha * ((phat[k] - p[k]) + (shat[k] - s[k]));
        if (noise) noise[k] = nn;
        if (image) image[k] = p[k] + s[k] + nn;
    }
    return 0;
}

/* Sec. 2.6, second Eq. 5: alpha = sqrt(n_sim / (zeta I)), I the mAs level and
 * zeta the effective source photons per mAs. */
double or_noise_scale(double n_sim, double zeta, double mas)
{
    if (!(n_sim > 0.0) || !(zeta > 0.0) || !(mas > 0.0)) return -1.0;
    return sqrt(n_sim / (zeta * mas));
}

/* Tests: the local majorant of the cube holding each position xyz[k] at
 * energy e[k] (macro > 0 required). */
int or_local_majorant_at(const or_problem* p, const double* xyz, const double* e, int64_t m, double* out)
{
    if (validate(p) || p->macro <= 0) return -1;
    or_ctx c;
    memset(&c, 0, sizeof(c));
    setup_geometry(p, &c);
    if (build_macro(p, &c)) { free_ctx(&c); return -1; }
    for (int64_t k = 0; k < m; ++k) {
        int b[3];
        for (int a = 0; a < 3; ++a)
            b[a] = clampi((int)floor((xyz[3 * k + a] - c.lo[a]) / (p->macro * c.vs[a])), 0, c.nb[a] - 1);
        out[k] = macro_mbar(p, &c, ((size_t)b[2] * c.nb[1] + b[1]) * c.nb[0] + b[0], e[k]);
    }
    free_ctx(&c);
    return 0;
}
