// Host side of libgdrr: argument checks, workspace layout, launch plans,
// the cached HIP graph of a batch, and the C ABI of include/gdrr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gdrr.h"
#include "gdrr_kernels.h"
#include "gdrr_raytrace.h"
#include "gdrr_denoise.h"

using namespace gdrr;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define GDRR_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail(GDRR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// --------------------------------------------------------------------------
// Device properties, read once per device.
// --------------------------------------------------------------------------
struct DevInfo {
    int cus = 0;
    size_t lds_max = 0;      // per workgroup
    bool ok = false;
};

std::mutex g_dev_mu;
DevInfo g_dev[64];

int device_info(DevInfo& out) {
    int dev = 0;
    GDRR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(GDRR_ENOTSUP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev[dev].ok) {
        hipDeviceProp_t prop;
        GDRR_HIP(hipGetDeviceProperties(&prop, dev));
        g_dev[dev].cus = prop.multiProcessorCount;
        g_dev[dev].lds_max = prop.sharedMemPerBlock;
        g_dev[dev].ok = true;
    }
    out = g_dev[dev];
    return GDRR_OK;
}

// --------------------------------------------------------------------------
// Workspace carving: the same walk sizes the workspace (base == nullptr) and
// lays it out.
// --------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// Rows of a source's spectrum table (one, or one per detector column); -1 if invalid.
int spec_rows(const gdrr_source& s) {
    if (s.spec_rows == 0 || s.spec_rows == 1) return 1;
    return s.spec_rows == s.fu && s.fu > 1 ? s.spec_rows : -1;
}

uint32_t guide_size(int n) {
    uint32_t k = 1;
    while ((int)k < n && k < (1u << 20)) k <<= 1;
    return k;
}

// --------------------------------------------------------------------------
// Argument checks.
// --------------------------------------------------------------------------
int check_volume(const gdrr_volume* v) {
    if (!v) return fail(GDRR_EINVAL, "volume is NULL");
    if (v->nx < 1 || v->ny < 1 || v->nz < 1) return fail(GDRR_EINVAL, "volume dimensions must be >= 1");
    if ((long long)v->nx * v->ny * v->nz >= (1ll << 31)) return fail(GDRR_EINVAL, "volume has 2^31 voxels or more");
    // cell records are indexed in 32-bit arithmetic
    if ((long long)(v->nx + 1) * (v->ny + 1) * (v->nz + 1) >= (1ll << 31))
        return fail(GDRR_EINVAL, "volume has 2^31 interpolation cells or more ((nx+1)(ny+1)(nz+1))");
    if (!(v->dx_mm > 0 && v->dy_mm > 0 && v->dz_mm > 0)) return fail(GDRR_EINVAL, "voxel sizes must be > 0");
    if (!v->density || !v->material) return fail(GDRR_EINVAL, "volume density/material pointer is NULL");
    if (v->macro < 0 || v->macro > 256) return fail(GDRR_EINVAL, "volume macro must be in [0, 256]");
    if (v->macro > 0 && (!(v->macro_margin >= 0.0f) || !std::isfinite(v->macro_margin)))
        return fail(GDRR_EINVAL, "volume macro_margin must be finite and >= 0");
    if (v->macro > 0 && (!(v->macro_rho_min >= 0.0f) || !std::isfinite(v->macro_rho_min)))
        return fail(GDRR_EINVAL, "volume macro_rho_min must be finite and >= 0");
    return GDRR_OK;
}

int cubes(int n, int m) { return (n + m - 1) / m; }

#ifndef GDRR_MACRO_LDS_MAX
#define GDRR_MACRO_LDS_MAX (32 << 10)
#endif
constexpr size_t kMacroLdsMax = GDRR_MACRO_LDS_MAX;   // bytes of cube records staged in LDS
// LDS allocation granule of a gfx950 workgroup (160 KiB / 128), as measured by
// calib/lds_granule: three 512-thread workgroups share a compute unit up to 42
// granules (53760 bytes) each, where hipOccupancyMaxActiveBlocksPerMultiprocessor
// still reports three up to 54528.
constexpr size_t kLdsGranule = 1280;

int check_physics(const gdrr_physics* p) {
    if (!p) return fail(GDRR_EINVAL, "physics is NULL");
    if (p->n_mat < 1 || p->n_mat > GDRR_MAX_MATERIALS) return fail(GDRR_EINVAL, "n_mat must be in [1, 16]");
    if (p->n_e < 2 || p->n_e > 1024) return fail(GDRR_EINVAL, "n_e must be in [2, 1024]");
    if (!(p->de_kev > 0) || !(p->e0_kev > 0)) return fail(GDRR_EINVAL, "energy grid must have e0 > 0 and de > 0");
    if (!p->mu_mass) return fail(GDRR_EINVAL, "mu_mass is NULL");
    if (!(p->e_cut_kev >= p->e0_kev)) return fail(GDRR_EINVAL, "e_cut must be >= e0");
    if (!(p->rayleigh_x0_invA > 0)) return fail(GDRR_EINVAL, "rayleigh x0 must be > 0");
    return GDRR_OK;
}

int check_source(const gdrr_source* s) {
    if (!s) return fail(GDRR_EINVAL, "source is NULL");
    if (s->n_spec < 1 || s->n_spec > 4096) return fail(GDRR_EINVAL, "n_spec must be in [1, 4096]");
    if (!s->spec_e_kev || !s->spec_prob || !s->fluence) return fail(GDRR_EINVAL, "source pointer is NULL");
    if (s->fu < 1 || s->fv < 1 || (long long)s->fu * s->fv > (1ll << 24))
        return fail(GDRR_EINVAL, "fluence grid must have 1 <= fu*fv <= 2^24");
    if (spec_rows(*s) < 0) return fail(GDRR_EINVAL, "spec_rows must be 0, 1 or fu");
    if ((long long)spec_rows(*s) * s->n_spec > (1ll << 24)) return fail(GDRR_EINVAL, "spec_rows * n_spec must be <= 2^24");
    return GDRR_OK;
}

int check_geometry(const gdrr_geometry* g, const gdrr_volume* v, const gdrr_source* s) {
    if (!g) return fail(GDRR_EINVAL, "geometry is NULL");
    if (!(g->sad_mm > 0 && g->aid_mm > 0)) return fail(GDRR_EINVAL, "SAD and AID must be > 0");
    if (g->nu < 1 || g->nv < 1 || !(g->du_mm > 0 && g->dv_mm > 0)) return fail(GDRR_EINVAL, "bad detector grid");
    if (!std::isfinite(g->phi_rad) || !std::isfinite(g->theta_rad)) return fail(GDRR_EINVAL, "angles must be finite");
    if (s && (s->fu != g->nu || s->fv != g->nv))
        return fail(GDRR_EINVAL, "the fluence grid must be the detector's pixel grid (fu = nu, fv = nv)");
    if (v) {
        const double hx = 0.5 * v->nx * v->dx_mm, hy = 0.5 * v->ny * v->dy_mm;
        const double r = std::sqrt(hx * hx + hy * hy);
        if (!(r < g->aid_mm) || !(r < g->sad_mm))
            return fail(GDRR_EINVAL, "the phantom must lie between the source and the detector at every angle");
    }
    return GDRR_OK;
}

// --------------------------------------------------------------------------
// Timing hook: HIP events around the transport kernel, on the call's stream.
// --------------------------------------------------------------------------
struct TimeEvents {
    hipEvent_t a = nullptr, b = nullptr;
    bool recorded = false;
};

std::mutex g_time_mu;
bool g_timing = false;
TimeEvents g_tev[64];

int timing_events(TimeEvents** out) {
    int dev = 0;
    GDRR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(GDRR_ENOTSUP, "device index out of range");
    TimeEvents& t = g_tev[dev];
    if (!t.a) GDRR_HIP(hipEventCreate(&t.a));
    if (!t.b) GDRR_HIP(hipEventCreate(&t.b));
    *out = &t;
    return GDRR_OK;
}

// --------------------------------------------------------------------------
// Launch list: every kernel takes one parameter struct by value, so a launch
// is (function, grid, block, LDS bytes, argument bytes).  The list runs either
// directly or as a HIP graph.
// --------------------------------------------------------------------------
struct Launch {
    const void* func;
    dim3 grid, block;
    size_t shmem;
    std::vector<char> args;
};

template <class P>
Launch make_launch(const void* f, dim3 g, dim3 b, size_t sh, const P& p) {
    Launch L{f, g, b, sh, std::vector<char>(sizeof(P))};
    std::memcpy(L.args.data(), &p, sizeof(P));
    return L;
}

// Launches [timed, timed_last] are bracketed with `ev` (timed = -1: none;
// timed_last = -1: the single launch `timed`).
int run_direct(std::vector<Launch>& ls, hipStream_t st, int timed = -1, TimeEvents* ev = nullptr,
               int timed_last = -1) {
    if (timed_last < 0) timed_last = timed;
    for (size_t i = 0; i < ls.size(); ++i) {
        Launch& L = ls[i];
        void* a[1] = {L.args.data()};
        if ((int)i == timed) GDRR_HIP(hipEventRecord(ev->a, st));
        GDRR_HIP(hipLaunchKernel(L.func, L.grid, L.block, a, L.shmem, st));
        if (timed >= 0 && (int)i == timed_last) {
            GDRR_HIP(hipEventRecord(ev->b, st));
            ev->recorded = true;
        }
    }
    return GDRR_OK;
}

std::vector<char> launch_key(const std::vector<Launch>& ls) {
    std::vector<char> k;
    for (auto& L : ls) {
        const char* f = (const char*)&L.func;
        k.insert(k.end(), f, f + sizeof(L.func));
        unsigned dims[7] = {L.grid.x, L.grid.y, L.grid.z, L.block.x, L.block.y, L.block.z, (unsigned)L.shmem};
        k.insert(k.end(), (const char*)dims, (const char*)dims + sizeof(dims));
        k.insert(k.end(), L.args.begin(), L.args.end());
    }
    return k;
}

struct GraphEntry {
    int device = -1;
    std::vector<char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

std::mutex g_graph_mu;
GraphEntry g_graphs[4];
int g_graph_next = 0;

int run_graph(std::vector<Launch>& ls, hipStream_t st, int timed = -1, TimeEvents* ev = nullptr) {
    int dev = 0;
    GDRR_HIP(hipGetDevice(&dev));
    std::vector<char> key = launch_key(ls);
    {
        const int t[1] = {timed};
        key.insert(key.end(), (const char*)t, (const char*)t + sizeof(t));
        const void* e[2] = {ev ? (const void*)ev->a : nullptr, ev ? (const void*)ev->b : nullptr};
        key.insert(key.end(), (const char*)e, (const char*)e + sizeof(e));
    }
    if (ev && timed >= 0) ev->recorded = true;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& e : g_graphs)
        if (e.exec && e.device == dev && e.key == key) {
            GDRR_HIP(hipGraphLaunch(e.exec, st));
            return GDRR_OK;
        }
    GraphEntry& e = g_graphs[g_graph_next];
    g_graph_next = (g_graph_next + 1) % 4;
    if (e.exec) { (void)hipGraphExecDestroy(e.exec); e.exec = nullptr; }
    if (e.graph) { (void)hipGraphDestroy(e.graph); e.graph = nullptr; }
    GDRR_HIP(hipGraphCreate(&e.graph, 0));
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; i < ls.size(); ++i) {
        Launch& L = ls[i];
        if ((int)i == timed) {
            hipGraphNode_t en;
            GDRR_HIP(hipGraphAddEventRecordNode(&en, e.graph, prev ? &prev : nullptr, prev ? 1 : 0, ev->a));
            prev = en;
        }
        hipKernelNodeParams kp{};
        void* a[1] = {L.args.data()};
        kp.func = const_cast<void*>(L.func);
        kp.gridDim = L.grid;
        kp.blockDim = L.block;
        kp.sharedMemBytes = (unsigned)L.shmem;
        kp.kernelParams = a;
        kp.extra = nullptr;
        hipGraphNode_t node;
        GDRR_HIP(hipGraphAddKernelNode(&node, e.graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = node;
        if ((int)i == timed) {
            hipGraphNode_t en;
            GDRR_HIP(hipGraphAddEventRecordNode(&en, e.graph, &prev, 1, ev->b));
            prev = en;
        }
    }
    GDRR_HIP(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
    e.device = dev;
    e.key = std::move(key);
    GDRR_HIP(hipGraphLaunch(e.exec, st));
    return GDRR_OK;
}

// --------------------------------------------------------------------------
// A batch plan: host-side tables and the workspace layout.
// --------------------------------------------------------------------------
struct SrcArea {
    double* spec_cdf;
    uint32_t* spec_guide;
    double* flu_cdf;
    uint32_t* flu_guide;
    uint32_t spec_k, flu_k;
};

struct Layout {
    unsigned long long* counter;      // [8]: dispenser, error word
    unsigned long long* chunk_prefix; // [n_jobs + 1]
    DJob* jobs;                       // [n_jobs]
    long long* out_off;               // [n_jobs]
    float* majorants;                 // [n_vols][n_e - 1] (when computed)
    unsigned int* rho_max;            // [n_vols][256]
    unsigned int* present;            // [n_vols][256]
    SrcArea src[GDRR_MAX_SOURCES];
    CellRec* cells[GDRR_MAX_VOLUMES]; // per-volume cell records
    uint2* macro[GDRR_MAX_VOLUMES];   // per-volume local majorants (volumes with macro > 0)
    unsigned long long* tally;        // fixed-point tallies
    size_t tally_elems;
    size_t bytes;
};

size_t cell_count(const gdrr_volume& v) {
    return (size_t)(v.nx + 1) * (size_t)(v.ny + 1) * (size_t)(v.nz + 1);
}

Layout carve(void* ws, const gdrr_volume* vols, const gdrr_physics* phys, const gdrr_source* srcs, int n_srcs,
             int n_jobs, int n_vols, size_t tally_elems, bool need_majorant) {
    Carver c(ws);
    Layout L{};
    L.counter = c.take<unsigned long long>(8);
    L.chunk_prefix = c.take<unsigned long long>((size_t)n_jobs + 1);
    L.jobs = c.take<DJob>((size_t)n_jobs);
    L.out_off = c.take<long long>((size_t)n_jobs);
    L.majorants = need_majorant ? c.take<float>((size_t)n_vols * (phys->n_e - 1)) : nullptr;
    L.rho_max = c.take<unsigned int>((size_t)n_vols * 256);
    L.present = c.take<unsigned int>((size_t)n_vols * 256);
    for (int s = 0; s < n_srcs; ++s) {
        const int npix = srcs[s].fu * srcs[s].fv;
        L.src[s].spec_k = guide_size(srcs[s].n_spec);
        L.src[s].flu_k = guide_size(npix);
        const size_t rows = (size_t)spec_rows(srcs[s]);
        L.src[s].spec_cdf = c.take<double>(rows * srcs[s].n_spec);
        L.src[s].spec_guide = c.take<uint32_t>(rows * L.src[s].spec_k);
        L.src[s].flu_cdf = c.take<double>((size_t)npix);
        L.src[s].flu_guide = c.take<uint32_t>(L.src[s].flu_k);
    }
    for (int v = 0; v < n_vols; ++v) L.cells[v] = c.take<CellRec>(cell_count(vols[v]));
    for (int v = 0; v < n_vols; ++v) {
        const gdrr_volume& V = vols[v];
        L.macro[v] = V.macro > 0 ? c.take<uint2>((size_t)cubes(V.nx, V.macro) * cubes(V.ny, V.macro) *
                                                 cubes(V.nz, V.macro))
                                 : nullptr;
    }
    L.tally = c.take<unsigned long long>(tally_elems);
    L.tally_elems = tally_elems;
    L.bytes = c.off + 256;
    return L;
}

size_t tally_elems_of(const gdrr_job* jobs, int n_jobs, const gdrr_source* srcs) {
    size_t e = 0;
    for (int k = 0; k < n_jobs; ++k) e += 4 * (size_t)jobs[k].geom.nu * jobs[k].geom.nv;
    (void)srcs;
    return e;
}

struct Batch {
    const gdrr_volume* vols;
    int n_vols;
    const gdrr_physics* phys;
    const gdrr_source* srcs;
    int n_srcs;
    const gdrr_job* jobs;
    int n_jobs;
    const float* majorants;     // caller's, or null
    uint64_t seed;
    uint32_t flags;
    const gdrr_tuning* tune;
    int mode;                   // kModeForward / kModeTrace / kModeBackward
    int only_volume;            // backward: jobs of this volume only (-1 = all)
    double* out;                // forward: caller tallies
    const double* adj;          // backward
    double* grad;               // backward
    int8_t* t_cls; int32_t* t_pixel; float* t_e; int32_t* t_steps; int32_t* t_nc; int32_t* t_nr;
    bool use_graph;
    bool tables_by_kernel = false;   // one job: its tables as kernel arguments, no host copy, no timing
};

// Host staging of the per-call tables.  It is pageable memory: a host-to-device
// hipMemcpyAsync from pageable memory returns only once the source has been
// copied out (into the runtime's own staging for the DMA), so the buffer can be
// refilled by the next call while the previous copy is still in flight.
thread_local std::vector<char> g_staging;

// Geometry part of a job record (Sec. 2.1), evaluated in double and stored as float.
DJob djob_of(const gdrr_job& J) {
    const gdrr_geometry& g = J.geom;
    const double phi = g.phi_rad, th = g.theta_rad;
    const double cq = std::cos(phi + th), sq = std::sin(phi + th);
    DJob d{};
    d.Sx = (float)(-g.sad_mm * std::cos(phi));
    d.Sy = (float)(-g.sad_mm * std::sin(phi));
    d.Sz = 0.0f;
    d.Px = (float)(g.aid_mm * cq);
    d.Py = (float)(g.aid_mm * sq);
    d.Pz = 0.0f;
    d.nx = (float)cq; d.ny = (float)sq; d.nz = 0.0f;
    d.ux = (float)(-sq); d.uy = (float)cq; d.uz = 0.0f;
    d.du = g.du_mm; d.dv = g.dv_mm;
    d.idu = (float)(1.0 / g.du_mm); d.idv = (float)(1.0 / g.dv_mm);
    d.nu = g.nu; d.nv = g.nv;
    d.src = J.source; d.vol = J.volume;
    d.job_id = J.job_id;
    return d;
}

int check_batch(const Batch& B) {
    if (B.n_vols < 1 || B.n_vols > GDRR_MAX_VOLUMES) return fail(GDRR_EINVAL, "n_vols must be in [1, 8]");
    if (B.n_srcs < 1 || B.n_srcs > GDRR_MAX_SOURCES) return fail(GDRR_EINVAL, "n_srcs must be in [1, 8]");
    if (B.n_jobs < 1 || B.n_jobs > (1 << 20)) return fail(GDRR_EINVAL, "n_jobs must be in [1, 2^20]");
    if (!B.vols || !B.srcs || !B.jobs) return fail(GDRR_EINVAL, "NULL array argument");
    int rc;
    if ((rc = check_physics(B.phys))) return rc;
    for (int v = 0; v < B.n_vols; ++v)
        if ((rc = check_volume(&B.vols[v]))) return rc;
    for (int s = 0; s < B.n_srcs; ++s)
        if ((rc = check_source(&B.srcs[s]))) return rc;
    for (int k = 0; k < B.n_jobs; ++k) {
        const gdrr_job& J = B.jobs[k];
        if (J.volume < 0 || J.volume >= B.n_vols) return fail(GDRR_EINVAL, "job volume index out of range");
        if (J.source < 0 || J.source >= B.n_srcs) return fail(GDRR_EINVAL, "job source index out of range");
        if (J.n_photons >= (1ull << 32) || (uint64_t)J.first_photon + J.n_photons >= (1ull << 32))
            return fail(GDRR_EINVAL, "a job's photon indices must stay below 2^32 (first_photon + n_photons)");
        if (J.tally_offset < 0) return fail(GDRR_EINVAL, "negative tally offset");
        if ((rc = check_geometry(&J.geom, &B.vols[J.volume], &B.srcs[J.source]))) return rc;
    }
    if (B.tune) {
        const gdrr_tuning& t = *B.tune;
        if (t.block && (t.block % 64 || t.block < 64 || t.block > 1024)) return fail(GDRR_EINVAL, "tune.block must be a multiple of 64 in [64, 1024]");
        if (t.chunk && (t.chunk % 64 || t.chunk < 64)) return fail(GDRR_EINVAL, "tune.chunk must be a positive multiple of 64");
        if (t.defer < 0 || t.defer > 64) return fail(GDRR_EINVAL, "tune.defer must be in [0, 64]");
        if (t.blocks_per_cu < 0 || t.blocks_per_cu > 64) return fail(GDRR_EINVAL, "tune.blocks_per_cu must be in [0, 64]");
        if (t.coll_defer < 0 || t.coll_defer > 64) return fail(GDRR_EINVAL, "tune.coll_defer must be in [0, 64]");
    }
    return GDRR_OK;
}

// local: 0 single majorants, 1 local majorants with records in global memory, 2 with records in LDS,
// 3 every traced volume with local majorants and records in LDS, interpolated density
template <int MODE>
const void* mc_func(int local) {
    if constexpr (MODE == kModeBackward)
        return local == 3 ? reinterpret_cast<const void*>(&mc_adjoint_kernel<3>)
             : local == 2 ? reinterpret_cast<const void*>(&mc_adjoint_kernel<2>)
             : local == 1 ? reinterpret_cast<const void*>(&mc_adjoint_kernel<1>)
                          : reinterpret_cast<const void*>(&mc_adjoint_kernel<0>);
    else
        return local == 3 ? reinterpret_cast<const void*>(&mc_kernel<MODE, 3>)
             : local == 2 ? reinterpret_cast<const void*>(&mc_kernel<MODE, 2>)
             : local == 1 ? reinterpret_cast<const void*>(&mc_kernel<MODE, 1>)
                          : reinterpret_cast<const void*>(&mc_kernel<MODE, 0>);
}

const void* mc_func_for(int mode, int local) {
    return mode == kModeForward ? mc_func<kModeForward>(local)
         : mode == kModeTrace ? mc_func<kModeTrace>(local) : mc_func<kModeBackward>(local);
}

// Does some job of the launch trace photons in volume v?
bool batch_uses(const Batch& B, int v) {
    for (int k = 0; k < B.n_jobs; ++k)
        if (B.jobs[k].volume == v && B.jobs[k].n_photons > 0 && (B.only_volume < 0 || v == B.only_volume))
            return true;
    return false;
}

int run_batch(const Batch& B, void* ws, size_t ws_bytes, hipStream_t st) {
    int rc = check_batch(B);
    if (rc) return rc;
    const gdrr_physics* phys = B.phys;
    const bool need_maj = B.majorants == nullptr;
    const Layout L0 = carve(nullptr, B.vols, phys, B.srcs, B.n_srcs, B.n_jobs, B.n_vols,
                            tally_elems_of(B.jobs, B.n_jobs, B.srcs), need_maj);
    if (!ws || ws_bytes < L0.bytes)
        return fail(GDRR_EINVAL, "workspace too small: need " + std::to_string(L0.bytes) + " bytes");
    DevInfo dev;
    if ((rc = device_info(dev))) return rc;
    char* wsa = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    const Layout L = carve(wsa, B.vols, phys, B.srcs, B.n_srcs, B.n_jobs, B.n_vols, L0.tally_elems, need_maj);
    const bool interp = (B.flags & GDRR_INTERP_DENSITY) != 0;

    // ---- host tables: jobs, chunk prefix, output offsets ----
    gdrr_tuning tune{};
    if (B.tune) tune = *B.tune;
    unsigned long long total_photons = 0;
    for (int k = 0; k < B.n_jobs; ++k)
        if (B.only_volume < 0 || B.jobs[k].volume == B.only_volume) total_photons += B.jobs[k].n_photons;
    bool local = false;
    for (int v = 0; v < B.n_vols; ++v) local |= B.vols[v].macro > 0;
    const int block = tune.block ? tune.block : 256;
    // the single-majorant tables are staged only if some traced volume tracks with them
    bool any_single = false;
    for (int v = 0; v < B.n_vols; ++v) any_single |= batch_uses(B, v) && B.vols[v].macro <= 0;
    const int n_maj = any_single ? B.n_vols : 0;
    // local majorants go to LDS (after the tables) while the records of all volumes that the
    // launch traces fit in kMacroLdsMax (one word per cube in the all-local instantiation)
    int macro_lds[GDRR_MAX_VOLUMES];
    int macro_lds_n = 0;
    for (int v = 0; v < GDRR_MAX_VOLUMES; ++v) macro_lds[v] = -1;
    // the all-local instantiation counts a flight's crossings in 9 bits per axis
    bool small_grids = true;
    for (int v = 0; v < B.n_vols; ++v)
        if (B.vols[v].macro > 0 && batch_uses(B, v))
            small_grids &= cubes(B.vols[v].nx, B.vols[v].macro) <= 512 && cubes(B.vols[v].ny, B.vols[v].macro) <= 512 &&
                           cubes(B.vols[v].nz, B.vols[v].macro) <= 512;
    const bool all_local = local && !any_single && interp && small_grids;
    const size_t rec_bytes = lds_record_bytes(all_local ? 3 : 2);
    if (local) {
        size_t n = 0;
        for (int v = 0; v < B.n_vols; ++v)
            if (B.vols[v].macro > 0 && batch_uses(B, v))
                n += (size_t)cubes(B.vols[v].nx, B.vols[v].macro) * cubes(B.vols[v].ny, B.vols[v].macro) *
                     cubes(B.vols[v].nz, B.vols[v].macro);
        if (n * rec_bytes <= kMacroLdsMax)
            for (int v = 0; v < B.n_vols; ++v)
                if (B.vols[v].macro > 0 && batch_uses(B, v)) {
                    macro_lds[v] = macro_lds_n;
                    macro_lds_n += cubes(B.vols[v].nx, B.vols[v].macro) * cubes(B.vols[v].ny, B.vols[v].macro) *
                                   cubes(B.vols[v].nz, B.vols[v].macro);
                }
    }
    const int local_kind = !local ? 0 : (macro_lds_n > 0 ? (all_local ? 3 : 2) : 1);
    // Rows for the material sets of cubes (all-local launches, at most 8 materials): as many
    // as keep the workgroups per compute unit that the launch has without them (or the tuned
    // count), as the runtime's occupancy calculation has it.
    const int n_mat = phys->n_mat;
    const auto lds_for = [&](int rows) {
        return draw_slots_offset_bytes(table_floats2(rows, phys->n_e, n_maj) * 8 +
                                       (size_t)macro_lds_n * lds_record_bytes(local_kind)) +
               (size_t)block * 16;
    };
    const void* mfunc = mc_func_for(B.mode, local_kind);
    // (the LDS of a workgroup is allocated in granules of kLdsGranule bytes, which the
    // runtime's occupancy calculation does not round to: the query gets the rounded size)
    const auto per_cu_with = [&](size_t bytes, int& nb) -> int {
        nb = 0;
        const size_t held = (bytes + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
        GDRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mfunc, block, held));
        return GDRR_OK;
    };
    int mask_rows = 0;
    if (local_kind == 3 && n_mat <= 8 && lds_for(n_mat) <= dev.lds_max) {
        int target = tune.blocks_per_cu;
        if (!target && (rc = per_cu_with(lds_for(n_mat), target))) return rc;
        const int sets = std::min((1 << n_mat) - 1 - n_mat, (int)kNoRow - n_mat);   // sets of two or more
        for (int r = sets; r > 0; --r) {                       // the most rows that keep the target
            if (lds_for(n_mat + r) > dev.lds_max) continue;
            int nb = 0;
            if ((rc = per_cu_with(lds_for(n_mat + r), nb))) return rc;
            if (nb >= target) {
                mask_rows = r;
                break;
            }
        }
    }
    const size_t lds = lds_for(n_mat + mask_rows);
    if (lds > dev.lds_max) return fail(GDRR_ENOTSUP, "tables exceed the LDS of a workgroup");
    int per_cu = tune.blocks_per_cu;
    if (!per_cu) {
        int nb = 0;
        if ((rc = per_cu_with(lds, nb))) return rc;
        per_cu = std::max(nb, 1);
    }
    const unsigned grid = (unsigned)(dev.cus * per_cu);
    const unsigned long long waves = (unsigned long long)grid * (block / 64);
    int chunk = tune.chunk;
    if (!chunk) {
        unsigned long long c = total_photons / (waves * 8ull);
        c = std::max<unsigned long long>(64, std::min<unsigned long long>(4096, c));
        chunk = (int)(c / 64 * 64);
    }
    const int defer = tune.defer ? tune.defer : 32;
    const int cdefer = tune.coll_defer ? tune.coll_defer : defer;

    const size_t n_jobs = (size_t)B.n_jobs;
    const size_t job_bytes = sizeof(unsigned long long) * (n_jobs + 1);
    std::vector<unsigned long long> prefix(n_jobs + 1);
    std::vector<DJob> dj(n_jobs);
    std::vector<long long> out_off(n_jobs);
    unsigned long long chunks = 0;
    size_t toff = 0;
    for (size_t k = 0; k < n_jobs; ++k) {
        const gdrr_job& J = B.jobs[k];
        const gdrr_geometry& g = J.geom;
        DJob d = djob_of(J);
        const bool run = B.only_volume < 0 || J.volume == B.only_volume;
        const unsigned long long n = run ? J.n_photons : 0ull;
        d.n_lo = (uint32_t)J.n_photons;
        d.n_hi = (uint32_t)(J.n_photons >> 32);
        d.first = J.first_photon;
        d.index = (uint32_t)k;
        d.tally_off = (long long)toff;
        d.adj_off = (long long)(2 * (size_t)g.nu * g.nv * k);
        toff += 4 * (size_t)g.nu * g.nv;
        dj[k] = d;
        out_off[k] = J.tally_offset;
        prefix[k] = chunks;
        chunks += (n + (unsigned long long)chunk - 1) / (unsigned long long)chunk;
    }
    prefix[n_jobs] = chunks;

    // The volume order of the dispenser: jobs are taken in array order; a
    // wavefront drains before it changes phantom, so callers group jobs by volume.
    std::vector<Launch> ls;
    if (B.tables_by_kernel) {
        if (n_jobs != 1) return fail(GDRR_EINVAL, "internal: kernel-written tables need one job");
        JobTableParams jt{L.chunk_prefix, L.jobs, L.out_off, prefix[0], prefix[1], out_off[0], dj[0]};
        ls.push_back(make_launch((const void*)&job_table_kernel, dim3(1), dim3(64), 0, jt));
    } else {
        g_staging.resize(job_bytes + sizeof(DJob) * n_jobs + sizeof(long long) * n_jobs + 1024);
        char* hs = g_staging.data();
        std::memcpy(hs, prefix.data(), job_bytes);
        GDRR_HIP(hipMemcpyAsync(L.chunk_prefix, hs, job_bytes, hipMemcpyHostToDevice, st));
        std::memcpy(hs + job_bytes, dj.data(), sizeof(DJob) * n_jobs);
        GDRR_HIP(hipMemcpyAsync(L.jobs, hs + job_bytes, sizeof(DJob) * n_jobs, hipMemcpyHostToDevice, st));
        std::memcpy(hs + job_bytes + sizeof(DJob) * n_jobs, out_off.data(), sizeof(long long) * n_jobs);
        GDRR_HIP(hipMemcpyAsync(L.out_off, hs + job_bytes + sizeof(DJob) * n_jobs, sizeof(long long) * n_jobs,
                                hipMemcpyHostToDevice, st));
    }

    unsigned int* status = (unsigned int*)(L.counter + 1);    // input-error bits of this call
    const bool resume = B.mode == kModeForward && (B.flags & GDRR_RESUME);
    // ---- clear counters, tallies (unless resuming), the gradient and the majorant scratch ----
    {
        FillParams f{L.counter, 8};
        ls.push_back(make_launch((const void*)&fill_zero_kernel, dim3(1), dim3(256), 0, f));
        FillParams t{L.tally, (long long)L.tally_elems};
        if (!resume)
            ls.push_back(make_launch((const void*)&fill_zero_kernel, dim3(std::max<unsigned>(1, std::min<size_t>(4096, (L.tally_elems + 255) / 256))), dim3(256), 0, t));
        if (B.mode == kModeBackward && !(B.flags & GDRR_ACCUMULATE)) {
            const gdrr_volume& V = B.vols[B.only_volume];
            GradClearParams g{B.grad, (long long)V.nx * V.ny * V.nz};
            ls.push_back(make_launch((const void*)&grad_zero_kernel, dim3(1024), dim3(256), 0, g));
        }
        FillParams r{(unsigned long long*)L.rho_max, (long long)B.n_vols * 128};   // 256 u32 per volume
        ls.push_back(make_launch((const void*)&fill_zero_kernel, dim3(4), dim3(256), 0, r));
        FillParams p{(unsigned long long*)L.present, (long long)B.n_vols * 128};
        ls.push_back(make_launch((const void*)&fill_zero_kernel, dim3(4), dim3(256), 0, p));
    }
    // ---- majorants ----
    const float* maj = B.majorants;
    if (need_maj) {
        for (int v = 0; v < B.n_vols; ++v) {
            const gdrr_volume& V = B.vols[v];
            MajParams m{V.density, V.material, V.nx, V.ny, V.nz, interp ? 1 : 0, phys->n_mat, L.rho_max + 256 * v,
                        L.present + 256 * v, status};
            const long long nvox = (long long)V.nx * V.ny * V.nz;
            const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>(dev.cus * 8, (nvox + 255) / 256));
            ls.push_back(make_launch((const void*)&rho_max_kernel, dim3(g), dim3(256), 0, m));
            MajFinParams fp{L.rho_max + 256 * v, L.present + 256 * v, phys->mu_mass, phys->n_mat, phys->n_e,
                            1.0 + (double)(1.0f / 1048576.0f), L.majorants + (size_t)v * (phys->n_e - 1),
                            status};
            ls.push_back(make_launch((const void*)&majorant_kernel, dim3((phys->n_e + 254) / 256), dim3(256), 0, fp));
        }
        maj = L.majorants;
    }
    // ---- cell records of every volume that has photons ----
    for (int v = 0; v < B.n_vols; ++v) {
        if (!batch_uses(B, v)) continue;
        const gdrr_volume& V = B.vols[v];
        CellParams cp{V.density, V.material, V.nx, V.ny, V.nz, phys->n_mat, L.cells[v], status};
        const size_t nc = cell_count(V);
        ls.push_back(make_launch((const void*)&cells_kernel,
                                 dim3((unsigned)std::max<size_t>(1, std::min<size_t>((size_t)dev.cus * 16, (nc + 255) / 256))),
                                 dim3(256), 0, cp));
        if (L.macro[v]) {
            MacroParams mp{V.density, V.material, V.nx, V.ny, V.nz, V.macro, cubes(V.nx, V.macro),
                           cubes(V.ny, V.macro), cubes(V.nz, V.macro), phys->n_mat,
                           1.0 + (double)V.macro_margin, V.macro_rho_min, L.macro[v]};
            const size_t nm = (size_t)mp.mnx * mp.mny * mp.mnz;
            // one workgroup of 256 per cube
            ls.push_back(make_launch((const void*)&macro_kernel,
                                     dim3((unsigned)std::max<size_t>(1, std::min<size_t>((size_t)dev.cus * 16, nm))),
                                     dim3(256), 0, mp));
        }
    }
    // ---- sources: CDFs and guide tables ----
    for (int s = 0; s < B.n_srcs; ++s) {
        const gdrr_source& S = B.srcs[s];
        const SrcArea& A = L.src[s];
        const int rows = spec_rows(S);
        SrcPrepParams sp{S.spec_prob, S.n_spec, rows, A.spec_cdf, A.spec_guide, (int)A.spec_k, status};
        ls.push_back(make_launch((const void*)&cdf_kernel, dim3(rows), dim3(1024), 0, sp));
        const unsigned gk = (unsigned)std::min<size_t>((size_t)dev.cus * 8, ((size_t)rows * A.spec_k + 255) / 256);
        ls.push_back(make_launch((const void*)&guide_kernel, dim3(gk), dim3(256), 0, sp));
        SrcPrepParams fp{S.fluence, S.fu * S.fv, 1, A.flu_cdf, A.flu_guide, (int)A.flu_k, status};
        ls.push_back(make_launch((const void*)&cdf_kernel, dim3(1), dim3(1024), 0, fp));
        ls.push_back(make_launch((const void*)&guide_kernel, dim3((A.flu_k + 255) / 256), dim3(256), 0, fp));
    }
    // ---- the persistent transport kernel ----
    KParams kp{};
    for (int v = 0; v < B.n_vols; ++v) {
        const gdrr_volume& V = B.vols[v];
        DVolume& d = kp.vol[v];
        d.density = V.density;
        d.material = V.material;
        d.cells = L.cells[v];
        d.cx = V.nx + 1;
        d.cxy = (V.nx + 1) * (V.ny + 1);
        d.nx = V.nx; d.ny = V.ny; d.nz = V.nz; d.nxy = V.nx * V.ny;
        d.lox = (float)(-0.5 * V.nx * V.dx_mm); d.hix = -d.lox;
        d.loy = (float)(-0.5 * V.ny * V.dy_mm); d.hiy = -d.loy;
        d.loz = (float)(-0.5 * V.nz * V.dz_mm); d.hiz = -d.loz;
        d.idx = (float)(1.0 / V.dx_mm); d.idy = (float)(1.0 / V.dy_mm); d.idz = (float)(1.0 / V.dz_mm);
        d.lds_majorant = n_maj ? v * (phys->n_e - 1) : -1;
        d.macro = L.macro[v];
        if (V.macro > 0) {
            d.mnx = cubes(V.nx, V.macro); d.mny = cubes(V.ny, V.macro); d.mnz = cubes(V.nz, V.macro);
            d.mcube = V.macro;
            d.mex = (float)((double)V.macro * V.dx_mm);
            d.mey = (float)((double)V.macro * V.dy_mm);
            d.mez = (float)((double)V.macro * V.dz_mm);
            d.imx = (float)(1.0 / ((double)V.macro * V.dx_mm));
            d.imy = (float)(1.0 / ((double)V.macro * V.dy_mm));
            d.imz = (float)(1.0 / ((double)V.macro * V.dz_mm));
        }
    }
    for (int s = 0; s < B.n_srcs; ++s) {
        DSource& d = kp.src[s];
        d.spec_e = B.srcs[s].spec_e_kev;
        d.spec_cdf = L.src[s].spec_cdf;
        d.spec_guide = L.src[s].spec_guide;
        d.flu_cdf = L.src[s].flu_cdf;
        d.flu_guide = L.src[s].flu_guide;
        d.n_spec = B.srcs[s].n_spec;
        d.spec_rows = spec_rows(B.srcs[s]);
        d.spec_k = (int)L.src[s].spec_k;
        d.npix = B.srcs[s].fu * B.srcs[s].fv;
        d.flu_k = (int)L.src[s].flu_k;
    }
    kp.jobs = L.jobs;
    kp.chunk_prefix = L.chunk_prefix;
    kp.counter = L.counter;
    kp.tally = L.tally;
    kp.mu_mass = phys->mu_mass;
    kp.response = phys->response;
    kp.majorants = maj;
    kp.total_chunks = chunks;
    kp.n_jobs = B.n_jobs;
    kp.n_vols = B.n_vols;
    kp.n_maj = n_maj;
    kp.n_mat = phys->n_mat;
    kp.tot_rows = phys->n_mat + mask_rows;
    kp.mask_rows = mask_rows;
    kp.n_e = phys->n_e;
    kp.e0 = phys->e0_kev;
    kp.inv_de = (float)(1.0 / phys->de_kev);
    kp.e_max = (float)(phys->e0_kev + (double)phys->de_kev * (phys->n_e - 1));
    kp.e_cut = phys->e_cut_kev;
    kp.x0 = phys->rayleigh_x0_invA;
    kp.k0 = (uint32_t)B.seed;
    kp.k1 = (uint32_t)(B.seed >> 32);
    kp.flags = B.flags;
    kp.chunk = chunk;
    kp.defer = defer;
    kp.cdefer = cdefer;
    kp.t_cls = B.t_cls; kp.t_pixel = B.t_pixel; kp.t_e = B.t_e;
    kp.t_steps = B.t_steps; kp.t_nc = B.t_nc; kp.t_nr = B.t_nr;
    kp.adj = B.adj;
    kp.grad = B.grad;
    for (int v = 0; v < kMaxVol; ++v) kp.macro_lds[v] = v < GDRR_MAX_VOLUMES ? macro_lds[v] : -1;
    kp.macro_lds_n = macro_lds_n;
    const void* mf = mc_func_for(B.mode, local_kind);
    int timed = -1;
    if (chunks > 0) {
        timed = (int)ls.size();
        ls.push_back(make_launch(mf, dim3(grid), dim3(block), lds, kp));
    }
    // ---- finalize ----
    if (B.mode == kModeForward) {
        int maxpix = 1;
        for (int k = 0; k < B.n_jobs; ++k) maxpix = std::max(maxpix, B.jobs[k].geom.nu * B.jobs[k].geom.nv);
        FinParams fp{L.jobs, B.n_jobs, L.tally, B.out, L.out_off, B.flags & (GDRR_TALLY_SUMSQ | GDRR_ACCUMULATE | GDRR_RESUME)};
        ls.push_back(make_launch((const void*)&finalize_kernel,
                                 dim3((unsigned)std::min(1024, (4 * maxpix + 255) / 256), (unsigned)B.n_jobs), dim3(256), 0, fp));
    }
    TimeEvents* ev = nullptr;
    if (!B.tables_by_kernel) {
        std::lock_guard<std::mutex> lk(g_time_mu);
        if (g_timing && timed >= 0 && (rc = timing_events(&ev))) return rc;
    }
    if (!ev) timed = -1;
    return B.use_graph ? run_graph(ls, st, timed, ev) : run_direct(ls, st, timed, ev);
}

size_t batch_bytes(const gdrr_volume* vols, int n_vols, const gdrr_physics* phys, const gdrr_source* srcs,
                   int n_srcs, const gdrr_job* jobs, int n_jobs, bool need_maj) {
    if (!vols || !phys || !srcs || !jobs || n_srcs < 1 || n_srcs > GDRR_MAX_SOURCES || n_jobs < 1 || n_vols < 1 ||
        n_vols > GDRR_MAX_VOLUMES)
        return 0;
    for (int v = 0; v < n_vols; ++v)
        if (vols[v].nx < 1 || vols[v].ny < 1 || vols[v].nz < 1) return 0;
    for (int s = 0; s < n_srcs; ++s)
        if (srcs[s].n_spec < 1 || spec_rows(srcs[s]) < 0) return 0;
    return carve(nullptr, vols, phys, srcs, n_srcs, n_jobs, n_vols, tally_elems_of(jobs, n_jobs, srcs), need_maj).bytes +
           256;
}

// --------------------------------------------------------------------------
// Ray-tracing primary (Eq. 1): workspace layout and launch.
// --------------------------------------------------------------------------
struct RtLayout {
    unsigned long long* head;            // [8] status block (word 1: input-error bits)
    DJob* jobs;                          // [n_jobs]
    int* unit_job;                       // [max units]
    unsigned int* unit_first;
    unsigned int* unit_pref;
    long long* out_off;                  // [n_jobs]
    float* coef[GDRR_MAX_SOURCES];       // [rows][n_spec]
    float* tab[GDRR_MAX_SOURCES];        // [n_spec][n_mat]
    double* inv_wsum[GDRR_MAX_SOURCES];  // [1]
    CellRec* cells[GDRR_MAX_VOLUMES];    // volumes that some job uses
    size_t bytes;
};

bool volume_used(const gdrr_job* jobs, int n_jobs, int v) {
    for (int k = 0; k < n_jobs; ++k)
        if (jobs[k].volume == v) return true;
    return false;
}


unsigned long long rt_tiles(const gdrr_geometry& g) {
    return (unsigned long long)((g.nu + 15) / 16) * (unsigned long long)((g.nv + 15) / 16);
}

// Work units: pieces of one tile row of one job, `run` tiles long (whole
// rows once there are enough of them to fill every XCD several times).
unsigned long long rt_run_length(const gdrr_job* jobs, int n_jobs) {
    unsigned long long total = 0, widest = 1;
    for (int k = 0; k < n_jobs; ++k) {
        total += rt_tiles(jobs[k].geom);
        widest = std::max(widest, (unsigned long long)((jobs[k].geom.nu + 15) / 16));
    }
    return std::min(widest, std::max<unsigned long long>(4, total / (8ull * kXcds)));
}

unsigned long long rt_row_units(const gdrr_geometry& g, unsigned long long run) {
    return (unsigned long long)((g.nv + 15) / 16) * (((unsigned long long)((g.nu + 15) / 16) + run - 1) / run);
}

size_t rt_max_units(const gdrr_job* jobs, int n_jobs) {
    const unsigned long long run = rt_run_length(jobs, n_jobs);
    size_t u = 0;
    for (int k = 0; k < n_jobs; ++k) u += (size_t)rt_row_units(jobs[k].geom, run);
    return u;
}

RtLayout rt_carve(void* ws, const gdrr_volume* vols, int n_vols, const gdrr_physics* phys, const gdrr_source* srcs,
                  int n_srcs, const gdrr_job* jobs, int n_jobs) {
    Carver c(ws);
    RtLayout L{};
    L.head = c.take<unsigned long long>(8);
    L.jobs = c.take<DJob>((size_t)n_jobs);
    const size_t units = rt_max_units(jobs, n_jobs);
    L.unit_job = c.take<int>(units);
    L.unit_first = c.take<unsigned int>(units);
    L.unit_pref = c.take<unsigned int>(units);
    L.out_off = c.take<long long>((size_t)n_jobs);
    for (int s = 0; s < n_srcs; ++s) {
        L.coef[s] = c.take<float>((size_t)spec_rows(srcs[s]) * srcs[s].n_spec);
        L.tab[s] = c.take<float>((size_t)srcs[s].n_spec * phys->n_mat);
        L.inv_wsum[s] = c.take<double>(1);
    }
    for (int v = 0; v < n_vols; ++v)
        L.cells[v] = volume_used(jobs, n_jobs, v) ? c.take<CellRec>(cell_count(vols[v])) : nullptr;
    L.bytes = c.off + 256;
    return L;
}

constexpr unsigned kRtMaxTiles = (1u << 24) - 1024u;    // grid * block stays below 2^32 work-items

int check_rt(const gdrr_volume* vols, int n_vols, const gdrr_physics* phys, const gdrr_source* srcs, int n_srcs,
             const gdrr_job* jobs, int n_jobs, uint32_t flags) {
    if (n_vols < 1 || n_vols > GDRR_MAX_VOLUMES) return fail(GDRR_EINVAL, "n_vols must be in [1, 8]");
    if (n_srcs < 1 || n_srcs > GDRR_MAX_SOURCES) return fail(GDRR_EINVAL, "n_srcs must be in [1, 8]");
    if (n_jobs < 1 || n_jobs > (1 << 20)) return fail(GDRR_EINVAL, "n_jobs must be in [1, 2^20]");
    if (!vols || !srcs || !jobs) return fail(GDRR_EINVAL, "NULL array argument");
    if (flags & ~(GDRR_INTERP_DENSITY | GDRR_ACCUMULATE))
        return fail(GDRR_EINVAL, "gdrr_primary takes only GDRR_INTERP_DENSITY and GDRR_ACCUMULATE");
    int rc;
    if ((rc = check_physics(phys))) return rc;
    for (int v = 0; v < n_vols; ++v)
        if ((rc = check_volume(&vols[v]))) return rc;
    for (int s = 0; s < n_srcs; ++s)
        if ((rc = check_source(&srcs[s]))) return rc;
    for (int k = 0; k < n_jobs; ++k) {
        const gdrr_job& J = jobs[k];
        if (J.volume < 0 || J.volume >= n_vols) return fail(GDRR_EINVAL, "job volume index out of range");
        if (J.source < 0 || J.source >= n_srcs) return fail(GDRR_EINVAL, "job source index out of range");
        if (J.tally_offset < 0) return fail(GDRR_EINVAL, "negative output offset");
        if ((rc = check_geometry(&J.geom, &vols[J.volume], &srcs[J.source]))) return rc;
    }
    return GDRR_OK;
}

int run_primary(const gdrr_volume* vols, int n_vols, const gdrr_physics* phys, const gdrr_source* srcs, int n_srcs,
                const gdrr_job* jobs, int n_jobs, float step_mm, uint32_t flags, double* out, void* ws,
                size_t ws_bytes, hipStream_t st) {
    int rc = check_rt(vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs, flags);
    if (rc) return rc;
    if (!out) return fail(GDRR_EINVAL, "out is NULL");
    if (!std::isfinite(step_mm)) return fail(GDRR_EINVAL, "step_mm must be finite");
    const RtLayout L0 = rt_carve(nullptr, vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs);
    if (!ws || ws_bytes < L0.bytes)
        return fail(GDRR_EINVAL, "workspace too small: need " + std::to_string(L0.bytes) + " bytes");
    RtParams rp{};
    for (int v = 0; v < n_vols; ++v) {
        const gdrr_volume& V = vols[v];
        const double edge = std::min(V.dx_mm, std::min(V.dy_mm, V.dz_mm));
        const double dl = step_mm > 0.0f ? (double)step_mm : 0.5 * edge;
        const double diag = std::sqrt((double)V.nx * V.dx_mm * V.nx * V.dx_mm + (double)V.ny * V.dy_mm * V.ny * V.dy_mm +
                                      (double)V.nz * V.dz_mm * V.nz * V.dz_mm);
        if (volume_used(jobs, n_jobs, v) && diag / dl > (double)(1 << 20))
            return fail(GDRR_EINVAL, "step_mm too small: more than 2^20 intervals across a phantom");
        rp.dl[v] = (float)dl;
    }
    const size_t lds = (size_t)phys->n_mat * kRtBlock * sizeof(float);
    DevInfo dev;
    if ((rc = device_info(dev))) return rc;
    if (lds > dev.lds_max) return fail(GDRR_ENOTSUP, "per-material accumulators exceed the LDS of a workgroup");
    char* wsa = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    const RtLayout L = rt_carve(wsa, vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs);
    const bool interp = (flags & GDRR_INTERP_DENSITY) != 0;

    const size_t nj = (size_t)n_jobs;
    std::vector<DJob> dj(nj);
    std::vector<long long> off(nj);
    unsigned long long tiles = 0;
    for (size_t k = 0; k < nj; ++k) {
        dj[k] = djob_of(jobs[k]);
        dj[k].index = (uint32_t)k;
        off[k] = jobs[k].tally_offset;
        tiles += rt_tiles(jobs[k].geom);
        if (tiles > kRtMaxTiles) return fail(GDRR_EINVAL, "too many pixels in one call (2^32 lanes)");
    }
    // Units in row-band order: for each phantom, tile row by tile row, that
    // row of every job on the phantom, dealt to the XCDs in turn.  All XCDs
    // then work through the same band of detector rows -- the same slab of
    // the phantom -- across all its projections at once, so the slab is read
    // from HBM about once and served from the last-level cache after that.
    const unsigned long long run = rt_run_length(jobs, n_jobs);
    std::vector<int> u_job[kXcds];
    std::vector<unsigned int> u_first[kXcds];
    std::vector<std::vector<int>> band[GDRR_MAX_VOLUMES];    // [volume][tile row] -> jobs in order
    for (size_t k = 0; k < nj; ++k) {
        std::vector<std::vector<int>>& b = band[jobs[k].volume];
        const size_t rows = (size_t)((jobs[k].geom.nv + 15) / 16);
        if (b.size() < rows) b.resize(rows);
        for (size_t r = 0; r < rows; ++r) b[r].push_back((int)k);
    }
    int deal = 0;
    for (int v = 0; v < n_vols; ++v)
        for (size_t r = 0; r < band[v].size(); ++r)
            for (const int k : band[v][r]) {
                const unsigned long long tu = (unsigned long long)((jobs[k].geom.nu + 15) / 16);
                for (unsigned long long c = 0; c < tu; c += run) {
                    u_job[deal].push_back(k);
                    u_first[deal].push_back((unsigned int)(r * tu + c));
                    deal = (deal + 1) % kXcds;
                }
            }
    std::vector<int> ujob;
    std::vector<unsigned int> ufirst, upref;
    unsigned int most = 0;
    for (int x = 0; x < kXcds; ++x) {
        rp.xcd_start[x] = (unsigned int)ujob.size();
        unsigned int acc = 0;
        for (size_t i = 0; i < u_job[x].size(); ++i) {
            const int k = u_job[x][i];
            ujob.push_back(k);
            ufirst.push_back(u_first[x][i]);
            upref.push_back(acc);
            const unsigned long long tu = (unsigned long long)((jobs[k].geom.nu + 15) / 16);
            acc += (unsigned int)std::min<unsigned long long>(run, tu - u_first[x][i] % tu);
        }
        rp.xcd_tiles[x] = acc;
        most = std::max(most, acc);
    }
    rp.xcd_start[kXcds] = (unsigned int)ujob.size();
    const size_t nu_ = ujob.size();
    const size_t b_jobs = sizeof(DJob) * nj, b_u = sizeof(unsigned int) * nu_, b_off = sizeof(long long) * nj;
    g_staging.resize(b_jobs + 3 * b_u + b_off);
    char* hs = g_staging.data();
    std::memcpy(hs, dj.data(), b_jobs);
    std::memcpy(hs + b_jobs, ujob.data(), b_u);
    std::memcpy(hs + b_jobs + b_u, ufirst.data(), b_u);
    std::memcpy(hs + b_jobs + 2 * b_u, upref.data(), b_u);
    std::memcpy(hs + b_jobs + 3 * b_u, off.data(), b_off);
    GDRR_HIP(hipMemcpyAsync(L.jobs, hs, b_jobs, hipMemcpyHostToDevice, st));
    GDRR_HIP(hipMemcpyAsync(L.unit_job, hs + b_jobs, b_u, hipMemcpyHostToDevice, st));
    GDRR_HIP(hipMemcpyAsync(L.unit_first, hs + b_jobs + b_u, b_u, hipMemcpyHostToDevice, st));
    GDRR_HIP(hipMemcpyAsync(L.unit_pref, hs + b_jobs + 2 * b_u, b_u, hipMemcpyHostToDevice, st));
    GDRR_HIP(hipMemcpyAsync(L.out_off, hs + b_jobs + 3 * b_u, b_off, hipMemcpyHostToDevice, st));

    std::vector<Launch> ls;
    unsigned int* status = (unsigned int*)(L.head + 1);
    {
        FillParams f{L.head, 8};
        ls.push_back(make_launch((const void*)&fill_zero_kernel, dim3(1), dim3(256), 0, f));
    }
    for (int v = 0; v < n_vols; ++v) {
        const gdrr_volume& V = vols[v];
        DVolume& d = rp.vol[v];
        d.density = V.density;
        d.material = V.material;
        d.cells = interp ? L.cells[v] : nullptr;
        d.cx = V.nx + 1;
        d.cxy = (V.nx + 1) * (V.ny + 1);
        d.nx = V.nx; d.ny = V.ny; d.nz = V.nz; d.nxy = V.nx * V.ny;
        d.lox = (float)(-0.5 * V.nx * V.dx_mm); d.hix = -d.lox;
        d.loy = (float)(-0.5 * V.ny * V.dy_mm); d.hiy = -d.loy;
        d.loz = (float)(-0.5 * V.nz * V.dz_mm); d.hiz = -d.loz;
        d.idx = (float)(1.0 / V.dx_mm); d.idy = (float)(1.0 / V.dy_mm); d.idz = (float)(1.0 / V.dz_mm);
        if (interp && L.cells[v]) {
            CellParams cp{V.density, V.material, V.nx, V.ny, V.nz, phys->n_mat, L.cells[v], status};
            const size_t nc = cell_count(V);
            ls.push_back(make_launch((const void*)&cells_kernel,
                                     dim3((unsigned)std::max<size_t>(1, std::min<size_t>((size_t)dev.cus * 16, (nc + 255) / 256))),
                                     dim3(256), 0, cp));
        } else if (volume_used(jobs, n_jobs, v)) {
            const long long nv = (long long)V.nx * V.ny * V.nz;
            VolCheckParams vc{V.density, V.material, nv, phys->n_mat, status};
            ls.push_back(make_launch((const void*)&volume_check_kernel,
                                     dim3((unsigned)std::max<long long>(1, std::min<long long>((long long)dev.cus * 8, (nv + 255) / 256))),
                                     dim3(256), 0, vc));
        }
    }
    for (int s = 0; s < n_srcs; ++s) {
        const gdrr_source& S = srcs[s];
        RtPrepParams pp{S.spec_e_kev, S.spec_prob, S.fluence, S.n_spec, S.fu * S.fv, phys->mu_mass, phys->response,
                        phys->n_mat, phys->n_e, (double)phys->e0_kev, (double)phys->de_kev, L.coef[s], L.tab[s],
                        L.inv_wsum[s], status};
        ls.push_back(make_launch((const void*)&raytrace_prep_kernel, dim3(spec_rows(S)), dim3(256), 0, pp));
        rp.src[s] = RtSource{S.fluence, L.coef[s], L.tab[s], L.inv_wsum[s], S.n_spec, spec_rows(S)};
    }
    rp.jobs = L.jobs;
    rp.unit_job = L.unit_job;
    rp.unit_first = L.unit_first;
    rp.unit_pref = L.unit_pref;
    rp.out_off = L.out_off;
    rp.out = out;
    rp.n_mat = phys->n_mat;
    rp.interp = interp ? 1 : 0;
    rp.accumulate = (flags & GDRR_ACCUMULATE) ? 1 : 0;
    const unsigned long long grid = (unsigned long long)kXcds * most;
    if (grid * kRtBlock >= (1ull << 32)) return fail(GDRR_EINVAL, "too many pixels in one call (2^32 lanes)");
    const int timed = (int)ls.size();
    ls.push_back(make_launch((const void*)&raytrace_kernel, dim3((unsigned)grid), dim3(kRtBlock), lds, rp));
    TimeEvents* ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_time_mu);
        if (g_timing && (rc = timing_events(&ev))) return rc;
    }
    return run_direct(ls, st, ev ? timed : -1, ev);
}

// --------------------------------------------------------------------------
// Denoising (Eq. 5) and noise assembly (Sec. 2.6).
// --------------------------------------------------------------------------
bool ranges_overlap(const void* a, size_t a_bytes, const void* b, size_t b_bytes) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + b_bytes && b0 < a0 + a_bytes;
}

size_t dn_buffer_bytes(int n_img, int nv, int nu) {
    return ((size_t)n_img * nv * nu * sizeof(float) + 255) & ~(size_t)255;
}

int run_denoise(const double* shat, long long stride, int n_img, int nv, int nu, float beta, float omega, int iters,
                float s_floor, double* out, void* ws, size_t ws_bytes, hipStream_t st) {
    if (!shat || !out) return fail(GDRR_EINVAL, "shat / out is NULL");
    if (n_img < 1 || nv < 1 || nu < 1) return fail(GDRR_EINVAL, "n_img, nv and nu must be >= 1");
    const long long npix = (long long)nv * nu;
    if (stride == 0) stride = npix;
    if (stride < npix) return fail(GDRR_EINVAL, "shat_stride must be 0 or >= nv * nu");
    if (!(beta > 0.0f) || !std::isfinite(beta)) return fail(GDRR_EINVAL, "beta must be finite and > 0");
    if (!(omega > 0.0f && omega < 2.0f)) return fail(GDRR_EINVAL, "omega must be in (0, 2)");
    if (iters < 0 || iters > (1 << 20)) return fail(GDRR_EINVAL, "iters must be in [0, 2^20]");
    if (!(s_floor > 0.0f) || !std::isfinite(s_floor)) return fail(GDRR_EINVAL, "s_floor must be finite and > 0");
    const int tiles_u = (nu + kDnTileU - 1) / kDnTileU, tiles_v = (nv + kDnTileV - 1) / kDnTileV;
    if ((long long)n_img * tiles_u * tiles_v >= (1ll << 31)) return fail(GDRR_EINVAL, "too many tiles in one call");
    const size_t in_bytes = ((size_t)(n_img - 1) * (size_t)stride + (size_t)npix) * sizeof(double);
    const size_t out_bytes = (size_t)n_img * (size_t)npix * sizeof(double);
    if (ranges_overlap(shat, in_bytes, out, out_bytes)) return fail(GDRR_EINVAL, "out must not overlap shat");
    const size_t buf = dn_buffer_bytes(n_img, nv, nu);
    if (!ws || ws_bytes < 2 * buf + 256) return fail(GDRR_EINVAL, "workspace too small: need " + std::to_string(2 * buf + 256) + " bytes");
    char* wsa = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    float* pp[2] = {(float*)wsa, (float*)(wsa + buf)};
    std::vector<Launch> ls;
    // whole images in one workgroup's registers: 64 C columns, R rows per wavefront
    const void* image_kernel = nullptr;
    int image_waves = 0;
    const int img_c[3] = {4, 2, 1}, img_r[3] = {12, 24, 48};
    const void* img_k[3] = {(const void*)&denoise_image_kernel<4, 12>, (const void*)&denoise_image_kernel<2, 24>,
                            (const void*)&denoise_image_kernel<1, 48>};
    for (int q = 0; q < 3 && !image_kernel; ++q)
        if (nu == 64 * img_c[q] && nv % img_r[q] == 0 && nv / img_r[q] <= 16) {
            image_kernel = img_k[q];
            image_waves = nv / img_r[q];
        }
    const int passes = image_kernel ? 0 : std::max(1, (iters + kDnHalo - 1) / kDnHalo);
    if (image_kernel) {
        DnParams d{};
        d.shat = shat;
        d.shat_stride = stride;
        d.out = out;
        d.n_img = n_img; d.nv = nv; d.nu = nu;
        d.iters = iters;
        d.omega = omega;
        d.inv_beta = 1.0f / beta;
        d.s_floor = s_floor;
        ls.push_back(make_launch(image_kernel, dim3((unsigned)n_img), dim3(64 * image_waves), 0, d));
    }
    for (int p = 0; p < passes; ++p) {
        DnParams d{};
        d.shat = shat;
        d.shat_stride = stride;
        d.s_in = p == 0 ? nullptr : pp[p & 1];
        d.s_out = p + 1 == passes ? nullptr : pp[(p + 1) & 1];
        d.out = p + 1 == passes ? out : nullptr;
        d.n_img = n_img; d.nv = nv; d.nu = nu; d.tiles_u = tiles_u; d.tiles_v = tiles_v;
        d.iters = std::min(kDnHalo, iters - p * kDnHalo);
        d.omega = omega;
        d.inv_beta = 1.0f / beta;
        d.s_floor = s_floor;
        const bool inside = nv >= kDnWaves * kDnRows && nu >= kDnCols;
        ls.push_back(make_launch(inside ? (const void*)&denoise_inside_kernel : (const void*)&denoise_kernel,
                                 dim3((unsigned)(n_img * tiles_u * tiles_v)), dim3(kDnBlock), 0, d));
    }
    TimeEvents* ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_time_mu);
        int rc;
        if (g_timing && (rc = timing_events(&ev))) return rc;
    }
    return run_direct(ls, st, ev ? 0 : -1, ev, ev ? (int)ls.size() - 1 : -1);
}

// --------------------------------------------------------------------------
// Scratch of gdrr_mc_project_static: one array per device in the code object.
// Host code never passes `scratch` itself (in host code the name stands for a
// host-side shadow); it passes the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device.
// --------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GDRR_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64];

int static_scratch(void** out) {
    int dev = 0;
    GDRR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(GDRR_ENOTSUP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GDRR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GDRR_EHIP, "hipGetSymbolAddress returned NULL for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GDRR_OK;
}

gdrr_job single_job(const gdrr_geometry* geom, uint64_t n, uint32_t job_id) {
    gdrr_job j{};
    j.volume = 0;
    j.source = 0;
    j.geom = *geom;
    j.n_photons = n;
    j.job_id = job_id;
    j.tally_offset = 0;
    return j;
}

}  // namespace

extern "C" {

const char* gdrr_last_error(void) { return g_err.c_str(); }

const char* gdrr_version(void) { return "gdrr-mi355x 0.1"; }

int gdrr_init(void) {
    DevInfo d;
    int rc = device_info(d);
    if (rc) return rc;
    void* p = nullptr;
    return static_scratch(&p);
}

int gdrr_enable_timing(int enable) {
    std::lock_guard<std::mutex> lk(g_time_mu);
    g_timing = enable != 0;
    return GDRR_OK;
}

int gdrr_last_kernel_ms(float* ms) {
    if (!ms) return fail(GDRR_EINVAL, "ms is NULL");
    int dev = 0;
    GDRR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_time_mu);
    if (dev < 0 || dev >= 64 || !g_tev[dev].recorded) return fail(GDRR_EINVAL, "no timed launch on this device");
    GDRR_HIP(hipEventSynchronize(g_tev[dev].b));
    GDRR_HIP(hipEventElapsedTime(ms, g_tev[dev].a, g_tev[dev].b));
    return GDRR_OK;
}

int gdrr_default_tuning(gdrr_tuning* out) {
    if (!out) return fail(GDRR_EINVAL, "out is NULL");
    out->block = 256;
    out->blocks_per_cu = 0;
    out->chunk = 0;
    out->defer = 32;
    out->coll_defer = 0;
    return GDRR_OK;
}

size_t gdrr_majorant_workspace(void) { return 4096; }

int gdrr_majorant(const gdrr_volume* vol, const gdrr_physics* phys, uint32_t flags, float margin, float* out,
                  void* workspace, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_volume(vol)) || (rc = check_physics(phys))) return rc;
    if (!out) return fail(GDRR_EINVAL, "out is NULL");
    if (!(margin >= 0.0f) || !std::isfinite(margin)) return fail(GDRR_EINVAL, "margin must be finite and >= 0");
    if (!workspace || ws_bytes < gdrr_majorant_workspace()) return fail(GDRR_EINVAL, "workspace too small");
    DevInfo dev;
    if ((rc = device_info(dev))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // the status block first (as in every workspace; word 1 holds the input-error bits), then the
    // per-material maxima and presence flags
    unsigned long long* head = (unsigned long long*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    unsigned int* err = (unsigned int*)(head + 1);
    unsigned int* rmax = (unsigned int*)(head + 8);
    unsigned int* pres = rmax + 256;
    std::vector<Launch> ls;
    FillParams f{head, 8 + 256};
    ls.push_back(make_launch((const void*)&fill_zero_kernel, dim3(2), dim3(256), 0, f));
    MajParams m{vol->density, vol->material, vol->nx, vol->ny, vol->nz, (flags & GDRR_INTERP_DENSITY) ? 1 : 0,
                phys->n_mat, rmax, pres, err};
    const long long nvox = (long long)vol->nx * vol->ny * vol->nz;
    const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>(dev.cus * 8, (nvox + 255) / 256));
    ls.push_back(make_launch((const void*)&rho_max_kernel, dim3(g), dim3(256), 0, m));
    MajFinParams fp{rmax, pres, phys->mu_mass, phys->n_mat, phys->n_e, 1.0 + (double)margin, out, err};
    ls.push_back(make_launch((const void*)&majorant_kernel, dim3((phys->n_e + 254) / 256), dim3(256), 0, fp));
    return run_direct(ls, st);
}

size_t gdrr_mc_project_workspace(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                                 const gdrr_geometry* geom) {
    if (!geom) return 0;
    gdrr_job j = single_job(geom, 0, 0);
    return batch_bytes(vol, 1, phys, src, 1, &j, 1, true);
}

int gdrr_mc_project(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                    const gdrr_geometry* geom, const float* majorant, uint64_t seed, uint64_t n_photons,
                    uint32_t job_id, uint32_t flags, double* tally, void* workspace, size_t ws_bytes,
                    void* stream) {
    if (!geom) return fail(GDRR_EINVAL, "geometry is NULL");
    if (!tally) return fail(GDRR_EINVAL, "tally is NULL");
    gdrr_job j = single_job(geom, n_photons, job_id);
    Batch B{vol, 1, phys, src, 1, &j, 1, majorant, seed, flags, nullptr, kModeForward, -1, tally,
            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false};
    return run_batch(B, workspace, ws_bytes, (hipStream_t)stream);
}

int gdrr_mc_project_static(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                           const gdrr_geometry* geom, const float* majorant, uint64_t seed, uint64_t n_photons,
                           uint32_t job_id, uint32_t flags, double* tally, void* stream) {
    if (!geom) return fail(GDRR_EINVAL, "geometry is NULL");
    if (!tally) return fail(GDRR_EINVAL, "tally is NULL");
    if (flags & GDRR_RESUME) return fail(GDRR_EINVAL, "gdrr_mc_project_static does not resume (GDRR_RESUME)");
    gdrr_job j = single_job(geom, n_photons, job_id);
    Batch B{vol, 1, phys, src, 1, &j, 1, majorant, seed, flags, nullptr, kModeForward, -1, tally,
            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false};
    B.tables_by_kernel = true;
    int rc = check_batch(B);
    if (rc) return rc;
    const size_t need = batch_bytes(vol, 1, phys, src, 1, &j, 1, majorant == nullptr);
    if (need > GDRR_STATIC_SCRATCH_BYTES)
        return fail(GDRR_EINVAL, "gdrr_mc_project_static: the call needs " + std::to_string(need) +
                                 " bytes of scratch; the static scratch holds " +
                                 std::to_string((size_t)GDRR_STATIC_SCRATCH_BYTES) + " (use gdrr_mc_project)");
    void* ws = nullptr;
    if ((rc = static_scratch(&ws))) return rc;
    return run_batch(B, ws, GDRR_STATIC_SCRATCH_BYTES, (hipStream_t)stream);
}

size_t gdrr_mc_project_batch_workspace(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                                       const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs,
                                       int32_t n_jobs) {
    return batch_bytes(vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs, true);
}

int gdrr_mc_project_batch(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                          const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs,
                          const float* majorants, uint64_t seed, uint32_t flags, const gdrr_tuning* tune,
                          double* tallies, void* workspace, size_t ws_bytes, void* stream) {
    if (!tallies) return fail(GDRR_EINVAL, "tallies is NULL");
    Batch B{vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs, majorants, seed, flags, tune, kModeForward, -1,
            tallies, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true};
    return run_batch(B, workspace, ws_bytes, (hipStream_t)stream);
}

int gdrr_mc_backward(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys, const gdrr_source* srcs,
                     int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs, int32_t volume, const float* majorants,
                     uint64_t seed, uint32_t flags, const gdrr_tuning* tune, const double* adj,
                     double* grad_density, void* workspace, size_t ws_bytes, void* stream) {
    if (!majorants) return fail(GDRR_EINVAL, "the adjoint needs the forward's majorants");
    if (!adj || !grad_density) return fail(GDRR_EINVAL, "adj / grad_density is NULL");
    if (volume < 0 || volume >= n_vols) return fail(GDRR_EINVAL, "volume index out of range");
    // (the gradient is cleared by run_batch's launch list, after every argument check)
    Batch B{vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs, majorants, seed, flags, tune, kModeBackward, volume,
            nullptr, adj, grad_density, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false};
    return run_batch(B, workspace, ws_bytes, (hipStream_t)stream);
}

size_t gdrr_primary_workspace(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys,
                              const gdrr_source* srcs, int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs) {
    if (!vols || !phys || !srcs || !jobs || n_vols < 1 || n_vols > GDRR_MAX_VOLUMES || n_srcs < 1 ||
        n_srcs > GDRR_MAX_SOURCES || n_jobs < 1)
        return 0;
    for (int k = 0; k < n_jobs; ++k)
        if (jobs[k].volume < 0 || jobs[k].volume >= n_vols) return 0;
    for (int v = 0; v < n_vols; ++v)
        if (vols[v].nx < 1 || vols[v].ny < 1 || vols[v].nz < 1) return 0;
    for (int s = 0; s < n_srcs; ++s)
        if (srcs[s].n_spec < 1 || spec_rows(srcs[s]) < 0) return 0;
    return rt_carve(nullptr, vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs).bytes + 256;
}

int gdrr_primary(const gdrr_volume* vols, int32_t n_vols, const gdrr_physics* phys, const gdrr_source* srcs,
                 int32_t n_srcs, const gdrr_job* jobs, int32_t n_jobs, float step_mm, uint32_t flags, double* out,
                 void* workspace, size_t ws_bytes, void* stream) {
    return run_primary(vols, n_vols, phys, srcs, n_srcs, jobs, n_jobs, step_mm, flags, out, workspace, ws_bytes,
                       (hipStream_t)stream);
}

size_t gdrr_denoise_workspace(int32_t n_img, int32_t nv, int32_t nu) {
    if (n_img < 1 || nv < 1 || nu < 1) return 0;
    return 2 * dn_buffer_bytes(n_img, nv, nu) + 256;
}

int gdrr_denoise(const double* shat, int64_t shat_stride, int32_t n_img, int32_t nv, int32_t nu, float beta,
                 float omega, int32_t iters, float s_floor, double* out, void* workspace, size_t ws_bytes,
                 void* stream) {
    return run_denoise(shat, shat_stride, n_img, nv, nu, beta, omega, iters, s_floor, out, workspace, ws_bytes,
                       (hipStream_t)stream);
}

int gdrr_noise(int32_t n_img, int64_t npix, const double* phat, int64_t phat_stride, const double* p,
               const double* shat, int64_t shat_stride, const double* s, double alpha, double* noise,
               double* image, void* stream) {
    if (!phat || !p || !shat || !s) return fail(GDRR_EINVAL, "input pointer is NULL");
    if (n_img < 1 || npix < 1) return fail(GDRR_EINVAL, "n_img and npix must be >= 1");
    if (phat_stride == 0) phat_stride = npix;
    if (shat_stride == 0) shat_stride = npix;
    if (phat_stride < npix || shat_stride < npix) return fail(GDRR_EINVAL, "strides must be 0 or >= npix");
    if (!std::isfinite(alpha)) return fail(GDRR_EINVAL, "alpha must be finite");
    NoiseParams q{phat, phat_stride, p, shat, shat_stride, s, alpha, noise, image, npix, n_img};
    const long long total = npix * (long long)n_img;
    const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(8192, (total + 255) / 256));
    void* a[1] = {&q};
    GDRR_HIP(hipLaunchKernel((const void*)&noise_kernel, dim3(grid), dim3(256), a, 0, (hipStream_t)stream));
    return GDRR_OK;
}

int gdrr_noise_scale(double n_sim, double zeta, double mas, double* alpha) {
    if (!alpha) return fail(GDRR_EINVAL, "alpha is NULL");
    if (!(n_sim > 0.0 && zeta > 0.0 && mas > 0.0) || !std::isfinite(n_sim) || !std::isfinite(zeta) ||
        !std::isfinite(mas))
        return fail(GDRR_EINVAL, "n_sim, zeta and mAs must be finite and > 0");
    *alpha = std::sqrt(n_sim / (zeta * mas));
    return GDRR_OK;
}

int gdrr_input_status(const void* workspace, void* stream) {
    if (!workspace) return fail(GDRR_EINVAL, "workspace is NULL");
    hipStream_t st = (hipStream_t)stream;
    const unsigned int* word = (const unsigned int*)((((uintptr_t)workspace + 255) & ~(uintptr_t)255) + 8);
    unsigned int bits = 0;
    GDRR_HIP(hipStreamSynchronize(st));
    GDRR_HIP(hipMemcpyAsync(&bits, word, sizeof(bits), hipMemcpyDeviceToHost, st));
    GDRR_HIP(hipStreamSynchronize(st));
    if (!bits) return GDRR_OK;
    std::string msg = "invalid device inputs:";
    if (bits & kErrDensity) msg += " densities negative, NaN or infinite (transported as 0);";
    if (bits & kErrMaterial) msg += " material indices >= n_mat (transported as n_mat - 1);";
    if (bits & kErrWeights) msg += " spectrum or fluence weights negative, non-finite or summing to 0;";
    msg.pop_back();
    return fail(GDRR_EINVAL, msg);
}

int gdrr_mc_trace(const gdrr_volume* vol, const gdrr_physics* phys, const gdrr_source* src,
                  const gdrr_geometry* geom, const float* majorant, uint64_t seed, uint64_t n_photons,
                  uint32_t job_id, uint32_t flags, int8_t* cls, int32_t* pixel, float* e_final, int32_t* steps,
                  int32_t* n_compton, int32_t* n_rayleigh, void* workspace, size_t ws_bytes, void* stream) {
    if (!geom) return fail(GDRR_EINVAL, "geometry is NULL");
    gdrr_job j = single_job(geom, n_photons, job_id);
    Batch B{vol, 1, phys, src, 1, &j, 1, majorant, seed, flags, nullptr, kModeTrace, -1, nullptr, nullptr,
            nullptr, cls, pixel, e_final, steps, n_compton, n_rayleigh, false};
    return run_batch(B, workspace, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
