// Event-queue variant of the transport kernel.
//
// Lanes only fly.  A photon that meets a real collision leaves its lane for a
// collision queue in LDS; collisions are processed by consecutive threads of
// the workgroup once a wavefront's worth has gathered, and fresh source
// photons are generated the same way.  Both kinds of result go to a ready
// queue in LDS, from which lanes whose photon left or ended take their next
// photon.  Interactions and source sampling thus run on packed lanes instead
// of on the few lanes of each wavefront that need them.  Per iteration:
//   A  lanes without a photon take ready photons;
//   F  flying lanes do one flight pair; real collisions are pushed to the
//      collision queue (a lane keeps its photon if the queue is full);
//   M  thread 0 decides how many collisions to process and fresh photons to
//      generate, and serves the chunk dispenser;
//   CG consecutive threads process the chosen collisions and generate the
//      fresh photons into the ready queue; lanes that kept a collision
//      process it in place.
// Barriers separate F | M | CG | A, and every decision is read from LDS after
// a barrier, so the workgroup stays in lockstep.  The loop ends when the
// dispenser is empty and no photon is in a lane or a queue.
#pragma once

#include "gdrr_kernels.h"

namespace gdrr {

constexpr int kQWords = 15;   // words per queued photon

struct QArrays {
    float *x, *y, *z, *dx, *dy, *dz, *E, *aux, *w;
    uint32_t *pid, *step, *pair, *nsc, *pix, *job;
};

__device__ __forceinline__ QArrays q_carve(float* base, int cap) {
    QArrays q;
    float* f = base;
    q.x = f; q.y = f + cap; q.z = f + 2 * cap; q.dx = f + 3 * cap; q.dy = f + 4 * cap; q.dz = f + 5 * cap;
    q.E = f + 6 * cap; q.aux = f + 7 * cap; q.w = f + 8 * cap;
    uint32_t* u = reinterpret_cast<uint32_t*>(f + 9 * cap);
    q.pid = u; q.step = u + cap; q.pair = u + 2 * cap; q.nsc = u + 3 * cap; q.pix = u + 4 * cap; q.job = u + 5 * cap;
    return q;
}

// aux = sel (collision queue) or trem (ready queue)
__device__ __forceinline__ void q_store(const QArrays& q, int i, const Photon& ph, float aux) {
    q.x[i] = ph.px; q.y[i] = ph.py; q.z[i] = ph.pz;
    q.dx[i] = ph.dx; q.dy[i] = ph.dy; q.dz[i] = ph.dz;
    q.E[i] = ph.E; q.aux[i] = aux; q.w[i] = ph.w;
    q.pid[i] = ph.pid; q.step[i] = ph.step; q.pair[i] = ph.pair; q.nsc[i] = ph.nsc;
    q.pix[i] = (uint32_t)ph.pix0 | ((uint32_t)ph.pm << 24) | (ph.passb ? 0x80000000u : 0u);
    q.job[i] = (uint32_t)ph.job;
}

__device__ __forceinline__ void q_load(const QArrays& q, int i, Photon& ph, float& aux) {
    ph.px = q.x[i]; ph.py = q.y[i]; ph.pz = q.z[i];
    ph.dx = q.dx[i]; ph.dy = q.dy[i]; ph.dz = q.dz[i];
    ph.E = q.E[i]; aux = q.aux[i]; ph.w = q.w[i];
    ph.pid = q.pid[i]; ph.step = q.step[i]; ph.pair = q.pair[i]; ph.nsc = q.nsc[i];
    const uint32_t px = q.pix[i];
    ph.pix0 = (int)(px & 0xFFFFFFu);
    ph.pm = (int)((px >> 24) & 0x7Fu);
    ph.passb = (px >> 31) != 0u;
    ph.job = (int)q.job[i];
}

__host__ __device__ inline int queue_cap(int block) { return max(64, 3 * block / 8); }

__host__ __device__ inline size_t queue_lds_bytes(int n_mat, int n_e, int n_vols, bool resp, int block) {
    const int qc = queue_cap(block), rc = 2 * queue_cap(block);
    return table_floats2(n_mat, n_e, n_vols, resp) * 8 + (size_t)kQWords * 4 * (qc + rc) + 64 * 4 + 2 * 16 * 4;
}

enum : int {
    kCtlQn = 0, kCtlRn, kCtlJob, kCtlNext, kCtlEnd, kCtlVol, kCtlExh, kCtlHold,
    kCtlCFirst, kCtlCCount, kCtlGCount, kCtlGPid, kCtlGJob, kCtlExit, kCtlHaveChunk, kCtlCount
};

template <int MODE>
__global__ __launch_bounds__(1024) void mc_queue_kernel(KParams P) {
    extern __shared__ float2 lds[];
    const Tables T = stage_tables(P, lds);
    const int B = blockDim.x;
    const int QCAP = queue_cap(B), RCAP = 2 * queue_cap(B), RTARGET = queue_cap(B);
    float* qbase = reinterpret_cast<float*>(lds + table_floats2(P.n_mat, P.n_e, P.n_vols, P.response != nullptr));
    const QArrays Q = q_carve(qbase, QCAP);
    const QArrays R = q_carve(qbase + kQWords * QCAP, RCAP);
    int* ctl = reinterpret_cast<int*>(qbase + kQWords * (QCAP + RCAP));
    int* w_free = ctl + 64;
    int* w_busy = w_free + 16;
    const int NW = B >> 6, wave = threadIdx.x >> 6, lane = __lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    if (threadIdx.x == 0) {
        for (int k = 0; k < kCtlCount; ++k) ctl[k] = 0;
        ctl[kCtlVol] = -1;
    }
    if (lane == 0) { w_free[wave] = 64; w_busy[wave] = 0; }
    __syncthreads();
    const bool interp = (P.flags & 1u) != 0;

    Photon ph;
    ph.st = kDead;
    ph.passb = false;
    ph.w = 0.0f;
    ph.job = 0; ph.pid = 0; ph.jid = 0; ph.nsc = 0; ph.sel = 0.0f; ph.pair = 0u; ph.pm = 0; ph.step = 0;

    for (;;) {
        const int vol = ctl[kCtlVol];
        const DVolume& V = P.vol[vol < 0 ? 0 : vol];
        const int vo = V.lds_majorant;
        // ---- A: lanes without a photon take ready photons (top of the ready stack) ----
        const int nr = ctl[kCtlRn];
        if (nr > 0) {
            int before = 0;
            for (int w = 0; w < wave; ++w) before += w_free[w];
            const bool fr = ph.st == kDead;
            const int g = before + __popcll(__ballot(fr) & lt);
            if (fr && g < nr) {
                float trem;
                q_load(R, nr - 1 - g, ph, trem);
                ph.trem = trem;
                ph.jid = P.jobs[ph.job].job_id;
                ph.ec = energy_cache(P, T, vo, ph.E);
                ph.st = kFly;
            }
        }
        // ---- F: one flight pair per flying lane ----
        if (ph.st == kFly) {
            ph.pair += 1u;
            const Block b = philox(ph.pid, ph.jid, ph.pair, 0u, P.k0, P.k1);
            if (flight<MODE>(P, T, V, vo, interp, ph, b.x, b.y)) flight<MODE>(P, T, V, vo, interp, ph, b.z, b.w);
        }
        {   // push real collisions to the collision queue (one LDS atomic per wavefront)
            const bool push = ph.st == kColl;
            const uint64_t pm = __ballot(push);
            if (pm) {
                const int first = __ffsll((long long)pm) - 1;
                int base = 0;
                if (lane == first) base = atomicAdd(&ctl[kCtlQn], __popcll(pm));
                base = __shfl(base, first);
                const int slot = base + __popcll(pm & lt);
                if (push && slot < QCAP) {
                    q_store(Q, slot, ph, ph.sel);
                    ph.st = kDead;
                }
            }
        }
        {
            const int busy = __popcll(__ballot(ph.st != kDead));
            if (lane == 0) w_busy[wave] = busy;
        }
        __syncthreads();
        // ---- M: decisions (thread 0) ----
        if (threadIdx.x == 0) {
            int nfree = 0, busy = 0;
            for (int w = 0; w < NW; ++w) { nfree += w_free[w]; busy += w_busy[w]; }
            const int taken = min(nfree, nr);
            const int nr_left = nr - taken;
            const int nq = min(ctl[kCtlQn], QCAP);
            // dispenser: make sure a chunk of the current phantom is at hand
            if (!ctl[kCtlExh] && !ctl[kCtlHaveChunk]) {
                const unsigned long long c = atomicAdd(P.counter, 1ull);
                if (c >= P.total_chunks) {
                    ctl[kCtlExh] = 1;
                } else {
                    int lo = 0, hi = P.n_jobs - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (P.chunk_prefix[mid] <= c) lo = mid; else hi = mid - 1;
                    }
                    const DJob& J = P.jobs[lo];
                    const unsigned long long nph = (unsigned long long)J.n_lo | ((unsigned long long)J.n_hi << 32);
                    const unsigned long long first = (c - P.chunk_prefix[lo]) * (unsigned long long)P.chunk;
                    const unsigned long long last = first + (unsigned long long)P.chunk < nph ? first + P.chunk : nph;
                    ctl[kCtlJob] = lo;
                    ctl[kCtlNext] = (int)(uint32_t)first;
                    ctl[kCtlEnd] = (int)(uint32_t)last;
                    ctl[kCtlHaveChunk] = 1;
                }
            }
            // a chunk of another phantom waits until this workgroup holds no photon
            if (ctl[kCtlHaveChunk]) {
                const int v = P.jobs[ctl[kCtlJob]].vol;
                if (v != ctl[kCtlVol]) {
                    if (busy == 0 && nq == 0 && nr_left == 0) ctl[kCtlVol] = v;
                }
            }
            const bool can_gen = ctl[kCtlHaveChunk] && P.jobs[ctl[kCtlJob]].vol == ctl[kCtlVol];
            int cc = 0;
            if (nq >= 64 || (!can_gen && nq > 0) || (nq > 0 && busy == 0 && nr_left == 0)) cc = min(nq, RCAP - nr_left);
            ctl[kCtlCFirst] = nq - cc;
            ctl[kCtlCCount] = cc;
            ctl[kCtlQn] = nq - cc;
            int gc = 0;
            if (can_gen) {
                const int room = RCAP - nr_left - cc;
                const int want = RTARGET - nr_left - cc;
                const int avail = (int)((uint32_t)ctl[kCtlEnd] - (uint32_t)ctl[kCtlNext]);
                gc = min(min(room, want > 0 ? want : 0), avail);
                if (gc < 0) gc = 0;
                ctl[kCtlGPid] = ctl[kCtlNext];
                ctl[kCtlGJob] = ctl[kCtlJob];
                ctl[kCtlNext] = (int)((uint32_t)ctl[kCtlNext] + (uint32_t)gc);
                if ((uint32_t)ctl[kCtlNext] >= (uint32_t)ctl[kCtlEnd]) ctl[kCtlHaveChunk] = 0;
            }
            ctl[kCtlGCount] = gc;
            ctl[kCtlRn] = nr_left;
            ctl[kCtlExit] = (ctl[kCtlExh] && !ctl[kCtlHaveChunk] && busy == 0 && nq == 0 && nr_left == 0) ? 1 : 0;
        }
        __syncthreads();
        if (ctl[kCtlExit]) break;
        // ---- CG: packed collisions and fresh photons ----
        {
            const int cc = ctl[kCtlCCount], gc = ctl[kCtlGCount], cf = ctl[kCtlCFirst];
            const int gpid = ctl[kCtlGPid], gjob = ctl[kCtlGJob];
            const int vnow = ctl[kCtlVol];
            const DVolume& V2 = P.vol[vnow < 0 ? 0 : vnow];
            const int vo2 = V2.lds_majorant;
            for (int t = threadIdx.x; t < cc + gc; t += B) {
                Photon tp;
                tp.passb = false;
                tp.w = 0.0f;
                tp.sel = 0.0f;
                tp.pm = 0;
                if (t < cc) {
                    float sel;
                    q_load(Q, cf + t, tp, sel);
                    tp.sel = sel;
                    tp.jid = P.jobs[tp.job].job_id;
                    tp.ec = energy_cache(P, T, vo2, tp.E);
                    tp.st = kColl;
                    collide<MODE>(P, T, V2, vo2, tp);
                } else {
                    tp.pid = (uint32_t)gpid + (uint32_t)(t - cc);
                    tp.job = gjob;
                    tp.jid = P.jobs[gjob].job_id;
                    tp.nsc = 0;
                    if (start_photon(P, T, V2, vo2, tp)) tp.st = kFly;
                    else finish<MODE>(P, T, V2, vo2, tp, kPrimary, tp.pix0);
                }
                if (tp.st == kFly) {
                    const int slot = atomicAdd(&ctl[kCtlRn], 1);
                    q_store(R, slot, tp, tp.trem);
                }
            }
            if (ph.st == kColl) collide<MODE>(P, T, V, vo, ph);   // the queue was full: in place
            const int nfree = __popcll(__ballot(ph.st == kDead));
            if (lane == 0) w_free[wave] = nfree;
        }
        __syncthreads();
    }
}

}  // namespace gdrr
