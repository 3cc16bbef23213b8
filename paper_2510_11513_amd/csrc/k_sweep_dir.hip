// Per-direction sweep order (SNX_DESIGNATION_DIRECTION).
//
// Each direction sweeps the mesh in its own upwind order, the mesh traversal of
// every direction that Section 2.1 describes: face f of cell K is inflow for
// direction n when Omega_n . A_f < 0.  On distorted meshes a direction's graph
// can have cycles; set-up breaks them by lagging only faces inside the
// strongly connected components of that graph (the upwind cell ranked after
// the downwind one by Omega_n . centroid), and levels the rest.
//
// The sweep is level-synchronous over those per-direction levels.  A work unit
// is one (cell, octant, direction) on the current level of that direction's
// order; a wave takes several units, stages their cells' element matrices in
// LDS and solves one (unit, group) system per lane, with the direction's own
// inflow faces.  An inflow neighbour sits on an earlier level
// of the same direction, so its angular flux in the hand-off array is this
// sweep's, except across a lagged face, which reads the neighbour's flux of
// the previous sweep from a snapshot taken before the first level.  The angle
// sums go to the octant slots afterwards (the reduction kernel combines them
// as for the other sweeps).
#include <algorithm>

#include "snx_internal.h"

namespace snx {

// Global address space: loads and stores through these pointers compile to
// global_* instructions instead of flat ones (device pass only), so that LDS
// reads do not wait on them.
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#else
#define GLOBAL
#endif

template <typename T>
__device__ __forceinline__ GLOBAL T *gp(T *p) { return (GLOBAL T *)p; }

namespace {

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// The k-th local vertex (increasing order) of face f = 2 axis + side: the 2-bit
// index k with the bit `side` inserted at position `axis`.
__host__ __device__ constexpr int face_vertex_of(int f, int k) {
    return (k & ((1 << (f >> 1)) - 1)) | ((f & 1) << (f >> 1)) | ((k >> (f >> 1)) << ((f >> 1) + 1));
}

__global__ void k_lag_snapshot(DirDev D, const DevProblem *__restrict__ probs, const int *stop) {
    if (stop && *stop) return;
    const DevProblem &P = probs[0];
    const long long G = P.G;
    const long long n = D.nlag * 4 * G;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        D.lagbuf[i] = P.psi[D.lagsrc[i / G] + i % G];
}

// One wave per up to `upw` work units of a level, a unit being one (cell,
// octant, direction) whose level in that direction's order is the current one;
// lane l solves group l % G of unit l / G (G <= 64), or, for G > 64, block y
// takes groups 64 y.. of a single unit.  Packing units rather than one (cell,
// octant) item per wave fills the lanes: an item holds 1.3 directions on
// average, so a wave per item left two thirds of its lanes idle.  Each unit's
// cell matrices and its direction's operators (B = Om . S - sum over the
// direction's inflow faces of Om . F_f, and each inflow face's Om . F_f) are
// built cooperatively in LDS first, so that a lane's row assembly has no face
// branches; only its right-hand side depends on which faces are inflow.
constexpr int kDirThreads = 64;
constexpr int kMaxUnits = 8;                 // units per wave (lanes of G <= 8 groups stay partly idle)
// M, S, F of the cell; B (stride 65); the inflow faces' Om . F; padded to whole
// float4s so that every unit's block is 16-byte aligned (units' B blocks then
// start 4 banks apart)
constexpr int kUnitFloats = 544 + 65 + 96 + 3;

// The units sTask/sDir[0, nu) of this wave (64 threads): their cells' data and
// operators into LDS, then one (unit, group) system per lane, whose angular
// flux goes to the hand-off array.  `gy` is the block of 64 groups (G > 64).
// The angular flux is stored and read with device-scope (sc1) accesses, which
// the dependency-driven sweep needs to hand it across CUs and XCDs (the level
// launches measured no faster with plain ones).
__device__ __forceinline__ void solve_units(const DirDev &D, const DevProblem &P, int nu, const int *sTask,
                                            const int *sDir, float *smem, int gy) {
    const int C = P.C, A = P.A, G = P.G;
    const int tid = threadIdx.x;
    __shared__ float sOm[kMaxUnits][3];
    __shared__ int sMk[kMaxUnits], sLag[kMaxUnits], sLidx[kMaxUnits];
    __shared__ int sNb[kDirThreads];        // [unit][face] neighbour
    __shared__ unsigned sPm[kDirThreads];   // [unit][face] neighbour's node map
    // The units' neighbours and node maps (lane = 6 unit + face) and their
    // directions, masks and lag slots (lane mod 8 = unit), loaded by every lane
    // at clamped indices so that no load waits on a branch; then the cell data
    // (M, S, F: 136 float4 per cell), each lane's share loaded before any of it
    // is stored, nine float4 at a time; the small values are stored after.
    const int tu = min(tid / 6, nu - 1), tf = tid % 6;
    const int tK = sTask[tu] >> 3;
    const int nbv = gp(P.nbr)[(size_t)tK * 6 + tf];
    const unsigned pmv = gp(P.perm)[(size_t)tK * 6 + tf];
    const int wu = min(tid & 7, nu - 1), wtask = sTask[wu], wa = sDir[wu];
    const int wo = wtask & 7, wn = wo * A + wa;
    const size_t woka = ((size_t)wo * C + (wtask >> 3)) * A + wa;
    const float om0 = gp(P.omega)[3 * wn], om1 = gp(P.omega)[3 * wn + 1], om2 = gp(P.omega)[3 * wn + 2];
    const int wmk = gp(D.amask)[woka], wlag = gp(D.lagbits)[woka], wlidx = gp(D.lagidx)[woka];
    const int n4 = nu * 136;
    for (int r0 = 0; r0 < n4; r0 += 9 * kDirThreads) {
        float4 v[9];
        int dst[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {   // past the end: the last float4 again (the same value to the same place)
            const int e = min(r0 + r * kDirThreads + tid, n4 - 1);
            const int u = e / 136, j = e - 136 * u;
            const int K = sTask[u] >> 3;
            const GLOBAL float *src = j < 16 ? gp(P.M) + (size_t)K * 64 + 4 * j
                                             : (j < 64 ? gp(P.S) + (size_t)K * 192 + 4 * (j - 16)
                                                       : gp(P.F) + (size_t)K * 288 + 4 * (j - 64));
            v[r] = *reinterpret_cast<const GLOBAL float4 *>(src);
            dst[r] = u * kUnitFloats + 4 * j;
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) *reinterpret_cast<float4 *>(smem + dst[r]) = v[r];
    }
    sNb[tid] = nbv;
    sPm[tid] = pmv;
    sOm[tid & 7][0] = om0;   // lanes of one slot store the same values
    sOm[tid & 7][1] = om1;
    sOm[tid & 7][2] = om2;
    sMk[tid & 7] = wmk;
    sLag[tid & 7] = wlag;
    sLidx[tid & 7] = wlidx;
    __syncthreads();
    for (int idx = tid; idx < nu * (64 + 96); idx += kDirThreads) {
        const int u = idx / (64 + 96), e = idx % (64 + 96);
        const float *sS = smem + u * kUnitFloats + 64, *sF = smem + u * kUnitFloats + 256;
        const float ox = sOm[u][0], oy = sOm[u][1], oz = sOm[u][2];
        const int mask = sMk[u];
        if (e < 64) {
            const int i = e >> 3, j = e & 7;
            float v = ox * sS[e] + oy * sS[64 + e] + oz * sS[128 + e];
            for (int f = 0; f < 6; ++f) {
                const int ax = f >> 1, sd = f & 1;
                if (!((mask >> f) & 1) || ((i >> ax) & 1) != sd || ((j >> ax) & 1) != sd) continue;
                // positions of i and j among the face's vertices: drop bit `ax`
                const int k = (i & ((1 << ax) - 1)) | ((i >> (ax + 1)) << ax);
                const int l = (j & ((1 << ax) - 1)) | ((j >> (ax + 1)) << ax);
                const float *F = sF + f * 48 + 4 * k + l;
                v -= ox * F[0] + oy * F[16] + oz * F[32];
            }
            smem[u * kUnitFloats + 544 + e] = v;
        } else {
            const int f = (e - 64) >> 4, kl = (e - 64) & 15;
            const float *F = sF + f * 48 + kl;
            smem[u * kUnitFloats + 544 + 65 + f * 16 + kl] = ((mask >> f) & 1) ? ox * F[0] + oy * F[16] + oz * F[32]
                                                                              : 0.f;
        }
    }
    __syncthreads();

    const int u = G <= kDirThreads ? tid / G : 0;
    const int g = G <= kDirThreads ? tid % G : gy * kDirThreads + tid;
    if (u >= nu || g >= G) return;   // (no barrier follows in this function)
    const int task = sTask[u], a = sDir[u];
    const int K = task >> 3, o = task & 7;
    const size_t AG = (size_t)A * G;
    const int mask = sMk[u], lagb = sLag[u], lbase = lagb ? sLidx[u] : 0;
    // every inflow trace first, from an address chosen per face (one block of
    // loads in flight together; faces without a trace read a valid dummy and
    // take zero), then the products
    const GLOBAL float *dummy = gp(P.sigt) + (size_t)K * G + g;
    float uu[6][4];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int N = sNb[6 * u + f];
        const unsigned pm = sPm[6 * u + f];
        const bool in = (mask >> f) & 1, lagged = N >= 0 && ((lagb >> f) & 1);
        const bool zero = !in || (N < 0 && !P.psib);
        const int slot = lbase + __popc(lagb & ((1 << f) - 1));
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int vn = (int)((pm >> (8 * l)) & 0xffu);
            const GLOBAL float *src =
                zero ? dummy
                     : (lagged ? gp(D.lagbuf) + ((size_t)slot * 4 + l) * G + g       // a face lagged to break a cycle
                               : (N >= 0 ? gp(P.psi) + (((size_t)o * C + N) * 8 + vn) * AG + (size_t)a * G + g
                                         : gp(P.psib) + g));                           // the boundary
            const float v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uu[f][l] = zero ? 0.f : v;
        }
    }
    const float sig = gp(P.sigt)[(size_t)K * G + g];
    const float4 r0 = *reinterpret_cast<const GLOBAL float4 *>(gp(P.r) + ((size_t)K * G + g) * 8);
    const float4 r1 = *reinterpret_cast<const GLOBAL float4 *>(gp(P.r) + ((size_t)K * G + g) * 8 + 4);
    const float *sM = smem + u * kUnitFloats;
    const float *Bk = sM + 544, *sOF = sM + 544 + 65;
    float m[64], b[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
    for (int e = 0; e < 64; ++e) m[e] = __builtin_fmaf(sig, sM[e], Bk[e]);
    // right-hand side: minus each inflow face's operator on the upwind trace
    // (zero operator rows on the other faces)
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const float *OF = sOF + f * 16;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
#pragma unroll
            for (int l = 0; l < 4; ++l) t = __builtin_fmaf(OF[4 * k + l], uu[f][l], t);
            b[face_vertex_of(f, k)] -= t;
        }
    }
    // unpivoted LU with forward elimination of b, then back substitution
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float inv = __builtin_amdgcn_rcpf(m[k * 8 + k]);
#pragma unroll
        for (int i = k + 1; i < 8; ++i) {
            const float l = m[i * 8 + k] * inv;
#pragma unroll
            for (int j = k + 1; j < 8; ++j) m[i * 8 + j] = __builtin_fmaf(-l, m[k * 8 + j], m[i * 8 + j]);
            b[i] = __builtin_fmaf(-l, b[k], b[i]);
        }
    }
#pragma unroll
    for (int i = 7; i >= 0; --i) {
        float s = b[i];
#pragma unroll
        for (int j = i + 1; j < 8; ++j) s = __builtin_fmaf(-m[i * 8 + j], b[j], s);
        b[i] = s * __builtin_amdgcn_rcpf(m[i * 8 + i]);
    }
    GLOBAL float *dst = gp(P.psi) + ((size_t)o * C + K) * 8 * AG + (size_t)a * G + g;
#pragma unroll
    for (int d = 0; d < 8; ++d) __hip_atomic_store(dst + d * AG, b[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


__global__ __launch_bounds__(kDirThreads) void k_sweep_dir(DirDev D, const DevProblem *__restrict__ probs,
                                                           long long begin, long long end, int upw, const int *stop) {
    if (stop && *stop) return;
    const DevProblem &P = probs[0];
    const long long u0 = begin + (long long)blockIdx.x * upw;
    const int nu = (int)min((long long)upw, end - u0);
    extern __shared__ __align__(16) float smem[];
    __shared__ int sTask[kMaxUnits], sDir[kMaxUnits];
    const int tid = threadIdx.x;
    if (tid < nu) {
        sTask[tid] = D.units[2 * (u0 + tid)];
        sDir[tid] = D.units[2 * (u0 + tid) + 1];
    }
    __syncthreads();
    solve_units(D, P, nu, sTask, sDir, smem, (int)blockIdx.y);
}

// The dependency-driven form of the same sweep.  A unit (cell, octant,
// direction) is ready when every non-lagged interior inflow face of its
// direction has been solved: a counter per unit, counted up across sweeps to
// in-degree x epoch.  Units of one (octant, direction) share a queue, fixed at
// set-up, and a wave serves the queue of its XCD first.  A wave solves up to
// upw units of one queue together, counts down their downwind neighbours and
// keeps up to upw of those that became ready for its next round (work first:
// most units never pass through a queue); the rest go to the queue in one
// reservation.  An idle wave flushes its solved count to the queue, then takes
// a slot and waits for it to be filled, moving to the next queue when this one
// is finished (its solved count reaches its units) and exiting when every queue
// is.  The angular flux is stored with device-scope stores and the wave waits
// for them to complete before its counter updates, and read with device-scope
// loads issued only after the units' ids came back: the hand-off argument of
// the octant sweep.  A wall-clock watchdog turns a stall into an abort.
__device__ __forceinline__ unsigned ld_agent(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for queue entry `slot` of this epoch; -1 when the queue finishes first
// (finished = true; only for a slot taken by an idle wave) or on abort.
__device__ __forceinline__ long long unit_wait(const unsigned long long *qs, const UnitQ *Q, long long qt,
                                               unsigned slot, unsigned epoch, unsigned *abortp,
                                               unsigned long long watchdog, bool &finished,
                                               unsigned long long &polls) {
    const unsigned long long t0 = wall_clock64();
    int backoff = 1;
    finished = false;
    for (unsigned k = 1;; ++k) {
        if ((long long)slot < qt) {
            const unsigned long long v = __hip_atomic_load(qs + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)(v >> 32) == epoch) return (long long)(v & 0xffffffffull);
        }
        if ((k & 7) == 0) {
            if ((long long)ld_agent(&Q->done) >= qt) { finished = true; return -1; }
            if (ld_agent(abortp)) return -1;
        }
        ++polls;
        if (wall_clock64() - t0 > watchdog) {
            __hip_atomic_store(abortp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(1);
        backoff = backoff < 8 ? 2 * backoff : 8;
    }
}

__device__ __forceinline__ int unit_xcc() {
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 15;   // HW_REG_XCC_ID[3:0]
}

__global__ __launch_bounds__(kDirThreads) void k_sweep_units(DirDev D, const DevProblem *__restrict__ probs,
                                                             int upw, unsigned *abortp,
                                                             unsigned long long watchdog, const int *stop,
                                                             int phase_stats) {
    if (stop && *stop) return;
    const DevProblem &P = probs[0];
    const int C = P.C, A = P.A;
    UnitCtl *ctl = D.uctl;
    const unsigned epoch = ctl->epoch;
    extern __shared__ __align__(16) float smem[];
    __shared__ int sTask[kMaxUnits], sDir[kMaxUnits];
    __shared__ unsigned sReady[kMaxUnits * 6];
    __shared__ int sN, sReadyN;
    const int tid = threadIdx.x;
    // lane 0's state: the queue served, units solved but not yet flushed, units carried over
    int q = unit_xcc() % kUnitQueues;
    const int home = q;
    unsigned unflushed = 0;
    int carried = 0;
    unsigned long long polls = 0, nunits = 0, rounds = 0, ncarried = 0, ph[4] = {0, 0, 0, 0}, mark = 0;
    const bool ph0 = phase_stats && tid == 0;   // lane 0 keeps the phase clock (optional)
    if (tid == 0) sReadyN = 0;
    for (;;) {
        if (ph0) mark = clock64();
        if (tid == 0) {
            int n = carried;   // sTask/sDir[0, carried) hold the continuation, in unit form
            ncarried += (unsigned long long)carried;
            if (n == 0) {
                if (unflushed) {
                    atomicAdd(&ctl->q[q].done, unflushed);
                    unflushed = 0;
                }
                // idle: take a slot of this queue, or of the next ones once it is finished
                for (int tried = 0; tried < kUnitQueues && n == 0; ++tried) {
                    UnitQ *Q = &ctl->q[q];
                    const long long qt = ctl->qtotal[q];
                    bool finished = (long long)ld_agent(&Q->done) >= qt;
                    if (!finished) {
                        const unsigned slot = atomicAdd(&Q->head, 1u);
                        const long long u = unit_wait(D.uqueue + ctl->qbase[q], Q, qt, slot, epoch, abortp,
                                                      watchdog, finished, polls);
                        if (u >= 0) {
                            sTask[0] = (int)u;
                            n = 1;
                        } else if (!finished) {
                            break;   // abort
                        }
                    }
                    if (n == 0) q = q + 1 < kUnitQueues ? q + 1 : 0;
                }
            }
            if (ph0) { const unsigned long long t = clock64(); ph[0] += t - mark; mark = t; }
            // a wave that has just taken a unit tops up from this queue with entries
            // already reserved by a push (never waiting while holding units); a wave
            // that carries units on does not (the queue's control line is the
            // contended resource: topping up every round measured 1.9x slower)
            if (n > 0 && carried == 0) {
                UnitQ *Q = &ctl->q[q];
                const long long qt = ctl->qtotal[q];
                while (n < upw) {
                    const unsigned h = ld_agent(&Q->head), t = ld_agent(&Q->tail);
                    unsigned hh = h;
                    if (h >= t || (long long)h >= qt ||
                        !__hip_atomic_compare_exchange_strong(&Q->head, &hh, h + 1u, __ATOMIC_RELAXED,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                        break;
                    bool fin;
                    const long long u = unit_wait(D.uqueue + ctl->qbase[q], Q, qt, h, epoch, abortp, watchdog,
                                                  fin, polls);
                    if (u < 0) break;   // abort
                    sTask[n++] = (int)u;
                }
            }
            // unit id (o C + K) A + a -> task 8 K + o and direction a
            for (int i = 0; i < n; ++i) {
                const int u = sTask[i], oc = u / A;
                sTask[i] = 8 * (oc % C) + oc / C;
                sDir[i] = u % A;
            }
            sN = n;
        }
        __syncthreads();
        const int nu = sN;
        if (nu == 0) break;
        if (ph0) { const unsigned long long t = clock64(); ph[1] += t - mark; mark = t; }
        solve_units(D, P, nu, sTask, sDir, smem, 0);   // G <= 64 (the host checks)
        if (ph0) { const unsigned long long t = clock64(); ph[2] += t - mark; mark = t; }
        // the angular flux of these units is visible at device scope before any
        // downwind counter moves
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid < nu * 6) {
            const int i = tid / 6, f = tid % 6;
            const int K = sTask[i] >> 3, o = sTask[i] & 7, a = sDir[i];
            const int N = P.nbr[(size_t)K * 6 + f];
            if (N >= 0) {
                const int nf = D.nbrf[(size_t)K * 6 + f];
                const unsigned un = (unsigned)(((size_t)o * C + N) * A + a);
                // face nf of N is inflow for the direction and not lagged: a dependency
                if (((D.amask[un] >> nf) & 1) && !((D.lagbits[un] >> nf) & 1)) {
                    const unsigned old = __hip_atomic_fetch_add(D.ucnt + un, 1u, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                    if (old + 1u == (unsigned)D.uindeg[un] * epoch) sReady[atomicAdd(&sReadyN, 1)] = un;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            const int nr = sReadyN;
            const int keep = nr < upw ? nr : upw;
            for (int i = 0; i < keep; ++i) sTask[i] = (int)sReady[i];
            carried = keep;
            unflushed += (unsigned)nu;
            nunits += (unsigned long long)nu;
            ++rounds;
            if (nr > keep) {   // the rest to the queue (the same queue: same octant and direction)
                UnitQ *Q = &ctl->q[q];
                const long long qt = ctl->qtotal[q];
                const unsigned s0 = atomicAdd(&Q->tail, (unsigned)(nr - keep));
                if ((long long)s0 + (nr - keep) <= qt) {
                    unsigned long long *qs = D.uqueue + ctl->qbase[q];
                    for (int i = keep; i < nr; ++i)
                        __hip_atomic_store(qs + s0 + (i - keep), ((unsigned long long)epoch << 32) | sReady[i],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {   // more units than the queue has: counters inconsistent with the orders
                    __hip_atomic_store(abortp, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    carried = 0;
                }
            }
            sReadyN = 0;
            if (ph0) ph[3] += clock64() - mark;
        }
        __syncthreads();
    }
    if (tid == 0) {
        UnitStat &S = ctl->st[home];
        atomicAdd(&S.units, nunits);
        atomicAdd(&S.rounds, rounds);
        atomicAdd(&S.carried, ncarried);
        atomicAdd(&S.polls, polls);
        if (phase_stats)
            for (int i = 0; i < 4; ++i) atomicAdd(&S.phase[i], ph[i]);
    }
}

// Starts a dependency-driven sweep: the next epoch, each queue empty but for
// its seeds (units without a non-lagged interior inflow face).  One block.
__global__ void k_unit_prologue(DirDev D, const int *stop) {
    if (stop && *stop) return;
    UnitCtl *ctl = D.uctl;
    __shared__ unsigned s_epoch;
    if (threadIdx.x == 0) {
        s_epoch = ctl->epoch + 1u;
        ctl->epoch = s_epoch;
    }
    if (threadIdx.x < kUnitQueues) {
        UnitQ &Q = ctl->q[threadIdx.x];
        Q.head = 0;
        Q.tail = (unsigned)(ctl->seed_off[threadIdx.x + 1] - ctl->seed_off[threadIdx.x]);
        Q.done = 0;
        ctl->st[threadIdx.x] = UnitStat{};
    }
    __syncthreads();
    for (int q = 0; q < kUnitQueues; ++q) {
        const long long b = ctl->seed_off[q], n = ctl->seed_off[q + 1] - b;
        for (long long i = threadIdx.x; i < n; i += blockDim.x)
            D.uqueue[ctl->qbase[q] + i] = ((unsigned long long)s_epoch << 32) | (unsigned)D.seeds[b + i];
    }
}

// Octant slots from the sweep's angular flux: per (octant, cell, group, dof)
// the compensated sum of w_n psi_n over the octant's directions in increasing
// order, as the other sweeps leave them.  Group fastest across threads, so the
// reads of one direction are contiguous.
__global__ void k_dir_slots(const DevProblem *__restrict__ probs, const int *stop) {
    if (stop && *stop) return;
    const DevProblem &P = probs[0];
    const long long G = P.G, A = P.A, C = P.C;
    const long long n = 8 * C * G * 8;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
        const long long g = t % G, d = (t / G) & 7, oc = t / (8 * G);   // oc = o * C + K
        const int o = (int)(oc / C);
        const GLOBAL float *src = gp(P.psi) + (oc * 8 + d) * A * G + g;
        const GLOBAL float *w = gp(P.w) + o * A;
        float s = 0.f, c = 0.f;
        // eight directions' loads in flight at a time, summed in direction order
        for (int a0 = 0; a0 < A; a0 += 8) {
            float v[8], wv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int a = min(a0 + j, (int)A - 1);
                v[j] = src[(size_t)a * G];
                wv[j] = w[a];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (a0 + j >= A) break;
                float u, e;
                two_sum(s, wv[j] * v[j], u, e);
                s = u;
                c += e;
            }
        }
        const size_t e = ((size_t)oc * G + g) * 8 + d;
        gp(P.slot)[e] = s;
        gp(P.slotc)[e] = c;
    }
}

unsigned grid_of(long long n, unsigned bs) {
    const long long g = (n + bs - 1) / bs;
    return (unsigned)std::max(1LL, std::min(g, 65535LL * 16));
}

}  // namespace

hipError_t launch_lag_snapshot(const DirDev &D, const DevProblem *probs, int G, const int *stop, hipStream_t s) {
    if (D.nlag == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lag_snapshot, dim3(grid_of(D.nlag * 4 * G, 256)), dim3(256), 0, s, D, probs, stop);
    return hipGetLastError();
}

hipError_t launch_sweep_dir_level(const DirDev &D, const DevProblem *probs, int threads, long long begin,
                                  long long end, const int *stop, hipStream_t s) {
    (void)threads;   // one wave per block
    if (end <= begin) return hipSuccess;
    const int upw = D.G <= kDirThreads ? std::min(kMaxUnits, kDirThreads / D.G) : 1;
    const size_t lds = sizeof(float) * (size_t)upw * kUnitFloats;
    const dim3 grid((unsigned)((end - begin + upw - 1) / upw), (unsigned)((D.G + kDirThreads - 1) / kDirThreads));
    hipLaunchKernelGGL(k_sweep_dir, grid, dim3(kDirThreads), lds, s, D, probs, begin, end, upw, stop);
    return hipGetLastError();
}

hipError_t launch_unit_sweep(const DirDev &D, const DevProblem *probs, unsigned *abortp, unsigned long long watchdog,
                             const int *stop, bool phase_stats, hipStream_t s) {
    hipLaunchKernelGGL(k_unit_prologue, dim3(1), dim3(256), 0, s, D, stop);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int upw = std::min(kMaxUnits, kDirThreads / D.G);
    const size_t lds = sizeof(float) * (size_t)upw * kUnitFloats;
    // resident waves for this (device, upw): queried once
    static thread_local int c_dev = -1, c_upw = -1, c_grid = 0;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if (dev != c_dev || upw != c_upw) {
        int cus = 0, per = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_units, kDirThreads, lds)) != hipSuccess)
            return e;
        c_dev = dev;
        c_upw = upw;
        c_grid = std::max(1, per * cus);
    }
    // every wave resident at once (not needed for progress: a wave that waits
    // for a queue slot holds no unit)
    const unsigned grid = (unsigned)c_grid;
    hipLaunchKernelGGL(k_sweep_units, dim3(grid), dim3(kDirThreads), lds, s, D, probs, upw, abortp, watchdog, stop,
                       phase_stats ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_dir_slots(const DevProblem *probs, int C, int G, const int *stop, hipStream_t s) {
    hipLaunchKernelGGL(k_dir_slots, dim3(grid_of(64LL * C * G, 256)), dim3(256), 0, s, probs, stop);
    return hipGetLastError();
}

}  // namespace snx
