// Persistent, dependency-driven S_N sweep on gfx950.
//
// The paper's many-task sweep (Section 3, Algorithm 1) starts one task per
// direction at the first element; a task solves its element for all groups
// and then generates the task of every downwind neighbour for which it was the
// last upwind dependency, found with per-element atomic counters; work-first
// generation runs the new task on the generating thread unless another thread
// steals it from that thread's queue.
//
// On the GPU a task is one (cell, octant) pair of one problem: every angle of
// the octant and every group of the cell is solved by one workgroup, one
// (angle, group) system per lane.  One designation serves all angles of an
// octant, so the cell's task covers the whole octant.  When a task completes
// the last dependency of downwind cells, its workgroup runs one of them next
// (work-first continuation) and pushes the others to a device queue; idle
// workgroups pop queue slots in order and wait for the slot to be filled.
//
// Per lane (angle n, group g) the upwind DG system of the cell is
//   A = sum_a Om_a S^a + sigma_t M - sum_{f in} Om.F_f       (8x8)
//   b = r_g - sum_{f in} (Om.F_f) psi_up_f,   r_g = M (Q + sigma_s phi) / (4 pi)
// assembled from a per-angle operator B_n = sum_a Om_a S^a - sum_in Om.F_f built
// once per task in LDS, and solved by unpivoted LU in registers, row by row.
//
// Hand-off across CUs and XCDs: psi is stored with agent-coherent (sc1)
// stores and read with agent-coherent loads; every wave waits for its stores
// to complete (vmcnt(0)) before the workgroup increments downstream counters.
// Everything else is read-only during the kernel and stays cacheable.
//
// The angle reduction phi = sum_n w_n psi_n (Eq. 2) is done in the task: each
// round's weighted solutions are staged in LDS and added in increasing angle
// order with a compensated (TwoSum) sum per (group, dof); the per-octant
// partial and its compensation go to the octant's slot.  The order is fixed,
// so results do not depend on the schedule.
#include "snx_internal.h"

namespace snx {
namespace {

#ifndef WAVES_ONE
#define WAVES_ONE 5
#endif

// Global address space: loads and stores through these pointers compile to
// global_* instructions instead of flat ones (device pass only).
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#else
#define GLOBAL
#endif

template <typename T>
__device__ __forceinline__ GLOBAL T *gp(T *p) { return (GLOBAL T *)p; }

__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Workgroup barrier ordering LDS accesses only.  Unlike __syncthreads it does
// not wait for the wave's global loads and stores, so psi stores and upwind
// trace requests stay in flight across it (LDS-destined loads still land
// before it).  Every hand-off through global memory in the sweep waits for its
// stores explicitly (wait_stores).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// Workgroup barrier for data written to LDS by ordinary LDS stores only: it
// waits for the wave's LDS operations, not for its LDS-destined loads (each
// wave waits for the ones whose data it reads) nor its global accesses.
__device__ __forceinline__ void lds_store_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// face f = 2*axis + side: face-local vertex k -> cell-local vertex
__device__ __forceinline__ int face_vertex(int f, int k) {
    const int axis = f >> 1, side = f & 1;
    if (axis == 0) return (k << 1) | side;
    if (axis == 1) return (k & 1) | (side << 1) | ((k >> 1) << 2);
    return (side << 2) | k;
}
// b[vertices of face F] -= t (face-local order)
template <int F>
__device__ __forceinline__ void sub_face(float (&b)[8], const float (&t)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) b[face_vertex(F, k)] -= t[k];
}
// The same for a wave-uniform face: one scalar branch, static register indices.
// The distinct empty asm statements keep the compiler from merging the cases
// into one update at a computed index, which would move b to scratch memory.
__device__ __forceinline__ void sub_face(int f, float (&b)[8], const float (&t)[4]) {
    switch (f) {
    case 0: sub_face<0>(b, t); asm volatile("; face 0"); break;
    case 1: sub_face<1>(b, t); asm volatile("; face 1"); break;
    case 2: sub_face<2>(b, t); asm volatile("; face 2"); break;
    case 3: sub_face<3>(b, t); asm volatile("; face 3"); break;
    case 4: sub_face<4>(b, t); asm volatile("; face 4"); break;
    default: sub_face<5>(b, t); asm volatile("; face 5"); break;
    }
}
// t = C u for a 4x4 face operator stored by rows in LDS
__device__ __forceinline__ void face_apply(const float *C, const float (&u)[4], float (&t)[4]) {
    const float4 *c = reinterpret_cast<const float4 *>(C);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 ck = c[k];
        t[k] = __builtin_fmaf(ck.w, u[3], __builtin_fmaf(ck.z, u[2], __builtin_fmaf(ck.y, u[1], ck.x * u[0])));
    }
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// floor(a / b) for 0 <= a < 2^20 and b >= 1 from inv_b ~ 1 / b (within a few ulp):
// (a + 0.5) / b lies at least 0.5 / b away from an integer, far more than the
// relative error of inv_b and of the product.
__device__ __forceinline__ int div_small(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

__device__ __forceinline__ int find_problem(const long long *__restrict__ base, int nprob, long long task) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= task) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The per-lane inputs of one (angle, group) system: source dofs, sigma_t, the
// boundary inflow and the upwind traces of every inflow face (mask-predicated,
// one slot per face).
struct LaneIn {
    float r[8];
    float sig;
    float psib;
    float up[6][4];
};

// sigma_t and boundary inflow of lane (n, g) of cell K (requested early: the
// values are used only at the solve).
__device__ __forceinline__ void load_sig(const DevProblem &P, int K, int g, LaneIn &L) {
    L.sig = gp(P.sigt)[(size_t)K * P.G + g];
    L.psib = P.psib ? gp(P.psib)[g] : 0.f;
}
// Source dofs, sigma_t and boundary inflow of lane (n, g) of cell K: no
// dependence on other tasks.
__device__ __forceinline__ void load_own(const DevProblem &P, int K, int g, LaneIn &L) {
    const GLOBAL float4 *rv = reinterpret_cast<const GLOBAL float4 *>(gp(P.r) + ((size_t)K * P.G + g) * 8);
    const float4 r0 = rv[0], r1 = rv[1];
    L.r[0] = r0.x; L.r[1] = r0.y; L.r[2] = r0.z; L.r[3] = r0.w;
    L.r[4] = r1.x; L.r[5] = r1.y; L.r[6] = r1.z; L.r[7] = r1.w;
    load_sig(P, K, g, L);
}

// psi of one (octant, cell) is [dof][angle][group]: lane p = n*G + g of a task
// finds dof d at float d*A*G + p.  Each cell's block is addressed through a
// buffer resource (base and size in scalar registers), so a lane's address is
// the 32-bit byte offset 4p and the dof offset is a scalar: no per-lane 64-bit
// address arithmetic.  kCoherentAccess is the sc1 cache policy of agent-scope
// accesses, so hand-offs between CUs and XCDs see each other's values.
constexpr int kCoherentAccess = 16;
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t cell_block(const float *psi_o, int cell, int cell_floats) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(psi_o) + (size_t)cell * cell_floats, (short)0,
                                             cell_floats * 4, kRawBufferWord3);
}

// Upwind traces of lane p on every inflow face; nb / pm are the task's (uniform)
// neighbour ids and node permutations, so all loads issue at once.  A boundary
// face reads dof 0 of cell K instead (any valid address); its value is replaced
// by the inflow psi_b where the traces are used.
__device__ __forceinline__ void load_up(int K, int mask, const int (&nb)[6], const unsigned (&pm)[6], int p,
                                        int AG, const float *psi_o, LaneIn &L) {
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!((mask >> f) & 1)) continue;
        const int N = nb[f] >= 0 ? nb[f] : K;
        const unsigned perm = nb[f] >= 0 ? pm[f] : 0u;
        const __amdgpu_buffer_rsrc_t rs = cell_block(psi_o, N, 8 * AG);
#pragma unroll
        for (int l = 0; l < 4; ++l)
            L.up[f][l] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                rs, 4 * p, (int)((perm >> (8 * l)) & 0xff) * AG * 4, kCoherentAccess));
    }
}

// Issues the upwind-trace loads of lane p for up to three inflow faces: the
// lowest set bits of `faces`.  Returns the faces taken; bit j of `bnd` marks a
// boundary slot (its loads read dof 0 of cell K, any valid address, and its
// value is replaced by psi_b where the traces are used).  desc holds the task's
// neighbour ids [6] and node permutations [6].
__device__ __forceinline__ int load_slots(int faces, int K, int p, int AG, const float *psi_o, const int *desc,
                                          float (&u)[3][4], int &bnd) {
    int m = faces, taken = 0;
    bnd = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const bool live = m != 0;
        const int f = live ? __builtin_ctz(m) : 0;
        m &= m - 1;
        const int Nf = live ? __builtin_amdgcn_readfirstlane(desc[f]) : -1;
        taken |= live ? 1 << f : 0;
        bnd |= Nf < 0 ? 1 << j : 0;
        const unsigned perm = Nf >= 0 ? (unsigned)__builtin_amdgcn_readfirstlane(desc[6 + f]) : 0u;
        const __amdgpu_buffer_rsrc_t rs = cell_block(psi_o, Nf >= 0 ? Nf : K, 8 * AG);
#pragma unroll
        for (int l = 0; l < 4; ++l)
            u[j][l] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                rs, 4 * p, (int)((perm >> (8 * l)) & 0xff) * AG * 4, kCoherentAccess));
    }
    return taken;
}

// Hardware id of the XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ int xcc_id() {
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & (kMaxXcc - 1);   // HW_REG_XCC_ID[3:0]
}

__device__ __forceinline__ unsigned ld_agent_u32(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pops the next slot of queue q and waits for it.  A workgroup whose queue has
// no task left moves on to the next queue (stealing); -1 when every queue is
// done or on abort.
__device__ long long pop_task(SweepCtl *ctl, unsigned long long *queue, int &q, int nq, unsigned epoch,
                              unsigned long long watchdog, unsigned long long &polls) {
    for (int tried = 0; tried < nq; ++tried, q = q + 1 < nq ? q + 1 : 0) {
        QueueCtl *Q = &ctl->q[q];
        const long long qt = ctl->qtotal[q];
        // take a slot at once (the finished-queue test below runs while waiting,
        // so the common case costs one atomic and one load)
        const unsigned slot = atomicAdd(&Q->head, 1u);
        const GLOBAL unsigned long long *qs = gp(queue) + ctl->qbase[q];
        const unsigned long long t0 = wall_clock64();
        int backoff = 1;
        for (unsigned k = 1;; ++k) {
            if ((long long)slot < qt) {
                const unsigned long long v = __hip_atomic_load(qs + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)(v >> 32) == epoch) return (long long)(v & 0xffffffffull);
            }
            if ((k & 7) == 0) {
                if ((long long)ld_agent_u32(&Q->done) >= qt) break;        // this queue is finished
                if (ld_agent_u32(&ctl->abort)) return -1;
            }
            ++polls;
            if (wall_clock64() - t0 > watchdog) {
                __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return -1;
            }
            for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(1);
            backoff = backoff < 8 ? 2 * backoff : 8;
        }
    }
    return -1;
}

// LDS layout (floats): stage buffers [ONE ? 2 : 1][stage_floats] (M, T of the
// octant, the face matrices, the task record, ONE: source dofs), om[A][4],
// Bop[A][64], Cop[A][maxin][16], multi-round wpsi[2][NT][8], red_s[G][8],
// red_c[G][8]; ONE: a static trace array [12][NT] that also takes wpsi.
// ONE: every problem of the launch has A*G <= NT, so a task is one round of
// lanes; nothing is prefetched for a next round, the upwind traces go to the
// static LDS array and wpsi reuses it, which lowers the register and LDS
// footprint and lets more workgroups be resident.
//
// BSP: the bulk-synchronous comparator of the paper (§2.1): the launch runs the
// tasks bsp_tasks[bsp_begin, bsp_end) of one level (of every octant and problem)
// with a grid-stride loop, and the next level is the next launch; no counters,
// queues or continuation.  Task bodies are the same code, so results are the
// same bits.  stops (nullable) marks converged problems of a batch.
//
// EXT: the variant for the optional physics of a problem: per-direction
// upwinding (lagged faces), reflective planes and anisotropic moments.  Each
// part is guarded by its own array being present, so the variant also runs
// plain problems of a mixed batch; without EXT none of its code is compiled.
template <int NT, bool ONE, bool BSP, bool EXT, int DEPTH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(ONE ? WAVES_ONE : 4))) void k_sweep(
    const DevProblem *__restrict__ probs, int nprob, const long long *__restrict__ task_base,
    SweepCtl *__restrict__ ctl, unsigned long long *__restrict__ queue, int maxA, int maxG, int maxin,
    unsigned long long watchdog, const long long *__restrict__ bsp_tasks, long long bsp_begin, long long bsp_end,
    const int *__restrict__ stops, int phase_stats) {
    constexpr int depth = DEPTH;
    extern __shared__ __align__(16) float lds[];
    __shared__ long long s_task;
    __shared__ int s_q;
    __shared__ int s_nready;
    __shared__ long long s_ready[6];
    __shared__ int s_rface[6];            // face of this task across which s_ready[i] lies
    __shared__ int s_npush, s_qpush;      // ready tasks s_ready[1..s_npush] still to be queued
    if (!BSP && ctl->nactive == 0) return;
    const unsigned epoch = ctl->epoch;
    const int nq = ctl->nq;
    const int tid = threadIdx.x;
    const bool ph0 = phase_stats && tid == 0;   // thread 0 keeps the phase clock (optional: it costs issue slots)
    // Per-(group, dof) work (partial sums, slots) starts at the second wave, so
    // the first wave, which also publishes to the downwind counters, carries the
    // least of it.
    const int rt = tid >= 64 ? tid - 64 : tid + NT - 64;
    int q = ctl->xcc_queue[xcc_id()];       // home queue: the one of this XCD

    // Stage buffers (stage_floats each): cell data, task record (own and
    // downwind descriptors, see kRecWords) and, ONE, source dofs.  ONE has two:
    // a task stages into buffer cur, and a continuation reads its descriptor from
    // the last task's record in the other buffer while its own is being loaded.
    const int SB = stage_floats(ONE, maxG);
    float *sOm = lds + stage_buffers(ONE) * SB;   // [maxA][4]: omega xyz, weight
    float *sB = sOm + 4 * maxA;           // [maxA][64]
    float *sC = sB + 64 * maxA;           // [maxA][maxin][16]
    float *sW = sC + 16 * maxin * maxA;   // multi-round: [2][NT][8] weighted psi
    float *sRs = sW + (ONE ? 0 : 16) * NT; // [maxG][8]
    float *sRc = sRs + 8 * maxG;          // [maxG][8]
    // ONE: [3 slots][4 face nodes][NT] upwind traces, filled by LDS-destined loads.
    // A separate LDS object: reads of the other LDS data then need not wait for
    // these loads to land.  Its first 8 rows then take the weighted psi, [8][NT]:
    // each lane overwrites only its own column, after its own trace reads.
    __shared__ __align__(16) float s_up[ONE ? 12 * NT : 4];
    float *sUp = s_up;

    // Workgroup statistics, kept in LDS and touched by thread 0 only: polls, tasks,
    // continued tasks, tasks not yet added to the queue's done count, and (when
    // phase_stats is set) the shader-clock cycles of the five phases of a task.
    __shared__ unsigned long long s_stat[4], s_ph[5], s_mark;
    if (tid == 0) {
        for (int i = 0; i < 4; ++i) s_stat[i] = 0;
        for (int i = 0; i < 5; ++i) s_ph[i] = 0;
        s_npush = 0;
    }
    // Queues the ready tasks the last task did not continue with: one atomic
    // reserves their slots.  One thread runs it during the next task (ONE: the
    // last wave's first lane after the operator build, else thread 0 while the
    // stage loads are in flight), so the round trip overlaps other work.
    auto push_ready = [&]() {
        const int np = s_npush;
        if (np <= 0) return;
        const int qo = s_qpush;
        const unsigned slot0 = atomicAdd(&ctl->q[qo].tail, (unsigned)np);
        for (int i = 0; i < np; ++i) {
            const unsigned long long v = ((unsigned long long)epoch << 32) | (unsigned long long)s_ready[1 + i];
            if ((long long)(slot0 + i) < ctl->qtotal[qo])
                __hip_atomic_store(gp(queue) + ctl->qbase[qo] + slot0 + i, v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            else   // more pushes than tasks: counters inconsistent with the DAG
                __hip_atomic_store(&ctl->abort, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_npush = 0;
    };
    long long cont = -1;
    long long bsp_i = bsp_begin + blockIdx.x;
    int cur = 0;                          // stage buffer of the current task
    int cface = -1, cbuf = 0;             // continuation: its face in the last task's record, and that record's buffer
    for (;;) {
        long long task = cont;
        if (ph0) s_mark = clock64();
        if constexpr (BSP) {
            if (bsp_i >= bsp_end) break;
            task = bsp_tasks[bsp_i];
            bsp_i += gridDim.x;
            if (stops && stops[uni(find_problem(task_base, nprob, task))]) continue;
        } else if (task < 0) {
            if (tid == 0) {
                if (s_stat[3]) {
                    __hip_atomic_fetch_add(&ctl->q[q].done, (unsigned)s_stat[3], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    s_stat[3] = 0;
                }
                unsigned long long polls = 0;
                s_task = pop_task(ctl, queue, q, nq, epoch, watchdog, polls);
                s_stat[0] += polls;
                s_q = q;
                if (phase_stats) {
                    const unsigned long long t = clock64();
                    s_ph[0] += t - s_mark;
                    s_mark = t;
                }
            }
            lds_barrier();
            task = s_task;
            q = s_q;
            if (task < 0) break;
        } else if (tid == 0) {
            ++s_stat[2];
        }

        // ---------------------------------------------------------- decode
        const int p = uni(find_problem(task_base, nprob, task));
        const DevProblem &P = probs[p];
        const int C = P.C, G = P.G, A = P.A;
        const unsigned epoch_p = *gp(P.epoch);        // the problem's sweep count: counter targets are indeg x epoch
        const long long local = task - P.task_base;
        const int o = uni((int)(local & 7));                 // task = 8 * cell + octant
        const int K = uni((int)(local >> 3));
        const int AG = A * G;
        const float invG = __builtin_amdgcn_rcpf((float)G);
        const int ln = div_small(tid, invG), lg = tid - ln * G;  // (angle, group) of this lane in the first round
        const size_t cell_psi = (size_t)8 * A * G;          // floats per (octant, cell)
        const float *psi_o = P.psi + (size_t)o * C * cell_psi;

        // --------------------------------------------- early upwind loads
        // A continuation already holds its descriptor (the last task's record), so
        // its first three inflow faces' traces are requested now, straight into
        // LDS (buffer loads with an LDS destination, one 64-lane run per wave),
        // together with the stage loads below; other tasks request them as soon
        // as their record is in LDS.
        int taken0 = 0, bnd0 = 0;
        auto early_up = [&](const int *d) {
            int m = uni(d[12]);
            const int wbase = uni(tid & ~63);
#pragma unroll 1
            for (int j = 0; j < 3 && m; ++j) {
                const int f = __builtin_ctz(m);
                m &= m - 1;
                taken0 |= 1 << f;
                const int Nf = uni(d[f]);
                bnd0 |= Nf < 0 ? 1 << j : 0;
                const unsigned perm = Nf >= 0 ? (unsigned)uni(d[6 + f]) : 0u;
                const __amdgpu_buffer_rsrc_t rs = cell_block(psi_o, Nf >= 0 ? Nf : K, 8 * AG);
                if (wbase < AG) {
#pragma unroll
                    for (int l = 0; l < 4; ++l)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(
                            rs, (__attribute__((address_space(3))) void *)(sUp + (j * 4 + l) * NT + wbase), 4,
                            4 * tid, (int)((perm >> (8 * l)) & 0xff) * AG * 4, 0, kCoherentAccess);
                }
            }
        };

        // ---------------------------------------------------------- stage
        // One round trip brings the cell data (M, T^a of this octant, the six
        // face matrices; 136 float4s) and the task record (24 int4s) to LDS, the
        // directions, and each lane's sigma_t; one-round tasks also stage the
        // cell's source dofs of every group (2 float4s per group).
        constexpr int kGeo = 16 + 48 + 72, kItems = kGeo + kRecWords / 4;
        float *const stg = lds + (ONE ? cur : 0) * SB;
        float *const sM = stg;                // M, then T^x, T^y, T^z of this (cell, octant),
        float *const sT = sM + 64;            // then the six face matrices F^x, F^y, F^z (48 each)
        float *const sF = sT + 192;
        int *const s_desc = reinterpret_cast<int *>(stg + 4 * kGeo);   // words 0..12: this task's descriptor
        const float *const sR = stg + 4 * kItems;                     // ONE: [G][8] source dofs
        const int *const prev_rec = reinterpret_cast<const int *>(lds + (ONE ? cbuf : 0) * SB + 4 * kGeo);
        float4 om4 = make_float4(0.f, 0.f, 0.f, 0.f);          // direction and weight of angle tid (A <= 64 <= NT)
        LaneIn L;
        // a continuation is in the same problem and octant: its directions are in LDS
        const bool new_om = !ONE || cface < 0;
        // per-angle designation: every wave holds the per-direction inflow masks
        // of this (octant, cell), lane a those of direction a (A <= 64)
        int amv = 0;
        if constexpr (EXT)
            if (P.amask && (tid & 63) < A) amv = gp(P.amask)[((size_t)o * C + K) * A + (tid & 63)];
        if (new_om && tid < A) {
            const int n = o * A + tid;
            om4 = make_float4(gp(P.omega)[3 * n + 0], gp(P.omega)[3 * n + 1], gp(P.omega)[3 * n + 2], gp(P.w)[n]);
        }
        // ONE: 16-byte LDS-destined loads of the stage items of cell Kc (octant o)
        // into buffer dst, 64-lane blocks first, first + step, ... (one block per
        // wave and step); no registers are held for the staged data
        auto stage_dma = [&](int Kc, float *dst, int first, int step) {
            const int nitems = kItems + 2 * G;
            const GLOBAL float *srcM = gp(P.M) + (size_t)Kc * 64;
            const GLOBAL float *srcT = gp(P.T) + ((size_t)o * C + Kc) * 192;
            const GLOBAL float *srcF = gp(P.F) + (size_t)Kc * 288;
            const GLOBAL float *srcRec =
                reinterpret_cast<const GLOBAL float *>(gp(P.rec) + ((size_t)o * C + Kc) * kRecWords);
            const GLOBAL float *srcR = gp(P.r) + (size_t)Kc * G * 8;
            for (int i0 = first; i0 < nitems; i0 += step) {
                const int i = i0 + (tid & 63);
                if (i < nitems) {
                    // the item's array and offset, picked by selects (no divergent branches)
                    unsigned long long a = (unsigned long long)srcM + 16ull * i;
                    a = i >= 16 ? (unsigned long long)srcT + 16ull * (i - 16) : a;
                    a = i >= 64 ? (unsigned long long)srcF + 16ull * (i - 64) : a;
                    a = i >= kGeo ? (unsigned long long)srcRec + 16ull * (i - kGeo) : a;
                    a = i >= kItems ? (unsigned long long)srcR + 16ull * (i - kItems) : a;
                    __builtin_amdgcn_global_load_lds((const void *)a,
                                                     (__attribute__((address_space(3))) void *)(dst + 4 * i0), 16, 0, 0);
                }
            }
        };
        if constexpr (ONE) {
            stage_dma(K, stg, uni(tid & ~63), NT);
            if (tid < AG) load_sig(P, K, lg, L);
            // a continuation's trace requests go after the stage loads (staging
            // depth 1: one round trip brings the cell data and the traces)
            if (cface >= 0 && depth > 0) early_up(prev_rec + 16 + 13 * cface);
        } else {
            auto stage_item = [&](int i) -> float4 {
                if (i < 16) return reinterpret_cast<const GLOBAL float4 *>(gp(P.M) + (size_t)K * 64)[i];
                if (i < 64) return reinterpret_cast<const GLOBAL float4 *>(gp(P.T) + ((size_t)o * C + K) * 192)[i - 16];
                if (i < kGeo) return reinterpret_cast<const GLOBAL float4 *>(gp(P.F) + (size_t)K * 288)[i - 64];
                return reinterpret_cast<const GLOBAL float4 *>(gp(P.rec) + ((size_t)o * C + K) * kRecWords)[i - kGeo];
            };
            if constexpr (NT >= kItems) {
                // at most one item per thread: all loads in flight together
                const float4 st = tid < kItems ? stage_item(tid) : make_float4(0.f, 0.f, 0.f, 0.f);
                if (tid < AG) load_own(P, K, lg, L);
                if (tid == 0) push_ready();                        // overlaps the loads above
                if (tid < kItems) reinterpret_cast<float4 *>(stg)[tid] = st;
            } else {
                if (tid < AG) load_own(P, K, lg, L);
                if (tid == 0) push_ready();
                for (int i = tid; i < kItems; i += NT) reinterpret_cast<float4 *>(stg)[i] = stage_item(i);
            }
        }
        if (new_om && tid < A) reinterpret_cast<float4 *>(sOm)[tid] = om4;
        for (int i = rt; i < G * 8; i += NT) { sRs[i] = 0.f; sRc[i] = 0.f; }
        lds_barrier();                // the staged data come from LDS-destined loads of every wave
        if (tid == 0) s_nready = 0;   // after the barrier: every thread has read the last task's count
        if constexpr (ONE)
            if (cface < 0 || depth == 0) early_up(s_desc);
        const int mask = uni(s_desc[12]);
        const int nin = __popc(mask);
        // faces where some direction's designation differs from the octant's
        const int lagm = EXT && P.amask ? uni((s_desc[13] >> 18) & 63) : 0;
        // faces on reflective planes and the first reflective slot of the cell
        const int rmask = EXT && P.refl_in ? uni((s_desc[13] >> 24) & 63) : 0;
        const int rbase = rmask ? uni(s_desc[14]) : 0;
        // Reflective plane: the inflow of a direction is its mirror image's outflow
        // at the same nodes, from the previous sweep.  The mirror image lies in the
        // octant o ^ (1 << axis) at the same index within its octant (the
        // quadrature's symmetry, checked at set-up), so lane p reads lane p of
        // that octant's record of the face.
        auto refl_row = [&](int f, float *base) {
            const int slot = rbase + __popc(rmask & ((1 << f) - 1));
            return base + (size_t)(((o ^ (1 << (f >> 1))) * P.nref + slot) * 4) * AG;
        };
        auto refl_own = [&](int f, float *base) {
            const int slot = rbase + __popc(rmask & ((1 << f) - 1));
            return base + (size_t)((o * P.nref + slot) * 4) * AG;
        };
        int nb[6];
        unsigned pm[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            nb[f] = uni(s_desc[f]);
            pm[f] = (unsigned)uni(s_desc[6 + f]);
        }
        // multi-round tasks: the first round's upwind traces are in flight during
        // the operator build; one-round tasks issue them after it, which keeps
        // their registers free while the operators are built
        if constexpr (!ONE)
            if (tid < AG) load_up(K, mask, nb, pm, tid, AG, psi_o, L);
        if (ph0) { const unsigned long long t = clock64(); s_ph[1] += t - s_mark; s_mark = t; }

        // ------------------------------------- per-angle operators B_n, C_n,f
        {   // Angles are dealt to waves (wave-uniform loop), entries to lanes: lane l
            // owns entry l of B (8x8) and entry l & 15 of the inflow operator of slot
            // l >> 4, so its three operator values are read once and each angle costs
            // one broadcast direction read, three FMAs per operator and the writes.
            const int lane = tid & 63, wv = uni(tid >> 6);
            constexpr int kWaves = NT / 64;
            const float bx = sT[lane], by = sT[64 + lane], bz = sT[128 + lane];
            auto slot_coef = [&](int s, float &cx, float &cy, float &cz) {
                int m = mask;                                   // face of inflow slot s: s-th set bit of mask
                for (int k = 0; k < s; ++k) m &= m - 1;
                const float *Fs = sF + (m ? __ffs(m) - 1 : 0) * 48;
                const int kl = lane & 15;
                cx = Fs[kl]; cy = Fs[16 + kl]; cz = Fs[32 + kl];
            };
            const int s0 = lane >> 4;                           // slots 0..3
            float cx, cy, cz;
            slot_coef(s0, cx, cy, cz);
            const bool c0 = s0 < nin;
            const float4 *om4s = reinterpret_cast<const float4 *>(sOm);
            auto put = [&](int n, float4 om) {
                sB[n * 64 + lane] = om.x * bx + om.y * by + om.z * bz;
                if (c0) sC[(n * maxin + s0) * 16 + (lane & 15)] = om.x * cx + om.y * cy + om.z * cz;
            };
            int n = wv;
            for (; n + kWaves < A; n += 2 * kWaves) {          // two angles' reads in flight together
                const float4 oa = om4s[n], ob = om4s[n + kWaves];
                put(n, oa);
                put(n + kWaves, ob);
            }
            if (n < A) put(n, om4s[n]);
            if (nin > 4) {                                      // slots 4, 5 (rare)
                const int s1 = 4 + s0;
                slot_coef(s1, cx, cy, cz);
                for (int n = wv; n < A; n += kWaves) {
                    const float4 om = reinterpret_cast<const float4 *>(sOm)[n];
                    if (s1 < nin) sC[(n * maxin + s1) * 16 + (lane & 15)] = om.x * cx + om.y * cy + om.z * cz;
                }
            }
            if (EXT && lagm) {
                // Per-angle designation: direction n's operator is
                // B_n = Om.S - sum over its own inflow faces of Om.F_f, so each face
                // where its designation differs from the octant's adds Om.F_f
                // (inflow for the octant only) or subtracts it (inflow for the
                // direction only), and the inflow slot of an octant-inflow face
                // that is outflow for the direction is cleared.  Each lane updates
                // the entries it wrote above, so no barrier is needed.
                auto slot_face = [&](int s) {
                    int m = mask;
                    for (int k = 0; k < s; ++k) m &= m - 1;
                    return m ? __ffs(m) - 1 : -1;
                };
                const int fs0 = s0 < nin ? slot_face(s0) : -1;
                const int fs1 = 4 + s0 < nin ? slot_face(4 + s0) : -1;
                const int i = lane >> 3, j = lane & 7;
                for (int n = wv; n < A; n += kWaves) {
                    const int dif = __builtin_amdgcn_readlane(amv, n) ^ mask;
                    if (!dif) continue;
                    const float4 om = om4s[n];
                    float dB = 0.f;
                    for (int m = dif; m; m &= m - 1) {
                        const int f = __builtin_ctz(m), axis = f >> 1, side = f & 1;
                        if (((i >> axis) & 1) == side && ((j >> axis) & 1) == side) {
                            const int ki = axis == 0 ? i >> 1 : (axis == 1 ? (i & 1) | ((i >> 2) << 1) : i & 3);
                            const int kj = axis == 0 ? j >> 1 : (axis == 1 ? (j & 1) | ((j >> 2) << 1) : j & 3);
                            const float *Ff = sF + 48 * f + 4 * ki + kj;
                            const float c = om.x * Ff[0] + om.y * Ff[16] + om.z * Ff[32];
                            dB += (mask >> f) & 1 ? c : -c;
                        }
                    }
                    sB[n * 64 + lane] += dB;
                    const int gone = dif & mask;
                    if (fs0 >= 0 && ((gone >> fs0) & 1)) sC[(n * maxin + s0) * 16 + (lane & 15)] = 0.f;
                    if (fs1 >= 0 && ((gone >> fs1) & 1)) sC[(n * maxin + 4 + s0) * 16 + (lane & 15)] = 0.f;
                }
            }
        }
        // only LDS stores cross this barrier: LDS-destined trace loads are read by
        // the wave that issued them, after its own wait
        lds_store_barrier();
        // one-round tasks: the last wave queues the last task's other ready tasks
        // while the lanes solve (it is idle there when A*G <= NT - 64)
        if constexpr (ONE)
            if (tid == NT - 64) push_ready();
        if (ph0) { const unsigned long long t = clock64(); s_ph[2] += t - s_mark; s_mark = t; }

        // ------------------------------------------------ rounds of lanes
        int buf = 0;
        for (int base = 0; ONE ? base == 0 : base < AG; base += NT, buf ^= 1) {
            const int pi = base + tid;
            // The task's inflow mask and neighbour ids, kept opaque to the compiler
            // in each round: the per-face tests made on them (inflow face, boundary
            // face) are then scalar instructions at their use, not 64-bit lane masks
            // computed once per task and held across the round loop, which ran out
            // of scalar registers (spilled to vector-register lanes and reloaded by
            // v_readlane in every round).
            int fmask = mask;
            int fnb[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) fnb[f] = nb[f];
            asm volatile("" : "+s"(fmask), "+s"(fnb[0]), "+s"(fnb[1]), "+s"(fnb[2]), "+s"(fnb[3]), "+s"(fnb[4]),
                         "+s"(fnb[5]));
            float *sWb = ONE ? sUp : sW + buf * NT * 8;   // dof d of lane l: ONE d*NT + l, else 8l + d
            if (pi < AG) {
                const int n = ONE ? ln : div_small(pi, invG), g = ONE ? lg : pi - n * G;
                if constexpr (!ONE)
                    if (depth == 0 && base > 0) {
                        load_own(P, K, g, L);
                        load_up(K, fmask, fnb, pm, pi, AG, psi_o, L);
                    }
                float b[8];
                if constexpr (ONE) {
                    const float4 r0 = reinterpret_cast<const float4 *>(sR + 8 * g)[0];
                    const float4 r1 = reinterpret_cast<const float4 *>(sR + 8 * g)[1];
                    b[0] = r0.x; b[1] = r0.y; b[2] = r0.z; b[3] = r0.w;
                    b[4] = r1.x; b[5] = r1.y; b[6] = r1.z; b[7] = r1.w;
                } else {
#pragma unroll
                    for (int d = 0; d < 8; ++d) b[d] = L.r[d];
                }
                if constexpr (EXT)
                    if (P.mom) {
                        // anisotropic scattering: sum over moments of degree >= 1 of
                        // Y_k(Omega_n) sigma_l M phi_lm on top of the isotropic source
                        const int nm = (P.L + 1) * (P.L + 1);
                        const float *y = P.ylm + (size_t)(o * A + n) * nm;
                        const float4 *rm = reinterpret_cast<const float4 *>(P.rmom + ((size_t)K * G + g) * nm * 8);
                        // four moments' loads in flight together
                        for (int k0 = 1; k0 < nm; k0 += 4) {
                            float yk[4];
                            float4 ra[4], rb[4];
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int k = k0 + j < nm ? k0 + j : k0;
                                yk[j] = k0 + j < nm ? y[k] : 0.f;
                                ra[j] = rm[2 * k];
                                rb[j] = rm[2 * k + 1];
                            }
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                b[0] = __builtin_fmaf(yk[j], ra[j].x, b[0]); b[1] = __builtin_fmaf(yk[j], ra[j].y, b[1]);
                                b[2] = __builtin_fmaf(yk[j], ra[j].z, b[2]); b[3] = __builtin_fmaf(yk[j], ra[j].w, b[3]);
                                b[4] = __builtin_fmaf(yk[j], rb[j].x, b[4]); b[5] = __builtin_fmaf(yk[j], rb[j].y, b[5]);
                                b[6] = __builtin_fmaf(yk[j], rb[j].z, b[6]); b[7] = __builtin_fmaf(yk[j], rb[j].w, b[7]);
                            }
                        }
                    }
                const float psib = L.psib;
                if constexpr (ONE) {
                    // Inflow faces in slot order (slot s = s-th set bit of the mask),
                    // three at a time.  The face of a slot is wave-uniform, so the
                    // node map is picked by one scalar branch per slot.  The first
                    // three arrived in LDS (requested early); hexahedra of the
                    // meshes here have three inflow faces per octant, so later groups
                    // (loaded into registers here) are rare.
                    // boundary slots (bit j of bnd) take the inflow psi_b; interior
                    // tasks skip the selects
                    auto set_boundary = [&](float (&u)[3][4], int bnd) {
                        if (bnd) {
#pragma unroll
                            for (int j = 0; j < 3; ++j)
#pragma unroll
                                for (int l = 0; l < 4; ++l) u[j][l] = (bnd >> j) & 1 ? psib : u[j][l];
                        }
                    };
                    // reflective slots among `taken` (faces in slot order) read the mirror
                    // image's outflow of the previous sweep
                    auto reflect = [&](float (&u)[3][4], int taken) {
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            if (!taken) break;
                            const int f = __builtin_ctz(taken);
                            taken &= taken - 1;
                            if ((rmask >> f) & 1) {
                                const float *src = refl_row(f, P.refl_in);
#pragma unroll
                                for (int l = 0; l < 4; ++l) u[j][l] = src[l * AG + pi];
                            }
                        }
                    };
                    auto apply = [&](int taken, int s0, const float (&u)[3][4]) {
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            if (!taken) break;
                            const int f = __builtin_ctz(taken);
                            taken &= taken - 1;
                            float t[4];
                            face_apply(sC + (n * maxin + s0 + j) * 16, u[j], t);
                            sub_face(f, b, t);
                        }
                    };
                    {
                        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the LDS-destined loads have landed
                        float u0[3][4];
#pragma unroll
                        for (int j = 0; j < 3; ++j)
#pragma unroll
                            for (int l = 0; l < 4; ++l) u0[j][l] = sUp[(j * 4 + l) * NT + tid];
                        set_boundary(u0, bnd0);
                        if constexpr (EXT)
                            if (rmask & taken0) reflect(u0, taken0);
                        apply(taken0, 0, u0);
                    }
                    int rest = fmask & ~taken0;
                    for (int s0 = 3; rest; s0 += 3) {
                        float u[3][4];
                        int bnd = 0;
                        const int taken = load_slots(rest, K, pi, AG, psi_o, s_desc, u, bnd);
                        rest &= ~taken;
                        set_boundary(u, bnd);
                        if constexpr (EXT)
                            if (rmask & taken) reflect(u, taken);
                        apply(taken, s0, u);
                    }
                } else {
#pragma unroll
                    for (int f = 0; f < 6; ++f) {
                        if (!((fmask >> f) & 1)) continue;
                        const float *Cs = sC + (n * maxin + __popc(fmask & ((1 << f) - 1))) * 16;
                        float u[4];
#pragma unroll
                        for (int l = 0; l < 4; ++l) u[l] = fnb[f] >= 0 ? L.up[f][l] : psib;
                        if constexpr (EXT)
                            if ((rmask >> f) & 1) {
                                const float *src = refl_row(f, P.refl_in);
#pragma unroll
                                for (int l = 0; l < 4; ++l) u[l] = src[l * AG + pi];
                            }
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            float t = Cs[k * 4] * u[0];
                            t = __builtin_fmaf(Cs[k * 4 + 1], u[1], t);
                            t = __builtin_fmaf(Cs[k * 4 + 2], u[2], t);
                            t = __builtin_fmaf(Cs[k * 4 + 3], u[3], t);
                            b[face_vertex(f, k)] -= t;
                        }
                    }
                }
                if (const int lf = EXT ? lagm & ~fmask : 0) {
                    // Per-angle designation: a face that is inflow for this direction
                    // but downwind in the octant's order takes the neighbour's trace
                    // from the previous sweep (its task runs after this one, so the
                    // value is still there), or psi_b on the boundary.
                    const int mine = __builtin_amdgcn_ds_bpermute(n << 2, amv);
                    const float4 om = reinterpret_cast<const float4 *>(sOm)[n];
#pragma unroll
                    for (int f = 0; f < 6; ++f) {
                        if (!((lf >> f) & 1) || !((mine >> f) & 1)) continue;
                        float u[4];
                        if (fnb[f] >= 0) {
                            const __amdgpu_buffer_rsrc_t rs = cell_block(psi_o, fnb[f], 8 * AG);
#pragma unroll
                            for (int l = 0; l < 4; ++l)
                                u[l] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                    rs, 4 * pi, (int)((pm[f] >> (8 * l)) & 0xff) * AG * 4, kCoherentAccess));
                        } else {
#pragma unroll
                            for (int l = 0; l < 4; ++l) u[l] = psib;
                        }
                        const float *Ff = sF + 48 * f;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            float t = 0.f;
#pragma unroll
                            for (int l = 0; l < 4; ++l) {
                                const float c = om.x * Ff[4 * k + l] + om.y * Ff[16 + 4 * k + l] + om.z * Ff[32 + 4 * k + l];
                                t = __builtin_fmaf(c, u[l], t);
                            }
                            b[face_vertex(f, k)] -= t;
                        }
                    }
                }
                const float sig = L.sig;
                // the next round's inputs are in flight during this round's solve
                // (staging depth 1; at depth 0 each round loads its own at its start)
                if constexpr (!ONE) {
                    const int pn = pi + NT;
                    if (depth > 0 && pn < AG) {
                        const int nn = div_small(pn, invG), gn = pn - nn * G;
                        load_own(P, K, gn, L);
                        load_up(K, fmask, fnb, pm, pn, AG, psi_o, L);
                    }
                }

                // Unpivoted LU, one row of A = B_n + sigma_t M at a time (Doolittle by rows):
                // row i is reduced by the finished rows k < i; only the strict upper
                // triangle and the pivots stay live.
                float U[8][8], inv[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    float row[8];
                    const float4 *bp = reinterpret_cast<const float4 *>(sB + n * 64 + i * 8);
                    const float4 *mp = reinterpret_cast<const float4 *>(sM + i * 8);
                    const float4 b0 = bp[0], b1 = bp[1], m0 = mp[0], m1 = mp[1];
                    row[0] = __builtin_fmaf(sig, m0.x, b0.x); row[1] = __builtin_fmaf(sig, m0.y, b0.y);
                    row[2] = __builtin_fmaf(sig, m0.z, b0.z); row[3] = __builtin_fmaf(sig, m0.w, b0.w);
                    row[4] = __builtin_fmaf(sig, m1.x, b1.x); row[5] = __builtin_fmaf(sig, m1.y, b1.y);
                    row[6] = __builtin_fmaf(sig, m1.z, b1.z); row[7] = __builtin_fmaf(sig, m1.w, b1.w);
#pragma unroll
                    for (int k = 0; k < i; ++k) {
                        const float l = row[k] * inv[k];
#pragma unroll
                        for (int j = k + 1; j < 8; ++j) row[j] = __builtin_fmaf(-l, U[k][j], row[j]);
                        b[i] = __builtin_fmaf(-l, b[k], b[i]);
                    }
                    inv[i] = __builtin_amdgcn_rcpf(row[i]);
#pragma unroll
                    for (int j = i + 1; j < 8; ++j) U[i][j] = row[j];
                    if constexpr (ONE) __builtin_amdgcn_sched_barrier(0);   // one row's loads in flight at a time
                }
#pragma unroll
                for (int k = 7; k >= 0; --k) {
                    float t = b[k];
#pragma unroll
                    for (int j = k + 1; j < 8; ++j) t = __builtin_fmaf(-U[k][j], b[j], t);
                    b[k] = t * inv[k];
                }
                if constexpr (EXT) {
                    // reflective faces this octant leaves through: their nodal outflow
                    // for the mirror images' next sweep
                    if (const int ro = rmask & ~fmask) {
#pragma unroll
                        for (int f = 0; f < 6; ++f) {
                            if (!((ro >> f) & 1)) continue;
                            float *dst = refl_own(f, P.refl_out);
#pragma unroll
                            for (int l = 0; l < 4; ++l) dst[l * AG + pi] = b[face_vertex(f, l)];
                        }
                    }
                }
                const __amdgpu_buffer_rsrc_t rk = cell_block(psi_o, K, 8 * AG);
                const float wn = sOm[4 * n + 3];
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, b[d]), rk, 4 * pi, d * AG * 4,
                                                          kCoherentAccess);
                    sWb[ONE ? d * NT + tid : tid * 8 + d] = wn * b[d];
                }
            }
            lds_store_barrier();   // the psi stores stay in flight until the publish
            // compensated accumulation in increasing angle order, one (group, dof) per reducer;
            // the other buffer takes the next round's values meanwhile
            const int hi = min(base + NT, AG);
            const int bm = ONE ? 0 : base % G;   // group of the round's first lane (wave-uniform)
            for (int e = rt; e < G * 8; e += NT) {
                const int g = e >> 3, d = e & 7;
                float s = sRs[e], c = sRc[e];
                // first lane of group g in this round: base + (g - bm) mod G, with
                // 0 <= g, bm < G (one conditional add, no per-lane division)
                const int q0 = ONE ? g : base + (g - bm) + (g < bm ? G : 0);
                constexpr int LS = ONE ? 1 : 8;   // stride between lanes
                const float *w = sWb + (q0 - base) * LS + d * (ONE ? NT : 1);
                const int st = G * LS;            // next angle, same group
                int q = q0;
                for (; q + 3 * G < hi; q += 4 * G, w += 4 * st) {   // four angles' reads in flight together
                    const float w0 = w[0], w1 = w[st], w2 = w[2 * st], w3 = w[3 * st];
                    float t, err;
                    two_sum(s, w0, t, err); s = t; c += err;
                    two_sum(s, w1, t, err); s = t; c += err;
                    two_sum(s, w2, t, err); s = t; c += err;
                    two_sum(s, w3, t, err); s = t; c += err;
                }
                for (; q < hi; q += G, w += st) {
                    float t, err;
                    two_sum(s, w[0], t, err);
                    s = t;
                    c += err;
                }
                sRs[e] = s;
                sRc[e] = c;
            }
        }

        if (ph0) { const unsigned long long t = clock64(); s_ph[3] += t - s_mark; s_mark = t; }
        // Octant slot: the task's compensated partial sums.  Only the reduction
        // kernel reads them, so in the dependency-driven sweep they are written
        // after the downwind counters: the wait before the counters covers only ψ.
        const size_t sbase = ((size_t)o * C + K) * G * 8;
        auto write_slot = [&]() {
            for (int e = rt; e < G * 8; e += NT) {
                gp(P.slot)[sbase + e] = sRs[e];
                gp(P.slotc)[sbase + e] = sRc[e];
            }
        };

        // --------------------------------------------- publish to downwind
        if constexpr (BSP) {               // the next level is the next launch
            write_slot();
            lds_barrier();
            continue;
        }
        wait_stores();
        __syncthreads();
        if (tid < 6) {
            const int f = tid;
            const int N = ((mask >> f) & 1) ? -1 : s_desc[f];
            if (N >= 0) {
                const unsigned old = __hip_atomic_fetch_add(gp(P.cnt) + (size_t)o * C + N, 1u, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                const unsigned target = (unsigned)((s_desc[13] >> (3 * f)) & 7) * epoch_p;
                if (old + 1u == target) {
                    const int i = atomicAdd(&s_nready, 1);
                    s_ready[i] = P.task_base + 8LL * N + o;
                    s_rface[i] = f;
                }
            }
        }
        lds_barrier();
        const int nr = s_nready;
        cont = nr > 0 ? s_ready[0] : -1;
        cface = nr > 0 ? s_rface[0] : -1;            // the continuation's descriptor is in this record
        cbuf = cur;
        cur ^= 1;
        write_slot();
        if (ph0) s_ph[4] += clock64() - s_mark;
        if (tid == 0) {
            ++s_stat[3];
            ++s_stat[1];
            // downwind cells are in the same octant, hence in this task's queue; the
            // others are queued during the continuation (nr > 1 implies one)
            s_npush = nr - 1;
            s_qpush = o % nq;

        }
    }
    if (!BSP && tid == 0) {
        QueueCtl *Q = &ctl->q[ctl->xcc_queue[xcc_id()]];
        atomicAdd(&Q->polls_empty, s_stat[0]);
        atomicAdd(&Q->tasks_done, s_stat[1]);
        atomicAdd(&Q->continued, s_stat[2]);
        for (int i = 0; i < 5; ++i) atomicAdd(&Q->phase[i], s_ph[i]);
    }
}

// Starts a sweep: advances the schedule's epoch and the epoch of every active
// problem (stops[p] == 0), sizes each queue for the active problems' tasks of
// its octants and pushes their level-0 tasks (cells with no interior upwind
// face) as seeds.  One workgroup; problems and seeds are few.
__global__ void k_sweep_prologue(SweepCtl *ctl, unsigned long long *queue, const DevProblem *__restrict__ probs,
                                 int nprob, const int *__restrict__ seeds, const int *__restrict__ seed_off,
                                 const int *__restrict__ stops) {
    __shared__ long long s_tail[kMaxQueues];
    const int nq = ctl->nq;
    if (threadIdx.x == 0) {
        const unsigned e = ctl->epoch + 1u;
        int nact = 0;
        for (int q = 0; q < nq; ++q) {
            long long tot = 0, tail = 0;
            for (int o = q; o < 8; o += nq)
                for (int p = 0; p < nprob; ++p) {
                    if (stops && stops[p]) continue;
                    tot += probs[p].C;
                    for (int i = seed_off[p * 8 + o]; i < seed_off[p * 8 + o + 1]; ++i)
                        queue[ctl->qbase[q] + tail++] =
                            ((unsigned long long)e << 32) | (unsigned long long)(probs[p].task_base + seeds[i]);
                }
            ctl->qtotal[q] = tot;
            s_tail[q] = tail;
        }
        for (int p = 0; p < nprob; ++p)
            if (!(stops && stops[p])) {
                *probs[p].epoch += 1u;
                ++nact;
            }
        ctl->nactive = nact;
        ctl->epoch = e;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        QueueCtl *Q = &ctl->q[q];
        Q->head = 0;
        Q->tail = (unsigned)s_tail[q];
        Q->done = 0;
        Q->polls_empty = 0;
        Q->tasks_done = 0;
        Q->continued = 0;
        for (int i = 0; i < 5; ++i) Q->phase[i] = 0;
    }
}

// Records the XCD id each workgroup runs on (set-up probe of the device's XCDs).
__global__ void k_xcc_probe(int *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

template <int NT, bool ONE, bool BSP>
hipError_t launch_nt(const DevProblem *probs, int nprob, const long long *task_base, SweepCtl *ctl,
                     unsigned long long *queue, int maxA, int maxG, int maxin, int grid, size_t lds,
                     unsigned long long watchdog, const long long *bsp_tasks, long long b0, long long b1,
                     const int *stops, int phase_stats, int depth, bool ext, hipStream_t s) {
#define SNX_K(E, D)                                                                                                \
    hipLaunchKernelGGL((k_sweep<NT, ONE, BSP, E, D>), dim3(grid), dim3(NT), lds, s, probs, nprob, task_base, ctl, \
                       queue, maxA, maxG, maxin, watchdog, bsp_tasks, b0, b1, stops, phase_stats)
    if (ext) {
        if (depth) SNX_K(true, 1); else SNX_K(true, 0);
    } else {
        if (depth) SNX_K(false, 1); else SNX_K(false, 0);
    }
#undef SNX_K
    return hipGetLastError();
}

template <int NT, bool ONE>
const void *kernel_ptr(bool ext, int depth) {
    if (depth)
        return ext ? reinterpret_cast<const void *>(&k_sweep<NT, ONE, false, true, 1>)
                   : reinterpret_cast<const void *>(&k_sweep<NT, ONE, false, false, 1>);
    return ext ? reinterpret_cast<const void *>(&k_sweep<NT, ONE, false, true, 0>)
               : reinterpret_cast<const void *>(&k_sweep<NT, ONE, false, false, 0>);
}

}  // namespace

bool sweep_threads_valid(int threads) {
    return threads == 64 || threads == 128 || threads == 192 || threads == 256 || threads == 512;
}

size_t sweep_lds_bytes(int threads, int maxA, int maxG, int maxin, bool one) {
    size_t floats = (size_t)stage_buffers(one) * stage_floats(one, maxG) + 4 * (size_t)maxA + 64 * (size_t)maxA +
                    16 * (size_t)maxin * maxA + (one ? 0 : 16) * (size_t)threads + 16 * (size_t)maxG;
    return floats * sizeof(float);
}

int sweep_occupancy(int threads, bool one, bool ext, int depth, size_t lds) {
    const void *k = nullptr;
    switch (threads) {
        case 64: k = one ? kernel_ptr<64, true>(ext, depth) : kernel_ptr<64, false>(ext, depth); break;
        case 128: k = one ? kernel_ptr<128, true>(ext, depth) : kernel_ptr<128, false>(ext, depth); break;
        case 192: k = one ? kernel_ptr<192, true>(ext, depth) : kernel_ptr<192, false>(ext, depth); break;
        case 256: k = one ? kernel_ptr<256, true>(ext, depth) : kernel_ptr<256, false>(ext, depth); break;
        case 512: k = one ? kernel_ptr<512, true>(ext, depth) : kernel_ptr<512, false>(ext, depth); break;
        default: return 0;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, lds) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_sweep_prologue(SweepCtl *ctl, unsigned long long *queue, const DevProblem *probs, int nprob,
                                 const int *seeds, const int *seed_off, const int *stops, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep_prologue, dim3(1), dim3(64), 0, s, ctl, queue, probs, nprob, seeds, seed_off, stops);
    return hipGetLastError();
}

hipError_t launch_xcc_probe(int *out, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_xcc_probe, dim3(nblocks), dim3(64), 0, s, out);
    return hipGetLastError();
}

hipError_t launch_sweep_kernel(const DevProblem *probs, int nprob, const long long *task_base, SweepCtl *ctl,
                               unsigned long long *queue, int threads, bool one, int grid, int maxA, int maxG,
                               int maxin, unsigned long long watchdog, bool phase_stats, int depth, bool ext,
                               hipStream_t s) {
    const size_t lds = sweep_lds_bytes(threads, maxA, maxG, maxin, one);
    const int ps = phase_stats ? 1 : 0;
#define SNX_LAUNCH(NT)                                                                                             \
    return one ? launch_nt<NT, true, false>(probs, nprob, task_base, ctl, queue, maxA, maxG, maxin, grid, lds,      \
                                            watchdog, nullptr, 0, 0, nullptr, ps, depth, ext, s)                    \
               : launch_nt<NT, false, false>(probs, nprob, task_base, ctl, queue, maxA, maxG, maxin, grid, lds,     \
                                             watchdog, nullptr, 0, 0, nullptr, ps, depth, ext, s)
    switch (threads) {
        case 64: SNX_LAUNCH(64);
        case 128: SNX_LAUNCH(128);
        case 192: SNX_LAUNCH(192);
        case 256: SNX_LAUNCH(256);
        case 512: SNX_LAUNCH(512);
        default: return hipErrorInvalidValue;
    }
#undef SNX_LAUNCH
}

hipError_t launch_sweep_level(const DevProblem *probs, int nprob, const long long *task_base, SweepCtl *ctl,
                              int threads, bool one, int grid, int maxA, int maxG, int maxin,
                              const long long *bsp_tasks, long long begin, long long end, const int *stops,
                              int depth, bool ext, hipStream_t s) {
    const size_t lds = sweep_lds_bytes(threads, maxA, maxG, maxin, one);
    const long long n = end - begin;
    if (n <= 0) return hipSuccess;
    const int g = (int)std::min<long long>(grid, n);
#define SNX_LAUNCH(NT)                                                                                             \
    return one ? launch_nt<NT, true, true>(probs, nprob, task_base, ctl, nullptr, maxA, maxG, maxin, g, lds, 0,     \
                                           bsp_tasks, begin, end, stops, 0, depth, ext, s)                          \
               : launch_nt<NT, false, true>(probs, nprob, task_base, ctl, nullptr, maxA, maxG, maxin, g, lds, 0,    \
                                            bsp_tasks, begin, end, stops, 0, depth, ext, s)
    switch (threads) {
        case 64: SNX_LAUNCH(64);
        case 128: SNX_LAUNCH(128);
        case 192: SNX_LAUNCH(192);
        case 256: SNX_LAUNCH(256);
        case 512: SNX_LAUNCH(512);
        default: return hipErrorInvalidValue;
    }
#undef SNX_LAUNCH
}

}  // namespace snx
