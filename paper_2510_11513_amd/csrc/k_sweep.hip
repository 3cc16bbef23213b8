// Persistent, dependency-driven S_N sweep on gfx950.
//
// The paper's many-task sweep (Section 3, Algorithm 1) starts one task per
// direction at the first element, and a task, after solving its element for
// all groups, generates the task of every downwind neighbour for which it was
// the last upwind dependency, detected with per-element atomic counters.
// On the GPU a task is one (cell, octant) pair of one problem: all A angles of
// the octant and all G groups of the cell are solved by one workgroup, one
// (angle, group) system per lane.  Tasks whose counters are complete are
// pushed to a device queue; resident workgroups pop queue slots in order and
// wait for the slot to be filled.  Every octant shares one upwind designation,
// so a cell's (octant) task covers every angle of that octant.
//
// Per task (lane = (angle n, group g)), the upwind DG system of the cell is
//   A = sum_a Om_a S^a + sigma_t M - sum_{f in} Om.F_f       (8x8)
//   b = r_g - sum_{f in} (Om.F_f) psi_up_f,   r_g = M (Q + sigma_s phi) / (4 pi)
// assembled from a per-angle operator B_n = sum_a Om_a S^a - sum_in Om.F_f built
// once per task in LDS, and solved by unpivoted LU in registers, row by row.
//
// Cross-CU / cross-XCD hand-off.  The solution psi of a task is stored with
// agent-coherent (sc1) stores and read by consumers with agent-coherent loads;
// every wave waits for its stores to complete (vmcnt(0)) before the workgroup
// increments downstream counters.  Other data is read-only during the kernel
// and stays cacheable.
//
// The angle reduction phi = sum_n w_n psi_n (Eq. 2) is done in the task: the
// weighted solutions of each round of lanes are staged in LDS and added in
// increasing angle order with a compensated (TwoSum) sum per (group, dof);
// the per-octant partial and its compensation go to the octant's slot.  The
// summation order is fixed, so results do not depend on the schedule.
#include "snx_internal.h"

namespace snx {
namespace {

__device__ inline float ld_agent(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// face f = 2*axis + side: face-local vertex k -> cell-local vertex
__device__ inline int face_vertex(int f, int k) {
    const int axis = f >> 1, side = f & 1;
    if (axis == 0) return (k << 1) | side;
    if (axis == 1) return (k & 1) | (side << 1) | ((k >> 1) << 2);
    return (side << 2) | k;
}
// cell-local vertex j on a face of the given axis -> face-local index
__device__ inline int face_index(int axis, int j) {
    if (axis == 0) return j >> 1;
    if (axis == 1) return (j & 1) | ((j >> 2) << 1);
    return j & 3;
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ inline void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ inline int find_problem(const long long *__restrict__ base, int nprob, long long task) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= task) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// LDS layout (floats): M[64] S[192] Fin[6][48] om[A][4] Bop[A][64] Cop[A][maxin][16]
//                      wpsi[NT][8] red_s[G][8] red_c[G][8]
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep(const DevProblem *__restrict__ probs, int nprob,
                                              const long long *__restrict__ task_base, long long total,
                                              QueueCtl *__restrict__ ctl, unsigned long long *__restrict__ queue,
                                              const int *__restrict__ stop_flag, int maxA, int maxG, int maxin,
                                              unsigned long long watchdog) {
    extern __shared__ __align__(16) float lds[];
    __shared__ long long s_task;
    if (stop_flag && *stop_flag) return;
    const unsigned epoch = ctl->epoch;
    const int tid = threadIdx.x;

    float *sM = lds;
    float *sS = sM + 64;
    float *sF = sS + 192;                 // up to 6 inflow faces x 48
    float *sOm = sF + 6 * 48;             // [maxA][4]: omega xyz, weight
    float *sB = sOm + 4 * maxA;           // [maxA][64]
    float *sC = sB + 64 * maxA;           // [maxA][maxin][16]
    float *sW = sC + 16 * maxin * maxA;   // [NT][8]
    float *sRs = sW + 8 * NT;             // [maxG][8]
    float *sRc = sRs + 8 * maxG;          // [maxG][8]

    unsigned long long my_polls = 0, my_tasks = 0;
    for (;;) {
        if (tid == 0) {
            long long task = -1;
            const unsigned slot = atomicAdd(&ctl->head, 1u);
            if ((long long)slot < total) {
                const unsigned long long t0 = wall_clock64();
                for (;;) {
                    const unsigned long long v =
                        __hip_atomic_load(&queue[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((unsigned)(v >> 32) == epoch) { task = (long long)(v & 0xffffffffull); break; }
                    if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                    ++my_polls;
                    if (wall_clock64() - t0 > watchdog) {
                        __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            s_task = task;
        }
        __syncthreads();
        const long long task = s_task;
        if (task < 0) break;

        // ---------------------------------------------------------- decode
        const int p = find_problem(task_base, nprob, task);
        const DevProblem &P = probs[p];
        const int C = P.C, G = P.G, A = P.A;
        const long long local = task - P.task_base;
        const int o = (int)(local / C);
        const int K = (int)(local - (long long)o * C);
        const int mask = P.inmask[(size_t)o * C + K];
        const int nin = __popc(mask);

        // ---------------------------------------------------- stage geometry
        for (int i = tid; i < 64; i += NT) sM[i] = P.M[(size_t)K * 64 + i];
        for (int i = tid; i < 192; i += NT) sS[i] = P.S[(size_t)K * 192 + i];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (!((mask >> f) & 1)) continue;
            const int s = __popc(mask & ((1 << f) - 1));   // slot of face f among the inflow faces
            for (int i = tid; i < 48; i += NT) sF[s * 48 + i] = P.F[((size_t)K * 6 + f) * 48 + i];
        }
        for (int i = tid; i < A; i += NT) {
            const int n = o * A + i;
            sOm[4 * i + 0] = P.omega[3 * n + 0];
            sOm[4 * i + 1] = P.omega[3 * n + 1];
            sOm[4 * i + 2] = P.omega[3 * n + 2];
            sOm[4 * i + 3] = P.w[n];
        }
        for (int i = tid; i < G * 8; i += NT) { sRs[i] = 0.f; sRc[i] = 0.f; }
        __syncthreads();

        // ------------------------------------- per-angle operators B_n, C_n,f
        for (int e = tid; e < A * 64; e += NT) {
            const int n = e >> 6, ij = e & 63, i = ij >> 3, j = ij & 7;
            const float ox = sOm[4 * n], oy = sOm[4 * n + 1], oz = sOm[4 * n + 2];
            float v = ox * sS[ij] + oy * sS[64 + ij] + oz * sS[128 + ij];
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const int axis = f >> 1, side = f & 1;
                if (((mask >> f) & 1) && ((i >> axis) & 1) == side && ((j >> axis) & 1) == side) {
                    const int kl = face_index(axis, i) * 4 + face_index(axis, j);
                    const float *Fs = sF + __popc(mask & ((1 << f) - 1)) * 48;
                    v -= ox * Fs[kl] + oy * Fs[16 + kl] + oz * Fs[32 + kl];
                }
            }
            sB[e] = v;
        }
        for (int e = tid; e < A * nin * 16; e += NT) {
            const int n = e / (nin * 16), rem = e - n * nin * 16, s = rem >> 4, kl = rem & 15;
            const float *Fs = sF + s * 48;
            sC[(n * maxin + s) * 16 + kl] =
                sOm[4 * n] * Fs[kl] + sOm[4 * n + 1] * Fs[16 + kl] + sOm[4 * n + 2] * Fs[32 + kl];
        }
        __syncthreads();

        // ------------------------------------------------ rounds of lanes
        const int AG = A * G;
        const size_t cell_psi = (size_t)8 * A * G;          // floats per (octant, cell)
        float *psi_o = P.psi + (size_t)o * C * cell_psi;
        for (int base = 0; base < AG; base += NT) {
            const int pi = base + tid;
            if (pi < AG) {
                const int n = pi / G, g = pi - n * G;
                const float sig = P.sigt[(size_t)K * G + g];
                float b[8];
                const float4 *rv = reinterpret_cast<const float4 *>(P.r + ((size_t)K * G + g) * 8);
                const float4 r0 = rv[0], r1 = rv[1];
                b[0] = r0.x; b[1] = r0.y; b[2] = r0.z; b[3] = r0.w;
                b[4] = r1.x; b[5] = r1.y; b[6] = r1.z; b[7] = r1.w;
                const float psib = P.psib ? P.psib[g] : 0.f;
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    if (!((mask >> f) & 1)) continue;
                    const int s = __popc(mask & ((1 << f) - 1));
                    float up[4];
                    const int N = P.nbr[(size_t)K * 6 + f];
                    if (N >= 0) {
                        const unsigned pm = P.perm[(size_t)K * 6 + f];
                        const float *pn = psi_o + (size_t)N * cell_psi + (size_t)n * G + g;
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            const int jn = (pm >> (8 * l)) & 0xff;
                            up[l] = ld_agent(pn + (size_t)jn * A * G);
                        }
                    } else {
#pragma unroll
                        for (int l = 0; l < 4; ++l) up[l] = psib;
                    }
                    const float *Cs = sC + (n * maxin + s) * 16;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        float t = Cs[k * 4] * up[0];
                        t = __builtin_fmaf(Cs[k * 4 + 1], up[1], t);
                        t = __builtin_fmaf(Cs[k * 4 + 2], up[2], t);
                        t = __builtin_fmaf(Cs[k * 4 + 3], up[3], t);
                        b[face_vertex(f, k)] -= t;
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
                }
#pragma unroll
                for (int k = 7; k >= 0; --k) {
                    float t = b[k];
#pragma unroll
                    for (int j = k + 1; j < 8; ++j) t = __builtin_fmaf(-U[k][j], b[j], t);
                    b[k] = t * inv[k];
                }
                float *pk = psi_o + (size_t)K * cell_psi + (size_t)n * G + g;
                const float wn = sOm[4 * n + 3];
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    st_agent(pk + (size_t)d * A * G, b[d]);
                    sW[tid * 8 + d] = wn * b[d];
                }
            }
            __syncthreads();
            // compensated accumulation in increasing angle order, one (group, dof) per reducer
            const int hi = min(base + NT, AG);
            for (int e = tid; e < G * 8; e += NT) {
                const int g = e >> 3, d = e & 7;
                float s = sRs[e], c = sRc[e];
                int p0 = base + ((g - base % G) % G + G) % G;
                for (int q = p0; q < hi; q += G) {
                    float t, err;
                    two_sum(s, sW[(q - base) * 8 + d], t, err);
                    s = t;
                    c += err;
                }
                sRs[e] = s;
                sRc[e] = c;
            }
            __syncthreads();
        }

        // ------------------------------------------------------ octant slot
        const size_t sbase = ((size_t)o * C + K) * G * 8;
        for (int e = tid; e < G * 8; e += NT) {
            P.slot[sbase + e] = sRs[e];
            P.slotc[sbase + e] = sRc[e];
        }

        // --------------------------------------------- publish to downwind
        wait_stores();
        __syncthreads();
        if (tid < 6) {
            const int f = tid;
            const int N = ((mask >> f) & 1) ? -1 : P.nbr[(size_t)K * 6 + f];
            if (N >= 0) {
                const unsigned old = __hip_atomic_fetch_add(&P.cnt[(size_t)o * C + N], 1u, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                const unsigned target = (unsigned)P.indeg[(size_t)o * C + N] * epoch;
                if (old + 1u == target) {
                    const unsigned slot = atomicAdd(&ctl->tail, 1u);
                    const unsigned long long v =
                        ((unsigned long long)epoch << 32) | (unsigned long long)(P.task_base + (long long)o * C + N);
                    if ((long long)slot < total)
                        __hip_atomic_store(&queue[slot], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    else   // more pushes than tasks: counters inconsistent with the DAG
                        __hip_atomic_store(&ctl->abort, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        ++my_tasks;
        __syncthreads();
    }
    if (tid == 0) {
        atomicAdd(&ctl->polls_empty, my_polls);
        atomicAdd(&ctl->tasks_done, my_tasks);
    }
}

// Starts a sweep: advances the epoch, empties the queue and pushes the tasks
// with no interior upwind face (level 0 of every octant).
__global__ void k_sweep_prologue(QueueCtl *ctl, unsigned long long *queue, const int *__restrict__ seeds, int nseed,
                                 const int *stop_flag) {
    if (stop_flag && *stop_flag) return;
    __shared__ unsigned s_epoch;
    if (threadIdx.x == 0) s_epoch = ctl->epoch + 1u;
    __syncthreads();
    const unsigned e = s_epoch;
    for (int i = threadIdx.x; i < nseed; i += blockDim.x)
        queue[i] = ((unsigned long long)e << 32) | (unsigned)seeds[i];
    if (threadIdx.x == 0) {
        ctl->epoch = e;
        ctl->head = 0;
        ctl->tail = (unsigned)nseed;
        ctl->polls_empty = 0;
        ctl->tasks_done = 0;
    }
}

template <int NT>
hipError_t launch_nt(const DevProblem *probs, int nprob, const long long *task_base, long long total, QueueCtl *ctl,
                     unsigned long long *queue, const int *stop_flag, int maxA, int maxG, int maxin, int grid,
                     size_t lds, unsigned long long watchdog, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep<NT>, dim3(grid), dim3(NT), lds, s, probs, nprob, task_base, total, ctl, queue,
                       stop_flag, maxA, maxG, maxin, watchdog);
    return hipGetLastError();
}

template <int NT>
const void *kernel_ptr() { return reinterpret_cast<const void *>(&k_sweep<NT>); }

}  // namespace

size_t sweep_lds_bytes(int threads, int maxA, int maxG, int maxin) {
    size_t floats = 64 + 192 + 6 * 48 + 4 * (size_t)maxA + 64 * (size_t)maxA + 16 * (size_t)maxin * maxA +
                    8 * (size_t)threads + 16 * (size_t)maxG;
    return floats * sizeof(float);
}

int sweep_occupancy(int threads, size_t lds) {
    const void *k = nullptr;
    switch (threads) {
        case 64: k = kernel_ptr<64>(); break;
        case 128: k = kernel_ptr<128>(); break;
        case 256: k = kernel_ptr<256>(); break;
        case 512: k = kernel_ptr<512>(); break;
        case 1024: k = kernel_ptr<1024>(); break;
        default: return 0;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, lds) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_sweep_prologue(QueueCtl *ctl, unsigned long long *queue, const int *seeds, int nseed,
                                 const int *stop_flag, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep_prologue, dim3(1), dim3(256), 0, s, ctl, queue, seeds, nseed, stop_flag);
    return hipGetLastError();
}

hipError_t launch_sweep_kernel(const DevProblem *probs, int nprob, const long long *task_base, long long total,
                               QueueCtl *ctl, unsigned long long *queue, const int *stop_flag, int threads, int grid,
                               int maxA, int maxG, int maxin, unsigned long long watchdog, hipStream_t s) {
    const size_t lds = sweep_lds_bytes(threads, maxA, maxG, maxin);
    switch (threads) {
        case 64: return launch_nt<64>(probs, nprob, task_base, total, ctl, queue, stop_flag, maxA, maxG, maxin, grid, lds, watchdog, s);
        case 128: return launch_nt<128>(probs, nprob, task_base, total, ctl, queue, stop_flag, maxA, maxG, maxin, grid, lds, watchdog, s);
        case 256: return launch_nt<256>(probs, nprob, task_base, total, ctl, queue, stop_flag, maxA, maxG, maxin, grid, lds, watchdog, s);
        case 512: return launch_nt<512>(probs, nprob, task_base, total, ctl, queue, stop_flag, maxA, maxG, maxin, grid, lds, watchdog, s);
        case 1024: return launch_nt<1024>(probs, nprob, task_base, total, ctl, queue, stop_flag, maxA, maxG, maxin, grid, lds, watchdog, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace snx
