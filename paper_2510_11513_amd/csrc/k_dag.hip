// Per-octant upwind designation and topological levelling on the device.
//
// The sweep of one direction visits cells after all their upwind neighbours
// (Section 2.1: the dependencies form a DAG; UnSNAP groups cells into t-level
// "buckets" and merges the buckets of all angles of an octant).  Here one
// designation serves a whole octant: face f of cell K is inflow for octant o
// when s_o . A_f < 0, with s_o the octant's sign vector and A_f the outward
// area vector.  A_f is antisymmetric across interior faces, so exactly one
// side of every face is upwind.  One workgroup per octant peels the DAG level
// by level: level(K) = 1 + max level of its upwind neighbours.
#include "snx_internal.h"

namespace snx {
namespace {

constexpr int kDagThreads = 1024;

__global__ __launch_bounds__(kDagThreads) void k_dag(int C, const int *__restrict__ nbr,
                                                     const double *__restrict__ area,
                                                     unsigned char *__restrict__ inmask, int *__restrict__ indeg,
                                                     int *__restrict__ level, int *__restrict__ hist,
                                                     int *__restrict__ nlev, int *__restrict__ seeds,
                                                     int *__restrict__ nseed, int *__restrict__ scratch,
                                                     int *__restrict__ err) {
    const int o = blockIdx.x;
    const double sx = (o & 1) ? -1.0 : 1.0, sy = (o & 2) ? -1.0 : 1.0, sz = (o & 4) ? -1.0 : 1.0;
    int *rem = scratch + (size_t)o * 3 * C;       // remaining upwind faces per cell
    int *cur = rem + C;                             // current frontier
    int *nxt = cur + C;                             // next frontier
    __shared__ int s_ncur, s_nnext, s_maxin;
    if (threadIdx.x == 0) { s_ncur = 0; s_nnext = 0; s_maxin = 0; }
    __syncthreads();
    for (int K = threadIdx.x; K < C; K += blockDim.x) {
        int mask = 0, nin = 0, nall = 0;
        for (int f = 0; f < 6; ++f) {
            const double *A = area + ((size_t)K * 6 + f) * 3;
            double d = sx * A[0] + sy * A[1] + sz * A[2];
            if (d == 0.0) atomicOr(err, 2);
            if (d < 0.0) {
                mask |= 1 << f;
                ++nall;
                if (nbr[(size_t)K * 6 + f] >= 0) ++nin;
            }
        }
        inmask[(size_t)o * C + K] = (unsigned char)mask;
        indeg[(size_t)o * C + K] = nin;
        rem[K] = nin;
        atomicMax(&s_maxin, nall);
        if (nin == 0) {
            int i = atomicAdd(&s_ncur, 1);
            cur[i] = K;
            level[(size_t)o * C + K] = 0;
        }
    }
    __syncthreads();
    int lev = 0, total = 0;
    for (;;) {
        const int n = s_ncur;
        if (n == 0) break;
        total += n;
        if (threadIdx.x == 0) hist[(size_t)o * (C + 1) + lev] = n;
        if (lev == 0) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) seeds[(size_t)o * C + i] = cur[i];
            if (threadIdx.x == 0) nseed[o] = n;
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int K = cur[i];
            const int mask = inmask[(size_t)o * C + K];
            for (int f = 0; f < 6; ++f) {
                if ((mask >> f) & 1) continue;
                const int N = nbr[(size_t)K * 6 + f];
                if (N < 0) continue;
                if (atomicSub(&rem[N], 1) == 1) {
                    level[(size_t)o * C + N] = lev + 1;
                    nxt[atomicAdd(&s_nnext, 1)] = N;
                }
            }
        }
        __syncthreads();
        int *t = cur; cur = nxt; nxt = t;
        ++lev;
        __syncthreads();
        if (threadIdx.x == 0) { s_ncur = s_nnext; s_nnext = 0; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        nlev[o] = lev;
        nlev[8 + o] = s_maxin;
        if (total != C) atomicOr(err, 4);
    }
}

}  // namespace

hipError_t launch_dag_one(int C, const int *nbr, const double *area, unsigned char *inmask, int *indeg, int *level,
                          int *hist, int *nlev, int *seeds, int *nseed, int *scratch, int *err, hipStream_t s) {
    hipLaunchKernelGGL(k_dag, dim3(8), dim3(kDagThreads), 0, s, C, nbr, area, inmask, indeg, level, hist, nlev,
                       seeds, nseed, scratch, err);
    return hipGetLastError();
}

}  // namespace snx

namespace snx {
namespace {

// T^a_ij = S^a_ij - sum over inflow faces f of octant o of F^a_f at (i, j) when both
// i and j lie on f: the angle-independent part of the upwind operator
// B_n = sum_a Omega_a T^a of every direction of the octant.
__global__ void k_octant_operators(int C, const float *__restrict__ S, const float *__restrict__ F,
                                   const unsigned char *__restrict__ inmask, float *__restrict__ T) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 8LL * C * 192) return;
    const int e = (int)(t % 192);
    const long long oc = t / 192;            // o * C + K
    const int K = (int)(oc % C);
    const int a = e >> 6, ij = e & 63, i = ij >> 3, j = ij & 7;
    const int mask = inmask[oc];
    float v = S[(size_t)K * 192 + e];
    for (int f = 0; f < 6; ++f) {
        const int axis = f >> 1, side = f & 1;
        if (!((mask >> f) & 1) || ((i >> axis) & 1) != side || ((j >> axis) & 1) != side) continue;
        const int ki = axis == 0 ? i >> 1 : (axis == 1 ? (i & 1) | ((i >> 2) << 1) : i & 3);
        const int kj = axis == 0 ? j >> 1 : (axis == 1 ? (j & 1) | ((j >> 2) << 1) : j & 3);
        v -= F[((size_t)K * 6 + f) * 48 + a * 16 + ki * 4 + kj];
    }
    T[t] = v;
}

// Task records (layout at kRecWords): a task's own descriptor and those of its
// downwind neighbours, so a task that continues with a downwind cell already
// holds that cell's descriptor when it starts it.
__global__ void k_task_records(int C, const int *__restrict__ nbr, const unsigned *__restrict__ perm,
                               const unsigned char *__restrict__ inmask, const int *__restrict__ indeg,
                               const unsigned char *__restrict__ lagm, const unsigned char *__restrict__ rmask,
                               const int *__restrict__ rbase, int *__restrict__ rec) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // o * C + K
    if (t >= 8LL * C) return;
    const int o = (int)(t / C), K = (int)(t - (long long)o * C);
    int *r = rec + t * kRecWords;
    auto desc = [&](int cell, int *d) {
        for (int f = 0; f < 6; ++f) {
            d[f] = nbr[(size_t)cell * 6 + f];
            d[6 + f] = (int)perm[(size_t)cell * 6 + f];
        }
        d[12] = inmask[(size_t)o * C + cell];
    };
    desc(K, r);
    r[13] = (lagm ? (int)lagm[t] << 18 : 0) | (rmask ? (int)rmask[K] << 24 : 0);
    r[14] = rmask ? rbase[K] : 0;
    r[15] = 0;
    const int mask = inmask[t];
    for (int f = 0; f < 6; ++f) {
        int *d = r + 16 + 13 * f;
        const int N = nbr[(size_t)K * 6 + f];
        if (!((mask >> f) & 1) && N >= 0) {
            desc(N, d);
            r[13] |= indeg[(size_t)o * C + N] << (3 * f);   // in-degree of the downwind cell (<= 6)
        } else {
            for (int w = 0; w < 13; ++w) d[w] = 0;
        }
    }
    r[94] = r[95] = 0;
}

// Per-angle designation (each direction's own mesh traversal, Section 2.1):
// face f of K is inflow for direction n when Omega_n . A_f < 0, decided in FP64.
// Tasks stay (cell, octant) and follow the octant's DAG; the sweep corrects the
// operators of the directions that differ from the octant's designation, and a
// face that is inflow for a direction but downwind in the octant's order takes
// the neighbour's angular flux of the previous sweep (a lagged face).  One
// thread per (octant, cell).
__global__ void k_angle_masks(int C, int A, const double *__restrict__ omega, const int *__restrict__ nbr,
                              const double *__restrict__ area, const unsigned char *__restrict__ inmask,
                              unsigned char *__restrict__ amask, unsigned char *__restrict__ lagm,
                              unsigned long long *__restrict__ counts, int *__restrict__ err) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // o * C + K
    if (t >= 8LL * C) return;
    const int o = (int)(t / C), K = (int)(t - (long long)o * C);
    const int om = inmask[t];
    int interior = 0;
    for (int f = 0; f < 6; ++f) interior |= nbr[(size_t)K * 6 + f] >= 0 ? 1 << f : 0;
    int any = 0;
    unsigned long long ndiff = 0, nlag = 0;
    for (int a = 0; a < A; ++a) {
        const double *w = omega + 3 * ((size_t)o * A + a);
        int mask = 0;
        for (int f = 0; f < 6; ++f) {
            const double *Af = area + ((size_t)K * 6 + f) * 3;
            const double d = w[0] * Af[0] + w[1] * Af[1] + w[2] * Af[2];
            if (d == 0.0) atomicOr(err, 8);
            mask |= d < 0.0 ? 1 << f : 0;
        }
        amask[(size_t)t * A + a] = (unsigned char)mask;
        any |= mask ^ om;
        ndiff += __popc(mask ^ om);
        nlag += __popc(mask & ~om & interior);
    }
    lagm[t] = (unsigned char)any;
    if (ndiff) {
        atomicAdd(&counts[0], ndiff);
        atomicAdd(&counts[1], nlag);
        atomicAdd(&counts[2], 1ull);
    }
}

}  // namespace

hipError_t launch_task_records(int C, const int *nbr, const unsigned *perm, const unsigned char *inmask,
                               const int *indeg, const unsigned char *lagm, const unsigned char *rmask,
                               const int *rbase, int *rec, hipStream_t s) {
    const long long n = 8LL * C;
    hipLaunchKernelGGL(k_task_records, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, nbr, perm, inmask,
                       indeg, lagm, rmask, rbase, rec);
    return hipGetLastError();
}

hipError_t launch_angle_masks(int C, int A, const double *omega, const int *nbr, const double *area,
                              const unsigned char *inmask, unsigned char *amask, unsigned char *lagm,
                              unsigned long long *counts, int *err, hipStream_t s) {
    const long long n = 8LL * C;
    hipLaunchKernelGGL(k_angle_masks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, A, omega, nbr, area,
                       inmask, amask, lagm, counts, err);
    return hipGetLastError();
}

hipError_t launch_octant_operators(int C, const float *S, const float *F, const unsigned char *inmask, float *T,
                                   hipStream_t s) {
    const long long n = 8LL * C * 192;
    hipLaunchKernelGGL(k_octant_operators, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, S, F, inmask, T);
    return hipGetLastError();
}

}  // namespace snx
