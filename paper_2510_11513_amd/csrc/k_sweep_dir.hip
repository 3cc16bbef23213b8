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
constexpr int kUnitFloats = 544 + 65 + 96;   // M, S, F of the cell; B (odd stride); the inflow faces' Om . F

__global__ __launch_bounds__(kDirThreads) void k_sweep_dir(DirDev D, const DevProblem *__restrict__ probs,
                                                           long long begin, long long end, int upw, const int *stop) {
    if (stop && *stop) return;
    const DevProblem &P = probs[0];
    const int C = P.C, A = P.A, G = P.G;
    const long long u0 = begin + (long long)blockIdx.x * upw;
    const int nu = (int)min((long long)upw, end - u0);
    extern __shared__ float smem[];
    __shared__ int sNb[kMaxUnits][6], sTask[kMaxUnits], sDir[kMaxUnits];
    __shared__ unsigned sPm[kMaxUnits][6];
    const int tid = threadIdx.x;
    if (tid < nu) {
        sTask[tid] = D.units[2 * (u0 + tid)];
        sDir[tid] = D.units[2 * (u0 + tid) + 1];
    }
    __syncthreads();
    // the cell data of every unit: all loads in flight together
    for (int e = tid; e < nu * 544; e += kDirThreads) {
        const int u = e / 544, i = e % 544;
        const int K = sTask[u] >> 3;
        float *sc = smem + u * kUnitFloats;
        sc[i] = i < 64 ? P.M[(size_t)K * 64 + i]
                       : (i < 256 ? P.S[(size_t)K * 192 + i - 64] : P.F[(size_t)K * 288 + i - 256]);
    }
    if (tid < nu * 6) {
        const int u = tid / 6, f = tid % 6;
        const int K = sTask[u] >> 3;
        sNb[u][f] = P.nbr[(size_t)K * 6 + f];
        sPm[u][f] = P.perm[(size_t)K * 6 + f];
    }
    __syncthreads();
    for (int idx = tid; idx < nu * (64 + 96); idx += kDirThreads) {
        const int u = idx / (64 + 96), e = idx % (64 + 96);
        const int task = sTask[u], a = sDir[u];
        const int K = task >> 3, o = task & 7, n = o * A + a;
        const float *sS = smem + u * kUnitFloats + 64, *sF = smem + u * kUnitFloats + 256;
        const float ox = P.omega[3 * n], oy = P.omega[3 * n + 1], oz = P.omega[3 * n + 2];
        const int mask = D.amask[((size_t)o * C + K) * A + a];
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
    const int g = G <= kDirThreads ? tid % G : (int)blockIdx.y * kDirThreads + tid;
    if (u >= nu || g >= G) return;
    const int task = sTask[u], a = sDir[u];
    const int K = task >> 3, o = task & 7;
    const size_t AG = (size_t)A * G;
    const size_t oka = ((size_t)o * C + K) * A + a;
    const int mask = D.amask[oka], lagb = D.lagbits[oka];
    const int lbase = lagb ? D.lagidx[oka] : 0;
    const float sig = P.sigt[(size_t)K * G + g];
    const float *sM = smem + u * kUnitFloats;
    const float *Bk = sM + 544, *sOF = sM + 544 + 65;
    float m[64], b[8];
#pragma unroll
    for (int e = 0; e < 64; ++e) m[e] = __builtin_fmaf(sig, sM[e], Bk[e]);
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = P.r[((size_t)K * G + g) * 8 + i];
    // right-hand side: minus each inflow face's operator on the upwind trace
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!((mask >> f) & 1)) continue;
        const int N = sNb[u][f];
        float uu[4];
        if (N >= 0 && ((lagb >> f) & 1)) {          // a face lagged to break a cycle: last sweep's flux
            const int slot = lbase + __popc(lagb & ((1 << f) - 1));
#pragma unroll
            for (int l = 0; l < 4; ++l) uu[l] = D.lagbuf[((size_t)slot * 4 + l) * G + g];
        } else if (N >= 0) {                        // an earlier level of this direction: this sweep's
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int vn = (int)((sPm[u][f] >> (8 * l)) & 0xffu);
                uu[l] = P.psi[(((size_t)o * C + N) * 8 + vn) * AG + (size_t)a * G + g];
            }
        } else {
#pragma unroll
            for (int l = 0; l < 4; ++l) uu[l] = P.psib ? P.psib[g] : 0.f;
        }
        const float *OF = sOF + f * 16;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
#pragma unroll
            for (int l = 0; l < 4; ++l) t = __builtin_fmaf(OF[4 * k + l], uu[l], t);
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
    float *dst = P.psi + ((size_t)o * C + K) * 8 * AG + (size_t)a * G + g;
#pragma unroll
    for (int d = 0; d < 8; ++d) dst[d * AG] = b[d];
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
        const float *src = P.psi + (oc * 8 + d) * A * G + g;
        float s = 0.f, c = 0.f;
        for (int a = 0; a < A; ++a) {
            float u, e;
            two_sum(s, P.w[o * A + a] * src[(size_t)a * G], u, e);
            s = u;
            c += e;
        }
        const size_t e = ((size_t)oc * G + g) * 8 + d;
        P.slot[e] = s;
        P.slotc[e] = c;
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

hipError_t launch_dir_slots(const DevProblem *probs, int C, int G, const int *stop, hipStream_t s) {
    hipLaunchKernelGGL(k_dir_slots, dim3(grid_of(64LL * C * G, 256)), dim3(256), 0, s, probs, stop);
    return hipGetLastError();
}

}  // namespace snx
