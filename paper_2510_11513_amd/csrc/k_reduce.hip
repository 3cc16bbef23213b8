// Angle reduction, source update, FP64 convergence residual and particle balance.
//
//   phi_K,g    = sum_o (slot_o + comp_o)             per-octant partials of Eq. 2,
//                                                   added in octant order with TwoSum
//   r_K,g      = M_K (Q_K,g + sigma_s,K,g phi_K,g + qo_K,g) / (4 pi)   next sweep's source,
//                qo the cross-group scattering source of the current outer
//                iteration (absent without a group-to-group matrix)
//   eps        = ||phi_new - phi_old||_inf / ||phi_new||_inf      in FP64
//   balance    : 1^T M (Q + sigma_s phi_in) = sigma_t 1^T M phi_out + sum_n w_n L_n
#include "snx_internal.h"

#include <algorithm>

namespace snx {
namespace {

__device__ inline void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ inline void source_dofs(const float *__restrict__ M, float q, float ss, const float (&phi)[8],
                                   const float *__restrict__ qo, float (&r)[8]) {
    float src[8];
    if (qo) {
#pragma unroll
        for (int j = 0; j < 8; ++j) src[j] = (q + (ss * phi[j] + qo[j])) * kInv4Pi;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) src[j] = (q + ss * phi[j]) * kInv4Pi;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc = __builtin_fmaf(M[i * 8 + j], src[j], acc);
        r[i] = acc;
    }
}

// r = M (Q + sigma_s phi) / (4 pi) from a given phi (NULL = zero flux).
__global__ void k_source(const DevProblem *__restrict__ probs, int prob, const float *__restrict__ phi,
                         const int *__restrict__ stop_flag) {
    if (stop_flag && *stop_flag) return;
    const DevProblem &P = probs[prob];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)P.C * P.G) return;
    const int K = (int)(t / P.G);
    float ph[8], r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) ph[j] = phi ? phi[t * 8 + j] : 0.f;
    source_dofs(P.M + (size_t)K * 64, P.q[t], P.sigs[t], ph, P.qo ? P.qo + t * 8 : nullptr, r);
    float4 *out = reinterpret_cast<float4 *>(P.r + t * 8);
    out[0] = make_float4(r[0], r[1], r[2], r[3]);
    out[1] = make_float4(r[4], r[5], r[6], r[7]);
}

// Cross-group scattering source of an outer iteration from a given phi (NULL =
// zero): qo_K,g = sum over g' != g of sigma(g' -> g) phi_K,g' at each node, in
// increasing g'.  One thread per (cell, group).
__global__ void k_outer_source(const DevProblem *__restrict__ probs, int prob, const float *__restrict__ phi,
                               const int *__restrict__ stop_flag) {
    if (stop_flag && *stop_flag) return;
    const DevProblem &P = probs[prob];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)P.C * P.G) return;
    const int G = P.G, K = (int)(t / G), g = (int)(t - (long long)K * G);
    const float *S = P.sgg + (size_t)P.cmat[K] * G * G;
    float v[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) v[d] = 0.f;
    if (phi) {
        for (int h = 0; h < G; ++h) {
            if (h == g) continue;
            const float sh = S[(size_t)h * G + g];
            const float *ph = phi + ((size_t)K * G + h) * 8;
#pragma unroll
            for (int d = 0; d < 8; ++d) v[d] = __builtin_fmaf(sh, ph[d], v[d]);
        }
    }
    float4 *out = reinterpret_cast<float4 *>(P.qo + t * 8);
    out[0] = make_float4(v[0], v[1], v[2], v[3]);
    out[1] = make_float4(v[4], v[5], v[6], v[7]);
}

// Anisotropic scattering (the flux-moment arrays of the paper's table of
// arrays).  Step 1: the degree >= 1 moments of the previous sweep's angular
// flux, phi_lm = sum_n w_n Y_lm(Omega_n) psi_n, one thread per (cell, node,
// group) with the group fastest, so each direction's reads are contiguous.
constexpr int kMaxMoments = 16;   // (L + 1)^2 for L <= 3
// The harmonics of every direction go to LDS (at most 8 * 64 * 16 floats) once
// per block; the launch passes that size as dynamic LDS.
__global__ __launch_bounds__(256) void k_moments(const DevProblem *__restrict__ probs, int prob,
                                                 const int *__restrict__ stop_flag) {
    if (stop_flag && *stop_flag) return;
    const DevProblem &P = probs[prob];
    const int C = P.C, G = P.G, A = P.A, nm = (P.L + 1) * (P.L + 1);
    extern __shared__ float s_ylm[];
    for (int i = threadIdx.x; i < 8 * A * nm; i += blockDim.x) s_ylm[i] = P.ylm[i];
    __syncthreads();
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)C * 8 * G) return;
    const int g = (int)(t % G), d = (int)((t / G) % 8), K = (int)(t / (8LL * G));
    float acc[kMaxMoments];
#pragma unroll
    for (int k = 0; k < kMaxMoments; ++k) acc[k] = 0.f;
    const size_t AG = (size_t)A * G;
    for (int o = 0; o < 8; ++o) {
        const float *ps = P.psi + (((size_t)o * C + K) * 8 + d) * AG + g;
        // eight directions' loads in flight together, then their moments
        for (int a0 = 0; a0 < A; a0 += 8) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = a0 + j < A ? ps[(size_t)(a0 + j) * G] : 0.f;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (a0 + j >= A) break;
                const int n = o * A + a0 + j;
                const float wv = P.w[n] * v[j];
                const float *y = s_ylm + n * nm;
#pragma unroll
                for (int k = 1; k < kMaxMoments; ++k)
                    if (k < nm) acc[k] = __builtin_fmaf(y[k], wv, acc[k]);
            }
        }
    }
    float *out = P.mom + ((size_t)K * G + g) * nm * 8 + d;
#pragma unroll
    for (int k = 1; k < kMaxMoments; ++k)
        if (k < nm) out[(size_t)k * 8] = acc[k];
}

// Step 2: the source dofs of each moment, sigma_l M phi_lm (degree >= 1), one
// thread per (cell, group).  A direction's source is then the isotropic
// r = M (Q + sigma_s phi + qo) / (4 pi) plus sum_k Y_k(Omega_n) of these, which
// the sweep adds per lane: the expansion of
// sum_l (2l+1)/(4 pi) sigma_l P_l(Omega . Omega') over real orthonormal harmonics.
__global__ __launch_bounds__(256) void k_moment_sources(const DevProblem *__restrict__ probs, int prob,
                                                        const int *__restrict__ stop_flag) {
    if (stop_flag && *stop_flag) return;
    const DevProblem &P = probs[prob];
    const int C = P.C, G = P.G, L = P.L, nm = (L + 1) * (L + 1);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // K * G + g
    if (t >= (long long)C * G) return;
    const int K = (int)(t / G);
    float Mr[64];                        // the cell's mass matrix, loaded once
    const float4 *M4 = reinterpret_cast<const float4 *>(P.M + (size_t)K * 64);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float4 v = M4[i];
        Mr[4 * i] = v.x; Mr[4 * i + 1] = v.y; Mr[4 * i + 2] = v.z; Mr[4 * i + 3] = v.w;
    }
    for (int l = 1; l <= L; ++l) {
        const float sl = P.sigl[t * L + (l - 1)];
        for (int k = l * l; k < (l + 1) * (l + 1); ++k) {
            const float4 *m4 = reinterpret_cast<const float4 *>(P.mom + ((size_t)t * nm + k) * 8);
            const float4 ma = m4[0], mb = m4[1];
            const float m[8] = {ma.x, ma.y, ma.z, ma.w, mb.x, mb.y, mb.z, mb.w};
            float r[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < 8; ++j) acc = __builtin_fmaf(Mr[d * 8 + j], m[j], acc);
                r[d] = sl * acc;
            }
            float4 *r4 = reinterpret_cast<float4 *>(P.rmom + ((size_t)t * nm + k) * 8);
            r4[0] = make_float4(r[0], r[1], r[2], r[3]);
            r4[1] = make_float4(r[4], r[5], r[6], r[7]);
        }
    }
}

// FP64 max-norm terms of a - b: out[0] = max |a - b|, out[1] = max |a| (both
// non-negative, so their bit patterns order like the values); out must be zero.
__global__ __launch_bounds__(256) void k_max_change(const float *__restrict__ a, const float *__restrict__ b,
                                                    long long n, unsigned long long *__restrict__ out) {
    double num = 0.0, den = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double x = (double)a[i], y = (double)b[i];
        num = fmax(num, fabs(x - y));
        den = fmax(den, fabs(x));
    }
    __shared__ double s_num[256], s_den[256];
    s_num[threadIdx.x] = num;
    s_den[threadIdx.x] = den;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_num[threadIdx.x] = fmax(s_num[threadIdx.x], s_num[threadIdx.x + w]);
            s_den[threadIdx.x] = fmax(s_den[threadIdx.x], s_den[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(s_num[0]));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(s_den[0]));
    }
}

__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// Octant-slot reduction of one (cell, group) of P: phi = sum_o (slot_o + comp_o)
// in octant order with TwoSum; optional source update r = M (Q + sigma_s phi)/(4 pi);
// returns the FP64 residual terms |phi - phi_old| and |phi| (maxima over dofs).
__device__ inline void reduce_one(const DevProblem &P, long long t, float *__restrict__ phi_out,
                                  const float *__restrict__ phi_old, int update_source, double &num, double &den) {
    const long long CG = (long long)P.C * P.G;
    float s[8], c[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) { s[d] = 0.f; c[d] = 0.f; }
    for (int o = 0; o < 8; ++o) {
        const size_t off = ((size_t)o * CG + t) * 8;
        const float4 *sv = reinterpret_cast<const float4 *>(P.slot + off);
        const float4 *cv = reinterpret_cast<const float4 *>(P.slotc + off);
        const float4 a0 = sv[0], a1 = sv[1], b0 = cv[0], b1 = cv[1];
        const float sa[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const float ca[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            float u, e;
            two_sum(s[d], sa[d], u, e);
            s[d] = u;
            c[d] += e + ca[d];
        }
    }
    float ph[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) ph[d] = s[d] + c[d];
    float4 *po = reinterpret_cast<float4 *>(phi_out + t * 8);
    po[0] = make_float4(ph[0], ph[1], ph[2], ph[3]);
    po[1] = make_float4(ph[4], ph[5], ph[6], ph[7]);
    if (update_source) {
        const int K = (int)(t / P.G);
        float r[8];
        source_dofs(P.M + (size_t)K * 64, P.q[t], P.sigs[t], ph, P.qo ? P.qo + t * 8 : nullptr, r);
        float4 *ro = reinterpret_cast<float4 *>(P.r + t * 8);
        ro[0] = make_float4(r[0], r[1], r[2], r[3]);
        ro[1] = make_float4(r[4], r[5], r[6], r[7]);
    }
    if (phi_old) {
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const double nw = (double)ph[d], od = (double)phi_old[t * 8 + d];
            num = fmax(num, fabs(nw - od));
            den = fmax(den, fabs(nw));
        }
    }
}

// Block maxima of the residual terms, then one atomicMax per block (non-negative
// doubles order like their bit patterns); the last block of the problem turns
// them into eps and sets the stop flag on convergence or at max_it.
__device__ inline void residual_finish(double num, double den, IterCtl *ic, int *stop_flag, unsigned nblocks) {
    __shared__ double s_num[256], s_den[256];
    s_num[threadIdx.x] = num;
    s_den[threadIdx.x] = den;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_num[threadIdx.x] = fmax(s_num[threadIdx.x], s_num[threadIdx.x + w]);
            s_den[threadIdx.x] = fmax(s_den[threadIdx.x], s_den[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&ic->num_bits, dbits(s_num[0]));
        atomicMax(&ic->den_bits, dbits(s_den[0]));
        // Both maxima are performed at the device's coherence point once their
        // returns arrive; waiting for them orders them before the count below
        // without a device-wide fence (which would write back the whole L2).
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const unsigned done = atomicAdd(&ic->blocks_done, 1u);
        if (done == nblocks - 1) {
            // every block's maxima precede its count; read them with atomics
            const double nm = __longlong_as_double((long long)atomicAdd(&ic->num_bits, 0ull));
            const double dn = __longlong_as_double((long long)atomicAdd(&ic->den_bits, 0ull));
            const double eps = dn > 0.0 ? nm / dn : (nm > 0.0 ? __builtin_inf() : 0.0);
            ic->last_eps = eps;
            ic->iter += 1;
            ic->num_bits = 0ull;
            ic->den_bits = 0ull;
            ic->blocks_done = 0u;
            if (eps <= ic->tol) *stop_flag = 1;
            else if (ic->iter >= ic->max_it) *stop_flag = 2;
        }
    }
}

// One thread per (cell, group) of one problem.
__global__ __launch_bounds__(256) void k_reduce(const DevProblem *__restrict__ probs, int prob,
                                                float *__restrict__ phi_out, const float *__restrict__ phi_old,
                                                int update_source, IterCtl *__restrict__ ic,
                                                int *__restrict__ stop_flag) {
    if (stop_flag && *stop_flag) return;
    const DevProblem &P = probs[prob];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double num = 0.0, den = 0.0;
    if (t < (long long)P.C * P.G) reduce_one(P, t, phi_out, phi_old, update_source, num, den);
    if (!ic || !phi_old) return;
    residual_finish(num, den, ic, stop_flag, gridDim.x);
}

__device__ inline int block_problem(const int *__restrict__ blk_base, int nprob, int b) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk_base[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same over every problem of a batch; blocks of one problem are contiguous.
__global__ __launch_bounds__(256) void k_reduce_batch(const DevProblem *__restrict__ probs, int nprob,
                                                      const int *__restrict__ blk_base, float *const *phi_out,
                                                      float *const *phi_old, int update_source,
                                                      IterCtl *__restrict__ ic, int *__restrict__ stops) {
    const int p = block_problem(blk_base, nprob, blockIdx.x);
    if (stops[p]) return;
    const DevProblem &P = probs[p];
    // kReduceItems (cell, group) items per thread, each pass a contiguous run of
    // blockDim items: fewer blocks, so fewer residual atomics per problem
    const long long t0 = (long long)(blockIdx.x - blk_base[p]) * blockDim.x * kReduceItems + threadIdx.x;
    double num = 0.0, den = 0.0;
    const float *old = phi_old ? phi_old[p] : nullptr;
    for (int k = 0; k < kReduceItems; ++k) {
        const long long t = t0 + (long long)k * blockDim.x;
        if (t < (long long)P.C * P.G) reduce_one(P, t, phi_out[p], old, update_source, num, den);
    }
    if (!ic || !old) return;
    residual_finish(num, den, ic + p, stops + p, blk_base[p + 1] - blk_base[p]);
}

__global__ __launch_bounds__(256) void k_source_batch(const DevProblem *__restrict__ probs, int nprob,
                                                      const int *__restrict__ blk_base, float *const *phi,
                                                      const int *__restrict__ stops) {
    const int p = block_problem(blk_base, nprob, blockIdx.x);
    if (stops && stops[p]) return;
    const DevProblem &P = probs[p];
    const long long t = (long long)(blockIdx.x - blk_base[p]) * blockDim.x + threadIdx.x;
    if (t >= (long long)P.C * P.G) return;
    const int K = (int)(t / P.G);
    float ph[8], r[8];
    const float *f = phi ? phi[p] : nullptr;
#pragma unroll
    for (int j = 0; j < 8; ++j) ph[j] = f ? f[t * 8 + j] : 0.f;
    source_dofs(P.M + (size_t)K * 64, P.q[t], P.sigs[t], ph, P.qo ? P.qo + t * 8 : nullptr, r);
    float4 *out = reinterpret_cast<float4 *>(P.r + t * 8);
    out[0] = make_float4(r[0], r[1], r[2], r[3]);
    out[1] = make_float4(r[4], r[5], r[6], r[7]);
}

// dst[p] = src[p] (or zero when src[p] is NULL), [C][G][8] floats per problem.
__global__ __launch_bounds__(256) void k_copy_batch(const DevProblem *__restrict__ probs, int nprob,
                                                    const int *__restrict__ blk_base, float *const *dst,
                                                    float *const *src) {
    const int p = block_problem(blk_base, nprob, blockIdx.x);
    const DevProblem &P = probs[p];
    const long long t = (long long)(blockIdx.x - blk_base[p]) * blockDim.x + threadIdx.x;
    if (t >= (long long)P.C * P.G) return;
    const float *s = src[p];
    float *d = dst[p];
    for (int j = 0; j < 8; ++j) d[t * 8 + j] = s ? s[t * 8 + j] : 0.f;
}

__global__ void k_iter_init_batch(IterCtl *ic, int *stops, int nprob, int max_it, double tol) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    ic[p].num_bits = 0ull;
    ic[p].den_bits = 0ull;
    ic[p].blocks_done = 0u;
    ic[p].iter = 0;
    ic[p].max_it = max_it;
    ic[p].tol = tol;
    ic[p].last_eps = __builtin_inf();
    stops[p] = 0;
}

__global__ void k_iter_init(IterCtl *ic, int *stop_flag, int max_it, double tol) {
    ic->num_bits = 0ull;
    ic->den_bits = 0ull;
    ic->blocks_done = 0u;
    ic->iter = 0;
    ic->max_it = max_it;
    ic->tol = tol;
    ic->last_eps = __builtin_inf();
    *stop_flag = 0;
}

// FP64 balance: one thread per (cell, group) -> (source, absorption, leakage).
__global__ __launch_bounds__(256) void k_balance(const DevProblem *__restrict__ probs, int prob,
                                                 const float *__restrict__ phi_in, const float *__restrict__ phi_out,
                                                 double *__restrict__ partial) {
    const DevProblem &P = probs[prob];
    const int C = P.C, G = P.G, A = P.A;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double src = 0.0, ab = 0.0, lk = 0.0;
    const bool live = t < (long long)C * G;
    if (live) {
        const int K = (int)(t / G), g = (int)(t - (long long)K * G);
        const float *M = P.M + (size_t)K * 64;
        const double q = P.q[t], ss = P.sigs[t], st = P.sigt[t];
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
                const double pin = phi_in ? (double)phi_in[t * 8 + j] : 0.0;
                const double qo = P.qo ? (double)P.qo[t * 8 + j] : 0.0;   // cross-group source from phi_in
                src += (double)M[i * 8 + j] * (q + ss * pin + qo);
                ab += (double)M[i * 8 + j] * st * (double)phi_out[t * 8 + j];
            }
        const size_t cell_psi = (size_t)8 * A * G;
        for (int o = 0; o < 8; ++o) {
            const float *psi_o = P.psi + (size_t)o * C * cell_psi;
            // reflective faces of the cell and their first slot (task record words 13, 14)
            const int *rec = P.rec + ((size_t)o * C + K) * kRecWords;
            const int rmask = P.refl_in ? (rec[13] >> 24) & 63 : 0, rbase = rec[14];
            for (int a = 0; a < A; ++a) {
                const int n = o * A + a;
                // upwind faces of the octant, or of the direction under per-angle
                // designation (whose lagged faces read this sweep's neighbour trace
                // here, so the cell imbalance also measures the lag)
                const int mask = P.amask ? (int)P.amask[((size_t)o * C + K) * A + a] : (int)P.inmask[(size_t)o * C + K];
                const double ox = P.omega[3 * n], oy = P.omega[3 * n + 1], oz = P.omega[3 * n + 2];
                double L = 0.0;
                for (int f = 0; f < 6; ++f) {
                    const float *F = P.F + ((size_t)K * 6 + f) * 48;
                    const int axis = f >> 1, side = f & 1;
                    double val[4];
                    const bool in = (mask >> f) & 1;
                    const int N = P.nbr[(size_t)K * 6 + f];
                    int k = 0;
                    for (int j = 0; j < 8; ++j) {
                        if (((j >> axis) & 1) != side) continue;
                        if (!in) {
                            val[k] = psi_o[(size_t)K * cell_psi + ((size_t)j * A + a) * G + g];
                        } else if (N >= 0) {
                            const int jn = (P.perm[(size_t)K * 6 + f] >> (8 * k)) & 0xff;
                            val[k] = psi_o[(size_t)N * cell_psi + ((size_t)jn * A + a) * G + g];
                        } else if ((rmask >> f) & 1) {
                            // the mirror image's outflow that this sweep read (see the sweep kernel)
                            const int slot = rbase + __popc(rmask & ((1 << f) - 1));
                            const int om = o ^ (1 << axis);
                            val[k] = P.refl_in[((size_t)(om * P.nref + slot) * 4 + k) * A * G + (size_t)a * G + g];
                        } else {
                            val[k] = P.psib ? (double)P.psib[g] : 0.0;
                        }
                        ++k;
                    }
                    for (int kk = 0; kk < 4; ++kk)
                        for (int l = 0; l < 4; ++l)
                            L += (ox * F[kk * 4 + l] + oy * F[16 + kk * 4 + l] + oz * F[32 + kk * 4 + l]) * val[l];
                }
                lk += (double)P.w[n] * L;
            }
        }
    }
    // deterministic per-block sums per group: rows of the block in order
    __shared__ double s_v[256][4];
    double scale = fmax(fabs(src), fmax(fabs(ab), fabs(lk)));
    s_v[threadIdx.x][0] = src;
    s_v[threadIdx.x][1] = ab;
    s_v[threadIdx.x][2] = lk;
    s_v[threadIdx.x][3] = (live && scale > 0.0) ? fabs(src - ab - lk) / scale : 0.0;
    __syncthreads();
    const long long first = (long long)blockIdx.x * blockDim.x;
    if (threadIdx.x < G) {
        const int g = threadIdx.x;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            const long long tt = first + i;
            if (tt >= (long long)C * G) break;
            if ((int)(tt % G) != g) continue;
            a0 += s_v[i][0]; a1 += s_v[i][1]; a2 += s_v[i][2]; a3 = fmax(a3, s_v[i][3]);
        }
        double *out = partial + ((size_t)blockIdx.x * G + g) * 4;
        out[0] = a0; out[1] = a1; out[2] = a2; out[3] = a3;
    }
}

// Sums per-block partial[nblk][G][4] in block order (max for the last column).
__global__ void k_finish_partials(const double *__restrict__ partial, int nblk, int G, int ncol_sum,
                                  double *__restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    double acc[4] = {0, 0, 0, 0};
    for (int b = 0; b < nblk; ++b)
        for (int c = 0; c < 4; ++c) {
            const double v = partial[((size_t)b * G + g) * 4 + c];
            acc[c] = c < ncol_sum ? acc[c] + v : fmax(acc[c], v);
        }
    for (int c = 0; c < 4; ++c) out[g * 4 + c] = acc[c];
}

// Eq. 3 integrated flux: per (cell, group) sum of dofs and 1^T M phi in FP64.
__global__ __launch_bounds__(256) void k_intflux(const float *__restrict__ Mall, const float *__restrict__ phi, int C,
                                                 int G, double *__restrict__ partial) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0, v = 0.0;
    if (t < (long long)C * G) {
        const int K = (int)(t / G);
        const float *M = Mall + (size_t)K * 64;
        for (int i = 0; i < 8; ++i) {
            s += (double)phi[t * 8 + i];
            for (int j = 0; j < 8; ++j) v += (double)M[i * 8 + j] * (double)phi[t * 8 + j];
        }
    }
    __shared__ double s_v[256][2];
    s_v[threadIdx.x][0] = s;
    s_v[threadIdx.x][1] = v;
    __syncthreads();
    const long long first = (long long)blockIdx.x * blockDim.x;
    if (threadIdx.x < G) {
        const int g = threadIdx.x;
        double a0 = 0, a1 = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            const long long tt = first + i;
            if (tt >= (long long)C * G) break;
            if ((int)(tt % G) != g) continue;
            a0 += s_v[i][0];
            a1 += s_v[i][1];
        }
        double *out = partial + ((size_t)blockIdx.x * G + g) * 4;
        out[0] = a0; out[1] = a1; out[2] = 0.0; out[3] = 0.0;
    }
}

__global__ void k_fill_f32(float *p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(unsigned *p, size_t n, unsigned v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_copy_f32(float *dst, const float *src, size_t n, const int *stop_flag) {
    if (stop_flag && *stop_flag) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// psi of one (angle, group) out of the sweep's hand-off array
// [8 octants][C][8 dofs][A][G]: out[K][d], K in the caller's cell order.
__global__ void k_gather_psi(const float *__restrict__ psi, int C, int A, int G, int o, int a, int g,
                             float *__restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < 8LL * C;
         i += (long long)gridDim.x * blockDim.x) {
        const long long K = i >> 3, d = i & 7;
        out[i] = psi[(((long long)o * C + K) * 8 + d) * A * G + (long long)a * G + g];
    }
}

unsigned grid_for(size_t n, unsigned bs, unsigned cap = 65535u * 4u) {
    size_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_source(const DevProblem *probs, int prob, int C, int G, const float *phi, int *stop_flag,
                         hipStream_t s) {
    const size_t n = (size_t)C * G;
    hipLaunchKernelGGL(k_source, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, probs, prob, phi, stop_flag);
    return hipGetLastError();
}

hipError_t launch_reduce(const DevProblem *probs, int prob, int C, int G, float *phi_out, const float *phi_old,
                         bool update_source, IterCtl *ic, int *stop_flag, hipStream_t s) {
    const size_t n = (size_t)C * G;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, probs, prob, phi_out, phi_old,
                       update_source ? 1 : 0, ic, stop_flag);
    return hipGetLastError();
}

hipError_t launch_balance(const DevProblem *probs, int prob, int C, int G, const float *phi_in, const float *phi_out,
                          double *partial, double *out, hipStream_t s) {
    const size_t n = (size_t)C * G;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_balance, dim3(nblk), dim3(256), 0, s, probs, prob, phi_in, phi_out, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish_partials, dim3((G + 63) / 64), dim3(64), 0, s, partial, (int)nblk, G, 3, out);
    return hipGetLastError();
}

size_t partial_blocks(int C, int G) { return ((size_t)C * G + 255) / 256; }

hipError_t launch_integrated_flux(const float *M, const float *phi, int C, int G, double *partial, double *out,
                                  hipStream_t s) {
    const size_t n = (size_t)C * G;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_intflux, dim3(nblk), dim3(256), 0, s, M, phi, C, G, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish_partials, dim3((G + 63) / 64), dim3(64), 0, s, partial, (int)nblk, G, 4, out);
    return hipGetLastError();
}

hipError_t launch_outer_source(const DevProblem *probs, int prob, int C, int G, const float *phi, hipStream_t s,
                               const int *stop_flag) {
    const long long n = (long long)C * G;
    hipLaunchKernelGGL(k_outer_source, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, probs, prob, phi,
                       stop_flag);
    return hipGetLastError();
}

hipError_t launch_moments(const DevProblem *probs, int prob, int C, int G, const int *stop_flag, hipStream_t s) {
    const long long n = (long long)C * 8 * G;
    const size_t ylm_bytes = sizeof(float) * 8 * kMaxAnglesPerOctant * kMaxMoments;   // 32 KB at most
    hipLaunchKernelGGL(k_moments, dim3((unsigned)((n + 255) / 256)), dim3(256), ylm_bytes, s, probs, prob,
                       stop_flag);
    const long long m = (long long)C * G;
    hipLaunchKernelGGL(k_moment_sources, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, probs, prob, stop_flag);
    return hipGetLastError();
}

hipError_t launch_max_change(const float *a, const float *b, long long n, unsigned long long *out, hipStream_t s) {
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_max_change, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, size_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_gather_psi(const float *psi, int C, int A, int G, int angle, int group, float *out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_gather_psi, dim3(grid_for(8 * (size_t)C, 256)), dim3(256), 0, s, psi, C, A, G, angle / A,
                       angle % A, group, out);
    return hipGetLastError();
}
hipError_t launch_copy_f32(float *dst, const float *src, size_t n, const int *stop_flag, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n, stop_flag);
    return hipGetLastError();
}
hipError_t launch_source_batch(const DevProblem *probs, int nprob, const int *blk_base, int nblk, float *const *phi,
                               const int *stops, hipStream_t s) {
    hipLaunchKernelGGL(k_source_batch, dim3(nblk), dim3(256), 0, s, probs, nprob, blk_base, phi, stops);
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const DevProblem *probs, int nprob, const int *blk_base, int nblk,
                               float *const *phi_out, float *const *phi_old, int update_source, IterCtl *ic,
                               int *stops, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_batch, dim3(nblk), dim3(256), 0, s, probs, nprob, blk_base, phi_out, phi_old,
                       update_source, ic, stops);
    return hipGetLastError();
}

hipError_t launch_copy_batch(const DevProblem *probs, int nprob, const int *blk_base, int nblk, float *const *dst,
                             float *const *src, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_batch, dim3(nblk), dim3(256), 0, s, probs, nprob, blk_base, dst, src);
    return hipGetLastError();
}

hipError_t launch_iter_init_batch(IterCtl *ic, int *stops, int nprob, int max_it, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_iter_init_batch, dim3((nprob + 63) / 64), dim3(64), 0, s, ic, stops, nprob, max_it, tol);
    return hipGetLastError();
}

hipError_t launch_iter_init(IterCtl *ic, int *stop_flag, int max_it, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_iter_init, dim3(1), dim3(1), 0, s, ic, stop_flag, max_it, tol);
    return hipGetLastError();
}

}  // namespace snx
