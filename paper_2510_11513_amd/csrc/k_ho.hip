// Higher-order elements (orders 2 and 3): element matrices, the sweep of one
// level of the octant DAGs, the source and the angle reduction.
//
// The element is the order-p Lagrange element on a trilinear hexahedron: nodes
// at the Gauss-Lobatto-Legendre points in each reference coordinate (local node
// j = a + m b + m^2 c with m = p + 1), integrals by the m-point Gauss rule per
// direction.  The paper's benchmarks run first-, second- and third-order
// elements (Section 3.6 and its table of run times); the equations of one
// (cell, direction, group) are those of first order with N = m^3 nodes:
//     (sum_a Om_a S^a + sigma_t M - sum_{f in} Om . F_f) psi = M q - sum_{f in} (Om . F_f) psi_up.
//
// A system has N unknowns, too many for one lane's registers at N = 27 or 64,
// so a wave solves it cooperatively: lane r holds row r of the matrix and
// entry r of the right-hand side, the pivot row goes to every lane through
// LDS, and unpivoted LU (the operator's symmetric part is positive
// definite: sigma_t M plus the upwind face terms) eliminates below it.  At
// order 2 each half-wave solves its own system.
//
// These systems are far less well conditioned than the first-order ones
// (condition numbers up to ~2e3 on the 16^3 shape, where sigma_t h ~ 0.05 makes
// them streaming-dominated), and an upwind error travels downstream almost
// undamped, so a plain FP32 solve loses accuracy along every path through the
// mesh.  Each solve is therefore followed by mixed-precision iterative
// refinement: the residual b - A x is formed in FP64 against the operator
// assembled in FP64 (B = Om . S - sum Om . F kept in LDS as an FP32 pair
// hi + lo, the right-hand side's face terms from the same operators), and the
// correction reuses the FP32 LU factors, whose multipliers stay in the row
// entries that elimination leaves behind.  The streaming and face matrices
// S and F are stored in FP64: rounded separately to FP32 they no longer satisfy
// the discrete divergence identity that makes the face terms cancel on a
// constant, an error these systems amplify (M stays FP32).
#include <utility>

#include "snx_internal.h"

namespace snx {

namespace {

constexpr double kFourPi = 12.566370614359172953850573533118;

// node index j -> its index along reference axis d
template <int P> __device__ __forceinline__ int node_axis(int j, int d) {
    constexpr int m = P + 1;
    return d == 0 ? j % m : d == 1 ? (j / m) % m : j / (m * m);
}
// the two free axes of face f in increasing order
__device__ __forceinline__ void face_axes(int f, int &u, int &v) {
    const int axis = f >> 1;
    u = axis == 0 ? 1 : 0;
    v = axis == 2 ? 1 : 2;
}
// position of node j on face f (index along u + m * index along v), or -1 when
// j is not on the face
template <int P> __device__ __forceinline__ int face_pos(int f, int j) {
    int u, v;
    face_axes(f, u, v);
    if (node_axis<P>(j, f >> 1) != (f & 1) * P) return -1;
    return node_axis<P>(j, u) + (P + 1) * node_axis<P>(j, v);
}

// trilinear vertex function v and its reference gradient at xi
__device__ __forceinline__ void trilinear(int v, const double xi[3], double &f, double df[3]) {
    double h[3], dh[3];
    for (int d = 0; d < 3; ++d) {
        const double c = ((v >> d) & 1) ? 1.0 : -1.0;
        h[d] = 0.5 * (1.0 + c * xi[d]);
        dh[d] = 0.5 * c;
    }
    f = h[0] * h[1] * h[2];
    df[0] = dh[0] * h[1] * h[2];
    df[1] = h[0] * dh[1] * h[2];
    df[2] = h[0] * h[1] * dh[2];
}

// Lagrange polynomial a of the nodes at x, and its derivative
template <int P> __device__ __forceinline__ void lagrange(const double *node, int a, double x, double &val,
                                                          double &der) {
    double v = 1.0, d = 0.0;
    for (int b = 0; b <= P; ++b) {
        if (b == a) continue;
        const double den = node[a] - node[b];
        d = d * (x - node[b]) / den + v / den;   // product rule, one factor at a time
        v *= (x - node[b]) / den;
    }
    val = v;
    der = d;
}

// ------------------------------------------------------------------ geometry

// One workgroup per cell: M_ij = int phi_i phi_j dV and
// S^a_ij = int phi_i d phi_j / d x_a dV in FP64 by the m^3-point Gauss rule.
template <int P>
__global__ __launch_bounds__(256) void k_ho_volume(const double *__restrict__ xyz, const int *__restrict__ cv, HoRef ref,
                                                   float *__restrict__ M, double *__restrict__ S, int *__restrict__ err) {
    constexpr int m = P + 1, N = m * m * m, Q = m * m * m;
    const int K = blockIdx.x, tid = threadIdx.x;
    __shared__ double sX[8][3];
    __shared__ double sWd[Q], sJi[Q][9];   // weight * det J; (J^-1)[b][a] = d xi_b / d x_a at [b * 3 + a]
    __shared__ double sL[m][m], sD[m][m];  // Lagrange value / derivative of node a at Gauss point t
    if (tid < 24) sX[tid / 3][tid % 3] = xyz[3 * (size_t)cv[8 * (size_t)K + tid / 3] + tid % 3];
    if (tid < m * m) lagrange<P>(ref.node, tid / m, ref.gx[tid % m], sL[tid / m][tid % m], sD[tid / m][tid % m]);
    __syncthreads();
    if (tid < Q) {
        const int qa = tid % m, qb = (tid / m) % m, qc = tid / (m * m);
        const double xi[3] = {ref.gx[qa], ref.gx[qb], ref.gx[qc]};
        double J[3][3] = {};
        for (int v = 0; v < 8; ++v) {
            double f, df[3];
            trilinear(v, xi, f, df);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) J[a][b] += sX[v][a] * df[b];
        }
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        const double c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        const double det = J[0][0] * c00 + J[1][0] * c01 + J[2][0] * c02;
        if (!(det > 0.0)) atomicOr(err, 1);
        const double id = 1.0 / det;
        // inverse by the adjugate: inv[b][a]
        sJi[tid][0] = c00 * id;
        sJi[tid][1] = c01 * id;
        sJi[tid][2] = c02 * id;
        sJi[tid][3] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
        sJi[tid][4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        sJi[tid][5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        sJi[tid][6] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
        sJi[tid][7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        sJi[tid][8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
        sWd[tid] = ref.gw[qa] * ref.gw[qb] * ref.gw[qc] * det;
    }
    __syncthreads();
    for (int e = tid; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        const int ia = node_axis<P>(i, 0), ib = node_axis<P>(i, 1), ic = node_axis<P>(i, 2);
        const int ja = node_axis<P>(j, 0), jb = node_axis<P>(j, 1), jc = node_axis<P>(j, 2);
        double mm = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < Q; ++q) {
            const int qa = q % m, qb = (q / m) % m, qc = q / (m * m);
            const double wp = sWd[q] * sL[ia][qa] * sL[ib][qb] * sL[ic][qc];
            const double la = sL[ja][qa], lb = sL[jb][qb], lc = sL[jc][qc];
            const double g0 = sD[ja][qa] * lb * lc, g1 = la * sD[jb][qb] * lc, g2 = la * lb * sD[jc][qc];
            const double *Ji = sJi[q];
            mm += wp * la * lb * lc;
            s0 += wp * (Ji[0] * g0 + Ji[3] * g1 + Ji[6] * g2);
            s1 += wp * (Ji[1] * g0 + Ji[4] * g1 + Ji[7] * g2);
            s2 += wp * (Ji[2] * g0 + Ji[5] * g1 + Ji[8] * g2);
        }
        const size_t NN = (size_t)N * N;
        M[K * NN + e] = (float)mm;
        S[(3 * (size_t)K + 0) * NN + e] = s0;
        S[(3 * (size_t)K + 1) * NN + e] = s1;
        S[(3 * (size_t)K + 2) * NN + e] = s2;
    }
}

// One workgroup per (cell, face): F^a_kl = int_f n_a phi_k phi_l dA over the
// face's nodes by the m^2-point Gauss rule, n dA = +-(dx/du x dx/dv) outward.
// An interior face is integrated on the side with the smaller (cell, face)
// index, which also writes the negated values at the neighbour's nodes.
template <int P>
__global__ __launch_bounds__(256) void k_ho_faces(const double *__restrict__ xyz, const int *__restrict__ cv,
                                                  const int *__restrict__ nbr, const int *__restrict__ nbrf,
                                                  const int *__restrict__ hoperm, HoRef ref, double *__restrict__ F) {
    constexpr int m = P + 1, NF = m * m, QF = m * m;
    const int K = blockIdx.x / 6, f = blockIdx.x % 6, tid = threadIdx.x;
    const int Nb = nbr[6 * K + f], g = nbrf[6 * K + f];
    if (Nb >= 0 && 6 * Nb + g < 6 * K + f) return;   // the neighbour's side writes this face
    __shared__ double sX[8][3], sN[QF][3], sL[m][m];
    if (tid < 24) sX[tid / 3][tid % 3] = xyz[3 * (size_t)cv[8 * (size_t)K + tid / 3] + tid % 3];
    if (tid < m * m) {
        double d;
        lagrange<P>(ref.node, tid / m, ref.gx[tid % m], sL[tid / m][tid % m], d);
    }
    __syncthreads();
    const int axis = f >> 1, side = f & 1;
    int u, v;
    face_axes(f, u, v);
    if (tid < QF) {
        const int qu = tid % m, qv = tid / m;
        double xi[3];
        xi[axis] = side ? 1.0 : -1.0;
        xi[u] = ref.gx[qu];
        xi[v] = ref.gx[qv];
        double tu[3] = {0, 0, 0}, tv[3] = {0, 0, 0};
        for (int vv = 0; vv < 8; ++vv) {
            double fv, df[3];
            trilinear(vv, xi, fv, df);
            for (int a = 0; a < 3; ++a) {
                tu[a] += sX[vv][a] * df[u];
                tv[a] += sX[vv][a] * df[v];
            }
        }
        // dx/du x dx/dv points along +xi_axis for axes 0 and 2, along -xi_axis for axis 1
        const double sgn = (axis == 1 ? -1.0 : 1.0) * (side ? 1.0 : -1.0) * ref.gw[qu] * ref.gw[qv];
        sN[tid][0] = sgn * (tu[1] * tv[2] - tu[2] * tv[1]);
        sN[tid][1] = sgn * (tu[2] * tv[0] - tu[0] * tv[2]);
        sN[tid][2] = sgn * (tu[0] * tv[1] - tu[1] * tv[0]);
    }
    __syncthreads();
    if (tid >= NF * NF) return;
    const int k = tid / NF, l = tid % NF;
    // face node at position k: index k % m along u, k / m along v (its factor along the axis is 1 on the face)
    double F3[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < QF; ++q) {
        const int qu = q % m, qv = q / m;
        const double pk = sL[k % m][qu] * sL[k / m][qv], pl = sL[l % m][qu] * sL[l / m][qv];
        for (int a = 0; a < 3; ++a) F3[a] += sN[q][a] * pk * pl;
    }
    const size_t FF = (size_t)NF * NF;
    for (int a = 0; a < 3; ++a) F[((6 * (size_t)K + f) * 3 + a) * FF + tid] = F3[a];
    if (Nb < 0) return;
    const int pk = face_pos<P>(g, hoperm[(6 * (size_t)K + f) * NF + k]);
    const int pl = face_pos<P>(g, hoperm[(6 * (size_t)K + f) * NF + l]);
    if (pk < 0 || pl < 0) return;   // not produced by the host's node maps; kept out of bounds-unsafe writes
    for (int a = 0; a < 3; ++a) F[((6 * (size_t)Nb + g) * 3 + a) * FF + pk * NF + pl] = -F3[a];
}

// --------------------------------------------------------------------- sweep

// Orders LDS accesses of one wave: what a lane wrote before is seen by every
// lane after.  A wave's LDS instructions execute in issue order, so keeping
// the compiler from moving memory accesses across this point is enough.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Elimination step k of the unpivoted LU by rows: lane k broadcasts its row
// (columns k.., and its right-hand side at [N]) through LDS, every lane below
// takes column k out of its own row.  A template per step keeps every row
// index static, so the row stays in registers.
constexpr int kChunks = 4;   // 16-byte pivot chunks (of each pivot row) loaded ahead at order 3

template <int N, int k>
__device__ __forceinline__ void lu_step(float (&row)[N], float &b, float *piv, int r) {
    if (r == k) {   // whole 16-byte chunks from the one holding column k (entries left of k go unread)
        float4 *w4 = reinterpret_cast<float4 *>(piv);
#pragma unroll
        for (int c = k / 4; c < (N + 3) / 4; ++c) {
            const int j = 4 * c;
            w4[c] = make_float4(row[j], j + 1 < N ? row[j + 1] : 0.f, j + 2 < N ? row[j + 2] : 0.f,
                                j + 3 < N ? row[j + 3] : 0.f);
        }
        piv[N] = b;
    }
    wave_lds_sync();
    const float4 *piv4 = reinterpret_cast<const float4 *>(piv);
    const float l = r > k ? row[k] * __builtin_amdgcn_rcpf(piv[k]) : 0.f;
#pragma unroll
    for (int c = (k + 1) / 4; c < (N + 3) / 4; ++c) {
        const float4 v = piv4[c];
        const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * c + e;
            if (j > k && j < N) row[j] = __builtin_fmaf(-l, vv[e], row[j]);
        }
        // at most kChunks pivot chunks in flight: fewer live registers, more resident waves
        if (N > 32 && (c + 1) % kChunks == 0) __builtin_amdgcn_sched_barrier(0);
    }
    b = __builtin_fmaf(-l, piv[N], b);
    // the next step's write comes after these reads in issue order
}
// Two elimination steps, pivots k and k+1, with one LDS round trip: lanes k
// and k+1 broadcast their rows, every lane forms row k+1 with column k
// eliminated from the two (its multiplier m1 and pivot d), then takes columns
// k and k+1 out of its own row at once: row -= c0 row_k + c1 row_k+1, with
// c1 = l1 and c0 = l0 - l1 m1 (l0, l1 its own multipliers).  Lane k+1 itself
// only takes out column k.  Same arithmetic as two single steps, up to
// rounding order.
template <int N, int LP, int k, bool KEEP>
__device__ __forceinline__ void lu_step2(float (&row)[N], float &b, float *piv, int r) {
    float *piv1 = piv + LP;
    if (r == k || r == k + 1) {
        float4 *w4 = reinterpret_cast<float4 *>(r == k ? piv : piv1);
#pragma unroll
        for (int c = k / 4; c < (N + 3) / 4; ++c) {
            const int j = 4 * c;
            w4[c] = make_float4(row[j], j + 1 < N ? row[j + 1] : 0.f, j + 2 < N ? row[j + 2] : 0.f,
                                j + 3 < N ? row[j + 3] : 0.f);
        }
        (r == k ? piv : piv1)[N] = b;
    }
    wave_lds_sync();
    const float4 *p0 = reinterpret_cast<const float4 *>(piv);
    const float4 *p1 = reinterpret_cast<const float4 *>(piv1);
    const float pk = piv[k], pk1 = piv[k + 1], qk = piv1[k], qk1 = piv1[k + 1];
    const float ipk = __builtin_amdgcn_rcpf(pk);
    const float m1 = qk * ipk;                                  // row k+1's multiplier of row k
    const float d = __builtin_fmaf(-m1, pk1, qk1);              // row k+1's pivot after that
    const float l0 = row[k] * ipk;
    const float l1 = __builtin_fmaf(-l0, pk1, row[k + 1]) * __builtin_amdgcn_rcpf(d);
    const float c0 = r > k + 1 ? __builtin_fmaf(-l1, m1, l0) : (r == k + 1 ? m1 : 0.f);
    const float c1 = r > k + 1 ? l1 : 0.f;
    // The multipliers go where this step leaves nothing of use (columns k and
    // k+1 of the rows below the pivots are never read again), for the
    // refinement's replay: c1 as column k+1 is updated, c0 after the loop.
#pragma unroll
    for (int c = (k + 1) / 4; c < (N + 3) / 4; ++c) {
        const float4 v = p0[c], w = p1[c];
        const float vv[4] = {v.x, v.y, v.z, v.w}, ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * c + e;
            if (j > k && j < N) {
                const float u = __builtin_fmaf(-c1, ww[e], __builtin_fmaf(-c0, vv[e], row[j]));
                row[j] = (KEEP && j == k + 1 && r > k + 1) ? c1 : u;
            }
        }
        if (N > 32 && (c + 1) % kChunks == 0) __builtin_amdgcn_sched_barrier(0);
    }
    b = __builtin_fmaf(-c1, piv1[N], __builtin_fmaf(-c0, piv[N], b));
    if constexpr (KEEP) row[k] = r > k ? c0 : row[k];
}

// x_k of lane k (or H + k in the upper half-wave) for every lane of its system
template <int H>
__device__ __forceinline__ float from_lane(float v, int k, int half) {
    const int bits = __builtin_bit_cast(int, v);
    if constexpr (H == 64) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(bits, k));
    } else {
        const float v0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(bits, k));
        const float v1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(bits, H + k));
        return half ? v1 : v0;
    }
}

// The elimination of the pivot pair (k, k+1) replayed on a new right-hand side
// with the stored multipliers: lane k+1 takes out m1 b_k, the lanes below
// c0 b_k + c1 b_k+1 (b_k+1 as it was before lane k+1's own update).
template <int N, int H, int k>
__device__ __forceinline__ void replay_step2(const float (&row)[N], float &b, int r, int half) {
    const float bk = from_lane<H>(b, k, half), bk1 = from_lane<H>(b, k + 1, half);
    const float c0 = r > k ? row[k] : 0.f;
    const float c1 = r > k + 1 ? row[k + 1] : 0.f;
    b = __builtin_fmaf(-c1, bk1, __builtin_fmaf(-c0, bk, b));
}

// Back substitution, column k = N-1-i: lane k finishes x_k, which every lane
// of its system reads straight from lane k's register (no LDS round trip),
// and the rows above take it out.  H: lanes per system (32: two systems per wave).
template <int N, int H, int i>
__device__ __forceinline__ void back_step(const float (&row)[N], float &b, float &x, int r, int half) {
    constexpr int k = N - 1 - i;
    const int cand = __builtin_bit_cast(int, b * __builtin_amdgcn_rcpf(row[k]));   // x_k in lane k
    float xk;
    if constexpr (H == 64) {
        xk = __builtin_bit_cast(float, __builtin_amdgcn_readlane(cand, k));
    } else {
        const float x0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(cand, k));
        const float x1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(cand, H + k));
        xk = half ? x1 : x0;
    }
    if (r == k) x = xk;
    b = __builtin_fmaf(r < k ? -row[k] : 0.f, xk, b);
}
template <int N, int H, int LP, bool KEEP, int... K, int... I>
__device__ __forceinline__ void lu_solve(float (&row)[N], float &b, float &x, float *piv, int r, int half,
                                         std::integer_sequence<int, K...>, std::integer_sequence<int, I...>) {
    (lu_step2<N, LP, 2 * I, KEEP>(row, b, piv, r), ...);       // pivots in pairs
    if constexpr (N % 2) lu_step<N, N - 1>(row, b, piv, r);      // the odd last one (no row below it)
    (back_step<N, H, K>(row, b, x, r, half), ...);
}
// A second solve with the factors of lu_solve: forward elimination replayed
// pair by pair, then back substitution.
template <int N, int H, int... K, int... I>
__device__ __forceinline__ void lu_resolve(const float (&row)[N], float &b, float &x, int r, int half,
                                           std::integer_sequence<int, K...>, std::integer_sequence<int, I...>) {
    (replay_step2<N, H, 2 * I>(row, b, r, half), ...);
    (back_step<N, H, K>(row, b, x, r, half), ...);
}

// One workgroup per (task, direction) of a level: B = Om . S - sum_{f in}
// Om . F_f and M go to LDS once, then the workgroup's wave halves solve the
// direction's groups, one system each.
template <int P, int REFINE>
__device__ __forceinline__ void ho_sweep_body(const HoDev &D, int begin) {
    constexpr int m = P + 1, N = m * m * m, NF = m * m;
    constexpr int LD = (N % 2 == 0) ? N + 1 : N + 2;        // odd row stride: lanes' rows sit in different banks
    constexpr int LP = ((N + 1) + 3) / 4 * 4;               // pivot buffer: row and rhs, 16-byte aligned
    constexpr int H = N <= 32 ? 32 : 64, SPW = 64 / H, SPB = 4 * SPW;
    __shared__ float sB[N * LD], sBlo[N * LD], sM[N * LD];   // B = hi + lo (FP64 assembly)
    __shared__ float sOF[6][NF * NF], sOFlo[6][NF * NF];     // Om . F_f = hi + lo (FP64 assembly)
    __shared__ __align__(16) float sPiv[4 * SPW][2 * LP];   // pivot rows k and k+1

    const int A = D.A, C = D.C, G = D.G;
    const int t = begin + (int)(blockIdx.x / (unsigned)A), dir = (int)(blockIdx.x % (unsigned)A);
    const int task = D.tasks[t];
    const int K = task >> 3, o = task & 7, n = o * A + dir;
    const int mask = D.inmask[(size_t)o * C + K];
    const double dx = D.omega64[3 * n], dy = D.omega64[3 * n + 1], dz = D.omega64[3 * n + 2];
    const int tid = threadIdx.x;
    const size_t NN = (size_t)N * N, FF = (size_t)NF * NF;
    const double *S = D.S + 3 * (size_t)K * NN;
    const float *Mk = D.M + (size_t)K * NN;
    const double *Fk = D.F + 6 * 3 * (size_t)K * FF;

    for (int e = tid; e < N * N; e += 256) {
        const int i = e / N, j = e % N;
        double b = dx * S[e] + dy * S[NN + e] + dz * S[2 * NN + e];
        for (int f = 0; f < 6; ++f) {
            if (!((mask >> f) & 1)) continue;
            const int pi = face_pos<P>(f, i), pj = face_pos<P>(f, j);
            if (pi < 0 || pj < 0) continue;
            const double *Ff = Fk + (size_t)f * 3 * FF + pi * NF + pj;
            b -= dx * Ff[0] + dy * Ff[FF] + dz * Ff[2 * FF];
        }
        const float hi = (float)b;
        sB[i * LD + j] = hi;
        sBlo[i * LD + j] = (float)(b - (double)hi);
        sM[i * LD + j] = Mk[e];
    }
    for (int e = tid; e < 6 * NF * NF; e += 256) {
        const int f = e / (NF * NF), kl = e % (NF * NF);
        if (!((mask >> f) & 1)) continue;
        const double *Ff = Fk + (size_t)f * 3 * FF + kl;
        const double of = dx * Ff[0] + dy * Ff[FF] + dz * Ff[2 * FF];
        const float hi = (float)of;
        sOF[f][kl] = hi;
        sOFlo[f][kl] = (float)(of - (double)hi);
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int half = lane / H, r = lane % H;
    const int rr = r < N ? r : N - 1;                        // lanes past the last row compute on a copy of it
    float *piv = sPiv[wave * SPW + half];
    int fpos[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) fpos[f] = ((mask >> f) & 1) ? face_pos<P>(f, rr) : -1;

    for (int g0 = 0; g0 < G; g0 += SPB) {
        const int g = g0 + wave * SPW + half;
        const bool valid = g < G && r < N;
        const int gg = g < G ? g : G - 1;
        const float sig = D.sigt[(size_t)K * G + gg];
        float row[N];
#pragma unroll
        for (int j = 0; j < N; ++j) row[j] = __builtin_fmaf(sig, sM[rr * LD + j], sB[rr * LD + j]);
        // right-hand side in FP64 with the same face operators as the matrix (an
        // FP32 one would break the exact cancellation of the face terms on a
        // constant solution)
        double bd = (double)D.R[((size_t)K * G + gg) * N + rr];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (fpos[f] < 0) continue;
            const int nb = D.nbr[6 * K + f];
            const float *of = sOF[f] + fpos[f] * NF, *ofl = sOFlo[f] + fpos[f] * NF;
            if (nb >= 0) {
                const float *up = D.psi + (((size_t)n * C + nb) * G + gg) * N;
                const int *pm = D.perm + (6 * (size_t)K + f) * NF;
                for (int l = 0; l < NF; ++l) bd -= ((double)of[l] + (double)ofl[l]) * (double)up[pm[l]];
            } else {
                const double pb = D.psib ? (double)D.psib[gg] : 0.0;
                double s = 0.0;
                for (int l = 0; l < NF; ++l) s += (double)of[l] + (double)ofl[l];
                bd -= s * pb;
            }
        }
        const double b0 = bd;
        float b = (float)bd;
        float x = 0.f;
        lu_solve<N, H, LP, (REFINE > 0)>(row, b, x, piv, r, half, std::make_integer_sequence<int, N>{},
                           std::make_integer_sequence<int, N / 2>{});
        // refinement: residual in FP64 against sigma_t M + (B hi + lo), then the
        // correction from the same factors.  x reaches every lane of the system
        // through its pivot buffer (a wave's LDS accesses run in issue order).
#pragma unroll 1
        for (int it = 0; it < REFINE; ++it) {
            if (r < N) piv[r] = x;
            wave_lds_sync();
            const float4 *x4 = reinterpret_cast<const float4 *>(piv);
            double res = b0;
#pragma unroll 1
            for (int c = 0; c < (N + 3) / 4; ++c) {
                const float4 xv = x4[c];
                const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = 4 * c + e;
                    if (j < N) {
                        const double a = (double)sig * (double)sM[rr * LD + j] +
                                         ((double)sB[rr * LD + j] + (double)sBlo[rr * LD + j]);
                        res = __builtin_fma(-a, (double)xs[e], res);
                    }
                }
            }
            float rb = (float)res, dxk = 0.f;
            lu_resolve<N, H>(row, rb, dxk, r, half, std::make_integer_sequence<int, N>{},
                             std::make_integer_sequence<int, N / 2>{});
            x += dxk;
            wave_lds_sync();      // every lane has read the old x before the next write
        }
        if (valid) D.psi[(((size_t)n * C + K) * G + g) * N + r] = x;
    }
}

// One kernel per order, each with one refinement step.  With pivots in pairs
// order 3 runs fastest at two waves per SIMD (each with twice the work between
// LDS round trips); the refinement's replay keeps the multipliers alive, so
// holding it there spills a few registers.
__global__ __launch_bounds__(256) void k_ho_sweep2(HoDev D, int begin) { ho_sweep_body<2, 1>(D, begin); }
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_ho_sweep3(HoDev D, int begin) {
    ho_sweep_body<3, 1>(D, begin);
}

// R = M (Q + sigma_s phi) / (4 pi) at every (cell, group, node); phi NULL = zero
__global__ __launch_bounds__(256) void k_ho_source(const float *__restrict__ M, const float *__restrict__ q,
                                                   const float *__restrict__ sigs, const float *__restrict__ phi,
                                                   float *__restrict__ R, int C, int G, int N) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)C * G * N) return;
    const long long kg = e / N;
    const int i = (int)(e % N), K = (int)(kg / G);
    const float Q = q[kg], ss = sigs[kg];
    const float *Mi = M + ((size_t)K * N + i) * N;
    const float *ph = phi ? phi + kg * N : nullptr;
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += (double)Mi[j] * (double)(ph ? Q + ss * ph[j] : Q);
    R[e] = (float)(s / kFourPi);
}

// phi = sum_n w_n psi_n at every (cell, group, node), in increasing n, FP64
__global__ __launch_bounds__(256) void k_ho_reduce(const float *__restrict__ psi, const float *__restrict__ w, int nang,
                                                   long long cgn, float *__restrict__ phi) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cgn) return;
    double s = 0.0;
    for (int n = 0; n < nang; ++n) s += (double)w[n] * (double)psi[(size_t)n * cgn + e];
    phi[e] = (float)s;
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_ho_geometry(int P, const double *xyz, const int *cv, const int *nbr, const int *nbrf,
                              const int *hoperm, int C, const HoRef &ref, float *M, double *S, double *F, int *err,
                              hipStream_t s) {
    if (P == 2) {
        hipLaunchKernelGGL(k_ho_volume<2>, dim3(C), dim3(256), 0, s, xyz, cv, ref, M, S, err);
        hipLaunchKernelGGL(k_ho_faces<2>, dim3(6 * C), dim3(256), 0, s, xyz, cv, nbr, nbrf, hoperm, ref, F);
    } else if (P == 3) {
        hipLaunchKernelGGL(k_ho_volume<3>, dim3(C), dim3(256), 0, s, xyz, cv, ref, M, S, err);
        hipLaunchKernelGGL(k_ho_faces<3>, dim3(6 * C), dim3(256), 0, s, xyz, cv, nbr, nbrf, hoperm, ref, F);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ho_sweep_level(int P, const HoDev &D, int begin, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const dim3 grid((unsigned)count * (unsigned)D.A);
    if (P == 2) hipLaunchKernelGGL(k_ho_sweep2, grid, dim3(256), 0, s, D, begin);
    else if (P == 3) hipLaunchKernelGGL(k_ho_sweep3, grid, dim3(256), 0, s, D, begin);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ho_source(const float *M, const float *q, const float *sigs, const float *phi, float *R, int C,
                            int G, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_ho_source, dim3(blocks_for((long long)C * G * N)), dim3(256), 0, s, M, q, sigs, phi, R, C,
                       G, N);
    return hipGetLastError();
}

hipError_t launch_ho_reduce(const float *psi, const float *w, int nang, long long cgn, float *phi, hipStream_t s) {
    hipLaunchKernelGGL(k_ho_reduce, dim3(blocks_for(cgn)), dim3(256), 0, s, psi, w, nang, cgn, phi);
    return hipGetLastError();
}

}  // namespace snx
