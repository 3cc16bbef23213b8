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
// assembled in FP64 (B = Om . S - sum Om . F kept in LDS in FP64, the
// right-hand side's face terms from the same FP64 operators), and the
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

// 16-byte pivot chunks (of each pivot row) loaded ahead at order 3; the order-3
// sweep takes 126.3 ms at 3, 126.9 at 2, 128.2 at 4, 134 at 8 and 135 at 1.
constexpr int kChunks = 3;
// Each lane keeps the inverse of its own pivot from the elimination (one select
// per step) instead of every lane taking a reciprocal at every back-substitution
// step, twice per system with the refinement.  That pays at order 3 (64 rows,
// 6 % faster); at order 2 the extra selects cost more than the 27 reciprocals
// (3 % slower), so there the back substitution takes the reciprocals.
template <int N> constexpr bool kKeepInversePivot = N > 32;

// Elimination step k of the unpivoted LU by rows: lane k broadcasts its row
// (columns k.., and its right-hand side at [N]) through LDS, every lane below
// takes column k out of its own row.  A template per step keeps every row
// index static, so the row stays in registers.
template <int N, int k>
__device__ __forceinline__ void lu_step(float (&row)[N], float &b, float &idg, float *piv, int r) {
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
    const float ip = __builtin_amdgcn_rcpf(piv[k]);
    const float l = r > k ? row[k] * ip : 0.f;
    if constexpr (kKeepInversePivot<N>) {
        idg = r == k ? ip : idg;
        asm volatile("" : "+v"(idg));
    }
#pragma unroll
    for (int c = (k + 1) / 4; c < (N + 3) / 4; ++c) {
        const float4 v = piv4[c];
        const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * c + e;
            if (j > k && j < N) row[j] = __builtin_fmaf(-l, vv[e], row[j]);
        }
        // at most kChunks pivot chunks in flight: fewer live registers
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
__device__ __forceinline__ void lu_step2(float (&row)[N], float &b, float &idg, float *piv, int r) {
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
    const float id = __builtin_amdgcn_rcpf(d);
    const float l1 = __builtin_fmaf(-l0, pk1, row[k + 1]) * id;
    if constexpr (kKeepInversePivot<N>) {
        idg = r == k ? ipk : (r == k + 1 ? id : idg);           // the lane's own inverse pivot
        asm volatile("" : "+v"(idg));   // taken here: the pivots need not stay live to the back substitution
    }
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

// v_writelane_b32 (lane `lane` of `old` takes the uniform `val`), reached through
// its LLVM intrinsic, which this compiler has no builtin for; being the
// intrinsic, the compiler knows it and inserts its hazard waits.
extern "C" __device__ int snx_writelane_i32(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// Back substitution, column k = N-1-i: lane k finishes x_k, which every lane
// of its system reads straight from lane k's register (no LDS round trip) and
// which is written into lane k of x; the rows above take it out.  The lanes at
// and below k hold their x already and never read b again, so they take out
// the same product unmasked.  H: lanes per system (32: two systems per wave).
template <int N, int H, int i>
__device__ __forceinline__ void back_step(const float (&row)[N], float idg, float &b, float &x, int half) {
    constexpr int k = N - 1 - i;
    const float inv = kKeepInversePivot<N> ? idg : __builtin_amdgcn_rcpf(row[k]);
    const int cand = __builtin_bit_cast(int, b * inv);   // x_k in lane k
    int xi = __builtin_bit_cast(int, x);
    float xk;
    if constexpr (H == 64) {
        const int s = __builtin_amdgcn_readlane(cand, k);
        xi = snx_writelane_i32(s, k, xi);
        xk = __builtin_bit_cast(float, s);
    } else {
        const int s0 = __builtin_amdgcn_readlane(cand, k), s1 = __builtin_amdgcn_readlane(cand, H + k);
        xi = snx_writelane_i32(s0, k, xi);
        xi = snx_writelane_i32(s1, H + k, xi);
        xk = __builtin_bit_cast(float, half ? s1 : s0);
    }
    x = __builtin_bit_cast(float, xi);
    b = __builtin_fmaf(-row[k], xk, b);
}
template <int N, int H, int LP, bool KEEP, int... K, int... I>
__device__ __forceinline__ void lu_solve(float (&row)[N], float &b, float &x, float &idg, float *piv, int r,
                                         int half, std::integer_sequence<int, K...>,
                                         std::integer_sequence<int, I...>) {
    (lu_step2<N, LP, 2 * I, KEEP>(row, b, idg, piv, r), ...);  // pivots in pairs
    if constexpr (N % 2) lu_step<N, N - 1>(row, b, idg, piv, r); // the odd last one (no row below it)
    asm volatile("" : "+v"(r), "+v"(half));                      // fresh lane masks for this pass
    (back_step<N, H, K>(row, idg, b, x, half), ...);
}
// A second solve with the factors of lu_solve: forward elimination replayed
// pair by pair, then back substitution.
template <int N, int H, int... K, int... I>
__device__ __forceinline__ void lu_resolve(const float (&row)[N], float idg, float &b, float &x, int r, int half,
                                           std::integer_sequence<int, K...>, std::integer_sequence<int, I...>) {
    (replay_step2<N, H, 2 * I>(row, b, r, half), ...);
    asm volatile("" : "+v"(r), "+v"(half));
    (back_step<N, H, K>(row, idg, b, x, half), ...);
}

// Node of face f at face position (pu, pv): the face's axis coordinate fixed at
// its side, the two free axes in increasing order (the inverse of face_pos).
template <int P> __device__ __forceinline__ int face_node(int f, int pu, int pv) {
    constexpr int m = P + 1;
    int u, v;
    face_axes(f, u, v);
    const int stride[3] = {1, m, m * m};
    return (f & 1) * P * stride[f >> 1] + pu * stride[u] + pv * stride[v];
}

// One workgroup per (task, direction) of a level: B = Om . S - sum_{f in}
// Om . F_f and M go to LDS once, then the workgroup's waves (order 3) or wave
// halves (order 2) solve the direction's groups, one system each.
//
// Every global load a system needs comes one group ahead: the source dofs,
// sigma_t and the upwind traces of the next group are requested before the
// current group's solve and land during it (the traces through a small LDS
// buffer per system, since every row of a system reads all of them).  The
// element data are requested all at once before any is used.
template <int P, int REFINE>
__device__ __forceinline__ void ho_sweep_body(const HoDev &D, int begin) {
    constexpr int m = P + 1, N = m * m * m, NF = m * m;
    constexpr int LD = (N % 2 == 0) ? N + 1 : N + 2;        // odd row stride: lanes' rows sit in different banks
    constexpr int LP = ((N + 1) + 3) / 4 * 4;               // pivot buffer: row and rhs, 16-byte aligned
    constexpr int H = N <= 32 ? 32 : 64, SPW = 64 / H, SPB = 4 * SPW;
    constexpr int NN = N * N, FF = NF * NF, PER = (NN + 255) / 256;
    static_assert(FF <= 256 && 6 * NF <= 2 * H, "one face entry per thread, two trace slots per lane");
    __shared__ double sB[N * LD];                             // B in FP64
    __shared__ float sM[N * LD];
    __shared__ double sOF[6][FF];                             // Om . F_f of the inflow faces in FP64
    __shared__ __align__(16) float sPiv[4 * SPW][2 * LP];    // pivot rows k and k+1; x (FP64) for the residual
    __shared__ float sTr[4 * SPW][6 * NF];                    // each system's upwind traces, inflow-face order
    __shared__ int sPm[6][NF], sNb[6], sFl[6];

    const int A = D.A, C = D.C, G = D.G;
    const int t = begin + (int)(blockIdx.x / (unsigned)A), dir = (int)(blockIdx.x % (unsigned)A);
    const int task = D.tasks[t];
    const int K = task >> 3, o = task & 7, n = o * A + dir;
    const int mask = D.inmask[(size_t)o * C + K];
    const int nin = __popc(mask);
    const double dx = D.omega64[3 * n], dy = D.omega64[3 * n + 1], dz = D.omega64[3 * n + 2];
    const int tid = threadIdx.x;
    const double *S = D.S + 3 * (size_t)K * NN;
    const float *Mk = D.M + (size_t)K * NN;
    const double *Fk = D.F + 6 * 3 * (size_t)K * FF;

    // element data: every load in flight before the first use
    double s0[PER], s1[PER], s2[PER];
    float mv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (e < NN) {
            s0[q] = S[e];
            s1[q] = S[NN + e];
            s2[q] = S[2 * NN + e];
            mv[q] = Mk[e];
        }
    }
    double fo[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        fo[f] = 0.0;
        if (((mask >> f) & 1) && tid < FF) {
            const double *Ff = Fk + (size_t)f * 3 * FF + tid;
            fo[f] = dx * Ff[0] + dy * Ff[FF] + dz * Ff[2 * FF];
        }
    }
    if (tid < 6 * NF) {
        const int f = tid / NF;
        sPm[f][tid % NF] = ((mask >> f) & 1) ? D.perm[(6 * (size_t)K + f) * NF + tid % NF] : 0;
    }
    if (tid < 6) {
        sNb[tid] = D.nbr[6 * K + tid];
        int mm = mask;
        for (int k = 0; k < tid && mm; ++k) mm &= mm - 1;
        sFl[tid] = mm ? __builtin_ctz(mm) : 0;             // the tid-th inflow face
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (e < NN) {
            const int i = e / N, j = e % N;
            sB[i * LD + j] = dx * s0[q] + dy * s1[q] + dz * s2[q];
            sM[i * LD + j] = mv[q];
        }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f)
        if (((mask >> f) & 1) && tid < FF) sOF[f][tid] = fo[f];
    __syncthreads();
    // the inflow faces' terms, one face at a time (faces share edge nodes)
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!((mask >> f) & 1)) continue;
        if (tid < FF) {
            const int pi = tid / NF, pj = tid % NF;
            const int i = face_node<P>(f, pi % m, pi / m), j = face_node<P>(f, pj % m, pj / m);
            sB[i * LD + j] -= fo[f];
        }
        __syncthreads();
    }

    const int lane = tid & 63, wave = tid >> 6;
    const int half = lane / H, r = lane % H;
    const int rr = r < N ? r : N - 1;                        // lanes past the last row compute on a copy of it
    const int sys = wave * SPW + half;
    float *piv = sPiv[sys];
    float *tr = sTr[sys];
    int fpos[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) fpos[f] = ((mask >> f) & 1) ? face_pos<P>(f, rr) : -1;

    // this lane's two trace slots: inflow face k = s / NF (in face order), node l = s % NF
    const int ntr = nin * NF;
    auto trace = [&](int s, int g) -> float {
        if (s >= ntr) return 0.f;
        const int f = sFl[s / NF], nb = sNb[f];
        if (nb < 0) return D.psib ? D.psib[g] : 0.f;
        return D.psi[(((size_t)n * C + nb) * G + g) * N + sPm[f][s % NF]];
    };
    float a0, a1, rv, sg;
    auto fetch = [&](int g) {
        const int gg = g < G ? g : G - 1;
        sg = D.sigt[(size_t)K * G + gg];
        rv = D.R[((size_t)K * G + gg) * N + rr];
        a0 = trace(r, gg);
        a1 = trace(r + H, gg);
    };
    fetch(sys);

    for (int g0 = 0; g0 < G; g0 += SPB) {
        const int g = g0 + sys;
        const bool valid = g < G && r < N;
        // The elimination compares the lane's row with each pivot index; kept
        // opaque here, those compares are made where they are used instead of
        // being hoisted out of the loop as hundreds of live lane masks.
        int rl = r, hl = half;
        asm volatile("" : "+v"(rl), "+v"(hl));
        if (r < ntr) tr[r] = a0;
        if (r + H < ntr) tr[r + H] = a1;
        wave_lds_sync();
        const float sig = sg;
        double bd = (double)rv;
        fetch(g + SPB);                                      // the next group's inputs land during this solve
        float row[N];
#pragma unroll
        for (int j = 0; j < N; ++j) row[j] = __builtin_fmaf(sig, sM[rr * LD + j], (float)sB[rr * LD + j]);
        // right-hand side in FP64 with the same face operators as the matrix (an
        // FP32 one would break the exact cancellation of the face terms on a
        // constant solution)
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (fpos[f] < 0) continue;                       // not inflow, or this row's node is not on it
            const double *of = sOF[f] + fpos[f] * NF;
            const float *u = tr + __popc(mask & ((1 << f) - 1)) * NF;   // its slot among the inflow faces
#pragma unroll
            for (int l = 0; l < NF; ++l) bd -= of[l] * (double)u[l];
        }
        const double b0 = bd;
        float b = (float)bd;
        float x = 0.f, idg = 0.f;   // idg: the inverse of this lane's pivot
        lu_solve<N, H, LP, (REFINE > 0)>(row, b, x, idg, piv, rl, hl, std::make_integer_sequence<int, N>{},
                                         std::make_integer_sequence<int, N / 2>{});
        // refinement: residual in FP64, b0 - B x - sigma_t M x with B in FP64, then
        // the correction from the same factors.  x reaches every lane of the system
        // in FP64 through its pivot buffer (a wave's LDS accesses run in issue order).
#pragma unroll 1
        for (int it = 0; it < REFINE; ++it) {
            double *xd = reinterpret_cast<double *>(piv);
            if (r < N) xd[r] = (double)x;
            wave_lds_sync();
            const double2 *x2 = reinterpret_cast<const double2 *>(piv);
            double sb = 0.0, sm = 0.0;
#pragma unroll 4
            for (int c = 0; c < N / 2; ++c) {
                const double2 xv = x2[c];
                sb = __builtin_fma(sB[rr * LD + 2 * c], xv.x, sb);
                sm = __builtin_fma((double)sM[rr * LD + 2 * c], xv.x, sm);
                sb = __builtin_fma(sB[rr * LD + 2 * c + 1], xv.y, sb);
                sm = __builtin_fma((double)sM[rr * LD + 2 * c + 1], xv.y, sm);
            }
            if constexpr (N % 2) {
                const double xl = xd[N - 1];
                sb = __builtin_fma(sB[rr * LD + N - 1], xl, sb);
                sm = __builtin_fma((double)sM[rr * LD + N - 1], xl, sm);
            }
            const double res = __builtin_fma(-(double)sig, sm, b0 - sb);
            float rb = (float)res, dxk = 0.f;
            asm volatile("" : "+v"(rl), "+v"(hl));   // not the masks of the first solve either
            lu_resolve<N, H>(row, idg, rb, dxk, rl, hl, std::make_integer_sequence<int, N>{},
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
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_ho_sweep2(HoDev D, int begin) {
    ho_sweep_body<2, 1>(D, begin);
}
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
