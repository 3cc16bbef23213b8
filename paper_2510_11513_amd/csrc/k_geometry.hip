// Element arrays of trilinear-hex DG (Table 1: fi_dfj_dx/dy/dz, fi_dfj, normals),
// integrated in FP64 on the device and stored in FP32 for the sweep.
//
//   M_ij   = int_K f_i f_j dV               2x2x2 Gauss, points +-1/sqrt(3)
//   S^a_ij = int_K f_i (df_j / dx_a) dV     same rule (exact for trilinear maps)
//   F^a_kl = int_f f_k f_l n_a dA           2x2 Gauss on the face, k, l face vertices
//   A_f    = int_f n dA                     outward area vector (FP64, designation)
//
// Reference element [-1,1]^3, local vertex j = a + 2b + 4c at (2a-1, 2b-1, 2c-1),
// basis f_j = prod_d (1 + c_jd xi_d) / 2.
#include "snx_internal.h"

namespace snx {
namespace {

__device__ inline double cj(int j, int d) { return ((j >> d) & 1) ? 1.0 : -1.0; }

struct Frame {
    double f[8];
    double dxi[8][3];
};

__device__ inline void eval_basis(double x0, double x1, double x2, Frame &fr) {
    const double xi[3] = {x0, x1, x2};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double h0 = 0.5 * (1.0 + cj(j, 0) * xi[0]);
        double h1 = 0.5 * (1.0 + cj(j, 1) * xi[1]);
        double h2 = 0.5 * (1.0 + cj(j, 2) * xi[2]);
        fr.f[j] = h0 * h1 * h2;
        fr.dxi[j][0] = 0.5 * cj(j, 0) * h1 * h2;
        fr.dxi[j][1] = h0 * 0.5 * cj(j, 1) * h2;
        fr.dxi[j][2] = h0 * h1 * 0.5 * cj(j, 2);
    }
}

// One thread per (cell, row i): row i of M and of S^x, S^y, S^z.
__global__ void k_volume(const double *__restrict__ xyz, const int *__restrict__ cv, int C,
                         float *__restrict__ M, float *__restrict__ S, int *__restrict__ err) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)C * 8) return;
    int K = (int)(t >> 3), i = (int)(t & 7);
    double X[8][3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int v = cv[(size_t)K * 8 + j];
        X[j][0] = xyz[3 * (size_t)v + 0];
        X[j][1] = xyz[3 * (size_t)v + 1];
        X[j][2] = xyz[3 * (size_t)v + 2];
    }
    double m[8] = {0}, s[3][8] = {{0}};
    const double g = 0.57735026918962576451;  // 1/sqrt(3)
    bool bad = false;
    for (int qp = 0; qp < 8; ++qp) {
        Frame fr;
        eval_basis(cj(qp, 0) * g, cj(qp, 1) * g, cj(qp, 2) * g, fr);
        double J[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < 8; ++j) acc += X[j][a] * fr.dxi[j][b];
                J[a][b] = acc;
            }
        // cofactor matrix: adj(J)^T = det(J) J^{-T}; grad_x f = J^{-T} grad_xi f
        double cof[3][3];
        cof[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        cof[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        cof[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        cof[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        cof[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        cof[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        cof[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        cof[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        cof[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        double det = J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
        if (!(det > 0.0)) bad = true;
        double fi = fr.f[i];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            m[j] += det * fi * fr.f[j];
            // det * (J^{-T} grad_xi f_j)_a = sum_b cof[a][b] dxi_b
#pragma unroll
            for (int a = 0; a < 3; ++a)
                s[a][j] += fi * (cof[a][0] * fr.dxi[j][0] + cof[a][1] * fr.dxi[j][1] + cof[a][2] * fr.dxi[j][2]);
        }
    }
    if (bad) atomicOr(err, 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        M[(size_t)K * 64 + i * 8 + j] = (float)m[j];
#pragma unroll
        for (int a = 0; a < 3; ++a) S[(size_t)K * 192 + a * 64 + i * 8 + j] = (float)s[a][j];
    }
}

// One thread per (cell, face).  Interior faces are integrated once, by the side
// with the smaller cell*6+face; the other side receives the negated matrices at
// the matching vertices, so the two sides cancel exactly.
__global__ void k_faces(const double *__restrict__ xyz, const int *__restrict__ cv, const int *__restrict__ nbr,
                        const int *__restrict__ nbr_face, const unsigned *__restrict__ perm, int C,
                        float *__restrict__ F, double *__restrict__ area) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)C * 6) return;
    int K = (int)(t / 6), f = (int)(t % 6);
    int N = nbr[t], gN = nbr_face[t];
    if (N >= 0 && (long long)N * 6 + gN < t) return;
    double X[8][3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int v = cv[(size_t)K * 8 + j];
        X[j][0] = xyz[3 * (size_t)v + 0];
        X[j][1] = xyz[3 * (size_t)v + 1];
        X[j][2] = xyz[3 * (size_t)v + 2];
    }
    const int axis = f >> 1, side = f & 1;
    const int u = axis == 0 ? 1 : 0, v = axis == 2 ? 1 : 2;
    // d x/d xi_u cross d x/d xi_v points along +xi_axis for axes 0, 2 and -xi_axis for axis 1
    const double sgn = (axis == 1 ? -1.0 : 1.0) * (side ? 1.0 : -1.0);
    int fv[4], k = 0;
    for (int j = 0; j < 8; ++j)
        if (((j >> axis) & 1) == side) fv[k++] = j;
    double Fl[3][16] = {{0}}, A[3] = {0, 0, 0};
    const double g = 0.57735026918962576451;
    for (int qp = 0; qp < 4; ++qp) {
        double xi[3];
        xi[axis] = side ? 1.0 : -1.0;
        xi[u] = ((qp & 1) ? 1.0 : -1.0) * g;
        xi[v] = ((qp & 2) ? 1.0 : -1.0) * g;
        Frame fr;
        eval_basis(xi[0], xi[1], xi[2], fr);
        double tu[3], tv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double su = 0.0, sv = 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                su += X[j][a] * fr.dxi[j][u];
                sv += X[j][a] * fr.dxi[j][v];
            }
            tu[a] = su;
            tv[a] = sv;
        }
        double n[3] = {sgn * (tu[1] * tv[2] - tu[2] * tv[1]), sgn * (tu[2] * tv[0] - tu[0] * tv[2]),
                       sgn * (tu[0] * tv[1] - tu[1] * tv[0])};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            A[a] += n[a];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int l = 0; l < 4; ++l) Fl[a][kk * 4 + l] += n[a] * fr.f[fv[kk]] * fr.f[fv[l]];
        }
    }
    float *FK = F + (size_t)t * 48;
    for (int a = 0; a < 3; ++a) {
        area[(size_t)t * 3 + a] = A[a];
        for (int e = 0; e < 16; ++e) FK[a * 16 + e] = (float)Fl[a][e];
    }
    if (N < 0) return;
    // position of each of my face vertices among the neighbour's face vertices
    const int axN = gN >> 1, sdN = gN & 1;
    int pos[4];
    unsigned pk = perm[t];
    for (int kk = 0; kk < 4; ++kk) {
        int jn = (pk >> (8 * kk)) & 0xff, m = 0;
        pos[kk] = 0;
        for (int j = 0; j < 8; ++j)
            if (((j >> axN) & 1) == sdN) {
                if (j == jn) pos[kk] = m;
                ++m;
            }
    }
    size_t tn = (size_t)N * 6 + gN;
    float *FN = F + tn * 48;
    for (int a = 0; a < 3; ++a) {
        area[tn * 3 + a] = -A[a];
        for (int kk = 0; kk < 4; ++kk)
            for (int l = 0; l < 4; ++l) FN[a * 16 + pos[kk] * 4 + pos[l]] = (float)(-Fl[a][kk * 4 + l]);
    }
}

}  // namespace

hipError_t launch_geometry(const double *xyz, const int *cell_vert, const int *nbr, const int *nbr_face,
                           const unsigned *perm, int C, float *M, float *S, float *F, double *area,
                           int *err_flag, hipStream_t s) {
    const int bs = 128;
    long long n1 = (long long)C * 8, n2 = (long long)C * 6;
    hipLaunchKernelGGL(k_volume, dim3((unsigned)((n1 + bs - 1) / bs)), dim3(bs), 0, s, xyz, cell_vert, C, M, S,
                       err_flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_faces, dim3((unsigned)((n2 + bs - 1) / bs)), dim3(bs), 0, s, xyz, cell_vert, nbr, nbr_face,
                       perm, C, F, area);
    return hipGetLastError();
}

}  // namespace snx
