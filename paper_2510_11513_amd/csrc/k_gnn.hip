// Face-adjacency message-passing network on gfx950: BF16 MFMA forward and
// backward kernels with FP32 accumulation.
//
// Nodes are (cell, group) pairs, v = K*G + g; a node's neighbours are the
// same group of the cells sharing a face.  With H = 64 hidden features:
//   h0 = relu(x W_in + b_in)                       (x: 8 features, FP32 FMA)
//   h_l = relu([h_{l-1}, mean_nbr h_{l-1}] W_l + b_l)   (64 x 128 . 128 x 64, MFMA)
//   z = h_L w_out + b_out                          (predicted log(phi_avg + delta))
// Activations are stored in BF16; the three GEMM shapes of a layer (forward
// A W, weight gradient A^T dP, input gradient dP W^T) run on
// v_mfma_f32_32x32x16_bf16 from 64-node tiles staged in LDS.  Per-block
// gradient partials are reduced in a fixed order, so gradients are
// deterministic.
#include "snx_internal.h"

namespace snx {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int H = 64;            // hidden width
constexpr int TILE = 64;         // nodes per tile
constexpr int AS = 2 * H + 8;    // LDS row stride (bf16) of a [node][h | m] tile
constexpr int TS = TILE + 8;     // LDS row stride of transposed tiles ([feature][node])
constexpr int PS = H + 8;        // LDS row stride of [node][H] and [2H][H] tiles
constexpr float kDelta = 1e-4f;  // log(phi_avg + delta) is the regression target

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// The row of element r (0..15) of a 32x32 MFMA accumulator held by lane l;
// its column is l % 32.
__device__ __forceinline__ int acc_row(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

// Loads 16 features [c0, c0+16) of node v as floats.
__device__ __forceinline__ void load16(const bf16 *__restrict__ h, long long v, int c0, float (&out)[16]) {
    const bf16x8 *p = reinterpret_cast<const bf16x8 *>(h + v * H + c0);
    const bf16x8 a = p[0], b = p[1];
#pragma unroll
    for (int i = 0; i < 8; ++i) { out[i] = (float)a[i]; out[8 + i] = (float)b[i]; }
}

// Rows v0..v0+63 of A = [h | mean of the neighbours' h], written as bf16 to
// sA[node][AS] and/or sAt[feature][TS] (either may be null); rows past Nn are 0.
// 256 threads: thread t covers node t/4, features (t%4)*16 .. +16 of h and of m.
__device__ void build_a(const bf16 *__restrict__ h, const int *__restrict__ nbr, const float *__restrict__ inv_deg,
                        int G, long long Nn, long long v0, bf16 *sA, bf16 *sAt) {
    const int t = threadIdx.x, r = t >> 2, c0 = (t & 3) * 16;
    const long long v = v0 + r;
    float own[16], acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) { own[i] = 0.f; acc[i] = 0.f; }
    if (v < Nn) {
        const long long K = v / G;
        const int g = (int)(v - K * G);
        load16(h, v, c0, own);
        for (int f = 0; f < 6; ++f) {
            const int N = nbr[K * 6 + f];
            if (N < 0) continue;
            float nb[16];
            load16(h, (long long)N * G + g, c0, nb);
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] += nb[i];
        }
        const float s = inv_deg[K];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] *= s;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const bf16 a = (bf16)own[i], m = (bf16)acc[i];
        if (sA) { sA[r * AS + c0 + i] = a; sA[r * AS + H + c0 + i] = m; }
        if (sAt) { sAt[(c0 + i) * TS + r] = a; sAt[(H + c0 + i) * TS + r] = m; }
    }
}

// h_out = relu([h_in, mean_nbr h_in] W + b); Wt = W^T as bf16 [H][2H].
__global__ __launch_bounds__(256) void k_layer_fwd(const bf16 *__restrict__ hin, bf16 *__restrict__ hout,
                                                   const int *__restrict__ nbr, const float *__restrict__ inv_deg,
                                                   int G, long long Nn, const bf16 *__restrict__ Wt,
                                                   const float *__restrict__ b) {
    __shared__ __align__(16) bf16 sA[TILE * AS];
    __shared__ __align__(16) bf16 sW[H * AS];
    const long long v0 = (long long)blockIdx.x * TILE;
    for (int i = threadIdx.x; i < H * 16; i += 256) {      // 64 rows of 16 x 8 bf16
        const int j = i >> 4, k8 = (i & 15) * 8;
        *reinterpret_cast<bf16x8 *>(&sW[j * AS + k8]) = *reinterpret_cast<const bf16x8 *>(&Wt[j * 2 * H + k8]);
    }
    build_a(hin, nbr, inv_deg, G, Nn, v0, sA, nullptr);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 2 * H / 16; ++s) {
        const int k = 16 * s + 8 * (l >> 5);
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sA[(rb + (l & 31)) * AS + k]);
        const bf16x8 bb = *reinterpret_cast<const bf16x8 *>(&sW[(cb + (l & 31)) * AS + k]);
        acc = mfma(a, bb, acc);
    }
    const int j = cb + (l & 31);
    const float bj = b[j];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const long long v = v0 + rb + acc_row(r, l);
        if (v < Nn) hout[v * H + j] = (bf16)fmaxf(acc[r] + bj, 0.f);
    }
}

// One layer's backward over a grid-stride set of 64-node tiles:
//   dP = dH_cur * [h_cur > 0]
//   dW += A^T dP, db += sum dP              (per-block partials)
//   [dh_self | dm] = dP W^T; dH_prev = dh_self, dM = dm / deg (scattered later)
// W is bf16 row-major [2H][H].
__global__ __launch_bounds__(256) void k_layer_bwd(const bf16 *__restrict__ hprev, const bf16 *__restrict__ hcur,
                                                   const float *__restrict__ dH, const int *__restrict__ nbr,
                                                   const float *__restrict__ inv_deg, int G, long long Nn,
                                                   const bf16 *__restrict__ W, float *__restrict__ dHprev,
                                                   float *__restrict__ dM, float *__restrict__ dWpart,
                                                   float *__restrict__ dbpart) {
    __shared__ __align__(16) bf16 sAt[2 * H * TS];   // A^T of the tile
    __shared__ __align__(16) bf16 sP[TILE * PS];     // dP
    __shared__ __align__(16) bf16 sPt[H * TS];       // dP^T
    __shared__ __align__(16) bf16 sW[2 * H * PS];    // W
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, t = threadIdx.x;
    for (int i = t; i < 2 * H * 8; i += 256) {          // 128 rows of 8 x 8 bf16
        const int row = i >> 3, k8 = (i & 7) * 8;
        *reinterpret_cast<bf16x8 *>(&sW[row * PS + k8]) = *reinterpret_cast<const bf16x8 *>(&W[row * H + k8]);
    }
    f32x16 accW0 = {}, accW1 = {};
    float db = 0.f;
    const long long ntiles = (Nn + TILE - 1) / TILE;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long long v0 = tile * TILE;
        build_a(hprev, nbr, inv_deg, G, Nn, v0, nullptr, sAt);
        {   // dP rows: thread t covers node t/4, features (t%4)*16 .. +16
            const int r = t >> 2, c0 = (t & 3) * 16;
            const long long v = v0 + r;
            float hc[16];
            if (v < Nn) load16(hcur, v, c0, hc);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float d = (v < Nn && hc[i] > 0.f) ? dH[v * H + c0 + i] : 0.f;
                const bf16 q = (bf16)d;
                sP[r * PS + c0 + i] = q;
                sPt[(c0 + i) * TS + r] = q;
            }
        }
        if (t < H) {   // bias gradient in FP32 from dH itself
            for (int r = 0; r < TILE; ++r) {
                const long long v = v0 + r;
                if (v < Nn && (float)hcur[v * H + t] > 0.f) db += dH[v * H + t];
            }
        }
        __syncthreads();
        // weight gradient: rows 32w..32w+31 of the 2H x H result, both column tiles; K = tile nodes
#pragma unroll
        for (int s = 0; s < TILE / 16; ++s) {
            const int k = 16 * s + 8 * (l >> 5);
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sAt[(32 * w + (l & 31)) * TS + k]);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(&sPt[(l & 31) * TS + k]);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(&sPt[(32 + (l & 31)) * TS + k]);
            accW0 = mfma(a, b0, accW0);
            accW1 = mfma(a, b1, accW1);
        }
        // input gradient dA = dP W^T: node rows 32*(w&1).., feature columns 64*(w>>1) .. +63
        const int n0 = 32 * (w & 1);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int i0 = 64 * (w >> 1) + 32 * ct;
            f32x16 acc = {};
#pragma unroll
            for (int s = 0; s < H / 16; ++s) {
                const int k = 16 * s + 8 * (l >> 5);
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sP[(n0 + (l & 31)) * PS + k]);
                const bf16x8 bb = *reinterpret_cast<const bf16x8 *>(&sW[(i0 + (l & 31)) * PS + k]);
                acc = mfma(a, bb, acc);
            }
            const int i = i0 + (l & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const long long v = v0 + n0 + acc_row(r, l);
                if (v >= Nn) continue;
                if (i < H) dHprev[v * H + i] = acc[r];
                else dM[v * H + (i - H)] = acc[r] * inv_deg[v / G];
            }
        }
        __syncthreads();
    }
    float *part = dWpart + (size_t)blockIdx.x * 2 * H * H;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 32 * w + acc_row(r, l);
        part[i * H + (l & 31)] = accW0[r];
        part[i * H + 32 + (l & 31)] = accW1[r];
    }
    if (t < H) dbpart[(size_t)blockIdx.x * H + t] = db;
}

// dH_prev[v] += sum over face neighbours u of dM[u] (dM already divided by deg(u)).
__global__ __launch_bounds__(256) void k_gather_bwd(float *__restrict__ dHprev, const float *__restrict__ dM,
                                                    const int *__restrict__ nbr, int G, long long Nn) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long v = t >> 2;
    if (v >= Nn) return;
    const int c0 = (int)(t & 3) * 16;
    const long long K = v / G;
    const int g = (int)(v - K * G);
    float acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = dHprev[v * H + c0 + i];
    for (int f = 0; f < 6; ++f) {
        const int N = nbr[K * 6 + f];
        if (N < 0) continue;
        const float *src = dM + ((long long)N * G + g) * H + c0;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] += src[i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) dHprev[v * H + c0 + i] = acc[i];
}

// h0 = relu(x W_in + b_in), FP32 arithmetic, bf16 output; thread = (node, 16 features).
__global__ __launch_bounds__(256) void k_input_fwd(const float *__restrict__ x, const float *__restrict__ Win,
                                                   const float *__restrict__ bin, bf16 *__restrict__ h0, long long Nn) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long v = t >> 2;
    if (v >= Nn) return;
    const int c0 = (int)(t & 3) * 16;
    float xv[kGnnFeatures];
#pragma unroll
    for (int f = 0; f < kGnnFeatures; ++f) xv[f] = x[v * kGnnFeatures + f];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float s = bin[c0 + i];
#pragma unroll
        for (int f = 0; f < kGnnFeatures; ++f) s = fmaf(xv[f], Win[f * H + c0 + i], s);
        h0[v * H + c0 + i] = (bf16)fmaxf(s, 0.f);
    }
}

// Input-layer gradients: dW_in = x^T dP0, db_in = sum dP0 (per-block partials);
// thread = (node lane t/64, feature t%64), 4 nodes per pass.
__global__ __launch_bounds__(256) void k_input_bwd(const float *__restrict__ x, const bf16 *__restrict__ h0,
                                                   const float *__restrict__ dH0, long long Nn,
                                                   float *__restrict__ dWpart, float *__restrict__ dbpart) {
    const int j = threadIdx.x & 63, lane = threadIdx.x >> 6;
    constexpr int NF = kGnnFeatures;
    float aw[NF], ab = 0.f;
#pragma unroll
    for (int f = 0; f < NF; ++f) aw[f] = 0.f;
    for (long long v = (long long)blockIdx.x * 4 + lane; v < Nn; v += (long long)gridDim.x * 4) {
        const float d = (float)h0[v * H + j] > 0.f ? dH0[v * H + j] : 0.f;
#pragma unroll
        for (int f = 0; f < NF; ++f) aw[f] = fmaf(x[v * NF + f], d, aw[f]);
        ab += d;
    }
    __shared__ float s[4][NF + 1][H];
#pragma unroll
    for (int f = 0; f < NF; ++f) s[lane][f][j] = aw[f];
    s[lane][NF][j] = ab;
    __syncthreads();
    if (lane == 0) {
        for (int f = 0; f <= NF; ++f) {
            const float tot = ((s[0][f][j] + s[1][f][j]) + s[2][f][j]) + s[3][f][j];
            if (f < NF) dWpart[(size_t)blockIdx.x * NF * H + f * H + j] = tot;
            else dbpart[(size_t)blockIdx.x * H + j] = tot;
        }
    }
}

// z = h_L w_out + b_out; thread per node.
__global__ __launch_bounds__(256) void k_head_fwd(const bf16 *__restrict__ h, const float *__restrict__ wout,
                                                  const float *__restrict__ bout, float *__restrict__ z, long long Nn) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Nn) return;
    float s = bout[0];
    for (int c = 0; c < H; c += 16) {
        float hv[16];
        load16(h, v, c, hv);
#pragma unroll
        for (int i = 0; i < 16; ++i) s = fmaf(hv[i], wout[c + i], s);
    }
    z[v] = s;
}

// Loss (z - y)^2 / Nn and the head's gradients: dH_L = dz w_out, dw_out, db_out
// (per-block partials); thread = (node lane t/64, feature t%64).
__global__ __launch_bounds__(256) void k_head_bwd(const bf16 *__restrict__ h, const float *__restrict__ z,
                                                  const float *__restrict__ y, const float *__restrict__ wout,
                                                  long long Nn, float *__restrict__ dH, float *__restrict__ part) {
    const int j = threadIdx.x & 63, lane = threadIdx.x >> 6;
    const float scale = 2.f / (float)Nn;
    float aw = 0.f, ab = 0.f, al = 0.f;
    for (long long v = (long long)blockIdx.x * 4 + lane; v < Nn; v += (long long)gridDim.x * 4) {
        const float r = z[v] - y[v];
        const float dz = scale * r;
        dH[v * H + j] = dz * wout[j];
        aw = fmaf(dz, (float)h[v * H + j], aw);
        if (j == 0) { ab += dz; al = fmaf(r, r, al); }
    }
    __shared__ float s[4][H + 2];
    s[lane][j] = aw;
    if (j == 0) { s[lane][H] = ab; s[lane][H + 1] = al; }
    __syncthreads();
    if (lane == 0) {
        float *p = part + (size_t)blockIdx.x * (H + 2);
        p[j] = ((s[0][j] + s[1][j]) + s[2][j]) + s[3][j];
        if (j == 0) {
            p[H] = ((s[0][H] + s[1][H]) + s[2][H]) + s[3][H];
            p[H + 1] = ((s[0][H + 1] + s[1][H + 1]) + s[2][H + 1]) + s[3][H + 1];
        }
    }
}

// out[i] = sum over blocks b of part[b][i] (in block order) * scale.
__global__ void k_sum_partials(const float *__restrict__ part, int nblk, int n, float *__restrict__ out, float scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + i];
    out[i] = s * scale;
}

// AdamW with bias correction on FP32 master weights.
__global__ void k_adamw(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float wd, float c1,
                        float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
}

// bf16 copies of a layer's weight W [2H][H]: row-major and transposed.
__global__ void k_to_bf16(const float *__restrict__ W, bf16 *__restrict__ Wb, bf16 *__restrict__ Wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * H * H) return;
    const int r = i / H, c = i % H;
    const bf16 q = (bf16)W[i];
    Wb[i] = q;
    Wt[c * 2 * H + r] = q;
}

// Node features of (cell, group) pairs from a problem's device tables: the
// cell's cross sections and source, its size in mean free paths, its boundary
// faces and its position in the mesh's bounding box (u in [0,1]^3 and the
// distance to the nearest side of the box).
__global__ void k_features(const float *__restrict__ sigt, const float *__restrict__ sigs, const float *__restrict__ q,
                           const float *__restrict__ M, const int *__restrict__ nbr, const double *__restrict__ xyz,
                           const int *__restrict__ cv, float3 lo, float3 hi, int C, int G, float *__restrict__ x,
                           int *__restrict__ nbr_out) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long long)C * G) return;
    const long long K = v / G;
    float vol = 0.f;
    for (int e = 0; e < 64; ++e) vol += M[K * 64 + e];
    int nb = 0;
    for (int f = 0; f < 6; ++f) nb += nbr[K * 6 + f] < 0;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int j = 0; j < 8; ++j) {
        const long long n = cv[K * 8 + j];
        cx += xyz[3 * n]; cy += xyz[3 * n + 1]; cz += xyz[3 * n + 2];
    }
    const float ux = (float)((cx * 0.125 - lo.x) / (hi.x - lo.x));
    const float uy = (float)((cy * 0.125 - lo.y) / (hi.y - lo.y));
    const float uz = (float)((cz * 0.125 - lo.z) / (hi.z - lo.z));
    const float db = fminf(fminf(fminf(ux, 1.f - ux), fminf(uy, 1.f - uy)), fminf(uz, 1.f - uz));
    const float st = sigt[v], ss = sigs[v], qq = q[v];
    const float c = ss / st, sa = st - ss;
    const float h = cbrtf(vol);
    float *o = x + v * kGnnFeatures;
    o[0] = logf(st);
    o[1] = c;
    o[2] = qq;
    o[3] = logf(qq / sa + 1e-2f);
    o[4] = (float)nb / 3.f;
    o[5] = logf(st * h);
    o[6] = logf(fmaxf(1.f - c, 1e-6f));
    o[7] = db;
    o[8] = ux;
    o[9] = uy;
    o[10] = uz;
    o[11] = logf(fmaxf(sa * h, 1e-12f));
    if (nbr_out && (v % G) == 0)
        for (int f = 0; f < 6; ++f) nbr_out[K * 6 + f] = nbr[K * 6 + f];
}

__global__ void k_inv_degree(const int *__restrict__ nbr, int C, float *__restrict__ inv_deg) {
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= C) return;
    int d = 0;
    for (int f = 0; f < 6; ++f) d += nbr[K * 6 + f] >= 0;
    inv_deg[K] = d > 0 ? 1.f / (float)d : 0.f;
}

__global__ void k_targets(const float *__restrict__ phi, long long Nn, float *__restrict__ y) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Nn) return;
    float s = 0.f;
    for (int d = 0; d < 8; ++d) s += phi[v * 8 + d];
    y[v] = logf(s * 0.125f + kDelta);
}

__global__ void k_expand(const float *__restrict__ z, long long Nn, float *__restrict__ phi) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Nn * 8) return;
    phi[t] = fmaxf(expf(z[t >> 3]) - kDelta, 0.f);
}

unsigned blocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t gnn_bwd_grid(long long Nn) {
    const long long tiles = (Nn + TILE - 1) / TILE;
    return (size_t)std::max(1LL, std::min(tiles, 512LL));
}

hipError_t gnn_layer_fwd(const void *hin, void *hout, const int *nbr, const float *inv_deg, int G, long long Nn,
                         const void *Wt, const float *b, hipStream_t s) {
    hipLaunchKernelGGL(k_layer_fwd, dim3(blocks(Nn, TILE)), dim3(256), 0, s, (const bf16 *)hin, (bf16 *)hout, nbr,
                       inv_deg, G, Nn, (const bf16 *)Wt, b);
    return hipGetLastError();
}

hipError_t gnn_layer_bwd(const void *hprev, const void *hcur, const float *dH, const int *nbr, const float *inv_deg,
                         int G, long long Nn, const void *W, float *dHprev, float *dM, float *dWpart, float *dbpart,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_layer_bwd, dim3((unsigned)gnn_bwd_grid(Nn)), dim3(256), 0, s, (const bf16 *)hprev,
                       (const bf16 *)hcur, dH, nbr, inv_deg, G, Nn, (const bf16 *)W, dHprev, dM, dWpart, dbpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_bwd, dim3(blocks(Nn * 4, 256)), dim3(256), 0, s, dHprev, dM, nbr, G, Nn);
    return hipGetLastError();
}

hipError_t gnn_input_fwd(const float *x, const float *Win, const float *bin, void *h0, long long Nn, hipStream_t s) {
    hipLaunchKernelGGL(k_input_fwd, dim3(blocks(Nn * 4, 256)), dim3(256), 0, s, x, Win, bin, (bf16 *)h0, Nn);
    return hipGetLastError();
}

hipError_t gnn_input_bwd(const float *x, const void *h0, const float *dH0, long long Nn, float *dWpart, float *dbpart,
                         int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_input_bwd, dim3(grid), dim3(256), 0, s, x, (const bf16 *)h0, dH0, Nn, dWpart, dbpart);
    return hipGetLastError();
}

hipError_t gnn_head_fwd(const void *h, const float *wout, const float *bout, float *z, long long Nn, hipStream_t s) {
    hipLaunchKernelGGL(k_head_fwd, dim3(blocks(Nn, 256)), dim3(256), 0, s, (const bf16 *)h, wout, bout, z, Nn);
    return hipGetLastError();
}

hipError_t gnn_head_bwd(const void *h, const float *z, const float *y, const float *wout, long long Nn, float *dH,
                        float *part, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_head_bwd, dim3(grid), dim3(256), 0, s, (const bf16 *)h, z, y, wout, Nn, dH, part);
    return hipGetLastError();
}

hipError_t gnn_sum_partials(const float *part, int nblk, int n, float *out, float scale, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks(n, 256)), dim3(256), 0, s, part, nblk, n, out, scale);
    return hipGetLastError();
}

hipError_t gnn_adamw(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adamw, dim3(blocks(n, 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

hipError_t gnn_to_bf16(const float *W, void *Wb, void *Wt, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(2 * H * H, 256)), dim3(256), 0, s, W, (bf16 *)Wb, (bf16 *)Wt);
    return hipGetLastError();
}

hipError_t gnn_features(const DevProblem &P, float *x, int *nbr_out, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3(blocks((long long)P.C * P.G, 256)), dim3(256), 0, s, P.sigt, P.sigs, P.q, P.M,
                       P.nbr, P.xyz, P.cv, make_float3(P.lo[0], P.lo[1], P.lo[2]),
                       make_float3(P.hi[0], P.hi[1], P.hi[2]), P.C, P.G, x, nbr_out);
    return hipGetLastError();
}

hipError_t gnn_inv_degree(const int *nbr, int C, float *inv_deg, hipStream_t s) {
    hipLaunchKernelGGL(k_inv_degree, dim3(blocks(C, 256)), dim3(256), 0, s, nbr, C, inv_deg);
    return hipGetLastError();
}

hipError_t gnn_targets(const float *phi, long long Nn, float *y, hipStream_t s) {
    hipLaunchKernelGGL(k_targets, dim3(blocks(Nn, 256)), dim3(256), 0, s, phi, Nn, y);
    return hipGetLastError();
}

hipError_t gnn_expand(const float *z, long long Nn, float *phi, hipStream_t s) {
    hipLaunchKernelGGL(k_expand, dim3(blocks(Nn * 8, 256)), dim3(256), 0, s, z, Nn, phi);
    return hipGetLastError();
}

}  // namespace snx
