// C ABI of the learned initial guess: a face-adjacency message-passing network
// that predicts the converged scalar flux of a problem from its data, trained on
// the GPU with the library's own BF16 MFMA forward and backward kernels.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>

#include "snx_internal.h"

using namespace snx;

namespace {

constexpr int H = 64;
constexpr int NFEAT = kGnnFeatures;

thread_local std::string g_gnn_error;

}  // namespace

struct snx_gnn {
    int device = 0;
    int layers = 4;
    std::string err;
    std::vector<void *> allocs;        // parameters and optimiser state
    std::vector<void *> ws_allocs;     // workspace sized for the largest graph seen
    float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    std::vector<void *> Wb, Wt;        // bf16 copies of the layer weights: [2H][H] and [H][2H]
    int nparams = 0;
    long long step = 0;
    float weight_decay = 1e-4f;        // of snx_gnn_train_step (the problem-level step)
    // workspace
    long long cap_nodes = 0;
    int cap_cells = 0;
    std::vector<void *> h;             // bf16 [Nn][H], layers + 1 of them
    float *dHa = nullptr, *dHb = nullptr, *dM = nullptr, *z = nullptr, *inv_deg = nullptr;
    float *x = nullptr, *y = nullptr;  // features and targets of predict()
    int *nbr = nullptr;
    float *wpart = nullptr, *bpart = nullptr, *hsum = nullptr;
    float *pinned = nullptr;

    int off_win() const { return 0; }
    int off_bin() const { return NFEAT * H; }
    int off_w(int l) const { return NFEAT * H + H + (l - 1) * (2 * H * H + H); }   // l = 1..layers
    int off_b(int l) const { return off_w(l) + 2 * H * H; }
    int off_wout() const { return off_w(layers + 1); }
    int off_bout() const { return off_wout() + H; }
};

namespace {

snx_status gfail(snx_gnn *g, snx_status code, const std::string &msg) {
    if (g) g->err = msg; else g_gnn_error = msg;
    return code;
}
snx_status ghip(snx_gnn *g, hipError_t e, const char *what) {
    return gfail(g, e == hipErrorOutOfMemory ? SNX_E_OOM : SNX_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define GCHK(g, expr, what)                                  \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return ghip((g), e_, (what));  \
    } while (0)

hipError_t galloc(std::vector<void *> &list, void **p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e == hipSuccess) list.push_back(*p);
    return e;
}

void free_list(std::vector<void *> &list) {
    for (void *p : list) (void)hipFree(p);
    list.clear();
}

snx_status refresh_bf16(snx_gnn *g, hipStream_t s) {
    for (int l = 1; l <= g->layers; ++l)
        GCHK(g, gnn_to_bf16(g->params + g->off_w(l), g->Wb[l - 1], g->Wt[l - 1], s), "bf16 copy");
    return SNX_OK;
}

snx_status ensure_workspace(snx_gnn *g, long long Nn, int C) {
    if (Nn <= g->cap_nodes && C <= g->cap_cells) return SNX_OK;
    free_list(g->ws_allocs);
    g->h.assign(g->layers + 1, nullptr);
    const long long nn = std::max(Nn, g->cap_nodes);
    const int cc = std::max(C, g->cap_cells);
    const size_t grid = gnn_bwd_grid(nn);
    auto &L = g->ws_allocs;
    for (auto &p : g->h) GCHK(g, galloc(L, &p, sizeof(uint16_t) * nn * H), "workspace");
    GCHK(g, galloc(L, (void **)&g->dHa, sizeof(float) * nn * H), "workspace");
    GCHK(g, galloc(L, (void **)&g->dHb, sizeof(float) * nn * H), "workspace");
    GCHK(g, galloc(L, (void **)&g->dM, sizeof(float) * nn * H), "workspace");
    GCHK(g, galloc(L, (void **)&g->z, sizeof(float) * nn), "workspace");
    GCHK(g, galloc(L, (void **)&g->x, sizeof(float) * nn * NFEAT), "workspace");
    GCHK(g, galloc(L, (void **)&g->y, sizeof(float) * nn), "workspace");
    GCHK(g, galloc(L, (void **)&g->inv_deg, sizeof(float) * cc), "workspace");
    GCHK(g, galloc(L, (void **)&g->nbr, sizeof(int) * 6 * (size_t)cc), "workspace");
    GCHK(g, galloc(L, (void **)&g->wpart, sizeof(float) * std::max<size_t>(512, grid) * 2 * H * H), "workspace");
    GCHK(g, galloc(L, (void **)&g->bpart, sizeof(float) * std::max<size_t>(512, grid) * (H + 2)), "workspace");
    GCHK(g, galloc(L, (void **)&g->hsum, sizeof(float) * (H + 2)), "workspace");
    g->cap_nodes = nn;
    g->cap_cells = cc;
    return SNX_OK;
}

// Forward pass over a graph of C cells x G groups; keeps every layer's output.
snx_status forward(snx_gnn *g, const float *x, const int *nbr, int C, int G, hipStream_t s) {
    const long long Nn = (long long)C * G;
    snx_status st = ensure_workspace(g, Nn, C);
    if (st) return st;
    GCHK(g, gnn_inv_degree(nbr, C, g->inv_deg, s), "degree");
    GCHK(g, gnn_input_fwd(x, g->params + g->off_win(), g->params + g->off_bin(), g->h[0], Nn, s), "input layer");
    for (int l = 1; l <= g->layers; ++l)
        GCHK(g, gnn_layer_fwd(g->h[l - 1], g->h[l], nbr, g->inv_deg, G, Nn, g->Wt[l - 1], g->params + g->off_b(l), s),
             "layer");
    GCHK(g, gnn_head_fwd(g->h[g->layers], g->params + g->off_wout(), g->params + g->off_bout(), g->z, Nn, s), "head");
    return SNX_OK;
}

// Forward and backward: gradients of the mean squared error into g->grad, the loss to *loss.
snx_status backward(snx_gnn *g, const float *x, const int *nbr, int C, int G, const float *y, float *loss,
                    hipStream_t s) {
    snx_status st = forward(g, x, nbr, C, G, s);
    if (st) return st;
    const long long Nn = (long long)C * G;
    const int hgrid = 512;
    GCHK(g, gnn_head_bwd(g->h[g->layers], g->z, y, g->params + g->off_wout(), Nn, g->dHa, g->bpart, hgrid, s), "head");
    GCHK(g, gnn_sum_partials(g->bpart, hgrid, H + 2, g->hsum, 1.f, s), "reduce");
    GCHK(g, hipMemcpyAsync(g->grad + g->off_wout(), g->hsum, sizeof(float) * (H + 1), hipMemcpyDeviceToDevice, s),
         "copy");
    GCHK(g, hipMemcpyAsync(g->pinned, g->hsum + H + 1, sizeof(float), hipMemcpyDeviceToHost, s), "copy");
    float *dH = g->dHa, *dHprev = g->dHb;
    const int grid = (int)gnn_bwd_grid(Nn);
    for (int l = g->layers; l >= 1; --l) {
        GCHK(g, gnn_layer_bwd(g->h[l - 1], g->h[l], dH, nbr, g->inv_deg, G, Nn, g->Wb[l - 1], dHprev, g->dM,
                              g->wpart, g->bpart, s), "layer backward");
        GCHK(g, gnn_sum_partials(g->wpart, grid, 2 * H * H, g->grad + g->off_w(l), 1.f, s), "reduce");
        GCHK(g, gnn_sum_partials(g->bpart, grid, H, g->grad + g->off_b(l), 1.f, s), "reduce");
        std::swap(dH, dHprev);
    }
    GCHK(g, gnn_input_bwd(x, g->h[0], dH, Nn, g->wpart, g->bpart, hgrid, s), "input backward");
    GCHK(g, gnn_sum_partials(g->wpart, hgrid, NFEAT * H, g->grad + g->off_win(), 1.f, s), "reduce");
    GCHK(g, gnn_sum_partials(g->bpart, hgrid, H, g->grad + g->off_bin(), 1.f, s), "reduce");
    GCHK(g, hipStreamSynchronize(s), "backward");
    if (loss) *loss = g->pinned[0] / (float)Nn;
    return SNX_OK;
}

}  // namespace

extern "C" {

snx_status snx_gnn_create_on(snx_gnn **out, int32_t device, int32_t hidden, int32_t layers, uint64_t seed) {
    if (!out) return gfail(nullptr, SNX_E_ARG, "out is NULL");
    *out = nullptr;
    if (hidden != H) return gfail(nullptr, SNX_E_ARG, "the network's hidden width is 64");
    if (layers < 1 || layers > 8) return gfail(nullptr, SNX_E_ARG, "1 <= layers <= 8");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return gfail(nullptr, SNX_E_ARG, "no such HIP device");
    snx_gnn *g = new (std::nothrow) snx_gnn();
    if (!g) return gfail(nullptr, SNX_E_OOM, "out of host memory");
    g->device = device;
    g->layers = layers;
    g->nparams = g->off_bout() + 1;
    hipError_t e = hipSetDevice(device);
    auto &L = g->allocs;
    if (e == hipSuccess) e = galloc(L, (void **)&g->params, sizeof(float) * g->nparams);
    if (e == hipSuccess) e = galloc(L, (void **)&g->grad, sizeof(float) * g->nparams);
    if (e == hipSuccess) e = galloc(L, (void **)&g->m, sizeof(float) * g->nparams);
    if (e == hipSuccess) e = galloc(L, (void **)&g->v, sizeof(float) * g->nparams);
    g->Wb.assign(layers, nullptr);
    g->Wt.assign(layers, nullptr);
    for (int l = 0; l < layers && e == hipSuccess; ++l) {
        e = galloc(L, &g->Wb[l], sizeof(uint16_t) * 2 * H * H);
        if (e == hipSuccess) e = galloc(L, &g->Wt[l], sizeof(uint16_t) * 2 * H * H);
    }
    if (e == hipSuccess) e = hipHostMalloc((void **)&g->pinned, 256, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_list(g->allocs);
        delete g;
        return gfail(nullptr, SNX_E_DEVICE, std::string("allocation failed: ") + hipGetErrorString(e));
    }
    // He initialisation (normal, variance 2 / fan_in) of every weight, zero biases
    std::mt19937_64 rng(seed);
    std::vector<float> p(g->nparams, 0.f);
    auto fill = [&](int off, int fan_in, int n) {
        std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / fan_in));
        for (int i = 0; i < n; ++i) p[off + i] = (float)nd(rng);
    };
    fill(g->off_win(), NFEAT, NFEAT * H);
    for (int l = 1; l <= layers; ++l) fill(g->off_w(l), 2 * H, 2 * H * H);
    fill(g->off_wout(), H, H);
    e = hipMemcpy(g->params, p.data(), sizeof(float) * g->nparams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(g->m, 0, sizeof(float) * g->nparams);
    if (e == hipSuccess) e = hipMemset(g->v, 0, sizeof(float) * g->nparams);
    if (e != hipSuccess || refresh_bf16(g, nullptr) || hipDeviceSynchronize() != hipSuccess) {
        free_list(g->allocs);
        (void)hipHostFree(g->pinned);
        delete g;
        return gfail(nullptr, SNX_E_DEVICE, "initialisation failed");
    }
    *out = g;
    return SNX_OK;
}

void snx_gnn_destroy(snx_gnn *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    free_list(g->ws_allocs);
    free_list(g->allocs);
    if (g->pinned) (void)hipHostFree(g->pinned);
    delete g;
}

const char *snx_gnn_last_error(const snx_gnn *g) { return g ? g->err.c_str() : g_gnn_error.c_str(); }

snx_status snx_gnn_num_params(const snx_gnn *g, int64_t *n) {
    if (!g || !n) return SNX_E_ARG;
    *n = g->nparams;
    return SNX_OK;
}

snx_status snx_gnn_get_params(snx_gnn *g, float *host) {
    if (!g || !host) return SNX_E_ARG;
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    GCHK(g, hipMemcpy(host, g->params, sizeof(float) * g->nparams, hipMemcpyDeviceToHost), "copy");
    return SNX_OK;
}

snx_status snx_gnn_set_params(snx_gnn *g, const float *host) {
    if (!g || !host) return SNX_E_ARG;
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    GCHK(g, hipMemcpy(g->params, host, sizeof(float) * g->nparams, hipMemcpyHostToDevice), "copy");
    GCHK(g, hipMemset(g->m, 0, sizeof(float) * g->nparams), "memset");
    GCHK(g, hipMemset(g->v, 0, sizeof(float) * g->nparams), "memset");
    g->step = 0;
    snx_status st = refresh_bf16(g, nullptr);
    if (st) return st;
    GCHK(g, hipDeviceSynchronize(), "sync");
    return SNX_OK;
}

snx_status snx_gnn_save(snx_gnn *g, const char *path) {
    if (!g || !path) return SNX_E_ARG;
    std::vector<float> p(g->nparams);
    snx_status st = snx_gnn_get_params(g, p.data());
    if (st) return st;
    FILE *f = std::fopen(path, "wb");
    if (!f) return gfail(g, SNX_E_ARG, "cannot open file for writing");
    const char magic[8] = {'S', 'N', 'X', 'G', 'N', 'N', '1', 0};
    const int32_t hdr[3] = {H, g->layers, g->nparams};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 3, f) == 3 &&
              std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SNX_OK : gfail(g, SNX_E_ARG, "write failed");
}

snx_status snx_gnn_load(snx_gnn *g, const char *path) {
    if (!g || !path) return SNX_E_ARG;
    FILE *f = std::fopen(path, "rb");
    if (!f) return gfail(g, SNX_E_ARG, "cannot open file");
    char magic[8];
    int32_t hdr[3];
    std::vector<float> p(g->nparams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "SNXGNN1", 8) == 0 &&
              std::fread(hdr, sizeof(int32_t), 3, f) == 3 && hdr[0] == H && hdr[1] == g->layers &&
              hdr[2] == g->nparams && std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
    std::fclose(f);
    if (!ok) return gfail(g, SNX_E_ARG, "not a network file of this shape");
    return snx_gnn_set_params(g, p.data());
}

snx_status snx_gnn_features(snx_problem *p, float *x, int32_t *nbr, void *stream) {
    DevProblem P;
    int dev = 0;
    if (!p || !x) return SNX_E_ARG;
    if (!problem_view(p, &P, &dev)) return SNX_E_STATE;
    if (hipSetDevice(dev) != hipSuccess) return SNX_E_DEVICE;
    if (gnn_features(P, x, nbr, (hipStream_t)stream) != hipSuccess) return SNX_E_DEVICE;
    return SNX_OK;
}

snx_status snx_gnn_targets(const float *phi, int64_t ncell, int32_t G, float *y, void *stream) {
    if (!phi || !y || ncell < 1 || G < 1) return SNX_E_ARG;
    return gnn_targets(phi, ncell * G, y, (hipStream_t)stream) == hipSuccess ? SNX_OK : SNX_E_DEVICE;
}

snx_status snx_gnn_forward(snx_gnn *g, const float *x, const int32_t *nbr, int64_t ncell, int32_t G, float *z,
                           void *stream) {
    if (!g || !x || !nbr || !z || ncell < 1 || G < 1) return SNX_E_ARG;
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    snx_status st = forward(g, x, nbr, (int)ncell, G, s);
    if (st) return st;
    GCHK(g, hipMemcpyAsync(z, g->z, sizeof(float) * ncell * G, hipMemcpyDeviceToDevice, s), "copy");
    return SNX_OK;
}

snx_status snx_gnn_grad(snx_gnn *g, const float *x, const int32_t *nbr, int64_t ncell, int32_t G, const float *y,
                        float *loss, float *grad_host, void *stream) {
    if (!g || !x || !nbr || !y || ncell < 1 || G < 1) return SNX_E_ARG;
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    snx_status st = backward(g, x, nbr, (int)ncell, G, y, loss, (hipStream_t)stream);
    if (st) return st;
    if (grad_host) GCHK(g, hipMemcpy(grad_host, g->grad, sizeof(float) * g->nparams, hipMemcpyDeviceToHost), "copy");
    return SNX_OK;
}

snx_status snx_gnn_train_step_graph(snx_gnn *g, const float *x, const int32_t *nbr, int64_t ncell, int32_t G,
                                    const float *y, float lr, float weight_decay, float *loss, void *stream) {
    if (!g || !x || !nbr || !y || ncell < 1 || G < 1 || !(lr > 0.f)) return SNX_E_ARG;
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    snx_status st = backward(g, x, nbr, (int)ncell, G, y, loss, s);
    if (st) return st;
    const float b1 = 0.9f, b2 = 0.999f;
    ++g->step;
    const float c1 = 1.f - std::pow(b1, (float)g->step), c2 = 1.f - std::pow(b2, (float)g->step);
    GCHK(g, gnn_adamw(g->params, g->grad, g->m, g->v, g->nparams, lr, b1, b2, 1e-8f, weight_decay, c1, c2, s), "adamw");
    return refresh_bf16(g, s);
}

snx_status snx_gnn_create(snx_gnn **out, int32_t hidden, int32_t layers, uint64_t seed) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return gfail(nullptr, SNX_E_DEVICE, "no current HIP device");
    return snx_gnn_create_on(out, device, hidden, layers, seed);
}

snx_status snx_gnn_set_weight_decay(snx_gnn *g, float weight_decay) {
    if (!g || !(weight_decay >= 0.f)) return SNX_E_ARG;
    g->weight_decay = weight_decay;
    return SNX_OK;
}

snx_status snx_gnn_train_step(snx_gnn *g, snx_problem *p, const float *phi_target, float lr, float *loss,
                              void *stream) {
    if (!g || !p || !phi_target || !(lr > 0.f)) return SNX_E_ARG;
    DevProblem P;
    int dev = 0;
    if (!problem_view(p, &P, &dev)) return gfail(g, SNX_E_STATE, "the problem is not set up");
    if (dev != g->device) return gfail(g, SNX_E_ARG, "network and problem are on different devices");
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    snx_status st = ensure_workspace(g, (long long)P.C * P.G, P.C);
    if (st) return st;
    GCHK(g, gnn_features(P, g->x, g->nbr, s), "features");
    GCHK(g, gnn_targets(phi_target, (long long)P.C * P.G, g->y, s), "targets");
    return snx_gnn_train_step_graph(g, g->x, g->nbr, P.C, P.G, g->y, lr, g->weight_decay, loss, stream);
}

snx_status snx_gnn_predict(snx_gnn *g, snx_problem *p, float *phi0, void *stream) {
    if (!g || !p || !phi0) return SNX_E_ARG;
    DevProblem P;
    int dev = 0;
    if (!problem_view(p, &P, &dev)) return gfail(g, SNX_E_STATE, "the problem is not set up");
    if (dev != g->device) return gfail(g, SNX_E_ARG, "network and problem are on different devices");
    GCHK(g, hipSetDevice(g->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const long long Nn = (long long)P.C * P.G;
    snx_status st = ensure_workspace(g, Nn, P.C);
    if (st) return st;
    GCHK(g, gnn_features(P, g->x, g->nbr, s), "features");
    st = forward(g, g->x, g->nbr, P.C, P.G, s);
    if (st) return st;
    GCHK(g, gnn_expand(g->z, Nn, phi0, s), "expand");
    return SNX_OK;
}

}  // extern "C"
