// C ABI of the gfx950 S_N sweep library: problem state, set-up orchestration,
// sweep and the graph-captured source-iteration loop.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "snx_internal.h"


using namespace snx;

namespace {

thread_local std::string g_create_error;

struct DevAlloc {
    std::vector<void *> ptrs;
    hipError_t alloc(void **p, size_t bytes) {
        *p = nullptr;
        hipError_t e = hipMalloc(p, bytes ? bytes : 1);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    void release() {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
};

}  // namespace

// Everything one sweep schedule needs: the merged problem table, the queue and
// the seed tasks.  A single problem is a schedule of one.
struct SweepSched {
    DevProblem *d_probs = nullptr;
    long long *d_base = nullptr;
    SweepCtl *d_ctl = nullptr;
    SweepCtl host_ctl{};                 // static part (queue layout, seeds, XCC map) uploaded on reset
    unsigned long long *d_queue = nullptr;
    int *d_seeds = nullptr;
    int nprob = 0, nseed = 0;
    long long total = 0;
    int maxA = 0, maxG = 0, maxin = 0;
    int threads = 256, wg_per_cu = 0, grid = 0;
};

struct snx_problem {
    int device = 0;
    std::string err;
    hipStream_t cap_stream = nullptr;
    void *pinned = nullptr;            // host staging for small read-backs

    // host inputs
    int C = 0, nvert = 0, nang = 0, A = 0, G = 0, bkind = 0;
    std::vector<double> xyz, omega, w, sigt, sigs, q, psib;
    std::vector<int> cv;
    bool have_mesh = false, have_quad = false, have_mat = false;

    // set-up results
    bool ready = false;
    DevAlloc mem;
    DevProblem hp{};
    SweepSched sched;
    std::vector<int> level, nlev;
    int *d_err = nullptr;
    IterCtl *d_ic = nullptr;
    int *d_stop = nullptr;
    float *d_phi[2] = {nullptr, nullptr};
    double *d_partial = nullptr, *d_out4 = nullptr;
    double *d_area = nullptr;
    unsigned long long watchdog_ticks = 0;
    int chunk = 8;
    int threads = 256, wg_per_cu = 0;   // requested sweep schedule
    int nq = 1;                         // task queues = XCDs seen on the device
    int xcc_queue[kMaxXcc] = {0};       // home queue of each hardware XCC id

    hipGraphExec_t graph[2] = {nullptr, nullptr};   // chunk starting from ping-pong buffer 0 / 1
};

static snx_status fail(snx_problem *p, snx_status code, const std::string &msg) {
    if (p) p->err = msg;
    return code;
}

static snx_status hip_fail(snx_problem *p, hipError_t e, const char *what) {
    return fail(p, e == hipErrorOutOfMemory ? SNX_E_OOM : SNX_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(p, expr, what)                                   \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_fail((p), e_, (what)); \
    } while (0)

static void drop_graph(snx_problem *p) {
    for (auto &g : p->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

static void drop_device(snx_problem *p) {
    drop_graph(p);
    p->mem.release();
    p->ready = false;
    p->hp = DevProblem{};
    p->sched = SweepSched{};
}

// Zero the scheduler state: counters, epoch, queue slots, abort flag and queue
// statistics, and upload the static queue layout.
static hipError_t reset_schedule(snx_problem *p, hipStream_t s) {
    hipError_t e = launch_fill_u32(p->hp.cnt, (size_t)8 * p->C, 0u, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->sched.d_queue, 0, sizeof(unsigned long long) * (size_t)p->sched.total, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->sched.d_ctl, &p->sched.host_ctl, sizeof(SweepCtl), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Queue layout of a sweep: octant o goes to queue o mod nq; each queue's slots
// hold every task of its octants, seeds first.
static void layout_queues(SweepCtl &c, int nq, const int *xcc_queue, const std::vector<long long> &cells_per_problem,
                          const std::vector<std::vector<int>> &seeds_by_octant, std::vector<int> &seeds) {
    c = SweepCtl{};
    c.nq = nq;
    for (int x = 0; x < kMaxXcc; ++x) c.xcc_queue[x] = xcc_queue[x];
    long long base = 0;
    seeds.clear();
    for (int q = 0; q < nq; ++q) {
        long long tot = 0;
        c.qseed_base[q] = (int)seeds.size();
        for (int o = q; o < 8; o += nq) {
            for (long long cp : cells_per_problem) tot += cp;
            seeds.insert(seeds.end(), seeds_by_octant[o].begin(), seeds_by_octant[o].end());
        }
        c.qseed_count[q] = (int)seeds.size() - c.qseed_base[q];
        c.qbase[q] = base;
        c.qtotal[q] = tot;
        base += tot;
    }
}

static int cu_count(int device) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
    return n;
}

static snx_status configure_grid(snx_problem *p, SweepSched &sc) {
    const size_t lds = sweep_lds_bytes(sc.threads, sc.maxA, sc.maxG, sc.maxin);
    if (lds > 64 * 1024) return fail(p, SNX_E_ARG, "task does not fit in 64 KB of LDS (too many angles or groups)");
    int occ = sweep_occupancy(sc.threads, lds);
    if (occ <= 0) return fail(p, SNX_E_ARG, "sweep kernel cannot be resident with this schedule");
    int per_cu = sc.wg_per_cu > 0 ? std::min(sc.wg_per_cu, occ) : occ;
    long long grid = (long long)cu_count(p->device) * per_cu;
    if (grid > sc.total) grid = sc.total;
    sc.grid = (int)std::max(1LL, grid);
    return SNX_OK;
}

extern "C" {

snx_status snx_create(snx_problem **out, int32_t device) {
    if (!out) { g_create_error = "out is NULL"; return SNX_E_ARG; }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_create_error = "no such HIP device";
        return SNX_E_ARG;
    }
    snx_problem *p = new (std::nothrow) snx_problem();
    if (!p) { g_create_error = "out of host memory"; return SNX_E_OOM; }
    p->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc(&p->pinned, 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        g_create_error = std::string("HIP initialisation failed: ") + hipGetErrorString(e);
        if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
        delete p;
        return SNX_E_DEVICE;
    }
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    // Which XCDs do workgroups land on?  Each distinct XCC id becomes one task queue.
    {
        const int nb = 8 * cu_count(device);
        int *d_ids = nullptr;
        std::vector<int> ids(nb, 0);
        e = hipMalloc((void **)&d_ids, sizeof(int) * nb);
        if (e == hipSuccess) e = launch_xcc_probe(d_ids, nb, p->cap_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ids.data(), d_ids, sizeof(int) * nb, hipMemcpyDeviceToHost, p->cap_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->cap_stream);
        if (d_ids) (void)hipFree(d_ids);
        if (e != hipSuccess) {
            g_create_error = std::string("XCD probe failed: ") + hipGetErrorString(e);
            (void)hipStreamDestroy(p->cap_stream);
            (void)hipHostFree(p->pinned);
            delete p;
            return SNX_E_DEVICE;
        }
        bool seen[kMaxXcc] = {false};
        for (int v : ids) seen[v & (kMaxXcc - 1)] = true;
        int nq = 0;
        for (int x = 0; x < kMaxXcc; ++x)
            if (seen[x] && nq < kMaxQueues) p->xcc_queue[x] = nq++;
        p->nq = std::max(1, nq);
    }
    p->watchdog_ticks = (unsigned long long)rate_khz * 1000ull * 20ull;   // 20 s without a ready task
    *out = p;
    return SNX_OK;
}

void snx_destroy(snx_problem *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    drop_device(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->pinned) (void)hipHostFree(p->pinned);
    delete p;
}

const char *snx_last_error(const snx_problem *p) { return p ? p->err.c_str() : g_create_error.c_str(); }

snx_status snx_set_mesh(snx_problem *p, int64_t ncell, int64_t nvert, const double *xyz, const int32_t *cell_vert) {
    if (!p) return SNX_E_ARG;
    if (ncell < 1 || ncell > (1 << 26) || nvert < 8 || nvert > (1LL << 30) || !xyz || !cell_vert)
        return fail(p, SNX_E_ARG, "bad mesh arguments");
    for (int64_t i = 0; i < ncell * 8; ++i)
        if (cell_vert[i] < 0 || cell_vert[i] >= nvert) return fail(p, SNX_E_ARG, "vertex id out of range");
    p->C = (int)ncell;
    p->nvert = (int)nvert;
    p->xyz.assign(xyz, xyz + 3 * nvert);
    p->cv.assign(cell_vert, cell_vert + 8 * ncell);
    p->have_mesh = true;
    p->have_mat = false;
    drop_device(p);
    return SNX_OK;
}

snx_status snx_quadrature_product(int32_t npolar, int32_t nazim, double *omega, double *w) {
    return product_quadrature(npolar, nazim, omega, w);
}

snx_status snx_set_quadrature(snx_problem *p, int32_t nang, const double *omega, const double *w) {
    if (!p) return SNX_E_ARG;
    if (nang < 8 || nang % 8 || nang / 8 > kMaxAnglesPerOctant || !omega || !w)
        return fail(p, SNX_E_ARG, "nang must be a multiple of 8 with at most 64 per octant");
    const int per = nang / 8;
    for (int n = 0; n < nang; ++n) {
        const double *om = omega + 3 * n;
        if (om[0] == 0.0 || om[1] == 0.0 || om[2] == 0.0) return fail(p, SNX_E_ARG, "direction on an octant plane");
        const int o = (om[0] < 0) + 2 * (om[1] < 0) + 4 * (om[2] < 0);
        if (o != n / per) return fail(p, SNX_E_ARG, "directions are not grouped by octant");
        if (!(w[n] > 0.0)) return fail(p, SNX_E_ARG, "weights must be positive");
    }
    p->nang = nang;
    p->A = per;
    p->omega.assign(omega, omega + 3 * nang);
    p->w.assign(w, w + nang);
    p->have_quad = true;
    drop_device(p);
    return SNX_OK;
}

snx_status snx_set_materials(snx_problem *p, int32_t ngroup, const double *sigma_t, const double *sigma_s,
                             const double *q) {
    if (!p) return SNX_E_ARG;
    if (!p->have_mesh) return fail(p, SNX_E_STATE, "set the mesh before the materials");
    if (ngroup < 1 || ngroup > kMaxGroups || !sigma_t || !sigma_s || !q)
        return fail(p, SNX_E_ARG, "bad material arguments (1 <= G <= 256)");
    const size_t n = (size_t)p->C * ngroup;
    for (size_t i = 0; i < n; ++i)
        if (!(sigma_t[i] > 0.0) || sigma_s[i] < 0.0 || !std::isfinite(q[i]))
            return fail(p, SNX_E_ARG, "need sigma_t > 0, sigma_s >= 0 and finite sources");
    p->G = ngroup;
    p->sigt.assign(sigma_t, sigma_t + n);
    p->sigs.assign(sigma_s, sigma_s + n);
    p->q.assign(q, q + n);
    p->have_mat = true;
    drop_device(p);
    return SNX_OK;
}

snx_status snx_set_boundary(snx_problem *p, int32_t kind, const double *psi_in) {
    if (!p) return SNX_E_ARG;
    if (kind != 0 && kind != 1) return fail(p, SNX_E_ARG, "boundary kind must be 0 or 1");
    if (kind == 1 && (!psi_in || !p->have_mat)) return fail(p, SNX_E_ARG, "inflow needs materials set and psi_in");
    p->bkind = kind;
    if (kind == 1) p->psib.assign(psi_in, psi_in + p->G); else p->psib.clear();
    drop_device(p);
    return SNX_OK;
}

snx_status snx_setup(snx_problem *p, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->have_mesh || !p->have_quad || !p->have_mat) return fail(p, SNX_E_STATE, "mesh, quadrature and materials must be set");
    if (p->bkind == 1 && (int)p->psib.size() != p->G) return fail(p, SNX_E_STATE, "boundary inflow size differs from G");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    drop_device(p);

    std::vector<int> nbr, nbrf;
    std::vector<unsigned> perm;
    std::string terr;
    int rc = topology(p->C, p->nvert, p->cv.data(), nbr, nbrf, perm, terr);
    if (rc) return fail(p, rc, terr);

    const size_t C = p->C, G = p->G, A = p->A;
    DevAlloc &m = p->mem;
    DevProblem &hp = p->hp;
    double *d_xyz; int *d_cv, *d_nbr, *d_nbrf; unsigned *d_perm;
    float *dM, *dS, *dF, *dsigt, *dsigs, *dq, *dr, *dom, *dw, *dpsib = nullptr, *dpsi, *dslot, *dslotc;
    unsigned char *dmask; int *dindeg, *dlevel, *dhist, *dnlev, *dseeds, *dnseed, *dscratch; unsigned *dcnt;
#define ALLOC(ptr, bytes) HIPCHK(p, m.alloc((void **)&(ptr), (bytes)), "device allocation")
    ALLOC(d_xyz, sizeof(double) * 3 * p->nvert);
    ALLOC(d_cv, sizeof(int) * 8 * C);
    ALLOC(d_nbr, sizeof(int) * 6 * C);
    ALLOC(d_nbrf, sizeof(int) * 6 * C);
    ALLOC(d_perm, sizeof(unsigned) * 6 * C);
    ALLOC(dM, sizeof(float) * 64 * C);
    ALLOC(dS, sizeof(float) * 192 * C);
    float *dT;
    ALLOC(dT, sizeof(float) * 8 * 192 * C);
    ALLOC(dF, sizeof(float) * 288 * C);
    ALLOC(p->d_area, sizeof(double) * 18 * C);
    ALLOC(dmask, 8 * C);
    ALLOC(dindeg, sizeof(int) * 8 * C);
    ALLOC(dlevel, sizeof(int) * 8 * C);
    ALLOC(dhist, sizeof(int) * 8 * (C + 1));
    ALLOC(dnlev, sizeof(int) * 16);
    ALLOC(dseeds, sizeof(int) * 8 * C);
    ALLOC(dnseed, sizeof(int) * 8);
    ALLOC(dscratch, sizeof(int) * 24 * C);
    ALLOC(p->d_err, sizeof(int));
    ALLOC(dsigt, sizeof(float) * C * G);
    ALLOC(dsigs, sizeof(float) * C * G);
    ALLOC(dq, sizeof(float) * C * G);
    ALLOC(dr, sizeof(float) * C * G * 8);
    ALLOC(dom, sizeof(float) * 3 * p->nang);
    ALLOC(dw, sizeof(float) * p->nang);
    if (p->bkind == 1) ALLOC(dpsib, sizeof(float) * G);
    ALLOC(dpsi, sizeof(float) * 8 * C * 8 * A * G);
    ALLOC(dslot, sizeof(float) * 8 * C * G * 8);
    ALLOC(dslotc, sizeof(float) * 8 * C * G * 8);
    ALLOC(dcnt, sizeof(unsigned) * 8 * C);
    ALLOC(p->d_ic, sizeof(IterCtl));
    ALLOC(p->d_stop, sizeof(int));
    ALLOC(p->d_phi[0], sizeof(float) * C * G * 8);
    ALLOC(p->d_phi[1], sizeof(float) * C * G * 8);
    ALLOC(p->d_partial, sizeof(double) * partial_blocks(p->C, p->G) * G * 4);
    ALLOC(p->d_out4, sizeof(double) * G * 4);
    SweepSched &sc = p->sched;
    ALLOC(sc.d_probs, sizeof(DevProblem));
    ALLOC(sc.d_base, sizeof(long long) * 2);
    ALLOC(sc.d_ctl, sizeof(SweepCtl));
    ALLOC(sc.d_queue, sizeof(unsigned long long) * 8 * C);
    ALLOC(sc.d_seeds, sizeof(int) * 8 * C);
#undef ALLOC

    // host -> device (FP64 mesh; FP32 materials and quadrature)
    std::vector<float> f32(std::max<size_t>({C * G, (size_t)3 * p->nang, G}));
    auto up32 = [&](float *dst, const std::vector<double> &src) {
        for (size_t i = 0; i < src.size(); ++i) f32[i] = (float)src[i];
        return hipMemcpyAsync(dst, f32.data(), sizeof(float) * src.size(), hipMemcpyHostToDevice, s);
    };
    HIPCHK(p, hipMemcpyAsync(d_xyz, p->xyz.data(), sizeof(double) * 3 * p->nvert, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_cv, p->cv.data(), sizeof(int) * 8 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_nbr, nbr.data(), sizeof(int) * 6 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_nbrf, nbrf.data(), sizeof(int) * 6 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_perm, perm.data(), sizeof(unsigned) * 6 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    HIPCHK(p, up32(dsigt, p->sigt), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    HIPCHK(p, up32(dsigs, p->sigs), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    HIPCHK(p, up32(dq, p->q), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    HIPCHK(p, up32(dom, p->omega), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    HIPCHK(p, up32(dw, p->w), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    if (dpsib) {
        HIPCHK(p, up32(dpsib, p->psib), "copy");
        HIPCHK(p, hipStreamSynchronize(s), "sync");
    }
    HIPCHK(p, hipMemsetAsync(p->d_err, 0, sizeof(int), s), "memset");
    HIPCHK(p, hipMemsetAsync(dF, 0, sizeof(float) * 288 * C, s), "memset");

    // element matrices, then designation and levels
    HIPCHK(p, launch_geometry(d_xyz, d_cv, d_nbr, d_nbrf, d_perm, p->C, dM, dS, dF, p->d_area, p->d_err, s), "geometry");
    int herr = 0;
    HIPCHK(p, hipMemcpyAsync(&herr, p->d_err, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "geometry");
    if (herr & 1) { drop_device(p); return fail(p, SNX_E_MESH, "non-positive Jacobian at a Gauss point"); }
    HIPCHK(p, launch_dag_one(p->C, d_nbr, p->d_area, dmask, dindeg, dlevel, dhist, dnlev, dseeds, dnseed, dscratch,
                             p->d_err, s), "levelling");
    std::vector<int> nlev(16), nseed(8);
    HIPCHK(p, hipMemcpyAsync(&herr, p->d_err, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipMemcpyAsync(nlev.data(), dnlev, sizeof(int) * 16, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipMemcpyAsync(nseed.data(), dnseed, sizeof(int) * 8, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "levelling");
    if (herr & 2) { drop_device(p); return fail(p, SNX_E_MESH, "a face is tangent to an octant diagonal"); }
    if (herr & 4) { drop_device(p); return fail(p, SNX_E_CYCLE, "the upwind graph of an octant has a cycle"); }
    p->level.resize(8 * C);
    HIPCHK(p, hipMemcpy(p->level.data(), dlevel, sizeof(int) * 8 * C, hipMemcpyDeviceToHost), "copy");
    p->nlev.assign(nlev.begin(), nlev.begin() + 8);
    int maxin = 0;
    for (int o = 0; o < 8; ++o) maxin = std::max(maxin, nlev[8 + o]);

    HIPCHK(p, launch_octant_operators(p->C, dS, dF, dmask, dT, s), "octant operators");

    // level-0 tasks of every octant become the queues' seeds
    std::vector<int> seeds_host(8 * C), seeds;
    std::vector<std::vector<int>> seeds_by_octant(8);
    HIPCHK(p, hipMemcpy(seeds_host.data(), dseeds, sizeof(int) * 8 * C, hipMemcpyDeviceToHost), "copy");
    for (int o = 0; o < 8; ++o)
        for (int i = 0; i < nseed[o]; ++i) seeds_by_octant[o].push_back(o * p->C + seeds_host[(size_t)o * C + i]);
    layout_queues(sc.host_ctl, p->nq, p->xcc_queue, std::vector<long long>{(long long)p->C}, seeds_by_octant, seeds);

    hp.C = p->C; hp.G = p->G; hp.A = p->A; hp.nang = p->nang; hp.task_base = 0;
    hp.M = dM; hp.S = dS; hp.T = dT; hp.F = dF; hp.nbr = d_nbr; hp.perm = d_perm; hp.inmask = dmask; hp.indeg = dindeg;
    hp.sigt = dsigt; hp.sigs = dsigs; hp.q = dq; hp.r = dr; hp.omega = dom; hp.w = dw; hp.psib = dpsib;
    hp.psi = dpsi; hp.slot = dslot; hp.slotc = dslotc; hp.cnt = dcnt;
    sc.nprob = 1;
    sc.total = 8LL * p->C;
    sc.nseed = (int)seeds.size();
    sc.maxA = p->A; sc.maxG = p->G; sc.maxin = std::max(1, maxin);
    sc.threads = p->threads;
    sc.wg_per_cu = p->wg_per_cu;
    while (sc.threads < p->G) sc.threads *= 2;
    long long base[2] = {0, sc.total};
    HIPCHK(p, hipMemcpy(sc.d_probs, &hp, sizeof(DevProblem), hipMemcpyHostToDevice), "copy");
    HIPCHK(p, hipMemcpy(sc.d_base, base, sizeof(base), hipMemcpyHostToDevice), "copy");
    HIPCHK(p, hipMemcpy(sc.d_seeds, seeds.data(), sizeof(int) * seeds.size(), hipMemcpyHostToDevice), "copy");
    HIPCHK(p, reset_schedule(p, s), "reset");
    HIPCHK(p, launch_fill_f32(dr, C * G * 8, 0.f, s), "fill");
    HIPCHK(p, hipStreamSynchronize(s), "setup");
    snx_status st = configure_grid(p, sc);
    if (st) { drop_device(p); return st; }
    p->ready = true;
    return SNX_OK;
}

static snx_status enqueue_sweep(snx_problem *p, const int *stop, hipStream_t s, hipEvent_t ev0 = nullptr,
                                hipEvent_t ev1 = nullptr) {
    SweepSched &sc = p->sched;
    HIPCHK(p, launch_sweep_prologue(sc.d_ctl, sc.d_queue, sc.d_seeds, stop, s), "sweep prologue");
    if (ev0) HIPCHK(p, hipEventRecord(ev0, s), "event");
    HIPCHK(p, launch_sweep_kernel(sc.d_probs, sc.nprob, sc.d_base, sc.d_ctl, sc.d_queue, stop, sc.threads, sc.grid,
                                  sc.maxA, sc.maxG, sc.maxin, p->watchdog_ticks, s),
           "sweep launch");
    if (ev1) HIPCHK(p, hipEventRecord(ev1, s), "event");
    return SNX_OK;
}

snx_status snx_sweep(snx_problem *p, const float *phi_in, float *phi_out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (!phi_out || phi_in == phi_out) return fail(p, SNX_E_ARG, "phi_out must be non-NULL and distinct from phi_in");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(p, launch_source(p->sched.d_probs, 0, p->C, p->G, phi_in, nullptr, s), "source");
    snx_status st = enqueue_sweep(p, nullptr, s);
    if (st) return st;
    HIPCHK(p, launch_reduce(p->sched.d_probs, 0, p->C, p->G, phi_out, nullptr, false, nullptr, nullptr, s), "reduce");
    return SNX_OK;
}

// Captures `chunk` source iterations whose first one reads ping-pong buffer `parity`.
static snx_status build_graph(snx_problem *p, int parity) {
    hipStream_t cs = p->cap_stream;
    HIPCHK(p, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    snx_status st = SNX_OK;
    for (int i = 0; i < p->chunk && !st; ++i) {
        st = enqueue_sweep(p, p->d_stop, cs);
        if (!st) {
            const int cur = (parity + i) & 1;
            hipError_t e = launch_reduce(p->sched.d_probs, 0, p->C, p->G, p->d_phi[cur ^ 1], p->d_phi[cur], true,
                                         p->d_ic, p->d_stop, cs);
            if (e != hipSuccess) st = hip_fail(p, e, "reduce launch");
        }
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(p, e, "end capture");
    e = hipGraphInstantiate(&p->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(p, e, "graph instantiate");
    return SNX_OK;
}

snx_status snx_solve(snx_problem *p, double tol, int32_t max_it, const float *phi0, float *phi, snx_solve_info *info,
                     void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (!phi || max_it < 1 || !(tol >= 0.0)) return fail(p, SNX_E_ARG, "bad solve arguments");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t nphi = (size_t)p->C * p->G * 8;
    HIPCHK(p, launch_iter_init(p->d_ic, p->d_stop, max_it, tol, s), "init");
    if (phi0) HIPCHK(p, launch_copy_f32(p->d_phi[0], phi0, nphi, nullptr, s), "copy");
    else HIPCHK(p, launch_fill_f32(p->d_phi[0], nphi, 0.f, s), "fill");
    HIPCHK(p, launch_source(p->sched.d_probs, 0, p->C, p->G, p->d_phi[0], nullptr, s), "source");
    IterCtl *hic = reinterpret_cast<IterCtl *>(p->pinned);
    unsigned *habort = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(p->pinned) + 1024);
    int *hstop = reinterpret_cast<int *>(reinterpret_cast<char *>(p->pinned) + 2048);
    const long long max_launch = (max_it + p->chunk - 1) / p->chunk + 1;
    int done_iters = 0;
    for (long long l = 0; l < max_launch; ++l) {
        const int parity = done_iters & 1;
        if (!p->graph[parity]) {
            snx_status st = build_graph(p, parity);
            if (st) return st;
        }
        HIPCHK(p, hipGraphLaunch(p->graph[parity], s), "graph launch");
        HIPCHK(p, hipMemcpyAsync(hic, p->d_ic, sizeof(IterCtl), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipMemcpyAsync(habort, &p->sched.d_ctl->abort, sizeof(unsigned), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipMemcpyAsync(hstop, p->d_stop, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipStreamSynchronize(s), "solve");
        if (*habort) {
            (void)reset_schedule(p, s);
            (void)hipStreamSynchronize(s);
            return fail(p, SNX_E_DEVICE, "sweep watchdog expired (no ready task)");
        }
        if (*hstop) break;
        done_iters = hic->iter;
    }
    const int iters = hic->iter;
    HIPCHK(p, launch_copy_f32(phi, p->d_phi[iters & 1], nphi, nullptr, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "solve");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const bool conv = *hstop == 1;
    if (info) {
        info->iterations = iters;
        info->status = conv ? SNX_OK : SNX_E_NOCONV;
        info->residual = hic->last_eps;
        info->wall_ms = ms;
        info->solves_per_s = ms > 0 ? (double)iters * p->C * p->nang * p->G / (ms * 1e-3) : 0.0;
    }
    return conv ? SNX_OK : fail(p, SNX_E_NOCONV, "max_it reached before the tolerance");
}

snx_status snx_balance(snx_problem *p, const float *phi_in, const float *phi_out, double *out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (!phi_out || !out) return fail(p, SNX_E_ARG, "phi_out and out are required");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(p, launch_balance(p->sched.d_probs, 0, p->C, p->G, phi_in, phi_out, p->d_partial, p->d_out4, s), "balance");
    HIPCHK(p, hipMemcpyAsync(out, p->d_out4, sizeof(double) * 4 * p->G, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "balance");
    return SNX_OK;
}

snx_status snx_integrated_flux(snx_problem *p, const float *phi, double *out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (!phi || !out) return fail(p, SNX_E_ARG, "phi and out are required");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(p, launch_integrated_flux(p->hp.M, phi, p->C, p->G, p->d_partial, p->d_out4, s), "integrated flux");
    std::vector<double> tmp(4 * p->G);
    HIPCHK(p, hipMemcpyAsync(tmp.data(), p->d_out4, sizeof(double) * 4 * p->G, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "integrated flux");
    for (int g = 0; g < p->G; ++g) { out[2 * g] = tmp[4 * g]; out[2 * g + 1] = tmp[4 * g + 1]; }
    return SNX_OK;
}

snx_status snx_get_levels(snx_problem *p, int32_t *level, int32_t *nlevels) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (level) std::memcpy(level, p->level.data(), sizeof(int) * p->level.size());
    if (nlevels) std::memcpy(nlevels, p->nlev.data(), sizeof(int) * 8);
    return SNX_OK;
}

snx_status snx_set_schedule(snx_problem *p, int32_t threads, int32_t wg_per_cu, int32_t chunk) {
    if (!p) return SNX_E_ARG;
    if (threads > 0) {
        if (threads != 64 && threads != 128 && threads != 256 && threads != 512)
            return fail(p, SNX_E_ARG, "threads must be 64, 128, 256 or 512");
        if (p->have_mat && threads < p->G) return fail(p, SNX_E_ARG, "threads must be at least G");
        p->threads = threads;
        p->sched.threads = threads;
    }
    if (wg_per_cu > 0) { p->wg_per_cu = wg_per_cu; p->sched.wg_per_cu = wg_per_cu; }
    if (chunk > 0) p->chunk = chunk;
    drop_graph(p);
    if (p->ready) return configure_grid(p, p->sched);
    return SNX_OK;
}

snx_status snx_profile_sweep(snx_problem *p, int32_t nsweeps, const float *phi_in, float *phi_out, double *ms,
                             void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (nsweeps < 1 || !phi_out || !ms || phi_in == phi_out) return fail(p, SNX_E_ARG, "bad profile arguments");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    std::vector<hipEvent_t> ev(2 * nsweeps, nullptr);
    snx_status st = SNX_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) { st = fail(p, SNX_E_DEVICE, "hipEventCreate failed"); break; }
    for (int i = 0; i < nsweeps && !st; ++i) {
        hipError_t e = launch_source(p->sched.d_probs, 0, p->C, p->G, phi_in, nullptr, s);
        if (e != hipSuccess) { st = hip_fail(p, e, "source"); break; }
        st = enqueue_sweep(p, nullptr, s, ev[2 * i], ev[2 * i + 1]);
        if (st) break;
        e = launch_reduce(p->sched.d_probs, 0, p->C, p->G, phi_out, nullptr, false, nullptr, nullptr, s);
        if (e != hipSuccess) st = hip_fail(p, e, "reduce");
    }
    double total = 0.0;
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail(p, SNX_E_DEVICE, "profile sync failed");
    for (int i = 0; i < nsweeps && !st; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) != hipSuccess) st = fail(p, SNX_E_DEVICE, "event timing");
        total += t;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (!st) *ms = total / nsweeps;
    return st;
}

snx_status snx_sweep_stats(snx_problem *p, int64_t *out) {
    if (!p || !out) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    std::vector<SweepCtl> h(1);
    HIPCHK(p, hipDeviceSynchronize(), "sync");
    HIPCHK(p, hipMemcpy(h.data(), p->sched.d_ctl, sizeof(SweepCtl), hipMemcpyDeviceToHost), "copy");
    for (int i = 0; i < 11; ++i) out[i] = 0;
    for (int q = 0; q < h[0].nq; ++q) {
        const QueueCtl &Q = h[0].q[q];
        out[0] += (int64_t)Q.tasks_done;
        out[1] += (int64_t)Q.polls_empty;
        out[4] += (int64_t)Q.continued;
        for (int i = 0; i < 5; ++i) out[6 + i] += (int64_t)Q.phase[i];
    }
    out[2] = (int64_t)h[0].abort;
    out[3] = (int64_t)p->sched.grid;
    out[5] = (int64_t)p->sched.threads;
    return SNX_OK;
}

}  // extern "C"
