// C ABI of the gfx950 S_N sweep library: problems, batches, the sweep schedule,
// the graph-captured source-iteration loop and the schedule autotuner.
//
// A schedule drives one persistent sweep launch over one or more problems:
// the merged problem table, the task queues (one per XCD), the seeds and the
// per-problem iteration records.  A problem owns a schedule of one; a batch
// owns a schedule over its problems, so many uneven problems share every
// launch of the graph-captured loop, and a converged problem simply stops
// contributing tasks to later sweeps.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "snx_internal.h"

using namespace snx;

// Fixed device scratch of the entry points that allocate nothing
// (snx_integrated_flux_noalloc): every device the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not a device address: kernels and copies get the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchDoubles = size_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};

// This device's copy of `scratch`, looked up once per device with the device current.
hipError_t scratch_address(int device, double **addr) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_addr[device]) {
        void *a = nullptr;
        hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = static_cast<double *>(a);
    }
    *addr = g_scratch_addr[device];
    return hipSuccess;
}

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

int cu_count(int device) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
    return n;
}

}  // namespace

// ----------------------------------------------------------------- schedule

struct Sched {
    int device = 0;
    std::vector<snx_problem *> probs;        // not owned
    DevAlloc mem;
    DevProblem *d_probs = nullptr;
    long long *d_base = nullptr;             // [nprob + 1] first task of each problem
    SweepCtl *d_ctl = nullptr;
    unsigned long long *d_queue = nullptr;   // [total] slots, queue q from host_ctl.qbase[q]
    int *d_seeds = nullptr, *d_seed_off = nullptr;
    int *d_blk_base = nullptr;               // [nprob + 1] first 256-item block of each problem
    int nblk = 0;
    int *d_rblk_base = nullptr;              // [nprob + 1] the same for the reduction's 256*kReduceItems blocks
    int nrblk = 0;
    float **d_buf = nullptr;                 // [2][nprob] ping-pong flux buffers of the problems
    float **d_user = nullptr;                // [2][nprob] caller pointers of the current call
    IterCtl *d_ic = nullptr;                 // [nprob]
    int *d_stop = nullptr;                   // [nprob]
    void *pinned = nullptr;                  // host staging: pointer arrays and read-backs
    SweepCtl host_ctl{};
    std::vector<DevProblem> hprobs;
    long long total = 0;
    int maxA = 0, maxG = 0, maxin = 1;
    int maxAG = 0;                           // largest (angles per octant) * G of the problems
    bool one = false;                        // every task is one round of lanes (maxAG <= threads)
    bool ext = false;                        // a problem uses per-angle designation or reflective planes:
                                             // the kernel variant with them
    int threads = 256, wg_per_cu = 0, grid = 0, chunk = 8;
    int mode = SNX_SWEEP_AMT;                // SNX_SWEEP_AMT or SNX_SWEEP_BSP
    int depth = 1;                           // staging depth (snx_set_staging_depth): 1 = a task's or
                                             // round's inputs requested one step ahead, 0 = at its start
    bool phase_stats = false;                // gather the per-phase cycle statistics (snx_set_sweep_stats)
    bool fixed_outer = false;                // group-to-group matrices: keep the cross-group source fixed
                                             // (inner iterations of an outer one); else renew it every iteration
    const snx_problem *dirp = nullptr;       // the schedule's one problem when it sweeps in per-direction
                                             // order (see enqueue_sweep)
    bool dir_units = false;                  // its last sweep was the dependency-driven unit sweep
    long long *d_bsp_tasks = nullptr;        // tasks of every problem ordered by level (BSP comparator)
    std::vector<long long> bsp_off;          // [levels + 1] offsets into d_bsp_tasks
    unsigned long long watchdog = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // chunk starting from ping-pong buffer 0 / 1
    std::string err;

    int nprob() const { return (int)probs.size(); }
    void drop_graphs() {
        for (auto &g : graph) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
    void release() {
        drop_graphs();
        mem.release();
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
    }
};

struct snx_problem {
    int device = 0;
    std::string err;
    void *pinned = nullptr;            // host staging for small read-backs (4096 bytes)
    double *scratch = nullptr;         // device address of this device's fixed scratch

    // host inputs
    int C = 0, nvert = 0, nang = 0, A = 0, G = 0, bkind = 0;
    std::vector<double> xyz, omega, w, sigt, sigs, q, psib;
    std::vector<int> cv;
    bool have_mesh = false, have_quad = false, have_mat = false;
    int designation = SNX_DESIGNATION_OCTANT;
    int L = 0;                          // anisotropic scattering degree (snx_set_anisotropy)
    std::vector<double> sigl;           // [C][G][L]
    int refl = 0;                       // reflective planes (snx_set_reflective), bit 2*axis + side
    int nref = 0;                       // reflective boundary faces found at setup
    int nmat = 0;                       // group-to-group scattering (snx_set_group_scattering), 0 = none
    std::vector<int> cmat;              // [C]
    std::vector<double> sgg;            // [nmat][G][G], from g' into g
    int order = 1;                      // element order (snx_set_order): 1, 2 or 3

    // set-up results
    bool ready = false;
    DevAlloc mem;
    DevProblem hp{};
    std::vector<int> level, nlev;
    std::vector<std::vector<int>> seeds_by_octant;   // local task ids (8*K + o) of level-0 cells
    unsigned long long desig_counts[3] = {0, 0, 0};  // per-angle designation statistics (snx_designation_stats)
    // per-direction sweep order (SNX_DESIGNATION_DIRECTION): work items, lagged faces
    struct Dir {
        std::vector<long long> level_off;   // [levels + 1] offsets into the work units
        long long nunits = 0;               // units per sweep (8 C A)
        UnitCtl uctl_host;                  // the unit queues' fixed layout (epoch and queue state zero)
        long long cyclic = 0;               // directions whose graph had a cycle
        DirDev dev{};
    } dir;
    int maxin = 1;
    int *d_err = nullptr;
    float *d_phi[2] = {nullptr, nullptr};
    float *d_outer = nullptr;                        // second iterate buffer of snx_solve_outer
    unsigned long long *d_change = nullptr;          // [2] FP64 bits of the outer change norm
    double *d_partial = nullptr, *d_out4 = nullptr;
    double *d_area = nullptr;
    unsigned long long watchdog_ticks = 0;  // sweep watchdog in wall-clock ticks (snx_set_watchdog)
    double tick_hz = 1e8;                   // the device's wall-clock rate
    int threads = 0, wg_per_cu = 0, chunk = 8;     // requested sweep schedule (threads 0: automatic)
    int mode = SNX_SWEEP_AMT;
    int depth = 1;                      // requested staging depth (snx_set_staging_depth)
    bool mode_set = false;              // snx_set_sweep_mode was called
    bool phase_stats = false;           // per-phase cycle statistics of the sweep (snx_set_sweep_stats)
    int nq = 1;                         // task queues = XCDs seen on the device
    int xcc_queue[kMaxXcc] = {0};       // home queue of each hardware XCC id
    Sched sched;                        // the problem's own schedule of one
    // higher-order elements (order > 1): their matrices, fluxes and level lists
    struct Ho {
        float *M = nullptr, *R = nullptr, *psi = nullptr;
        double *S = nullptr, *F = nullptr;   // streaming and face matrices in FP64
        float *phi[2] = {nullptr, nullptr};
        int *perm = nullptr, *tasks = nullptr;
        double *omega64 = nullptr;      // [nang][3] directions in FP64
        std::vector<int> off;           // [levels + 1] offsets into tasks (all octants, by level)
        HoDev dev{};
    } ho;
};

struct snx_batch {
    int device = 0;
    Sched sched;
    int threads = 0, wg_per_cu = 0, chunk = 8;
    int mode = SNX_SWEEP_AMT;
};

namespace {

snx_status fail_msg(std::string &err, snx_status code, const std::string &msg) {
    err = msg;
    return code;
}
snx_status fail(snx_problem *p, snx_status code, const std::string &msg) {
    if (p) p->err = msg;
    return code;
}
snx_status hip_fail_msg(std::string &err, hipError_t e, const char *what) {
    return fail_msg(err, e == hipErrorOutOfMemory ? SNX_E_OOM : SNX_E_DEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK_E(err, expr, what)                                      \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return hip_fail_msg((err), e_, (what));  \
    } while (0)
#define HIPCHK(p, expr, what) HIPCHK_E((p)->err, expr, what)

void drop_device(snx_problem *p) {
    p->sched.release();
    p->sched = Sched{};
    p->mem.release();
    p->ready = false;
    p->hp = DevProblem{};
    p->ho = snx_problem::Ho{};
    p->dir = snx_problem::Dir{};
}

// ------------------------------------------------------- higher-order elements

int ho_nodes(const snx_problem *p) { return (p->order + 1) * (p->order + 1) * (p->order + 1); }

// Node map of each shared face at order P: for my face node at position
// i + m j (i along the face's first free axis u, j along the second v) the
// neighbour's local node.  The shared face's corners fix it: byte l of perm is
// the neighbour's local vertex at my face corner l = bu + 2 bv, so each of the
// neighbour's free axes follows one of mine, possibly reversed, and the nodes,
// symmetric about 0 on each axis, follow with it.
snx_status ho_node_maps(snx_problem *p, int P, const std::vector<int> &nbr, const std::vector<int> &nbrf,
                        const std::vector<unsigned> &perm, std::vector<int> &out) {
    const int m = P + 1, NF = m * m;
    out.assign((size_t)p->C * 6 * NF, -1);
    auto axes = [](int f, int &u, int &v) {
        const int a = f >> 1;
        u = a == 0 ? 1 : 0;
        v = a == 2 ? 1 : 2;
    };
    for (int K = 0; K < p->C; ++K)
        for (int f = 0; f < 6; ++f) {
            const int N = nbr[6 * (size_t)K + f], g = nbrf[6 * (size_t)K + f];
            if (N < 0) continue;
            int u2, v2;
            axes(g, u2, v2);
            int cu[4], cw[4];   // the neighbour's corner bits along u2 and v2 at my corner l
            for (int l = 0; l < 4; ++l) {
                const int w = (int)((perm[6 * (size_t)K + f] >> (8 * l)) & 0xffu);
                if (((w >> (g >> 1)) & 1) != (g & 1)) return fail(p, SNX_E_MESH, "neighbour vertex off the shared face");
                cu[l] = (w >> u2) & 1;
                cw[l] = (w >> v2) & 1;
            }
            const bool u_follows_u = cu[1] != cu[0];
            for (int l = 0; l < 4; ++l) {   // the map is one of the square's eight symmetries
                const int bu = l & 1, bv = l >> 1;
                const int eu = cu[0] ^ (u_follows_u ? bu : bv), ev = cw[0] ^ (u_follows_u ? bv : bu);
                if (eu != cu[l] || ev != cw[l]) return fail(p, SNX_E_MESH, "shared face corners do not match");
            }
            for (int j = 0; j < m; ++j)
                for (int i = 0; i < m; ++i) {
                    const int a = u_follows_u ? i : j, b = u_follows_u ? j : i;
                    int idx[3];
                    idx[g >> 1] = (g & 1) * P;
                    idx[u2] = cu[0] ? P - a : a;
                    idx[v2] = cw[0] ? P - b : b;
                    out[((size_t)K * 6 + f) * NF + i + m * j] = idx[0] + m * idx[1] + m * m * idx[2];
                }
        }
    return SNX_OK;
}

// Reference tables of the order-P element: Gauss-Lobatto-Legendre nodes and
// the (P+1)-point Gauss-Legendre rule (closed forms).
HoRef ho_reference(int P) {
    HoRef r{};
    if (P == 2) {
        const double a = std::sqrt(0.6);
        const double node[3] = {-1.0, 0.0, 1.0}, gx[3] = {-a, 0.0, a}, gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
        for (int i = 0; i < 3; ++i) { r.node[i] = node[i]; r.gx[i] = gx[i]; r.gw[i] = gw[i]; }
    } else {
        const double s5 = std::sqrt(0.2), t = 2.0 / 7.0 * std::sqrt(1.2);
        const double x1 = std::sqrt(3.0 / 7.0 - t), x2 = std::sqrt(3.0 / 7.0 + t);
        const double w1 = (18.0 + std::sqrt(30.0)) / 36.0, w2 = (18.0 - std::sqrt(30.0)) / 36.0;
        const double node[4] = {-1.0, -s5, s5, 1.0}, gx[4] = {-x2, -x1, x1, x2}, gw[4] = {w2, w1, w1, w2};
        for (int i = 0; i < 4; ++i) { r.node[i] = node[i]; r.gx[i] = gx[i]; r.gw[i] = gw[i]; }
    }
    return r;
}

// Workgroup width: the requested one if valid and at least G, else the
// narrowest width that holds a whole task in one round (at most 256), and never
// less than G.
int pick_threads(int requested, int maxG, int maxAG) {
    static const int kWidths[] = {64, 128, 192, 256, 512};
    if (requested > 0 && sweep_threads_valid(requested) && requested >= maxG) return requested;
    const int want = requested > 0 ? std::max(requested, maxG) : std::max(maxG, std::min(maxAG, 256));
    for (int w : kWidths)
        if (w >= want) return w;
    return 512;
}

// Grid of the persistent sweep: resident workgroups per CU times the CUs.
snx_status configure_grid(Sched &sc) {
    sc.one = sc.maxAG <= sc.threads;
    const size_t lds = sweep_lds_bytes(sc.threads, sc.maxA, sc.maxG, sc.maxin, sc.one);
    if (lds > 64 * 1024) return fail_msg(sc.err, SNX_E_ARG, "task does not fit in 64 KB of LDS (too many angles or groups)");
    const int occ = sweep_occupancy(sc.threads, sc.one, sc.ext, sc.depth, lds);
    if (occ <= 0) return fail_msg(sc.err, SNX_E_ARG, "sweep kernel cannot be resident with this schedule");
    const int per_cu = sc.wg_per_cu > 0 ? std::min(sc.wg_per_cu, occ) : occ;
    long long grid = (long long)cu_count(sc.device) * per_cu;
    if (grid > sc.total) grid = sc.total;
    sc.grid = (int)std::max(1LL, grid);
    return SNX_OK;
}

constexpr double kWatchdogSeconds = 20.0;   // default sweep watchdog: this long without a ready task

// Zero the scheduler state of every problem of the schedule (counters, epochs)
// and of the schedule (queue slots, abort flag, statistics); upload the layout.
hipError_t reset_schedule(Sched &sc, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (const DevProblem &P : sc.hprobs) {
        if (e == hipSuccess) e = launch_fill_u32(P.cnt, (size_t)8 * P.C, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(P.epoch, 1, 0u, s);
    }
    if (e == hipSuccess) e = hipMemsetAsync(sc.d_queue, 0, sizeof(unsigned long long) * (size_t)sc.total, s);
    if (sc.dirp && e == hipSuccess) {   // the per-direction order's counters, queue and epoch
        const DirDev &D = sc.dirp->dir.dev;
        const long long NU = sc.dirp->dir.nunits;
        e = launch_fill_u32(D.ucnt, (size_t)NU, 0u, s);
        if (e == hipSuccess) e = hipMemsetAsync(D.uqueue, 0, sizeof(unsigned long long) * (size_t)NU, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(D.uctl, &sc.dirp->dir.uctl_host, sizeof(UnitCtl), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(sc.d_ctl, &sc.host_ctl, sizeof(SweepCtl), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Builds a schedule over set-up problems (all on one device).
snx_status build_sched(Sched &sc, const std::vector<snx_problem *> &probs, int threads, int wg_per_cu, int chunk,
                       hipStream_t s) {
    sc.release();
    sc.probs = probs;
    snx_problem *p0 = probs[0];
    sc.device = p0->device;
    sc.watchdog = p0->watchdog_ticks;
    const int n = (int)probs.size();
    HIPCHK_E(sc.err, hipStreamCreateWithFlags(&sc.cap_stream, hipStreamNonBlocking), "stream");
    HIPCHK_E(sc.err, hipHostMalloc(&sc.pinned, 64 * (size_t)n + 4096, hipHostMallocDefault), "pinned");

    sc.hprobs.clear();
    std::vector<long long> base(n + 1, 0);
    std::vector<int> blk(n + 1, 0), rblk(n + 1, 0), seed_off(8 * n + 1, 0), seeds;
    sc.maxA = sc.maxG = sc.maxAG = 0;
    sc.maxin = 1;
    sc.ext = false;
    sc.dirp = nullptr;
    for (snx_problem *p : probs)
        if (p->designation == SNX_DESIGNATION_DIRECTION) {
            if (n > 1) return fail_msg(sc.err, SNX_E_ARG, "a problem swept in per-direction order cannot join a batch");
            sc.dirp = p;
        }
    for (int i = 0; i < n; ++i) {
        snx_problem *p = probs[i];
        DevProblem P = p->hp;
        P.task_base = base[i];
        sc.hprobs.push_back(P);
        base[i + 1] = base[i] + 8LL * p->C;
        blk[i + 1] = blk[i] + (int)(((long long)p->C * p->G + 255) / 256);
        rblk[i + 1] = rblk[i] + (int)(((long long)p->C * p->G + 256 * kReduceItems - 1) / (256 * kReduceItems));
        sc.maxA = std::max(sc.maxA, p->A);
        sc.maxG = std::max(sc.maxG, p->G);
        sc.maxAG = std::max(sc.maxAG, p->A * p->G);
        sc.maxin = std::max(sc.maxin, p->maxin);
        sc.ext = sc.ext || p->hp.amask != nullptr || p->hp.refl_in != nullptr || p->hp.mom != nullptr;
        for (int o = 0; o < 8; ++o) {
            seed_off[i * 8 + o] = (int)seeds.size();
            seeds.insert(seeds.end(), p->seeds_by_octant[o].begin(), p->seeds_by_octant[o].end());
        }
    }
    seed_off[8 * n] = (int)seeds.size();
    sc.total = base[n];
    // level lists of the bulk-synchronous comparator: task ids bucketed by level
    int maxlev = 0;
    for (snx_problem *p : probs)
        for (int l : p->level) maxlev = std::max(maxlev, l);
    sc.bsp_off.assign(maxlev + 2, 0);
    for (snx_problem *p : probs)
        for (int l : p->level) ++sc.bsp_off[l + 1];
    for (int l = 0; l <= maxlev; ++l) sc.bsp_off[l + 1] += sc.bsp_off[l];
    std::vector<long long> bsp(sc.total), fill(sc.bsp_off.begin(), sc.bsp_off.end() - 1);
    for (int i = 0; i < n; ++i) {
        const snx_problem *p = probs[i];
        for (int o = 0; o < 8; ++o)
            for (int K = 0; K < p->C; ++K)
                bsp[fill[p->level[(size_t)o * p->C + K]]++] = base[i] + 8LL * K + o;
    }
    sc.nblk = blk[n];
    sc.nrblk = rblk[n];
    sc.threads = pick_threads(threads, sc.maxG, sc.maxAG);
    sc.wg_per_cu = wg_per_cu;
    sc.chunk = chunk;

    // queue layout: octant o to queue o mod nq; each queue can hold all tasks of its octants
    SweepCtl &c = sc.host_ctl;
    c = SweepCtl{};
    c.nq = p0->nq;
    for (int x = 0; x < kMaxXcc; ++x) c.xcc_queue[x] = p0->xcc_queue[x];
    long long qb = 0;
    for (int q = 0; q < c.nq; ++q) {
        long long tot = 0;
        for (int o = q; o < 8; o += c.nq)
            for (snx_problem *p : probs) tot += p->C;
        c.qbase[q] = qb;
        c.qtotal[q] = tot;
        qb += tot;
    }

    DevAlloc &m = sc.mem;
#define SALLOC(ptr, bytes) HIPCHK_E(sc.err, m.alloc((void **)&(ptr), (bytes)), "device allocation")
    SALLOC(sc.d_probs, sizeof(DevProblem) * n);
    SALLOC(sc.d_base, sizeof(long long) * (n + 1));
    SALLOC(sc.d_ctl, sizeof(SweepCtl));
    SALLOC(sc.d_queue, sizeof(unsigned long long) * sc.total);
    SALLOC(sc.d_bsp_tasks, sizeof(long long) * sc.total);
    SALLOC(sc.d_seeds, sizeof(int) * std::max<size_t>(1, seeds.size()));
    SALLOC(sc.d_seed_off, sizeof(int) * (8 * n + 1));
    SALLOC(sc.d_blk_base, sizeof(int) * (n + 1));
    SALLOC(sc.d_rblk_base, sizeof(int) * (n + 1));
    SALLOC(sc.d_buf, sizeof(float *) * 2 * n);
    SALLOC(sc.d_user, sizeof(float *) * 2 * n);
    SALLOC(sc.d_ic, sizeof(IterCtl) * n);
    SALLOC(sc.d_stop, sizeof(int) * n);
#undef SALLOC
    std::vector<float *> bufs(2 * n);
    for (int i = 0; i < n; ++i) {
        bufs[i] = probs[i]->d_phi[0];
        bufs[n + i] = probs[i]->d_phi[1];
    }
    HIPCHK_E(sc.err, hipMemcpy(sc.d_probs, sc.hprobs.data(), sizeof(DevProblem) * n, hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemcpy(sc.d_base, base.data(), sizeof(long long) * (n + 1), hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemcpy(sc.d_bsp_tasks, bsp.data(), sizeof(long long) * sc.total, hipMemcpyHostToDevice),
             "copy");
    if (!seeds.empty())
        HIPCHK_E(sc.err, hipMemcpy(sc.d_seeds, seeds.data(), sizeof(int) * seeds.size(), hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemcpy(sc.d_seed_off, seed_off.data(), sizeof(int) * (8 * n + 1), hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemcpy(sc.d_blk_base, blk.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemcpy(sc.d_rblk_base, rblk.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemcpy(sc.d_buf, bufs.data(), sizeof(float *) * 2 * n, hipMemcpyHostToDevice), "copy");
    HIPCHK_E(sc.err, hipMemset(sc.d_stop, 0, sizeof(int) * n), "memset");
    HIPCHK_E(sc.err, reset_schedule(sc, s), "reset");
    return configure_grid(sc);
}

// Prologue and persistent sweep of the schedule; events (optional) bracket the
// sweep kernel alone.
snx_status enqueue_sweep(Sched &sc, const int *stops, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr) {
    if (sc.dirp) {   // per-direction order: lag snapshot, the sweep (dependency-driven or by level), octant slots
        const snx_problem *p = sc.dirp;
        const DirDev &D = p->dir.dev;
        if (ev0) HIPCHK_E(sc.err, hipEventRecord(ev0, s), "event");
        HIPCHK_E(sc.err, launch_lag_snapshot(D, sc.d_probs, p->G, stops, s), "lag snapshot");
        sc.dir_units = sc.mode == SNX_SWEEP_AMT && p->G <= 64;
        if (sc.mode == SNX_SWEEP_AMT && p->G <= 64) {   // dependency-driven: one persistent launch
            HIPCHK_E(sc.err, launch_unit_sweep(D, sc.d_probs, &sc.d_ctl->abort, sc.watchdog, stops, sc.phase_stats, s),
                     "unit sweep");
        } else {                                        // level by level
            for (size_t l = 0; l + 1 < p->dir.level_off.size(); ++l)
                HIPCHK_E(sc.err, launch_sweep_dir_level(D, sc.d_probs, sc.threads, p->dir.level_off[l],
                                                        p->dir.level_off[l + 1], stops, s), "level launch");
        }
        HIPCHK_E(sc.err, launch_dir_slots(sc.d_probs, p->C, p->G, stops, s), "slots");
        if (ev1) HIPCHK_E(sc.err, hipEventRecord(ev1, s), "event");
        return SNX_OK;
    }
    // reflective planes: the last sweep's outflow becomes this sweep's inflow
    for (int i = 0; i < sc.nprob(); ++i) {
        const DevProblem &P = sc.hprobs[i];
        if (P.refl_in)
            HIPCHK_E(sc.err, launch_copy_f32(P.refl_in, P.refl_out, (size_t)8 * P.nref * 4 * P.A * P.G,
                                             stops ? stops + i : nullptr, s), "reflective copy");
    }
    if (sc.mode == SNX_SWEEP_BSP) {   // one launch per level; the kernel boundary is the barrier
        if (ev0) HIPCHK_E(sc.err, hipEventRecord(ev0, s), "event");
        for (size_t l = 0; l + 1 < sc.bsp_off.size(); ++l)
            HIPCHK_E(sc.err, launch_sweep_level(sc.d_probs, sc.nprob(), sc.d_base, sc.d_ctl, sc.threads, sc.one,
                                                sc.grid, sc.maxA, sc.maxG, sc.maxin, sc.d_bsp_tasks, sc.bsp_off[l],
                                                sc.bsp_off[l + 1], stops, sc.depth, sc.ext, s), "level launch");
        if (ev1) HIPCHK_E(sc.err, hipEventRecord(ev1, s), "event");
        return SNX_OK;
    }
    HIPCHK_E(sc.err, launch_sweep_prologue(sc.d_ctl, sc.d_queue, sc.d_probs, sc.nprob(), sc.d_seeds, sc.d_seed_off,
                                           stops, s), "sweep prologue");
    if (ev0) HIPCHK_E(sc.err, hipEventRecord(ev0, s), "event");
    HIPCHK_E(sc.err, launch_sweep_kernel(sc.d_probs, sc.nprob(), sc.d_base, sc.d_ctl, sc.d_queue, sc.threads, sc.one,
                                         sc.grid, sc.maxA, sc.maxG, sc.maxin, sc.watchdog, sc.phase_stats, sc.depth,
                                         sc.ext, s),
             "sweep launch");
    if (ev1) HIPCHK_E(sc.err, hipEventRecord(ev1, s), "event");
    return SNX_OK;
}

// Inner iterations of outer ones, for the lifetime of the object: the graph
// chunk is the inner count and the cross-group source stays fixed; both are
// restored after (graphs are rebuilt when either changes).
struct OuterScope {
    Sched &sc;
    int saved;
    OuterScope(Sched &s, int chunk) : sc(s), saved(s.chunk) {
        if (chunk != saved || !sc.fixed_outer) {
            sc.chunk = chunk;
            sc.fixed_outer = true;
            sc.drop_graphs();
        }
    }
    ~OuterScope() {
        sc.chunk = saved;
        sc.fixed_outer = false;
        sc.drop_graphs();
    }
};

// Anisotropic problems of the schedule: flux moments of their last sweep's psi
// and the moments' source dofs; stops (device, nullable) retires problems.  The
// isotropic source comes from the source update as before.
snx_status enqueue_ang_sources(Sched &sc, const int *stops, hipStream_t s) {
    for (int i = 0; i < sc.nprob(); ++i) {
        const DevProblem &P = sc.hprobs[i];
        if (!P.mom) continue;
        HIPCHK_E(sc.err, launch_moments(sc.d_probs, i, P.C, P.G, stops ? stops + i : nullptr, s), "moments");
    }
    return SNX_OK;
}

// Uploads caller pointers: d_user[0][p] = a[p], d_user[1][p] = b[p] (either array may be NULL).
snx_status upload_user(Sched &sc, const float *const *a, const float *const *b, hipStream_t s) {
    const int n = sc.nprob();
    const float **h = reinterpret_cast<const float **>(sc.pinned);
    HIPCHK_E(sc.err, hipStreamSynchronize(s), "sync");        // the staging area may still be read
    for (int i = 0; i < n; ++i) {
        h[i] = a ? a[i] : nullptr;
        h[n + i] = b ? b[i] : nullptr;
    }
    HIPCHK_E(sc.err, hipMemcpyAsync(sc.d_user, h, sizeof(float *) * 2 * n, hipMemcpyHostToDevice, s), "copy");
    HIPCHK_E(sc.err, hipStreamSynchronize(s), "sync");
    return SNX_OK;
}

// One source iteration of every problem: source from d_user[0], sweep, reduction into d_user[1].
snx_status sched_sweep(Sched &sc, const float *const *phi_in, float *const *phi_out, hipStream_t s) {
    snx_status st = upload_user(sc, phi_in, phi_out, s);
    if (st) return st;
    const int n = sc.nprob();
    HIPCHK_E(sc.err, launch_iter_init_batch(sc.d_ic, sc.d_stop, n, 1, 0.0, s), "init");
    for (int i = 0; i < n; ++i)   // group-to-group matrices: one Jacobi step over groups
        if (sc.hprobs[i].qo)
            HIPCHK_E(sc.err, launch_outer_source(sc.d_probs, i, sc.hprobs[i].C, sc.hprobs[i].G, phi_in ? phi_in[i] : nullptr,
                                                 s), "outer source");
    HIPCHK_E(sc.err, launch_source_batch(sc.d_probs, n, sc.d_blk_base, sc.nblk, sc.d_user, nullptr, s), "source");
    st = enqueue_ang_sources(sc, nullptr, s);
    if (st) return st;
    st = enqueue_sweep(sc, nullptr, s);
    if (st) return st;
    HIPCHK_E(sc.err, launch_reduce_batch(sc.d_probs, n, sc.d_rblk_base, sc.nrblk, sc.d_user + n, nullptr, 0, nullptr,
                                         sc.d_stop, s), "reduce");
    return SNX_OK;
}

// Captures `chunk` source iterations whose first one reads ping-pong buffer `parity`.
snx_status build_graph(Sched &sc, int parity) {
    hipStream_t cs = sc.cap_stream;
    const int n = sc.nprob();
    HIPCHK_E(sc.err, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    snx_status st = SNX_OK;
    for (int i = 0; i < sc.chunk && !st; ++i) {
        st = enqueue_sweep(sc, sc.d_stop, cs);
        if (!st) {
            const int cur = (parity + i) & 1;
            hipError_t e = launch_reduce_batch(sc.d_probs, n, sc.d_rblk_base, sc.nrblk, sc.d_buf + (cur ^ 1) * n,
                                               sc.d_buf + cur * n, 1, sc.d_ic, sc.d_stop, cs);
            if (e != hipSuccess) st = hip_fail_msg(sc.err, e, "reduce launch");
            if (!st) st = enqueue_ang_sources(sc, sc.d_stop, cs);   // anisotropic: moments of this sweep
            for (int k = 0; k < n && !st && !sc.fixed_outer; ++k) {
                // group-to-group matrices: the next sweep's cross-group source from the new
                // flux, then its source dofs again (the reduction used the previous one)
                const DevProblem &P = sc.hprobs[k];
                if (!P.qo) continue;
                hipError_t e2 = launch_outer_source(sc.d_probs, k, P.C, P.G, sc.probs[k]->d_phi[cur ^ 1], cs,
                                                    sc.d_stop + k);
                if (e2 == hipSuccess) e2 = launch_source(sc.d_probs, k, P.C, P.G, sc.probs[k]->d_phi[cur ^ 1],
                                                         sc.d_stop + k, cs);
                if (e2 != hipSuccess) st = hip_fail_msg(sc.err, e2, "outer source launch");
            }
        }
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail_msg(sc.err, e, "end capture");
    e = hipGraphInstantiate(&sc.graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail_msg(sc.err, e, "graph instantiate");
    return SNX_OK;
}

// Source iteration of every problem of the schedule until each one's FP64
// relative change is <= tol or max_it; graph replays of `chunk` iterations,
// with converged problems retired from later sweeps.
snx_status sched_solve(Sched &sc, double tol, int max_it, const float *const *phi0, float *const *phi,
                       snx_solve_info *infos, hipStream_t s, const std::vector<int> *retired = nullptr) {
    const int n = sc.nprob();
    const auto t0 = std::chrono::steady_clock::now();
    snx_status st = upload_user(sc, phi0, nullptr, s);
    if (st) return st;
    HIPCHK_E(sc.err, launch_iter_init_batch(sc.d_ic, sc.d_stop, n, max_it, tol, s), "init");
    if (retired) {   // problems left out of this solve (their phi is passed through unchanged)
        std::vector<int> init(n);
        for (int i = 0; i < n; ++i) init[i] = (*retired)[i] ? 3 : 0;
        HIPCHK_E(sc.err, hipMemcpyAsync(sc.d_stop, init.data(), sizeof(int) * n, hipMemcpyHostToDevice, s), "copy");
        HIPCHK_E(sc.err, hipStreamSynchronize(s), "copy");
    }
    HIPCHK_E(sc.err, launch_copy_batch(sc.d_probs, n, sc.d_blk_base, sc.nblk, sc.d_buf, sc.d_user, s), "copy");
    if (!sc.fixed_outer)   // group-to-group matrices: the whole source from the start flux (Jacobi over groups)
        for (int i = 0; i < n; ++i)
            if (sc.hprobs[i].qo)
                HIPCHK_E(sc.err, launch_outer_source(sc.d_probs, i, sc.hprobs[i].C, sc.hprobs[i].G,
                                                     sc.probs[i]->d_phi[0], s, sc.d_stop + i), "outer source");
    HIPCHK_E(sc.err, launch_source_batch(sc.d_probs, n, sc.d_blk_base, sc.nblk, sc.d_buf, sc.d_stop, s), "source");
    st = enqueue_ang_sources(sc, sc.d_stop, s);
    if (st) return st;
    char *pin = reinterpret_cast<char *>(sc.pinned);
    IterCtl *hic = reinterpret_cast<IterCtl *>(pin + 16 * (size_t)n);
    int *hstop = reinterpret_cast<int *>(pin + 64 * (size_t)n);
    unsigned *habort = reinterpret_cast<unsigned *>(pin + 64 * (size_t)n + 2048);
    static_assert(sizeof(IterCtl) <= 48, "IterCtl staging");
    const long long max_launch = (max_it + sc.chunk - 1) / sc.chunk + 1;
    int done_iters = 0;
    for (long long l = 0; l < max_launch; ++l) {
        const int parity = done_iters & 1;
        if (!sc.graph[parity]) {
            st = build_graph(sc, parity);
            if (st) return st;
        }
        HIPCHK_E(sc.err, hipGraphLaunch(sc.graph[parity], s), "graph launch");
        HIPCHK_E(sc.err, hipMemcpyAsync(hstop, sc.d_stop, sizeof(int) * n, hipMemcpyDeviceToHost, s), "copy");
        HIPCHK_E(sc.err, hipMemcpyAsync(habort, &sc.d_ctl->abort, sizeof(unsigned), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK_E(sc.err, hipStreamSynchronize(s), "solve");
        if (*habort) {
            (void)reset_schedule(sc, s);
            return fail_msg(sc.err, SNX_E_DEVICE, "sweep watchdog expired (no ready task)");
        }
        bool all = true;
        for (int i = 0; i < n; ++i) all = all && hstop[i];
        if (all) break;
        // every problem still running has done chunk more iterations
        done_iters += sc.chunk;
    }
    HIPCHK_E(sc.err, hipMemcpyAsync(hic, sc.d_ic, sizeof(IterCtl) * n, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK_E(sc.err, hipStreamSynchronize(s), "solve");
    // each problem's final iterate sits in buffer (its iterations mod 2)
    std::vector<const float *> src(n);
    for (int i = 0; i < n; ++i) src[i] = sc.probs[i]->d_phi[hic[i].iter & 1];
    std::vector<IterCtl> ic(hic, hic + n);
    std::vector<int> stops(hstop, hstop + n);
    st = upload_user(sc, src.data(), phi, s);
    if (st) return st;
    HIPCHK_E(sc.err, launch_copy_batch(sc.d_probs, n, sc.d_blk_base, sc.nblk, sc.d_user + n, sc.d_user, s), "copy");
    HIPCHK_E(sc.err, hipStreamSynchronize(s), "solve");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool conv = true;
    for (int i = 0; i < n; ++i) {
        conv = conv && stops[i] == 1;
        if (infos) {
            const snx_problem *p = sc.probs[i];
            infos[i].iterations = ic[i].iter;
            infos[i].status = stops[i] == 1 ? SNX_OK : SNX_E_NOCONV;
            infos[i].residual = ic[i].last_eps;
            infos[i].wall_ms = ms;
            infos[i].solves_per_s = ms > 0 ? (double)ic[i].iter * p->C * p->nang * p->G / (ms * 1e-3) : 0.0;
        }
    }
    return conv ? SNX_OK : fail_msg(sc.err, SNX_E_NOCONV, "max_it reached before the tolerance");
}

// Statistics of the most recent sweep of the schedule (see snx_sweep_stats).
snx_status sched_stats(Sched &sc, int64_t *out) {
    std::vector<SweepCtl> h(1);
    HIPCHK_E(sc.err, hipDeviceSynchronize(), "sync");
    HIPCHK_E(sc.err, hipMemcpy(h.data(), sc.d_ctl, sizeof(SweepCtl), hipMemcpyDeviceToHost), "copy");
    for (int i = 0; i < 11; ++i) out[i] = 0;
    for (int q = 0; q < h[0].nq; ++q) {
        const QueueCtl &Q = h[0].q[q];
        out[0] += (int64_t)Q.tasks_done;
        out[1] += (int64_t)Q.polls_empty;
        out[4] += (int64_t)Q.continued;
        for (int i = 0; i < 5; ++i) out[6 + i] += (int64_t)Q.phase[i];
    }
    out[2] = (int64_t)h[0].abort;
    out[3] = (int64_t)sc.grid;
    out[5] = (int64_t)sc.threads;
    // an aborted sweep leaves counters, queues and epochs inconsistent: re-arm
    // them (the statistics below are read first)
    const bool rearm = h[0].abort != 0;
    if (sc.dirp && sc.dir_units) {   // the per-direction unit sweep's own statistics
        UnitCtl u;
        HIPCHK_E(sc.err, hipMemcpy(&u, sc.dirp->dir.dev.uctl, sizeof(UnitCtl), hipMemcpyDeviceToHost), "copy");
        for (int i = 0; i < 11; ++i)
            if (i != 2 && i != 5) out[i] = 0;
        for (int q = 0; q < kUnitQueues; ++q) {
            const UnitStat &S = u.st[q];
            out[0] += (int64_t)S.units;
            out[1] += (int64_t)S.polls;
            out[3] += (int64_t)S.rounds;
            out[4] += (int64_t)S.carried;
            for (int i = 0; i < 4; ++i) out[6 + i] += (int64_t)S.phase[i];
        }
        out[5] = 64;
    }
    if (rearm) {
        hipStream_t s0 = nullptr;
        HIPCHK_E(sc.err, reset_schedule(sc, s0), "re-arm after an abort");
        HIPCHK_E(sc.err, hipDeviceSynchronize(), "sync");
    }
    return SNX_OK;
}

// Mean duration (ms) of the sweep kernel over `reps` sweeps, from events on s.
snx_status time_sweeps(Sched &sc, int reps, hipStream_t s, double *ms) {
    std::vector<hipEvent_t> ev(2 * reps, nullptr);
    snx_status st = SNX_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) { st = fail_msg(sc.err, SNX_E_DEVICE, "hipEventCreate failed"); break; }
    for (int i = 0; i < reps && !st; ++i) st = enqueue_sweep(sc, nullptr, s, ev[2 * i], ev[2 * i + 1]);
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail_msg(sc.err, SNX_E_DEVICE, "sync failed");
    double total = 0.0;
    for (int i = 0; i < reps && !st; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) != hipSuccess) st = fail_msg(sc.err, SNX_E_DEVICE, "event");
        total += t;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (!st) *ms = total / reps;
    return st;
}

// ---------------------------------------------------------------- autotuner
//
// The schedule's knobs are the workgroup width (threads, i.e. how many of a
// task's (angle, group) solves run side by side: 64 per wavefront) and the
// resident workgroups per CU.  The tuner times a few sweeps of every candidate
// on the actual problems and keeps the fastest; results are cached in a text
// file of JSON lines keyed by device, problem shape and sweep-kernel revision
// (kSweepRevision: a schedule tuned for another kernel is not reused).

std::string tune_key(const Sched &sc) {
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, sc.device);
    long long cells = 0, solves = 0;
    for (const snx_problem *p : sc.probs) {
        cells += p->C;
        solves += (long long)p->C * p->nang * p->G;
    }
    int cb = 0, sb = 0;   // size buckets: log2 of cells and solves
    while ((1LL << (cb + 1)) <= cells) ++cb;
    while ((1LL << (sb + 1)) <= solves) ++sb;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|cu%d|np%d|A%d|G%d|c%d|s%d|k%d%s", prop.gcnArchName, cu_count(sc.device),
                  sc.nprob(), sc.maxA, sc.maxG, cb, sb, kSweepRevision, sc.ext ? "|ext" : "");
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, int &threads, int &wg, int &mode, int &depth) {
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[300];
        int t = 0, w = 0, m = SNX_SWEEP_AMT, d = 1;   // entries written before the depth knob: depth 1
        const int got = std::sscanf(line, "{\"key\": \"%299[^\"]\", \"threads\": %d, \"wg_per_cu\": %d, \"mode\": %d, "
                                    "\"depth\": %d", k, &t, &w, &m, &d);
        if (got >= 4 && key == k && (m == SNX_SWEEP_AMT || m == SNX_SWEEP_BSP) && (d == 0 || d == 1)) {
            threads = t;
            wg = w;
            mode = m;
            depth = got == 5 ? d : 1;
            found = true;   // the last entry for a key wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, int threads, int wg, int mode, int depth, double ms) {
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"wg_per_cu\": %d, \"mode\": %d, \"depth\": %d, \"ms\": %.6f}\n",
                 key.c_str(), threads, wg, mode, depth, ms);
    std::fclose(f);
}

snx_status tune_sched(Sched &sc, const char *cache, hipStream_t s, int *out_threads, int *out_wg, double *out_ms) {
    const std::string key = tune_key(sc);
    int t = 0, w = 0, md = SNX_SWEEP_AMT, dp = 1;
    if (cache_lookup(cache, key, t, w, md, dp) && t >= sc.maxG) {
        sc.threads = t;
        sc.wg_per_cu = w;
        sc.mode = md;
        sc.depth = dp;
        sc.drop_graphs();
        if (!configure_grid(sc)) {
            *out_threads = t;
            *out_wg = w;
            *out_ms = -1.0;
            return SNX_OK;
        }
    }
    // Candidates: the dependency-driven sweep at every (threads, workgroups per CU)
    // and the level-synchronous one at every width (its grid only caps a level's
    // workgroups).  Small meshes favour the second: a level launch costs less than
    // the latency of a chain of dependent tasks through device-coherent memory.
    // The dependency-driven candidates also try both staging depths (inputs
    // requested one task or round ahead, or at its start).
    // Two passes, each candidate's best pass counts (clock and thermal drift
    // during the first pass does not decide).
    struct Cand { int th, wg, mode, depth; double ms; };
    std::vector<Cand> cands;
    for (int th : {64, 128, 192, 256, 512}) {
        if (th < sc.maxG) continue;
        for (int dp : {1, 0})
            for (int wg : {0, 2, 4, 8}) cands.push_back({th, wg, SNX_SWEEP_AMT, dp, 1e300});
        cands.push_back({th, 0, SNX_SWEEP_BSP, 1, 1e300});
    }
    for (int pass = 0; pass < 2; ++pass)
        for (Cand &c : cands) {
            sc.threads = c.th;
            sc.wg_per_cu = c.wg;
            sc.mode = c.mode;
            sc.depth = c.depth;
            if (configure_grid(sc)) continue;
            double ms = 0.0;
            snx_status st = time_sweeps(sc, 1, s, &ms);           // warm-up
            if (!st) st = time_sweeps(sc, 3, s, &ms);
            if (st) return st;
            c.ms = std::min(c.ms, ms);
        }
    double best = 1e300;
    int bt = sc.threads, bw = sc.wg_per_cu, bm = sc.mode, bd = sc.depth;
    for (const Cand &c : cands)
        if (c.ms < best) { best = c.ms; bt = c.th; bw = c.wg; bm = c.mode; bd = c.depth; }
    sc.threads = bt;
    sc.wg_per_cu = bw;
    sc.mode = bm;
    sc.depth = bd;
    sc.drop_graphs();
    snx_status st = configure_grid(sc);
    if (st) return st;
    cache_store(cache, key, bt, bw, bm, bd, best);
    *out_threads = bt;
    *out_wg = bw;
    *out_ms = best;
    return SNX_OK;
}

}  // namespace

extern "C" {

// ----------------------------------------------------------------- problems

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
    if (e == hipSuccess) e = hipHostMalloc(&p->pinned, 4096, hipHostMallocDefault);
    if (e == hipSuccess) e = scratch_address(device, &p->scratch);
    if (e != hipSuccess) {
        g_create_error = std::string("HIP initialisation failed: ") + hipGetErrorString(e);
        if (p->pinned) (void)hipHostFree(p->pinned);
        delete p;
        return SNX_E_DEVICE;
    }
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    p->tick_hz = (double)rate_khz * 1000.0;
    p->watchdog_ticks = (unsigned long long)(p->tick_hz * kWatchdogSeconds);   // without a ready task
    // Which XCDs do workgroups land on?  Each distinct XCC id becomes one task queue.
    {
        const int nb = 8 * cu_count(device);
        int *d_ids = nullptr;
        std::vector<int> ids(nb, 0);
        e = hipMalloc((void **)&d_ids, sizeof(int) * nb);
        if (e == hipSuccess) e = launch_xcc_probe(d_ids, nb, nullptr);
        if (e == hipSuccess) e = hipMemcpy(ids.data(), d_ids, sizeof(int) * nb, hipMemcpyDeviceToHost);
        if (d_ids) (void)hipFree(d_ids);
        if (e != hipSuccess) {
            g_create_error = std::string("XCD probe failed: ") + hipGetErrorString(e);
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
    *out = p;
    return SNX_OK;
}

void snx_destroy(snx_problem *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    drop_device(p);
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

snx_status snx_set_anisotropy(snx_problem *p, int32_t L, const double *sigma_l) {
    if (!p) return SNX_E_ARG;
    if (!p->have_mat) return fail(p, SNX_E_STATE, "set the materials before the anisotropy");
    if (L < 0 || L > 3 || (L > 0 && !sigma_l)) return fail(p, SNX_E_ARG, "0 <= L <= 3 and sigma_l required");
    const size_t n = (size_t)p->C * p->G * L;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(sigma_l[i])) return fail(p, SNX_E_ARG, "sigma_l must be finite");
    p->L = L;
    p->sigl.assign(sigma_l, sigma_l + n);
    drop_device(p);
    return SNX_OK;
}

snx_status snx_set_reflective(snx_problem *p, int32_t planes) {
    if (!p) return SNX_E_ARG;
    if (planes < 0 || planes > 63) return fail(p, SNX_E_ARG, "planes is a 6-bit mask (bit 2*axis + side)");
    p->refl = planes;
    drop_device(p);
    return SNX_OK;
}

snx_status snx_set_group_scattering(snx_problem *p, int32_t nmat, const int32_t *cell_mat, const double *sigma_gg) {
    if (!p) return SNX_E_ARG;
    if (!p->have_mat) return fail(p, SNX_E_STATE, "set the materials before the group scattering");
    if (nmat == 0) {
        p->nmat = 0;
        p->cmat.clear();
        p->sgg.clear();
        drop_device(p);
        return SNX_OK;
    }
    if (nmat < 0 || !cell_mat || !sigma_gg) return fail(p, SNX_E_ARG, "bad group scattering arguments");
    for (int K = 0; K < p->C; ++K)
        if (cell_mat[K] < 0 || cell_mat[K] >= nmat) return fail(p, SNX_E_ARG, "material index out of range");
    const size_t n = (size_t)nmat * p->G * p->G;
    for (size_t i = 0; i < n; ++i)
        if (!(sigma_gg[i] >= 0.0) || !std::isfinite(sigma_gg[i]))
            return fail(p, SNX_E_ARG, "scattering cross sections must be finite and >= 0");
    p->nmat = nmat;
    p->cmat.assign(cell_mat, cell_mat + p->C);
    p->sgg.assign(sigma_gg, sigma_gg + n);
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

snx_status snx_set_designation(snx_problem *p, int32_t kind) {
    if (!p) return SNX_E_ARG;
    if (kind != SNX_DESIGNATION_OCTANT && kind != SNX_DESIGNATION_ANGLE && kind != SNX_DESIGNATION_DIRECTION)
        return fail(p, SNX_E_ARG, "designation must be SNX_DESIGNATION_OCTANT, _ANGLE or _DIRECTION");
    p->designation = kind;
    drop_device(p);
    return SNX_OK;
}

snx_status snx_setup(snx_problem *p, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->have_mesh || !p->have_quad || !p->have_mat) return fail(p, SNX_E_STATE, "mesh, quadrature and materials must be set");
    if (p->bkind == 1 && (int)p->psib.size() != p->G) return fail(p, SNX_E_STATE, "boundary inflow size differs from G");
    if (p->order > 1 && (p->designation != SNX_DESIGNATION_OCTANT || p->refl || p->L || p->nmat))
        return fail(p, SNX_E_ARG, "per-angle designation, reflective planes, anisotropic and group-to-group "
                                  "scattering are not available at order > 1");
    if (p->designation == SNX_DESIGNATION_DIRECTION && (p->refl || p->L))
        return fail(p, SNX_E_ARG, "reflective planes and anisotropic scattering are not available with the "
                                  "per-direction sweep order");
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
    float *dM, *dS, *dT, *dF, *dsigt, *dsigs, *dq, *dr, *dom, *dw, *dpsib = nullptr, *dpsi, *dslot, *dslotc;
    unsigned char *dmask; int *dindeg, *dlevel, *dhist, *dnlev, *dseeds, *dnseed, *dscratch, *drec; unsigned *dcnt, *depoch;
#define ALLOC(ptr, bytes) HIPCHK(p, m.alloc((void **)&(ptr), (bytes)), "device allocation")
    ALLOC(d_xyz, sizeof(double) * 3 * p->nvert);
    ALLOC(d_cv, sizeof(int) * 8 * C);
    ALLOC(d_nbr, sizeof(int) * 6 * C);
    ALLOC(d_nbrf, sizeof(int) * 6 * C);
    ALLOC(d_perm, sizeof(unsigned) * 6 * C);
    ALLOC(dM, sizeof(float) * 64 * C);
    ALLOC(dS, sizeof(float) * 192 * C);
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
    ALLOC(drec, sizeof(int) * 8 * C * kRecWords);
    ALLOC(depoch, sizeof(unsigned));
    ALLOC(p->d_phi[0], sizeof(float) * C * G * 8);
    ALLOC(p->d_phi[1], sizeof(float) * C * G * 8);
    ALLOC(p->d_partial, sizeof(double) * partial_blocks(p->C, p->G) * G * 4);
    ALLOC(p->d_out4, sizeof(double) * G * 4);
    ALLOC(p->d_outer, sizeof(float) * C * G * 8);
    ALLOC(p->d_change, sizeof(unsigned long long) * 2);
#undef ALLOC

    // host -> device (FP64 mesh; FP32 materials and quadrature)
    std::vector<float> f32(std::max<size_t>({C * G, (size_t)3 * p->nang, G}));
    auto up32 = [&](float *dst, const std::vector<double> &src) {
        for (size_t i = 0; i < src.size(); ++i) f32[i] = (float)src[i];
        hipError_t e = hipMemcpyAsync(dst, f32.data(), sizeof(float) * src.size(), hipMemcpyHostToDevice, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;     // f32 is reused by the next upload
    };
    HIPCHK(p, hipMemcpyAsync(d_xyz, p->xyz.data(), sizeof(double) * 3 * p->nvert, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_cv, p->cv.data(), sizeof(int) * 8 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_nbr, nbr.data(), sizeof(int) * 6 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_nbrf, nbrf.data(), sizeof(int) * 6 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipMemcpyAsync(d_perm, perm.data(), sizeof(unsigned) * 6 * C, hipMemcpyHostToDevice, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "sync");
    HIPCHK(p, up32(dsigt, p->sigt), "copy");
    if (p->nmat) {
        // the group matrix's diagonal is the within-group scattering
        std::vector<double> diag(C * G);
        for (size_t K = 0; K < C; ++K)
            for (size_t g = 0; g < G; ++g) diag[K * G + g] = p->sgg[((size_t)p->cmat[K] * G + g) * G + g];
        HIPCHK(p, up32(dsigs, diag), "copy");
    } else {
        HIPCHK(p, up32(dsigs, p->sigs), "copy");
    }
    HIPCHK(p, up32(dq, p->q), "copy");
    HIPCHK(p, up32(dom, p->omega), "copy");
    HIPCHK(p, up32(dw, p->w), "copy");
    if (dpsib) HIPCHK(p, up32(dpsib, p->psib), "copy");
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
    p->maxin = 1;
    for (int o = 0; o < 8; ++o) p->maxin = std::max(p->maxin, nlev[8 + o]);

    // group-to-group scattering: matrix, materials, cross-group source and outer iterates
    float *dqo = nullptr, *dsgg = nullptr;
    int *dcmat = nullptr;
    if (p->nmat) {
        const size_t nm = (size_t)p->nmat * G * G;
        HIPCHK(p, m.alloc((void **)&dsgg, sizeof(float) * nm), "device allocation");
        HIPCHK(p, m.alloc((void **)&dcmat, sizeof(int) * C), "device allocation");
        HIPCHK(p, m.alloc((void **)&dqo, sizeof(float) * C * G * 8), "device allocation");
        std::vector<float> sf(nm);
        for (size_t i = 0; i < nm; ++i) sf[i] = (float)p->sgg[i];
        HIPCHK(p, hipMemcpyAsync(dsgg, sf.data(), sizeof(float) * nm, hipMemcpyHostToDevice, s), "copy");
        HIPCHK(p, hipMemcpyAsync(dcmat, p->cmat.data(), sizeof(int) * C, hipMemcpyHostToDevice, s), "copy");
        HIPCHK(p, launch_fill_f32(dqo, C * G * 8, 0.f, s), "fill");
        HIPCHK(p, hipStreamSynchronize(s), "copy");     // sf is a local buffer
    }

    // per-angle designation: each direction's inflow faces, decided in FP64
    unsigned char *damask = nullptr, *dlagm = nullptr;
    std::fill(p->desig_counts, p->desig_counts + 3, 0ull);
    if (p->designation != SNX_DESIGNATION_OCTANT) {
        double *d_om64;
        unsigned long long *dcounts;
        HIPCHK(p, m.alloc((void **)&damask, 8 * C * A), "device allocation");
        HIPCHK(p, m.alloc((void **)&dlagm, 8 * C), "device allocation");
        HIPCHK(p, m.alloc((void **)&d_om64, sizeof(double) * 3 * p->nang), "device allocation");
        HIPCHK(p, m.alloc((void **)&dcounts, sizeof(unsigned long long) * 3), "device allocation");
        HIPCHK(p, hipMemcpyAsync(d_om64, p->omega.data(), sizeof(double) * 3 * p->nang, hipMemcpyHostToDevice, s),
               "copy");
        HIPCHK(p, hipMemsetAsync(dcounts, 0, sizeof(unsigned long long) * 3, s), "memset");
        HIPCHK(p, launch_angle_masks(p->C, p->A, d_om64, d_nbr, p->d_area, dmask, damask, dlagm, dcounts, p->d_err, s),
               "per-angle designation");
        HIPCHK(p, hipMemcpyAsync(&herr, p->d_err, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipMemcpyAsync(p->desig_counts, dcounts, sizeof(unsigned long long) * 3, hipMemcpyDeviceToHost, s),
               "copy");
        HIPCHK(p, hipStreamSynchronize(s), "per-angle designation");
        if (herr & 8) { drop_device(p); return fail(p, SNX_E_MESH, "a face is tangent to a direction"); }
        // lagged faces read the previous sweep's angular flux: zero before the first
        HIPCHK(p, launch_fill_f32(dpsi, 8 * C * 8 * A * G, 0.f, s), "fill");
    }
    if (p->designation == SNX_DESIGNATION_DIRECTION) {
        // each direction's own order: components, lagged faces and levels on the host
        std::vector<unsigned char> am(8 * C * A);
        HIPCHK(p, hipMemcpy(am.data(), damask, 8 * C * A, hipMemcpyDeviceToHost), "copy");
        DirHost dh;
        std::string derr;
        const int drc = direction_orders(p->C, p->A, nbr, nbrf, am, p->xyz, p->cv, p->omega, dh, derr);
        if (drc) { drop_device(p); return fail(p, drc, derr); }
        const size_t nl = dh.lag.size();
        std::vector<long long> src(std::max<size_t>(1, 4 * nl), 0);
        for (size_t i = 0; i < nl; ++i) {
            const DirHost::Lag &L = dh.lag[i];
            const int N = nbr[(size_t)L.K * 6 + L.f];
            for (int l = 0; l < 4; ++l) {
                const long long vn = (perm[(size_t)L.K * 6 + L.f] >> (8 * l)) & 0xffu;
                src[4 * i + l] = ((((long long)L.o * p->C + N) * 8 + vn) * p->A + L.a) * p->G;
            }
        }
        // work units (task, direction), level by level: every direction of an item
        std::vector<int> units;
        std::vector<long long> unit_off(dh.level_off.size(), 0);
        units.reserve(2 * (size_t)C * p->nang);
        for (size_t l = 0; l + 1 < dh.level_off.size(); ++l) {
            unit_off[l] = (long long)(units.size() / 2);
            for (long long i = dh.level_off[l]; i < dh.level_off[l + 1]; ++i)
                for (unsigned long long d = dh.dirs[i]; d; d &= d - 1) {
                    units.push_back(dh.items[i]);
                    units.push_back(__builtin_ctzll(d));
                }
        }
        unit_off.back() = (long long)(units.size() / 2);
        DirDev &D = p->dir.dev;
        int *dunits; unsigned char *dlagb; int *dlagi; long long *dsrc; float *dlbuf;
        HIPCHK(p, m.alloc((void **)&dunits, sizeof(int) * std::max<size_t>(2, units.size())), "device allocation");
        HIPCHK(p, m.alloc((void **)&dlagb, 8 * C * A), "device allocation");
        HIPCHK(p, m.alloc((void **)&dlagi, sizeof(int) * 8 * C * A), "device allocation");
        HIPCHK(p, m.alloc((void **)&dsrc, sizeof(long long) * src.size()), "device allocation");
        HIPCHK(p, m.alloc((void **)&dlbuf, sizeof(float) * std::max<size_t>(1, 4 * nl * G)), "device allocation");
        HIPCHK(p, hipMemcpy(dunits, units.data(), sizeof(int) * units.size(), hipMemcpyHostToDevice), "copy");
        HIPCHK(p, hipMemcpy(dlagb, dh.lagbits.data(), 8 * C * A, hipMemcpyHostToDevice), "copy");
        HIPCHK(p, hipMemcpy(dlagi, dh.lagidx.data(), sizeof(int) * 8 * C * A, hipMemcpyHostToDevice), "copy");
        HIPCHK(p, hipMemcpy(dsrc, src.data(), sizeof(long long) * src.size(), hipMemcpyHostToDevice), "copy");
        D.units = dunits; D.amask = damask; D.lagbits = dlagb; D.lagidx = dlagi;
        D.lagsrc = dsrc; D.lagbuf = dlbuf; D.nlag = (long long)nl; D.G = p->G; D.A = p->A;
        p->dir.level_off = unit_off;
        p->dir.cyclic = dh.cyclic_directions;
        // the dependency-driven form: each unit's in-degree (non-lagged interior
        // inflow faces of its direction), the seeds, the neighbours' faces
        {
            const size_t NU = (size_t)8 * C * A;
            std::vector<unsigned char> uindeg(NU), nbrf8((size_t)C * 6, 255);
            std::vector<int> qseeds[kUnitQueues], useeds;
            UnitCtl &H = p->dir.uctl_host;
            H = UnitCtl{};
            for (size_t e = 0; e < (size_t)C * 6; ++e)
                if (nbr[e] >= 0) nbrf8[e] = (unsigned char)nbrf[e];
            for (size_t u = 0; u < NU; ++u) {   // u = (o C + K) A + a; queue (o A + a) mod kUnitQueues
                const size_t K = (u / A) % C, oa = (u / ((size_t)A * C)) * A + u % A;
                const int q = (int)(oa % kUnitQueues);
                int interior = 0;
                for (int f = 0; f < 6; ++f) interior |= nbr[K * 6 + f] >= 0 ? 1 << f : 0;
                uindeg[u] = (unsigned char)__builtin_popcount(am[u] & interior & ~dh.lagbits[u]);
                ++H.qtotal[q];
                if (!uindeg[u]) qseeds[q].push_back((int)u);
            }
            for (int q = 0; q < kUnitQueues; ++q) {
                H.qbase[q] = q ? H.qbase[q - 1] + H.qtotal[q - 1] : 0;
                H.seed_off[q] = (long long)useeds.size();
                useeds.insert(useeds.end(), qseeds[q].begin(), qseeds[q].end());
            }
            H.seed_off[kUnitQueues] = (long long)useeds.size();
            unsigned *ducnt; unsigned char *dindeg, *dnbrf; int *dseeds; UnitCtl *dctl; unsigned long long *dq;
            HIPCHK(p, m.alloc((void **)&ducnt, sizeof(unsigned) * NU), "device allocation");
            HIPCHK(p, m.alloc((void **)&dindeg, NU), "device allocation");
            HIPCHK(p, m.alloc((void **)&dnbrf, (size_t)C * 6), "device allocation");
            HIPCHK(p, m.alloc((void **)&dseeds, sizeof(int) * std::max<size_t>(1, useeds.size())), "device allocation");
            HIPCHK(p, m.alloc((void **)&dctl, sizeof(UnitCtl)), "device allocation");
            HIPCHK(p, m.alloc((void **)&dq, sizeof(unsigned long long) * NU), "device allocation");
            HIPCHK(p, hipMemcpy(dindeg, uindeg.data(), NU, hipMemcpyHostToDevice), "copy");
            HIPCHK(p, hipMemcpy(dnbrf, nbrf8.data(), (size_t)C * 6, hipMemcpyHostToDevice), "copy");
            if (!useeds.empty())
                HIPCHK(p, hipMemcpy(dseeds, useeds.data(), sizeof(int) * useeds.size(), hipMemcpyHostToDevice), "copy");
            D.ucnt = ducnt; D.uindeg = dindeg; D.nbrf = dnbrf; D.seeds = dseeds;
            D.uctl = dctl; D.uqueue = dq;
            p->dir.nunits = (long long)NU;
        }
        p->desig_counts[1] = nl;   // lagged triples: only the faces that break cycles
    }

    // anisotropic scattering: harmonics of the directions (FP64 on the host, from
    // the standard library's associated Legendre functions), moments, sources
    float *dsigl = nullptr, *dylm = nullptr, *dmom = nullptr, *drmom = nullptr;
    if (p->L) {
        const int L = p->L, nm = (L + 1) * (L + 1);
        std::vector<float> y((size_t)p->nang * nm);
        for (int n = 0; n < p->nang; ++n) {
            const double *om = &p->omega[3 * n];
            const double mu = std::max(-1.0, std::min(1.0, om[2])), az = std::atan2(om[1], om[0]);
            for (int l = 0; l <= L; ++l)
                for (int mm = 0; mm <= l; ++mm) {
                    const double norm = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * std::tgamma(l - mm + 1.0) /
                                                  std::tgamma(l + mm + 1.0));
                    const double plm = std::assoc_legendre(l, mm, mu);
                    if (mm == 0) {
                        y[(size_t)n * nm + l * l + l] = (float)(norm * plm);
                    } else {
                        y[(size_t)n * nm + l * l + l + mm] = (float)(M_SQRT2 * norm * plm * std::cos(mm * az));
                        y[(size_t)n * nm + l * l + l - mm] = (float)(M_SQRT2 * norm * plm * std::sin(mm * az));
                    }
                }
        }
        std::vector<float> sl(p->sigl.begin(), p->sigl.end());
        HIPCHK(p, m.alloc((void **)&dsigl, sizeof(float) * sl.size()), "device allocation");
        HIPCHK(p, m.alloc((void **)&dylm, sizeof(float) * y.size()), "device allocation");
        HIPCHK(p, m.alloc((void **)&dmom, sizeof(float) * C * G * nm * 8), "device allocation");
        HIPCHK(p, m.alloc((void **)&drmom, sizeof(float) * C * G * nm * 8), "device allocation");
        HIPCHK(p, hipMemcpy(dsigl, sl.data(), sizeof(float) * sl.size(), hipMemcpyHostToDevice), "copy");
        HIPCHK(p, hipMemcpy(dylm, y.data(), sizeof(float) * y.size(), hipMemcpyHostToDevice), "copy");
        HIPCHK(p, launch_fill_f32(dmom, C * G * nm * 8, 0.f, s), "fill");
        HIPCHK(p, launch_fill_f32(drmom, C * G * nm * 8, 0.f, s), "fill");
        // the moments of the first sweep come from a zero angular flux
        HIPCHK(p, launch_fill_f32(dpsi, 8 * C * 8 * A * G, 0.f, s), "fill");
    }

    // reflective planes: boundary faces whose area vector lies along a reflective
    // axis direction (tangential parts within 1e-12 of its length), one slot each
    unsigned char *drmask = nullptr;
    int *drbase = nullptr;
    float *drefl_in = nullptr, *drefl_out = nullptr;
    p->nref = 0;
    if (p->refl) {
        // the mirror image of direction a of octant o must be direction a of octant o ^ (1 << axis)
        for (int n = 0; n < p->nang; ++n)
            for (int ax = 0; ax < 3; ++ax) {
                if (!((p->refl >> (2 * ax)) & 3)) continue;
                const int m = (int)(((n / A) ^ (1 << ax)) * A + n % A);
                double d = 0.0;
                for (int c = 0; c < 3; ++c) d += std::fabs(p->omega[3 * m + c] - (c == ax ? -1.0 : 1.0) * p->omega[3 * n + c]);
                if (!(d < 1e-12)) {
                    drop_device(p);
                    return fail(p, SNX_E_ARG, "the quadrature is not symmetric under the reflective planes");
                }
            }
        std::vector<double> harea(18 * C);
        HIPCHK(p, hipMemcpy(harea.data(), p->d_area, sizeof(double) * 18 * C, hipMemcpyDeviceToHost), "copy");
        std::vector<unsigned char> rm(C, 0);
        std::vector<int> rb(C, 0);
        for (size_t K = 0; K < C; ++K) {
            rb[K] = p->nref;
            for (int f = 0; f < 6; ++f) {
                if (nbr[K * 6 + f] >= 0) continue;
                const double *Af = &harea[(K * 6 + f) * 3];
                const double len = std::sqrt(Af[0] * Af[0] + Af[1] * Af[1] + Af[2] * Af[2]);
                for (int ax = 0; ax < 3; ++ax) {
                    if (std::fabs(Af[(ax + 1) % 3]) > 1e-12 * len || std::fabs(Af[(ax + 2) % 3]) > 1e-12 * len) continue;
                    if ((p->refl >> (2 * ax + (Af[ax] > 0.0))) & 1) {
                        rm[K] |= (unsigned char)(1 << f);
                        ++p->nref;
                    }
                    break;
                }
            }
        }
        if (p->nref) {
            const size_t nr = (size_t)8 * p->nref * 4 * A * G;
            HIPCHK(p, m.alloc((void **)&drmask, C), "device allocation");
            HIPCHK(p, m.alloc((void **)&drbase, sizeof(int) * C), "device allocation");
            HIPCHK(p, m.alloc((void **)&drefl_in, sizeof(float) * nr), "device allocation");
            HIPCHK(p, m.alloc((void **)&drefl_out, sizeof(float) * nr), "device allocation");
            HIPCHK(p, hipMemcpy(drmask, rm.data(), C, hipMemcpyHostToDevice), "copy");
            HIPCHK(p, hipMemcpy(drbase, rb.data(), sizeof(int) * C, hipMemcpyHostToDevice), "copy");
            HIPCHK(p, launch_fill_f32(drefl_in, nr, 0.f, s), "fill");
            HIPCHK(p, launch_fill_f32(drefl_out, nr, 0.f, s), "fill");
        }
    }

    HIPCHK(p, launch_octant_operators(p->C, dS, dF, dmask, dT, s), "octant operators");
    HIPCHK(p, launch_task_records(p->C, d_nbr, d_perm, dmask, dindeg, dlagm, drmask, drbase, drec, s),
           "task records");

    // level-0 tasks of every octant are the seeds of a sweep
    std::vector<int> seeds_host(8 * C);
    HIPCHK(p, hipMemcpy(seeds_host.data(), dseeds, sizeof(int) * 8 * C, hipMemcpyDeviceToHost), "copy");
    p->seeds_by_octant.assign(8, {});
    for (int o = 0; o < 8; ++o)
        for (int i = 0; i < nseed[o]; ++i) p->seeds_by_octant[o].push_back(8 * seeds_host[(size_t)o * C + i] + o);

    hp.C = p->C; hp.G = p->G; hp.A = p->A; hp.nang = p->nang; hp.task_base = 0; hp.epoch = depoch;
    hp.M = dM; hp.S = dS; hp.T = dT; hp.F = dF; hp.nbr = d_nbr; hp.perm = d_perm; hp.inmask = dmask; hp.indeg = dindeg;
    hp.amask = damask;
    hp.qo = dqo; hp.sgg = dsgg; hp.cmat = dcmat;
    hp.refl_in = drefl_in; hp.refl_out = drefl_out; hp.nref = p->nref;
    hp.L = p->L; hp.sigl = dsigl; hp.ylm = dylm; hp.mom = dmom; hp.rmom = drmom;
    hp.sigt = dsigt; hp.sigs = dsigs; hp.q = dq; hp.r = dr; hp.omega = dom; hp.w = dw; hp.psib = dpsib;
    hp.psi = dpsi; hp.slot = dslot; hp.slotc = dslotc; hp.cnt = dcnt; hp.rec = drec;
    hp.xyz = d_xyz; hp.cv = d_cv;
    for (int a = 0; a < 3; ++a) {
        double lo = p->xyz[a], hi = p->xyz[a];
        for (int v = 1; v < p->nvert; ++v) {
            lo = std::min(lo, p->xyz[3 * v + a]);
            hi = std::max(hi, p->xyz[3 * v + a]);
        }
        hp.lo[a] = (float)lo;
        hp.hi[a] = (float)hi;
    }
    HIPCHK(p, launch_fill_f32(dr, C * G * 8, 0.f, s), "fill");
    HIPCHK(p, hipStreamSynchronize(s), "setup");
    snx_status st = build_sched(p->sched, {p}, p->threads, p->wg_per_cu, p->chunk, s);
    // per-direction order: level by level unless a mode was chosen (the unit
    // sweep measured slower at every size tried)
    p->sched.mode = p->designation == SNX_DESIGNATION_DIRECTION && !p->mode_set ? SNX_SWEEP_BSP : p->mode;
    p->sched.depth = p->depth;
    p->sched.phase_stats = p->phase_stats;
    if (st) {
        std::string msg = p->sched.err;
        drop_device(p);
        return fail(p, st, msg);
    }
    if (p->order > 1) {
        // higher-order elements: node maps of the shared faces, element
        // matrices, and the tasks of all octants bucketed by level
        const int P = p->order, N = ho_nodes(p), NF = (P + 1) * (P + 1);
        std::vector<int> hmap;
        st = ho_node_maps(p, P, nbr, nbrf, perm, hmap);
        if (st) {
            std::string msg = p->err;
            drop_device(p);
            return fail(p, st, msg);
        }
        snx_problem::Ho &H = p->ho;
        const size_t NN = (size_t)N * N;
#define HALLOC(ptr, bytes) HIPCHK(p, m.alloc((void **)&(ptr), (bytes)), "device allocation")
        HALLOC(H.M, sizeof(float) * C * NN);
        HALLOC(H.S, sizeof(double) * 3 * C * NN);
        HALLOC(H.F, sizeof(double) * 18 * C * NF * NF);
        HALLOC(H.R, sizeof(float) * C * G * N);
        HALLOC(H.psi, sizeof(float) * p->nang * C * G * N);
        HALLOC(H.phi[0], sizeof(float) * C * G * N);
        HALLOC(H.phi[1], sizeof(float) * C * G * N);
        HALLOC(H.perm, sizeof(int) * 6 * C * NF);
        HALLOC(H.tasks, sizeof(int) * 8 * C);
        HALLOC(H.omega64, sizeof(double) * 3 * p->nang);
#undef HALLOC
        int maxlev = 0;
        for (int l : p->level) maxlev = std::max(maxlev, l);
        H.off.assign(maxlev + 2, 0);
        for (int l : p->level) ++H.off[l + 1];
        for (int l = 0; l <= maxlev; ++l) H.off[l + 1] += H.off[l];
        std::vector<int> tasks(8 * C), fillp(H.off.begin(), H.off.end() - 1);
        for (int o = 0; o < 8; ++o)
            for (size_t K = 0; K < C; ++K) tasks[fillp[p->level[(size_t)o * C + K]]++] = (int)(8 * K + o);
        HIPCHK(p, hipMemcpyAsync(H.perm, hmap.data(), sizeof(int) * hmap.size(), hipMemcpyHostToDevice, s), "copy");
        HIPCHK(p, hipMemcpyAsync(H.tasks, tasks.data(), sizeof(int) * tasks.size(), hipMemcpyHostToDevice, s), "copy");
        HIPCHK(p, hipMemcpyAsync(H.omega64, p->omega.data(), sizeof(double) * 3 * p->nang, hipMemcpyHostToDevice, s),
               "copy");
        HIPCHK(p, hipMemsetAsync(p->d_err, 0, sizeof(int), s), "memset");
        HIPCHK(p, launch_ho_geometry(P, d_xyz, d_cv, d_nbr, d_nbrf, H.perm, p->C, ho_reference(P), H.M, H.S, H.F,
                                     p->d_err, s), "geometry");
        HIPCHK(p, hipMemcpyAsync(&herr, p->d_err, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipStreamSynchronize(s), "geometry");
        if (herr & 1) { drop_device(p); return fail(p, SNX_E_MESH, "non-positive Jacobian at a Gauss point"); }
        HoDev &D = H.dev;
        D.C = p->C; D.G = p->G; D.A = p->A;
        D.M = H.M; D.S = H.S; D.F = H.F; D.perm = H.perm; D.nbr = hp.nbr; D.inmask = hp.inmask;
        D.sigt = hp.sigt; D.omega = hp.omega; D.omega64 = H.omega64; D.psib = hp.psib; D.R = H.R; D.psi = H.psi;
        D.tasks = H.tasks;
    }
    p->ready = true;
    return SNX_OK;
}

#define SCHED_ERR(p, expr)                                   \
    do {                                                     \
        snx_status st_ = (expr);                             \
        if (st_) return fail((p), st_, (p)->sched.err);      \
    } while (0)

}  // extern "C"

namespace {

// One higher-order sweep: the source from phi_in, the levels in order, the
// angle reduction into phi_out.  e0/e1 (optional) bracket the level launches.
snx_status ho_sweep(snx_problem *p, const float *phi_in, float *phi_out, hipStream_t s, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr) {
    snx_problem::Ho &H = p->ho;
    const int N = ho_nodes(p);
    HIPCHK(p, launch_ho_source(H.M, p->hp.q, p->hp.sigs, phi_in, H.R, p->C, p->G, N, s), "source");
    if (e0) HIPCHK(p, hipEventRecord(e0, s), "event");
    for (size_t l = 0; l + 1 < H.off.size(); ++l)
        HIPCHK(p, launch_ho_sweep_level(p->order, H.dev, H.off[l], H.off[l + 1] - H.off[l], s), "level launch");
    if (e1) HIPCHK(p, hipEventRecord(e1, s), "event");
    HIPCHK(p, launch_ho_reduce(H.psi, p->hp.w, p->nang, (long long)p->C * p->G * N, phi_out, s), "reduce");
    return SNX_OK;
}

// Source iteration at order > 1 until the FP64 relative max-norm change of phi
// is <= tol or max_it sweeps.
snx_status ho_solve(snx_problem *p, double tol, int max_it, const float *phi0, float *phi, snx_solve_info *info,
                    hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = (size_t)p->C * p->G * ho_nodes(p);
    float *cur = p->ho.phi[0], *nxt = p->ho.phi[1];
    if (phi0) HIPCHK(p, hipMemcpyAsync(cur, phi0, sizeof(float) * n, hipMemcpyDeviceToDevice, s), "copy");
    else HIPCHK(p, launch_fill_f32(cur, n, 0.f, s), "fill");
    int it = 0;
    double eps = INFINITY;
    while (it < max_it) {
        snx_status st = ho_sweep(p, cur, nxt, s);
        if (st) return st;
        HIPCHK(p, hipMemsetAsync(p->d_change, 0, 2 * sizeof(unsigned long long), s), "memset");
        HIPCHK(p, launch_max_change(nxt, cur, (long long)n, p->d_change, s), "change");
        unsigned long long h[2] = {0, 0};
        HIPCHK(p, hipMemcpyAsync(h, p->d_change, sizeof h, hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipStreamSynchronize(s), "solve");
        double num, den;
        std::memcpy(&num, &h[0], sizeof num);
        std::memcpy(&den, &h[1], sizeof den);
        eps = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
        ++it;
        std::swap(cur, nxt);
        if (eps <= tol) break;
    }
    HIPCHK(p, hipMemcpyAsync(phi, cur, sizeof(float) * n, hipMemcpyDeviceToDevice, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "solve");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const bool conv = eps <= tol;
    if (info) {
        info->iterations = it;
        info->status = conv ? SNX_OK : SNX_E_NOCONV;
        info->residual = eps;
        info->wall_ms = ms;
        info->solves_per_s = ms > 0 ? (double)p->C * p->nang * p->G * it / (ms * 1e-3) : 0.0;
    }
    return conv ? SNX_OK : fail(p, SNX_E_NOCONV, "source iteration ended before the tolerance");
}

}  // namespace

extern "C" {

snx_status snx_set_order(snx_problem *p, int32_t order) {
    if (!p) return SNX_E_ARG;
    if (order < 1 || order > 3) return fail(p, SNX_E_ARG, "order must be 1, 2 or 3");
    p->order = order;
    drop_device(p);
    return SNX_OK;
}

snx_status snx_get_order(snx_problem *p, int32_t *order, int32_t *nodes) {
    if (!p) return SNX_E_ARG;
    if (order) *order = p->order;
    if (nodes) *nodes = ho_nodes(p);
    return SNX_OK;
}

snx_status snx_sweep(snx_problem *p, const float *phi_in, float *phi_out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (!phi_out || phi_in == phi_out) return fail(p, SNX_E_ARG, "phi_out must be non-NULL and distinct from phi_in");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (p->order > 1) return ho_sweep(p, phi_in, phi_out, s);
    if (p->nmat)   // one Jacobi step over groups: the cross-group source from phi_in too
        HIPCHK(p, launch_outer_source(p->sched.d_probs, 0, p->C, p->G, phi_in, s), "outer source");
    HIPCHK(p, launch_source(p->sched.d_probs, 0, p->C, p->G, phi_in, nullptr, s), "source");
    if (p->hp.mom)   // anisotropic: moments of the last sweep's psi and their source dofs
        HIPCHK(p, launch_moments(p->sched.d_probs, 0, p->C, p->G, nullptr, s), "moments");
    SCHED_ERR(p, enqueue_sweep(p->sched, nullptr, s));
    HIPCHK(p, launch_reduce(p->sched.d_probs, 0, p->C, p->G, phi_out, nullptr, false, nullptr, nullptr, s), "reduce");
    return SNX_OK;
}

snx_status snx_solve(snx_problem *p, double tol, int32_t max_it, const float *phi0, float *phi, snx_solve_info *info,
                     void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (!phi || max_it < 1 || !(tol >= 0.0)) return fail(p, SNX_E_ARG, "bad solve arguments");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    if (p->order > 1) return ho_solve(p, tol, max_it, phi0, phi, info, (hipStream_t)stream);
    const float *in[1] = {phi0};
    float *out[1] = {phi};
    snx_status st = sched_solve(p->sched, tol, max_it, in, out, info, (hipStream_t)stream);
    if (st) return fail(p, st, p->sched.err);
    return SNX_OK;
}

snx_status snx_solve_outer(snx_problem *p, int32_t outer, int32_t inner, double tol, const float *phi0, float *phi,
                           snx_solve_info *info, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (p->order > 1) return fail(p, SNX_E_ARG, "snx_solve_outer is not available at order > 1");
    if (!phi || outer < 1 || inner < 1 || !(tol >= 0.0)) return fail(p, SNX_E_ARG, "bad solve arguments");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = (size_t)p->C * p->G * 8;
    // The outer iterates alternate between the caller's phi and a library
    // buffer.  Without a group matrix the cross-group source is zero: inner x
    // outer source iterations with the change measured every `inner`.
    float *bufs[2] = {phi, p->d_outer};
    int cur = 0;
    if (phi0 && phi0 != phi)
        HIPCHK(p, hipMemcpyAsync(bufs[0], phi0, sizeof(float) * n, hipMemcpyDeviceToDevice, s), "copy");
    else if (!phi0)
        HIPCHK(p, launch_fill_f32(bufs[0], n, 0.f, s), "fill");
    unsigned long long *hch = reinterpret_cast<unsigned long long *>(p->pinned);
    OuterScope outer_scope(p->sched, inner);   // replays of exactly the inner iterations, fixed cross-group source
    int k = 0, total = 0;
    double eps = INFINITY;
    while (k < outer) {
        if (p->nmat) HIPCHK(p, launch_outer_source(p->sched.d_probs, 0, p->C, p->G, bufs[cur], s), "outer source");
        const float *in[1] = {bufs[cur]};
        float *out[1] = {bufs[cur ^ 1]};
        snx_status st = sched_solve(p->sched, 0.0, inner, in, out, nullptr, s);
        if (st && st != SNX_E_NOCONV) return fail(p, st, p->sched.err);
        total += inner;
        HIPCHK(p, hipMemsetAsync(p->d_change, 0, sizeof(unsigned long long) * 2, s), "memset");
        HIPCHK(p, launch_max_change(bufs[cur ^ 1], bufs[cur], (long long)n, p->d_change, s), "change");
        HIPCHK(p, hipMemcpyAsync(hch, p->d_change, sizeof(unsigned long long) * 2, hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(p, hipStreamSynchronize(s), "solve");
        double num, den;
        std::memcpy(&num, &hch[0], sizeof(double));
        std::memcpy(&den, &hch[1], sizeof(double));
        eps = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
        cur ^= 1;
        ++k;
        if (tol > 0.0 && eps <= tol) break;
    }
    if (bufs[cur] != phi) HIPCHK(p, hipMemcpyAsync(phi, bufs[cur], sizeof(float) * n, hipMemcpyDeviceToDevice, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "solve");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const bool conv = tol == 0.0 || eps <= tol;
    if (info) {
        info->iterations = total;
        info->status = conv ? SNX_OK : SNX_E_NOCONV;
        info->residual = eps;
        info->wall_ms = ms;
        info->solves_per_s = ms > 0 ? (double)total * p->C * p->nang * p->G / (ms * 1e-3) : 0.0;
    }
    return conv ? SNX_OK : fail(p, SNX_E_NOCONV, "outer iterations ended before the tolerance");
}

snx_status snx_balance(snx_problem *p, const float *phi_in, const float *phi_out, double *out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (p->order > 1) return fail(p, SNX_E_ARG, "snx_balance is not available at order > 1");
    if (!phi_out || !out) return fail(p, SNX_E_ARG, "phi_out and out are required");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (p->nmat)   // the cross-group part of the source is the one phi_in gives
        HIPCHK(p, launch_outer_source(p->sched.d_probs, 0, p->C, p->G, phi_in, s), "outer source");
    HIPCHK(p, launch_balance(p->sched.d_probs, 0, p->C, p->G, phi_in, phi_out, p->d_partial, p->d_out4, s), "balance");
    HIPCHK(p, hipMemcpyAsync(out, p->d_out4, sizeof(double) * 4 * p->G, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "balance");
    return SNX_OK;
}

snx_status snx_integrated_flux(snx_problem *p, const float *phi, double *out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (p->order > 1) return fail(p, SNX_E_ARG, "snx_integrated_flux is not available at order > 1");
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

snx_status snx_integrated_flux_noalloc(snx_problem *p, const float *phi, double *out, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (p->order > 1) return fail(p, SNX_E_ARG, "snx_integrated_flux_noalloc is not available at order > 1");
    if (!phi || !out) return fail(p, SNX_E_ARG, "phi and out are required");
    // the same kernels as snx_integrated_flux: per-block partial[nblk][G][4], then out4[G][4]
    const size_t nblk = partial_blocks(p->C, p->G);
    const size_t need = (nblk + 1) * (size_t)p->G * 4;
    if (need > kScratchDoubles)
        return fail(p, SNX_E_ARG, "ncell * G is too large for the fixed scratch of snx_integrated_flux_noalloc "
                                  "((ceil(ncell * G / 256) + 1) * G * 4 doubles must fit in 2^20)");
    if (!p->scratch) return fail(p, SNX_E_STATE, "no fixed scratch on this device");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    double *partial = p->scratch, *out4 = p->scratch + nblk * (size_t)p->G * 4;
    HIPCHK(p, launch_integrated_flux(p->hp.M, phi, p->C, p->G, partial, out4, s), "integrated flux");
    // columns 0 and 1 of out4 into the pinned staging (G <= 256: at most 4096 bytes), then to out
    HIPCHK(p, hipMemcpy2DAsync(p->pinned, 2 * sizeof(double), out4, 4 * sizeof(double), 2 * sizeof(double),
                               (size_t)p->G, hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(p, hipStreamSynchronize(s), "integrated flux");
    std::memcpy(out, p->pinned, sizeof(double) * 2 * p->G);
    return SNX_OK;
}

snx_status snx_get_levels(snx_problem *p, int32_t *level, int32_t *nlevels) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (level) std::memcpy(level, p->level.data(), sizeof(int) * p->level.size());
    if (nlevels) std::memcpy(nlevels, p->nlev.data(), sizeof(int) * 8);
    return SNX_OK;
}

snx_status snx_designation_stats(snx_problem *p, int64_t *out) {
    if (!p || !out) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    out[0] = p->designation;
    for (int i = 0; i < 3; ++i) out[1 + i] = (int64_t)p->desig_counts[i];
    return SNX_OK;
}

snx_status snx_get_psi(snx_problem *p, int32_t angle, int32_t group, float *out, void *stream) {
    if (!p || !out) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (angle < 0 || angle >= p->nang || group < 0 || group >= p->G)
        return fail(p, SNX_E_ARG, "angle or group out of range");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    if (p->order > 1) {
        // order p keeps psi[nang][C][G][N]: C rows of N floats, G * N apart
        const size_t N = (size_t)(p->order + 1) * (p->order + 1) * (p->order + 1);
        const float *src = p->ho.psi + ((size_t)angle * p->C * p->G + group) * N;
        HIPCHK(p, hipMemcpy2DAsync(out, N * sizeof(float), src, (size_t)p->G * N * sizeof(float), N * sizeof(float),
                                   (size_t)p->C, hipMemcpyDeviceToDevice, (hipStream_t)stream), "copy");
        return SNX_OK;
    }
    HIPCHK(p, launch_gather_psi(p->hp.psi, p->C, p->A, p->G, angle, group, out, (hipStream_t)stream), "gather");
    return SNX_OK;
}

snx_status snx_set_sweep_mode(snx_problem *p, int32_t mode) {
    if (!p) return SNX_E_ARG;
    if (mode != SNX_SWEEP_AMT && mode != SNX_SWEEP_BSP) return fail(p, SNX_E_ARG, "unknown sweep mode");
    p->mode = mode;
    p->mode_set = true;
    if (p->ready) {
        p->sched.mode = mode;
        p->sched.drop_graphs();
    }
    return SNX_OK;
}

snx_status snx_set_sweep_stats(snx_problem *p, int32_t phases) {
    if (!p) return SNX_E_ARG;
    p->phase_stats = phases != 0;
    if (p->ready) {
        p->sched.phase_stats = p->phase_stats;
        p->sched.drop_graphs();
    }
    return SNX_OK;
}

snx_status snx_set_schedule(snx_problem *p, int32_t threads, int32_t wg_per_cu, int32_t chunk) {
    if (!p) return SNX_E_ARG;
    if (threads > 0) {
        if (!sweep_threads_valid(threads)) return fail(p, SNX_E_ARG, "threads must be 64, 128, 192, 256 or 512");
        if (p->have_mat && threads < p->G) return fail(p, SNX_E_ARG, "threads must be at least G");
        p->threads = threads;
    }
    if (wg_per_cu > 0) p->wg_per_cu = wg_per_cu;
    if (chunk > 0) p->chunk = chunk;
    if (!p->ready) return SNX_OK;
    if (p->threads > 0) p->sched.threads = p->threads;
    p->sched.wg_per_cu = p->wg_per_cu;
    p->sched.chunk = p->chunk;
    p->sched.drop_graphs();
    SCHED_ERR(p, configure_grid(p->sched));
    return SNX_OK;
}

snx_status snx_tune(snx_problem *p, const char *cache_path, int32_t *chosen, void *stream) {
    if (!p) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    if (p->order > 1) return fail(p, SNX_E_ARG, "snx_tune is not available at order > 1");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    int t = 0, w = 0;
    double ms = 0;
    SCHED_ERR(p, tune_sched(p->sched, cache_path, (hipStream_t)stream, &t, &w, &ms));
    p->threads = t;
    p->wg_per_cu = w;
    p->mode = p->sched.mode;
    p->depth = p->sched.depth;
    if (chosen) { chosen[0] = t; chosen[1] = w; }
    return SNX_OK;
}

snx_status snx_set_staging_depth(snx_problem *p, int32_t depth) {
    if (!p) return SNX_E_ARG;
    if (depth != 0 && depth != 1) return fail(p, SNX_E_ARG, "staging depth must be 0 or 1");
    p->depth = depth;
    if (p->ready) {
        p->sched.depth = depth;
        p->sched.drop_graphs();
        SCHED_ERR(p, configure_grid(p->sched));   // the two variants' occupancy may differ
    }
    return SNX_OK;
}

snx_status snx_get_staging_depth(snx_problem *p, int32_t *depth) {
    if (!p || !depth) return SNX_E_ARG;
    *depth = p->ready ? p->sched.depth : p->depth;
    return SNX_OK;
}

snx_status snx_get_schedule(snx_problem *p, int32_t *out) {
    if (!p || !out) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    out[0] = p->sched.threads;
    out[1] = p->sched.wg_per_cu;
    out[2] = p->sched.chunk;
    out[3] = p->sched.mode;
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
    for (int i = 0; i < nsweeps && !st && p->order > 1; ++i) st = ho_sweep(p, phi_in, phi_out, s, ev[2 * i], ev[2 * i + 1]);
    for (int i = 0; i < nsweeps && !st && p->order == 1; ++i) {
        hipError_t e = launch_source(p->sched.d_probs, 0, p->C, p->G, phi_in, nullptr, s);
        if (e != hipSuccess) { st = fail(p, SNX_E_DEVICE, "source launch failed"); break; }
        st = enqueue_sweep(p->sched, nullptr, s, ev[2 * i], ev[2 * i + 1]);
        if (st) { st = fail(p, st, p->sched.err); break; }
        e = launch_reduce(p->sched.d_probs, 0, p->C, p->G, phi_out, nullptr, false, nullptr, nullptr, s);
        if (e != hipSuccess) st = fail(p, SNX_E_DEVICE, "reduce launch failed");
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

}  // extern "C"

bool snx::problem_view(const snx_problem *p, DevProblem *out, int *device) {
    if (!p || !p->ready || p->order > 1) return false;
    *out = p->hp;
    *device = p->device;
    return true;
}

extern "C" {

snx_status snx_set_watchdog(snx_problem *p, double seconds) {
    if (!p) return SNX_E_ARG;
    if (!(seconds == seconds) || seconds > 3600.0) return fail(p, SNX_E_ARG, "watchdog outside (0, 3600] s");
    p->watchdog_ticks = (unsigned long long)(p->tick_hz * (seconds > 0.0 ? seconds : kWatchdogSeconds));
    if (p->ready) {
        p->sched.watchdog = p->watchdog_ticks;
        p->sched.drop_graphs();   // the limit is a kernel argument of the captured sweeps
    }
    return SNX_OK;
}

snx_status snx_sweep_stats(snx_problem *p, int64_t *out) {
    if (!p || !out) return SNX_E_ARG;
    if (!p->ready) return fail(p, SNX_E_STATE, "snx_setup has not succeeded");
    HIPCHK(p, hipSetDevice(p->device), "hipSetDevice");
    SCHED_ERR(p, sched_stats(p->sched, out));
    return SNX_OK;
}

// ------------------------------------------------------------------ batches

snx_status snx_batch_create(snx_batch **out, int32_t n, snx_problem *const *probs) {
    if (!out || n < 1 || !probs) { g_create_error = "bad batch arguments"; return SNX_E_ARG; }
    *out = nullptr;
    std::vector<snx_problem *> v(probs, probs + n);
    for (snx_problem *p : v) {
        if (!p || !p->ready) { g_create_error = "every problem of a batch must be set up"; return SNX_E_STATE; }
        if (p->order > 1) { g_create_error = "batches hold first-order problems only"; return SNX_E_ARG; }
        if (p->device != v[0]->device) { g_create_error = "the problems of a batch must share a device"; return SNX_E_ARG; }
    }
    snx_batch *b = new (std::nothrow) snx_batch();
    if (!b) { g_create_error = "out of host memory"; return SNX_E_OOM; }
    b->device = v[0]->device;
    if (hipSetDevice(b->device) != hipSuccess) { delete b; g_create_error = "hipSetDevice failed"; return SNX_E_DEVICE; }
    snx_status st = build_sched(b->sched, v, b->threads, b->wg_per_cu, b->chunk, nullptr);
    if (st) {
        g_create_error = b->sched.err;
        b->sched.release();
        delete b;
        return st;
    }
    *out = b;
    return SNX_OK;
}

void snx_batch_destroy(snx_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    b->sched.release();
    delete b;
}

const char *snx_batch_last_error(const snx_batch *b) { return b ? b->sched.err.c_str() : g_create_error.c_str(); }

snx_status snx_batch_set_sweep_mode(snx_batch *b, int32_t mode) {
    if (!b) return SNX_E_ARG;
    if (mode != SNX_SWEEP_AMT && mode != SNX_SWEEP_BSP) return fail_msg(b->sched.err, SNX_E_ARG, "unknown sweep mode");
    b->mode = mode;
    b->sched.mode = mode;
    b->sched.drop_graphs();
    return SNX_OK;
}

snx_status snx_batch_set_staging_depth(snx_batch *b, int32_t depth) {
    if (!b) return SNX_E_ARG;
    if (depth != 0 && depth != 1) return fail_msg(b->sched.err, SNX_E_ARG, "staging depth must be 0 or 1");
    b->sched.depth = depth;
    b->sched.drop_graphs();
    return configure_grid(b->sched);
}

snx_status snx_batch_set_sweep_stats(snx_batch *b, int32_t phases) {
    if (!b) return SNX_E_ARG;
    b->sched.phase_stats = phases != 0;
    b->sched.drop_graphs();
    return SNX_OK;
}

snx_status snx_batch_set_schedule(snx_batch *b, int32_t threads, int32_t wg_per_cu, int32_t chunk) {
    if (!b) return SNX_E_ARG;
    if (threads > 0) {
        if (!sweep_threads_valid(threads))
            return fail_msg(b->sched.err, SNX_E_ARG, "threads must be 64, 128, 192, 256 or 512");
        if (threads < b->sched.maxG) return fail_msg(b->sched.err, SNX_E_ARG, "threads must be at least the largest G");
        b->sched.threads = threads;
    }
    if (wg_per_cu > 0) b->sched.wg_per_cu = wg_per_cu;
    if (chunk > 0) b->sched.chunk = chunk;
    b->sched.drop_graphs();
    return configure_grid(b->sched);
}

snx_status snx_batch_tune(snx_batch *b, const char *cache_path, int32_t *chosen, void *stream) {
    if (!b) return SNX_E_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return fail_msg(b->sched.err, SNX_E_DEVICE, "hipSetDevice failed");
    int t = 0, w = 0;
    double ms = 0;
    snx_status st = tune_sched(b->sched, cache_path, (hipStream_t)stream, &t, &w, &ms);
    if (st) return st;
    b->mode = b->sched.mode;
    if (chosen) { chosen[0] = t; chosen[1] = w; }
    return SNX_OK;
}

snx_status snx_batch_sweep(snx_batch *b, const float *const *phi_in, float *const *phi_out, void *stream) {
    if (!b) return SNX_E_ARG;
    if (!phi_out) return fail_msg(b->sched.err, SNX_E_ARG, "phi_out is required");
    for (int i = 0; i < b->sched.nprob(); ++i)
        if (!phi_out[i] || (phi_in && phi_in[i] == phi_out[i]))
            return fail_msg(b->sched.err, SNX_E_ARG, "each phi_out must be non-NULL and distinct from its phi_in");
    if (hipSetDevice(b->device) != hipSuccess) return fail_msg(b->sched.err, SNX_E_DEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    snx_status st = sched_sweep(b->sched, phi_in, phi_out, s);
    if (st) return st;
    HIPCHK_E(b->sched.err, hipStreamSynchronize(s), "batch sweep");
    return SNX_OK;
}

snx_status snx_batch_solve(snx_batch *b, double tol, int32_t max_it, const float *const *phi0, float *const *phi,
                           snx_solve_info *infos, void *stream) {
    if (!b) return SNX_E_ARG;
    if (!phi || max_it < 1 || !(tol >= 0.0)) return fail_msg(b->sched.err, SNX_E_ARG, "bad solve arguments");
    for (int i = 0; i < b->sched.nprob(); ++i)
        if (!phi[i]) return fail_msg(b->sched.err, SNX_E_ARG, "every phi must be non-NULL");
    if (hipSetDevice(b->device) != hipSuccess) return fail_msg(b->sched.err, SNX_E_DEVICE, "hipSetDevice failed");
    return sched_solve(b->sched, tol, max_it, phi0, phi, infos, (hipStream_t)stream);
}

snx_status snx_batch_solve_outer(snx_batch *b, int32_t outer, int32_t inner, double tol, const float *const *phi0,
                                 float *const *phi, snx_solve_info *infos, void *stream) {
    if (!b) return SNX_E_ARG;
    Sched &sc = b->sched;
    if (!phi || outer < 1 || inner < 1 || !(tol >= 0.0)) return fail_msg(sc.err, SNX_E_ARG, "bad solve arguments");
    const int n = sc.nprob();
    for (int i = 0; i < n; ++i)
        if (!phi[i]) return fail_msg(sc.err, SNX_E_ARG, "every phi must be non-NULL");
    if (hipSetDevice(b->device) != hipSuccess) return fail_msg(sc.err, SNX_E_DEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    // each problem's outer iterates alternate between the caller's phi and its library buffer
    std::vector<float *> bufs[2];
    for (int i = 0; i < n; ++i) {
        snx_problem *p = sc.probs[i];
        const size_t cnt = (size_t)p->C * p->G * 8;
        bufs[0].push_back(phi[i]);
        bufs[1].push_back(p->d_outer);
        if (phi0 && phi0[i] && phi0[i] != phi[i])
            HIPCHK_E(sc.err, hipMemcpyAsync(phi[i], phi0[i], sizeof(float) * cnt, hipMemcpyDeviceToDevice, s), "copy");
        else if (!phi0 || !phi0[i])
            HIPCHK_E(sc.err, launch_fill_f32(phi[i], cnt, 0.f, s), "fill");
    }
    std::vector<int> retired(n, 0), total(n, 0);
    std::vector<double> eps(n, INFINITY);
    OuterScope outer_scope(sc, inner);          // replays of exactly the inner iterations, fixed cross-group source
    int cur = 0;
    for (int k = 0; k < outer; ++k) {
        for (int i = 0; i < n; ++i)
            if (!retired[i] && sc.hprobs[i].qo)
                HIPCHK_E(sc.err, launch_outer_source(sc.d_probs, i, sc.hprobs[i].C, sc.hprobs[i].G, bufs[cur][i], s),
                         "outer source");
        snx_status st = sched_solve(sc, 0.0, inner, bufs[cur].data(), bufs[cur ^ 1].data(), nullptr, s, &retired);
        if (st && st != SNX_E_NOCONV) return st;
        for (int i = 0; i < n; ++i) {
            if (retired[i]) continue;
            snx_problem *p = sc.probs[i];
            total[i] += inner;
            HIPCHK_E(sc.err, hipMemsetAsync(p->d_change, 0, sizeof(unsigned long long) * 2, s), "memset");
            HIPCHK_E(sc.err, launch_max_change(bufs[cur ^ 1][i], bufs[cur][i], (long long)p->C * p->G * 8, p->d_change,
                                               s), "change");
        }
        std::vector<unsigned long long> bits(2 * (size_t)n, 0ull);
        for (int i = 0; i < n; ++i)
            if (!retired[i])
                HIPCHK_E(sc.err, hipMemcpyAsync(&bits[2 * i], sc.probs[i]->d_change, sizeof(unsigned long long) * 2,
                                                hipMemcpyDeviceToHost, s), "copy");
        HIPCHK_E(sc.err, hipStreamSynchronize(s), "solve");
        cur ^= 1;
        bool all = true;
        for (int i = 0; i < n; ++i) {
            if (retired[i]) continue;
            double num, den;
            std::memcpy(&num, &bits[2 * i], sizeof(double));
            std::memcpy(&den, &bits[2 * i + 1], sizeof(double));
            eps[i] = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
            // a retired problem's later solves pass its iterate through, so both of
            // its buffers end up holding it
            if (tol > 0.0 && eps[i] <= tol) retired[i] = 1;
            all = all && retired[i];
        }
        if (all) break;
    }
    for (int i = 0; i < n; ++i)
        if (bufs[cur][i] != phi[i])
            HIPCHK_E(sc.err, hipMemcpyAsync(phi[i], bufs[cur][i], sizeof(float) * sc.probs[i]->C * sc.probs[i]->G * 8,
                                            hipMemcpyDeviceToDevice, s), "copy");
    HIPCHK_E(sc.err, hipStreamSynchronize(s), "solve");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool conv = true;
    for (int i = 0; i < n; ++i) {
        const bool ok = tol == 0.0 || eps[i] <= tol;
        conv = conv && ok;
        if (infos) {
            const snx_problem *p = sc.probs[i];
            infos[i].iterations = total[i];
            infos[i].status = ok ? SNX_OK : SNX_E_NOCONV;
            infos[i].residual = eps[i];
            infos[i].wall_ms = ms;
            infos[i].solves_per_s = ms > 0 ? (double)total[i] * p->C * p->nang * p->G / (ms * 1e-3) : 0.0;
        }
    }
    return conv ? SNX_OK : fail_msg(sc.err, SNX_E_NOCONV, "outer iterations ended before the tolerance");
}

snx_status snx_batch_profile_sweep(snx_batch *b, int32_t nsweeps, double *ms, void *stream) {
    if (!b || nsweeps < 1 || !ms) return SNX_E_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return fail_msg(b->sched.err, SNX_E_DEVICE, "hipSetDevice failed");
    return time_sweeps(b->sched, nsweeps, (hipStream_t)stream, ms);
}

snx_status snx_batch_stats(snx_batch *b, int64_t *out) {
    if (!b || !out) return SNX_E_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return fail_msg(b->sched.err, SNX_E_DEVICE, "hipSetDevice failed");
    return sched_stats(b->sched, out);
}

}  // extern "C"
