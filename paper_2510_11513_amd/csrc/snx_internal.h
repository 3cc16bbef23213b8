// Internal declarations of the gfx950 S_N sweep library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "snx.h"

namespace snx {

constexpr int kMaxAnglesPerOctant = 64;
constexpr int kMaxGroups = 256;
constexpr float kInv4Pi = 0.0795774715459476679f;

constexpr int kMaxQueues = 16;   // task queues of a sweep (one per XCD of the device)
constexpr int kMaxXcc = 32;      // range of hardware XCC ids mapped to queues
constexpr int kReduceItems = 4;  // (cell, group) items per thread of the batched reduction
constexpr int kGnnFeatures = 12; // node features of the learned initial guess (see snx_gnn_features)
// Task record of one (octant, cell), 96 ints (24 int4): words 0..12 the cell's
// descriptor (neighbour ids [6], node permutations [6], inflow mask of the
// octant), word 13 the in-degree of the downwind neighbour across face f in
// bits 3f..3f+2, under per-angle designation in bits 18..23 the faces on
// which some direction of the octant differs from the octant's designation,
// and in bits 24..29 the cell's faces on reflective planes; word 14 the first
// reflective slot of the cell (its reflective faces take consecutive slots in
// face order), 15 zero, then for each face f at 16 + 13 f the descriptor
// of the neighbour across f when f is a downwind face (zero otherwise), 94..95
// zero.
constexpr int kRecWords = 96;
// Revision of the sweep kernel's schedule behaviour: part of the autotuner's
// cache key, raised when a kernel change can move the best schedule.
constexpr int kSweepRevision = 3;

// LDS stage buffer of one sweep task (floats): the cell data M, T of the octant
// and the six face matrices (136 float4s) and the task record (24 int4s); for
// one-round tasks also the cell's source dofs of every group (2 float4s per
// group), rounded up to whole 64-lane blocks of 16-byte LDS-destined loads.
// One-round sweep workgroups hold two (stage_buffers).
__host__ __device__ constexpr int stage_floats(bool one, int maxG) {
    return one ? 256 * ((160 + 2 * maxG + 63) / 64) : 4 * 160;
}
__host__ __device__ constexpr int stage_buffers(bool one) { return one ? 2 : 1; }

// One task queue: octants are assigned to queues (o mod nq), and each queue is
// served by the workgroups of one XCD, so a sweep's hand-offs stay in that
// XCD's L2.  head, tail and done each sit on a 128-byte cache line of their
// own (so do the statistics), so the workgroups that pop (head), push (tail)
// and poll for the queue's end (done) never contend for one line: that took
// the 32^3 / 96 / 16 sweep from 1.70 to 1.61 ms and left the 64^3 one as it
// was.
struct alignas(128) QueueCtl {
    unsigned head;      // next slot to pop
    unsigned pad0[31];
    unsigned tail;      // next slot to fill
    unsigned pad1[31];
    unsigned done;      // tasks of this queue completed, flushed before a workgroup waits
    unsigned pad2[31];
    unsigned long long polls_empty;  // polls that found the popped slot not yet filled
    unsigned long long tasks_done;   // tasks executed (statistics)
    unsigned long long continued;    // tasks run by the workgroup that made them ready (statistics)
    unsigned long long phase[5];     // shader-clock cycles summed over workgroups: waiting on the queue,
                                     // staging, operator build, solve rounds, publishing to downwind
};

// Control block of one sweep launch.
struct SweepCtl {
    unsigned epoch;     // sweep number of this schedule (tags queue entries)
    unsigned abort;     // set by a watchdog expiry (1) or a queue overflow (2); every worker then exits
    int nq;             // queues in use
    int nactive;        // problems swept this time (0: the sweep kernel returns at once)
    int xcc_queue[kMaxXcc];                 // home queue of the workgroups of each XCC id
    long long qbase[kMaxQueues];            // first slot of each queue in the slot array
    long long qtotal[kMaxQueues];           // tasks of each queue in this sweep (active problems only)
    QueueCtl q[kMaxQueues];
};

// Per-problem view used by the device kernels.  All pointers are device memory.
struct DevProblem {
    int C, G, A;                 // cells, groups, angles per octant
    int nang;
    long long task_base;         // first global task id of this problem (task = base + 8*K + o)
    unsigned *epoch;             // sweeps of this problem so far; its counters count to indeg * epoch
    const float *M;              // [C][64]       mass M_ij = int f_i f_j
    const float *S;              // [C][3][64]    stiffness S^a_ij = int f_i df_j/dx_a
    const float *F;              // [C][6][3][16] face matrices F^a_kl on face nodes
    const int *nbr;              // [C][6]        neighbour across face, -1 on the boundary
    const unsigned *perm;        // [C][6]        neighbour's local vertex at my face node k, 8 bits each
    const unsigned char *inmask; // [8][C]        inflow-face bit mask per octant
    const unsigned char *amask;  // [8][C][A]     per-angle designation: inflow faces of each direction; nullptr
                                 //               for per-octant designation
    const float *T;              // [8][C][3][64] T^a = S^a - sum_{f inflow} F^a_f (embedded), per octant
    const int *indeg;            // [8][C]        interior inflow faces per octant
    const float *sigt;           // [C][G]
    const float *sigs;           // [C][G]
    const float *q;              // [C][G]
    float *r;                    // [C][G][8]     M (Q + sigma_s phi) / (4 pi)
    const float *omega;          // [8*A][3]
    const float *w;              // [8*A]
    const float *psib;           // [G] isotropic inflow, or nullptr (vacuum)
    float *psi;                  // [8][C][8][A][G] angular flux handoff
    float *slot;                 // [8][C][G][8]  per-octant compensated partial sums
    float *slotc;                // [8][C][G][8]  their compensation terms
    unsigned *cnt;               // [8][C]        dependency counters (count up across sweeps)
    const int *rec;              // [8][C][kRecWords] task records (see kRecWords)
    float *qo;                   // [C][G][8]     cross-group scattering source of the current outer
                                 //               iteration; nullptr without a group-to-group matrix
    const float *sgg;            // [nmat][G][G]  group-to-group scattering, from g' (row) into g
    float *refl_in;              // [8][nref][4][A][G] reflective planes: outflow of the previous sweep at
                                 //               each reflective face's nodes per octant (read), or nullptr
    float *refl_out;             // the same written by this sweep (copied to refl_in before the next one)
    int nref;                    // reflective boundary faces
    int L;                       // anisotropic scattering degree (0: isotropic)
    const float *sigl;           // [C][G][L]     Legendre moments sigma_1..sigma_L of the scattering law
    const float *ylm;            // [8*A][(L+1)^2] real orthonormal spherical harmonics of the directions
    float *mom;                  // [C][G][(L+1)^2][8] flux moments of the previous sweep (degree >= 1),
                                 //               nullptr when isotropic
    float *rmom;                 // [C][G][(L+1)^2][8] their source dofs sigma_l M phi_lm (degree >= 1)
    const int *cmat;             // [C]           material of each cell (group-to-group matrix)
    const double *xyz;           // [nvert][3]    vertex coordinates (the network's cell positions)
    const int *cv;               // [C][8]        cell vertices
    float lo[3], hi[3];          // bounding box of the mesh
};

// Queues of the dependency-driven per-direction sweep.  A unit (cell, octant,
// direction) belongs to queue (o A + a) mod kUnitQueues, as do its downwind
// units; each queue's slots, units and seeds are fixed at set-up.
constexpr int kUnitQueues = 8;
// Each word on a cache line of its own: the waves that take slots (head),
// push ready units (tail) and poll for the queue's end (done) then never
// contend for one line (measured 9.4 -> 7.4 ms per cfg2 sweep).
struct alignas(128) UnitQ {
    unsigned head;   // next slot to take
    unsigned pad0[31];
    unsigned tail;   // next slot to fill
    unsigned pad1[31];
    unsigned done;   // units of the queue solved, flushed before a wave waits
    unsigned pad2[31];
};
// Statistics of a unit sweep, summed over the waves that start on each XCD.
struct alignas(128) UnitStat {
    unsigned long long units;       // units solved
    unsigned long long rounds;      // rounds of a wave (units solved together)
    unsigned long long carried;     // units solved by the wave that made them ready
    unsigned long long polls;       // polls of a queue slot that found it empty
    unsigned long long phase[4];    // shader-clock cycles: waiting for a unit, taking more units,
                                    // solving (staging, operators, systems), publishing downwind
};
struct UnitCtl {
    unsigned epoch;                          // sweeps so far (tags entries; counters count to in-degree x epoch)
    unsigned pad[31];
    long long qbase[kUnitQueues];            // first slot of each queue
    long long qtotal[kUnitQueues];           // units of each queue
    long long seed_off[kUnitQueues + 1];     // each queue's seeds in DirDev::seeds
    UnitQ q[kUnitQueues];
    UnitStat st[kUnitQueues];
};

// Per-direction sweep order (SNX_DESIGNATION_DIRECTION): the work items of the
// level-synchronous sweep and the faces lagged to break cycles.  Device memory.
struct DirDev {
    const int *units;                 // [nunits][2]   (task 8 K + o, direction a of octant o), bucketed by level
    const unsigned char *amask;       // [8][C][A]     inflow faces of each direction (the problem's amask)
    const unsigned char *lagbits;     // [8][C][A]     interior inflow faces lagged to break cycles
    const int *lagidx;                // [8][C][A]     first lag slot of the direction's lagged faces (face order)
    const long long *lagsrc;          // [nlag * 4]    hand-off index of the upwind node, group 0
    float *lagbuf;                    // [nlag * 4][G] upwind values of the previous sweep
    long long nlag;                   // lagged (direction, cell, face) triples
    int G;                            // groups: the systems of one unit
    int A;                            // directions per octant
    // dependency-driven form (units in natural order (o C + K) A + a)
    unsigned *ucnt;                   // [8][C][A]     dependency counters (count up across sweeps)
    const unsigned char *uindeg;      // [8][C][A]     non-lagged interior inflow faces of the unit's direction
    const unsigned char *nbrf;        // [C][6]        the neighbour's face across face f (255 on the boundary)
    const int *seeds;                 // [nseeds]      units with in-degree 0, by queue
    UnitCtl *uctl;
    unsigned long long *uqueue;       // [8 C A]       ready units by queue, epoch << 32 | unit
};
hipError_t launch_lag_snapshot(const DirDev &D, const DevProblem *probs, int G, const int *stop, hipStream_t s);
hipError_t launch_sweep_dir_level(const DirDev &D, const DevProblem *probs, int threads, long long begin,
                                  long long end, const int *stop, hipStream_t s);
hipError_t launch_dir_slots(const DevProblem *probs, int C, int G, const int *stop, hipStream_t s);
hipError_t launch_unit_sweep(const DirDev &D, const DevProblem *probs, unsigned *abortp, unsigned long long watchdog,
                             const int *stop, bool phase_stats, hipStream_t s);

// Higher-order elements (orders 2 and 3).  Reference tables of the order-p
// element: the Gauss-Lobatto-Legendre nodes and the Gauss points and weights,
// p + 1 of each.
struct HoRef {
    double node[4], gx[4], gw[4];
};
// Device view of a higher-order problem (N = (p+1)^3 nodes, NF = (p+1)^2 per face).
struct HoDev {
    int C, G, A;
    const float *M;              // [C][N][N]          mass
    const double *S;              // [C][3][N][N]       streaming S^a_ij (FP64) = int phi_i d phi_j / d x_a
    const double *F;              // [C][6][3][NF][NF]  face matrices on the face's nodes (FP64)
    const int *perm;             // [C][6][NF]         neighbour's local node at my face node k
    const int *nbr;              // [C][6]
    const unsigned char *inmask; // [8][C]             inflow faces per octant
    const float *sigt;           // [C][G]
    const float *omega;          // [8*A][3]
    const double *omega64;       // [8*A][3]           the directions in FP64 (operator assembly)
    const float *psib;           // [G] or nullptr
    const float *R;              // [C][G][N]          M (Q + sigma_s phi) / (4 pi)
    float *psi;                  // [8*A][C][G][N]
    const int *tasks;            // 8*K + o, ordered by level of the octant DAGs
};

// Iteration record of snx_solve's device-side control.
struct IterCtl {
    unsigned long long num_bits;  // max |phi_new - phi_old| (FP64 bit pattern, non-negative)
    unsigned long long den_bits;  // max |phi_new|
    unsigned blocks_done;
    int iter;                     // completed iterations
    int stop;                     // 1 = converged, 2 = max_it reached, 3 = device error
    int max_it;
    double tol;
    double last_eps;
};

// ------------------------------------------------------------- launchers
hipError_t launch_geometry(const double *xyz, const int *cell_vert, const int *nbr, const int *nbr_face,
                           const unsigned *perm, int C, float *M, float *S, float *F, double *area,
                           int *err_flag, hipStream_t s);
hipError_t launch_dag_one(int C, const int *nbr, const double *area, unsigned char *inmask, int *indeg, int *level,
                          int *hist, int *nlev, int *seeds, int *nseed, int *scratch, int *err, hipStream_t s);
hipError_t launch_sweep_prologue(SweepCtl *ctl, unsigned long long *queue, const DevProblem *probs, int nprob,
                                 const int *seeds, const int *seed_off, const int *stops, hipStream_t s);
hipError_t launch_sweep_kernel(const DevProblem *probs, int nprob, const long long *task_base, SweepCtl *ctl,
                               unsigned long long *queue, int threads, bool one, int grid, int maxA, int maxG, int maxin,
                               unsigned long long watchdog, bool phase_stats, int depth, bool ext, hipStream_t s);
// One level of the bulk-synchronous comparator: tasks bsp_tasks[begin, end).
hipError_t launch_sweep_level(const DevProblem *probs, int nprob, const long long *task_base, SweepCtl *ctl,
                              int threads, bool one, int grid, int maxA, int maxG, int maxin,
                              const long long *bsp_tasks, long long begin, long long end, const int *stops,
                              int depth, bool ext, hipStream_t s);
hipError_t launch_xcc_probe(int *out, int nblocks, hipStream_t s);
hipError_t launch_task_records(int C, const int *nbr, const unsigned *perm, const unsigned char *inmask,
                               const int *indeg, const unsigned char *lagm, const unsigned char *rmask,
                               const int *rbase, int *rec, hipStream_t s);
// Per-angle designation: amask[8][C][A] (bit f: Omega_n . A_f < 0), lagm[8][C]
// (faces where a direction of the octant differs from the octant's mask) and
// counts[3] += differing (direction, cell, face) triples, lagged ones (interior
// faces inflow for the direction and outflow for the octant), cells x octants
// with a difference; err |= 8 for a face tangent to a direction.
hipError_t launch_angle_masks(int C, int A, const double *omega, const int *nbr, const double *area,
                              const unsigned char *inmask, unsigned char *amask, unsigned char *lagm,
                              unsigned long long *counts, int *err, hipStream_t s);
hipError_t launch_octant_operators(int C, const float *S, const float *F, const unsigned char *inmask, float *T,
                                   hipStream_t s);
// Workgroup widths of the sweep kernel: 64, 128, 192, 256 or 512.
bool sweep_threads_valid(int threads);
// `one`: every problem of the launch has (angles per octant) * G <= threads.
size_t sweep_lds_bytes(int threads, int maxA, int maxG, int maxin, bool one);
// ext: the kernel variant with per-angle designation and reflective planes (any
// problem of the schedule uses one of them)
int sweep_occupancy(int threads, bool one, bool ext, int depth, size_t lds);
hipError_t launch_source(const DevProblem *probs, int prob, int C, int G, const float *phi, int *stop_flag,
                         hipStream_t s);
hipError_t launch_reduce(const DevProblem *probs, int prob, int C, int G, float *phi_out, const float *phi_old,
                         bool update_source, IterCtl *ic, int *stop_flag, hipStream_t s);
hipError_t launch_balance(const DevProblem *probs, int prob, int C, int G, const float *phi_in, const float *phi_out,
                          double *partial, double *out, hipStream_t s);
hipError_t launch_integrated_flux(const float *M, const float *phi, int C, int G, double *partial, double *out,
                                  hipStream_t s);
size_t partial_blocks(int C, int G);
hipError_t launch_fill_f32(float *p, size_t n, float v, hipStream_t s);
// P.qo of problem `prob` from phi (NULL = zero): sum over g' != g of sigma(g' -> g) phi_g'.
hipError_t launch_outer_source(const DevProblem *probs, int prob, int C, int G, const float *phi, hipStream_t s,
                               const int *stop_flag = nullptr);
// out[0] |= max |a - b|, out[1] |= max |a| as FP64 bit patterns (out zeroed by the caller).
// Anisotropic scattering: flux moments of degree >= 1 from P.psi (P.mom), then
// their source dofs sigma_l M phi_lm (P.rmom), which the sweep weighs by each
// direction's harmonics.
hipError_t launch_moments(const DevProblem *probs, int prob, int C, int G, const int *stop_flag, hipStream_t s);
hipError_t launch_max_change(const float *a, const float *b, long long n, unsigned long long *out, hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s);
hipError_t launch_copy_f32(float *dst, const float *src, size_t n, const int *stop_flag, hipStream_t s);
hipError_t launch_gather_psi(const float *psi, int C, int A, int G, int angle, int group, float *out, hipStream_t s);
hipError_t launch_iter_init(IterCtl *ic, int *stop_flag, int max_it, double tol, hipStream_t s);
// Batched forms over the problems of a schedule: per-problem stop flags and
// iteration records; blk_base[p] is the first block of problem p (256 (cell,
// group) pairs per block), phi pointer arrays live in device memory.
hipError_t launch_source_batch(const DevProblem *probs, int nprob, const int *blk_base, int nblk,
                               float *const *phi, const int *stops, hipStream_t s);
hipError_t launch_reduce_batch(const DevProblem *probs, int nprob, const int *blk_base, int nblk,
                               float *const *phi_out, float *const *phi_old, int update_source, IterCtl *ic,
                               int *stops, hipStream_t s);
hipError_t launch_iter_init_batch(IterCtl *ic, int *stops, int nprob, int max_it, double tol, hipStream_t s);
hipError_t launch_copy_batch(const DevProblem *probs, int nprob, const int *blk_base, int nblk, float *const *dst,
                             float *const *src, hipStream_t s);

// message-passing network (hidden width 64); bf16 buffers are passed as void*
size_t gnn_bwd_grid(long long Nn);
hipError_t gnn_layer_fwd(const void *hin, void *hout, const int *nbr, const float *inv_deg, int G, long long Nn,
                         const void *Wt, const float *b, hipStream_t s);
hipError_t gnn_layer_bwd(const void *hprev, const void *hcur, const float *dH, const int *nbr, const float *inv_deg,
                         int G, long long Nn, const void *W, float *dHprev, float *dM, float *dWpart, float *dbpart,
                         hipStream_t s);
hipError_t gnn_input_fwd(const float *x, const float *Win, const float *bin, void *h0, long long Nn, hipStream_t s);
hipError_t gnn_input_bwd(const float *x, const void *h0, const float *dH0, long long Nn, float *dWpart, float *dbpart,
                         int grid, hipStream_t s);
hipError_t gnn_head_fwd(const void *h, const float *wout, const float *bout, float *z, long long Nn, hipStream_t s);
hipError_t gnn_head_bwd(const void *h, const float *z, const float *y, const float *wout, long long Nn, float *dH,
                        float *part, int grid, hipStream_t s);
hipError_t gnn_sum_partials(const float *part, int nblk, int n, float *out, float scale, hipStream_t s);
hipError_t gnn_adamw(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, hipStream_t s);
hipError_t gnn_to_bf16(const float *W, void *Wb, void *Wt, hipStream_t s);
hipError_t gnn_features(const DevProblem &P, float *x, int *nbr_out, hipStream_t s);
hipError_t gnn_inv_degree(const int *nbr, int C, float *inv_deg, hipStream_t s);
hipError_t gnn_targets(const float *phi, long long Nn, float *y, hipStream_t s);
hipError_t gnn_expand(const float *z, long long Nn, float *phi, hipStream_t s);

hipError_t launch_ho_geometry(int P, const double *xyz, const int *cv, const int *nbr, const int *nbrf,
                              const int *hoperm, int C, const HoRef &ref, float *M, double *S, double *F, int *err,
                              hipStream_t s);
// Tasks D.tasks[begin, begin + count) of one level, one workgroup per (task, direction).
hipError_t launch_ho_sweep_level(int P, const HoDev &D, int begin, int count, hipStream_t s);
hipError_t launch_ho_source(const float *M, const float *q, const float *sigs, const float *phi, float *R, int C,
                            int G, int N, hipStream_t s);
hipError_t launch_ho_reduce(const float *psi, const float *w, int nang, long long cgn, float *phi, hipStream_t s);

// Device view of a set-up problem (false if it is not set up).
bool problem_view(const snx_problem *p, DevProblem *out, int *device);

// ------------------------------------------------------------- host helpers
int topology(int C, int nvert, const int *cell_vert, std::vector<int> &nbr, std::vector<int> &nbr_face,
             std::vector<unsigned> &perm, std::string &err);
int product_quadrature(int npolar, int nazim, double *omega, double *w);
// Host result of the per-direction ordering (see direction_orders in host.cpp).
struct DirHost {
    std::vector<int> items;                  // task 8 K + o of each work item, bucketed by level
    std::vector<unsigned long long> dirs;    // directions of the item's octant it solves (bit a)
    std::vector<long long> level_off;        // [levels + 1] offsets into items
    std::vector<unsigned char> lagbits;      // [8][C][A] lagged inflow faces
    std::vector<int> lagidx;                 // [8][C][A] first index into lag of the direction's lagged faces
    struct Lag { int o, K, a, f; };
    std::vector<Lag> lag;                    // lagged (octant, cell, direction, face), in that order
    long long cyclic_directions = 0;         // directions whose graph had a cycle
};
int direction_orders(int C, int A, const std::vector<int> &nbr, const std::vector<int> &nbr_face,
                     const std::vector<unsigned char> &amask, const std::vector<double> &xyz,
                     const std::vector<int> &cell_vert, const std::vector<double> &omega, DirHost &out,
                     std::string &err);

}  // namespace snx
