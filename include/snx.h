/*
 * snx.h -- C ABI of the MI355X (gfx950) unstructured S_N transport sweep.
 *
 * The library solves steady, fixed-source, multigroup linear Boltzmann
 * transport (Eq. 1 of "An Asynchronous Many-Task Algorithm for Unstructured
 * S_N Transport on Shared Memory Systems") on unstructured hexahedral meshes,
 * with within-group isotropic scattering by default and, optionally,
 * group-to-group scattering with inner/outer iterations, anisotropic
 * scattering moments, reflective boundary planes and per-direction upwinding,
 * discretised by S_N discrete ordinates grouped in octants (Section 2) and
 * first-order discontinuous Galerkin finite elements (one 8x8 "assemble and
 * solve" per cell, angle and group; Table 1 lists the element arrays).  One
 * source iteration is a sweep over the upwind dependency DAG of every
 * direction (Section 2.1) followed by the angle reduction phi = sum_n w_n
 * psi_n (Eq. 2); the GPU sweep schedules (cell, octant) tasks from a device
 * queue fed by atomic dependency counters, the GPU form of the work-first
 * many-task sweep of Algorithm 1 (Section 3).
 *
 * Conventions shared by every entry point:
 *   - Every call returns snx_status; the library never throws across the ABI.
 *     On failure snx_last_error() describes the cause.
 *   - "host" pointers are read during the call only (the library copies
 *     them); "device" pointers are caller-owned device memory on the
 *     problem's device and must stay valid until the work enqueued on the
 *     given stream has completed.
 *   - stream is a hipStream_t (NULL = the default stream).
 *   - Scalar flux layout (exchange format): phi[ncell][G][8] float32, cell
 *     ids as given to snx_set_mesh, local dof j = vertex j of the cell.
 *   - Local vertex j = a + 2b + 4c of a cell is the reference corner
 *     (2a-1, 2b-1, 2c-1) of [-1,1]^3; face f = 2*axis + side holds the
 *     vertices whose bit `axis` equals side.
 *   - Directions: omega[nang][3], unit vectors grouped by octant
 *     o = 4[Oz<0] + 2[Oy<0] + [Ox<0], the same count in every octant;
 *     weights w[nang] sum to 4 pi; phi = sum_n w_n psi_n.
 *   - A problem object is used by one host thread at a time; distinct
 *     problems are independent.
 */
#ifndef SNX_H
#define SNX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t snx_status;
#define SNX_OK        0
#define SNX_E_ARG    (-1)  /* invalid argument (NULL, size out of range)            */
#define SNX_E_STATE  (-2)  /* call out of order (e.g. sweep before setup)           */
#define SNX_E_MESH   (-3)  /* non-conforming face, detJ <= 0, face on an octant diagonal */
#define SNX_E_CYCLE  (-4)  /* the upwind graph of some octant has a cycle           */
#define SNX_E_DEVICE (-5)  /* HIP runtime error or sweep watchdog expiry            */
#define SNX_E_OOM    (-6)  /* device or host allocation failed                      */
#define SNX_E_NOCONV (-7)  /* max_it reached; info and phi still filled             */

typedef struct snx_problem snx_problem;
typedef struct snx_batch snx_batch;

typedef struct snx_solve_info {
    int32_t iterations;      /* sweeps performed                                   */
    int32_t status;          /* SNX_OK or SNX_E_NOCONV                             */
    double  residual;        /* last ||phi_l+1 - phi_l||_inf / ||phi_l+1||_inf (FP64) */
    double  wall_ms;         /* host wall time of the solve                        */
    double  solves_per_s;    /* cell-angle-group solves per second over the solve  */
} snx_solve_info;

/* Create a problem bound to HIP device `device`: one instance of the
 * fixed-source transport problem of Eq. 1 (mesh, quadrature, cross sections,
 * source and boundary condition, set below) with everything the sweep keeps
 * on the device.  *out receives the handle.  Errors: SNX_E_ARG (no such
 * device), SNX_E_DEVICE, SNX_E_OOM. */
snx_status snx_create(snx_problem **out, int32_t device);
/* Free the problem and every device buffer it owns.  NULL is ignored. */
void snx_destroy(snx_problem *p);
/* Last error message of p (or of the most recent failed snx_create if p is NULL). */
const char *snx_last_error(const snx_problem *p);

/* Mesh of hexahedra: host xyz[nvert][3] (float64), host cell_vert[ncell][8]
 * (int32 vertex ids, local vertex convention above).  Faces are matched by
 * their vertex sets (Table 1: face_nodes, elem_neighbors); unmatched faces are
 * boundary faces.  Invalidates a previous setup.  Errors: SNX_E_ARG. */
snx_status snx_set_mesh(snx_problem *p, int64_t ncell, int64_t nvert,
                        const double *xyz, const int32_t *cell_vert);

/* Angular quadrature (Section 2: S_N directions grouped by octant): host
 * omega[nang][3], host w[nang].  nang must be a positive multiple of 8 with
 * nang/8 <= 64.  Errors: SNX_E_ARG (not grouped by octant, zero component). */
snx_status snx_set_quadrature(snx_problem *p, int32_t nang, const double *omega, const double *w);

/* Product quadrature helper (no problem needed): the npolar positive nodes of
 * the 2*npolar-point Gauss-Legendre rule in mu = Omega_z times nazim equal
 * azimuths (k + 1/2) (pi/2) / nazim per octant, weight w_mu * pi / (2 nazim);
 * octant-major, then polar-major.  Host omega[8*npolar*nazim][3] and
 * w[8*npolar*nazim] are written.  Errors: SNX_E_ARG. */
snx_status snx_quadrature_product(int32_t npolar, int32_t nazim, double *omega, double *w);

/* Per-cell per-group data (Eq. 1 cross sections and fixed source): host
 * sigma_t, sigma_s, q, each [ncell][G] float64; q is the isotropic source
 * density, the angular source being q / (4 pi).  1 <= G <= 256, set after
 * the mesh.  Errors: SNX_E_ARG, SNX_E_STATE. */
snx_status snx_set_materials(snx_problem *p, int32_t ngroup, const double *sigma_t,
                             const double *sigma_s, const double *q);

/* Boundary condition of Eq. 1 on the inflow boundary faces (Omega . n < 0),
 * which the upwind traces of the sweep (Section 2) take there in place of a
 * neighbour's: kind 0 = vacuum (default, psi = 0), kind 1 = isotropic inflow
 * psi = psi_in[g] for every incoming direction (host float64 [G]).  Errors:
 * SNX_E_ARG (another kind, or kind 1 without psi_in or before the materials
 * fix G). */
snx_status snx_set_boundary(snx_problem *p, int32_t kind, const double *psi_in);

/* Anisotropic within-group scattering through flux moments (the moment
 * dimension of the paper's table of arrays: source, scalar_flux_moments and
 * the expansion coefficients ec; after snx_set_materials, before snx_setup;
 * L = 0 restores isotropic scattering).
 * - The law is sum over l = 0..L of (2l+1)/(4 pi) sigma_l P_l(Omega . Omega').
 *   sigma_0 is the within-group sigma_s.  sigma_l is host float64
 *   [ncell][G][L], holding sigma_1..sigma_L.  L <= 3.
 * - Direction n gets sum over l >= 1 of sigma_l sum over m of
 *   Y_lm(Omega_n) phi_lm on top of the isotropic source.  Y are real
 *   orthonormal spherical harmonics; phi_lm = sum_n w_n Y_lm(Omega_n) psi_n are
 *   the moments of the problem's previous sweep (zero after snx_setup).  The
 *   scalar flux comes from phi_in as before, so the exchange layout is unchanged.
 * - Before each sweep one pass over the last angular flux forms the moments
 *   and their source dofs sigma_l M phi_lm ([ncell][G][(L+1)^2][8]); the
 *   sweep adds each direction's harmonic-weighted sum per lane.
 * - Errors: SNX_E_STATE before the materials; SNX_E_ARG for L > 3 or a
 *   non-finite sigma_l. */
snx_status snx_set_anisotropy(snx_problem *p, int32_t L, const double *sigma_l);

/* Reflective boundary planes (UnSNAP's reason not to sweep octants
 * concurrently, §2.1; before snx_setup, a change undoes any earlier setup).
 * planes: bit 2*axis + side (0..5) marks the boundary faces whose area vector
 * points along -axis (side 0) or +axis (side 1) as reflective.  A face counts
 * when its area vector's other components are within 1e-12 of its length.
 * On such a face the inflow of direction n, at each face node, is the outflow
 * of its mirror image (n with that component negated) at the same node.  The
 * octants still run concurrently: that outflow is the one of the problem's
 * previous sweep (zero after snx_setup), and source iteration converges to the
 * reflective solution.  snx_setup returns SNX_E_ARG when the quadrature lacks
 * the mirror images at the same index of the mirrored octant (product sets have
 * them). */
snx_status snx_set_reflective(snx_problem *p, int32_t planes);

/* Group-to-group isotropic scattering (the energy coupling that the paper's
 * outer iterations resolve, §3.6; after snx_set_materials, before snx_setup;
 * nmat = 0 removes it).  cell_mat: host int32 [ncell], the material of each
 * cell (0 <= m < nmat).  sigma_gg: host float64 [nmat][G][G], entry [m][g'][g]
 * the cross section from group g' into group g (finite, >= 0).  Its diagonal
 * replaces the sigma_s of snx_set_materials, and the source of group g becomes
 * Q_g + sum over g' of sigma(g' -> g) phi_g'.  Under a matrix:
 * - snx_sweep takes the whole source from phi_in (one Jacobi step over groups);
 * - snx_solve renews the whole source from every sweep's flux: its iterates
 *   are those of snx_solve_outer with one inner iteration, all of them inside
 *   the solve's graph replays, stopped by snx_solve's own convergence test;
 * - snx_balance counts the cross-group source;
 * - in a batch, snx_batch_sweep and snx_batch_solve do the same per problem.
 * Errors: SNX_E_STATE before the materials, SNX_E_ARG for an index out of
 * range or a negative or non-finite entry. */
snx_status snx_set_group_scattering(snx_problem *p, int32_t nmat, const int32_t *cell_mat, const double *sigma_gg);

/* Element order, used by the next snx_setup (a change undoes any earlier
 * setup): 1 (default), 2 or 3.  The paper's benchmarks run first-, second- and
 * third-order elements (Section 3.6 and its table of run times).  Order p is
 * the Lagrange element of degree p in each reference coordinate on the
 * trilinear hexahedron, with N = (p+1)^3 nodes at the Gauss-Lobatto-Legendre
 * points (local node j = a + (p+1) b + (p+1)^2 c along the reference axes) and
 * integrals by the (p+1)-point Gauss rule per direction; order 1 is the
 * element of the rest of this header.  At order p > 1 every flux array of
 * snx_sweep, snx_solve and snx_profile_sweep holds [ncell][G][N] floats in
 * that node order, the sweep runs level by level over the octant DAGs (one
 * launch per level; snx_set_schedule and snx_set_sweep_mode do not apply),
 * and these are refused with SNX_E_ARG: per-angle
 * designation, reflective planes, anisotropic and group-to-group scattering
 * (at snx_setup), snx_solve_outer, snx_balance, snx_integrated_flux,
 * snx_tune, batches and the learned initial guess.
 * Errors: SNX_E_ARG for an order outside 1..3. */
snx_status snx_set_order(snx_problem *p, int32_t order);
/* The order and the nodes per cell, N = (order+1)^3 (either pointer may be NULL). */
snx_status snx_get_order(snx_problem *p, int32_t *order, int32_t *nodes);

/* Upwind designation, used by the next snx_setup (a change undoes any earlier
 * setup).
 * SNX_DESIGNATION_OCTANT (default): face f of cell K is inflow for every
 *   direction of octant o when s_o . A_f < 0 (s_o the octant's sign vector,
 *   A_f the outward area vector); one acyclic dependency graph per octant.
 * SNX_DESIGNATION_ANGLE: face f of K is inflow for direction n when
 *   Omega_n . A_f < 0, decided in FP64 (the per-direction mesh traversal of
 *   §2.1).  On distorted meshes these graphs can contain cycles.  Tasks still
 *   follow the octant's graph: a face that is inflow for a direction but
 *   downwind in the octant's order reads the neighbour's angular flux from the
 *   problem's previous sweep (zero after snx_setup).  Every cycle is broken
 *   this way, and source iteration converges to the per-direction upwind
 *   solution, independently of which faces lag.
 * SNX_DESIGNATION_DIRECTION: the same inflow faces, and each direction sweeps
 *   the mesh in its own upwind order (the traversal of §2.1).  snx_setup finds
 *   the strongly connected components of every direction's graph (Tarjan's
 *   algorithm, on the host) and lags only faces inside them: a face whose
 *   upwind cell has the larger Omega_n . centroid (vertex mean; the larger cell
 *   id on a tie) reads the neighbour's angular flux of the previous sweep.
 *   Every other inflow face reads this sweep's flux.  The work unit is one
 *   cell, octant and direction (several units per wavefront).  By default, and
 *   under SNX_SWEEP_BSP or with G > 64, one launch per level of the directions'
 *   own levels; under SNX_SWEEP_AMT (set explicitly) with G <= 64 one
 *   persistent launch runs the units as their counters say they are ready (a
 *   counter per unit, device queues of ready units, the watchdog of the octant
 *   sweep).  Both give the same bits (snx_sweep_stats counts units after the
 *   second).  Not
 *   available with reflective planes, anisotropic scattering, in batches or
 *   at order > 1 (SNX_E_ARG).  snx_designation_stats counts the lagged faces.
 * SNX_E_ARG for another kind; snx_setup returns SNX_E_MESH when a face is
 * tangent to a direction. */
#define SNX_DESIGNATION_OCTANT 0
#define SNX_DESIGNATION_ANGLE 1
#define SNX_DESIGNATION_DIRECTION 2
snx_status snx_set_designation(snx_problem *p, int32_t kind);

/* Build everything one mesh needs, on the device: face matching, element
 * matrices (FP64 integration, FP32 storage), per-octant upwind designation
 * (face f of cell K is inflow for octant o when s_o . A_f < 0, A_f the face's
 * outward area vector), DAG levelling and dependency counters.  Synchronous.
 * Errors: SNX_E_STATE (inputs missing), SNX_E_MESH, SNX_E_CYCLE, SNX_E_OOM,
 * SNX_E_DEVICE. */
snx_status snx_setup(snx_problem *p, void *stream);

/* One source iteration: the scattering source from device phi_in
 * (NULL = zero flux), one full sweep of all octants, angles and groups, and
 * the compensated angle reduction into device phi_out (Eq. 2).  phi_in and
 * phi_out may not alias.  Asynchronous on stream.  Errors: SNX_E_STATE,
 * SNX_E_ARG; device faults surface at the next synchronising call. */
snx_status snx_sweep(snx_problem *p, const float *phi_in, float *phi_out, void *stream);

/* Source iteration from device phi0 (NULL = zero start) until the FP64
 * relative max-norm change is <= tol or max_it sweeps; the final iterate is
 * written to device phi.  info (host, nullable) is filled.  Synchronous.
 * Returns SNX_E_NOCONV when max_it is reached first (phi and info filled),
 * SNX_E_DEVICE on a watchdog expiry. */
snx_status snx_solve(snx_problem *p, double tol, int32_t max_it, const float *phi0,
                     float *phi, snx_solve_info *info, void *stream);

/* Inner and outer iterations (the paper's benchmark runs five of each, §3.6).
 * - Each outer iteration computes the cross-group scattering source
 *   sum over g' != g of sigma(g' -> g) phi_g' from its starting flux.
 * - It then runs `inner` source iterations with the within-group scattering,
 *   graph-captured as in snx_solve.
 * - It ends with the FP64 relative max-norm change of the flux over the outer
 *   iteration.
 * The solve stops after `outer` outer iterations, or earlier when tol > 0 and
 * the change is <= tol.  Without a group matrix the cross-group source is zero.
 * phi0: device [ncell][G][8], or NULL for a zero start; it may equal phi.
 * phi: device out.
 * info (nullable) receives the total inner iterations, the last outer change,
 * the wall time and the solve rate.
 * Synchronous on stream.  Returns SNX_E_NOCONV when tol > 0 is not reached;
 * phi then still holds the last iterate. */
snx_status snx_solve_outer(snx_problem *p, int32_t outer, int32_t inner, double tol, const float *phi0, float *phi,
                           snx_solve_info *info, void *stream);

/* Particle balance (FP64) of the most recent sweep, which must have started
 * from device phi_in (NULL = zero) and produced device phi_out.  host out[G][4]
 * = total source, absorption, net leakage, and the largest per-cell relative
 * imbalance |src - abs - leak| / max(|src|, |abs|, |leak|).  Synchronous. */
snx_status snx_balance(snx_problem *p, const float *phi_in, const float *phi_out,
                       double *out, void *stream);

/* Integrated flux of Eq. 3 per group, FP64: host out[G][2] = (sum of phi over
 * cells and dofs, volume integral 1^T M phi).  Synchronous. */
snx_status snx_integrated_flux(snx_problem *p, const float *phi, double *out, void *stream);

/* As snx_integrated_flux, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, with the per-block partial sums in a fixed
 * 8 MiB device array that the library holds on each device from the first
 * snx_create on it until the process ends.  The call allocates nothing.
 * Limit: (ceil(ncell * G / 256) + 1) * G * 4 <= 2^20 (e.g. 32^3 cells with 16
 * groups); larger problems get SNX_E_ARG.  Every call on one device shares
 * that array and leaves its last contents there (each call writes every
 * entry it reads), so calls that overlap on one device, from several threads
 * or streams, race.  Synchronous; host out[G][2] as snx_integrated_flux. */
snx_status snx_integrated_flux_noalloc(snx_problem *p, const float *phi, double *out, void *stream);

/* Level structure from setup: host level[8][ncell] (t-level of each cell per
 * octant) and host nlevels[8]; either may be NULL.  Synchronous. */
snx_status snx_get_levels(snx_problem *p, int32_t *level, int32_t *nlevels);

/* Designation statistics from setup, host out[4]: the designation, the
 * (direction, cell, face) triples whose inflow bit differs from the octant's,
 * the lagged triples (SNX_DESIGNATION_ANGLE: interior faces inflow for the
 * direction and downwind in the octant's order; SNX_DESIGNATION_DIRECTION: the
 * faces lagged to break cycles), and the (cell, octant) tasks with at least
 * one differing direction.  The counts are zero under per-octant designation.
 * Synchronous. */
snx_status snx_designation_stats(snx_problem *p, int64_t *out);

/* The angular flux psi (Eq. 1) of one direction and group from the most recent
 * sweep of this problem (alone or in a batch): device out[ncell][8] (FP32, the
 * caller's cell order; the direction index is the one of snx_set_quadrature);
 * at order p > 1, out[ncell][(p+1)^3] in the node order of snx_set_order.
 * Before any sweep the values are unspecified.  SNX_E_ARG for an angle or
 * group out of range.  Asynchronous on `stream`. */
snx_status snx_get_psi(snx_problem *p, int32_t angle, int32_t group, float *out, void *stream);

/* Sweep schedule knobs: threads per task workgroup (64, 128, 192, 256 or
 * 512, at least G; a (cell, octant) task's (angle, group) solves run 64 per
 * wavefront, in rounds when there are more solves than threads), resident
 * workgroups per CU (capped at the occupancy maximum) and the graph chunk
 * length of snx_solve (iterations captured per host check).  Any argument
 * <= 0 keeps the current value; until threads is set, the narrowest width
 * that holds a whole task in one round (at most 256, at least G) is used. */
snx_status snx_set_schedule(snx_problem *p, int32_t threads, int32_t wg_per_cu, int32_t chunk);

/* Sweep scheme.  SNX_SWEEP_AMT (default): the persistent dependency-driven
 * sweep (one launch, tasks generated by atomic counters, paper §3).
 * SNX_SWEEP_BSP: the bulk-synchronous comparator of the paper (§2.1): one
 * launch per level of the per-octant DAGs (all octants and problems of the
 * schedule together), the launch boundary acting as the barrier.  Both run the
 * same task code, so they give the same bits; the mode applies to snx_sweep,
 * snx_solve and snx_profile_sweep.  snx_sweep_stats reports the last AMT sweep.
 * Under SNX_DESIGNATION_DIRECTION the default is SNX_SWEEP_BSP (see
 * snx_set_designation). */
#define SNX_SWEEP_AMT 0
#define SNX_SWEEP_BSP 1
snx_status snx_set_sweep_mode(snx_problem *p, int32_t mode);

/* LDS staging depth of the first-order sweep (the paper's task data staged
 * ahead of its use, §3.3).  1 (default): a continuation task's upwind traces
 * are requested into LDS together with its cell data (one round trip), and a
 * multi-round task requests the next round's source dofs, sigma_t and traces
 * during the current round's solve.  0: each task requests its traces after
 * its cell data has arrived, and each round its inputs at its start.  The bits
 * are the same; snx_tune picks it.  SNX_E_ARG for another value. */
snx_status snx_set_staging_depth(snx_problem *p, int32_t depth);
snx_status snx_get_staging_depth(snx_problem *p, int32_t *depth);

/* Schedule autotuner: times a few sweeps of every candidate on this problem
 * and keeps the fastest.  The candidates are the dependency-driven sweep at
 * every (threads, workgroups per CU, staging depth) and the bulk-synchronous
 * one at every width, so the tuner also picks the sweep mode (small meshes
 * favour the bulk-synchronous one, whose level launch costs less than a chain
 * of dependent tasks) and the staging depth.  cache_path (nullable) is a text file of JSON lines keyed
 * by device and problem shape: a hit skips the timing, a miss appends the
 * result.  host chosen[2] (nullable) receives (threads, workgroups per CU);
 * snx_get_schedule reports the mode.  Synchronous. */
snx_status snx_tune(snx_problem *p, const char *cache_path, int32_t *chosen, void *stream);

/* The problem's sweep schedule after setup or tuning, host out[4]: threads per
 * task workgroup, the workgroups-per-CU cap (0: occupancy), the graph chunk
 * length of snx_solve, and the sweep mode (SNX_SWEEP_AMT or SNX_SWEEP_BSP). */
snx_status snx_get_schedule(snx_problem *p, int32_t *out);

/* Times the sweep kernel alone: nsweeps source iterations from device phi_in
 * (NULL = zero) into device phi_out, with HIP events recorded on `stream`
 * immediately around each sweep-kernel launch; host *ms receives the mean
 * sweep-kernel duration in milliseconds.  Synchronous. */
snx_status snx_profile_sweep(snx_problem *p, int32_t nsweeps, const float *phi_in, float *phi_out, double *ms,
                             void *stream);

/* Statistics of the most recent sweep, host out[11]: tasks executed, queue
 * polls that found no ready task, abort flag (1 watchdog, 2 queue overflow),
 * resident workgroups of the sweep launch, tasks run by the workgroup that made
 * them ready, threads per workgroup, then shader-clock cycles summed over
 * workgroups spent waiting on the queue, staging cell data, building the
 * per-angle operators, solving, and publishing to downwind cells (zero unless
 * enabled by snx_set_sweep_stats).  After a dependency-driven per-direction
 * sweep (SNX_DESIGNATION_DIRECTION) the entries are: units (cell, octant,
 * direction) solved, polls that found no ready unit, abort flag, rounds of the
 * waves (units solved together), units run by the wave that made them ready,
 * 64, then cycles waiting for a unit, taking more units, solving, publishing,
 * and 0.  A sweep that aborted leaves its dependency counters and queues
 * inconsistent; this call reports the abort once and re-arms them, so the next
 * sweep starts clean (snx_solve does the same itself before it returns
 * SNX_E_DEVICE).  Synchronous. */
snx_status snx_sweep_stats(snx_problem *p, int64_t *out);

/* Watchdog of the dependency-driven sweeps (octant tasks and per-direction
 * units): a workgroup that waits longer than `seconds` of wall-clock time for
 * a ready task sets the abort flag, and every workgroup then leaves the sweep
 * (abort 1 in snx_sweep_stats; snx_solve returns SNX_E_DEVICE).  seconds <= 0
 * restores the default of 20 s; a tiny value makes any wait abort, which tests
 * the abort path.  Applies to the next sweep.  Not a fault handler: kernels
 * always exit normally.  Errors: SNX_E_ARG for NaN or more than 3600 s. */
snx_status snx_set_watchdog(snx_problem *p, double seconds);

/* Turns the per-phase cycle statistics of the dependency-driven sweep on
 * (phases != 0) or off (the default: reading the shader clock at every phase
 * of every task costs about 2 % of sweep time).  Counts of tasks, polls and
 * continuations are always gathered. */
snx_status snx_set_sweep_stats(snx_problem *p, int32_t phases);

/* ------------------------------------------------------------------ batches
 * Many independent problems (uneven sizes, group and angle counts) share one
 * persistent sweep launch per source iteration: their (cell, octant) tasks are
 * interleaved in the same device queues, and snx_batch_solve replays one
 * graph-captured chunk of iterations for all of them, retiring each problem
 * from later sweeps once it has converged.  The problems must have been set up
 * (snx_setup) on one device and must outlive the batch; a batch never changes
 * a problem's data, only its sweep counters and flux buffers. */

/* Create a batch over n set-up problems.  Errors: SNX_E_ARG, SNX_E_STATE,
 * SNX_E_OOM; the message is available from snx_batch_last_error(NULL). */
snx_status snx_batch_create(snx_batch **out, int32_t n, snx_problem *const *probs);
void snx_batch_destroy(snx_batch *b);
const char *snx_batch_last_error(const snx_batch *b);
/* As snx_set_sweep_mode, for every problem of the batch. */
snx_status snx_batch_set_sweep_mode(snx_batch *b, int32_t mode);
/* As snx_set_staging_depth, for the batch's shared sweep (snx_batch_tune also picks it). */
snx_status snx_batch_set_staging_depth(snx_batch *b, int32_t depth);
/* As snx_set_schedule, with threads at least the largest G of the batch. */
snx_status snx_batch_set_schedule(snx_batch *b, int32_t threads, int32_t wg_per_cu, int32_t chunk);
/* As snx_tune, over the whole batch. */
snx_status snx_batch_tune(snx_batch *b, const char *cache_path, int32_t *chosen, void *stream);
/* As snx_solve_outer, for every problem of the batch at once.  The inner
 * iterations of all problems share each graph replay.  Each problem's outer
 * change is measured on its own, and a problem whose change is <= tol (tol > 0)
 * sits out the later outer iterations.  phi0 (nullable, or NULL entries) and
 * phi are arrays of n device pointers.  infos[n] (nullable) is filled per
 * problem.  Synchronous.  Returns SNX_E_NOCONV when any problem misses tol. */
snx_status snx_batch_solve_outer(snx_batch *b, int32_t outer, int32_t inner, double tol, const float *const *phi0,
                                 float *const *phi, snx_solve_info *infos, void *stream);
/* One source iteration of every problem: host arrays of n device pointers
 * phi_in (nullable array, nullable entries = zero flux) and phi_out.
 * Synchronous. */
snx_status snx_batch_sweep(snx_batch *b, const float *const *phi_in, float *const *phi_out, void *stream);
/* Source iteration of every problem to tol or max_it, as snx_solve; host
 * arrays of n device pointers phi0 (nullable array or entries = zero start)
 * and phi; host infos[n] (nullable).  Returns SNX_E_NOCONV when any problem
 * stopped at max_it.  Synchronous. */
snx_status snx_batch_solve(snx_batch *b, double tol, int32_t max_it, const float *const *phi0, float *const *phi,
                           snx_solve_info *infos, void *stream);
/* Mean duration (ms) of the batch's sweep kernel over nsweeps sweeps of every
 * problem, from HIP events on stream (the sources in place are reused).
 * Synchronous. */
snx_status snx_batch_profile_sweep(snx_batch *b, int32_t nsweeps, double *ms, void *stream);
/* As snx_sweep_stats, for the most recent sweep of the batch. */
snx_status snx_batch_stats(snx_batch *b, int64_t *out);
/* As snx_set_sweep_stats, for the batch's sweeps. */
snx_status snx_batch_set_sweep_stats(snx_batch *b, int32_t phases);


/* ---- learned initial guess ------------------------------------------------
 * A face-adjacency message-passing network predicts the converged cell-average
 * scalar flux of every (cell, group) from the problem's data; the prediction,
 * broadcast to the 8 dofs, seeds source iteration (the fixed point of the
 * iteration does not depend on the start, so the result is unchanged; only
 * the number of sweeps is).  The method of the paper starts from zero; the
 * network is an addition of this library.
 *
 * Nodes are (cell, group) pairs v = K*G + g; node v's neighbours are group g
 * of the cells across K's faces.  With hidden width H = 64 and L layers:
 *   h0 = relu(x W_in + b_in), h_l = relu([h_{l-1}, mean_nbr h_{l-1}] W_l + b_l),
 *   z = h_L w_out + b_out,  z predicts y = log(mean of the 8 dofs of phi + 1e-4).
 * Parameters are one FP32 vector in the order W_in [12][H], b_in [H],
 * (W_l [2H][H], b_l [H]) for l = 1..L, w_out [H], b_out [1], row-major.  The
 * layer products run in BF16 (weights and activations) with FP32 accumulation.
 * Node features x [C*G][12] FP32: log sigma_t, c = sigma_s/sigma_t, q,
 * log(q/sigma_a + 1e-2), (boundary faces)/3, log(sigma_t * h),
 * log(max(1 - c, 1e-6)), the cell centroid's distance to the nearest side of
 * the mesh's bounding box and its coordinates u in [0,1]^3 relative to the box,
 * log(max(sigma_a * h, 1e-12)), with h = volume^(1/3).  nbr is [C][6] int32,
 * -1 on the boundary.
 * The loss is the mean over nodes of (z - y)^2; training is AdamW
 * (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay).  Gradients are
 * reduced in a fixed order, so training is deterministic.  Every call is
 * stream-ordered on `stream` unless it says synchronous. */
typedef struct snx_gnn snx_gnn;

/* Network on the calling thread's current HIP device; hidden must be 64,
 * 1 <= layers <= 8.  Weights are drawn normal with variance 2/fan_in from a
 * 64-bit Mersenne twister seeded with `seed`; biases are zero.  Errors:
 * SNX_E_ARG, SNX_E_DEVICE (message from snx_gnn_last_error(NULL)). */
snx_status snx_gnn_create(snx_gnn **out, int32_t hidden, int32_t layers, uint64_t seed);
/* As snx_gnn_create, on HIP device `device`. */
snx_status snx_gnn_create_on(snx_gnn **out, int32_t device, int32_t hidden, int32_t layers, uint64_t seed);
/* Free the network and its device memory.  NULL is ignored. */
void snx_gnn_destroy(snx_gnn *g);
const char *snx_gnn_last_error(const snx_gnn *g);
/* Number of FP32 parameters (33921 for 4 layers). */
snx_status snx_gnn_num_params(const snx_gnn *g, int64_t *n);
/* Copy the parameters to / from a host array of snx_gnn_num_params floats.
 * Setting them also resets the optimiser state.  Synchronous. */
snx_status snx_gnn_get_params(snx_gnn *g, float *host);
snx_status snx_gnn_set_params(snx_gnn *g, const float *host);
/* Parameter file: "SNXGNN1\0", int32 {64, layers, nparams}, then the FP32
 * parameters (little-endian).  Load rejects a file of another shape with
 * SNX_E_ARG.  Synchronous. */
snx_status snx_gnn_save(snx_gnn *g, const char *path);
snx_status snx_gnn_load(snx_gnn *g, const char *path);
/* Node features of a set-up problem into device x [C*G][12], and its face
 * adjacency into device nbr [C][6] (nbr may be NULL).  SNX_E_STATE if p is
 * not set up. */
snx_status snx_gnn_features(snx_problem *p, float *x, int32_t *nbr, void *stream);
/* Regression targets y [ncell*G] = log(mean of the 8 dofs + 1e-4) of a
 * device flux phi [ncell][G][8]. */
snx_status snx_gnn_targets(const float *phi, int64_t ncell, int32_t G, float *y, void *stream);
/* Forward pass on device inputs: z [ncell*G] (device, caller-owned).  The
 * network keeps a workspace sized for the largest graph it has seen. */
snx_status snx_gnn_forward(snx_gnn *g, const float *x, const int32_t *nbr, int64_t ncell, int32_t G, float *z,
                           void *stream);
/* Loss and its gradient: *loss (host, may be NULL) and grad_host (host array
 * of snx_gnn_num_params floats, may be NULL).  Synchronous. */
snx_status snx_gnn_grad(snx_gnn *g, const float *x, const int32_t *nbr, int64_t ncell, int32_t G, const float *y,
                        float *loss, float *grad_host, void *stream);
/* One AdamW step towards a converged flux of a set-up problem: the features
 * of p and the targets of device phi_target [C][G][8] (snx_gnn_features,
 * snx_gnn_targets) into the network's workspace, then the step of
 * snx_gnn_train_step_graph with learning rate lr > 0 and the network's weight
 * decay (1e-4 unless set).  *loss (may be NULL) is the loss before the step.
 * SNX_E_STATE if p is not set up, SNX_E_ARG if it lives on another device.
 * Synchronous (the loss is read back). */
snx_status snx_gnn_train_step(snx_gnn *g, snx_problem *p, const float *phi_target, float lr, float *loss,
                              void *stream);
/* Decoupled weight decay (>= 0) of snx_gnn_train_step. */
snx_status snx_gnn_set_weight_decay(snx_gnn *g, float weight_decay);
/* One AdamW step on a graph given as device arrays (x, nbr, y), as a training
 * loop over many stored instances runs it, with learning rate lr > 0 and
 * decoupled weight decay; *loss (may be NULL) is the loss before the step.
 * Synchronous (the loss is read back). */
snx_status snx_gnn_train_step_graph(snx_gnn *g, const float *x, const int32_t *nbr, int64_t ncell, int32_t G,
                                    const float *y, float lr, float weight_decay, float *loss, void *stream);
/* Predicted starting flux of a set-up problem into device phi0 [C][G][8]:
 * max(exp(z) - 1e-4, 0) on every dof of a cell.  SNX_E_STATE if p is not set
 * up, SNX_E_ARG if it lives on another device. */
snx_status snx_gnn_predict(snx_gnn *g, snx_problem *p, float *phi0, void *stream);

#ifdef __cplusplus
}
#endif
#endif
