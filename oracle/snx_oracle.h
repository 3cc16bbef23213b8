/*
 * snx_oracle.h -- plain, slow FP64 CPU reference for the unstructured S_N sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link
 * or call this code; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against an obviously
 * correct implementation written straight from the method's definition:
 *
 *   - steady linear Boltzmann transport, Eq. 1, with a fixed isotropic source,
 *     within-group isotropic scattering, vacuum or isotropic-inflow boundaries;
 *   - S_N discrete ordinates grouped by octant (Section 2) with a product
 *     quadrature; scalar flux phi = sum_n w_n psi_n (Eq. 2);
 *   - first-order (trilinear) discontinuous Galerkin on hexahedra, one 8x8
 *     "assemble + solve" per (cell, angle, group) using the element arrays of
 *     Table 1 (mass, stiffness, face normals, face nodes, neighbours);
 *   - the sweep: cells visited in a topological order of the upwind
 *     dependency DAG (Section 2.1), octant by octant, angle by angle;
 *   - upwind faces designated once per octant, or per angle (the mesh
 *     traversal of each direction, Section 2.1), either in the octant's order
 *     with lagged faces where a direction's own dependencies go against it, or
 *     in each direction's own order with cycles broken deterministically;
 *   - reflective planes with the octants in sequence (the reason UnSNAP keeps
 *     them so, Section 2.1) or concurrent;
 *   - source iteration, inner and outer iterations over a group-to-group
 *     scattering matrix (the benchmark of Section 3.6), and the integrated
 *     flux of Eq. 3.
 *
 * All arithmetic is double precision; local systems use LU with partial
 * pivoting.  Every reading of a point the paper leaves open (node ordering,
 * quadrature set, normalisation, upwind designation, convergence norm) is
 * listed in the repository's design notes.
 *
 * Layouts (row-major C arrays, all host memory, owned by the caller unless
 * stated): xyz[nvert][3]; cell_vert[ncell][8] with local vertex j = a+2b+4c at
 * reference corner (2a-1, 2b-1, 2c-1); omega[nang][3]; w[nang];
 * sigma_t, sigma_s, q: [ncell][G]; phi: [ncell][G][8].
 */
#ifndef SNX_ORACLE_H
#define SNX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SNXO_OK = 0,
    SNXO_E_ARG = -1,
    SNXO_E_STATE = -2,
    SNXO_E_MESH = -3,
    SNXO_E_CYCLE = -4,
    SNXO_E_OOM = -6,
    SNXO_E_NOCONV = -7
};

typedef struct snxo_problem snxo_problem;

/* n-point Gauss-Legendre rule on [-1,1], nodes ascending. */
int snxo_gauss_legendre(int n, double *x, double *w);

/* Product quadrature: npolar positive nodes of the 2*npolar-point
 * Gauss-Legendre rule in mu = Omega_z, nazim equal azimuths per octant.
 * Fills omega[8*npolar*nazim][3], w[8*npolar*nazim]; sum w = 4 pi.
 * Octant o = 4[Oz<0] + 2[Oy<0] + [Ox<0]; within an octant polar-major. */
int snxo_quadrature(int npolar, int nazim, double *omega, double *w);

int  snxo_create(snxo_problem **out);
void snxo_destroy(snxo_problem *p);
int  snxo_set_mesh(snxo_problem *p, int ncell, int nvert, const double *xyz, const int32_t *cell_vert);
int  snxo_set_quadrature(snxo_problem *p, int nang, const double *omega, const double *w);
int  snxo_set_materials(snxo_problem *p, int ngroup, const double *sigma_t,
                        const double *sigma_s, const double *q);
/* kind 0 = vacuum, 1 = isotropic inflow psi_b[g] on every inflow boundary face. */
int  snxo_set_boundary(snxo_problem *p, int kind, const double *psi_b);
/* Anisotropic within-group scattering (after snxo_set_materials, before
 * snxo_setup; L = 0 clears): the scattering law
 * sum_{l=0..L} (2l+1)/(4 pi) sigma_l P_l(Omega . Omega') with sigma_0 the
 * sigma_s of snxo_set_materials (or of the group matrix's diagonal) and
 * sigma_l[ncell][G][L] holding sigma_1..sigma_L.  The degree >= 1 flux moments
 * come from the previous sweep's angular flux (psi_prev), the scalar flux from
 * phi_in; L <= 7. */
int  snxo_set_anisotropy(snxo_problem *p, int L, const double *sigma_l);
/* Real orthonormal spherical harmonics of the directions used by the
 * anisotropic source: y[nang][(L+1)^2], index l*l + l + m. */
int  snxo_get_harmonics(snxo_problem *p, double *y);
/* Reflective boundary planes (before snxo_setup; default none): bit
 * 2*axis + side makes the boundary faces whose outward area vector points
 * along -axis (side 0) or +axis (side 1) reflective.  On such a face the inflow
 * of direction n is the outflow of its mirror image (the direction with that
 * component negated, which the quadrature must hold) at the same nodes.  Where
 * that outflow comes from is set by snxo_set_octant_order.
 * snxo_sweep_angle refuses reflective problems. */
int  snxo_set_reflective(snxo_problem *p, int planes);
/* Octant order of a sweep, for reflective planes (default 0; any time).
 * 1: the octants are swept in sequence 0..7, as UnSNAP does so that reflective
 *    faces can use the newest values (Section 2.1 and its footnote): the
 *    mirrored outflow is the current sweep's when the mirror image's octant
 *    came earlier in the sequence, else the previous sweep's (psi_prev).  On
 *    the planes x = 1, y = 1, z = 1 of the unit cube (side 1) every reflected
 *    inflow is then current.
 * 0: the octants are concurrent: every mirrored outflow is the previous
 *    sweep's, as on the GPU.
 * Both iterations converge to the same reflective solution. */
int  snxo_set_octant_order(snxo_problem *p, int sequential);
/* Group-to-group isotropic scattering (after snxo_set_materials; nmat = 0
 * clears it): cell_mat[ncell] material of each cell, sigma_gg[nmat][G][G]
 * with [m][g'][g] the cross section from group g' into group g.  When set, its
 * diagonal replaces sigma_s and the source of group g is
 * Q + sum_g' sigma(g' -> g) phi_g'. */
int  snxo_set_group_scattering(snxo_problem *p, int nmat, const int32_t *cell_mat, const double *sigma_gg);
/* Test hooks (may be NULL to clear).  ang_src[ncell][nang][G][8]: nodal values
 * of an angle-dependent source replacing (Q + sigma_s phi)/(4 pi).
 * bnd_in[ncell][6][nang][G][4]: nodal inflow values on boundary faces. */
int  snxo_set_hooks(snxo_problem *p, const double *ang_src, const double *bnd_in);
/* Upwind designation (before snxo_setup; default 0).
 * kind 0: per octant, face f of cell K is inflow for every angle of octant o
 *         when s_o . A_f < 0 (s_o the octant's sign vector, A_f the outward
 *         area vector).
 * kind 1: per angle, face f of K is inflow for angle n when Omega_n . A_f < 0.
 *         Cells are still visited in the octant's topological order; an
 *         inflow face whose neighbour comes later in that order reads the
 *         neighbour's angular flux of the previous sweep (psi_prev), so every
 *         cycle of a direction's own dependency graph is broken at the faces
 *         that go against the octant's order (the GPU's reading).
 * kind 2: per angle as kind 1, each direction swept in its own topological
 *         order (the mesh traversal of Section 2.1).  Cycles are broken only
 *         inside the strongly connected components of the direction's graph:
 *         there a face whose upwind cell has the larger Omega_n . centroid
 *         (cell id on a tie) is lagged and reads the neighbour's angular flux
 *         of the previous sweep (psi_prev).  See snxo_get_angle_order.
 * All three converge to a solution independent of which faces lag; kinds 1
 * and 2 to the same one. */
int  snxo_set_designation(snxo_problem *p, int kind);
/* Topology, geometry, upwind designation and levelling. */
int  snxo_setup(snxo_problem *p);

/* One source iteration: phi_out = sum_n w_n psi_n where psi solves the sweep
 * with scattering source from phi_in.  psi_prev[nang][ncell][G][8] (NULL =
 * zero) is the previous sweep's angular flux, read on lagged faces of
 * designation 1 only.  Optional outputs (NULL to skip):
 * psi_all[nang][ncell][G][8], leak[ncell][G] (angle-weighted net outflow),
 * leak_ang[nang][ncell][G] (per-angle net outflow). */
int  snxo_sweep(snxo_problem *p, const double *phi_in, const double *psi_prev, double *phi_out,
                double *psi_all, double *leak, double *leak_ang);

/* The sweep of one (angle n, group g) alone (angles and groups of a source
 * iteration are independent given phi_in and psi_prev): psi_out[ncell][8];
 * psi_prev[ncell][8] of the same (n, g), nullable as in snxo_sweep. */
int  snxo_sweep_angle(snxo_problem *p, const double *phi_in, int n, int g, const double *psi_prev,
                      double *psi_out);

/* Source iteration from phi0 (NULL = zero) until the relative max-norm change
 * is <= tol or max_it sweeps.  hist[max_it] (nullable) receives each change.
 * Designation 1 carries the angular flux from sweep to sweep, zero at the start. */
int  snxo_solve(snxo_problem *p, double tol, int max_it, const double *phi0,
                double *phi_out, int *iters, double *eps, double *hist);

/* Inner and outer iterations: each outer iteration fixes the cross-group
 * source sum_{g' != g} sigma(g' -> g) phi_g' from its starting flux and runs
 * `inner` source iterations with the within-group scattering; it ends with the
 * relative max-norm change over the outer iteration.  Runs `outer` outer
 * iterations, or stops earlier when tol > 0 and the change is <= tol (then
 * SNXO_E_NOCONV if it never is).  Counts and the last change are returned. */
int  snxo_solve_outer(snxo_problem *p, int outer, int inner, double tol, const double *phi0, double *phi_out,
                      int *outers_done, int *inners_done, double *eps);

/* Particle balance of one sweep phi_in -> phi_out with its leak[ncell][G]:
 * out[G][4] = source, absorption, leakage, max cell relative imbalance. */
int  snxo_balance(snxo_problem *p, const double *phi_in, const double *phi_out,
                  const double *leak, double *out);

/* Integrated flux (Eq. 3): per group the sum over cells and dofs of phi, and
 * the volume integral 1^T M phi; out[G][2]. */
int  snxo_integrated_flux(snxo_problem *p, const double *phi, double *out);

/* Exports for tests.  M[ncell][64], S[ncell][3][64], F[ncell][6][3][16],
 * area[ncell][6][3], nbr[ncell][6] (-1 boundary), nbr_face[ncell][6],
 * perm[ncell][6][4] (neighbour local vertex at each of my face nodes). */
int  snxo_get_geometry(snxo_problem *p, double *M, double *S, double *F, double *area,
                       int32_t *nbr, int32_t *nbr_face, int32_t *perm);
/* inflow[8][ncell] bit f set when face f is inflow; level[8][ncell];
 * order[8][ncell] the topological order used by the sweep. */
int  snxo_get_dag(snxo_problem *p, int32_t *inflow, int32_t *level, int32_t *order);
/* Designations 1 and 2: ain[nang][ncell], bit f set when face f is inflow for angle n. */
int  snxo_get_angle_inflow(snxo_problem *p, int32_t *ain);
/* Designation 2: order[nang][ncell] each direction's sweep order and
 * lag[nang][ncell] the inflow faces lagged to break its cycles (bit f);
 * either may be NULL. */
int  snxo_get_angle_order(snxo_problem *p, int32_t *order, int32_t *lag);
const char *snxo_last_error(snxo_problem *p);

#ifdef __cplusplus
}
#endif
#endif
