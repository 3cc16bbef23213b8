/*
 * snx_oracle.c -- FP64 CPU reference of the unstructured S_N sweep.
 *
 * TEST INFRASTRUCTURE ONLY (see snx_oracle.h).  Plain loops, double precision,
 * no blocking or fusion: each function follows the definition it cites so that
 * it can be checked against the paper by eye.
 */
#include "snx_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

struct snxo_problem {
    int ncell, nvert, nang, G;
    double *xyz;        /* [nvert][3] */
    int32_t *cv;        /* [ncell][8] */
    double *omega, *w;  /* [nang][3], [nang] */
    double *sigt, *sigs, *q; /* [ncell][G] */
    int bkind;
    double *psib;       /* [G] */
    const double *ang_src, *bnd_in; /* test hooks, not owned */
    int ready;
    /* derived by setup */
    double *M, *S, *F, *area;       /* [C][64], [C][3][64], [C][6][3][16], [C][6][3] */
    int32_t *nbr, *nbrf, *perm;     /* [C][6], [C][6], [C][6][4] */
    int32_t *inflow, *level, *order;/* [8][C] each */
    int designation;                /* 0 per octant, 1 per angle in the octant's order, 2 per angle in
                                       each direction's own order (snxo_set_designation) */
    int octseq;                     /* 1: octants in sequence, reflected inflow from the current sweep
                                       where the mirrored octant came earlier (snxo_set_octant_order) */
    int refl;                       /* reflective planes (snxo_set_reflective): bit 2*axis + side */
    int L;                          /* anisotropic scattering order (snxo_set_anisotropy), 0 = isotropic */
    double *sigl;                   /* [C][G][L] Legendre moments sigma_1..sigma_L of the within-group law */
    double *ylm;                    /* [nang][(L+1)^2] real orthonormal spherical harmonics (setup) */
    int32_t *rdir;                  /* [nang][3] the direction mirrored across each axis (setup) */
    int nmat;                       /* group-to-group scattering (snxo_set_group_scattering), 0 = none */
    int32_t *cmat;                  /* [C] material of each cell */
    double *sgg;                    /* [nmat][G][G] from group g' (row) into group g (column) */
    int32_t *ain;                   /* designations 1, 2: [nang][C] inflow faces of each angle */
    int32_t *aord;                  /* designation 2: [nang][C] each direction's topological order */
    int32_t *alag;                  /* designation 2: [nang][C] inflow faces lagged to break cycles */
    char err[256];
};

/* ---------------------------------------------------------------- helpers */

static int fail(snxo_problem *p, int code, const char *msg) {
    if (p) snprintf(p->err, sizeof p->err, "%s", msg);
    return code;
}

const char *snxo_last_error(snxo_problem *p) { return p ? p->err : "null problem"; }

/* Local vertex j = a + 2b + 4c sits at reference corner (2a-1, 2b-1, 2c-1). */
static double corner(int j, int d) { return ((j >> d) & 1) ? 1.0 : -1.0; }

/* Trilinear basis f_j(xi) = prod_d (1 + corner_jd xi_d)/2 and its reference gradient. */
static void basis(const double xi[3], double f[8], double df[8][3]) {
    for (int j = 0; j < 8; ++j) {
        double h[3], dh[3];
        for (int d = 0; d < 3; ++d) {
            h[d] = 0.5 * (1.0 + corner(j, d) * xi[d]);
            dh[d] = 0.5 * corner(j, d);
        }
        f[j] = h[0] * h[1] * h[2];
        df[j][0] = dh[0] * h[1] * h[2];
        df[j][1] = h[0] * dh[1] * h[2];
        df[j][2] = h[0] * h[1] * dh[2];
    }
}

/* Face f = 2*axis + side holds the local vertices whose bit `axis` equals side,
 * listed in increasing local index. */
static void face_nodes(int f, int fn[4]) {
    int axis = f / 2, side = f % 2, k = 0;
    for (int j = 0; j < 8; ++j)
        if (((j >> axis) & 1) == side) fn[k++] = j;
}

static double det3(const double J[3][3]) {
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* x(xi) Jacobian J[a][b] = d x_a / d xi_b. */
static void jacobian(const double X[8][3], const double df[8][3], double J[3][3]) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int j = 0; j < 8; ++j) s += X[j][a] * df[j][b];
            J[a][b] = s;
        }
}

/* Solve the n x n system A x = b by LU with partial pivoting (A, b overwritten). */
static int lu_solve(int n, double *A, double *b, double *x) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); piv = i; }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
        x[i] = s / A[i * n + i];
    }
    return 0;
}

/* Octant sign vector s_o: bit 0 -> x negative, bit 1 -> y, bit 2 -> z. */
static void octant_signs(int o, double s[3]) {
    for (int d = 0; d < 3; ++d) s[d] = ((o >> d) & 1) ? -1.0 : 1.0;
}

static int octant_of(const double om[3]) {
    return (om[0] < 0.0 ? 1 : 0) + (om[1] < 0.0 ? 2 : 0) + (om[2] < 0.0 ? 4 : 0);
}

/* ------------------------------------------------------------ quadrature */

int snxo_gauss_legendre(int n, double *x, double *w) {
    if (n < 1 || !x || !w) return SNXO_E_ARG;
    /* Newton iteration on P_n from the Chebyshev-like initial guess. */
    for (int i = 0; i < n; ++i) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = z;                       /* ascending order */
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return SNXO_OK;
}

int snxo_quadrature(int npolar, int nazim, double *omega, double *w) {
    if (npolar < 1 || nazim < 1 || !omega || !w) return SNXO_E_ARG;
    int m = 2 * npolar;
    double *gx = malloc(sizeof(double) * m), *gw = malloc(sizeof(double) * m);
    if (!gx || !gw) { free(gx); free(gw); return SNXO_E_OOM; }
    snxo_gauss_legendre(m, gx, gw);
    int per = npolar * nazim;
    for (int o = 0; o < 8; ++o) {
        double s[3];
        octant_signs(o, s);
        for (int k = 0; k < npolar; ++k) {
            double mu = gx[npolar + k];         /* positive half, ascending */
            double wmu = gw[npolar + k];
            double st = sqrt(1.0 - mu * mu);
            for (int j = 0; j < nazim; ++j) {
                double om = (j + 0.5) * (0.5 * PI) / nazim;
                int n = o * per + k * nazim + j;
                omega[3 * n + 0] = s[0] * st * cos(om);
                omega[3 * n + 1] = s[1] * st * sin(om);
                omega[3 * n + 2] = s[2] * mu;
                w[n] = wmu * (0.5 * PI) / nazim;
            }
        }
    }
    free(gx); free(gw);
    return SNXO_OK;
}

/* ------------------------------------------------------------ lifecycle */

static void free_derived(snxo_problem *p) {
    free(p->M); free(p->S); free(p->F); free(p->area);
    free(p->nbr); free(p->nbrf); free(p->perm);
    free(p->inflow); free(p->level); free(p->order); free(p->ain); free(p->rdir); free(p->ylm);
    free(p->aord); free(p->alag);
    p->ylm = NULL;
    p->aord = p->alag = NULL;
    p->M = p->S = p->F = p->area = NULL;
    p->nbr = p->nbrf = p->perm = p->inflow = p->level = p->order = p->ain = p->rdir = NULL;
    p->ready = 0;
}

int snxo_create(snxo_problem **out) {
    if (!out) return SNXO_E_ARG;
    *out = calloc(1, sizeof(snxo_problem));
    return *out ? SNXO_OK : SNXO_E_OOM;
}

void snxo_destroy(snxo_problem *p) {
    if (!p) return;
    free_derived(p);
    free(p->xyz); free(p->cv); free(p->omega); free(p->w);
    free(p->sigt); free(p->sigs); free(p->q); free(p->psib);
    free(p->cmat); free(p->sgg); free(p->sigl);
    free(p);
}

static double *dup_d(const double *src, size_t n) {
    double *d = malloc(sizeof(double) * (n ? n : 1));
    if (d && src) memcpy(d, src, sizeof(double) * n);
    return d;
}

int snxo_set_mesh(snxo_problem *p, int ncell, int nvert, const double *xyz, const int32_t *cv) {
    if (!p || ncell < 1 || nvert < 8 || !xyz || !cv) return fail(p, SNXO_E_ARG, "bad mesh arguments");
    for (long i = 0; i < 8L * ncell; ++i)
        if (cv[i] < 0 || cv[i] >= nvert) return fail(p, SNXO_E_ARG, "vertex index out of range");
    free(p->xyz); free(p->cv);
    p->xyz = dup_d(xyz, 3 * (size_t)nvert);
    p->cv = malloc(sizeof(int32_t) * 8 * (size_t)ncell);
    if (!p->xyz || !p->cv) return fail(p, SNXO_E_OOM, "out of memory");
    memcpy(p->cv, cv, sizeof(int32_t) * 8 * (size_t)ncell);
    p->ncell = ncell; p->nvert = nvert;
    free_derived(p);
    return SNXO_OK;
}

int snxo_set_quadrature(snxo_problem *p, int nang, const double *omega, const double *w) {
    if (!p || nang < 8 || nang % 8 || !omega || !w) return fail(p, SNXO_E_ARG, "bad quadrature");
    int per = nang / 8;
    for (int n = 0; n < nang; ++n) {
        if (omega[3 * n] == 0.0 || omega[3 * n + 1] == 0.0 || omega[3 * n + 2] == 0.0)
            return fail(p, SNXO_E_ARG, "direction on an octant boundary");
        if (octant_of(omega + 3 * n) != n / per)
            return fail(p, SNXO_E_ARG, "directions not grouped by octant");
    }
    free(p->omega); free(p->w);
    p->omega = dup_d(omega, 3 * (size_t)nang);
    p->w = dup_d(w, (size_t)nang);
    if (!p->omega || !p->w) return fail(p, SNXO_E_OOM, "out of memory");
    p->nang = nang;
    return SNXO_OK;
}

int snxo_set_materials(snxo_problem *p, int G, const double *st, const double *ss, const double *q) {
    if (!p || G < 1 || !st || !ss || !q || p->ncell < 1) return fail(p, SNXO_E_ARG, "bad materials");
    size_t n = (size_t)p->ncell * G;
    free(p->sigt); free(p->sigs); free(p->q);
    p->sigt = dup_d(st, n); p->sigs = dup_d(ss, n); p->q = dup_d(q, n);
    if (!p->sigt || !p->sigs || !p->q) return fail(p, SNXO_E_OOM, "out of memory");
    p->G = G;
    return SNXO_OK;
}

int snxo_set_boundary(snxo_problem *p, int kind, const double *psi_b) {
    if (!p || (kind != 0 && kind != 1) || (kind == 1 && (!psi_b || p->G < 1)))
        return fail(p, SNXO_E_ARG, "bad boundary");
    free(p->psib);
    p->psib = NULL;
    p->bkind = kind;
    if (kind == 1) {
        p->psib = dup_d(psi_b, (size_t)p->G);
        if (!p->psib) return fail(p, SNXO_E_OOM, "out of memory");
    }
    return SNXO_OK;
}

int snxo_set_designation(snxo_problem *p, int kind) {
    if (!p || kind < 0 || kind > 2) return fail(p, SNXO_E_ARG, "designation must be 0, 1 or 2");
    p->designation = kind;
    free_derived(p);
    return SNXO_OK;
}

int snxo_set_anisotropy(snxo_problem *p, int L, const double *sigma_l) {
    if (!p || p->G < 1 || p->ncell < 1) return fail(p, SNXO_E_STATE, "set the mesh and materials first");
    if (L < 0 || L > 7 || (L > 0 && !sigma_l)) return fail(p, SNXO_E_ARG, "0 <= L <= 7 and sigma_l required");
    free(p->sigl);
    p->sigl = NULL;
    p->L = 0;
    free_derived(p);
    if (L == 0) return SNXO_OK;
    size_t n = (size_t)p->ncell * p->G * L;
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(sigma_l[i])) return fail(p, SNXO_E_ARG, "sigma_l must be finite");
    p->sigl = dup_d(sigma_l, n);
    if (!p->sigl) return fail(p, SNXO_E_OOM, "out of memory");
    p->L = L;
    return SNXO_OK;
}

int snxo_set_octant_order(snxo_problem *p, int sequential) {
    if (!p || (sequential != 0 && sequential != 1)) return fail(p, SNXO_E_ARG, "octant order must be 0 or 1");
    p->octseq = sequential;
    return SNXO_OK;
}

int snxo_set_reflective(snxo_problem *p, int planes) {
    if (!p || planes < 0 || planes > 63) return fail(p, SNXO_E_ARG, "planes is a 6-bit mask");
    p->refl = planes;
    free_derived(p);
    return SNXO_OK;
}

int snxo_set_group_scattering(snxo_problem *p, int nmat, const int32_t *cell_mat, const double *sigma_gg) {
    if (!p || p->G < 1 || p->ncell < 1) return fail(p, SNXO_E_STATE, "set the mesh and materials first");
    free(p->cmat); free(p->sgg);
    p->cmat = NULL; p->sgg = NULL; p->nmat = 0;
    if (nmat == 0) return SNXO_OK;
    if (nmat < 0 || !cell_mat || !sigma_gg) return fail(p, SNXO_E_ARG, "bad group scattering arguments");
    for (int K = 0; K < p->ncell; ++K)
        if (cell_mat[K] < 0 || cell_mat[K] >= nmat) return fail(p, SNXO_E_ARG, "material index out of range");
    size_t n = (size_t)nmat * p->G * p->G;
    for (size_t i = 0; i < n; ++i)
        if (!(sigma_gg[i] >= 0.0)) return fail(p, SNXO_E_ARG, "scattering cross sections must be >= 0");
    p->cmat = malloc(sizeof(int32_t) * (size_t)p->ncell);
    p->sgg = dup_d(sigma_gg, n);
    if (!p->cmat || !p->sgg) return fail(p, SNXO_E_OOM, "out of memory");
    memcpy(p->cmat, cell_mat, sizeof(int32_t) * (size_t)p->ncell);
    p->nmat = nmat;
    return SNXO_OK;
}

int snxo_set_hooks(snxo_problem *p, const double *ang_src, const double *bnd_in) {
    if (!p) return SNXO_E_ARG;
    p->ang_src = ang_src;
    p->bnd_in = bnd_in;
    return SNXO_OK;
}

/* --------------------------------------------------------------- topology */

typedef struct { int32_t key[4]; int32_t cell, face; } face_rec;

static int cmp_rec(const void *a, const void *b) {
    const face_rec *x = a, *y = b;
    for (int i = 0; i < 4; ++i)
        if (x->key[i] != y->key[i]) return x->key[i] < y->key[i] ? -1 : 1;
    long ix = 6L * x->cell + x->face, iy = 6L * y->cell + y->face;
    return ix < iy ? -1 : (ix > iy);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

/* Faces are matched across cells by their sorted global-vertex 4-tuples. */
static int build_topology(snxo_problem *p) {
    int C = p->ncell;
    face_rec *r = malloc(sizeof(face_rec) * 6 * (size_t)C);
    if (!r) return fail(p, SNXO_E_OOM, "out of memory");
    for (int K = 0; K < C; ++K)
        for (int f = 0; f < 6; ++f) {
            int fn[4];
            face_nodes(f, fn);
            face_rec *e = &r[6 * K + f];
            for (int k = 0; k < 4; ++k) e->key[k] = p->cv[8 * K + fn[k]];
            qsort(e->key, 4, sizeof(int32_t), cmp_i32);
            for (int k = 1; k < 4; ++k)
                if (e->key[k] == e->key[k - 1]) { free(r); return fail(p, SNXO_E_MESH, "degenerate face"); }
            e->cell = K; e->face = f;
        }
    qsort(r, 6 * (size_t)C, sizeof(face_rec), cmp_rec);
    for (long i = 0; i < 6L * C; ++i) { p->nbr[i] = -1; p->nbrf[i] = -1; }
    long i = 0;
    while (i < 6L * C) {
        long j = i + 1;
        while (j < 6L * C && memcmp(r[j].key, r[i].key, sizeof r[i].key) == 0) ++j;
        if (j - i > 2) { free(r); return fail(p, SNXO_E_MESH, "face shared by more than two cells"); }
        if (j - i == 2) {
            int K = r[i].cell, f = r[i].face, N = r[i + 1].cell, g = r[i + 1].face;
            if (K == N) { free(r); return fail(p, SNXO_E_MESH, "cell glued to itself"); }
            p->nbr[6 * K + f] = N; p->nbrf[6 * K + f] = g;
            p->nbr[6 * N + g] = K; p->nbrf[6 * N + g] = f;
        }
        i = j;
    }
    free(r);
    /* Neighbour's local vertex at each of my face nodes. */
    for (int K = 0; K < C; ++K)
        for (int f = 0; f < 6; ++f) {
            int fn[4];
            face_nodes(f, fn);
            int N = p->nbr[6 * K + f];
            for (int k = 0; k < 4; ++k) {
                int32_t v = p->cv[8 * K + fn[k]], found = -1;
                if (N >= 0)
                    for (int jj = 0; jj < 8; ++jj)
                        if (p->cv[8 * N + jj] == v) found = jj;
                p->perm[24 * K + 4 * f + k] = found;
                if (N >= 0 && found < 0) return fail(p, SNXO_E_MESH, "face vertices do not match");
            }
        }
    return SNXO_OK;
}

/* --------------------------------------------------------------- geometry */

/* Mass and stiffness by 2x2x2 Gauss (points +-1/sqrt3, unit weights):
 * M_ij = int f_i f_j dV,  S^a_ij = int f_i d f_j / d x_a dV. */
static int cell_volume_matrices(snxo_problem *p, int K) {
    double X[8][3];
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) X[j][a] = p->xyz[3 * p->cv[8 * K + j] + a];
    double *M = p->M + 64L * K, *S = p->S + 192L * K;
    memset(M, 0, sizeof(double) * 64);
    memset(S, 0, sizeof(double) * 192);
    const double g = 1.0 / sqrt(3.0);
    for (int qp = 0; qp < 8; ++qp) {
        double xi[3] = { corner(qp, 0) * g, corner(qp, 1) * g, corner(qp, 2) * g };
        double f[8], df[8][3], J[3][3];
        basis(xi, f, df);
        jacobian(X, df, J);
        double dJ = det3(J);
        if (!(dJ > 0.0)) return fail(p, SNXO_E_MESH, "non-positive Jacobian at a Gauss point");
        /* physical gradient: solve J^T grad_x = grad_xi, via the inverse J^{-1} */
        double inv[3][3];
        inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / dJ;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / dJ;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / dJ;
        inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / dJ;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / dJ;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / dJ;
        inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / dJ;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / dJ;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / dJ;
        double gx[8][3];
        for (int j = 0; j < 8; ++j)
            for (int a = 0; a < 3; ++a)   /* (J^{-T} grad_xi)_a = sum_b inv[b][a] dxi_b */
                gx[j][a] = inv[0][a] * df[j][0] + inv[1][a] * df[j][1] + inv[2][a] * df[j][2];
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
                M[8 * i + j] += dJ * f[i] * f[j];
                for (int a = 0; a < 3; ++a) S[64 * a + 8 * i + j] += dJ * f[i] * gx[j][a];
            }
    }
    return SNXO_OK;
}

/* Face matrices by 2x2 Gauss on the face parametrised by the two remaining
 * reference coordinates (s, t) in increasing axis order; N = +-(dx/ds x dx/dt)
 * oriented outward.  F^a_kl = sum_q N_a f_k f_l over face nodes k, l;
 * area vector A = sum_q N. */
static void face_matrices(snxo_problem *p, int K, int f, double F[3][16], double A[3]) {
    double X[8][3];
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) X[j][a] = p->xyz[3 * p->cv[8 * K + j] + a];
    int axis = f / 2, side = f % 2, fn[4];
    face_nodes(f, fn);
    int u = (axis == 0) ? 1 : 0, v = (axis == 2) ? 1 : 2;
    /* dx/du x dx/dv points along +xi_axis for axis 0 and 2, along -xi_axis for axis 1 */
    double sgn = (axis == 1 ? -1.0 : 1.0) * (side ? 1.0 : -1.0);
    const double g = 1.0 / sqrt(3.0);
    memset(F, 0, sizeof(double) * 48);
    A[0] = A[1] = A[2] = 0.0;
    for (int qp = 0; qp < 4; ++qp) {
        double xi[3];
        xi[axis] = side ? 1.0 : -1.0;
        xi[u] = corner(qp, 0) * g;
        xi[v] = corner(qp, 1) * g;
        double fb[8], df[8][3], J[3][3];
        basis(xi, fb, df);
        jacobian(X, df, J);
        double tu[3] = { J[0][u], J[1][u], J[2][u] }, tv[3] = { J[0][v], J[1][v], J[2][v] };
        double N[3] = { sgn * (tu[1] * tv[2] - tu[2] * tv[1]),
                        sgn * (tu[2] * tv[0] - tu[0] * tv[2]),
                        sgn * (tu[0] * tv[1] - tu[1] * tv[0]) };
        for (int a = 0; a < 3; ++a) {
            A[a] += N[a];
            for (int k = 0; k < 4; ++k)
                for (int l = 0; l < 4; ++l) F[a][4 * k + l] += N[a] * fb[fn[k]] * fb[fn[l]];
        }
    }
}

static int build_geometry(snxo_problem *p) {
    int C = p->ncell;
    for (int K = 0; K < C; ++K) {
        int rc = cell_volume_matrices(p, K);
        if (rc) return rc;
    }
    /* Each interior face is integrated once, on the side with the smaller
     * (cell, face) index; the other side takes the negated values at the
     * matching nodes so the two sides cancel exactly. */
    for (int K = 0; K < C; ++K)
        for (int f = 0; f < 6; ++f) {
            int N = p->nbr[6 * K + f], g = p->nbrf[6 * K + f];
            if (N >= 0 && 6L * N + g < 6L * K + f) continue;
            double F[3][16], A[3];
            face_matrices(p, K, f, F, A);
            double *FK = p->F + 288L * K + 48 * f, *AK = p->area + 18L * K + 3 * f;
            memcpy(FK, F, sizeof F);
            memcpy(AK, A, sizeof A);
            if (N < 0) continue;
            int fnN[4], pos[4];
            face_nodes(g, fnN);
            for (int k = 0; k < 4; ++k) {
                pos[k] = -1;
                for (int m = 0; m < 4; ++m)
                    if (fnN[m] == p->perm[24 * K + 4 * f + k]) pos[k] = m;
                if (pos[k] < 0) return fail(p, SNXO_E_MESH, "neighbour node not on matched face");
            }
            double *FN = p->F + 288L * N + 48 * g, *AN = p->area + 18L * N + 3 * g;
            for (int a = 0; a < 3; ++a) {
                AN[a] = -A[a];
                for (int k = 0; k < 4; ++k)
                    for (int l = 0; l < 4; ++l) FN[16 * a + 4 * pos[k] + pos[l]] = -F[a][4 * k + l];
            }
        }
    return SNXO_OK;
}

/* ------------------------------------------------- designation and levels */

/* Face f of K is inflow for octant o when s_o . A_f < 0 (one designation per
 * octant); Kahn's algorithm gives a topological order and the t-levels. */
static int build_dag(snxo_problem *p) {
    int C = p->ncell;
    int32_t *indeg = malloc(sizeof(int32_t) * C), *queue = malloc(sizeof(int32_t) * C);
    if (!indeg || !queue) { free(indeg); free(queue); return fail(p, SNXO_E_OOM, "out of memory"); }
    for (int o = 0; o < 8; ++o) {
        double s[3];
        octant_signs(o, s);
        int32_t *in = p->inflow + (long)o * C, *lev = p->level + (long)o * C, *ord = p->order + (long)o * C;
        for (int K = 0; K < C; ++K) {
            int mask = 0;
            indeg[K] = 0;
            for (int f = 0; f < 6; ++f) {
                const double *A = p->area + 18L * K + 3 * f;
                double d = s[0] * A[0] + s[1] * A[1] + s[2] * A[2];
                if (d == 0.0) { free(indeg); free(queue); return fail(p, SNXO_E_MESH, "face tangent to an octant diagonal"); }
                if (d < 0.0) {
                    mask |= 1 << f;
                    if (p->nbr[6 * K + f] >= 0) indeg[K]++;
                }
            }
            in[K] = mask;
            lev[K] = 0;
        }
        int head = 0, tail = 0;
        for (int K = 0; K < C; ++K)
            if (indeg[K] == 0) queue[tail++] = K;
        while (head < tail) {
            int K = queue[head++];
            ord[head - 1] = K;
            for (int f = 0; f < 6; ++f) {
                int N = p->nbr[6 * K + f];
                if (N < 0 || (in[K] >> f) & 1) continue;
                if (lev[N] < lev[K] + 1) lev[N] = lev[K] + 1;
                if (--indeg[N] == 0) queue[tail++] = N;
            }
        }
        if (tail != C) { free(indeg); free(queue); return fail(p, SNXO_E_CYCLE, "upwind graph has a cycle"); }
    }
    free(indeg); free(queue);
    return SNXO_OK;
}

/* Designation 1: face f of K is inflow for angle n when Omega_n . A_f < 0 (the
 * mesh traversal of each direction, Section 2.1).  These graphs may have
 * cycles; the sweep keeps the octant's order and lags the faces that go
 * against it, so no order is derived from them here. */
static int build_angle_inflow(snxo_problem *p) {
    int C = p->ncell;
    for (int n = 0; n < p->nang; ++n) {
        const double *om = p->omega + 3 * n;
        for (int K = 0; K < C; ++K) {
            int mask = 0;
            for (int f = 0; f < 6; ++f) {
                const double *A = p->area + 18L * K + 3 * f;
                double d = om[0] * A[0] + om[1] * A[1] + om[2] * A[2];
                if (d == 0.0) return fail(p, SNXO_E_MESH, "face tangent to a direction");
                if (d < 0.0) mask |= 1 << f;
            }
            p->ain[(long)n * C + K] = mask;
        }
    }
    return SNXO_OK;
}

/* Designation 2: each direction sweeps the mesh in its own upwind order
 * (Section 2.1).  Cell K depends on its neighbour N across every face f with
 * Omega_n . A_f^K < 0.  On distorted meshes this graph can have cycles; the
 * paper does not say how to treat them.  Here they are broken as follows.
 *   1. The strongly connected components of the direction's graph are found
 *      (Tarjan's algorithm).  An edge between two components never lies on a
 *      cycle and is kept.
 *   2. Inside a component, cells are ranked by the upwind distance
 *      Omega_n . c_K of their vertex centroid c_K (cell id on a tie).  An edge
 *      N -> K from a cell ranked after K is lagged: K reads N's angular flux of
 *      the previous sweep on that face.  The kept edges inside a component all
 *      go up in rank, so the rest of the graph is acyclic.
 *   3. Kahn's algorithm over the kept edges gives the direction's order.
 * The rank uses the geometry only, so a renumbering of the cells changes
 * neither the lagged faces nor the result. */
static double upwind_key(const snxo_problem *p, int K, const double *om) {
    double c[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) c[a] += p->xyz[3 * p->cv[8 * K + j] + a] / 8.0;
    return om[0] * c[0] + om[1] * c[1] + om[2] * c[2];
}

static int ranked_after(const double *key, int N, int K) {
    return key[N] > key[K] || (key[N] == key[K] && N > K);
}

static int build_angle_order(snxo_problem *p) {
    int C = p->ncell;
    int32_t *idx = malloc(sizeof(int32_t) * C), *low = malloc(sizeof(int32_t) * C);
    int32_t *comp = malloc(sizeof(int32_t) * C), *stk = malloc(sizeof(int32_t) * C);
    int32_t *cs_v = malloc(sizeof(int32_t) * C), *cs_f = malloc(sizeof(int32_t) * C);
    int32_t *indeg = malloc(sizeof(int32_t) * C);
    char *onstk = malloc((size_t)C);
    double *key = malloc(sizeof(double) * C);
    int rc = SNXO_OK;
    if (!idx || !low || !comp || !stk || !cs_v || !cs_f || !indeg || !onstk || !key) {
        rc = fail(p, SNXO_E_OOM, "out of memory");
        goto done;
    }
    for (int n = 0; n < p->nang; ++n) {
        const int32_t *in = p->ain + (long)n * C;
        int32_t *lag = p->alag + (long)n * C, *ord = p->aord + (long)n * C;
        for (int K = 0; K < C; ++K) {
            idx[K] = -1;
            onstk[K] = 0;
            key[K] = upwind_key(p, K, p->omega + 3 * n);
        }
        /* 1. Tarjan's strongly connected components, iteratively.  The
         * successors of v are its neighbours across its outflow faces. */
        int counter = 0, sp = 0, ncomp = 0;
        for (int r = 0; r < C; ++r) {
            if (idx[r] >= 0) continue;
            int cp = 0;
            cs_v[cp] = r; cs_f[cp] = 0; ++cp;
            idx[r] = low[r] = counter++;
            stk[sp++] = r; onstk[r] = 1;
            while (cp > 0) {
                int v = cs_v[cp - 1];
                if (cs_f[cp - 1] < 6) {
                    int f = cs_f[cp - 1]++;
                    int w = p->nbr[6 * v + f];
                    if (w < 0 || ((in[v] >> f) & 1)) continue;
                    if (idx[w] < 0) {
                        idx[w] = low[w] = counter++;
                        stk[sp++] = w; onstk[w] = 1;
                        cs_v[cp] = w; cs_f[cp] = 0; ++cp;
                    } else if (onstk[w] && idx[w] < low[v]) {
                        low[v] = idx[w];
                    }
                } else {
                    --cp;
                    if (low[v] == idx[v]) {
                        int w;
                        do { w = stk[--sp]; onstk[w] = 0; comp[w] = ncomp; } while (w != v);
                        ++ncomp;
                    }
                    if (cp > 0 && low[v] < low[cs_v[cp - 1]]) low[cs_v[cp - 1]] = low[v];
                }
            }
        }
        /* 2. lag the edges inside a component that go down in rank */
        for (int K = 0; K < C; ++K) {
            int m = 0;
            indeg[K] = 0;
            for (int f = 0; f < 6; ++f) {
                int N = p->nbr[6 * K + f];
                if (N < 0 || !((in[K] >> f) & 1)) continue;
                if (comp[N] == comp[K] && ranked_after(key, N, K)) m |= 1 << f;
                else indeg[K]++;
            }
            lag[K] = m;
        }
        /* 3. Kahn's algorithm over the kept edges, first-in first-out from the
         * cells in id order */
        int head = 0, tail = 0;
        for (int K = 0; K < C; ++K)
            if (indeg[K] == 0) ord[tail++] = K;
        while (head < tail) {
            int v = ord[head++];
            for (int f = 0; f < 6; ++f) {
                int w = p->nbr[6 * v + f];
                if (w < 0 || ((in[v] >> f) & 1)) continue;
                int g = p->nbrf[6 * v + f];
                if ((lag[w] >> g) & 1) continue;
                if (--indeg[w] == 0) ord[tail++] = w;
            }
        }
        if (tail != C) { rc = fail(p, SNXO_E_CYCLE, "cycle left after lagging"); goto done; }
    }
done:
    free(idx); free(low); free(comp); free(stk); free(cs_v); free(cs_f); free(indeg); free(onstk); free(key);
    return rc;
}

/* Real orthonormal spherical harmonics of every direction up to degree L,
 * index l*l + l + m (m = -l..l): Y_l0 = N_l0 P_l(mu), Y_lm = sqrt2 N_lm P_l^m(mu)
 * cos(m phi) and Y_l,-m = sqrt2 N_lm P_l^m(mu) sin(m phi) for m > 0, with
 * N_lm^2 = (2l+1)/(4 pi) (l-m)!/(l+m)!, mu = Omega_z, phi the azimuth of
 * (Omega_x, Omega_y) and P_l^m from the three-term recurrence in l. */
static int build_harmonics(snxo_problem *p) {
    int L = p->L, nm = (L + 1) * (L + 1);
    p->ylm = malloc(sizeof(double) * (size_t)p->nang * nm);
    if (!p->ylm) return fail(p, SNXO_E_OOM, "out of memory");
    for (int n = 0; n < p->nang; ++n) {
        const double *om = p->omega + 3 * n;
        double mu = om[2], phi = atan2(om[1], om[0]), st = sqrt(fmax(0.0, 1.0 - mu * mu));
        double P[8][8];                 /* P[l][m] */
        for (int m = 0; m <= L; ++m) {
            double pmm = 1.0;           /* (2m-1)!! sin^m */
            for (int k = 1; k <= m; ++k) pmm *= (2.0 * k - 1.0) * st;
            P[m][m] = pmm;
            if (m + 1 <= L) P[m + 1][m] = (2.0 * m + 1.0) * mu * pmm;
            for (int l = m + 2; l <= L; ++l)
                P[l][m] = ((2.0 * l - 1.0) * mu * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (l - m);
        }
        double *y = p->ylm + (size_t)n * nm;
        for (int l = 0; l <= L; ++l)
            for (int m = 0; m <= l; ++m) {
                double ratio = 1.0;     /* (l-m)!/(l+m)! */
                for (int k = l - m + 1; k <= l + m; ++k) ratio /= k;
                double N = sqrt((2.0 * l + 1.0) / (4.0 * PI) * ratio);
                if (m == 0) {
                    y[l * l + l] = N * P[l][0];
                } else {
                    y[l * l + l + m] = sqrt(2.0) * N * P[l][m] * cos(m * phi);
                    y[l * l + l - m] = sqrt(2.0) * N * P[l][m] * sin(m * phi);
                }
            }
    }
    return SNXO_OK;
}

/* Reflective planes: for each direction and axis, the direction with that
 * component negated (it must be in the quadrature set). */
static int build_reflection(snxo_problem *p) {
    p->rdir = malloc(sizeof(int32_t) * 3 * (size_t)p->nang);
    if (!p->rdir) return fail(p, SNXO_E_OOM, "out of memory");
    for (int n = 0; n < p->nang; ++n)
        for (int a = 0; a < 3; ++a) {
            double want[3] = {p->omega[3 * n], p->omega[3 * n + 1], p->omega[3 * n + 2]};
            want[a] = -want[a];
            int found = -1;
            for (int m = 0; m < p->nang && found < 0; ++m) {
                const double *om = p->omega + 3 * m;
                if (fabs(om[0] - want[0]) + fabs(om[1] - want[1]) + fabs(om[2] - want[2]) < 1e-12) found = m;
            }
            if (found < 0) return fail(p, SNXO_E_ARG, "quadrature not symmetric under reflection");
            p->rdir[3 * n + a] = found;
        }
    return SNXO_OK;
}

/* Reflective plane of boundary face f of K, or -1: the face's area vector lies
 * along an axis (its other two components at most 1e-12 of its length, which
 * rounding leaves on faces of a coordinate plane), and bit 2*axis + side (side
 * 1 for the outward +axis) of the mask is set. */
static int reflective_axis(const snxo_problem *p, int K, int f) {
    if (!p->refl || p->nbr[6 * K + f] >= 0) return -1;
    const double *A = p->area + 18L * K + 3 * f;
    double len = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        if (fabs(A[b]) <= 1e-12 * len && fabs(A[c]) <= 1e-12 * len) {
            int side = A[a] > 0.0;
            return (p->refl >> (2 * a + side)) & 1 ? a : -1;
        }
    }
    return -1;
}

int snxo_setup(snxo_problem *p) {
    if (!p || !p->cv || !p->omega || !p->sigt) return fail(p, SNXO_E_STATE, "mesh, quadrature and materials must be set");
    free_derived(p);
    size_t C = (size_t)p->ncell;
    p->M = malloc(sizeof(double) * 64 * C);
    p->S = malloc(sizeof(double) * 192 * C);
    p->F = calloc(288 * C, sizeof(double));
    p->area = calloc(18 * C, sizeof(double));
    p->nbr = malloc(sizeof(int32_t) * 6 * C);
    p->nbrf = malloc(sizeof(int32_t) * 6 * C);
    p->perm = malloc(sizeof(int32_t) * 24 * C);
    p->inflow = malloc(sizeof(int32_t) * 8 * C);
    p->level = malloc(sizeof(int32_t) * 8 * C);
    p->order = malloc(sizeof(int32_t) * 8 * C);
    if (p->designation >= 1) p->ain = malloc(sizeof(int32_t) * (size_t)p->nang * C);
    if (p->designation == 2) {
        p->aord = malloc(sizeof(int32_t) * (size_t)p->nang * C);
        p->alag = malloc(sizeof(int32_t) * (size_t)p->nang * C);
    }
    if (!p->M || !p->S || !p->F || !p->area || !p->nbr || !p->nbrf || !p->perm || !p->inflow || !p->level || !p->order
        || (p->designation >= 1 && !p->ain) || (p->designation == 2 && (!p->aord || !p->alag))) {
        free_derived(p);
        return fail(p, SNXO_E_OOM, "out of memory");
    }
    int rc = build_topology(p);
    if (!rc) rc = build_geometry(p);
    if (!rc) rc = build_dag(p);
    if (!rc && p->designation >= 1) rc = build_angle_inflow(p);
    if (!rc && p->designation == 2) rc = build_angle_order(p);
    if (!rc && p->refl) rc = build_reflection(p);
    if (!rc && p->L) rc = build_harmonics(p);
    if (rc) { free_derived(p); return rc; }
    p->ready = 1;
    return SNXO_OK;
}

/* ------------------------------------------------------------------ sweep */

/* One (cell, angle, group) local system of the upwind DG form:
 *   A = sum_a Om_a S^a + sigma_t M - sum_{f in} sum_a Om_a F^a_f
 *   b = M q - sum_{f in} (Om . F_f) psi_up_f
 * with q the nodal source values and psi_up the upwind trace at f's nodes.
 * "in" is the octant's inflow set (designation 0) or the angle's own
 * (designations 1 and 2).  psi_up is read from psi_cur, which holds the newest
 * value of every cell: this sweep's for cells already visited, the previous
 * sweep's (or zero) for the rest.  Two exceptions:
 *   - designation 2, a face lagged to break a cycle: the neighbour's value of
 *     the previous sweep, psi_lag[N * lag_stride + node] (NULL = zero);
 *   - a reflective face: the mirrored direction m's own trace at these nodes,
 *     from this sweep (psi_now, octants in sequence) when m's octant came
 *     earlier, else from the previous sweep (psi_prev). */
static int solve_local(const snxo_problem *p, int K, int n, int g, const double *qnodal,
                       const double *psi_cur /*[C][8] this angle and group*/,
                       const double *psi_prev /*[nang][C][G][8] or NULL*/,
                       const double *psi_lag, long lag_stride,
                       const double *psi_now /*[nang][C][8] this group, or NULL*/, double x[8], double *leak_out) {
    const double *om = p->omega + 3 * n;
    const double *M = p->M + 64L * K, *S = p->S + 192L * K;
    int per = p->nang / 8, o = n / per;
    int mask = p->designation >= 1 ? p->ain[(long)n * p->ncell + K] : p->inflow[(long)o * p->ncell + K];
    int lagged = p->designation == 2 ? p->alag[(long)n * p->ncell + K] : 0;
    double sigt = p->sigt[(long)K * p->G + g];
    double A[64], b[8], up[6][4];
    for (int i = 0; i < 8; ++i) {
        double s = 0.0;
        for (int j = 0; j < 8; ++j) {
            A[8 * i + j] = om[0] * S[8 * i + j] + om[1] * S[64 + 8 * i + j] + om[2] * S[128 + 8 * i + j]
                         + sigt * M[8 * i + j];
            s += M[8 * i + j] * qnodal[j];
        }
        b[i] = s;
    }
    for (int f = 0; f < 6; ++f) {
        if (!((mask >> f) & 1)) continue;
        int fn[4];
        face_nodes(f, fn);
        const double *F = p->F + 288L * K + 48 * f;
        int N = p->nbr[6 * K + f];
        for (int l = 0; l < 4; ++l) {
            if (N >= 0 && ((lagged >> f) & 1))
                up[f][l] = psi_lag ? psi_lag[(long)N * lag_stride + p->perm[24 * K + 4 * f + l]] : 0.0;
            else if (N >= 0) up[f][l] = psi_cur[8L * N + p->perm[24 * K + 4 * f + l]];
            else if (reflective_axis(p, K, f) >= 0) {
                int m = p->rdir[3 * n + reflective_axis(p, K, f)];
                if (psi_now && m / per < o)
                    up[f][l] = psi_now[((long)m * p->ncell + K) * 8 + fn[l]];
                else
                    up[f][l] = psi_prev ? psi_prev[(((long)m * p->ncell + K) * p->G + g) * 8 + fn[l]] : 0.0;
            }
            else if (p->bnd_in) up[f][l] = p->bnd_in[((((long)K * 6 + f) * p->nang + n) * p->G + g) * 4 + l];
            else if (p->bkind == 1) up[f][l] = p->psib[g];
            else up[f][l] = 0.0;
        }
        for (int k = 0; k < 4; ++k) {
            double s = 0.0;
            for (int l = 0; l < 4; ++l) {
                double of = om[0] * F[4 * k + l] + om[1] * F[16 + 4 * k + l] + om[2] * F[32 + 4 * k + l];
                A[8 * fn[k] + fn[l]] -= of;
                s += of * up[f][l];
            }
            b[fn[k]] -= s;
        }
    }
    if (lu_solve(8, A, b, x)) return -1;
    if (leak_out) {
        /* net outflow through the upwind traces: own values on outflow faces,
         * upwind values on inflow faces */
        double L = 0.0;
        for (int f = 0; f < 6; ++f) {
            int fn[4];
            face_nodes(f, fn);
            const double *F = p->F + 288L * K + 48 * f;
            int in = (mask >> f) & 1;
            for (int k = 0; k < 4; ++k)
                for (int l = 0; l < 4; ++l) {
                    double of = om[0] * F[4 * k + l] + om[1] * F[16 + 4 * k + l] + om[2] * F[32 + 4 * k + l];
                    L += of * (in ? up[f][l] : x[fn[l]]);
                }
        }
        *leak_out = L;
    }
    return 0;
}

/* Nodal isotropic source of (cell K, group g) per unit solid angle:
 * (Q + scattering into g) / (4 pi) at each of the 8 nodes (Eq. 1 with
 * isotropic scattering).  Without a group matrix the scattering is
 * sigma_s phi_g (within the group).  With one it is
 * sum over g' of sigma(g' -> g) phi_g', the diagonal taken from phi_in and the
 * other groups from qouter when given (the cross-group source of an outer
 * iteration, held fixed during its inner iterations), else from phi_in too. */
static void source_nodal(const snxo_problem *p, const double *phi_in, const double *qouter, int K, int g,
                         double qn[8]) {
    int G = p->G;
    for (int j = 0; j < 8; ++j) {
        double ph = phi_in ? phi_in[((long)K * G + g) * 8 + j] : 0.0;
        double sc;
        if (!p->sgg) {
            sc = p->sigs[(long)K * G + g] * ph;
        } else {
            const double *S = p->sgg + (size_t)p->cmat[K] * G * G;
            sc = S[(long)g * G + g] * ph;
            if (qouter) {
                sc += qouter[((long)K * G + g) * 8 + j];
            } else {
                for (int h = 0; h < G; ++h)
                    if (h != g && phi_in) sc += S[(long)h * G + g] * phi_in[((long)K * G + h) * 8 + j];
            }
        }
        qn[j] = (p->q[(long)K * G + g] + sc) / (4.0 * PI);
    }
}

/* The cells of an angle are visited in the octant's topological order, so
 * under designation 0 every inflow neighbour is already done.  Under
 * designation 1 an inflow neighbour that comes later in that order still
 * holds the previous sweep's value in psi_cur (initialised from psi_prev):
 * that face is lagged.  Under designation 2 the cells of direction n are
 * visited in n's own order, where every inflow neighbour is done except
 * across the faces lagged to break cycles, which read psi_prev.  Octants run
 * in the order 0..7 (a group's whole sweep is sequential). */
static int sweep_src(snxo_problem *p, const double *phi_in, const double *qouter, const double *psi_prev,
                     double *phi_out, double *psi_all, double *leak, double *leak_ang) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (!phi_out) return fail(p, SNXO_E_ARG, "phi_out is NULL");
    int C = p->ncell, G = p->G, nang = p->nang, per = nang / 8;
    memset(phi_out, 0, sizeof(double) * 8 * (size_t)C * G);
    if (leak) memset(leak, 0, sizeof(double) * (size_t)C * G);
    /* Anisotropic scattering: the flux moments phi_lm = sum_n w_n Y_lm(Omega_n)
     * psi_n of degree 1..L, from the previous sweep's angular flux (the scalar
     * flux phi_in carries degree 0).  The source of direction n then gains
     * sum_{l>=1} sigma_l sum_m Y_lm(Omega_n) phi_lm, the expansion of the
     * scattering law sum_l (2l+1)/(4 pi) sigma_l P_l(Omega . Omega'). */
    int nm = (p->L + 1) * (p->L + 1);
    double *mom = NULL;
    if (p->L) {
        mom = calloc((size_t)C * G * nm * 8, sizeof(double));
        if (!mom) return fail(p, SNXO_E_OOM, "out of memory");
        if (psi_prev)
            for (int n = 0; n < nang; ++n)
                for (long K = 0; K < C; ++K)
                    for (int g = 0; g < G; ++g)
                        for (int k = 1; k < nm; ++k)
                            for (int j = 0; j < 8; ++j)
                                mom[(((size_t)K * G + g) * nm + k) * 8 + j] +=
                                    p->w[n] * p->ylm[(size_t)n * nm + k] * psi_prev[(((long)n * C + K) * G + g) * 8 + j];
    }
    int bad = 0;
    /* Groups are independent: each group's angle sum runs sequentially over
     * (octant, angle) so the result does not depend on the thread count. */
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int g = 0; g < G; ++g) {
        double *psi_cur = malloc(sizeof(double) * 8 * (size_t)C);
        /* octants in sequence: this group's angular flux of the current sweep,
         * read by reflective faces whose mirrored octant came earlier */
        double *psi_now = (p->refl && p->octseq) ? malloc(sizeof(double) * 8 * (size_t)C * nang) : NULL;
        if (!psi_cur || (p->refl && p->octseq && !psi_now)) { free(psi_cur); free(psi_now); bad = 1; continue; }
        for (int o = 0; o < 8; ++o)
            for (int a = 0; a < per; ++a) {
                int n = o * per + a;
                for (long K = 0; K < C; ++K)
                    for (int j = 0; j < 8; ++j)
                        psi_cur[8 * K + j] = psi_prev ? psi_prev[(((long)n * C + K) * G + g) * 8 + j] : 0.0;
                const int32_t *ord = p->designation == 2 ? p->aord + (long)n * C : p->order + (long)o * C;
                const double *lag = psi_prev ? psi_prev + ((long)n * C * G + g) * 8 : NULL;
                for (int t = 0; t < C; ++t) {
                    int K = ord[t];
                    double qn[8], x[8], L = 0.0;
                    if (p->ang_src) {
                        for (int j = 0; j < 8; ++j) qn[j] = p->ang_src[(((long)K * nang + n) * G + g) * 8 + j];
                    } else {
                        source_nodal(p, phi_in, qouter, K, g, qn);
                        for (int l = 1; l <= p->L; ++l) {
                            double sl = p->sigl[((size_t)K * G + g) * p->L + (l - 1)];
                            for (int k = l * l; k < (l + 1) * (l + 1); ++k)
                                for (int j = 0; j < 8; ++j)
                                    qn[j] += sl * p->ylm[(size_t)n * nm + k] * mom[(((size_t)K * G + g) * nm + k) * 8 + j];
                        }
                    }
                    if (solve_local(p, K, n, g, qn, psi_cur, psi_prev, lag, 8L * G, psi_now, x,
                                    (leak || leak_ang) ? &L : NULL)) {
                        bad = 1;
                        break;
                    }
                    for (int j = 0; j < 8; ++j) {
                        psi_cur[8L * K + j] = x[j];
                        if (psi_now) psi_now[((long)n * C + K) * 8 + j] = x[j];
                        phi_out[((long)K * G + g) * 8 + j] += p->w[n] * x[j];
                        if (psi_all) psi_all[(((long)n * C + K) * G + g) * 8 + j] = x[j];
                    }
                    if (leak) leak[(long)K * G + g] += p->w[n] * L;
                    if (leak_ang) leak_ang[((long)n * C + K) * G + g] = L;
                }
            }
        free(psi_cur);
        free(psi_now);
    }
    free(mom);
    if (bad) return fail(p, SNXO_E_MESH, "singular local system or out of memory");
    return SNXO_OK;
}

int snxo_sweep(snxo_problem *p, const double *phi_in, const double *psi_prev, double *phi_out,
               double *psi_all, double *leak, double *leak_ang) {
    return sweep_src(p, phi_in, NULL, psi_prev, phi_out, psi_all, leak, leak_ang);
}

/* The sweep of one (angle n, group g) alone: psi_out[ncell][8] receives that
 * angle's and group's psi.  For a given phi_in the angles and groups of one
 * source iteration are independent (Eq. 1 with the scattering source taken
 * from phi_in), so this is the same loop as one (n, g) pass of snxo_sweep;
 * it lets large problems be checked on sampled (angle, group) pairs. */
int snxo_sweep_angle(snxo_problem *p, const double *phi_in, int n, int g, const double *psi_prev,
                     double *psi_out) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (!psi_out) return fail(p, SNXO_E_ARG, "psi_out is NULL");
    int C = p->ncell, G = p->G, nang = p->nang, per = nang / 8;
    if (n < 0 || n >= nang || g < 0 || g >= G) return fail(p, SNXO_E_ARG, "angle or group out of range");
    if (p->refl || p->L) return fail(p, SNXO_E_ARG, "reflective planes and anisotropy couple directions: use snxo_sweep");
    int o = n / per;
    const int32_t *ord = p->designation == 2 ? p->aord + (long)n * C : p->order + (long)o * C;
    for (long i = 0; i < 8L * C; ++i) psi_out[i] = psi_prev ? psi_prev[i] : 0.0;
    for (int t = 0; t < C; ++t) {
        int K = ord[t];
        double qn[8], x[8];
        if (p->ang_src) {
            for (int j = 0; j < 8; ++j) qn[j] = p->ang_src[(((long)K * nang + n) * G + g) * 8 + j];
        } else {
            source_nodal(p, phi_in, NULL, K, g, qn);
        }
        if (solve_local(p, K, n, g, qn, psi_out, NULL, psi_prev, 8, NULL, x, NULL))
            return fail(p, SNXO_E_MESH, "singular local system");
        for (int j = 0; j < 8; ++j) psi_out[8L * K + j] = x[j];
    }
    return SNXO_OK;
}

/* Relative max-norm change ||phi_new - phi_old||_inf / ||phi_new||_inf. */
static double rel_change(const double *a, const double *b, size_t n) {
    double num = 0.0, den = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double d = fabs(a[i] - b[i]);
        if (d > num) num = d;
        if (fabs(a[i]) > den) den = fabs(a[i]);
    }
    return den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
}

int snxo_solve(snxo_problem *p, double tol, int max_it, const double *phi0,
               double *phi_out, int *iters, double *eps, double *hist) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (!phi_out || max_it < 1) return fail(p, SNXO_E_ARG, "bad solve arguments");
    size_t n = 8 * (size_t)p->ncell * p->G;
    double *cur = malloc(sizeof(double) * n);
    /* designation 1 and reflective planes: the angular flux carried between
     * sweeps (previous and next kept apart: a reflective face reads another
     * direction's previous values) */
    int carry = p->designation >= 1 || p->refl || p->L;
    double *psi = carry ? calloc(n * (size_t)p->nang, sizeof(double)) : NULL;
    double *psi2 = carry ? calloc(n * (size_t)p->nang, sizeof(double)) : NULL;
    if (!cur || (carry && (!psi || !psi2))) {
        free(cur); free(psi); free(psi2);
        return fail(p, SNXO_E_OOM, "out of memory");
    }
    if (phi0) memcpy(cur, phi0, sizeof(double) * n); else memset(cur, 0, sizeof(double) * n);
    int it = 0, rc = SNXO_OK;
    double e = INFINITY;
    while (it < max_it) {
        rc = snxo_sweep(p, cur, psi, phi_out, psi2, NULL, NULL);
        { double *t = psi; psi = psi2; psi2 = t; }
        if (rc) break;
        e = rel_change(phi_out, cur, n);
        if (hist) hist[it] = e;
        ++it;
        memcpy(cur, phi_out, sizeof(double) * n);
        if (e <= tol) break;
    }
    free(cur);
    free(psi);
    free(psi2);
    if (iters) *iters = it;
    if (eps) *eps = e;
    if (rc) return rc;
    return e <= tol ? SNXO_OK : SNXO_E_NOCONV;
}

/* Inner and outer iterations (the benchmark of Section 3.6 runs five of each):
 * each outer iteration fixes the cross-group scattering source from its
 * starting flux, then runs `inner` source iterations with the within-group
 * scattering only; it ends with the relative max-norm change of the flux over
 * the outer iteration.  Stops after `outer` outer iterations, or earlier when
 * tol > 0 and the change is <= tol.  Without a group matrix the cross-group
 * source is zero.  Designation 1 carries the angular flux across all sweeps. */
int snxo_solve_outer(snxo_problem *p, int outer, int inner, double tol, const double *phi0, double *phi_out,
                     int *outers_done, int *inners_done, double *eps) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (!phi_out || outer < 1 || inner < 1 || !(tol >= 0.0)) return fail(p, SNXO_E_ARG, "bad solve arguments");
    int C = p->ncell, G = p->G;
    size_t n = 8 * (size_t)C * G;
    double *start = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n), *qo = calloc(n, sizeof(double));
    int carry = p->designation >= 1 || p->refl || p->L;
    double *psi = carry ? calloc(n * (size_t)p->nang, sizeof(double)) : NULL;
    double *psi2 = carry ? calloc(n * (size_t)p->nang, sizeof(double)) : NULL;
    if (!start || !x || !qo || (carry && (!psi || !psi2))) {
        free(start); free(x); free(qo); free(psi); free(psi2);
        return fail(p, SNXO_E_OOM, "out of memory");
    }
    if (phi0) memcpy(start, phi0, sizeof(double) * n); else memset(start, 0, sizeof(double) * n);
    int k = 0, it = 0, rc = SNXO_OK;
    double e = INFINITY;
    while (k < outer) {
        if (p->sgg)
            for (int K = 0; K < C; ++K) {
                const double *S = p->sgg + (size_t)p->cmat[K] * G * G;
                for (int g = 0; g < G; ++g)
                    for (int j = 0; j < 8; ++j) {
                        double v = 0.0;
                        for (int h = 0; h < G; ++h)
                            if (h != g) v += S[(long)h * G + g] * start[((long)K * G + h) * 8 + j];
                        qo[((long)K * G + g) * 8 + j] = v;
                    }
            }
        memcpy(x, start, sizeof(double) * n);
        for (int i = 0; i < inner && !rc; ++i) {
            rc = sweep_src(p, x, qo, psi, phi_out, psi2, NULL, NULL);
            { double *t = psi; psi = psi2; psi2 = t; }
            if (!rc) memcpy(x, phi_out, sizeof(double) * n);
            ++it;
        }
        if (rc) break;
        e = rel_change(x, start, n);
        memcpy(start, x, sizeof(double) * n);
        ++k;
        if (tol > 0.0 && e <= tol) break;
    }
    memcpy(phi_out, start, sizeof(double) * n);
    free(start); free(x); free(qo); free(psi); free(psi2);
    if (outers_done) *outers_done = k;
    if (inners_done) *inners_done = it;
    if (eps) *eps = e;
    if (rc) return rc;
    return (tol == 0.0 || e <= tol) ? SNXO_OK : SNXO_E_NOCONV;
}

/* Cell balance of one sweep: source 1^T M (Q + sigma_s phi_in) equals
 * absorption sigma_t 1^T M phi_out plus angle-weighted net outflow. */
int snxo_balance(snxo_problem *p, const double *phi_in, const double *phi_out,
                 const double *leak, double *out) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (!phi_out || !leak || !out) return fail(p, SNXO_E_ARG, "bad balance arguments");
    int C = p->ncell, G = p->G;
    for (int g = 0; g < G; ++g) {
        double src = 0.0, ab = 0.0, lk = 0.0, worst = 0.0;
        for (int K = 0; K < C; ++K) {
            const double *M = p->M + 64L * K;
            double s = 0.0, a = 0.0, qn[8];
            source_nodal(p, phi_in, NULL, K, g, qn);
            for (int i = 0; i < 8; ++i)
                for (int j = 0; j < 8; ++j) {
                    s += M[8 * i + j] * 4.0 * PI * qn[j];
                    a += M[8 * i + j] * p->sigt[(long)K * G + g] * phi_out[((long)K * G + g) * 8 + j];
                }
            double l = leak[(long)K * G + g];
            double scale = fmax(fabs(s), fmax(fabs(a), fabs(l)));
            double rel = scale > 0.0 ? fabs(s - a - l) / scale : 0.0;
            if (rel > worst) worst = rel;
            src += s; ab += a; lk += l;
        }
        out[4 * g + 0] = src; out[4 * g + 1] = ab; out[4 * g + 2] = lk; out[4 * g + 3] = worst;
    }
    return SNXO_OK;
}

int snxo_integrated_flux(snxo_problem *p, const double *phi, double *out) {
    if (!p || !p->ready || !phi || !out) return fail(p, SNXO_E_ARG, "bad arguments");
    int C = p->ncell, G = p->G;
    for (int g = 0; g < G; ++g) {
        double s = 0.0, v = 0.0;
        for (int K = 0; K < C; ++K) {
            const double *M = p->M + 64L * K;
            for (int i = 0; i < 8; ++i) {
                s += phi[((long)K * G + g) * 8 + i];
                for (int j = 0; j < 8; ++j) v += M[8 * i + j] * phi[((long)K * G + g) * 8 + j];
            }
        }
        out[2 * g] = s; out[2 * g + 1] = v;
    }
    return SNXO_OK;
}

int snxo_get_geometry(snxo_problem *p, double *M, double *S, double *F, double *area,
                      int32_t *nbr, int32_t *nbr_face, int32_t *perm) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    size_t C = (size_t)p->ncell;
    if (M) memcpy(M, p->M, sizeof(double) * 64 * C);
    if (S) memcpy(S, p->S, sizeof(double) * 192 * C);
    if (F) memcpy(F, p->F, sizeof(double) * 288 * C);
    if (area) memcpy(area, p->area, sizeof(double) * 18 * C);
    if (nbr) memcpy(nbr, p->nbr, sizeof(int32_t) * 6 * C);
    if (nbr_face) memcpy(nbr_face, p->nbrf, sizeof(int32_t) * 6 * C);
    if (perm) memcpy(perm, p->perm, sizeof(int32_t) * 24 * C);
    return SNXO_OK;
}

int snxo_get_dag(snxo_problem *p, int32_t *inflow, int32_t *level, int32_t *order) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    size_t C = (size_t)p->ncell;
    if (inflow) memcpy(inflow, p->inflow, sizeof(int32_t) * 8 * C);
    if (level) memcpy(level, p->level, sizeof(int32_t) * 8 * C);
    if (order) memcpy(order, p->order, sizeof(int32_t) * 8 * C);
    return SNXO_OK;
}

int snxo_get_angle_inflow(snxo_problem *p, int32_t *ain) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (p->designation < 1 || !ain) return fail(p, SNXO_E_ARG, "per-angle masks exist under designations 1 and 2 only");
    memcpy(ain, p->ain, sizeof(int32_t) * (size_t)p->nang * p->ncell);
    return SNXO_OK;
}

int snxo_get_angle_order(snxo_problem *p, int32_t *order, int32_t *lag) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (p->designation != 2) return fail(p, SNXO_E_ARG, "per-direction orders exist under designation 2 only");
    size_t n = (size_t)p->nang * p->ncell;
    if (order) memcpy(order, p->aord, sizeof(int32_t) * n);
    if (lag) memcpy(lag, p->alag, sizeof(int32_t) * n);
    return SNXO_OK;
}

int snxo_get_harmonics(snxo_problem *p, double *y) {
    if (!p || !p->ready) return fail(p, SNXO_E_STATE, "setup has not run");
    if (!p->L || !y) return fail(p, SNXO_E_ARG, "harmonics exist with anisotropic scattering only");
    memcpy(y, p->ylm, sizeof(double) * (size_t)p->nang * (p->L + 1) * (p->L + 1));
    return SNXO_OK;
}
