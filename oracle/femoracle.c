/*
 * femoracle.c -- plain, slow, obviously correct FP64 reference for the
 * Laplace / Jacobi-PCG solve path.  TEST INFRASTRUCTURE ONLY: it is loaded by
 * the tests, by the smoke check and by the CPU-baseline leg of the benchmark,
 * never by the library.  It shares no code, header or table with the HIP
 * library.
 *
 * What it computes, step by step, with the passage each step follows:
 *
 *  1. DOF numbering.  P1: the mesh vertices.  P2: the vertices, then one DOF
 *     per mesh edge, edges ordered by their (min, max) vertex pair.  The
 *     paper's Table 7 (Sect. 4.2, "polynomial basis") varies the FEM degree
 *     from 1 to 4 on a triangle mesh; P3 and P4 (triangles only) number the
 *     vertices, then k-1 DOFs per edge (edges in (min, max) order, the DOF t
 *     of an edge at ((k-t) x_min + t x_max) / k), then (k-1)(k-2)/2 DOFs per
 *     cell (cells in order; inside a cell, interior lattice points in
 *     decreasing lexicographic order of their barycentric index).  A DOF on
 *     a boundary facet whose vertices are all flagged is a Dirichlet DOF
 *     (Sect. 2.2: u = f on the boundary).
 *  2. Element matrices K^e_ij = integral over T of grad(phi_i).grad(phi_j).
 *     P1 is written in gradient form, |T| grad(l_i).grad(l_j), and separately
 *     in the paper's cotangent form (Sect. 2.2: w(i,j) = (1/6) sum l_k cot a_k
 *     for tetrahedra, (cot a + cot b)/2 for triangles), where K_ij = -w(i,j)
 *     and K_ii = sum_j w(i,j).  The sign is flipped with respect to the
 *     paper's A(i,j) so that K is positive semi-definite.  P2 is integrated
 *     with a quadrature rule exact for the quadratic integrand.  P3/P4: the
 *     nodal basis of the degree-k polynomials at the lattice points, from the
 *     inverse of their monomial Vandermonde matrix, integrated with a
 *     collapsed (Duffy) Gauss-Legendre product rule that is exact for the
 *     degree 2k-2 integrand.
 *  3. Assembly: coordinate triplets, stable counting sort by column and then
 *     by row, duplicates summed in element order.  The structural pattern
 *     (every DOF pair sharing an element) is kept, zeros included.
 *  4. Dirichlet lifting with zero source: A = K_II, b = -K_ID g_D.
 *  5. Jacobi-preconditioned CG (Sect. 2.1, preconditioned system with
 *     M = diag(A)), one column at a time, zero initial guess, stopping test
 *     of Eq. (2) on the recursive residual, then the true residual
 *     ||b - A x|| / ||b||; if that exceeds tol the solve restarts from x
 *     (at most 3 times).  Iterations count the products A p.
 *  6. Eq. (1) error and Eq. (2) residual helpers.
 *  7. The paper's own iterative solver (Sect. 3.2): BiCGStab, right
 *     preconditioned by Block-Jacobi with exact solves of blocks of bs
 *     consecutive rows (dense LU with partial pivoting).
 *
 * Every function returns 0 on success and a negative code on failure.
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_EMESH -3
#define ORC_EBREAK -4

/* ------------------------------------------------------------------------- */
/* small dense helpers                                                        */
/* ------------------------------------------------------------------------- */

/* Jacobian J[r][c] = x_{c+1}[r] - x_0[r]; returns det J and writes the
 * gradients of the barycentric coordinates, G[i][r] = d l_i / d x_r. */
static double bary_gradients(int dim, const double *X, double *G)
{
    double J[3][3], inv[3][3], det;
    for (int r = 0; r < dim; r++)
        for (int c = 0; c < dim; c++)
            J[r][c] = X[(c + 1) * dim + r] - X[r];
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        inv[0][0] = J[1][1] / det;
        inv[0][1] = -J[0][1] / det;
        inv[1][0] = -J[1][0] / det;
        inv[1][1] = J[0][0] / det;
    } else {
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
            - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
            + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    /* lambda_{c+1}(x) = (J^{-1} (x - x_0))_c, so grad lambda_{c+1} = row c */
    for (int r = 0; r < dim; r++) G[0 * dim + r] = 0.0;
    for (int c = 0; c < dim; c++)
        for (int r = 0; r < dim; r++) {
            G[(c + 1) * dim + r] = inv[c][r];
            G[0 * dim + r] -= inv[c][r];
        }
    return det;
}

static double simplex_measure(int dim, double det)
{
    return dim == 2 ? det / 2.0 : det / 6.0;
}

/* ------------------------------------------------------------------------- */
/* element matrices                                                           */
/* ------------------------------------------------------------------------- */

/* P1 gradient form: K_ij = |T| grad(l_i) . grad(l_j). */
int orc_p1_element(int dim, const double *X, double *K)
{
    double G[12];
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    double det = bary_gradients(dim, X, G);
    if (!(det > 0.0)) return ORC_EMESH;
    double vol = simplex_measure(dim, det);
    int nl = dim + 1;
    for (int i = 0; i < nl; i++)
        for (int j = 0; j < nl; j++) {
            double s = 0.0;
            for (int r = 0; r < dim; r++) s += G[i * dim + r] * G[j * dim + r];
            K[i * nl + j] = vol * s;
        }
    return 0;
}

static void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* P1 cotangent form (the paper's Laplacian weights, Sect. 2.2).
 * Triangle: w_ij = cot(angle at the third vertex) / 2.
 * Tetrahedron: w_ij = l_kl cot(theta_kl) / 6, where (k,l) is the edge opposite
 * to (i,j), l_kl its length and theta_kl the dihedral angle along it.
 * K_ij = -w_ij (i != j), K_ii = sum_{j != i} w_ij. */
int orc_p1_element_cot(int dim, const double *X, double *K)
{
    int nl = dim + 1;
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    for (int i = 0; i < nl * nl; i++) K[i] = 0.0;
    for (int i = 0; i < nl; i++)
        for (int j = i + 1; j < nl; j++) {
            double w;
            if (dim == 2) {
                int l = 3 - i - j;
                double a[2] = {X[i * 2] - X[l * 2], X[i * 2 + 1] - X[l * 2 + 1]};
                double b[2] = {X[j * 2] - X[l * 2], X[j * 2 + 1] - X[l * 2 + 1]};
                double cr = a[0] * b[1] - a[1] * b[0];
                double dt = a[0] * b[0] + a[1] * b[1];
                if (cr == 0.0) return ORC_EMESH;
                w = 0.5 * dt / fabs(cr);
            } else {
                int kl[2], c = 0;
                for (int t = 0; t < 4; t++)
                    if (t != i && t != j) kl[c++] = t;
                const double *xk = X + 3 * kl[0], *xl = X + 3 * kl[1];
                double e[3], a[3], b[3], u[3], v[3], uxv[3];
                sub3(xl, xk, e);
                sub3(X + 3 * i, xk, a);
                sub3(X + 3 * j, xk, b);
                double len = sqrt(dot3(e, e));
                double eh[3] = {e[0] / len, e[1] / len, e[2] / len};
                double ae = dot3(a, eh), be = dot3(b, eh);
                for (int r = 0; r < 3; r++) {
                    u[r] = a[r] - ae * eh[r];
                    v[r] = b[r] - be * eh[r];
                }
                cross3(u, v, uxv);
                double sn = sqrt(dot3(uxv, uxv));
                if (sn == 0.0) return ORC_EMESH;
                w = len * (dot3(u, v) / sn) / 6.0;
            }
            K[i * nl + j] = -w;
            K[j * nl + i] = -w;
            K[i * nl + i] += w;
            K[j * nl + j] += w;
        }
    return 0;
}

/* local P2 numbering: vertices 0..d, then the edges (a,b), a<b, in
 * lexicographic order */
static int p2_local_edges(int dim, int E[6][2])
{
    int c = 0;
    for (int a = 0; a <= dim; a++)
        for (int b = a + 1; b <= dim; b++) {
            E[c][0] = a;
            E[c][1] = b;
            c++;
        }
    return c;
}

/* Gradients of the P2 basis at barycentric point L:
 * vertex i: phi = l_i (2 l_i - 1), grad = (4 l_i - 1) grad l_i;
 * edge (a,b): phi = 4 l_a l_b, grad = 4 (l_a grad l_b + l_b grad l_a). */
static void p2_grads(int dim, const double *G, const double *L, double *out)
{
    int E[6][2];
    int ne = p2_local_edges(dim, E);
    int nv = dim + 1;
    for (int i = 0; i < nv; i++)
        for (int r = 0; r < dim; r++)
            out[i * dim + r] = (4.0 * L[i] - 1.0) * G[i * dim + r];
    for (int e = 0; e < ne; e++) {
        int a = E[e][0], b = E[e][1];
        for (int r = 0; r < dim; r++)
            out[(nv + e) * dim + r] = 4.0 * (L[a] * G[b * dim + r] + L[b] * G[a * dim + r]);
    }
}

/* P2: K_ij = integral of grad(phi_i).grad(phi_j); the integrand is a
 * quadratic polynomial, integrated exactly by
 *   triangle: the three edge midpoints, weight |T|/3 each;
 *   tetrahedron: the symmetric 4-point rule with barycentric coordinates
 *   (a,b,b,b), a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20, weight |T|/4. */
int orc_p2_element(int dim, const double *X, double *K)
{
    double G[12], Q[10 * 3];
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    double det = bary_gradients(dim, X, G);
    if (!(det > 0.0)) return ORC_EMESH;
    double vol = simplex_measure(dim, det);
    int nl = dim == 2 ? 6 : 10;
    int nq = dim == 2 ? 3 : 4;
    double pts[4][4];
    if (dim == 2) {
        double m[3][3] = {{0.5, 0.5, 0.0}, {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}};
        for (int q = 0; q < 3; q++)
            for (int i = 0; i < 3; i++) pts[q][i] = m[q][i];
    } else {
        double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0, b = (5.0 - sqrt(5.0)) / 20.0;
        for (int q = 0; q < 4; q++)
            for (int i = 0; i < 4; i++) pts[q][i] = (i == q) ? a : b;
    }
    for (int i = 0; i < nl * nl; i++) K[i] = 0.0;
    for (int q = 0; q < nq; q++) {
        p2_grads(dim, G, pts[q], Q);
        double w = vol / nq;
        for (int i = 0; i < nl; i++)
            for (int j = 0; j < nl; j++) {
                double s = 0.0;
                for (int r = 0; r < dim; r++) s += Q[i * dim + r] * Q[j * dim + r];
                K[i * nl + j] += w * s;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* P3 / P4 triangles                                                          */
/* ------------------------------------------------------------------------- */

/* Local Pk numbering of the oracle: lattice points (i/k, j/k) of the
 * reference triangle (0,0), (1,0), (0,1), i outer (0..k), j inner (0..k-i);
 * barycentric index (k-i-j, i, j). */
static int pk_local_points(int k, int A[15][3])
{
    int c = 0;
    for (int i = 0; i <= k; i++)
        for (int j = 0; j <= k - i; j++) {
            A[c][0] = k - i - j;
            A[c][1] = i;
            A[c][2] = j;
            c++;
        }
    return c;
}

/* Gauss-Legendre rule with n points on [0,1]: Newton's method on the
 * Legendre polynomial P_n (three-term recurrence) from the starting guesses
 * cos(pi (i + 3/4) / (n + 1/2)); weight 1 / ((1 - z^2) P_n'(z)^2). */
static void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(acos(-1.0) * (i + 0.75) / (n + 0.5)), p0 = 1.0, p1 = z, dp = 1.0;
        for (int it = 0; it < 100; it++) {
            p0 = 1.0;
            p1 = z;
            for (int j = 2; j <= n; j++) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        p0 = 1.0;
        p1 = z;
        for (int j = 2; j <= n; j++) {
            double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 + z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* inverse of the n x n matrix M (row-major) by Gauss-Jordan elimination
 * with partial pivoting; returns 0 or ORC_EINVAL when singular */
static int invert(int n, const double *M, double *out)
{
    double a[15][30];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++) a[i][j] = j < n ? M[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
        if (a[p][c] == 0.0) return ORC_EINVAL;
        for (int j = 0; j < 2 * n; j++) { double t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t; }
        double d = a[c][c];
        for (int j = 0; j < 2 * n; j++) a[c][j] /= d;
        for (int r = 0; r < n; r++)
            if (r != c && a[r][c] != 0.0) {
                double f = a[r][c];
                for (int j = 0; j < 2 * n; j++) a[r][j] -= f * a[c][j];
            }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) out[i * n + j] = a[i][n + j];
    return 0;
}

/* P3/P4 triangle stiffness K_ij = integral of grad(phi_i).grad(phi_j) in the
 * local numbering of pk_local_points.  phi_j = sum_m C[m][j] xi^p eta^q over
 * the monomials p + q <= k, C the inverse Vandermonde matrix at the lattice
 * points.  Reference gradients map to the cell by grad_x = J^-T grad_xi.
 * Quadrature: xi = u (1 - v), eta = v over the unit square with n = k + 1
 * Gauss points per direction (weight w_u w_v (1 - v)), exact for
 * polynomials of degree 2n - 2 >= 2k - 2. */
int orc_pk_element(int k, const double *X, double *K)
{
    if (k < 3 || k > 4) return ORC_EINVAL;
    double G[12];
    double det = bary_gradients(2, X, G);
    if (!(det > 0.0)) return ORC_EMESH;
    int A[15][3], mono[15][2];
    int nl = pk_local_points(k, A), nm = 0;
    for (int d = 0; d <= k; d++)
        for (int q = 0; q <= d; q++) {
            mono[nm][0] = d - q;
            mono[nm][1] = q;
            nm++;
        }
    double V[225], Cm[225];
    for (int i = 0; i < nl; i++) {
        double xi = (double)A[i][1] / k, eta = (double)A[i][2] / k;
        for (int m = 0; m < nm; m++) V[i * nm + m] = pow(xi, mono[m][0]) * pow(eta, mono[m][1]);
    }
    int rc = invert(nl, V, Cm);
    if (rc) return rc;
    int n = k + 1;
    double gx[8], gw[8];
    gauss_legendre01(n, gx, gw);
    for (int i = 0; i < nl * nl; i++) K[i] = 0.0;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            double xi = gx[a] * (1.0 - gx[b]), eta = gx[b];
            double wq = gw[a] * gw[b] * (1.0 - gx[b]) * det;
            double dm[15][2], grad[15][2];
            for (int m = 0; m < nm; m++) {
                int p = mono[m][0], q = mono[m][1];
                dm[m][0] = p ? p * pow(xi, p - 1) * pow(eta, q) : 0.0;
                dm[m][1] = q ? q * pow(xi, p) * pow(eta, q - 1) : 0.0;
            }
            for (int j = 0; j < nl; j++) {
                double dxi = 0.0, deta = 0.0;
                for (int m = 0; m < nm; m++) {
                    dxi += Cm[m * nl + j] * dm[m][0];
                    deta += Cm[m * nl + j] * dm[m][1];
                }
                /* grad lambda_1 = grad xi, grad lambda_2 = grad eta */
                for (int r = 0; r < 2; r++) grad[j][r] = dxi * G[1 * 2 + r] + deta * G[2 * 2 + r];
            }
            for (int i = 0; i < nl; i++)
                for (int j = 0; j < nl; j++)
                    K[i * nl + j] += wq * (grad[i][0] * grad[j][0] + grad[i][1] * grad[j][1]);
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* the assembled system                                                       */
/* ------------------------------------------------------------------------- */

typedef struct {
    int dim, order;
    int64_t nverts, ncells, nedges, ndofs, nfree;
    int nloc;
    int32_t *cell_dofs;  /* [ncells][nloc] global DOF of each local DOF */
    double *dof_coords;  /* [ndofs][dim] */
    uint8_t *dirichlet;  /* [ndofs] */
    int64_t *dof2free;   /* [ndofs], -1 on Dirichlet DOFs */
    int64_t *free2dof;   /* [nfree] */
    /* full stiffness K (structural pattern) */
    int64_t nnz;
    int64_t *rowptr;
    int32_t *col;
    double *val;
    /* A = K_II in free numbering */
    int64_t a_nnz;
    int64_t *a_rowptr;
    int32_t *a_col;
    double *a_val;
    double *a_diag;
    int64_t n_bad_cells;
} orc_system;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct { int32_t v[3]; } face3;
static int cmp_face(const void *a, const void *b)
{
    const face3 *x = a, *y = b;
    for (int i = 0; i < 3; i++) {
        if (x->v[i] < y->v[i]) return -1;
        if (x->v[i] > y->v[i]) return 1;
    }
    return 0;
}

static int64_t find_key(const int64_t *keys, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (keys[mid] == key) return mid;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

void orc_free(orc_system *s)
{
    if (!s) return;
    free(s->cell_dofs);
    free(s->dof_coords);
    free(s->dirichlet);
    free(s->dof2free);
    free(s->free2dof);
    free(s->rowptr);
    free(s->col);
    free(s->val);
    free(s->a_rowptr);
    free(s->a_col);
    free(s->a_val);
    free(s->a_diag);
    free(s);
}

static void sort3(int32_t *a)
{
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (a[j] < a[i]) { int32_t t = a[i]; a[i] = a[j]; a[j] = t; }
}

/* Build DOFs, element matrices, K and the lifted A.  *err receives a code. */
orc_system *orc_build(int dim, int64_t nverts, const double *coords, int64_t ncells,
                      const int32_t *cells, const uint8_t *on_boundary, int order, int *err)
{
    *err = 0;
    if ((dim != 2 && dim != 3) || order < 1 || order > 4 || (order > 2 && dim != 2) || nverts <= 0 ||
        ncells <= 0) {
        *err = ORC_EINVAL;
        return NULL;
    }
    orc_system *s = calloc(1, sizeof(orc_system));
    if (!s) { *err = ORC_ENOMEM; return NULL; }
    s->dim = dim;
    s->order = order;
    s->nverts = nverts;
    s->ncells = ncells;
    int nv = dim + 1;
    int ne_loc = dim == 2 ? 3 : 6;
    s->nloc = order == 1 ? nv : (order == 2 ? nv + ne_loc : (order + 1) * (order + 2) / 2);
    int nloc = s->nloc;
    int ke = order - 1;                          /* DOFs per edge */
    int ci = (order - 1) * (order - 2) / 2;      /* DOFs inside a cell */

    /* ---- DOFs ---- */
    int64_t *ekeys = NULL, *uniq = NULL;
    int64_t nek = 0, nuniq = 0;
    if (order >= 2) {
        int E[6][2];
        p2_local_edges(dim, E);
        nek = ncells * ne_loc;
        ekeys = malloc(sizeof(int64_t) * nek);
        if (!ekeys) goto nomem;
        for (int64_t c = 0; c < ncells; c++)
            for (int e = 0; e < ne_loc; e++) {
                int64_t a = cells[c * nv + E[e][0]], b = cells[c * nv + E[e][1]];
                int64_t lo = a < b ? a : b, hi = a < b ? b : a;
                ekeys[c * ne_loc + e] = lo * nverts + hi;
            }
        uniq = malloc(sizeof(int64_t) * nek);
        if (!uniq) goto nomem;
        memcpy(uniq, ekeys, sizeof(int64_t) * nek);
        qsort(uniq, nek, sizeof(int64_t), cmp_i64);
        for (int64_t i = 0; i < nek; i++)
            if (i == 0 || uniq[i] != uniq[i - 1]) uniq[nuniq++] = uniq[i];
        s->nedges = nuniq;
    }
    s->ndofs = nverts + ke * s->nedges + ci * ncells;
    s->dof_coords = malloc(sizeof(double) * s->ndofs * dim);
    s->dirichlet = calloc(s->ndofs, 1);
    s->cell_dofs = malloc(sizeof(int32_t) * ncells * nloc);
    if (!s->dof_coords || !s->dirichlet || !s->cell_dofs) goto nomem;
    memcpy(s->dof_coords, coords, sizeof(double) * nverts * dim);
    for (int64_t v = 0; v < nverts; v++) s->dirichlet[v] = on_boundary[v] ? 1 : 0;
    for (int64_t e = 0; e < s->nedges; e++) {
        int64_t a = uniq[e] / nverts, b = uniq[e] % nverts;
        for (int r = 0; r < dim; r++) {
            if (order == 2) {
                s->dof_coords[(nverts + e) * dim + r] = 0.5 * (coords[a * dim + r] + coords[b * dim + r]);
            } else {
                for (int t = 1; t <= ke; t++)
                    s->dof_coords[(nverts + ke * e + t - 1) * dim + r] =
                        ((order - t) * coords[a * dim + r] + t * coords[b * dim + r]) / order;
            }
        }
    }
    if (order <= 2) {
        for (int64_t c = 0; c < ncells; c++) {
            for (int i = 0; i < nv; i++) s->cell_dofs[c * nloc + i] = cells[c * nv + i];
            if (order == 2)
                for (int e = 0; e < ne_loc; e++) {
                    int64_t idx = find_key(uniq, nuniq, ekeys[c * ne_loc + e]);
                    s->cell_dofs[c * nloc + nv + e] = (int32_t)(nverts + idx);
                }
        }
    } else {
        /* P3/P4 triangles: classify each local lattice point */
        int A[15][3];
        pk_local_points(order, A);
        int inter[3][3], ninter = 0; /* interior indices, decreasing lexicographic order */
        for (int a0 = order; a0 >= 0; a0--)
            for (int a1 = order - a0; a1 >= 0; a1--) {
                int a2 = order - a0 - a1;
                if (a0 > 0 && a1 > 0 && a2 > 0) {
                    inter[ninter][0] = a0;
                    inter[ninter][1] = a1;
                    inter[ninter][2] = a2;
                    ninter++;
                }
            }
        int64_t ibase = nverts + ke * s->nedges;
        for (int64_t c = 0; c < ncells; c++) {
            const int32_t *cv = cells + c * 3;
            for (int i = 0; i < nloc; i++) {
                int nz = 0, m0 = -1;
                for (int m = 0; m < 3; m++)
                    if (A[i][m] == 0) nz++;
                    else if (m0 < 0) m0 = m;
                int64_t g;
                if (nz == 2) {
                    g = cv[m0];  /* vertex m0 */
                } else if (nz == 1) {
                    int p = -1, q = -1;
                    for (int m = 0; m < 3; m++)
                        if (A[i][m] > 0) { if (p < 0) p = m; else q = m; }
                    int64_t gp = cv[p], gq = cv[q];
                    int64_t lo = gp < gq ? gp : gq, hi = gp < gq ? gq : gp;
                    int t = gp > gq ? A[i][p] : A[i][q];  /* weight of the larger vertex */
                    int64_t idx = find_key(uniq, nuniq, lo * nverts + hi);
                    g = nverts + ke * idx + (t - 1);
                } else {
                    int r = 0;
                    while (!(inter[r][0] == A[i][0] && inter[r][1] == A[i][1] && inter[r][2] == A[i][2])) r++;
                    g = ibase + ci * c + r;
                    for (int d = 0; d < dim; d++)
                        s->dof_coords[g * dim + d] = ((double)A[i][0] * coords[(int64_t)cv[0] * dim + d] +
                                                      (double)A[i][1] * coords[(int64_t)cv[1] * dim + d] +
                                                      (double)A[i][2] * coords[(int64_t)cv[2] * dim + d]) / order;
                }
                s->cell_dofs[c * nloc + i] = (int32_t)g;
            }
        }
    }
    /* Dirichlet edges: edges of boundary facets (facets in exactly one cell)
     * whose two vertices are flagged (all k-1 DOFs of such an edge) */
    if (order >= 2) {
        if (dim == 2) {
            /* facets are edges: count occurrences in the sorted key list */
            int64_t *cnt = calloc(nuniq, sizeof(int64_t));
            if (!cnt) goto nomem;
            for (int64_t i = 0; i < nek; i++) cnt[find_key(uniq, nuniq, ekeys[i])]++;
            for (int64_t e = 0; e < nuniq; e++) {
                int64_t a = uniq[e] / nverts, b = uniq[e] % nverts;
                if (cnt[e] == 1 && on_boundary[a] && on_boundary[b])
                    for (int t = 0; t < ke; t++) s->dirichlet[nverts + ke * e + t] = 1;
            }
            free(cnt);
        } else {
            int64_t nf = ncells * 4;
            face3 *f = malloc(sizeof(face3) * nf);
            if (!f) goto nomem;
            for (int64_t c = 0; c < ncells; c++)
                for (int o = 0; o < 4; o++) {
                    int q = 0;
                    for (int t = 0; t < 4; t++)
                        if (t != o) f[c * 4 + o].v[q++] = cells[c * 4 + t];
                    sort3(f[c * 4 + o].v);
                }
            qsort(f, nf, sizeof(face3), cmp_face);
            for (int64_t i = 0; i < nf;) {
                int64_t j = i;
                while (j < nf && cmp_face(&f[i], &f[j]) == 0) j++;
                if (j - i == 1) {
                    const int32_t *v = f[i].v;
                    if (on_boundary[v[0]] && on_boundary[v[1]] && on_boundary[v[2]]) {
                        int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
                        for (int p = 0; p < 3; p++) {
                            int64_t key = (int64_t)v[pr[p][0]] * nverts + v[pr[p][1]];
                            int64_t idx = find_key(uniq, nuniq, key);
                            s->dirichlet[nverts + idx] = 1;
                        }
                    }
                }
                i = j;
            }
            free(f);
        }
    }
    free(ekeys);
    ekeys = NULL;
    free(uniq);
    uniq = NULL;

    /* ---- element matrices into coordinate triplets ---- */
    {
        int64_t ncoo = ncells * (int64_t)nloc * nloc;
        int32_t *ri = malloc(sizeof(int32_t) * ncoo);
        int32_t *ci = malloc(sizeof(int32_t) * ncoo);
        double *vv = malloc(sizeof(double) * ncoo);
        if (!ri || !ci || !vv) { free(ri); free(ci); free(vv); goto nomem; }
        double Ke[225], X[4 * 3];
        for (int64_t c = 0; c < ncells; c++) {
            for (int i = 0; i < nv; i++)
                for (int r = 0; r < dim; r++) X[i * dim + r] = coords[(int64_t)cells[c * nv + i] * dim + r];
            int rc = order == 1 ? orc_p1_element(dim, X, Ke)
                   : (order == 2 ? orc_p2_element(dim, X, Ke) : orc_pk_element(order, X, Ke));
            if (rc) { s->n_bad_cells++; continue; }
            for (int i = 0; i < nloc; i++)
                for (int j = 0; j < nloc; j++) {
                    int64_t t = (c * nloc + i) * nloc + j;
                    ri[t] = s->cell_dofs[c * nloc + i];
                    ci[t] = s->cell_dofs[c * nloc + j];
                    vv[t] = Ke[i * nloc + j];
                }
        }
        if (s->n_bad_cells) {
            free(ri); free(ci); free(vv);
            *err = ORC_EMESH;
            orc_free(s);
            return NULL;
        }
        /* stable counting sort by column, then by row: triplets end up
         * ordered by (row, col, element order) */
        int64_t n = s->ndofs;
        int64_t *cnt = calloc(n + 1, sizeof(int64_t));
        int32_t *r2 = malloc(sizeof(int32_t) * ncoo);
        int32_t *c2 = malloc(sizeof(int32_t) * ncoo);
        double *v2 = malloc(sizeof(double) * ncoo);
        if (!cnt || !r2 || !c2 || !v2) {
            free(ri); free(ci); free(vv); free(cnt); free(r2); free(c2); free(v2);
            goto nomem;
        }
        for (int64_t t = 0; t < ncoo; t++) cnt[ci[t] + 1]++;
        for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
        for (int64_t t = 0; t < ncoo; t++) {
            int64_t d = cnt[ci[t]]++;
            r2[d] = ri[t]; c2[d] = ci[t]; v2[d] = vv[t];
        }
        memset(cnt, 0, sizeof(int64_t) * (n + 1));
        for (int64_t t = 0; t < ncoo; t++) cnt[r2[t] + 1]++;
        for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
        for (int64_t t = 0; t < ncoo; t++) {
            int64_t d = cnt[r2[t]]++;
            ri[d] = r2[t]; ci[d] = c2[t]; vv[d] = v2[t];
        }
        free(r2); free(c2); free(v2); free(cnt);
        /* sum duplicates */
        s->rowptr = calloc(n + 1, sizeof(int64_t));
        int64_t nnz = 0;
        for (int64_t t = 0; t < ncoo; t++)
            if (t == 0 || ri[t] != ri[t - 1] || ci[t] != ci[t - 1]) nnz++;
        s->col = malloc(sizeof(int32_t) * nnz);
        s->val = malloc(sizeof(double) * nnz);
        if (!s->rowptr || !s->col || !s->val) { free(ri); free(ci); free(vv); goto nomem; }
        int64_t w = -1;
        for (int64_t t = 0; t < ncoo; t++) {
            if (t == 0 || ri[t] != ri[t - 1] || ci[t] != ci[t - 1]) {
                w++;
                s->col[w] = ci[t];
                s->val[w] = vv[t];
                s->rowptr[ri[t] + 1]++;
            } else {
                s->val[w] += vv[t];
            }
        }
        for (int64_t i = 0; i < n; i++) s->rowptr[i + 1] += s->rowptr[i];
        s->nnz = nnz;
        free(ri); free(ci); free(vv);
    }

    /* ---- lifting: A = K_II ---- */
    {
        int64_t n = s->ndofs;
        s->dof2free = malloc(sizeof(int64_t) * n);
        if (!s->dof2free) goto nomem;
        int64_t nf = 0;
        for (int64_t d = 0; d < n; d++) s->dof2free[d] = s->dirichlet[d] ? -1 : nf++;
        s->nfree = nf;
        s->free2dof = malloc(sizeof(int64_t) * (nf ? nf : 1));
        s->a_rowptr = calloc(nf + 1, sizeof(int64_t));
        s->a_diag = calloc(nf ? nf : 1, sizeof(double));
        if (!s->free2dof || !s->a_rowptr || !s->a_diag) goto nomem;
        for (int64_t d = 0; d < n; d++)
            if (s->dof2free[d] >= 0) s->free2dof[s->dof2free[d]] = d;
        int64_t annz = 0;
        for (int64_t f = 0; f < nf; f++) {
            int64_t d = s->free2dof[f];
            for (int64_t t = s->rowptr[d]; t < s->rowptr[d + 1]; t++)
                if (s->dof2free[s->col[t]] >= 0) annz++;
            s->a_rowptr[f + 1] = annz;
        }
        s->a_col = malloc(sizeof(int32_t) * (annz ? annz : 1));
        s->a_val = malloc(sizeof(double) * (annz ? annz : 1));
        if (!s->a_col || !s->a_val) goto nomem;
        int64_t w = 0;
        for (int64_t f = 0; f < nf; f++) {
            int64_t d = s->free2dof[f];
            for (int64_t t = s->rowptr[d]; t < s->rowptr[d + 1]; t++) {
                int64_t cf = s->dof2free[s->col[t]];
                if (cf >= 0) {
                    s->a_col[w] = (int32_t)cf;
                    s->a_val[w] = s->val[t];
                    if (cf == f) s->a_diag[f] = s->val[t];
                    w++;
                }
            }
        }
        s->a_nnz = annz;
    }
    return s;
nomem:
    free(ekeys);
    free(uniq);
    orc_free(s);
    *err = ORC_ENOMEM;
    return NULL;
}

/* sizes: ndofs, nedges, nfree, nnz(K), nnz(A), nloc */
int orc_sizes(const orc_system *s, int64_t *out)
{
    out[0] = s->ndofs;
    out[1] = s->nedges;
    out[2] = s->nfree;
    out[3] = s->nnz;
    out[4] = s->a_nnz;
    out[5] = s->nloc;
    return 0;
}

int orc_copy_dofs(const orc_system *s, double *coords, uint8_t *dirichlet, int64_t *free2dof)
{
    if (coords) memcpy(coords, s->dof_coords, sizeof(double) * s->ndofs * s->dim);
    if (dirichlet) memcpy(dirichlet, s->dirichlet, s->ndofs);
    if (free2dof) memcpy(free2dof, s->free2dof, sizeof(int64_t) * s->nfree);
    return 0;
}

int orc_copy_K(const orc_system *s, int64_t *rowptr, int32_t *col, double *val)
{
    memcpy(rowptr, s->rowptr, sizeof(int64_t) * (s->ndofs + 1));
    memcpy(col, s->col, sizeof(int32_t) * s->nnz);
    memcpy(val, s->val, sizeof(double) * s->nnz);
    return 0;
}

int orc_copy_A(const orc_system *s, int64_t *rowptr, int32_t *col, double *val)
{
    memcpy(rowptr, s->a_rowptr, sizeof(int64_t) * (s->nfree + 1));
    memcpy(col, s->a_col, sizeof(int32_t) * s->a_nnz);
    memcpy(val, s->a_val, sizeof(double) * s->a_nnz);
    return 0;
}

/* b = -K_ID g_D for k columns; g is [ndofs][k], B is [nfree][k]. */
int orc_rhs(const orc_system *s, const double *g, int k, double *B)
{
    if (k <= 0) return ORC_EINVAL;
    for (int64_t f = 0; f < s->nfree; f++) {
        int64_t d = s->free2dof[f];
        for (int j = 0; j < k; j++) {
            double acc = 0.0;
            for (int64_t t = s->rowptr[d]; t < s->rowptr[d + 1]; t++) {
                int32_t c = s->col[t];
                if (s->dirichlet[c]) acc += s->val[t] * g[(int64_t)c * k + j];
            }
            B[f * k + j] = -acc;
        }
    }
    return 0;
}

/* y = A x for k interleaved columns ([nfree][k]) */
int orc_spmv(const orc_system *s, const double *x, int k, double *y)
{
    for (int64_t i = 0; i < s->nfree; i++)
        for (int j = 0; j < k; j++) {
            double acc = 0.0;
            for (int64_t t = s->a_rowptr[i]; t < s->a_rowptr[i + 1]; t++)
                acc += s->a_val[t] * x[(int64_t)s->a_col[t] * k + j];
            y[i * k + j] = acc;
        }
    return 0;
}

/* ---- single-column kernels of the PCG ---- */

typedef struct {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *diag;
} csr_view;

static csr_view view_A(const orc_system *s)
{
    csr_view v = {s->nfree, s->a_rowptr, s->a_col, s->a_val, s->a_diag};
    return v;
}

static void spmv1(const csr_view *A, const double *x, double *y)
{
    for (int64_t i = 0; i < A->n; i++) {
        double acc = 0.0;
        for (int64_t t = A->rowptr[i]; t < A->rowptr[i + 1]; t++)
            acc += A->val[t] * x[A->col[t]];
        y[i] = acc;
    }
}

static double dot1(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* Eq. (2) for k interleaved columns: relres[j] = ||b_j - A x_j|| / ||b_j||
 * (0 when b_j = 0 and x_j = 0). */
int orc_relres(const orc_system *s, const double *B, const double *X, int k, double *relres)
{
    int64_t n = s->nfree;
    double *x = malloc(sizeof(double) * (n ? n : 1));
    double *ax = malloc(sizeof(double) * (n ? n : 1));
    if (!x || !ax) { free(x); free(ax); return ORC_ENOMEM; }
    csr_view A = view_A(s);
    for (int j = 0; j < k; j++) {
        for (int64_t i = 0; i < n; i++) x[i] = X[i * k + j];
        spmv1(&A, x, ax);
        double rr = 0.0, bb = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double b = B[i * k + j], r = b - ax[i];
            rr += r * r;
            bb += b * b;
        }
        relres[j] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
    }
    free(x);
    free(ax);
    return 0;
}

/* Jacobi-PCG for column j of B (Sect. 2.1 with M = diag(A); exit test
 * Eq. (2)), zero initial guess; w holds 6 work vectors of n doubles.
 * iters[j] = number of products A p; relres[j] = true residual of Eq. (2);
 * restarts[j] = restarts after a drifted recursive residual.
 * Returns 0, or 1 if the column misses Eq. (2) (iteration cap or last
 * restart), or ORC_EBREAK on p.Ap <= 0. */
static int pcg_column(const csr_view *A, const double *B, int k, int j, double tol, int64_t max_iter,
                      double *w, double *X, int64_t *iters, double *relres, int32_t *restarts)
{
    int64_t n = A->n;
    int status = 0;
    size_t stride = (size_t)(n ? n : 1);
    double *b = w, *x = w + stride, *r = w + 2 * stride, *z = w + 3 * stride;
    double *p = w + 4 * stride, *q = w + 5 * stride;
    for (int64_t i = 0; i < n; i++) b[i] = B[i * k + j];
    double bnorm = sqrt(dot1(n, b, b));
    int64_t its = 0;
    int rs = 0;
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    if (bnorm == 0.0) {
        iters[j] = 0;
        relres[j] = 0.0;
        if (restarts) restarts[j] = 0;
        for (int64_t i = 0; i < n; i++) X[i * k + j] = 0.0;
        return 0;
    }
    double rel = 0.0;
    for (;;) {
        /* (re)start from x: r = b - A x, z = D^-1 r, p = z */
        spmv1(A, x, q);
        for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
        for (int64_t i = 0; i < n; i++) z[i] = r[i] / A->diag[i];
        for (int64_t i = 0; i < n; i++) p[i] = z[i];
        double rho = dot1(n, r, z);
        double rnorm = sqrt(dot1(n, r, r));
        while (rnorm > tol * bnorm && its < max_iter) {
            spmv1(A, p, q);
            double pq = dot1(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) {
                status = ORC_EBREAK;
                break;
            }
            double alpha = rho / pq;
            for (int64_t i = 0; i < n; i++) x[i] += alpha * p[i];
            for (int64_t i = 0; i < n; i++) r[i] -= alpha * q[i];
            its++;
            rnorm = sqrt(dot1(n, r, r));
            if (rnorm <= tol * bnorm) break;
            for (int64_t i = 0; i < n; i++) z[i] = r[i] / A->diag[i];
            double rho_new = dot1(n, r, z);
            double beta = rho_new / rho;
            rho = rho_new;
            for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
        /* true residual */
        spmv1(A, x, q);
        double rr = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double t = b[i] - q[i];
            rr += t * t;
        }
        rel = sqrt(rr) / bnorm;
        if (status == ORC_EBREAK || rel <= tol || its >= max_iter || rs >= 3) break;
        rs++;
    }
    /* Eq. (2) not met, either at the iteration cap or after the last
     * allowed restart: a warning, not success */
    if (rel > tol && status == 0) status = 1;
    iters[j] = its;
    relres[j] = rel;
    if (restarts) restarts[j] = rs;
    for (int64_t i = 0; i < n; i++) X[i * k + j] = x[i];
    return status;
}

/* Jacobi-PCG on the k columns of B, [nfree][k] (X is overwritten, zero
 * initial guess).  The columns are independent solves (Sect. 4.3: an
 * iterative solver treats each right-hand side on its own).  The default
 * build runs them one after another.  Built with -fopenmp (the CPU-baseline
 * timing build only) the columns run on separate threads; each column's
 * arithmetic is the same, so the results are identical.
 * Returns ORC_EBREAK if any column broke down, else 1 if any column missed
 * Eq. (2), else 0. */
static int pcg_csr(const csr_view *A, const double *B, int k, double tol, int64_t max_iter,
                   double *X, int64_t *iters, double *relres, int32_t *restarts)
{
    size_t stride = (size_t)(A->n ? A->n : 1);
    int worst = 0, broke = 0, nomem = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst) reduction(| : broke, nomem)
#endif
    for (int j = 0; j < k; j++) {
        double *w = malloc(sizeof(double) * 6 * stride);
        if (!w) {
            nomem = 1;
            continue;
        }
        int st = pcg_column(A, B, k, j, tol, max_iter, w, X, iters, relres, restarts);
        free(w);
        if (st == ORC_EBREAK) broke = 1;
        else if (st > worst) worst = st;
    }
    if (nomem) return ORC_ENOMEM;
    return broke ? ORC_EBREAK : worst;
}

int orc_pcg(const orc_system *s, const double *B, int k, double tol, int64_t max_iter,
            double *X, int64_t *iters, double *relres, int32_t *restarts)
{
    csr_view A = view_A(s);
    return pcg_csr(&A, B, k, tol, max_iter, X, iters, relres, restarts);
}

/* Threads that pcg_csr runs columns on: 1 in the default build; in the
 * -fopenmp timing build, `want` (if positive) becomes the thread count. */
int orc_threads(int want)
{
#ifdef _OPENMP
    if (want > 0) omp_set_num_threads(want);
    return omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

/* The same PCG on a caller-given CSR matrix (used by tests that plant a
 * defect, e.g. an indefinite matrix, into an oracle-built system). */
int orc_pcg_csr(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                const double *B, int k, double tol, int64_t max_iter, double *X, int64_t *iters,
                double *relres, int32_t *restarts)
{
    double *diag = malloc(sizeof(double) * (n ? n : 1));
    if (!diag) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++) {
        diag[i] = 0.0;
        for (int64_t t = rowptr[i]; t < rowptr[i + 1]; t++)
            if (col[t] == i) diag[i] = val[t];
    }
    csr_view A = {n, rowptr, col, val, diag};
    int rc = pcg_csr(&A, B, k, tol, max_iter, X, iters, relres, restarts);
    free(diag);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* BiCGStab with a Block-Jacobi preconditioner                                */
/* ------------------------------------------------------------------------- */

/* The paper's iterative solver is BiCGStab with a Block-Jacobi
 * preconditioner (Sect. 3.2).  Blocks here: the consecutive rows
 * [b bs, min(n, (b+1) bs)) of the matrix, the last one possibly shorter; the
 * block systems are solved exactly, by a dense LU factorisation with partial
 * pivoting of each diagonal block (taken once per solve), then two
 * triangular solves per application.  bs = 1 is the Jacobi preconditioner. */
typedef struct {
    int64_t n, nb;
    int bs;
    double *lu;    /* [nb][bs][bs] row-major LU factors (unit lower implied) */
    int32_t *piv;  /* [nb][bs] row interchanges */
} bj_fact;

static void bj_free(bj_fact *F)
{
    free(F->lu);
    free(F->piv);
}

static int bj_factor(const csr_view *A, int bs, bj_fact *F)
{
    int64_t n = A->n;
    F->n = n;
    F->bs = bs;
    F->nb = (n + bs - 1) / bs;
    F->lu = calloc((size_t)(F->nb ? F->nb : 1) * bs * bs, sizeof(double));
    F->piv = calloc((size_t)(F->nb ? F->nb : 1) * bs, sizeof(int32_t));
    if (!F->lu || !F->piv) { bj_free(F); return ORC_ENOMEM; }
    for (int64_t b = 0; b < F->nb; b++) {
        int64_t r0 = b * bs;
        int m = (int)((r0 + bs <= n) ? bs : n - r0);
        double *M = F->lu + (size_t)b * bs * bs;
        int32_t *pv = F->piv + (size_t)b * bs;
        for (int i = 0; i < m; i++)
            for (int64_t t = A->rowptr[r0 + i]; t < A->rowptr[r0 + i + 1]; t++) {
                int64_t c = A->col[t];
                if (c >= r0 && c < r0 + m) M[i * bs + (c - r0)] += A->val[t];
            }
        for (int c = 0; c < m; c++) {
            int p = c;
            for (int r = c + 1; r < m; r++)
                if (fabs(M[r * bs + c]) > fabs(M[p * bs + c])) p = r;
            if (M[p * bs + c] == 0.0) { bj_free(F); return ORC_EBREAK; }
            pv[c] = p;
            if (p != c)
                for (int j = 0; j < m; j++) {
                    double t = M[c * bs + j]; M[c * bs + j] = M[p * bs + j]; M[p * bs + j] = t;
                }
            for (int r = c + 1; r < m; r++) {
                double l = M[r * bs + c] / M[c * bs + c];
                M[r * bs + c] = l;
                for (int j = c + 1; j < m; j++) M[r * bs + j] -= l * M[c * bs + j];
            }
        }
    }
    return 0;
}

/* z = M^-1 r, block by block: permute, forward (unit lower), backward */
static void bj_apply(const bj_fact *F, const double *r, double *z)
{
    int bs = F->bs;
    for (int64_t b = 0; b < F->nb; b++) {
        int64_t r0 = b * bs;
        int m = (int)((r0 + bs <= F->n) ? bs : F->n - r0);
        const double *M = F->lu + (size_t)b * bs * bs;
        const int32_t *pv = F->piv + (size_t)b * bs;
        double y[64];
        for (int i = 0; i < m; i++) y[i] = r[r0 + i];
        for (int c = 0; c < m; c++)
            if (pv[c] != c) { double t = y[c]; y[c] = y[pv[c]]; y[pv[c]] = t; }
        for (int i = 0; i < m; i++)
            for (int j = 0; j < i; j++) y[i] -= M[i * bs + j] * y[j];
        for (int i = m - 1; i >= 0; i--) {
            for (int j = i + 1; j < m; j++) y[i] -= M[i * bs + j] * y[j];
            y[i] /= M[i * bs + i];
        }
        for (int i = 0; i < m; i++) z[r0 + i] = y[i];
    }
}

/* z = M^-1 r for a caller-given CSR matrix (bs <= 64) */
int orc_bj_apply(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int bs,
                 const double *r, double *z)
{
    if (bs < 1 || bs > 64) return ORC_EINVAL;
    csr_view A = {n, rowptr, col, val, NULL};
    bj_fact F;
    int rc = bj_factor(&A, bs, &F);
    if (rc) return rc;
    bj_apply(&F, r, z);
    bj_free(&F);
    return 0;
}

/* BiCGStab (van der Vorst), right preconditioned by M, zero initial guess,
 * one right-hand side:
 *   r = b - A x, rh = r;  rho_old = alpha = omega = 1;  v = p = 0
 *   repeat:  rho = (rh, r);  beta = (rho / rho_old)(alpha / omega)
 *            p = r + beta (p - omega v);  ph = M^-1 p;  v = A ph
 *            alpha = rho / (rh, v);  s = r - alpha v
 *            if ||s|| <= tol ||b||:  x += alpha ph, r = s, stop
 *            sh = M^-1 s;  t = A sh;  omega = (t, s) / (t, t)
 *            x += alpha ph + omega sh;  r = s - omega t;  rho_old = rho
 * until ||r|| <= tol ||b|| (the Eq. (2) test on the recursive residual),
 * then the true residual ||b - A x|| / ||b||, restarting from x when it is
 * above tol (at most 3 times).  One iteration = one pass of the loop (two
 * products with A, one when it stops at s).  A Lanczos near-breakdown,
 * |rho| <= 1e-14 ||rh|| ||r|| (rho = 0 included), restarts the iteration
 * from x with rh = r (at most 100 times): with zero source the lifted b,
 * hence rh, lives on the rows next to the boundary only, and rho then decays
 * far faster than r.  (rh, v) = 0, omega = 0 or a non-finite scalar is a
 * breakdown. */
int orc_bicgstab_csr(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                     const double *bvec, int bs, double tol, int64_t max_iter, double *xout,
                     int64_t *iters, double *relres, int32_t *restarts)
{
    if (bs < 1 || bs > 64 || n < 0) return ORC_EINVAL;
    csr_view A = {n, rowptr, col, val, NULL};
    bj_fact F;
    int rc = bj_factor(&A, bs, &F);
    if (rc) return rc;
    size_t bytes = sizeof(double) * (n ? n : 1);
    double *x = calloc(n ? n : 1, sizeof(double)), *r = malloc(bytes), *rh = malloc(bytes);
    double *p = malloc(bytes), *ph = malloc(bytes), *v = malloc(bytes), *sv = malloc(bytes);
    double *sh = malloc(bytes), *t = malloc(bytes);
    int status = 0;
    if (!x || !r || !rh || !p || !ph || !v || !sv || !sh || !t) { status = ORC_ENOMEM; goto done; }
    double bnorm = sqrt(dot1(n, bvec, bvec));
    int64_t its = 0;
    int rs = 0, soft = 0;
    double rel = 0.0;
    if (bnorm == 0.0) goto finish;
    for (;;) {
        spmv1(&A, x, t);
        for (int64_t i = 0; i < n; i++) {
            r[i] = bvec[i] - t[i];
            rh[i] = r[i];
            p[i] = v[i] = 0.0;
        }
        double rho_old = 1.0, alpha = 1.0, omega = 1.0;
        double rhrh = dot1(n, rh, rh);
        double rnorm = sqrt(dot1(n, r, r));
        int lanczos = 0;
        while (rnorm > tol * bnorm && its < max_iter) {
            double rho = dot1(n, rh, r);
            if (!isfinite(rho)) { status = ORC_EBREAK; break; }
            if (!(fabs(rho) > 1e-14 * sqrt(rhrh) * rnorm)) { lanczos = 1; break; }
            double beta = (rho / rho_old) * (alpha / omega);
            for (int64_t i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            bj_apply(&F, p, ph);
            spmv1(&A, ph, v);
            double sig = dot1(n, rh, v);
            if (sig == 0.0 || !isfinite(sig)) { status = ORC_EBREAK; break; }
            alpha = rho / sig;
            for (int64_t i = 0; i < n; i++) sv[i] = r[i] - alpha * v[i];
            its++;
            double snorm = sqrt(dot1(n, sv, sv));
            if (snorm <= tol * bnorm) {
                for (int64_t i = 0; i < n; i++) {
                    x[i] += alpha * ph[i];
                    r[i] = sv[i];
                }
                rnorm = snorm;
                break;
            }
            bj_apply(&F, sv, sh);
            spmv1(&A, sh, t);
            double tt = dot1(n, t, t), ts = dot1(n, t, sv);
            omega = ts / tt;
            if (omega == 0.0 || !isfinite(omega)) { status = ORC_EBREAK; break; }
            for (int64_t i = 0; i < n; i++) {
                x[i] += alpha * ph[i] + omega * sh[i];
                r[i] = sv[i] - omega * t[i];
            }
            rho_old = rho;
            rnorm = sqrt(dot1(n, r, r));
        }
        spmv1(&A, x, t);
        double rr = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double d = bvec[i] - t[i];
            rr += d * d;
        }
        rel = sqrt(rr) / bnorm;
        if (lanczos && status == 0) {
            if (soft >= 100 || its >= max_iter) { status = ORC_EBREAK; break; }
            soft++;
            continue;
        }
        if (status == ORC_EBREAK || rel <= tol || its >= max_iter || rs >= 3) break;
        rs++;
    }
    if (rel > tol && status == 0) status = 1;  /* cap or restarts spent: Eq. (2) not met */
finish:
    *iters = its;
    *relres = rel;
    if (restarts) *restarts = rs + soft;
    for (int64_t i = 0; i < n; i++) xout[i] = x[i];
done:
    free(x); free(r); free(rh); free(p); free(ph); free(v); free(sv); free(sh); free(t);
    bj_free(&F);
    return status;
}

/* Count of the nonzeros of the paper's regular-grid matrix read as a
 * 7-point finite-difference stencil (w(i,j) = 1, Sect. 2.2) on an m^3 grid
 * with one identity row per Dirichlet node (Table 1 row counts = m^3). */
int64_t orc_fd7_identity_nnz(int64_t m)
{
    int64_t nnz = 0;
    for (int64_t l = 0; l < m; l++)
        for (int64_t j = 0; j < m; j++)
            for (int64_t i = 0; i < m; i++) {
                int bnd = i == 0 || j == 0 || l == 0 || i == m - 1 || j == m - 1 || l == m - 1;
                if (bnd) {
                    nnz += 1;
                } else {
                    int nb = 0;
                    int64_t d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
                    for (int t = 0; t < 6; t++) {
                        int64_t a = i + d[t][0], b = j + d[t][1], c = l + d[t][2];
                        if (a >= 0 && a < m && b >= 0 && b < m && c >= 0 && c < m) nb++;
                    }
                    nnz += 1 + nb;
                }
            }
    return nnz;
}

/* Dense Cholesky (Sect. 4.3: a direct solver factorises the matrix once and
 * solves two triangular systems per right-hand side; A is symmetric
 * positive definite, so A = L L^T).  A given in CSR (n rows) is expanded to
 * a dense n x n array; L (row-major, lower triangle, zeros above) is written
 * to L_out when it is not NULL, and X = A^-1 B for the k columns of B
 * ([n][k]) when X is not NULL: forward substitution L y = b, then backward
 * substitution L^T x = y.  Returns 0, ORC_ENOMEM, or ORC_EBREAK when a pivot
 * is not positive (A not positive definite). */
int orc_dense_cholesky(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                       const double *B, int k, double *X, double *L_out)
{
    double *L = calloc((size_t)(n ? n : 1) * (size_t)(n ? n : 1), sizeof(double));
    if (!L) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++)
        for (int64_t t = rowptr[i]; t < rowptr[i + 1]; t++)
            if (col[t] <= i) L[i * n + col[t]] += val[t];
    /* column by column: L_jj = sqrt(a_jj - sum_m L_jm^2),
     * L_ij = (a_ij - sum_m L_im L_jm) / L_jj for i > j */
    for (int64_t j = 0; j < n; j++) {
        double d = L[j * n + j];
        for (int64_t m = 0; m < j; m++) d -= L[j * n + m] * L[j * n + m];
        if (!(d > 0.0)) {
            free(L);
            return ORC_EBREAK;
        }
        double ljj = sqrt(d);
        L[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; i++) {
            double s = L[i * n + j];
            for (int64_t m = 0; m < j; m++) s -= L[i * n + m] * L[j * n + m];
            L[i * n + j] = s / ljj;
        }
    }
    if (X) {
        for (int c = 0; c < k; c++) {
            for (int64_t i = 0; i < n; i++) {
                double s = B[i * k + c];
                for (int64_t m = 0; m < i; m++) s -= L[i * n + m] * X[m * k + c];
                X[i * k + c] = s / L[i * n + i];
            }
            for (int64_t i = n - 1; i >= 0; i--) {
                double s = X[i * k + c];
                for (int64_t m = i + 1; m < n; m++) s -= L[m * n + i] * X[m * k + c];
                X[i * k + c] = s / L[i * n + i];
            }
        }
    }
    if (L_out) memcpy(L_out, L, sizeof(double) * (size_t)n * (size_t)n);
    free(L);
    return 0;
}
