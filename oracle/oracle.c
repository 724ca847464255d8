/*
 * oracle.c -- plain, slow, single-threaded FP64 reference for the cell-loop
 * finite element assembly.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  The HIP library never
 * links, includes or calls it, and it shares no code, header or table with
 * the HIP library.
 *
 * What it computes is the plain definition of global assembly that the
 * paper's parallel loop reaches (PyOP2 "Parloops and kernels": a kernel is
 * applied to every cell with data gathered through Maps; "Access descriptors":
 * INC contributions are summed; "Matrix arguments": a Mat takes a row Map and
 * a column Map):
 *
 *   A[i][j] = sum over cells K containing nodes i and j of
 *             integral over K of ( cstiff * kappa grad(phi_j).grad(phi_i)
 *                                  + cmass * phi_j phi_i ) dx
 *   b[i]    = sum over cells K containing i of integral over K of f phi_i dx
 *   y       = sum over cells K of  P_K^T A_K P_K x      (matrix-free action)
 *
 * kappa and f are P1 fields (values on the mesh vertices, read through the
 * cell-to-vertex Map); the test/trial space is degree-k Lagrange (k = 1..3)
 * on triangles or tetrahedra, read through the cell-to-node Map.  The
 * coordinates are a P1 vector field (Firedrake layer, "The mesh
 * abstraction"), so cells are affine.
 *
 * Integration is done point by point at physical quadrature points with a
 * collapsed-coordinate (Stroud conical product) Gauss-Jacobi rule with q
 * points per direction, exact for polynomials of degree 2q-1.  Cells are
 * visited in index order and every sum is accumulated in that order.
 *
 * The oracle builds its own sparsity: for every row, the columns of every
 * cell incident to it, sorted and made unique (structural zeros kept).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 8
#define MAXLOC 20

/* ------------------------------------------------------------------ */
/* Jacobi polynomials and Gauss-Jacobi rules                            */
/* ------------------------------------------------------------------ */

/* P_n^{(a,b)}(x) by the three-term recurrence; also returns P_{n-1}. */
static double jacobi_p(int n, double a, double b, double x, double *pnm1)
{
    double p0 = 1.0, p1 = 0.5 * (a - b) + 0.5 * (a + b + 2.0) * x;
    if (n == 0) { if (pnm1) *pnm1 = 0.0; return p0; }
    for (int k = 2; k <= n; ++k) {
        double s = 2.0 * k + a + b;
        double c1 = 2.0 * k * (k + a + b) * (s - 2.0);
        double c2 = (s - 1.0) * (s * (s - 2.0) * x + a * a - b * b);
        double c3 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * s;
        double p2 = (c2 * p1 - c3 * p0) / c1;
        p0 = p1; p1 = p2;
    }
    if (pnm1) *pnm1 = p0;
    return p1;
}

/* d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)} */
static double jacobi_dp(int n, double a, double b, double x)
{
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x, NULL);
}

/*
 * n-point Gauss-Jacobi rule for the weight (1-t)^alpha on [0,1].
 * Roots of P_n^{(alpha,0)} on [-1,1] are bracketed on a fine grid, bisected,
 * then polished by Newton; weights from the classical closed form
 *   w = G(n+a+1)G(n+b+1) / (G(n+a+b+1) n!) * 2^(a+b+1) / ((1-x^2) P_n'(x)^2)
 * and mapped to [0,1] (scale 2^-(alpha+1)).
 */
int oracle_gauss_jacobi(int n, int alpha, double *t, double *w)
{
    if (n < 1 || n > MAXQ) return -1;
    const double a = alpha, b = 0.0;
    const int grid = 4000;
    int found = 0;
    double xl = -1.0, fl = jacobi_p(n, a, b, xl, NULL);
    double roots[MAXQ];
    for (int g = 1; g <= grid && found < n; ++g) {
        double xr = -1.0 + 2.0 * g / grid, fr = jacobi_p(n, a, b, xr, NULL);
        if (fl == 0.0) { roots[found++] = xl; }
        else if (fl * fr < 0.0) {
            double lo = xl, hi = xr, flo = fl;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), fm = jacobi_p(n, a, b, mid, NULL);
                if (flo * fm <= 0.0) hi = mid; else { lo = mid; flo = fm; }
            }
            double x = 0.5 * (lo + hi);
            for (int it = 0; it < 3; ++it) {
                double d = jacobi_dp(n, a, b, x);
                if (d != 0.0) x -= jacobi_p(n, a, b, x, NULL) / d;
            }
            roots[found++] = x;
        }
        xl = xr; fl = fr;
    }
    if (found != n) return -2;
    double lg = lgamma(n + a + 1.0) + lgamma(n + b + 1.0) - lgamma(n + a + b + 1.0) - lgamma(n + 1.0);
    double c = exp(lg) * pow(2.0, a + b + 1.0);
    for (int i = 0; i < n; ++i) {
        double x = roots[i], d = jacobi_dp(n, a, b, x);
        double wx = c / ((1.0 - x * x) * d * d);
        t[i] = 0.5 * (x + 1.0);
        w[i] = wx * pow(2.0, -(a + 1.0));
    }
    return 0;
}

/*
 * Collapsed-coordinate rule on the reference simplex (vertices 0, e_1..e_d):
 *   triangle: x = t1, y = (1-t1) t2                    weight (1-t1)
 *   tet:      x = t1, y = (1-t1) t2, z = (1-t1)(1-t2) t3 weight (1-t1)^2 (1-t2)
 * t1 ~ Gauss-Jacobi(alpha=d-1), t2 ~ Gauss-Jacobi(alpha=d-2), t3 ~ Gauss-Legendre.
 * Writes q^d points (reference coordinates) and weights; returns the count.
 */
int oracle_simplex_rule(int dim, int q, double *pts, double *wts)
{
    double t1[MAXQ], w1[MAXQ], t2[MAXQ], w2[MAXQ], t3[MAXQ], w3[MAXQ];
    if (dim == 1) {                      /* the segment [0, 1]: Gauss-Legendre */
        if (oracle_gauss_jacobi(q, 0, t1, w1)) return -1;
        for (int a = 0; a < q; ++a) { pts[a] = t1[a]; wts[a] = w1[a]; }
        return q;
    }
    if (dim == 2) {
        if (oracle_gauss_jacobi(q, 1, t1, w1) || oracle_gauss_jacobi(q, 0, t2, w2)) return -1;
        int k = 0;
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
                pts[2 * k + 0] = t1[a];
                pts[2 * k + 1] = (1.0 - t1[a]) * t2[b];
                wts[k] = w1[a] * w2[b];
                ++k;
            }
        return k;
    }
    if (dim == 3) {
        if (oracle_gauss_jacobi(q, 2, t1, w1) || oracle_gauss_jacobi(q, 1, t2, w2) ||
            oracle_gauss_jacobi(q, 0, t3, w3)) return -1;
        int k = 0;
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int c = 0; c < q; ++c) {
                    pts[3 * k + 0] = t1[a];
                    pts[3 * k + 1] = (1.0 - t1[a]) * t2[b];
                    pts[3 * k + 2] = (1.0 - t1[a]) * (1.0 - t2[b]) * t3[c];
                    wts[k] = w1[a] * w2[b] * w3[c];
                    ++k;
                }
        return k;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Lagrange bases in barycentric coordinates                           */
/* ------------------------------------------------------------------ */

int oracle_nloc(int dim, int degree)
{
    if (dim == 1) return degree >= 1 && degree <= 3 ? degree + 1 : -1;
    if (dim == 2) return degree == 1 ? 3 : degree == 2 ? 6 : degree == 3 ? 10 : -1;
    if (dim == 3) return degree == 1 ? 4 : degree == 2 ? 10 : degree == 3 ? 20 : -1;
    return -1;
}

/*
 * phi[i] and dphi[i][m] = d phi_i / d lambda_m at barycentric point lam
 * (nv = dim+1 barycentrics).  Local order: vertices; edges (a<b,
 * lexicographic), two nodes per edge at P3 ordered from a; tet faces (a<b<c,
 * lexicographic) or the triangle's interior node at P3.
 */
void oracle_basis(int dim, int degree, const double *lam, double *phi, double *dphi)
{
    const int nv = dim + 1;
    int n = oracle_nloc(dim, degree);
    memset(dphi, 0, sizeof(double) * (size_t)n * nv);
    int k = 0;
    for (int i = 0; i < nv; ++i, ++k) {
        double l = lam[i];
        if (degree == 1) { phi[k] = l; dphi[k * nv + i] = 1.0; }
        else if (degree == 2) { phi[k] = l * (2.0 * l - 1.0); dphi[k * nv + i] = 4.0 * l - 1.0; }
        else { phi[k] = 0.5 * l * (3.0 * l - 1.0) * (3.0 * l - 2.0);
               dphi[k * nv + i] = 0.5 * (27.0 * l * l - 18.0 * l + 2.0); }
    }
    if (degree == 1) return;
    for (int a = 0; a < nv; ++a)
        for (int b = a + 1; b < nv; ++b) {
            double la = lam[a], lb = lam[b];
            if (degree == 2) {
                phi[k] = 4.0 * la * lb;
                dphi[k * nv + a] = 4.0 * lb;
                dphi[k * nv + b] = 4.0 * la;
                ++k;
            } else {
                phi[k] = 4.5 * la * lb * (3.0 * la - 1.0);          /* nearer a */
                dphi[k * nv + a] = 4.5 * lb * (6.0 * la - 1.0);
                dphi[k * nv + b] = 4.5 * la * (3.0 * la - 1.0);
                ++k;
                phi[k] = 4.5 * la * lb * (3.0 * lb - 1.0);          /* nearer b */
                dphi[k * nv + a] = 4.5 * lb * (3.0 * lb - 1.0);
                dphi[k * nv + b] = 4.5 * la * (6.0 * lb - 1.0);
                ++k;
            }
        }
    if (degree == 3) {
        for (int a = 0; a < nv; ++a)
            for (int b = a + 1; b < nv; ++b)
                for (int c = b + 1; c < nv; ++c) {
                    double la = lam[a], lb = lam[b], lc = lam[c];
                    phi[k] = 27.0 * la * lb * lc;
                    dphi[k * nv + a] = 27.0 * lb * lc;
                    dphi[k * nv + b] = 27.0 * la * lc;
                    dphi[k * nv + c] = 27.0 * la * lb;
                    ++k;
                }
    }
}

/* ------------------------------------------------------------------ */
/* Cell geometry                                                       */
/* ------------------------------------------------------------------ */

/* J[r][c] = x_{c+1}[r] - x_0[r]; returns det J, writes Jinv. */
static double cell_geometry(int dim, const double *xv, double *J, double *Jinv)
{
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            J[r * dim + c] = xv[(c + 1) * dim + r] - xv[r];
    double det;
    if (dim == 2) {
        det = J[0] * J[3] - J[1] * J[2];
        Jinv[0] = J[3] / det; Jinv[1] = -J[1] / det;
        Jinv[2] = -J[2] / det; Jinv[3] = J[0] / det;
    } else {
        double a = J[0], b = J[1], c = J[2], d = J[3], e = J[4], f = J[5], g = J[6], h = J[7], i = J[8];
        det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
        Jinv[0] = (e * i - f * h) / det; Jinv[1] = (c * h - b * i) / det; Jinv[2] = (b * f - c * e) / det;
        Jinv[3] = (f * g - d * i) / det; Jinv[4] = (a * i - c * g) / det; Jinv[5] = (c * d - a * f) / det;
        Jinv[6] = (d * h - e * g) / det; Jinv[7] = (b * g - a * h) / det; Jinv[8] = (a * e - b * d) / det;
    }
    return det;
}

/* Quadrature points per direction for an integrand of total degree deg:
 * the smallest exact count plus one. */
static int points_for_degree(int deg) { return (deg + 2) / 2 + 1; }

struct rule { int np; double pts[MAXQ * MAXQ * MAXQ * 3]; double wts[MAXQ * MAXQ * MAXQ]; };

static int make_rule(int dim, int deg, struct rule *R)
{
    int q = points_for_degree(deg);
    if (q > MAXQ) return -1;
    R->np = oracle_simplex_rule(dim, q, R->pts, R->wts);
    return R->np > 0 ? 0 : -1;
}

/*
 * Physical-point data at one reference point of one cell: barycentrics of
 * the physical point x = x_0 + J xhat (recovered through J^{-1}), basis
 * values and physical gradients.
 */
static void eval_at_point(int dim, int degree, const double *xv, const double *Jinv,
                          const double *xhat, double *lam, double *phi, double *gphi)
{
    const int nv = dim + 1, n = oracle_nloc(dim, degree);
    double x[3], rel[3], xh[3];
    double J[9];
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            J[r * dim + c] = xv[(c + 1) * dim + r] - xv[r];
    for (int r = 0; r < dim; ++r) {
        x[r] = xv[r];
        for (int c = 0; c < dim; ++c) x[r] += J[r * dim + c] * xhat[c];
    }
    for (int r = 0; r < dim; ++r) rel[r] = x[r] - xv[r];
    double s = 0.0;
    for (int m = 0; m < dim; ++m) {
        xh[m] = 0.0;
        for (int r = 0; r < dim; ++r) xh[m] += Jinv[m * dim + r] * rel[r];
        lam[m + 1] = xh[m];
        s += xh[m];
    }
    lam[0] = 1.0 - s;
    /* grad lambda_m for m >= 1 is row m-1 of J^{-1}; grad lambda_0 = -sum. */
    double glam[4][3];
    for (int r = 0; r < dim; ++r) glam[0][r] = 0.0;
    for (int m = 1; m < nv; ++m)
        for (int r = 0; r < dim; ++r) {
            glam[m][r] = Jinv[(m - 1) * dim + r];
            glam[0][r] -= glam[m][r];
        }
    double dphi[MAXLOC * 4];
    oracle_basis(dim, degree, lam, phi, dphi);
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < dim; ++r) {
            double g = 0.0;
            for (int m = 0; m < nv; ++m) g += dphi[i * nv + m] * glam[m][r];
            gphi[i * dim + r] = g;
        }
}

/*
 * Element matrix of  cstiff * kappa grad(u).grad(v) + cmass * u v  on one
 * cell: A[i][j] (row = test function i).  xv: vertex coordinates [dim+1][dim];
 * kv: kappa at the vertices [dim+1].
 */
int oracle_element_matrix(int dim, int degree, const double *xv, const double *kv,
                          double cstiff, double cmass, double *A, double *Aabs)
{
    const int n = oracle_nloc(dim, degree), nv = dim + 1;
    if (n < 0) return -1;
    struct rule R;
    if (make_rule(dim, 2 * degree, &R)) return -1;
    double J[9], Jinv[9];
    double det = cell_geometry(dim, xv, J, Jinv);
    double adet = fabs(det);
    memset(A, 0, sizeof(double) * n * n);
    if (Aabs) memset(Aabs, 0, sizeof(double) * n * n);
    for (int p = 0; p < R.np; ++p) {
        double lam[4], phi[MAXLOC], gphi[MAXLOC * 3];
        eval_at_point(dim, degree, xv, Jinv, &R.pts[p * dim], lam, phi, gphi);
        double kap = 0.0;
        for (int m = 0; m < nv; ++m) kap += kv[m] * lam[m];
        double w = R.wts[p] * adet;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double g = 0.0, ga = 0.0;
                for (int r = 0; r < dim; ++r) {
                    g += gphi[i * dim + r] * gphi[j * dim + r];
                    ga += fabs(gphi[i * dim + r] * gphi[j * dim + r]);
                }
                A[i * n + j] += w * (cstiff * kap * g + cmass * phi[i] * phi[j]);
                /* magnitude of the summed terms: the scale of the rounding
                 * error of this entry (sum of |terms| bounds it) */
                if (Aabs) Aabs[i * n + j] += fabs(w) * (fabs(cstiff * kap) * ga + fabs(cmass * phi[i] * phi[j]));
            }
    }
    return 0;
}

/* Element vector of  f v  with f a P1 field (fv: f at the vertices). */
int oracle_element_vector(int dim, int degree, const double *xv, const double *fv, double *b,
                          double *babs)
{
    const int n = oracle_nloc(dim, degree), nv = dim + 1;
    if (n < 0) return -1;
    struct rule R;
    if (make_rule(dim, degree + 1, &R)) return -1;
    double J[9], Jinv[9];
    double adet = fabs(cell_geometry(dim, xv, J, Jinv));
    memset(b, 0, sizeof(double) * n);
    if (babs) memset(babs, 0, sizeof(double) * n);
    for (int p = 0; p < R.np; ++p) {
        double lam[4], phi[MAXLOC], gphi[MAXLOC * 3];
        eval_at_point(dim, degree, xv, Jinv, &R.pts[p * dim], lam, phi, gphi);
        double fx = 0.0, fa = 0.0;
        for (int m = 0; m < nv; ++m) { fx += fv[m] * lam[m]; fa += fabs(fv[m] * lam[m]); }
        for (int i = 0; i < n; ++i) {
            b[i] += R.wts[p] * adet * fx * phi[i];
            if (babs) babs[i] += fabs(R.wts[p] * adet * phi[i]) * fa;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gathers (staging in)                                                */
/* ------------------------------------------------------------------ */

static void gather_cell(int dim, int64_t c, const int32_t *cell_vertex, const double *coords,
                        const double *field, double *xv, double *fv)
{
    const int nv = dim + 1;
    for (int m = 0; m < nv; ++m) {
        int64_t v = cell_vertex[c * nv + m];
        for (int r = 0; r < dim; ++r) xv[m * dim + r] = coords[v * dim + r];
        if (fv) fv[m] = field ? field[v] : 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* Sparsity                                                            */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Row -> incident (cell, local index) lists of a Map, cells in index order. */
static int incidence(int64_t ncells, int nloc, const int32_t *map, int64_t nrows,
                     int64_t **ptr_out, int64_t **ent_out)
{
    int64_t *ptr = calloc((size_t)nrows + 1, sizeof(int64_t));
    int64_t *ent = malloc(sizeof(int64_t) * (size_t)(ncells * nloc + 1));
    int64_t *cur = malloc(sizeof(int64_t) * (size_t)(nrows + 1));
    if (!ptr || !ent || !cur) { free(ptr); free(ent); free(cur); return -1; }
    for (int64_t e = 0; e < ncells * nloc; ++e) {
        int32_t r = map[e];
        if (r < 0 || r >= nrows) { free(ptr); free(ent); free(cur); return -2; }
        ptr[r + 1]++;
    }
    for (int64_t r = 0; r < nrows; ++r) ptr[r + 1] += ptr[r];
    memcpy(cur, ptr, sizeof(int64_t) * (size_t)nrows);
    for (int64_t e = 0; e < ncells * nloc; ++e) ent[cur[map[e]]++] = e;   /* e = c*nloc + l */
    free(cur);
    *ptr_out = ptr; *ent_out = ent;
    return 0;
}

/*
 * CSR sparsity of the Mat with row Map rmap and column Map cmap: row i holds
 * every column of every cell incident to i, sorted ascending, unique.
 * Pass col_idx == NULL to count: fills row_ptr[0..nrows] and returns nnz.
 * With col_idx != NULL (row_ptr from the counting call) fills the columns.
 * Returns a negative value on an out-of-range Map entry or allocation failure.
 */
int64_t oracle_sparsity(int64_t ncells, int nloc_r, const int32_t *rmap, int nloc_c,
                        const int32_t *cmap, int64_t nrows, int64_t ncols,
                        int64_t *row_ptr, int32_t *col_idx)
{
    for (int64_t e = 0; e < ncells * nloc_c; ++e)
        if (cmap[e] < 0 || cmap[e] >= ncols) return -2;
    int64_t *ptr, *ent;
    int rc = incidence(ncells, nloc_r, rmap, nrows, &ptr, &ent);
    if (rc) return rc;
    int64_t maxdeg = 0;
    for (int64_t r = 0; r < nrows; ++r)
        if (ptr[r + 1] - ptr[r] > maxdeg) maxdeg = ptr[r + 1] - ptr[r];
    int32_t *buf = malloc(sizeof(int32_t) * (size_t)(maxdeg * nloc_c + 1));
    if (!buf) { free(ptr); free(ent); return -1; }
    int64_t total = 0;
    if (!col_idx) row_ptr[0] = 0;
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t m = 0;
        for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k) {
            int64_t c = ent[k] / nloc_r;
            for (int l = 0; l < nloc_c; ++l) buf[m++] = cmap[c * nloc_c + l];
        }
        qsort(buf, (size_t)m, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t k = 0; k < m; ++k)
            if (k == 0 || buf[k] != buf[k - 1]) buf[u++] = buf[k];
        if (col_idx) memcpy(col_idx + row_ptr[r], buf, sizeof(int32_t) * (size_t)u);
        else row_ptr[r + 1] = row_ptr[r] + u;
        total += u;
    }
    free(buf); free(ptr); free(ent);
    return total;
}

static int64_t find_col(const int64_t *row_ptr, const int32_t *col_idx, int64_t r, int32_t c)
{
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col_idx[mid] == c) return mid;
        if (col_idx[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Global assembly (par_loop over all cells, INC into Mat / Dat)        */
/* ------------------------------------------------------------------ */

/*
 * values[k] (k indexes the CSR given by row_ptr/col_idx, which must contain
 * the assembled pattern) is overwritten with the assembled matrix; absval[k]
 * (optional) with the magnitude scale of the rounding error: the sum over
 * cells and quadrature points of |weight * integrand term|.  Returns 0, or -3 if a
 * contribution falls outside the pattern.
 */
int oracle_assemble_mat(int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                        const double *coords, const int32_t *cell_node, const double *kappa,
                        double cstiff, double cmass, const int64_t *row_ptr,
                        const int32_t *col_idx, int64_t nrows, double *values, double *absval,
                        double *cabsval)
{
    const int n = oracle_nloc(dim, degree);
    if (n < 0) return -1;
    int64_t nnz = row_ptr[nrows];
    memset(values, 0, sizeof(double) * (size_t)nnz);
    if (absval) memset(absval, 0, sizeof(double) * (size_t)nnz);
    if (cabsval) memset(cabsval, 0, sizeof(double) * (size_t)nnz);
    double xv[12], kv[4], A[MAXLOC * MAXLOC], Aa[MAXLOC * MAXLOC];
    for (int64_t c = 0; c < ncells; ++c) {
        gather_cell(dim, c, cell_vertex, coords, kappa, xv, kv);
        if (oracle_element_matrix(dim, degree, xv, kv, cstiff, cmass, A, Aa)) return -1;
        for (int i = 0; i < n; ++i) {
            int32_t r = cell_node[c * n + i];
            for (int j = 0; j < n; ++j) {
                int64_t k = find_col(row_ptr, col_idx, r, cell_node[c * n + j]);
                if (k < 0) return -3;
                values[k] += A[i * n + j];
                if (absval) absval[k] += Aa[i * n + j];
                /* contribution-level scale: sum over cells of |element entry| */
                if (cabsval) cabsval[k] += fabs(A[i * n + j]);
            }
        }
    }
    return 0;
}

/* b (length nrows) overwritten with the assembled vector of f v. */
int oracle_assemble_vec(int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                        const double *coords, const int32_t *cell_node, const double *f,
                        int64_t nrows, double *b, double *absb)
{
    const int n = oracle_nloc(dim, degree);
    if (n < 0) return -1;
    memset(b, 0, sizeof(double) * (size_t)nrows);
    if (absb) memset(absb, 0, sizeof(double) * (size_t)nrows);
    double xv[12], fv[4], be[MAXLOC], ba[MAXLOC];
    for (int64_t c = 0; c < ncells; ++c) {
        gather_cell(dim, c, cell_vertex, coords, f, xv, fv);
        if (oracle_element_vector(dim, degree, xv, fv, be, ba)) return -1;
        for (int i = 0; i < n; ++i) {
            int32_t r = cell_node[c * n + i];
            if (r < 0 || r >= nrows) return -2;
            b[r] += be[i];
            if (absb) absb[r] += ba[i];
        }
    }
    return 0;
}

/* y (length nrows) overwritten with sum_K P_K^T A_K P_K x, cell by cell. */
int oracle_apply_action(int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                        const double *coords, const int32_t *cell_node, const double *kappa,
                        double cstiff, double cmass, const double *x, int64_t nrows,
                        double *y, double *absy)
{
    const int n = oracle_nloc(dim, degree);
    if (n < 0) return -1;
    memset(y, 0, sizeof(double) * (size_t)nrows);
    if (absy) memset(absy, 0, sizeof(double) * (size_t)nrows);
    double xv[12], kv[4], A[MAXLOC * MAXLOC], Aa[MAXLOC * MAXLOC];
    for (int64_t c = 0; c < ncells; ++c) {
        gather_cell(dim, c, cell_vertex, coords, kappa, xv, kv);
        if (oracle_element_matrix(dim, degree, xv, kv, cstiff, cmass, A, Aa)) return -1;
        for (int i = 0; i < n; ++i) {
            int32_t r = cell_node[c * n + i];
            if (r < 0 || r >= nrows) return -2;
            double s = 0.0, sa = 0.0;
            for (int j = 0; j < n; ++j) {
                double xj = x[cell_node[c * n + j]];
                s += A[i * n + j] * xj;
                sa += Aa[i * n + j] * fabs(xj);
            }
            y[r] += s;
            if (absy) absy[r] += sa;
        }
    }
    return 0;
}

/*
 * Selected rows of the assembled matrix, for meshes too large to assemble
 * whole.  rows[0..nsel) are distinct row ids.  Every cell is visited in index
 * order; each contribution to a selected row is added to that row's column
 * list (found by linear search, appended when new), then each row's list is
 * sorted by column.  Output for selected row s: out_ptr[s]..out_ptr[s+1] in
 * out_cols/out_vals/out_abs (capacity cap entries).  Returns total entries,
 * or a negative value on error / insufficient capacity.
 */
int64_t oracle_mat_rows(int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                        const double *coords, const int32_t *cell_node, const double *kappa,
                        double cstiff, double cmass, int64_t nrows, int64_t nsel,
                        const int64_t *rows, int64_t cap, int64_t *out_ptr,
                        int32_t *out_cols, double *out_vals, double *out_abs, double *out_cabs)
{
    const int n = oracle_nloc(dim, degree);
    if (n < 0) return -1;
    int64_t *slot = malloc(sizeof(int64_t) * (size_t)nrows);
    const int64_t per = 1024;                       /* max columns per selected row */
    int32_t *cols = malloc(sizeof(int32_t) * (size_t)(nsel * per));
    double *vals = calloc((size_t)(nsel * per), sizeof(double));
    double *abss = calloc((size_t)(nsel * per), sizeof(double));
    double *cabs = calloc((size_t)(nsel * per), sizeof(double));
    int64_t *cnt = calloc((size_t)nsel, sizeof(int64_t));
    if (!slot || !cols || !vals || !abss || !cabs || !cnt) {
        free(slot); free(cols); free(vals); free(abss); free(cabs); free(cnt);
        return -1;
    }
    for (int64_t r = 0; r < nrows; ++r) slot[r] = -1;
    for (int64_t s = 0; s < nsel; ++s) slot[rows[s]] = s;
    double xv[12], kv[4], A[MAXLOC * MAXLOC], Aa[MAXLOC * MAXLOC];
    int64_t rc = 0;
    for (int64_t c = 0; c < ncells && rc == 0; ++c) {
        int any = 0;
        for (int i = 0; i < n; ++i) any |= slot[cell_node[c * n + i]] >= 0;
        if (!any) continue;
        gather_cell(dim, c, cell_vertex, coords, kappa, xv, kv);
        oracle_element_matrix(dim, degree, xv, kv, cstiff, cmass, A, Aa);
        for (int i = 0; i < n; ++i) {
            int64_t s = slot[cell_node[c * n + i]];
            if (s < 0) continue;
            for (int j = 0; j < n; ++j) {
                int32_t col = cell_node[c * n + j];
                int64_t k = 0;
                while (k < cnt[s] && cols[s * per + k] != col) ++k;
                if (k == cnt[s]) {
                    if (k == per) { rc = -4; break; }
                    cols[s * per + k] = col; cnt[s]++;
                }
                vals[s * per + k] += A[i * n + j];
                abss[s * per + k] += Aa[i * n + j];
                cabs[s * per + k] += fabs(A[i * n + j]);
            }
        }
    }
    int64_t total = 0;
    if (rc == 0) {
        out_ptr[0] = 0;
        for (int64_t s = 0; s < nsel; ++s) {
            /* insertion sort of this row's (col, val, abs, cabs) tuples by col */
            int32_t *cc = cols + s * per;
            double *vv = vals + s * per, *aa = abss + s * per, *ca = cabs + s * per;
            for (int64_t a = 1; a < cnt[s]; ++a) {
                int32_t kc = cc[a]; double kv2 = vv[a], ka = aa[a], kca = ca[a];
                int64_t b = a - 1;
                while (b >= 0 && cc[b] > kc) {
                    cc[b + 1] = cc[b]; vv[b + 1] = vv[b]; aa[b + 1] = aa[b]; ca[b + 1] = ca[b]; --b;
                }
                cc[b + 1] = kc; vv[b + 1] = kv2; aa[b + 1] = ka; ca[b + 1] = kca;
            }
            if (total + cnt[s] > cap) { rc = -5; break; }
            memcpy(out_cols + total, cc, sizeof(int32_t) * (size_t)cnt[s]);
            memcpy(out_vals + total, vv, sizeof(double) * (size_t)cnt[s]);
            memcpy(out_abs + total, aa, sizeof(double) * (size_t)cnt[s]);
            if (out_cabs) memcpy(out_cabs + total, ca, sizeof(double) * (size_t)cnt[s]);
            total += cnt[s];
            out_ptr[s + 1] = total;
        }
    }
    free(slot); free(cols); free(vals); free(abss); free(cabs); free(cnt);
    return rc ? rc : total;
}

/*
 * Selected entries of the assembled vector (kind 0: f v with field = f) or of
 * the action y = A x (kind 1: field = kappa).  Visits every cell in order.
 */
int oracle_vec_rows(int kind, int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                    const double *coords, const int32_t *cell_node, const double *field,
                    double cstiff, double cmass, const double *x, int64_t nrows, int64_t nsel,
                    const int64_t *rows, double *out, double *out_abs)
{
    const int n = oracle_nloc(dim, degree);
    if (n < 0) return -1;
    int64_t *slot = malloc(sizeof(int64_t) * (size_t)nrows);
    if (!slot) return -1;
    for (int64_t r = 0; r < nrows; ++r) slot[r] = -1;
    for (int64_t s = 0; s < nsel; ++s) { slot[rows[s]] = s; out[s] = 0.0; out_abs[s] = 0.0; }
    double xv[12], fv[4], A[MAXLOC * MAXLOC], Aa[MAXLOC * MAXLOC], be[MAXLOC], ba[MAXLOC];
    for (int64_t c = 0; c < ncells; ++c) {
        int any = 0;
        for (int i = 0; i < n; ++i) any |= slot[cell_node[c * n + i]] >= 0;
        if (!any) continue;
        gather_cell(dim, c, cell_vertex, coords, field, xv, fv);
        if (kind == 0) oracle_element_vector(dim, degree, xv, fv, be, ba);
        else oracle_element_matrix(dim, degree, xv, fv, cstiff, cmass, A, Aa);
        for (int i = 0; i < n; ++i) {
            int64_t s = slot[cell_node[c * n + i]];
            if (s < 0) continue;
            if (kind == 0) { out[s] += be[i]; out_abs[s] += ba[i]; }
            else {
                double t = 0.0, ta = 0.0;
                for (int j = 0; j < n; ++j) {
                    double xj = x[cell_node[c * n + j]];
                    t += A[i * n + j] * xj; ta += Aa[i * n + j] * fabs(xj);
                }
                out[s] += t; out_abs[s] += ta;
            }
        }
    }
    free(slot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Nonlinear residual and its vector-Jacobian products (P1)             */
/* ------------------------------------------------------------------ */

/*
 * The residual of the differentiation benchmark,
 *
 *   F_i(u, kappa) = integral of  kappa grad(u).grad(phi_i) + u^3 phi_i - f phi_i,
 *
 * and, for a vector lambda (a P1 field lambda_h = sum_i lambda_i phi_i), the
 * vector-Jacobian products
 *
 *   (lambda^T dF/du)_j     = integral of  kappa grad(phi_j).grad(lambda_h)
 *                                         + 3 u^2 phi_j lambda_h,
 *   (lambda^T dF/dkappa)_k = integral of  phi_k grad(u).grad(lambda_h),
 *
 * obtained by differentiating the integrand of F_i with respect to u_j and
 * kappa_k and contracting with lambda_i.  The adjoint of the residual is what
 * the paper's closing discussion (adjoint models through the same
 * abstractions) points to.  u, kappa, f and lambda are P1 fields on the nodes
 * of the degree-1 space (read through the cell-to-node Map).  The integrand
 * has degree 4; the rule is exact for it.
 *
 * Element level: uv, kv, fv, lv are the nodal values of the cell; any output
 * may be NULL.  The *_abs outputs sum the magnitudes of the terms.
 */
static void nl_element_rule(int dim, const struct rule *R, const double *xv, const double *uv,
                            const double *kv, const double *fv, const double *lv, double *F, double *Fabs,
                            double *gu, double *guabs, double *gk, double *gkabs)
{
    const int n = dim + 1;
    double J[9], Jinv[9];
    double adet = fabs(cell_geometry(dim, xv, J, Jinv));
    for (int i = 0; i < n; ++i) {
        if (F) F[i] = 0.0;
        if (Fabs) Fabs[i] = 0.0;
        if (gu) gu[i] = 0.0;
        if (guabs) guabs[i] = 0.0;
        if (gk) gk[i] = 0.0;
        if (gkabs) gkabs[i] = 0.0;
    }
    for (int p = 0; p < R->np; ++p) {
        double lam[4], phi[MAXLOC], gphi[MAXLOC * 3];
        eval_at_point(dim, 1, xv, Jinv, &R->pts[p * dim], lam, phi, gphi);
        const double w = R->wts[p] * adet;
        double uq = 0, ua = 0, kq = 0, ka = 0, fq = 0, fa = 0, lq = 0, la = 0;
        double gu_[3] = {0, 0, 0}, gl_[3] = {0, 0, 0};
        for (int m = 0; m < n; ++m) {
            uq += uv[m] * phi[m]; ua += fabs(uv[m] * phi[m]);
            kq += kv[m] * phi[m]; ka += fabs(kv[m] * phi[m]);
            if (fv) { fq += fv[m] * phi[m]; fa += fabs(fv[m] * phi[m]); }
            if (lv) { lq += lv[m] * phi[m]; la += fabs(lv[m] * phi[m]); }
            for (int r = 0; r < dim; ++r) {
                gu_[r] += uv[m] * gphi[m * dim + r];
                if (lv) gl_[r] += lv[m] * gphi[m * dim + r];
            }
        }
        double gul = 0, gula = 0;
        for (int r = 0; r < dim; ++r) { gul += gu_[r] * gl_[r]; gula += fabs(gu_[r] * gl_[r]); }
        for (int i = 0; i < n; ++i) {
            double gg = 0, gga = 0, gil = 0, gila = 0;
            for (int r = 0; r < dim; ++r) {
                gg += gu_[r] * gphi[i * dim + r];
                gga += fabs(gu_[r] * gphi[i * dim + r]);
                gil += gphi[i * dim + r] * gl_[r];
                gila += fabs(gphi[i * dim + r] * gl_[r]);
            }
            if (F) F[i] += w * (kq * gg + uq * uq * uq * phi[i] - fq * phi[i]);
            if (Fabs) Fabs[i] += fabs(w) * (ka * gga + ua * ua * ua * fabs(phi[i]) + fa * fabs(phi[i]));
            if (gu) gu[i] += w * (kq * gil + 3.0 * uq * uq * phi[i] * lq);
            if (guabs) guabs[i] += fabs(w) * (ka * gila + 3.0 * ua * ua * fabs(phi[i]) * la);
            if (gk) gk[i] += w * phi[i] * gul;
            if (gkabs) gkabs[i] += fabs(w * phi[i]) * gula;
        }
    }
}

int oracle_nl_element(int dim, const double *xv, const double *uv, const double *kv, const double *fv,
                      const double *lv, double *F, double *Fabs, double *gu, double *guabs, double *gk,
                      double *gkabs)
{
    struct rule R;
    if (make_rule(dim, 4, &R)) return -1;
    nl_element_rule(dim, &R, xv, uv, kv, fv, lv, F, Fabs, gu, guabs, gk, gkabs);
    return 0;
}

static void gather_nodal(int n, int64_t c, const int32_t *cell_node, const double *a, double *av)
{
    for (int i = 0; i < n; ++i) av[i] = a ? a[cell_node[c * n + i]] : 0.0;
}

/* Global residual F[nnodes] (and its magnitude scale), cells in index order. */
int oracle_nl_residual(int dim, int64_t ncells, const int32_t *cell_vertex, const double *coords,
                       const int32_t *cell_node, int64_t nnodes, const double *u, const double *kappa,
                       const double *f, double *F, double *Fabs)
{
    const int n = dim + 1;
    memset(F, 0, sizeof(double) * nnodes);
    memset(Fabs, 0, sizeof(double) * nnodes);
    double xv[12], uv[4], kv[4], fv[4], Fe[4], Fa[4], dummy[4];
    struct rule R;
    if (make_rule(dim, 4, &R)) return -1;
    for (int64_t c = 0; c < ncells; ++c) {
        gather_cell(dim, c, cell_vertex, coords, NULL, xv, dummy);
        gather_nodal(n, c, cell_node, u, uv);
        gather_nodal(n, c, cell_node, kappa, kv);
        gather_nodal(n, c, cell_node, f, fv);
        nl_element_rule(dim, &R, xv, uv, kv, fv, NULL, Fe, Fa, NULL, NULL, NULL, NULL);
        for (int i = 0; i < n; ++i) {
            F[cell_node[c * n + i]] += Fe[i];
            Fabs[cell_node[c * n + i]] += Fa[i];
        }
    }
    return 0;
}

/* Global vector-Jacobian products gu = lambda^T dF/du, gk = lambda^T dF/dkappa. */
int oracle_nl_adjoint(int dim, int64_t ncells, const int32_t *cell_vertex, const double *coords,
                      const int32_t *cell_node, int64_t nnodes, const double *u, const double *kappa,
                      const double *lambda, double *gu, double *guabs, double *gk, double *gkabs)
{
    const int n = dim + 1;
    memset(gu, 0, sizeof(double) * nnodes);
    memset(guabs, 0, sizeof(double) * nnodes);
    memset(gk, 0, sizeof(double) * nnodes);
    memset(gkabs, 0, sizeof(double) * nnodes);
    double xv[12], uv[4], kv[4], lv[4], a[4], aa[4], b[4], ba[4], dummy[4];
    struct rule R;
    if (make_rule(dim, 4, &R)) return -1;
    for (int64_t c = 0; c < ncells; ++c) {
        gather_cell(dim, c, cell_vertex, coords, NULL, xv, dummy);
        gather_nodal(n, c, cell_node, u, uv);
        gather_nodal(n, c, cell_node, kappa, kv);
        gather_nodal(n, c, cell_node, lambda, lv);
        nl_element_rule(dim, &R, xv, uv, kv, NULL, lv, NULL, NULL, a, aa, b, ba);
        for (int i = 0; i < n; ++i) {
            const int32_t r = cell_node[c * n + i];
            gu[r] += a[i]; guabs[r] += aa[i];
            gk[r] += b[i]; gkabs[r] += ba[i];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Vector Lagrange linear elasticity (the precision benchmark)          */
/* ------------------------------------------------------------------ */

/*
 * a(u, v) = integral of 2 mu eps(u):eps(v) + lam div(u) div(v), with eps the
 * symmetric gradient and mu, lam P1 fields.  u and v lie in the vector
 * Lagrange space of the given degree with dim components; with the basis
 * phi_i e_a (DOF dim*node + a, node-major) the entry is
 *
 *   A[(i,a),(j,b)] = integral of  mu (delta_ab grad phi_i . grad phi_j
 *                                     + d_b phi_i d_a phi_j)
 *                                + lam d_a phi_i d_b phi_j,
 *
 * because 2 eps(phi_j e_b):eps(phi_i e_a) = delta_ab grad phi_i . grad phi_j
 * + d_b phi_i d_a phi_j and div(phi e_b) = d_b phi.  The integrand has degree
 * 2 degree - 1 on affine cells.  A is [dim*n][dim*n], row (i, a) = i*dim + a;
 * Aabs sums the magnitudes of the terms (the rounding scale of each entry).
 * xv: the cell's vertex coordinates [dim+1][dim]; muv, lav: mu and lam at the
 * vertices.
 */
int oracle_elasticity_element(int dim, int degree, const double *xv, const double *muv, const double *lav,
                              double *A, double *Aabs)
{
    const int n = oracle_nloc(dim, degree), nv = dim + 1, N = dim * n;
    if (n < 0) return -1;
    struct rule R;
    if (make_rule(dim, 2 * degree - 1, &R)) return -1;
    double J[9], Jinv[9];
    const double adet = fabs(cell_geometry(dim, xv, J, Jinv));
    memset(A, 0, sizeof(double) * N * N);
    if (Aabs) memset(Aabs, 0, sizeof(double) * N * N);
    for (int p = 0; p < R.np; ++p) {
        double lam[4], phi[MAXLOC], gphi[MAXLOC * 3];
        eval_at_point(dim, degree, xv, Jinv, &R.pts[p * dim], lam, phi, gphi);
        double mu = 0.0, la = 0.0;
        for (int m = 0; m < nv; ++m) { mu += muv[m] * lam[m]; la += lav[m] * lam[m]; }
        const double w = R.wts[p] * adet;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double g = 0.0, ga = 0.0;
                for (int r = 0; r < dim; ++r) {
                    g += gphi[i * dim + r] * gphi[j * dim + r];
                    ga += fabs(gphi[i * dim + r] * gphi[j * dim + r]);
                }
                for (int a = 0; a < dim; ++a)
                    for (int b = 0; b < dim; ++b) {
                        const double cross = gphi[i * dim + b] * gphi[j * dim + a];
                        const double dd = gphi[i * dim + a] * gphi[j * dim + b];
                        const double t = mu * ((a == b ? g : 0.0) + cross) + la * dd;
                        const int64_t k = (int64_t)(i * dim + a) * N + (j * dim + b);
                        A[k] += w * t;
                        if (Aabs)
                            Aabs[k] += fabs(w) * (fabs(mu) * ((a == b ? ga : 0.0) + fabs(cross)) + fabs(la * dd));
                    }
            }
    }
    return 0;
}

/*
 * Global elasticity matrix.  Coordinates are per cell: xdg[c][m][r] (a
 * discontinuous coordinate field); mu and lam are vertex fields read through
 * cell_vertex; cell_node is the scalar node Map, vector DOFs are dim*node + a.
 * row_ptr/col_idx: the vector CSR (rows dim*nnodes).  Cells in index order,
 * each contribution found by binary search in its row.
 */
int oracle_elasticity_mat(int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                          const double *xdg, const int32_t *cell_node, const double *mu, const double *lam,
                          const int64_t *row_ptr, const int32_t *col_idx, int64_t nrows, double *values,
                          double *absval)
{
    const int n = oracle_nloc(dim, degree), nv = dim + 1, N = dim * n;
    if (n < 0) return -1;
    const int64_t nnz = row_ptr[nrows];
    memset(values, 0, sizeof(double) * (size_t)nnz);
    if (absval) memset(absval, 0, sizeof(double) * (size_t)nnz);
    double *A = malloc(sizeof(double) * N * N), *Aa = malloc(sizeof(double) * N * N);
    if (!A || !Aa) { free(A); free(Aa); return -1; }
    double muv[4], lav[4];
    int rc = 0;
    for (int64_t c = 0; c < ncells && !rc; ++c) {
        for (int m = 0; m < nv; ++m) {
            muv[m] = mu[cell_vertex[c * nv + m]];
            lav[m] = lam[cell_vertex[c * nv + m]];
        }
        if (oracle_elasticity_element(dim, degree, xdg + c * nv * dim, muv, lav, A, Aa)) { rc = -1; break; }
        for (int i = 0; i < n && !rc; ++i)
            for (int a = 0; a < dim && !rc; ++a) {
                const int64_t r = (int64_t)dim * cell_node[c * n + i] + a;
                if (r < 0 || r >= nrows) { rc = -2; break; }
                for (int j = 0; j < n; ++j)
                    for (int b = 0; b < dim; ++b) {
                        const int64_t k = find_col(row_ptr, col_idx, r, dim * cell_node[c * n + j] + b);
                        if (k < 0) { rc = -3; break; }
                        values[k] += A[(int64_t)(i * dim + a) * N + j * dim + b];
                        if (absval) absval[k] += Aa[(int64_t)(i * dim + a) * N + j * dim + b];
                    }
            }
    }
    free(A); free(Aa);
    return rc;
}

/*
 * Selected rows of the global elasticity matrix (vector DOF rows, distinct),
 * for meshes too large to assemble whole; same output convention as
 * oracle_mat_rows.
 */
int64_t oracle_elasticity_rows(int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                               const double *xdg, const int32_t *cell_node, const double *mu,
                               const double *lam, int64_t nrows, int64_t nsel, const int64_t *rows,
                               int64_t cap, int64_t *out_ptr, int32_t *out_cols, double *out_vals,
                               double *out_abs)
{
    const int n = oracle_nloc(dim, degree), nv = dim + 1, N = dim * n;
    if (n < 0) return -1;
    const int64_t per = 1024;
    int64_t *slot = malloc(sizeof(int64_t) * (size_t)nrows);
    int32_t *cols = malloc(sizeof(int32_t) * (size_t)(nsel * per));
    double *vals = calloc((size_t)(nsel * per), sizeof(double));
    double *abss = calloc((size_t)(nsel * per), sizeof(double));
    int64_t *cnt = calloc((size_t)nsel, sizeof(int64_t));
    double *A = malloc(sizeof(double) * N * N), *Aa = malloc(sizeof(double) * N * N);
    int64_t rc = 0;
    if (!slot || !cols || !vals || !abss || !cnt || !A || !Aa) rc = -1;
    if (!rc) {
        for (int64_t r = 0; r < nrows; ++r) slot[r] = -1;
        for (int64_t s = 0; s < nsel; ++s) slot[rows[s]] = s;
    }
    double muv[4], lav[4];
    for (int64_t c = 0; c < ncells && rc == 0; ++c) {
        int any = 0;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < dim; ++a) any |= slot[(int64_t)dim * cell_node[c * n + i] + a] >= 0;
        if (!any) continue;
        for (int m = 0; m < nv; ++m) {
            muv[m] = mu[cell_vertex[c * nv + m]];
            lav[m] = lam[cell_vertex[c * nv + m]];
        }
        oracle_elasticity_element(dim, degree, xdg + c * nv * dim, muv, lav, A, Aa);
        for (int i = 0; i < n && rc == 0; ++i)
            for (int a = 0; a < dim && rc == 0; ++a) {
                const int64_t s = slot[(int64_t)dim * cell_node[c * n + i] + a];
                if (s < 0) continue;
                for (int j = 0; j < n; ++j)
                    for (int b = 0; b < dim; ++b) {
                        const int32_t col = dim * cell_node[c * n + j] + b;
                        int64_t k = 0;
                        while (k < cnt[s] && cols[s * per + k] != col) ++k;
                        if (k == cnt[s]) {
                            if (k == per) { rc = -4; break; }
                            cols[s * per + k] = col; cnt[s]++;
                        }
                        vals[s * per + k] += A[(int64_t)(i * dim + a) * N + j * dim + b];
                        abss[s * per + k] += Aa[(int64_t)(i * dim + a) * N + j * dim + b];
                    }
            }
    }
    int64_t total = 0;
    if (rc == 0) {
        out_ptr[0] = 0;
        for (int64_t s = 0; s < nsel; ++s) {
            int32_t *cc = cols + s * per; double *vv = vals + s * per, *aa = abss + s * per;
            for (int64_t a = 1; a < cnt[s]; ++a) {
                int32_t kc = cc[a]; double kv2 = vv[a], ka = aa[a];
                int64_t b = a - 1;
                while (b >= 0 && cc[b] > kc) { cc[b + 1] = cc[b]; vv[b + 1] = vv[b]; aa[b + 1] = aa[b]; --b; }
                cc[b + 1] = kc; vv[b + 1] = kv2; aa[b + 1] = ka;
            }
            if (total + cnt[s] > cap) { rc = -5; break; }
            memcpy(out_cols + total, cc, sizeof(int32_t) * (size_t)cnt[s]);
            memcpy(out_vals + total, vv, sizeof(double) * (size_t)cnt[s]);
            memcpy(out_abs + total, aa, sizeof(double) * (size_t)cnt[s]);
            total += cnt[s];
            out_ptr[s + 1] = total;
        }
    }
    free(slot); free(cols); free(vals); free(abss); free(cnt); free(A); free(Aa);
    return rc ? rc : total;
}

/* ------------------------------------------------------------------ */
/* Global reductions over cells (PyOP2 Globals: SUM, MIN, MAX)          */
/* ------------------------------------------------------------------ */

/*
 * Per-cell contributions to a Global: the cell energy of the bilinear form,
 * q_K = x_K^T A_K x_K (kind 0; A_K the element matrix of cstiff kappa
 * grad u.grad v + cmass u v, x a field of the P_k space), or the integral of
 * the P1 field f over K (kind 1).  q[c] and its magnitude scale qa[c]; the
 * totals in cell index order go to *sum and *sum_abs.
 */
int oracle_cell_values(int kind, int dim, int degree, int64_t ncells, const int32_t *cell_vertex,
                       const double *coords, const int32_t *cell_node, const double *field, double cstiff,
                       double cmass, const double *x, double *q, double *qa, double *sum, double *sum_abs)
{
    const int n = oracle_nloc(dim, degree);
    if (n < 0) return -1;
    double xv[12], fv[4], A[MAXLOC * MAXLOC], Aa[MAXLOC * MAXLOC], be[MAXLOC], ba[MAXLOC];
    double s = 0.0, sa = 0.0;
    for (int64_t c = 0; c < ncells; ++c) {
        gather_cell(dim, c, cell_vertex, coords, field, xv, fv);
        double t = 0.0, ta = 0.0;
        if (kind == 0) {
            if (oracle_element_matrix(dim, degree, xv, fv, cstiff, cmass, A, Aa)) return -1;
            for (int i = 0; i < n; ++i) {
                const double xi = x[cell_node[c * n + i]];
                for (int j = 0; j < n; ++j) {
                    const double xj = x[cell_node[c * n + j]];
                    t += xi * A[i * n + j] * xj;
                    ta += fabs(xi) * Aa[i * n + j] * fabs(xj);
                }
            }
        } else {
            if (oracle_element_vector(dim, degree, xv, fv, be, ba)) return -1;
            for (int i = 0; i < n; ++i) { t += be[i]; ta += ba[i]; }
        }
        q[c] = t; qa[c] = ta;
        s += t; sa += ta;
    }
    *sum = s; *sum_abs = sa;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Mixed function spaces: the monolithic matrix                          */
/* ------------------------------------------------------------------ */

/*
 * The monolithic matrix of a bilinear form on the mixed space W = V^nf (nf
 * copies of the scalar P_k space V, DOF f*nnodes + node for field f) whose
 * (test field a, trial field b) part is  cstiff[a*nf+b] kappa_ab
 * grad(u_b).grad(v_a) + cmass[a*nf+b] u_b v_a,  kappa_ab the P1 vertex field
 * kap[a*nf+b] (NULL: 1).  The mixed element matrix of each cell is formed
 * over the combined basis (field-major local order) and added entry by entry
 * into the monolithic CSR row_ptr/col_idx (rows nf*nnodes), cells in index
 * order.  This is the single mixed kernel and monolithic matrix that the
 * paper contrasts with Firedrake's split, per-block assembly.
 */
int oracle_mixed_mat(int dim, int degree, int nf, int64_t ncells, const int32_t *cell_vertex, const double *coords,
                     const int32_t *cell_node, int64_t nnodes, const double *const *kap, const double *cstiff,
                     const double *cmass, const int64_t *row_ptr, const int32_t *col_idx, double *values,
                     double *absval)
{
    const int n = oracle_nloc(dim, degree), nv = dim + 1, NN = nf * n;
    if (n < 0 || nf < 1 || nf > 4) return -1;
    const int64_t nnz = row_ptr[nf * nnodes];
    memset(values, 0, sizeof(double) * (size_t)nnz);
    memset(absval, 0, sizeof(double) * (size_t)nnz);
    double *A = malloc(sizeof(double) * NN * NN), *Aa = malloc(sizeof(double) * NN * NN);
    double Ab[MAXLOC * MAXLOC], Aab[MAXLOC * MAXLOC], xv[12], kv[4], dummy[4];
    int rc = 0;
    if (!A || !Aa) rc = -1;
    for (int64_t c = 0; c < ncells && !rc; ++c) {
        gather_cell(dim, c, cell_vertex, coords, NULL, xv, dummy);
        for (int a = 0; a < nf && !rc; ++a)
            for (int b = 0; b < nf && !rc; ++b) {
                const double *kf = kap[a * nf + b];
                for (int m = 0; m < nv; ++m) kv[m] = kf ? kf[cell_vertex[c * nv + m]] : 1.0;
                if (oracle_element_matrix(dim, degree, xv, kv, cstiff[a * nf + b], cmass[a * nf + b], Ab, Aab)) rc = -1;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        A[(int64_t)(a * n + i) * NN + b * n + j] = Ab[i * n + j];
                        Aa[(int64_t)(a * n + i) * NN + b * n + j] = Aab[i * n + j];
                    }
            }
        for (int I = 0; I < NN && !rc; ++I) {
            const int64_t r = (I / n) * nnodes + cell_node[c * n + I % n];
            for (int J = 0; J < NN; ++J) {
                const int64_t k = find_col(row_ptr, col_idx, r, (int32_t)((J / n) * nnodes + cell_node[c * n + J % n]));
                if (k < 0) { rc = -3; break; }
                values[k] += A[(int64_t)I * NN + J];
                absval[k] += Aa[(int64_t)I * NN + J];
            }
        }
    }
    free(A); free(Aa);
    return rc;
}


/* ------------------------------------------------------------------ */
/* Exterior facet integrals                                            */
/* ------------------------------------------------------------------ */

/*
 * b_i = sum over exterior facets F of the integral over F of g v_i ds, g a P1
 * field (vertex values), v_i the degree-k Lagrange basis restricted to F: the
 * basis of the (dim-1)-simplex F in its own local order (facet vertices in
 * the facet_vertex order, then edge nodes, then the P3 triangle's face
 * node).  facet_vertex [nf][dim], facet_node [nf][nloc(dim-1, k)].
 * Quadrature on the reference (dim-1)-simplex with the measure of F:
 * integral over F = |F| (dim-1)! sum_q w_q h(xi_q).
 */
int oracle_facet_vec(int dim, int degree, int64_t nfacets, const int32_t *facet_vertex, const double *coords,
                     const int32_t *facet_node, const double *g, int64_t nrows, double *b, double *babs)
{
    const int e = dim - 1, n = oracle_nloc(e, degree), nv = dim;
    if (n < 0 || e < 1) return -1;
    struct rule R;
    if (make_rule(e, degree + 1, &R)) return -1;
    memset(b, 0, sizeof(double) * (size_t)nrows);
    memset(babs, 0, sizeof(double) * (size_t)nrows);
    for (int64_t f = 0; f < nfacets; ++f) {
        double x[3][3], gv[3];
        for (int m = 0; m < nv; ++m) {
            const int64_t v = facet_vertex[f * nv + m];
            for (int r = 0; r < dim; ++r) x[m][r] = coords[v * dim + r];
            gv[m] = g[v];
        }
        double meas;
        if (e == 1) {
            double s2 = 0.0;
            for (int r = 0; r < dim; ++r) s2 += (x[1][r] - x[0][r]) * (x[1][r] - x[0][r]);
            meas = sqrt(s2);
        } else {
            const double u[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
            const double w[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
            const double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
            meas = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
        }
        const double scale = meas * (e == 2 ? 2.0 : 1.0);     /* |F| (dim-1)! */
        for (int q = 0; q < R.np; ++q) {
            double lam[4], phi[MAXLOC], dphi[MAXLOC * 4];
            double s = 0.0;
            for (int m = 0; m < e; ++m) { lam[m + 1] = R.pts[q * e + m]; s += lam[m + 1]; }
            lam[0] = 1.0 - s;
            oracle_basis(e, degree, lam, phi, dphi);
            double gq = 0.0, ga = 0.0;
            for (int m = 0; m < nv; ++m) { gq += gv[m] * lam[m]; ga += fabs(gv[m] * lam[m]); }
            const double w = R.wts[q] * scale;
            for (int i = 0; i < n; ++i) {
                const int64_t r = facet_node[f * n + i];
                if (r < 0 || r >= nrows) return -2;
                b[r] += w * gq * phi[i];
                babs[r] += fabs(w * phi[i]) * ga;
            }
        }
    }
    return 0;
}
