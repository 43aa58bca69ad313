/*
 * CPU oracle for the P1 pressure system -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path never calls it.  It
 * shares no source with the HIP library: different element formulas
 * (Gaussian elimination instead of an adjugate), an assembled CSR matrix
 * instead of a matrix-free gather, sequential loops throughout.
 *
 * What it computes (paper: Sec. 3.4 "Projection stage", the weak problem):
 * find dP in the P1 space such that for every test function z
 *     alpha * int dP z  +  beta * int c grad dP . grad z  =  rhs(z),
 * with alpha = 1/(gamma-1), beta = dt^2 and c = H piecewise constant per
 * primal element (Sec. 3.3, pre-projection).  The printed weak form carries
 * a minus sign in front of the stiffness integral; Green's formula applied
 * to the strong pressure equation of Sec. 3 gives a plus sign, and only the
 * plus sign yields the symmetric positive definite system the paper
 * states, so the plus sign is used.  The mass matrix is consistent (the
 * paper applies no lumping, Sec. 3.4).  Dirichlet pressure nodes
 * (Sec. 3.6, Neumann boundaries of the finite-volume stage) are imposed by
 * symmetric elimination: their rows and columns are cleared and the
 * diagonal set to 1.  The system is solved by the classical conjugate
 * gradient method (Hestenes-Stiefel; e.g. Saad, Iterative Methods for
 * Sparse Linear Systems, Alg. 6.18), as the paper prescribes (Sec. 3.4).
 *
 * Layout pieces (Morton renumbering, element order, node-to-element lists)
 * are not part of the paper; they are recomputed here from their written
 * definitions so the library's integer work can be compared bit for bit.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_EDEGENERATE (-2)
#define ORC_ENOMEM (-3)
#define ORC_EBREAKDOWN (-4)

/* ------------------------------------------------------------------ */
/* Element geometry: J = [x1-x0, ..., xd-x0] (columns), by elimination. */

/* Invert the d x d matrix J (row-major, J[r*d + c]) by Gauss-Jordan
 * elimination with partial pivoting.  Returns det(J); inv is valid only
 * when the returned determinant is nonzero. */
static double orc_invert(int d, const double *J, double *inv)
{
    double a[3][6];
    double det = 1.0;
    for (int r = 0; r < d; ++r) {
        for (int c = 0; c < d; ++c) {
            a[r][c] = J[r * d + c];
            a[r][d + c] = (r == c) ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < d; ++col) {
        int piv = col;
        for (int r = col + 1; r < d; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return 0.0;
        if (piv != col) {
            for (int c = 0; c < 2 * d; ++c) {
                double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
            det = -det;
        }
        double pv = a[col][col];
        det *= pv;
        for (int c = 0; c < 2 * d; ++c) a[col][c] /= pv;
        for (int r = 0; r < d; ++r) {
            if (r == col) continue;
            double f = a[r][col];
            if (f == 0.0) continue;
            for (int c = 0; c < 2 * d; ++c) a[r][c] -= f * a[col][c];
        }
    }
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) inv[r * d + c] = a[r][d + c];
    return det;
}

static void orc_jacobian(int d, const double *xv, double *J)
{
    /* xv: (d+1) vertices x d coordinates, row-major.  J[r][c] = x_{c+1}[r] - x_0[r]. */
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) J[r * d + c] = xv[(c + 1) * d + r] - xv[r];
}

/* Signed determinant of the element Jacobian. */
double orc_element_det(int dim, const double *xv)
{
    double J[9], inv[9];
    orc_jacobian(dim, xv, J);
    return orc_invert(dim, J, inv);
}

/* Element matrix (row-major (d+1)x(d+1)):
 *   A_ab = beta*c*|T| grad(phi_a).grad(phi_b) + alpha*|T|*(1 + delta_ab)/((d+1)(d+2)),
 * |T| = |det J| / d!, grad(phi_a) = row (a-1) of J^{-1} for a >= 1,
 * grad(phi_0) = -(sum of the others).  Returns the signed det, 0 when degenerate. */
double orc_element_matrix(int dim, const double *xv, double c, double alpha, double beta, double *A)
{
    const int d = dim, nv = dim + 1;
    double J[9], inv[9], g[4][3];
    orc_jacobian(d, xv, J);
    double det = orc_invert(d, J, inv);
    if (det == 0.0 || !isfinite(det)) return 0.0;
    double fact = (d == 2) ? 2.0 : 6.0;
    double vol = fabs(det) / fact;
    for (int k = 0; k < d; ++k) g[0][k] = 0.0;
    for (int a = 1; a < nv; ++a)
        for (int k = 0; k < d; ++k) {
            g[a][k] = inv[(a - 1) * d + k];
            g[0][k] -= g[a][k];
        }
    double mass = alpha * vol / (double)((d + 1) * (d + 2));
    for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
            double dot = 0.0;
            for (int k = 0; k < d; ++k) dot += g[a][k] * g[b][k];
            A[a * nv + b] = beta * c * vol * dot + mass * (a == b ? 2.0 : 1.0);
        }
    return det;
}

static void orc_gather_vertices(int dim, const double *coords, const int32_t *conn, double *xv)
{
    for (int a = 0; a <= dim; ++a)
        for (int k = 0; k < dim; ++k) xv[a * dim + k] = coords[(int64_t)conn[a] * dim + k];
}

/* Check indices, orient elements in place (swap local vertices 1 and 2 when
 * det < 0), reject det == 0.  Returns 0, -1 (bad index) or -2 (degenerate). */
int orc_orient(int dim, int64_t n_nodes, int64_t n_elems, const double *coords, int32_t *elems)
{
    const int nv = dim + 1;
    double xv[12];
    for (int64_t e = 0; e < n_elems; ++e) {
        int32_t *cn = elems + e * nv;
        for (int a = 0; a < nv; ++a)
            if (cn[a] < 0 || cn[a] >= n_nodes) return ORC_EINVAL;
        orc_gather_vertices(dim, coords, cn, xv);
        double det = orc_element_det(dim, xv);
        if (det == 0.0 || !isfinite(det)) return ORC_EDEGENERATE;
        if (det < 0.0) {
            int32_t t = cn[1];
            cn[1] = cn[2];
            cn[2] = t;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Assembled operator A_D in CSR.                                      */

typedef struct {
    int64_t n;
    int64_t *rowptr;
    int32_t *col;
    double *val;
} orc_csr;

void orc_csr_free(void *h);

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Node -> element incidence by counting (elements ascending in each list). */
static int orc_incidence(int dim, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                         int64_t **off_out, int64_t **lst_out)
{
    const int nv = dim + 1;
    int64_t *off = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t *lst = malloc(sizeof(int64_t) * (size_t)(n_elems * nv + 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    if (!off || !lst || !fill) {
        free(off); free(lst); free(fill);
        return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < nv; ++a) off[elems[e * nv + a] + 1]++;
    for (int64_t i = 0; i < n_nodes; ++i) off[i + 1] += off[i];
    memcpy(fill, off, sizeof(int64_t) * (size_t)n_nodes);
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < nv; ++a) {
            int32_t v = elems[e * nv + a];
            lst[fill[v]++] = e * nv + a;
        }
    free(fill);
    *off_out = off;
    *lst_out = lst;
    return ORC_OK;
}

/* Build the sparsity pattern and values of A_D.  The caller frees with
 * orc_csr_free.  Duplicate contributions are summed in ascending element
 * order.  Returns NULL on failure (bad input or no memory). */
void *orc_assemble(int dim, int64_t n_nodes, int64_t n_elems, const double *coords,
                   const int32_t *elems, const double *coef, double alpha, double beta,
                   const uint8_t *dirichlet)
{
    const int nv = dim + 1;
    if (dim != 2 && dim != 3) return NULL;
    int64_t *ioff = NULL, *ilst = NULL;
    if (orc_incidence(dim, n_nodes, n_elems, elems, &ioff, &ilst) != ORC_OK) return NULL;

    orc_csr *A = calloc(1, sizeof(orc_csr));
    A->n = n_nodes;
    A->rowptr = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int32_t *scratch = malloc(sizeof(int32_t) * 4096);
    int64_t cap = n_nodes * 16 + 16, used = 0;
    A->col = malloc(sizeof(int32_t) * (size_t)cap);
    /* Pattern: sorted unique neighbours (incl. self) of every node. */
    for (int64_t i = 0; i < n_nodes; ++i) {
        int64_t cnt = 0;
        for (int64_t k = ioff[i]; k < ioff[i + 1]; ++k) {
            int64_t e = ilst[k] / nv;
            for (int b = 0; b < nv; ++b) {
                if (cnt < 4096) scratch[cnt] = elems[e * nv + b];
                cnt++;
            }
        }
        if (cnt == 0) { scratch[0] = (int32_t)i; cnt = 1; }
        if (cnt > 4096) { free(scratch); free(ioff); free(ilst); free(A->rowptr); free(A->col); free(A); return NULL; }
        qsort(scratch, (size_t)cnt, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t k = 0; k < cnt; ++k)
            if (u == 0 || scratch[k] != scratch[u - 1]) scratch[u++] = scratch[k];
        if (used + u > cap) {
            cap = 2 * cap + u;
            A->col = realloc(A->col, sizeof(int32_t) * (size_t)cap);
        }
        memcpy(A->col + used, scratch, sizeof(int32_t) * (size_t)u);
        used += u;
        A->rowptr[i + 1] = used;
    }
    free(scratch);
    A->val = calloc((size_t)used + 1, sizeof(double));
    /* Values: element by element, ascending element index. */
    double xv[12], Ae[16];
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *cn = elems + e * nv;
        orc_gather_vertices(dim, coords, cn, xv);
        if (orc_element_matrix(dim, xv, coef[e], alpha, beta, Ae) == 0.0) {
            free(ioff); free(ilst);
            orc_csr_free(A);
            return NULL;
        }
        for (int a = 0; a < nv; ++a) {
            int32_t row = cn[a];
            int64_t lo = A->rowptr[row], hi = A->rowptr[row + 1];
            for (int b = 0; b < nv; ++b) {
                int32_t colid = cn[b];
                int64_t L = lo, H = hi - 1;
                while (L < H) {
                    int64_t M = (L + H) / 2;
                    if (A->col[M] < colid) L = M + 1; else H = M;
                }
                A->val[L] += Ae[a * nv + b];
            }
        }
    }
    /* Symmetric elimination of the Dirichlet nodes. */
    if (dirichlet) {
        for (int64_t i = 0; i < n_nodes; ++i)
            for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
                int32_t j = A->col[k];
                if (dirichlet[i] || dirichlet[j]) A->val[k] = (i == j) ? 1.0 : 0.0;
            }
    }
    free(ioff);
    free(ilst);
    return A;
}

int64_t orc_csr_nnz(const void *h) { const orc_csr *A = h; return A->rowptr[A->n]; }

void orc_csr_export(const void *h, int64_t *rowptr, int32_t *col, double *val)
{
    const orc_csr *A = h;
    memcpy(rowptr, A->rowptr, sizeof(int64_t) * (size_t)(A->n + 1));
    memcpy(col, A->col, sizeof(int32_t) * (size_t)A->rowptr[A->n]);
    memcpy(val, A->val, sizeof(double) * (size_t)A->rowptr[A->n]);
}

/* A CSR handle holding a copy of the given arrays (an operator formed
 * outside this file, e.g. the merged operator of a periodic mesh). */
void *orc_csr_from(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val)
{
    orc_csr *A = calloc(1, sizeof(orc_csr));
    if (!A) return NULL;
    const int64_t nnz = rowptr[n];
    A->n = n;
    A->rowptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    A->col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    A->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!A->rowptr || !A->col || !A->val) {
        orc_csr_free(A);
        return NULL;
    }
    memcpy(A->rowptr, rowptr, sizeof(int64_t) * (size_t)(n + 1));
    memcpy(A->col, col, sizeof(int32_t) * (size_t)nnz);
    memcpy(A->val, val, sizeof(double) * (size_t)nnz);
    return A;
}

void orc_csr_free(void *h)
{
    orc_csr *A = h;
    if (!A) return;
    free(A->rowptr);
    free(A->col);
    free(A->val);
    free(A);
}

/* Host threads of the CG loops (the CPU baseline's all-core leg; default
 * 1).  With T > 1 the SpMV rows and the vector updates are split over T
 * OpenMP threads (each row still sums in CSR order, so the SpMV gives the
 * same bits), and a dot product is the sum, in chunk order, of T sequential
 * sums over contiguous chunks: a fixed order for a given T. */
static int orc_nthreads = 1;

void orc_set_threads(int t) { orc_nthreads = t < 1 ? 1 : t; }

void orc_spmv(const void *h, const double *x, double *y)
{
    const orc_csr *A = h;
    const int T = orc_nthreads;
#pragma omp parallel for schedule(static) num_threads(T) if (T > 1)
    for (int64_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) s += A->val[k] * x[A->col[k]];
        y[i] = s;
    }
}

static double orc_dot(int64_t n, const double *a, const double *b)
{
    const int T = orc_nthreads;
    if (T == 1) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
        return s;
    }
    double part[256];
    const int nc = T < 256 ? T : 256;
#pragma omp parallel for schedule(static, 1) num_threads(T)
    for (int c = 0; c < nc; ++c) {
        const int64_t lo = n * c / nc, hi = n * (c + 1) / nc;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += part[c];
    return s;
}

/* ------------------------------------------------------------------ */
/* Conjugate gradient on the assembled A_D.
 *
 * r0 = b - A x0, p0 = r0; while ||r_k|| > rtol ||b|| and k < max_iter:
 *   q = A p, a = r.r / p.q (breakdown if p.q <= 0), x += a p, r -= a q,
 *   beta = r'.r' / r.r, p = r' + beta p.
 * hist[k] = ||r_k|| / ||b|| (capacity max_iter + 1).  When the recursive
 * residual has converged the true residual ||b - A x|| / ||b|| is computed;
 * if it is above rtol the residual is replaced by the true one and the
 * iteration resumes (at most twice).  Dirichlet rows start from x_B = b_B.
 * b = 0 gives x = 0 after 0 iterations. */
int orc_cg(const void *h, const uint8_t *dirichlet, const double *b, double *x,
           double rtol, int32_t max_iter, double *hist, int32_t *iters, double *true_relres)
{
    const orc_csr *A = h;
    const int64_t n = A->n;
    if (!(rtol > 0.0) || max_iter < 0) return ORC_EINVAL;
    double bnorm = sqrt(orc_dot(n, b, b));
    if (!isfinite(bnorm)) return ORC_EINVAL;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        *iters = 0;
        if (hist) hist[0] = 0.0;
        *true_relres = 0.0;
        return ORC_OK;
    }
    if (dirichlet)
        for (int64_t i = 0; i < n; ++i)
            if (dirichlet[i]) x[i] = b[i];
    double *r = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    if (!r || !p || !q) { free(r); free(p); free(q); return ORC_ENOMEM; }
    orc_spmv(A, x, q);
    for (int64_t i = 0; i < n; ++i) { r[i] = b[i] - q[i]; p[i] = r[i]; }
    double rr = orc_dot(n, r, r);
    int32_t k = 0;
    int replaced = 0, status = ORC_OK;
    if (hist) hist[0] = sqrt(rr) / bnorm;
    double tres = 0.0;
    for (;;) {
        while (sqrt(rr) > rtol * bnorm && k < max_iter) {
            orc_spmv(A, p, q);
            double pq = orc_dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; goto done; }
            double a = rr / pq;
            const int T = orc_nthreads;
#pragma omp parallel for schedule(static) num_threads(T) if (T > 1)
            for (int64_t i = 0; i < n; ++i) { x[i] += a * p[i]; r[i] -= a * q[i]; }
            double rr1 = orc_dot(n, r, r);
            double bt = rr1 / rr;
            rr = rr1;
#pragma omp parallel for schedule(static) num_threads(T) if (T > 1)
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + bt * p[i];
            ++k;
            if (hist) hist[k] = sqrt(rr) / bnorm;
        }
        orc_spmv(A, x, q);
        for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
        tres = sqrt(orc_dot(n, q, q)) / bnorm;
        if (tres <= rtol || replaced >= 2 || k >= max_iter) break;
        /* residual replacement */
        for (int64_t i = 0; i < n; ++i) { r[i] = q[i]; p[i] = q[i]; }
        rr = orc_dot(n, r, r);
        replaced++;
    }
    status = (tres <= rtol) ? ORC_OK : ORC_NOT_CONVERGED;
done:
    *iters = k;
    *true_relres = tres;
    free(r); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Mixed precision: FP64 defect correction around an FP32 inner CG.
 *
 * outer: r = b - A x (FP64); stop when ||r|| <= rtol ||b||;
 * inner: CG on A32 d = r32, A32 = the FP64 entries rounded to FP32,
 *        FP32 vectors, dot products accumulated in FP64, stopped when the
 *        inner residual is below inner_rtol * ||r32||;
 * update: x += d in FP64.  Returns the total number of inner iterations in
 * *inner_iters and the number of outer steps in *outer_iters. */
int orc_cg_mixed(const void *h, const uint8_t *dirichlet, const double *b, double *x,
                 double rtol, double inner_rtol, int32_t max_outer, int32_t max_inner,
                 int32_t *outer_iters, int32_t *inner_iters, double *true_relres)
{
    const orc_csr *A = h;
    const int64_t n = A->n, nnz = A->rowptr[n];
    double bnorm = sqrt(orc_dot(n, b, b));
    *outer_iters = 0;
    *inner_iters = 0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        *true_relres = 0.0;
        return ORC_OK;
    }
    if (dirichlet)
        for (int64_t i = 0; i < n; ++i)
            if (dirichlet[i]) x[i] = b[i];
    float *v32 = malloc(sizeof(float) * (size_t)nnz);
    double *r = malloc(sizeof(double) * (size_t)n);
    float *rf = malloc(sizeof(float) * (size_t)n), *d = malloc(sizeof(float) * (size_t)n);
    float *s = malloc(sizeof(float) * (size_t)n), *p = malloc(sizeof(float) * (size_t)n);
    float *q = malloc(sizeof(float) * (size_t)n);
    for (int64_t k = 0; k < nnz; ++k) v32[k] = (float)A->val[k];
    int status = ORC_NOT_CONVERGED;
    double tres = 0.0;
    for (int32_t o = 0; o <= max_outer; ++o) {
        orc_spmv(A, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        tres = sqrt(orc_dot(n, r, r)) / bnorm;
        if (tres <= rtol) { status = ORC_OK; break; }
        if (o == max_outer) break;
        *outer_iters = o + 1;
        /* inner FP32 CG from d = 0 */
        double s2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            rf[i] = (float)r[i];
            d[i] = 0.0f;
            s[i] = rf[i];
            p[i] = rf[i];
            s2 += (double)s[i] * (double)s[i];
        }
        double r0 = sqrt(s2);
        int32_t it = 0;
        while (sqrt(s2) > inner_rtol * r0 && it < max_inner) {
            double pq = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                float acc = 0.0f;
                for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) acc += v32[k] * p[A->col[k]];
                q[i] = acc;
                pq += (double)p[i] * (double)acc;
            }
            if (!(pq > 0.0)) break;
            float a = (float)(s2 / pq);
            double s2n = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                d[i] += a * p[i];
                s[i] -= a * q[i];
                s2n += (double)s[i] * (double)s[i];
            }
            float bt = (float)(s2n / s2);
            s2 = s2n;
            for (int64_t i = 0; i < n; ++i) p[i] = s[i] + bt * p[i];
            ++it;
        }
        *inner_iters += it;
        for (int64_t i = 0; i < n; ++i) x[i] += (double)d[i];
    }
    *true_relres = tres;
    free(v32); free(r); free(rf); free(d); free(s); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Matrix-free definition of y = A_D x, element by element (no assembly),
 * for sizes where the assembled matrix is too large.  Free rows:
 *   y_i = sum_{e containing i} sum_b A^e_{ib} x_b  with x_b = 0 for Dirichlet b;
 * Dirichlet rows: y_i = x_i.  If rows != NULL only those rows are computed
 * (out[k] = y_{rows[k]}). */
int orc_apply_elements(int dim, int64_t n_nodes, int64_t n_elems, const double *coords,
                       const int32_t *elems, const double *coef, double alpha, double beta,
                       const uint8_t *dirichlet, const double *x, double *y,
                       const int64_t *rows, int64_t n_rows, double *out)
{
    const int nv = dim + 1;
    double xv[12], Ae[16];
    if (rows == NULL) {
        for (int64_t i = 0; i < n_nodes; ++i) y[i] = 0.0;
        for (int64_t e = 0; e < n_elems; ++e) {
            const int32_t *cn = elems + e * nv;
            orc_gather_vertices(dim, coords, cn, xv);
            if (orc_element_matrix(dim, xv, coef[e], alpha, beta, Ae) == 0.0) return ORC_EDEGENERATE;
            for (int a = 0; a < nv; ++a) {
                if (dirichlet && dirichlet[cn[a]]) continue;
                double s = 0.0;
                for (int b = 0; b < nv; ++b)
                    if (!(dirichlet && dirichlet[cn[b]])) s += Ae[a * nv + b] * x[cn[b]];
                y[cn[a]] += s;
            }
        }
        if (dirichlet)
            for (int64_t i = 0; i < n_nodes; ++i)
                if (dirichlet[i]) y[i] = x[i];
        return ORC_OK;
    }
    int64_t *ioff = NULL, *ilst = NULL;
    if (orc_incidence(dim, n_nodes, n_elems, elems, &ioff, &ilst) != ORC_OK) return ORC_ENOMEM;
    for (int64_t k = 0; k < n_rows; ++k) {
        int64_t i = rows[k];
        if (dirichlet && dirichlet[i]) { out[k] = x[i]; continue; }
        double s = 0.0;
        for (int64_t t = ioff[i]; t < ioff[i + 1]; ++t) {
            int64_t e = ilst[t] / nv;
            int a = (int)(ilst[t] % nv);
            const int32_t *cn = elems + e * nv;
            orc_gather_vertices(dim, coords, cn, xv);
            orc_element_matrix(dim, xv, coef[e], alpha, beta, Ae);
            for (int b = 0; b < nv; ++b)
                if (!(dirichlet && dirichlet[cn[b]])) s += Ae[a * nv + b] * x[cn[b]];
        }
        out[k] = s;
    }
    free(ioff);
    free(ilst);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Layout definitions (integer, compared bit for bit with the library).
 *
 * Morton key of a node: bit b of its per-axis integer coordinate q_ax is
 * placed at bit (dim*b + ax) of the key (x in the lowest bit).  q is the
 * lattice coordinate when given, else
 *   q_ax = floor(((x_ax - min_ax) / (max_ax - min_ax)) * 2097151.0)
 * (0 when max_ax == min_ax).  Nodes are ordered by (key, old id); the new
 * id of a node is its rank.  Elements are ordered by (smallest new vertex
 * id, old id).  The node-to-element list of new node i holds
 * 4*e + a for every new element e whose local vertex a is i, ascending. */

typedef struct { uint64_t key; int64_t id; } orc_kv;

static int cmp_kv(const void *a, const void *b)
{
    const orc_kv *x = a, *y = b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->id > y->id) - (x->id < y->id);
}

static uint64_t orc_interleave(int dim, const uint32_t *q)
{
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b)
        for (int ax = 0; ax < dim; ++ax)
            if ((q[ax] >> b) & 1u) key |= (uint64_t)1 << (dim * b + ax);
    return key;
}

int orc_layout(int dim, int64_t n_nodes, int64_t n_elems, const double *coords,
               const int32_t *lattice, const int32_t *elems_oriented,
               int32_t *node_new2old, int32_t *elem_new2old, int32_t *elems_new,
               int32_t *n2e_off, int32_t *n2e_ent)
{
    const int nv = dim + 1;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (!lattice) {
        for (int ax = 0; ax < dim; ++ax) { lo[ax] = INFINITY; hi[ax] = -INFINITY; }
        for (int64_t i = 0; i < n_nodes; ++i)
            for (int ax = 0; ax < dim; ++ax) {
                double v = coords[i * dim + ax];
                if (v < lo[ax]) lo[ax] = v;
                if (v > hi[ax]) hi[ax] = v;
            }
    }
    orc_kv *kv = malloc(sizeof(orc_kv) * (size_t)(n_nodes > n_elems ? n_nodes : n_elems));
    int32_t *old2new = malloc(sizeof(int32_t) * (size_t)n_nodes);
    if (!kv || !old2new) { free(kv); free(old2new); return ORC_ENOMEM; }
    for (int64_t i = 0; i < n_nodes; ++i) {
        uint32_t q[3] = {0, 0, 0};
        for (int ax = 0; ax < dim; ++ax) {
            if (lattice) {
                int32_t v = lattice[i * dim + ax];
                if (v < 0 || v > 2097151) { free(kv); free(old2new); return ORC_EINVAL; }
                q[ax] = (uint32_t)v;
            } else if (hi[ax] > lo[ax]) {
                double t = ((coords[i * dim + ax] - lo[ax]) / (hi[ax] - lo[ax])) * 2097151.0;
                q[ax] = (uint32_t)floor(t);
            }
        }
        kv[i].key = orc_interleave(dim, q);
        kv[i].id = i;
    }
    qsort(kv, (size_t)n_nodes, sizeof(orc_kv), cmp_kv);
    for (int64_t r = 0; r < n_nodes; ++r) {
        node_new2old[r] = (int32_t)kv[r].id;
        old2new[kv[r].id] = (int32_t)r;
    }
    for (int64_t e = 0; e < n_elems; ++e) {
        int32_t mn = INT32_MAX;
        for (int a = 0; a < nv; ++a) {
            int32_t v = old2new[elems_oriented[e * nv + a]];
            if (v < mn) mn = v;
        }
        kv[e].key = (uint64_t)mn;
        kv[e].id = e;
    }
    qsort(kv, (size_t)n_elems, sizeof(orc_kv), cmp_kv);
    for (int64_t r = 0; r < n_elems; ++r) {
        elem_new2old[r] = (int32_t)kv[r].id;
        for (int a = 0; a < nv; ++a) elems_new[r * nv + a] = old2new[elems_oriented[kv[r].id * nv + a]];
    }
    for (int64_t i = 0; i <= n_nodes; ++i) n2e_off[i] = 0;
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < nv; ++a) n2e_off[elems_new[e * nv + a] + 1]++;
    for (int64_t i = 0; i < n_nodes; ++i) n2e_off[i + 1] += n2e_off[i];
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)(n_nodes + 1));
    memcpy(fill, n2e_off, sizeof(int32_t) * (size_t)n_nodes);
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < nv; ++a) {
            int32_t v = elems_new[e * nv + a];
            n2e_ent[fill[v]++] = (int32_t)(4 * e + a);
        }
    free(fill);
    free(kv);
    free(old2new);
    return ORC_OK;
}
