/*
 * rsm_oracle.c -- CPU oracle of the RSM repetitive task.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes.  The paper models its data-parallel operations (the
 * sparse DGEMV and vector operations of its conjugate-gradient case study,
 * Sec. 7) as repetitive tasks of the MARTE Repetitive Structure Modeling
 * package (named in Sec. 3; the Shaped multiplicity in Sec. 6.1).  The paper
 * does not restate the package's tiler semantics; this file writes out the
 * standard Array-OL / MARTE RSM definition:
 *
 *   index   e(r, i) = (o + P r + F i) mod s      componentwise, floored mod
 *   gather  pat_t(r)[i] = A_t[e_t(r, i)]          for every input tiler t
 *   task    y(r) = T(pat_1(r), pat_2(r), ...)     independently per r
 *   scatter B[e_out(r, j)] = y(r)[j]
 *
 * with r over the repetition space and i, j over the pattern shapes, both in
 * row-major order (dimension 0 slowest).  Arrays are dense row-major.  All
 * arithmetic is FP64 over inputs widened exactly by the caller; the per-output
 * sum of |terms| is returned for tolerance checks.  The adjoint of the linear
 * weighted-sum task follows from the same definition by transposing the
 * gather: gx[e_in(r,i)] += c[i] gy[e_out(r)], gc[i] += gy[e_out(r)] x[e_in(r,i)].
 *
 * The weighted sum may also have an output pattern of q > 1 elements (an
 * elementary task that produces a pattern, as every Array-OL task may: a
 * polyphase filter, where one repetition reads a window and writes several
 * outputs, each with its own taps).  Its coefficients are then a q x |s_p|
 * matrix, row j holding the taps of output element j:
 *     y(r)[j] = sum_i c[j][i] pat(r)[i]
 * and its adjoint is gx[e_in(r,i)] += sum_j c[j][i] gy[e_out(r,j)],
 * gc[j][i] += gy[e_out(r,j)] x[e_in(r,i)].  With q = 1 this is the plain
 * weighted sum above.
 *
 * Nothing here is blocked, fused or reordered: every loop is the definition.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_MAXR 8

typedef struct {
    int32_t arr_rank;
    int32_t pat_rank;
    int64_t shape[OR_MAXR];
    int64_t origin[OR_MAXR];
    int64_t paving[OR_MAXR * OR_MAXR];   /* arr_rank x rep_rank, row-major */
    int64_t fitting[OR_MAXR * OR_MAXR];  /* arr_rank x pat_rank, row-major */
    int64_t pat_shape[OR_MAXR];
} or_tiler;

enum { OR_COPY = 0, OR_SUM = 1, OR_WSUM = 2, OR_DOT = 3 };

/* Floored modulo: result in [0, m) for m > 0, also for negative a. */
static int64_t floor_mod(int64_t a, int64_t m)
{
    int64_t q = a % m;
    if (q < 0) q += m;
    return q;
}

static int64_t prod(const int64_t* v, int n)
{
    int64_t p = 1;
    for (int k = 0; k < n; ++k) p *= v[k];
    return p;
}

/* Row-major multi-index of a flat position. */
static void unflatten(int64_t flat, const int64_t* shape, int n, int64_t* idx)
{
    for (int k = n - 1; k >= 0; --k) {
        idx[k] = flat % shape[k];
        flat /= shape[k];
    }
}

/* e(r, i) as a linear offset into the tiler's array. */
static int64_t element_offset(const or_tiler* t, int rep_rank,
                              const int64_t* r, const int64_t* i)
{
    int64_t lin = 0;
    for (int d = 0; d < t->arr_rank; ++d) {
        int64_t v = t->origin[d];
        for (int k = 0; k < rep_rank; ++k) v += t->paving[d * rep_rank + k] * r[k];
        for (int k = 0; k < t->pat_rank; ++k) v += t->fitting[d * t->pat_rank + k] * i[k];
        lin = lin * t->shape[d] + floor_mod(v, t->shape[d]);
    }
    return lin;
}

/* Index table: out[r_flat * |s_p| + i_flat] = e(r, i) (linear). */
int oracle_indices(int32_t rep_rank, const int64_t* rep_shape,
                   const or_tiler* t, int64_t* out)
{
    int64_t nr = prod(rep_shape, rep_rank);
    int64_t np = prod(t->pat_shape, t->pat_rank);
    int64_t r[OR_MAXR], i[OR_MAXR];
    for (int64_t rf = 0; rf < nr; ++rf) {
        unflatten(rf, rep_shape, rep_rank, r);
        for (int64_t pf = 0; pf < np; ++pf) {
            unflatten(pf, t->pat_shape, t->pat_rank, i);
            out[rf * np + pf] = element_offset(t, rep_rank, r, i);
        }
    }
    return 0;
}

/* y(r) for one repetition; writes n_out values and their |term| sums.
 * Returns 0, or -1 for an unknown task or incompatible pattern sizes. */
static int task_one(int32_t rep_rank, const int64_t* r,
                    int32_t n_in, const or_tiler* in, const double* const* x,
                    int32_t kind, const double* coeffs, int64_t n_out,
                    double* y, double* yabs)
{
    int64_t i[OR_MAXR];
    int64_t np = prod(in[0].pat_shape, in[0].pat_rank);
    if (kind == OR_COPY) {
        if (np != n_out || n_in != 1) return -1;
        for (int64_t pf = 0; pf < np; ++pf) {
            unflatten(pf, in[0].pat_shape, in[0].pat_rank, i);
            y[pf] = x[0][element_offset(&in[0], rep_rank, r, i)];
            yabs[pf] = fabs(y[pf]);
        }
        return 0;
    }
    if (kind == OR_WSUM && n_out > 1) {
        /* output pattern of n_out elements: one row of taps per element */
        if (n_in != 1) return -1;
        for (int64_t jf = 0; jf < n_out; ++jf) {
            double acc = 0.0, aabs = 0.0;
            for (int64_t pf = 0; pf < np; ++pf) {
                unflatten(pf, in[0].pat_shape, in[0].pat_rank, i);
                double term = coeffs[jf * np + pf] * x[0][element_offset(&in[0], rep_rank, r, i)];
                acc += term;
                aabs += fabs(term);
            }
            y[jf] = acc;
            yabs[jf] = aabs;
        }
        return 0;
    }
    if (n_out != 1) return -1;
    double acc = 0.0, aabs = 0.0;
    if (kind == OR_SUM || kind == OR_WSUM) {
        if (n_in != 1) return -1;
        for (int64_t pf = 0; pf < np; ++pf) {
            unflatten(pf, in[0].pat_shape, in[0].pat_rank, i);
            double term = x[0][element_offset(&in[0], rep_rank, r, i)];
            if (kind == OR_WSUM) term *= coeffs[pf];
            acc += term;
            aabs += fabs(term);
        }
    } else if (kind == OR_DOT) {
        if (n_in != 2) return -1;
        if (prod(in[1].pat_shape, in[1].pat_rank) != np) return -1;
        int64_t i2[OR_MAXR];
        for (int64_t pf = 0; pf < np; ++pf) {
            unflatten(pf, in[0].pat_shape, in[0].pat_rank, i);
            unflatten(pf, in[1].pat_shape, in[1].pat_rank, i2);
            double term = x[0][element_offset(&in[0], rep_rank, r, i)]
                        * x[1][element_offset(&in[1], rep_rank, r, i2)];
            acc += term;
            aabs += fabs(term);
        }
    } else {
        return -1;
    }
    y[0] = acc;
    yabs[0] = aabs;
    return 0;
}

/*
 * Full repetitive task.  `out` holds the prior contents of the output array
 * (elements no repetition writes keep them); `hits` (zeroed by the caller)
 * counts writes per output element, so hits > 1 exposes a tiler that is not
 * single-assignment; `out_abs` receives the |term| sum of the value written.
 * Returns 0, or -1 on an unsupported task/shape combination.
 */
int oracle_run(int32_t rep_rank, const int64_t* rep_shape,
               int32_t n_in, const or_tiler* in, const double* const* x,
               const or_tiler* out_t, double* out, int64_t* hits, double* out_abs,
               int32_t kind, const double* coeffs)
{
    int64_t nr = prod(rep_shape, rep_rank);
    int64_t n_out = prod(out_t->pat_shape, out_t->pat_rank);
    double* y = (double*)malloc(sizeof(double) * (size_t)n_out);
    double* ya = (double*)malloc(sizeof(double) * (size_t)n_out);
    int64_t r[OR_MAXR], j[OR_MAXR];
    int rc = 0;
    for (int64_t rf = 0; rf < nr && rc == 0; ++rf) {
        unflatten(rf, rep_shape, rep_rank, r);
        rc = task_one(rep_rank, r, n_in, in, x, kind, coeffs, n_out, y, ya);
        if (rc) break;
        for (int64_t jf = 0; jf < n_out; ++jf) {
            unflatten(jf, out_t->pat_shape, out_t->pat_rank, j);
            int64_t lin = element_offset(out_t, rep_rank, r, j);
            out[lin] = y[jf];
            out_abs[lin] = ya[jf];
            hits[lin] += 1;
        }
    }
    free(y);
    free(ya);
    return rc;
}

/*
 * y(r) for a list of repetitions (flat row-major indices), for checking a few
 * outputs of a task too large to evaluate whole.  y / yabs are [n, |out pattern|].
 */
int oracle_run_sample(int32_t rep_rank, const int64_t* rep_shape,
                      int32_t n_in, const or_tiler* in, const double* const* x,
                      int64_t n_out, int32_t kind, const double* coeffs,
                      int64_t n, const int64_t* rep_flat, double* y, double* yabs)
{
    int64_t r[OR_MAXR];
    for (int64_t s = 0; s < n; ++s) {
        unflatten(rep_flat[s], rep_shape, rep_rank, r);
        int rc = task_one(rep_rank, r, n_in, in, x, kind, coeffs, n_out,
                          y + s * n_out, yabs + s * n_out);
        if (rc) return rc;
    }
    return 0;
}

/*
 * Adjoint of the weighted sum (SUM is the weighted sum with unit weights,
 * coeffs == NULL, and a scalar output pattern).  A weighted sum may have an
 * output pattern of q elements, coeffs then being q x |s_p| (row j = taps of
 * output element j).  gx (array-shaped) and gc (q x |s_p|) are accumulated
 * into (caller zeroes them); *_abs receive the |term| sums for tolerance
 * checks.  gc / gc_abs may be NULL.
 */
int oracle_adjoint(int32_t rep_rank, const int64_t* rep_shape,
                   const or_tiler* in, const double* x,
                   const or_tiler* out_t, const double* gy,
                   const double* coeffs,
                   double* gx, double* gx_abs, double* gc, double* gc_abs)
{
    int64_t nr = prod(rep_shape, rep_rank);
    int64_t np = prod(in->pat_shape, in->pat_rank);
    int64_t nq = prod(out_t->pat_shape, out_t->pat_rank);
    if (nq != 1 && !coeffs) return -1;
    int64_t r[OR_MAXR], i[OR_MAXR], j[OR_MAXR];
    for (int64_t rf = 0; rf < nr; ++rf) {
        unflatten(rf, rep_shape, rep_rank, r);
        for (int64_t jf = 0; jf < nq; ++jf) {
            unflatten(jf, out_t->pat_shape, out_t->pat_rank, j);
            double g = gy[element_offset(out_t, rep_rank, r, j)];
            for (int64_t pf = 0; pf < np; ++pf) {
                unflatten(pf, in->pat_shape, in->pat_rank, i);
                int64_t a = element_offset(in, rep_rank, r, i);
                double c = coeffs ? coeffs[jf * np + pf] : 1.0;
                gx[a] += c * g;
                gx_abs[a] += fabs(c * g);
                if (gc) {
                    gc[jf * np + pf] += g * x[a];
                    gc_abs[jf * np + pf] += fabs(g * x[a]);
                }
            }
        }
    }
    return 0;
}

/*
 * Repetitive task with data-dependent (indirect) tilers: the sparse
 * matrix-vector product of the paper's conjugate-gradient case study (Sec. 7,
 * "DGEMV(sparse)").  Repetition r reads the pattern vals[row_ptr[r] ..
 * row_ptr[r+1]) through a contiguous tiler and x[col_idx[k]] through the
 * indirect one, applies DOT and writes y[r].  yabs[r] = sum of |terms|.
 */
int oracle_run_csr(int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                   const double* vals, const double* x, double* y, double* yabs)
{
    for (int64_t r = 0; r < n_rows; ++r) {
        double acc = 0.0, aabs = 0.0;
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            double term = vals[k] * x[col_idx[k]];
            acc += term;
            aabs += fabs(term);
        }
        y[r] = acc;
        yabs[r] = aabs;
    }
    return 0;
}

/* Plain sequential FP64 inner product. */
static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Conjugate gradient on the CSR matrix, the loop of the paper's case study
 * (Sec. 7): every matrix-vector product is the indirect-tiler task above, the
 * inner products and vector updates are element-wise repetitions, and the
 * loop runs while the continue-condition holds.  The recurrences are the
 * Hestenes-Stiefel ones in the textbook the paper cites (Golub & Van Loan):
 *
 *   r0 = b - A x0,  p0 = r0,  rho0 = <r0, r0>
 *   while ||r_k|| > tol ||b|| and k < max_iter:
 *     q = A p_k;  alpha = rho_k / <p_k, q>
 *     x_{k+1} = x_k + alpha p_k;  r_{k+1} = r_k - alpha q
 *     rho_{k+1} = <r_{k+1}, r_{k+1}>;  beta = rho_{k+1} / rho_k
 *     p_{k+1} = r_{k+1} + beta p_k
 *
 * The relative residual test with tol follows the stopping rule of the
 * paper's Table 1 (tol = 1e-10, Matlab pcg's criterion).  x holds x0 on entry
 * and the last iterate on exit.  res (nullable, max_iter + 1 entries)
 * receives ||r_k||, alpha / beta (nullable, max_iter entries) the step
 * scalars.  Returns the number of iterations taken, or -1 on a breakdown
 * (<p, A p> <= 0: the matrix is not positive definite).
 */
int64_t oracle_cg(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                  const double* vals, const double* b, double* x, double tol,
                  int64_t max_iter, double* res, double* alpha_out, double* beta_out)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double* p = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double* scratch = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    oracle_run_csr(n, row_ptr, col_idx, vals, x, q, scratch);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - q[i];
        p[i] = r[i];
    }
    double rho = dot(n, r, r);
    const double bnorm = sqrt(dot(n, b, b));
    int64_t k = 0;
    if (res) res[0] = sqrt(rho);
    while (k < max_iter && sqrt(rho) > tol * bnorm) {
        oracle_run_csr(n, row_ptr, col_idx, vals, p, q, scratch);
        const double pq = dot(n, p, q);
        if (!(pq > 0.0)) {
            k = -1;
            break;
        }
        const double alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        const double rho_next = dot(n, r, r);
        const double beta = rho_next / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        if (alpha_out) alpha_out[k] = alpha;
        if (beta_out) beta_out[k] = beta;
        rho = rho_next;
        ++k;
        if (res) res[k] = sqrt(rho);
    }
    free(r);
    free(p);
    free(q);
    free(scratch);
    return k;
}
