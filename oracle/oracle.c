/*
 * Batched Krylov oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential FP64 implementation of what the fused batched
 * solver computes, written from the paper (Nguyen, Nayak, Anzt, "Porting
 * Batched Iterative Solvers onto Intel GPUs with SYCL", SC-W 2023) and the
 * textbook methods it composes (Saad 2003; van der Vorst 1992).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code with the HIP library.
 *
 * Rules kept on purpose so a reader can check it by eye:
 *   - every sum is a left-to-right loop in storage order, no blocking;
 *   - built with -ffp-contract=off: products are rounded before they are added;
 *   - one system at a time; OpenMP only distributes whole systems.
 *
 * Readings of the paper used here (it is silent on them):
 *   - stop test: ||r||_2 <= tol * ||b||_2 (relative) or ||r||_2 <= tol
 *     (absolute; Tab. 2 lists both criteria) on the recurrence residual, then a
 *     confirmation on the true residual b - A x; if that fails and iterations
 *     remain, the method restarts from the true residual;
 *   - BiCGSTAB and GMRES are right-preconditioned, so the monitored residual is
 *     the unpreconditioned one; CG follows Sec. 3.5, Alg. 1, step for step;
 *   - a BiCGSTAB half step that already meets the test counts as a full
 *     iteration; GMRES counts Arnoldi steps across restarts;
 *   - breakdown means an exact zero of the quantity that is divided by;
 *   - scalar Jacobi uses 1 where the diagonal entry is zero or not stored;
 *   - ILU(0) is the incomplete factorization on the pattern of A (Saad 2003,
 *     Sec. 10.3.2), without pivoting; if a pivot is zero or an entry of the
 *     factors is not finite, the system is solved without a preconditioner;
 *   - BatchTrsv solves with the lower (or upper) triangle of A, diagonal
 *     included; a zero or absent diagonal entry is a breakdown (x = 0);
 *   - ||b|| = 0 returns x = 0 with zero iterations, converged.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_CSR = 0, OR_ELL = 1 };
enum { OR_CG = 0, OR_BICGSTAB = 1, OR_GMRES = 2, OR_TRSV_LOWER = 3, OR_TRSV_UPPER = 4 };
/* OR_PREC_ILU_COL: ILU(0) with the column-oriented backward substitution (the
 * same factors and operations, the backward sums taken in decreasing column
 * order); the library computes only OR_PREC_ILU's result, the oracle offers
 * both orders so that a test can see how far rounding order alone moves a
 * solve. */
enum { OR_PREC_NONE = 0, OR_PREC_JACOBI = 1, OR_PREC_BLOCK_JACOBI = 2, OR_PREC_ILU = 3,
       OR_PREC_ILU_COL = 4 };
enum { OR_MAX_BLOCK = 16 };
enum { OR_CONVERGED = 0, OR_MAX_ITER = 1, OR_BREAKDOWN = 2, OR_NONFINITE = 3 };

/* One system's matrix: the shared pattern plus this system's values.
 * BatchCsr (Sec. 3.1): row_ptr[n+1], col[nnz], val[nnz].
 * BatchEll (Sec. 3.1): ecol[W][n] slot-major ("column-major" in the paper),
 * padding marked by column -1, val[W][n] in the same layout.              */
typedef struct {
    int fmt, n, width;
    const int *row_ptr, *col, *ecol;
    const double *val;
} or_mat;

/* y = A x, each row summed in storage order. */
static void spmv(const or_mat *A, const double *x, double *y)
{
    int n = A->n;
    if (A->fmt == OR_CSR) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                acc += A->val[k] * x[A->col[k]];
            y[i] = acc;
        }
    } else {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int s = 0; s < A->width; ++s) {
                int c = A->ecol[(size_t)s * n + i];
                if (c >= 0) acc += A->val[(size_t)s * n + i] * x[c];
            }
            y[i] = acc;
        }
    }
}

static double dot(int n, const double *a, const double *b)
{
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

/* Scalar Jacobi (Tab. 2): d_i = 1 / a_ii, or 1 if a_ii is zero or absent. */
static void jacobi_diag(const or_mat *A, int precond, double *d)
{
    int n = A->n;
    for (int i = 0; i < n; ++i) d[i] = 1.0;
    if (precond != OR_PREC_JACOBI) return;
    for (int i = 0; i < n; ++i) {
        double a = 0.0;
        int found = 0;
        if (A->fmt == OR_CSR) {
            for (int k = A->row_ptr[i]; k < A->row_ptr[i + 1] && !found; ++k)
                if (A->col[k] == i) { a = A->val[k]; found = 1; }
        } else {
            for (int s = 0; s < A->width && !found; ++s)
                if (A->ecol[(size_t)s * n + i] == i) { a = A->val[(size_t)s * n + i]; found = 1; }
        }
        if (found && a != 0.0) d[i] = 1.0 / a;
    }
}

/* Block Jacobi: blocks of bs consecutive rows (the last one may be shorter);
 * D_b = the entries of A in the rows and columns of block b (absent entries
 * zero).  Its inverse by Gauss-Jordan elimination of [D_b | I] without
 * pivoting: for each pivot p, divide row p by its pivot, then subtract
 * multiples of it from every other row.  A zero or non-finite pivot, or a
 * non-finite entry of the result, makes the block the identity (as scalar
 * Jacobi takes 1 for a zero diagonal).  inv[i*bs + j] = entry (i, b0 + j) of
 * the inverse for row i of block b0 (0 past the last row).  work: 2*bs*bs. */
static void block_jacobi(const or_mat *A, int bs, double *inv, double *work)
{
    int n = A->n;
    for (int b0 = 0; b0 < n; b0 += bs) {
        int m = n - b0 < bs ? n - b0 : bs, w2 = 2 * m, ok = 1;
        double *G = work;                               /* m x 2m, row-major */
        for (int r = 0; r < m; ++r) {
            for (int c = 0; c < w2; ++c) G[r * w2 + c] = 0.0;
            G[r * w2 + m + r] = 1.0;
            int i = b0 + r;
            if (A->fmt == OR_CSR) {
                for (int k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                    if (A->col[k] >= b0 && A->col[k] < b0 + m) G[r * w2 + A->col[k] - b0] = A->val[k];
            } else {
                for (int sl = 0; sl < A->width; ++sl) {
                    int c = A->ecol[(size_t)sl * n + i];
                    if (c >= b0 && c < b0 + m) G[r * w2 + c - b0] = A->val[(size_t)sl * n + i];
                }
            }
        }
        for (int p = 0; p < m && ok; ++p) {
            double piv = G[p * w2 + p];
            if (piv == 0.0 || !isfinite(piv)) { ok = 0; break; }
            for (int c = 0; c < w2; ++c) G[p * w2 + c] = G[p * w2 + c] / piv;
            for (int r = 0; r < m; ++r) {
                if (r == p) continue;
                double f = G[r * w2 + p];
                for (int c = 0; c < w2; ++c) G[r * w2 + c] = G[r * w2 + c] - f * G[p * w2 + c];
            }
        }
        for (int r = 0; r < m && ok; ++r)
            for (int c = 0; c < m; ++c)
                if (!isfinite(G[r * w2 + m + c])) ok = 0;
        for (int r = 0; r < m; ++r)
            for (int j = 0; j < bs; ++j)
                inv[(size_t)(b0 + r) * bs + j] =
                    j >= m ? 0.0 : ok ? G[r * w2 + m + j] : (j == r ? 1.0 : 0.0);
    }
}

/* A as a dense row-major n x n array F (absent entries 0) and its pattern as
 * a 0/1 mask P of the same shape. */
static void to_dense(const or_mat *A, double *F, unsigned char *P)
{
    int n = A->n;
    for (size_t e = 0; e < (size_t)n * n; ++e) { F[e] = 0.0; P[e] = 0; }
    for (int i = 0; i < n; ++i) {
        if (A->fmt == OR_CSR) {
            for (int k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
                F[(size_t)i * n + A->col[k]] = A->val[k];
                P[(size_t)i * n + A->col[k]] = 1;
            }
        } else {
            for (int s = 0; s < A->width; ++s) {
                int c = A->ecol[(size_t)s * n + i];
                if (c < 0) continue;
                F[(size_t)i * n + c] = A->val[(size_t)s * n + i];
                P[(size_t)i * n + c] = 1;
            }
        }
    }
}

/* ILU(0) (Tab. 2's BatchIlu; Saad 2003, Sec. 10.3.2, the IKJ form): on the
 * dense copy F of A, for each row i and each k < i in the pattern of row i,
 * in increasing k: F_ik /= F_kk, then F_ij -= F_ik F_kj for every j > k in the
 * pattern of row i (F_kj is zero off the pattern, as it is never written).
 * Afterwards F holds L (strictly below the diagonal, unit diagonal implied)
 * and U (diagonal and above).  Returns 1, or 0 if a pivot F_kk is zero or an
 * entry of the factors is not finite. */
static int ilu0(int n, double *F, const unsigned char *P)
{
    for (int i = 1; i < n; ++i)
        for (int k = 0; k < i; ++k) {
            if (!P[(size_t)i * n + k]) continue;
            F[(size_t)i * n + k] = F[(size_t)i * n + k] / F[(size_t)k * n + k];
            for (int j = k + 1; j < n; ++j)
                if (P[(size_t)i * n + j])
                    F[(size_t)i * n + j] = F[(size_t)i * n + j] -
                                           F[(size_t)i * n + k] * F[(size_t)k * n + j];
        }
    for (int k = 0; k < n; ++k)
        if (F[(size_t)k * n + k] == 0.0) return 0;
    for (size_t e = 0; e < (size_t)n * n; ++e)
        if (P[e] && !isfinite(F[e])) return 0;
    return 1;
}

/* z = (L U)^{-1} v: forward substitution with the unit lower factor, then
 * backward substitution with the upper one.  The forward sums run in
 * increasing column order over the pattern.  The backward substitution is
 * row-oriented (row i sums its terms u_ij z_j in increasing j, then divides by
 * u_ii) unless col is set; then it is column-oriented (the other textbook
 * form: z_j is divided by u_jj as soon as column j is reached, and every row
 * above subtracts u_ij z_j, so row i takes its terms in decreasing j).  Both
 * are the same operations in a different order. */
static void ilu_apply(int n, const double *F, const unsigned char *P, const double *v, double *z,
                      int col)
{
    for (int i = 0; i < n; ++i) {
        double acc = v[i];
        for (int k = 0; k < i; ++k)
            if (P[(size_t)i * n + k]) acc = acc - F[(size_t)i * n + k] * z[k];
        z[i] = acc;
    }
    if (col) {
        for (int j = n - 1; j >= 0; --j) {
            z[j] = z[j] / F[(size_t)j * n + j];
            for (int i = 0; i < j; ++i)
                if (P[(size_t)i * n + j]) z[i] = z[i] - F[(size_t)i * n + j] * z[j];
        }
        return;
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc = z[i];
        for (int j = i + 1; j < n; ++j)
            if (P[(size_t)i * n + j]) acc = acc - F[(size_t)i * n + j] * z[j];
        z[i] = acc / F[(size_t)i * n + i];
    }
}

/* The preconditioner as solvers apply it: z = M v, with M = diag(d) (scalar
 * Jacobi, or d = 1 for none), the block-Jacobi inverse (bs > 1) or the ILU(0)
 * factors (lu non-null). */
typedef struct { int bs, col; const double *d, *inv, *lu; const unsigned char *mask; } or_prec;

static void prec_apply(const or_prec *M, int n, const double *v, double *z)
{
    if (M->lu) {
        ilu_apply(n, M->lu, M->mask, v, z, M->col);
        return;
    }
    if (M->bs <= 1) {
        for (int i = 0; i < n; ++i) z[i] = M->d[i] * v[i];
        return;
    }
    for (int i = 0; i < n; ++i) {
        int b0 = i - i % M->bs;
        const double *row = M->inv + (size_t)i * M->bs;
        double acc = 0.0;
        for (int j = 0; j < M->bs && b0 + j < n; ++j) acc += row[j] * v[b0 + j];
        z[i] = acc;
    }
}

/* r = b - A x, returns ||r||_2; t is scratch. */
static double true_residual(const or_mat *A, const double *b, const double *x,
                            double *r, double *t)
{
    spmv(A, x, t);
    for (int i = 0; i < A->n; ++i) r[i] = b[i] - t[i];
    return nrm2(A->n, r);
}

typedef struct { int iters, status; double resid; } or_result;

/* Common exit: report the true residual of the returned x divided by rs
 * (||b||_2 for the relative criterion, 1 for the absolute one). */
static or_result finish(const or_mat *A, const double *b, const double *x, double rs,
                        int k, int status, double *r, double *t)
{
    or_result res;
    res.iters = k;
    res.status = status;
    res.resid = true_residual(A, b, x, r, t) / rs;
    return res;
}

/* Restart log (reading P2): when log is not NULL, log[0] counts the restarts
 * from the true residual and log[1..cap-1] receive the iteration count at
 * which each of the first cap-1 of them happened.  It only records; it never
 * changes what the solvers compute. */
static void log_restart(int *log, int cap, int k)
{
    if (!log) return;
    if (log[0] + 1 < cap) log[log[0] + 1] = k;
    log[0] += 1;
}

/* ---- CG: Sec. 3.5, Alg. 1, with the residual-norm stop test ------------ */
static or_result solve_cg(const or_mat *A, const or_prec *M, const double *b, double *x,
                          double rs, double lim, int max_iter, double *ws, int *log, int cap)
{
    int n = A->n, k = 0, r_true;
    double *r = ws, *z = ws + n, *p = ws + 2 * n, *t = ws + 3 * n;
    double rho, rn;

    rn = true_residual(A, b, x, r, t);
    r_true = 1;
restart:
    prec_apply(M, n, r, z);
    for (int i = 0; i < n; ++i) p[i] = z[i];
    rho = dot(n, r, z);
    for (;;) {
        if (!isfinite(rn) || !isfinite(rho)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (rn <= lim) {
            if (r_true) return finish(A, b, x, rs, k, OR_CONVERGED, r, t);
            rn = true_residual(A, b, x, r, t);
            r_true = 1;
            if (rn <= lim) return finish(A, b, x, rs, k, OR_CONVERGED, r, t);
            if (k >= max_iter) return finish(A, b, x, rs, k, OR_MAX_ITER, r, t);
            log_restart(log, cap, k);
            goto restart;
        }
        if (k >= max_iter) return finish(A, b, x, rs, k, OR_MAX_ITER, r, t);
        if (rho == 0.0) return finish(A, b, x, rs, k, OR_BREAKDOWN, r, t);
        spmv(A, p, t);                                   /* t = A p          */
        double pt = dot(n, p, t);
        if (!isfinite(pt)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (pt == 0.0) return finish(A, b, x, rs, k, OR_BREAKDOWN, r, t);
        double alpha = rho / pt;                         /* alpha = rho/(p.t) */
        for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * t[i];
        r_true = 0;
        prec_apply(M, n, r, z);                          /* z = precond(r)   */
        double rho_new = dot(n, r, z);
        rn = nrm2(n, r);
        double beta = rho_new / rho;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
        k += 1;
    }
}

/* ---- BiCGSTAB, right-preconditioned (van der Vorst 1992) --------------- */
static or_result solve_bicgstab(const or_mat *A, const or_prec *M, const double *b, double *x,
                                double rs, double lim, int max_iter, double *ws, int *log,
                                int cap)
{
    int n = A->n, k = 0, r_true;
    double *r = ws, *rh = ws + n, *p = ws + 2 * n, *v = ws + 3 * n;
    double *ph = ws + 4 * n, *s = ws + 5 * n, *sh = ws + 6 * n, *t = ws + 7 * n;
    double rho0, alpha, omega, rn;

    rn = true_residual(A, b, x, r, t);
    r_true = 1;
restart:
    for (int i = 0; i < n; ++i) { rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
    rho0 = alpha = omega = 1.0;
    for (;;) {
        if (!isfinite(rn)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (rn <= lim) {
            if (r_true) return finish(A, b, x, rs, k, OR_CONVERGED, r, t);
            rn = true_residual(A, b, x, r, t);
            r_true = 1;
            if (rn <= lim) return finish(A, b, x, rs, k, OR_CONVERGED, r, t);
            if (k >= max_iter) return finish(A, b, x, rs, k, OR_MAX_ITER, r, t);
            log_restart(log, cap, k);
            goto restart;
        }
        if (k >= max_iter) return finish(A, b, x, rs, k, OR_MAX_ITER, r, t);
        k += 1;
        double rho = dot(n, rh, r);
        if (!isfinite(rho)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (rho == 0.0) return finish(A, b, x, rs, k, OR_BREAKDOWN, r, t);
        double beta = (rho / rho0) * (alpha / omega);
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        prec_apply(M, n, p, ph);
        spmv(A, ph, v);                                  /* v = A M p        */
        double sigma = dot(n, rh, v);
        if (!isfinite(sigma)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (sigma == 0.0) return finish(A, b, x, rs, k, OR_BREAKDOWN, r, t);
        alpha = rho / sigma;
        for (int i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double sn = nrm2(n, s);
        if (!isfinite(sn)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (sn <= lim) {                                 /* half-step exit   */
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
            for (int i = 0; i < n; ++i) r[i] = s[i];
            r_true = 0;
            rn = sn;
            continue;
        }
        prec_apply(M, n, s, sh);
        spmv(A, sh, t);                                  /* t = A M s        */
        double tt = dot(n, t, t), ts = dot(n, t, s);
        if (!isfinite(tt) || !isfinite(ts)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        omega = (tt == 0.0) ? 0.0 : ts / tt;
        for (int i = 0; i < n; ++i) x[i] = (x[i] + alpha * ph[i]) + omega * sh[i];
        for (int i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        r_true = 0;
        rho0 = rho;
        rn = nrm2(n, r);
        if (omega == 0.0 && !(rn <= lim)) return finish(A, b, x, rs, k, OR_BREAKDOWN, r, t);
    }
}

/* ---- GMRES(m), right-preconditioned, modified Gram-Schmidt Arnoldi and
 *      Givens rotations (Saad 2003, Alg. 6.9 with right preconditioning) -- */
static or_result solve_gmres(const or_mat *A, const or_prec *M, const double *b, double *x,
                             double rs, double lim, int max_iter, int m, double *ws)
{
    int n = A->n, k = 0;
    double *r = ws, *t = ws + n, *w = ws + 2 * n, *z = ws + 3 * n;
    double *V = ws + 4 * n;                          /* (m+1) x n            */
    double *H = V + (size_t)(m + 1) * n;             /* (m+1) x m, H[i*m+j]  */
    double *cs = H + (size_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *y = g + m + 1;

    for (;;) {
        double beta = true_residual(A, b, x, r, t);
        if (!isfinite(beta)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
        if (beta <= lim) return finish(A, b, x, rs, k, OR_CONVERGED, r, t);
        if (k >= max_iter) return finish(A, b, x, rs, k, OR_MAX_ITER, r, t);
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int jend = -1;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n;
            prec_apply(M, n, vj, z);
            spmv(A, z, w);                               /* w = A M v_j      */
            for (int i = 0; i <= j; ++i) {               /* MGS              */
                double *vi = V + (size_t)i * n;
                double h = dot(n, w, vi);
                H[(size_t)i * m + j] = h;
                for (int l = 0; l < n; ++l) w[l] = w[l] - h * vi[l];
            }
            double hn = nrm2(n, w);
            H[(size_t)(j + 1) * m + j] = hn;
            k += 1;
            if (!isfinite(hn)) return finish(A, b, x, rs, k, OR_NONFINITE, r, t);
            for (int i = 0; i < j; ++i) {                /* old rotations    */
                double h0 = H[(size_t)i * m + j], h1 = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * h0 + sn[i] * h1;
                H[(size_t)(i + 1) * m + j] = -sn[i] * h0 + cs[i] * h1;
            }
            double hjj = H[(size_t)j * m + j];
            double dd = sqrt(hjj * hjj + hn * hn);
            if (dd == 0.0) return finish(A, b, x, rs, k, OR_BREAKDOWN, r, t);
            cs[j] = hjj / dd;
            sn[j] = hn / dd;
            H[(size_t)j * m + j] = dd;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jend = j;
            if (fabs(g[j + 1]) <= lim || hn == 0.0 || k >= max_iter) break;
            double *vn = V + (size_t)(j + 1) * n;
            for (int i = 0; i < n; ++i) vn[i] = w[i] / hn;
        }
        for (int i = jend; i >= 0; --i) {                /* back substitution */
            double acc = g[i];
            for (int l = i + 1; l <= jend; ++l) acc = acc - H[(size_t)i * m + l] * y[l];
            y[i] = acc / H[(size_t)i * m + i];
        }
        for (int i = 0; i < n; ++i) z[i] = 0.0;
        for (int j = 0; j <= jend; ++j) {
            double *vj = V + (size_t)j * n;
            for (int i = 0; i < n; ++i) z[i] = z[i] + y[j] * vj[i];
        }
        prec_apply(M, n, z, w);                      /* x += M (V y)     */
        for (int i = 0; i < n; ++i) x[i] = x[i] + w[i];
    }
}

/* ---- BatchTrsv (Tab. 2): T x = b with T the lower (or upper) triangle of A,
 *      diagonal included, by forward (backward) substitution.  A zero
 *      diagonal entry is a breakdown: x = 0.  Iterations: 0. ---------------- */
static or_result solve_trsv(const or_mat *A, int lower, const double *b, double *x,
                            double rs, double *F, unsigned char *P, double *t)
{
    int n = A->n;
    or_result res;
    to_dense(A, F, P);
    for (int i = 0; i < n; ++i)
        if (F[(size_t)i * n + i] == 0.0) {
            for (int j = 0; j < n; ++j) x[j] = 0.0;
            res.iters = 0; res.status = OR_BREAKDOWN; res.resid = nrm2(n, b) / rs;
            return res;
        }
    for (int q = 0; q < n; ++q) {
        int i = lower ? q : n - 1 - q;
        double acc = b[i];
        int j0 = lower ? 0 : i + 1, j1 = lower ? i : n;
        for (int j = j0; j < j1; ++j)
            if (P[(size_t)i * n + j]) acc = acc - F[(size_t)i * n + j] * x[j];
        x[i] = acc / F[(size_t)i * n + i];
    }
    /* true residual of the triangular system */
    double acc2 = 0.0;
    int fin = 1;
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        int j0 = lower ? 0 : i, j1 = lower ? i + 1 : n;
        for (int j = j0; j < j1; ++j)
            if (P[(size_t)i * n + j]) acc += F[(size_t)i * n + j] * x[j];
        t[i] = b[i] - acc;
        acc2 += t[i] * t[i];
        if (!isfinite(x[i])) fin = 0;
    }
    res.iters = 0;
    res.resid = sqrt(acc2) / rs;
    res.status = (fin && isfinite(res.resid)) ? OR_CONVERGED : OR_NONFINITE;
    return res;
}

static size_t workspace_doubles(int solver, int n, int m)
{
    if (solver == OR_CG) return (size_t)4 * n + n;
    if (solver == OR_BICGSTAB) return (size_t)8 * n + n;
    return (size_t)4 * n + (size_t)(m + 1) * n + (size_t)(m + 1) * m + 4 * (size_t)m + 2 + n;
}

/* absolute: 0 tests ||r|| <= tol * ||b|| and reports ||b - A x|| / ||b||,
 * 1 tests ||r|| <= tol and reports ||b - A x||. */
static or_result solve_one(const or_mat *A, int solver, int precond, int bs,
                           const double *b, double *x, double tol, int absolute, int max_iter,
                           int m, double *ws, double *F, unsigned char *P, int *log, int cap)
{
    int n = A->n;
    double *d = ws;                         /* n doubles: d */
    double *inv = ws + n;                   /* n * OR_MAX_BLOCK: block inverse rows */
    double *gj = inv + (size_t)n * OR_MAX_BLOCK;   /* 2 * OR_MAX_BLOCK^2: elimination */
    double *work = gj + 2 * OR_MAX_BLOCK * OR_MAX_BLOCK;
    or_prec M;
    or_result res;
    double bn = nrm2(n, b);
    if (!isfinite(bn)) {
        res.iters = 0; res.status = OR_NONFINITE; res.resid = bn;
        return res;
    }
    if (bn == 0.0) {                        /* b = 0: x = 0 solves it exactly */
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        res.iters = 0; res.status = OR_CONVERGED; res.resid = 0.0;
        return res;
    }
    /* blocks of one row are scalar Jacobi */
    double lim = absolute ? tol : tol * bn, rs = absolute ? 1.0 : bn;
    if (solver == OR_TRSV_LOWER || solver == OR_TRSV_UPPER)
        return solve_trsv(A, solver == OR_TRSV_LOWER, b, x, rs, F, P, work);
    jacobi_diag(A, precond == OR_PREC_BLOCK_JACOBI && bs <= 1 ? OR_PREC_JACOBI : precond, d);
    M.bs = 1; M.col = precond == OR_PREC_ILU_COL; M.d = d; M.inv = inv; M.lu = NULL;
    M.mask = NULL;
    if (precond == OR_PREC_BLOCK_JACOBI && bs > 1) {
        block_jacobi(A, bs, inv, gj);
        M.bs = bs;
    }
    if (precond == OR_PREC_ILU || precond == OR_PREC_ILU_COL) {
        to_dense(A, F, P);
        if (ilu0(A->n, F, P)) { M.lu = F; M.mask = P; }
    }
    if (solver == OR_CG) return solve_cg(A, &M, b, x, rs, lim, max_iter, work, log, cap);
    if (solver == OR_BICGSTAB)
        return solve_bicgstab(A, &M, b, x, rs, lim, max_iter, work, log, cap);
    return solve_gmres(A, &M, b, x, rs, lim, max_iter, m, work);
}

static void make_mat(or_mat *A, int fmt, int n, const int *row_ptr, const int *col,
                     int width, const int *ecol, const double *val)
{
    A->fmt = fmt; A->n = n; A->width = width;
    A->row_ptr = row_ptr; A->col = col; A->ecol = ecol; A->val = val;
}

/* ------------------------------- exports -------------------------------- */

/* Solve every system of the batch; x holds x0 on entry and the result on exit.
 * values: CSR [n_batch][nnz], ELL [n_batch][width][n].  restart_log (may be
 * NULL): [n_batch][log_cap] int32, the restart log of each system (CG and
 * BiCGSTAB; see log_restart).  Returns 0. */
int or_batch_solve_log(int fmt, int64_t n_batch, int n, const int *row_ptr, const int *col_idx,
                       int nnz, int width, const int *ell_col, const double *values,
                       const double *b, double *x, int solver, int precond, int block_size,
                       double tol, int absolute, int max_iter, int restart, int *iters,
                       double *resid, int *status, int nthreads, int *restart_log, int log_cap)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    int m = restart > 0 ? restart : 30;
    size_t wsz = workspace_doubles(solver, n, m) + n + (size_t)n * OR_MAX_BLOCK +
                 2 * OR_MAX_BLOCK * OR_MAX_BLOCK;
    int dense = precond == OR_PREC_ILU || precond == OR_PREC_ILU_COL ||
                solver == OR_TRSV_LOWER || solver == OR_TRSV_UPPER;
    if (block_size < 1 || block_size > OR_MAX_BLOCK) block_size = 1;
    if (nthreads < 1) nthreads = 1;
    if (log_cap < 1) restart_log = NULL;
    #pragma omp parallel num_threads(nthreads)
    {
        double *ws = (double *)malloc(wsz * sizeof(double));
        double *F = dense ? (double *)malloc((size_t)n * n * sizeof(double)) : NULL;
        unsigned char *P = dense ? (unsigned char *)malloc((size_t)n * n) : NULL;
        #pragma omp for schedule(dynamic, 8)
        for (int64_t s = 0; s < n_batch; ++s) {
            or_mat A;
            int *log = restart_log ? restart_log + (size_t)s * log_cap : NULL;
            if (log) for (int i = 0; i < log_cap; ++i) log[i] = 0;
            make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
            or_result res = solve_one(&A, solver, precond, block_size, b + (size_t)s * n,
                                      x + (size_t)s * n, tol, absolute, max_iter, m, ws, F, P,
                                      log, log_cap);
            iters[s] = res.iters;
            status[s] = res.status;
            resid[s] = res.resid;
        }
        free(ws);
        free(F);
        free(P);
    }
    return 0;
}

/* As or_batch_solve_log without the restart log. */
int or_batch_solve(int fmt, int64_t n_batch, int n, const int *row_ptr, const int *col_idx,
                   int nnz, int width, const int *ell_col, const double *values,
                   const double *b, double *x, int solver, int precond, int block_size,
                   double tol, int absolute, int max_iter, int restart, int *iters,
                   double *resid, int *status, int nthreads)
{
    return or_batch_solve_log(fmt, n_batch, n, row_ptr, col_idx, nnz, width, ell_col, values,
                              b, x, solver, precond, block_size, tol, absolute, max_iter,
                              restart, iters, resid, status, nthreads, NULL, 0);
}

/* y = A x for every system. */
void or_batch_spmv(int fmt, int64_t n_batch, int n, const int *row_ptr, const int *col_idx,
                   int nnz, int width, const int *ell_col, const double *values,
                   const double *x, double *y)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    for (int64_t s = 0; s < n_batch; ++s) {
        or_mat A;
        make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
        spmv(&A, x + (size_t)s * n, y + (size_t)s * n);
    }
}

/* ||b - A x|| / ||b|| per system (||b - A x|| when ||b|| = 0). */
void or_batch_true_residual(int fmt, int64_t n_batch, int n, const int *row_ptr,
                            const int *col_idx, int nnz, int width, const int *ell_col,
                            const double *values, const double *b, const double *x,
                            double *out, int nthreads)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    if (nthreads < 1) nthreads = 1;
    #pragma omp parallel num_threads(nthreads)
    {
        double *r = (double *)malloc(2 * (size_t)n * sizeof(double));
        #pragma omp for schedule(static)
        for (int64_t s = 0; s < n_batch; ++s) {
            or_mat A;
            make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
            double rn = true_residual(&A, b + (size_t)s * n, x + (size_t)s * n, r, r + n);
            double bn = nrm2(n, b + (size_t)s * n);
            out[s] = bn == 0.0 ? rn : rn / bn;
        }
        free(r);
    }
}

/* Jacobi diagonal d_i per system (for pinning the preconditioner). */
void or_batch_jacobi(int fmt, int64_t n_batch, int n, const int *row_ptr, const int *col_idx,
                     int nnz, int width, const int *ell_col, const double *values, double *d)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    for (int64_t s = 0; s < n_batch; ++s) {
        or_mat A;
        make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
        jacobi_diag(&A, OR_PREC_JACOBI, d + (size_t)s * n);
    }
}

/* Block-Jacobi inverse rows per system (for pinning): inv [n_batch][n][bs]. */
void or_batch_block_jacobi(int fmt, int64_t n_batch, int n, const int *row_ptr,
                           const int *col_idx, int nnz, int width, const int *ell_col,
                           const double *values, int bs, double *inv)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    double work[2 * OR_MAX_BLOCK * OR_MAX_BLOCK];
    for (int64_t s = 0; s < n_batch; ++s) {
        or_mat A;
        make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
        block_jacobi(&A, bs, inv + (size_t)s * n * bs, work);
    }
}

/* ILU(0) factors per system (for pinning): lu [n_batch][n][n] dense row-major,
 * L strictly below the diagonal, U on and above, zero off the pattern;
 * ok[s] = 0 where the factorization failed (zero pivot, non-finite entry). */
void or_batch_ilu0(int fmt, int64_t n_batch, int n, const int *row_ptr, const int *col_idx,
                   int nnz, int width, const int *ell_col, const double *values, double *lu,
                   int *ok)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    unsigned char *P = (unsigned char *)malloc((size_t)n * n);
    for (int64_t s = 0; s < n_batch; ++s) {
        or_mat A;
        double *F = lu + (size_t)s * n * n;
        make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
        to_dense(&A, F, P);
        ok[s] = ilu0(n, F, P);
    }
    free(P);
}

/* z = (L U)^{-1} v per system with the factors of or_batch_ilu0 (for pinning);
 * col selects the column-oriented backward substitution. */
void or_batch_ilu0_apply(int fmt, int64_t n_batch, int n, const int *row_ptr,
                         const int *col_idx, int nnz, int width, const int *ell_col,
                         const double *values, const double *lu, const double *v, double *z,
                         int col)
{
    size_t stride = fmt == OR_CSR ? (size_t)nnz : (size_t)width * n;
    unsigned char *P = (unsigned char *)malloc((size_t)n * n);
    double *G = (double *)malloc((size_t)n * n * sizeof(double));
    for (int64_t s = 0; s < n_batch; ++s) {
        or_mat A;
        make_mat(&A, fmt, n, row_ptr, col_idx, width, ell_col, values + (size_t)s * stride);
        to_dense(&A, G, P);
        ilu_apply(n, lu + (size_t)s * n * n, P, v + (size_t)s * n, z + (size_t)s * n, col);
    }
    free(G);
    free(P);
}

double or_dot(int n, const double *a, const double *b) { return dot(n, a, b); }

/* BatchEll from BatchCsr (Sec. 3.1): width = longest row; slot s of row i is
 * the s-th stored entry of that row in CSR order, -1 where the row is short.
 * Call with ell_col = NULL to query the width only.  Returns the width. */
int or_csr_to_ell(int n, const int *row_ptr, const int *col_idx, int *ell_col)
{
    int width = 0;
    for (int i = 0; i < n; ++i)
        if (row_ptr[i + 1] - row_ptr[i] > width) width = row_ptr[i + 1] - row_ptr[i];
    if (!ell_col) return width;
    for (int s = 0; s < width; ++s)
        for (int i = 0; i < n; ++i) {
            int k = row_ptr[i] + s;
            ell_col[(size_t)s * n + i] = k < row_ptr[i + 1] ? col_idx[k] : -1;
        }
    return width;
}

/* Values of every system moved from CSR order to the ELL slot layout
 * (padding slots set to 0). */
void or_csr_values_to_ell(int64_t n_batch, int n, const int *row_ptr, int nnz, int width,
                          const double *csr_vals, double *ell_vals)
{
    for (int64_t s = 0; s < n_batch; ++s) {
        const double *src = csr_vals + (size_t)s * nnz;
        double *dst = ell_vals + (size_t)s * width * n;
        for (int sl = 0; sl < width; ++sl)
            for (int i = 0; i < n; ++i) {
                int k = row_ptr[i] + sl;
                dst[(size_t)sl * n + i] = k < row_ptr[i + 1] ? src[k] : 0.0;
            }
    }
}

/* Dense LU with partial pivoting: A (row-major n x n) is overwritten by its
 * factors, b by the solution.  Returns 0, or 1 if a zero pivot is met. */
int or_dense_solve(int n, double *A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(A[(size_t)i * n + c]) > fabs(A[(size_t)piv * n + c])) piv = i;
        if (A[(size_t)piv * n + c] == 0.0) return 1;
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                double tmp = A[(size_t)c * n + j];
                A[(size_t)c * n + j] = A[(size_t)piv * n + j];
                A[(size_t)piv * n + j] = tmp;
            }
            double tb = b[c]; b[c] = b[piv]; b[piv] = tb;
        }
        for (int i = c + 1; i < n; ++i) {
            double l = A[(size_t)i * n + c] / A[(size_t)c * n + c];
            A[(size_t)i * n + c] = l;
            for (int j = c + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)c * n + j];
            b[i] -= l * b[c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc = b[i];
        for (int j = i + 1; j < n; ++j) acc -= A[(size_t)i * n + j] * b[j];
        b[i] = acc / A[(size_t)i * n + i];
    }
    return 0;
}
