/*
 * batchsolve -- batched sparse Krylov solvers for AMD Instinct MI355X (gfx950).
 *
 * Solves A_i x_i = b_i for very many small sparse systems i that share one
 * sparsity pattern (paper Sec. 1 and Sec. 3: "batched iterative solvers" with a
 * shared pattern, each system monitored individually).  One fused kernel runs
 * the whole solve of every system: SpMV, scalar Jacobi, dot products, vector
 * updates and the stop test (Sec. 3.2, Sec. 3.4).
 *
 * Conventions for every entry point:
 *   - Return value: BS_OK (0) or a negative bs_error code.  A negative code means
 *     nothing was launched and no output was written.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library never
 *     frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Solves are
 *     asynchronous on that stream; results are valid after the stream is
 *     synchronised.  The library performs no host synchronisation in a solve.
 *   - Matrix values, right-hand sides and solutions are FP64.  Indexes are int32.
 */
#ifndef BATCHSOLVE_H
#define BATCHSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Matrix formats of Sec. 3.1.  BS_CSR: shared row_ptr[n+1] and col_idx[nnz];
 * values [n_batch][nnz] in CSR order.  BS_ELL: rows padded to the width W of
 * the longest row, shared slot-major column array [W][n] (the paper's
 * "column-major" layout; slot s of row i at s*n + i, padding = -1); values
 * [n_batch][W][n] in the same layout, padding values ignored.  BS_DENSE
 * (BatchDense): every entry stored, values [n_batch][n][n] row-major, solved on
 * the full pattern of bs_pattern_create_dense. */
typedef enum { BS_CSR = 0, BS_ELL = 1, BS_DENSE = 2 } bs_format;

/* Solvers of Tab. 2.  BS_CG follows Sec. 3.5, Alg. 1 (stop test replaced by the
 * relative residual); BS_BICGSTAB is right-preconditioned BiCGSTAB; BS_GMRES is
 * right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and Givens
 * rotations.  BS_TRSV_LOWER / BS_TRSV_UPPER (BatchTrsv) solve T x = b directly
 * for T the lower / upper triangle of A, diagonal included (entries of the
 * other triangle are ignored), by substitution: iterations 0, resid the true
 * residual of T, status BS_BREAKDOWN with x = 0 where a diagonal entry is zero
 * or not stored, BS_NONFINITE where x is not finite; the preconditioner, tol
 * and max_iter are validated but unused; systems of at most 1024 rows (one
 * row per lane: one wave up to 64 rows, else a workgroup of the next power of
 * two lanes, the substitution taken level by level with the levels the
 * pattern derives at creation), FP64 (BS_ERR_UNSUPPORTED otherwise and on the
 * uneven-batch entry points). */
typedef enum {
  BS_CG = 0, BS_BICGSTAB = 1, BS_GMRES = 2, BS_TRSV_LOWER = 3, BS_TRSV_UPPER = 4
} bs_solver;

/* Preconditioners (Tab. 2): none; scalar Jacobi (d_i = 1/a_ii, 1 where the
 * diagonal entry is zero or not stored); block Jacobi: the inverse of the
 * block diagonal of A with blocks of bs_options.block_size consecutive rows
 * (2, 4 or 8; the last block may be shorter), each block inverted by
 * Gauss-Jordan elimination without pivoting, a block that meets a zero or
 * non-finite pivot (or gives a non-finite inverse) taken as the identity;
 * ILU(0) (BatchIlu): the incomplete LU factorization on the pattern of A
 * without pivoting, applied by a forward and a backward substitution, the
 * identity for a system whose factorization meets a zero pivot or gives a
 * non-finite entry.  ILU(0) takes one row per lane: systems of up to 64 rows
 * on one wave (dense factors in LDS), up to 1024 rows on a workgroup of the
 * next power of two lanes (sparse factors in LDS, factorization and both
 * substitutions taken level by level: a row's level is one more than the
 * largest among the rows its entries of that triangle name, as the pattern
 * derives at creation); BS_GMRES with ILU(0) up to 512 rows, where its basis
 * stays in registers; BS_ERR_UNSUPPORTED beyond, or where the factors do not
 * fit the 160 KiB of LDS of a workgroup (with rows of at most 16 entries a
 * 1024-row system fits).  BS_BICGSTAB or BS_GMRES in FP64 only (CG needs a
 * symmetric preconditioner: BS_ERR_UNSUPPORTED), and not the uneven-batch
 * entry points.  Block Jacobi and ILU(0) are FP64 only. */
typedef enum {
  BS_PREC_NONE = 0, BS_PREC_JACOBI = 1, BS_PREC_BLOCK_JACOBI = 2, BS_PREC_ILU = 3
} bs_precond;

/* BS_FP64: everything in FP64.  BS_MIXED: iterative refinement whose outer loop
 * (true residual b - A x, its norm, the update of x) is FP64 and whose inner
 * Krylov solve (SpMV, Krylov vectors, inner reductions) is FP32: BiCGSTAB, or
 * one GMRES(m) cycle per refinement step (its rotations and triangular solve
 * in FP64).  Not for CG (BS_ERR_UNSUPPORTED). */
typedef enum { BS_FP64 = 0, BS_MIXED = 1 } bs_precision;

/* Per-system outcome written to status[]. */
enum {
  BS_CONVERGED = 0, /* true relative (or absolute) residual <= tol            */
  BS_MAX_ITER = 1,  /* iteration budget used up                               */
  BS_BREAKDOWN = 2, /* an exact zero divisor (rho, sigma, omega, p.Ap, Givens) */
  BS_NONFINITE = 3  /* a NaN or Inf appeared (input or arithmetic)             */
};

typedef enum {
  BS_OK = 0,
  BS_ERR_INVALID_ARG = -1, /* bad size, tolerance, enum, or NULL pointer          */
  BS_ERR_PATTERN = -2,     /* malformed pattern (see bs_pattern_create_csr)       */
  BS_ERR_UNSUPPORTED = -3, /* shape outside the fused kernels' limits             */
  BS_ERR_HIP = -4,         /* a HIP runtime call failed (message in last error)   */
  BS_ERR_NO_DEVICE = -5    /* no HIP device is present                            */
} bs_error;

/* Flags for bs_options.flags. */
#define BS_FLAG_X0_ZERO 1 /* ignore x on entry and start from x0 = 0 (x is not read) */
#define BS_FLAG_ABS_TOL 4 /* absolute stop criterion (Tab. 2): converged when
                             ||b - A x||_2 <= tol instead of tol * ||b||_2, and
                             resid[] reports ||b - A x||_2 itself */
#define BS_FLAG_PLAIN_LAYOUT 2 /* one-wave teams: lane i owns row i, x_i at buffer
                                  element i, CSR windows at min(row start, nnz - slots)
                                  (the pattern's bank-aware layout is not used) */

/* Largest system the register kernels take: one row per lane, up to 1024
 * lanes per system, and 2 or 4 rows per lane beyond that (rows of up to 8
 * entries there); longest row held in registers.  GMRES takes one row per lane
 * (up to 1024 rows).  Where no register shape holds the rows (more than
 * BS_MAX_ROW_NNZ entries, or more than 8 beyond 1024 rows), CG, BiCGSTAB and
 * GMRES (FP64, or BiCGSTAB and GMRES mixed) with scalar Jacobi or none take the
 * streamed placement (the spill tier of Sec. 3.5: the rows stay in global
 * memory and are read at every product): CG and BiCGSTAB up to BS_MAX_ROWS
 * rows, GMRES up to 1024 rows, and FP64 GMRES up to BS_MAX_ROWS with its
 * basis in device memory (31 x 2048 doubles per resident workgroup, taken
 * with hipMallocAsync on the solve's stream and freed after the launch). */
#define BS_MAX_ROWS 2048
#define BS_MAX_ROW_NNZ 64
#define BS_MAX_RESTART 30

typedef struct bs_pattern_s *bs_pattern;

/* Create a shared pattern from CSR arrays in HOST memory (Sec. 3.1: one copy of
 * the pattern for the whole batch).  The library validates it once, derives the
 * ELL slot layout, the diagonal position of every row and the per-wave row
 * lengths, and uploads them to the current device (it owns that copy).
 * row_ptr[n_rows+1] must start at 0, be nondecreasing and end at nnz; every
 * col_idx must lie in [0, n_rows) with no duplicate column within a row.
 * Errors: BS_ERR_INVALID_ARG (n_rows < 1, nnz < 0, NULL pointer),
 * BS_ERR_PATTERN (the rules above), BS_ERR_NO_DEVICE / BS_ERR_HIP on upload. */
int bs_pattern_create_csr(int32_t n_rows, int32_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, bs_pattern *out);

/* Same, from an ELL slot-major column array [ell_width][n_rows] in HOST memory;
 * padding slots are -1 and must follow a row's stored entries. */
int bs_pattern_create_ell(int32_t n_rows, int32_t ell_width, const int32_t *ell_col,
                          bs_pattern *out);

/* Release the pattern's device copy.  NULL is accepted. */
int bs_pattern_destroy(bs_pattern pattern);

/* Shape of a pattern (any output pointer may be NULL). */
int bs_pattern_query(bs_pattern pattern, int32_t *n_rows, int32_t *nnz, int32_t *ell_width,
                     int32_t *max_row_nnz);

/* Bank-aware layout of a one-wave team (one system per 64-lane wave, one row per
 * lane, CSR rows read through windows of `slots` register slots).  This is the
 * library's own refinement of the on-chip placement of Sec. 3.5 for the LDS of
 * gfx950, not a step of the paper: the SpMV gathers x[col] from LDS, a 64-lane
 * read of 8-byte elements is served as two 32-lane halves, and within a half the
 * distinct elements on one bank pair ((address / 8) mod 32) are served one after
 * another.  The layout permutes which lane owns which row, which buffer element
 * holds which x_j, and where each row's CSR window starts, to lower
 *   cost = 5 * (gathers + vector writes) + register copy of the values
 * counted per half and per slot as the largest number of distinct elements on
 * one bank pair.  Deterministic simulated annealing (`steps` moves) from the
 * plain layout; the result never costs more than the plain layout's.
 * Host only (no device is touched).  Outputs, HOST memory:
 *   lane_row[64]: row owned by lane l, -1 for none (each row exactly once);
 *   lane_win[64]: CSR position where lane l's window starts: for its row i,
 *     max(0, row_ptr[i+1] - slots) <= w <= min(row_ptr[i], nnz - slots); an idle
 *     lane repeats a window of a lane of its own half;
 *   col_pos[n_rows]: buffer element 0..63 of x_j, all distinct;
 *   cost[2]: the chosen layout's cost and the plain layout's.
 * Errors: BS_ERR_INVALID_ARG (NULL pointer, n_rows < 1, nnz < 0, slots < 1,
 * steps < 0), BS_ERR_PATTERN (as bs_pattern_create_csr), BS_ERR_UNSUPPORTED
 * (n_rows outside 33..64, nnz < slots, or a row longer than slots). */
int bs_wave_layout(int32_t n_rows, int32_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                   int32_t slots, int32_t steps, int32_t *lane_row, int32_t *lane_win,
                   int32_t *col_pos, int64_t *cost);

/* The layout a pattern holds (made at creation for 33..64 rows, with the slot
 * count the planner takes for one-wave teams; bs_batch_solve uses it whenever
 * it runs such a shape on CSR values, unless BS_FLAG_PLAIN_LAYOUT is set).
 * *slots = 0 when the pattern has none; else, when layout is not NULL, it
 * receives lane_row[64] | lane_win[64] | col_pos[n_rows] (HOST memory). */
int bs_pattern_layout(bs_pattern pattern, int32_t *slots, int32_t *layout);

/* The full pattern of n_rows x n_rows entries, for BatchDense values (Sec. 3.1,
 * Tab. 2): a dense batch stores every entry of every matrix, [n_batch][n][n]
 * row-major, which is the CSR order of this pattern; bs_batch_solve with
 * BS_DENSE runs the BatchCsr kernels on it.  Rows longer than BS_MAX_ROW_NNZ
 * (n_rows > 64) take the streamed placement (CG, BiCGSTAB and FP64 GMRES with
 * n_rows <= 2048, mixed GMRES with n_rows <= 1024); other requests on them
 * fail with BS_ERR_UNSUPPORTED at solve time.
 * Errors: BS_ERR_INVALID_ARG (NULL out, n_rows < 1, n_rows^2 beyond int32),
 * BS_ERR_NO_DEVICE / BS_ERR_HIP on upload. */
int bs_pattern_create_dense(int32_t n_rows, bs_pattern *out);

/* Copy the ELL slot-major column array [ell_width][n_rows] to HOST memory. */
int bs_pattern_ell_cols(bs_pattern pattern, int32_t *ell_col_out);

/* Rewrite CSR-ordered values [n_batch][nnz] (device) into the ELL layout
 * [n_batch][W][n] (device), zeros in padding slots.  Asynchronous on stream. */
int bs_values_csr_to_ell(bs_pattern pattern, int64_t n_batch, const double *csr_values,
                         double *ell_values, void *stream);

/* Number of stored values and indexes of a batched matrix (Sec. 3.1 storage
 * list): CSR n_batch*nnz values + (n_rows+1)+nnz indexes; ELL n_batch*W*n values
 * + W*n indexes; dense n_batch*n*n values, no indexes.  Pure host function. */
int bs_matrix_storage(bs_format fmt, int64_t n_batch, int32_t n_rows, int32_t nnz,
                      int32_t ell_width, int64_t *value_count, int64_t *index_count);

typedef struct {
  int32_t restart;      /* GMRES restart length m in [1, 30]; 0 selects 30       */
  int32_t precision;    /* bs_precision; 0 = BS_FP64                             */
  double inner_tol;     /* BS_MIXED inner relative tolerance; 0 selects 1e-6     */
  int32_t flags;        /* BS_FLAG_*                                             */
  int32_t team;         /* lanes per system (16..1024, power of two); 0 = planner */
  int32_t rows_per_lane;/* 1, 2 or 4; 0 = planner                                */
  int32_t *outer_iters; /* BS_MIXED: optional device int32[n_batch] of refinement
                           steps; NULL = not written                              */
  const double *x_alt;  /* optional device [n_batch][n_rows]: a second initial
                           guess.  Each system starts from whichever of x and
                           x_alt has the smaller ||b - A x||_2 (x on a tie; x_alt
                           also when only x's norm is NaN), one extra SpMV.  Not
                           with BS_FLAG_X0_ZERO (BS_ERR_INVALID_ARG)              */
  int32_t *alt_used;    /* optional device int32[n_batch]: 1 where x_alt was
                           taken, 0 where x was; written only with x_alt          */
  int32_t block_size;   /* BS_PREC_BLOCK_JACOBI: rows per block, 2, 4 or 8;
                           0 selects 8 (BS_ERR_INVALID_ARG otherwise)             */
  int32_t n_rhs;        /* right-hand sides per matrix, k >= 1; 0 selects 1.  With
                           k > 1, n_batch counts matrices and every matrix is
                           solved k times: b and x are [n_batch][k][n_rows], and
                           iters, resid, status, outer_iters, x_alt and alt_used
                           hold n_batch*k entries in the same order; each solve
                           reads its matrix's values (bs_batch_solve only;
                           BS_ERR_UNSUPPORTED on the uneven-batch entry points) */
  int32_t varlen_policy;/* bs_batch_solve_varlen: queue policy + 1, 1..18 (the
                           policies of bs_varbatch_set_policy); 0 selects policy 3
                           (workgroups of 512 lanes x 2 rows, largest tasks first;
                           12, the streamed placement, for rows over 16 entries) */
  int32_t structure_generation; /* bs_batch_solve_varlen and bs_batch_solve_dev:
                           the caller's count of changes to the structure
                           arrays (batch structure, or the shared pattern).  The
                           library reads and validates those arrays once per
                           (addresses, shape, device, generation); a caller that
                           rewrites them in place must change this number */
} bs_options;

/* The fused batched solve (Sec. 3.2-3.6): one kernel launch solves all n_batch
 * systems, each by one team of lanes (a sub-wave, a wave or a workgroup).
 *   fmt, pattern   format of `values` and the shared pattern (its n must equal n_rows)
 *   values         device, CSR [n_batch][nnz], ELL [n_batch][W][n_rows] or dense
 *                  [n_batch][n_rows][n_rows] (BS_DENSE needs the full pattern,
 *                  BS_ERR_PATTERN otherwise)
 *   b              device [n_batch][n_rows]
 *   x              device [n_batch][n_rows]; in: initial guess (unless
 *                  BS_FLAG_X0_ZERO), out: the last iterate
 *   tol            relative tolerance: stop when ||b - A x||_2 <= tol ||b||_2
 *                  (with BS_FLAG_ABS_TOL: <= tol), confirmed on the true
 *                  residual; tol > 0 and finite
 *   max_iter       >= 0; CG/BiCGSTAB iterations, GMRES Arnoldi steps (BS_MIXED:
 *                  inner iterations summed over refinement steps)
 *   iters, resid,  device int32/FP64/int32 [n_batch]: iterations, true relative
 *   status         residual of the returned x (absolute when ||b|| = 0 or with
 *                  BS_FLAG_ABS_TOL), and the bs status code; status may be NULL
 *   opts           NULL for defaults
 * Errors: BS_ERR_INVALID_ARG (n_batch < 0, n_rows mismatch, bad enum, tol <= 0 or
 * non-finite, max_iter < 0, bad restart/team, NULL required pointer),
 * BS_ERR_UNSUPPORTED (n_rows > BS_MAX_ROWS, or no kernel for the request: a
 * row longer than BS_MAX_ROW_NNZ outside the streamed placement's reach, see
 * BS_MAX_ROWS), BS_ERR_HIP (launch failure, or the allocation of GMRES's basis
 * beyond 1024 rows).  n_batch = 0 is a no-op. */
int bs_batch_solve(bs_format fmt, int64_t n_batch, int32_t n_rows, bs_pattern pattern,
                   const double *values, const double *b, double *x, bs_solver solver,
                   bs_precond precond, double tol, int32_t max_iter, int32_t *iters,
                   double *resid, int32_t *status, const bs_options *opts, void *stream);

/* The kernel shape bs_batch_solve would use (Sec. 3.6: work-group size from the
 * row count; Sec. 3.5: what is kept on chip).  Pure host function.
 *   team           lanes per system;  rows_per_lane  rows held by each lane
 *   slots          register slots per row (>= longest row); 0 for the
 *                  streamed placement (rows read from memory at every product;
 *                  workgroups of 512 lanes x 2 rows, 1024 x 2 beyond 1024
 *                  rows, GMRES 1024 x 1, and 1024 x 2 beyond 1024 rows)
 *   group_size     threads per workgroup; systems_per_group
 *   lds_bytes      dynamic LDS per workgroup
 *   stage_values   how the values reach the registers: 0 straight from HBM;
 *                  1 one-wave groups prefetch the next system's values and b
 *                  into LDS while solving the current one; 2 multi-wave teams
 *                  (CSR, rows of 32 slots or more) copy the next system's
 *                  values into LDS with the whole group while solving the
 *                  current one (the launch falls back to 0 where that LDS
 *                  would cost a resident workgroup) */
typedef struct {
  int32_t team, rows_per_lane, slots, group_size, systems_per_group, lds_bytes, stage_values;
} bs_plan_info;

int bs_plan(bs_format fmt, int32_t n_rows, int32_t nnz, int32_t max_row_nnz, bs_solver solver,
            const bs_options *opts, bs_plan_info *out);

/* As bs_plan, for the given preconditioner (the LDS of the block-Jacobi
 * inverse or of the ILU(0) factors included).  Same errors as bs_batch_solve's
 * planning: BS_ERR_INVALID_ARG for a bad enum or block size,
 * BS_ERR_UNSUPPORTED where no kernel shape serves the request. */
int bs_plan_precond(bs_format fmt, int32_t n_rows, int32_t nnz, int32_t max_row_nnz,
                    bs_solver solver, bs_precond precond, const bs_options *opts,
                    bs_plan_info *out);

/* ---------------------------------------------------------------------------
 * Uneven batches: systems of different sizes and patterns solved by ONE
 * persistent kernel launch (the paper's batched solvers take one shared
 * pattern, Sec. 3.1; its per-device size thresholds, Sec. 3.6, become an
 * autotuned choice here).  Systems are grouped by size class into tasks of one
 * to sixteen systems, ordered largest first, and taken from an atomic work
 * queue by the workgroups of a persistent launch; each system is solved by a
 * team of 64 or more lanes that own R rows each (n_rows <= 1024).  Workgroup
 * shapes: 1024 lanes x 1 row, 512 x 2, 256 x 4.
 *
 * Placement of the matrix (Sec. 3.5 keeps what fits on chip and leaves the rest
 * in global memory): "registers" holds every row's values and gather addresses
 * in registers through the solve (rows of at most 16 entries); "streamed"
 * keeps only where each row starts and reads the entries and values again from
 * memory at every product (rows of any length; fewer registers, more resident
 * waves).  Walk order: "csr" reads a row's entries one after another, "ell"
 * reads slot k of every row of the team together (the slot-major ELL order of
 * Sec. 3.1).  A solve runs either as one launch for the whole batch (a queue
 * policy, bs_varbatch_set_policy) or as one launch per size class, each with its
 * own shape, walk and placement (a plan, bs_varbatch_set_plan); the autotuner
 * bs_varbatch_tune times both and keeps the faster.
 * ------------------------------------------------------------------------- */
typedef struct bs_varbatch_s *bs_varbatch;

/* Describe an uneven batch from HOST arrays (copied; the library owns the
 * device copy and a work counter).  Patterns are CSR: pattern p has
 * pat_rows[p] rows, row_ptr at rowptr_all[pat_rowptr_off[p] ..] (pat_rows[p]+1
 * entries) and columns at col_all[pat_col_off[p] ..]; system s uses pattern
 * sys_pat[s].  Values of system s are its pattern's nnz doubles in CSR order,
 * stored after those of system s-1; b and x likewise with n_rows doubles.
 * The initial policy is 0 (registers) when no row is longer than 16, else 9
 * (streamed).
 * Errors: BS_ERR_INVALID_ARG, BS_ERR_PATTERN (as for bs_pattern_create_csr, or
 * sys_pat out of range), BS_ERR_UNSUPPORTED (a pattern with more than 1024
 * rows), BS_ERR_NO_DEVICE / BS_ERR_HIP. */
int bs_varbatch_create(int64_t n_batch, int32_t n_patterns, const int32_t *pat_rows,
                       const int64_t *pat_rowptr_off, const int32_t *rowptr_all,
                       const int64_t *pat_col_off, const int32_t *col_all, const int32_t *sys_pat,
                       bs_varbatch *out);

/* Same for ELL patterns (BatchEll, Sec. 3.1): pattern p has pat_rows[p] rows
 * and pat_width[p] slots, its slot-major columns [pat_width[p]][pat_rows[p]] at
 * col_all[pat_col_off[p] ..] (slot k of row i at k*rows + i; -1 = padding,
 * which must follow a row's stored entries).  Values of system s are
 * pat_width*pat_rows doubles in the same slot-major layout (padding values are
 * not read), stored after those of system s-1.  The library derives each
 * pattern's row-ordered and slot-major walks from the columns.
 * Errors as bs_varbatch_create (BS_ERR_PATTERN also for an entry after
 * padding; BS_ERR_UNSUPPORTED for a width above 1024). */
int bs_varbatch_create_ell(int64_t n_batch, int32_t n_patterns, const int32_t *pat_rows,
                           const int32_t *pat_width, const int64_t *pat_col_off,
                           const int32_t *col_all, const int32_t *sys_pat, bs_varbatch *out);

int bs_varbatch_destroy(bs_varbatch vb);

/* Totals: rows (= length of b and x), values, queue tasks, current policy
 * (-1 while a per-class plan is in force). */
int bs_varbatch_query(bs_varbatch vb, int64_t *total_rows, int64_t *total_values, int32_t *n_tasks,
                      int32_t *policy);

/* One launch for the whole batch under policy p (0..17): placement p / 9
 * (0 registers, 1 streamed), workgroup shape (p % 9) / 3 (0: 1024 lanes x 1 row
 * per lane, 1: 512 x 2, 2: 256 x 4) and queue order p % 3: 0 = team of the next
 * power of two >= n / R lanes (at least 64), largest tasks first; 1 = teams
 * twice that size (fewer systems per task); 2 = as 0 with the systems of a
 * class kept in batch order.  The walk is the input's own order (csr for CSR
 * patterns, ell for ELL patterns).  A solve under a register policy with a row
 * longer than 16 fails with BS_ERR_UNSUPPORTED.
 * BS_ERR_INVALID_ARG for p outside 0..17. */
int bs_varbatch_set_policy(bs_varbatch vb, int32_t policy);

/* One launch per size class (n <= 64, <= 128, <= 256, <= 512, <= 1024 rows;
 * largest class first, each taking its own tasks from its own counter):
 * class_codes[5], one per class, code = shape + 3 * walk + 6 * placement with
 * shape as above (0..2), walk 0 csr / 1 ell, placement 0 registers / 1
 * streamed; codes of classes without systems are not used but must be valid.
 * A solve fails with BS_ERR_UNSUPPORTED when a class's choice has no kernel
 * (registers with a row longer than 16, or streamed with block Jacobi).
 * BS_ERR_INVALID_ARG for a code outside 0..11. */
int bs_varbatch_set_plan(bs_varbatch vb, const int32_t *class_codes);

/* The plan in force: *policy as bs_varbatch_query, class_codes[5] the
 * per-class codes (all -1 under a single-launch policy).  Either pointer may
 * be NULL. */
int bs_varbatch_get_plan(bs_varbatch vb, int32_t *policy, int32_t *class_codes);

/* Solve all systems (BS_CG or BS_BICGSTAB; BS_MIXED for BiCGSTAB), arguments
 * as in bs_batch_solve with the concatenated layouts above.  One launch of
 * the counter reset and one of the persistent solver, asynchronous. */
int bs_varbatch_solve(bs_varbatch vb, const double *values, const double *b, double *x,
                      bs_solver solver, bs_precond precond, double tol, int32_t max_iter,
                      int32_t *iters, double *resid, int32_t *status, const bs_options *opts,
                      void *stream);

/* Autotuner: on these inputs (1 warm-up and `reps` timed solves per
 * candidate, synchronising `stream`) time every single-launch policy, then
 * every class choice for each size class launched alone, then the plan of the
 * best choice per class as a whole; keep the fastest of that plan and the
 * best policy.  One-line report (report may be NULL): "policy=<p or
 * split:c0,..,c4> times_ms=<t0>,..,<t17> classes=<class>:<code>=<lanes>x<rows>/
 * <walk>/<placement>:<ms>,.. split_ms=<t> key=<key>", '-' for a policy with no
 * kernel for this request.  If cache_path is not NULL the choice is looked up
 * in / appended to that text file, keyed by the format, the size-class
 * histogram and longest rows, solver, precision and preconditioner; a cached
 * choice is applied without timing or solving.  Each timed solve
 * starts from the caller's x (kept in a temporary device copy) unless
 * opts->flags has BS_FLAG_X0_ZERO; after timing, one more solve with the
 * chosen policy leaves x/iters/resid/status as bs_varbatch_solve would. */
int bs_varbatch_tune(bs_varbatch vb, const double *values, const double *b, double *x,
                     bs_solver solver, bs_precond precond, double tol, int32_t max_iter,
                     int32_t *iters, double *resid, int32_t *status, const bs_options *opts,
                     int32_t reps, const char *cache_path, char *report, size_t report_len,
                     void *stream);

/* Capture the counter reset and the solve's launches (with these arguments)
 * into a HIP graph owned by the handle, replacing any previous one;
 * bs_varbatch_replay launches it on `stream`.  The graph holds no memset
 * nodes.  A change of plan (bs_varbatch_set_policy, bs_varbatch_set_plan,
 * bs_varbatch_tune) drops the graph;
 * bs_varbatch_replay then fails with BS_ERR_INVALID_ARG until the next
 * capture. */
int bs_varbatch_capture(bs_varbatch vb, const double *values, const double *b, double *x,
                        bs_solver solver, bs_precond precond, double tol, int32_t max_iter,
                        int32_t *iters, double *resid, int32_t *status, const bs_options *opts);
int bs_varbatch_replay(bs_varbatch vb, void *stream);

/* Uneven batch on caller-owned DEVICE arrays (the boundary of the batched
 * solve for systems of different sizes; paper Sec. 3.1 describes one shared
 * pattern per batch, here each system names one of n_patterns CSR patterns).
 *   sys_rows  [n_batch] rows of system s (1..1024; equal to its pattern's rows)
 *   row_off   [n_batch+1] first row of system s in b and x; row_off[0] = 0,
 *             row_off[s+1] - row_off[s] = sys_rows[s]
 *   val_off   [n_batch+1] first value of system s; val_off[0] = 0, each system
 *             holds its pattern's nnz values in CSR order
 *   pat_id    [n_batch] pattern of system s, 0..n_patterns-1
 *   pat_rowptr_off, pat_col_off [n_patterns]: where pattern p's row_ptr
 *             (rows+1 entries, starting at 0) and columns start in rowptr_all
 *             and col_all; patterns no system uses are not read
 *   values, b, x, iters, resid, status: as bs_varbatch_solve
 *   ws, ws_bytes  device workspace of at least bs_varlen_workspace_size(n_batch)
 *             bytes, 256-byte aligned; it holds the task queue of this call and
 *             must not be changed by the caller between calls that use it
 * No column twice in a row, all in range.  Policy: opts->varlen_policy - 1
 * (a single-launch policy of bs_varbatch_set_policy, 0..17); 0 selects 3
 * (512 x 2, registers), or 12 (streamed) when a row holds more than 16
 * entries.  The first call for a structure copies the structure arrays to the
 * host (one synchronisation of `stream`), validates them and builds the task queue; later
 * calls with the same addresses, shape and opts->structure_generation launch
 * at once (asynchronously), re-uploading the task queue only when ws or the
 * queue policy changed.  Solvers and options as bs_varbatch_solve.
 * Errors: BS_ERR_INVALID_ARG (NULL pointer, inconsistent offsets or rows,
 * workspace too small or misaligned, bad option), BS_ERR_PATTERN (malformed
 * pattern, pat_id out of range), BS_ERR_UNSUPPORTED (more than 1024 rows, a
 * row longer than 16 under a register policy, unsupported solver or
 * preconditioner), BS_ERR_HIP.
 * n_batch = 0 is a no-op. */
int bs_batch_solve_varlen(int64_t n_batch, const int32_t *sys_rows, const int64_t *row_off,
                          const int64_t *val_off, int32_t n_patterns, const int32_t *pat_id,
                          const int64_t *pat_rowptr_off, const int64_t *pat_col_off,
                          const int32_t *rowptr_all, const int32_t *col_all,
                          const double *values, const double *b, double *x, bs_solver solver,
                          bs_precond precond, double tol, int32_t max_iter, int32_t *iters,
                          double *resid, int32_t *status, const bs_options *opts, void *ws,
                          size_t ws_bytes, void *stream);

/* Bytes of workspace bs_batch_solve_varlen needs for n_batch systems (the task
 * counter, up to n_batch tasks and the queue order).  Pure host function;
 * 0 for n_batch < 0. */
size_t bs_varlen_workspace_size(int64_t n_batch);

/* A shared pattern held in caller-owned DEVICE memory. */
typedef struct {
  const int32_t *row_ptr; /* BS_CSR: [n_rows+1], starting at 0, nondecreasing; else NULL */
  const int32_t *col_idx; /* BS_CSR: [nnz]; BS_ELL: [ell_width][n_rows] slot-major, -1 padding
                             after a row's entries; BS_DENSE: unused */
  int32_t nnz;            /* BS_CSR: stored entries; BS_ELL: ell_width * n_rows */
  int32_t ell_width;      /* BS_ELL: slots per row; else 0 */
} bs_pattern_dev;

/* The batched solve with the shared pattern (Sec. 3.1) given as caller-owned
 * DEVICE arrays instead of a handle.  The first call for a pattern -- its
 * array addresses, format, n_rows, nnz, ell_width, the current device and
 * opts->structure_generation -- copies the arrays to the host (one
 * synchronisation of `stream`), validates them as bs_pattern_create_csr/_ell
 * do and keeps the derived pattern (8 patterns are kept; the least recently
 * used is released); later calls launch at once, asynchronously.  A caller
 * that rewrites the arrays in place passes a new structure_generation.
 * BS_DENSE reads no arrays (pattern may be NULL): the full pattern of n_rows
 * rows is built once.  workspace, workspace_bytes: bs_workspace_size bytes
 * (0: both may be NULL/0).  Everything else as bs_batch_solve.
 * Errors: BS_ERR_INVALID_ARG (NULL pattern or arrays for CSR/ELL, nnz
 * inconsistent with ell_width * n_rows, n_rows < 1, n_batch < 0, and those of
 * bs_batch_solve), BS_ERR_PATTERN (as bs_pattern_create_csr/_ell),
 * BS_ERR_UNSUPPORTED, BS_ERR_NO_DEVICE, BS_ERR_HIP.  n_batch = 0 is a no-op. */
int bs_batch_solve_dev(bs_format fmt, int64_t n_batch, int32_t n_rows,
                       const bs_pattern_dev *pattern, const double *values, const double *b,
                       double *x, bs_solver solver, bs_precond precond, double tol,
                       int32_t max_iter, int32_t *iters, double *resid, int32_t *status,
                       const bs_options *opts, void *workspace, size_t workspace_bytes,
                       void *stream);

/* Bytes of device workspace bs_batch_solve needs for this request: 0.  The
 * fused fixed-size kernels keep every Krylov vector on chip (registers and
 * LDS) and read and write only the caller's arrays, so the solve takes no
 * workspace; GMRES beyond 1024 rows, whose basis does not fit on chip, takes
 * its device memory itself (a stream-ordered allocation on the solve's stream,
 * freed after the launch).  The query exists so that a caller written against
 * a workspace protocol can size one.  Pure host function; 0 also for invalid
 * arguments. */
size_t bs_workspace_size(bs_format fmt, int64_t n_batch, int32_t n_rows, bs_pattern pattern,
                         bs_solver solver, const bs_options *opts);

/* ---------------------------------------------------------------------------
 * Learned initial guess for sequences of related batches (systems that drift
 * from one time step to the next, as along an integration in time; the paper
 * solves such sequences, Sec. 4.3).  A three-layer perceptron maps the
 * features f = [diag(A_t), b_t - x_{t-1}, x_{t-1}] of a system (3n values: the
 * information of diag(A_t), b_t and x_{t-1}, with the difference formed in FP64
 * so that the small step change survives the BF16 inputs; normalised by
 * training-set means and standard deviations) through two hidden ReLU layers
 * of width 256 to y (n values); the guess is x0 = x_{t-1} + sigma_d * y, with
 * sigma_d the per-component standard deviation of x_t - x_{t-1} over the
 * training data.  Training minimises the mean squared error between y and
 * (x_t - x_{t-1}) / sigma_d with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * Products run on BF16 matrix cores with FP32 accumulation; the master
 * weights, Adam moments, biases and losses are FP32, the scaling FP64.
 *
 * Parameter vector (FP32, this order, row-major): W1 [3n][256], b1 [256],
 * W2 [256][256], b2 [256], W3 [256][n], b3 [n].
 * Device arrays: feat [rows][3n] and delta [rows][n] FP32; rows (optional)
 * selects the samples of a minibatch; values/b/x FP64 as in bs_batch_solve
 * (CSR values of the model's pattern).  Calls taking a stream are
 * asynchronous on it; the others synchronise the device.
 * ------------------------------------------------------------------------- */
typedef struct bs_ws_model_s *bs_ws_model;

/* Model for systems with the given CSR pattern (host arrays; n <= 64).
 * Weights start at zero and the scaling at mean 0 / deviation 1.
 * Errors: BS_ERR_INVALID_ARG, BS_ERR_PATTERN, BS_ERR_UNSUPPORTED (n > 64),
 * BS_ERR_NO_DEVICE, BS_ERR_HIP. */
int bs_ws_create(int32_t n, int32_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                 bs_ws_model *out);
int bs_ws_destroy(bs_ws_model m);
int bs_ws_param_count(bs_ws_model m, int64_t *count);

/* Copy the FP32 parameter vector in (and reset Adam) or out (host arrays). */
int bs_ws_set_params(bs_ws_model m, const float *host_params);
int bs_ws_get_params(bs_ws_model m, float *host_params);

/* Raw features of n_batch systems and, if x_next is not NULL, their change
 * delta = x_next - x_prev (FP32). */
int bs_ws_features(bs_ws_model m, int64_t n_batch, const double *values, const double *b,
                   const double *x_prev, const double *x_next, float *feat, float *delta,
                   void *stream);

/* Fit the scaling (feature means and deviations, and sigma_d) to n_samples
 * training rows; get/set copy it from/to host arrays (F = 3n, n, n values). */
int bs_ws_fit_scaling(bs_ws_model m, int64_t n_samples, const float *feat, const float *delta,
                      void *stream);
int bs_ws_get_scaling(bs_ws_model m, double *mu_f, double *sd_f, double *sd_d);
int bs_ws_set_scaling(bs_ws_model m, const double *mu_f, const double *sd_f, const double *sd_d);

/* Network output y [n_samples][n] for raw feature rows. */
int bs_ws_forward(bs_ws_model m, int64_t n_samples, const float *feat, const int32_t *rows,
                  float *y, void *stream);

/* Loss (device scalar) and gradient (device [param_count]) of a batch,
 * without changing the model; bs_ws_train_step takes one Adam step with
 * learning rate lr on it (loss may be NULL). */
int bs_ws_grad(bs_ws_model m, int64_t n_samples, const float *feat, const float *delta,
               const int32_t *rows, float *grad, float *loss, void *stream);
int bs_ws_train_step(bs_ws_model m, int64_t n_samples, const float *feat, const float *delta,
                     const int32_t *rows, float lr, float *loss, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): bs_ws_train_step without its
 * workspace allocation.  The step's workspace (activations, their gradients,
 * the weight-gradient partials, the per-tile losses) is a file-scope device
 * array of 7 MiB on each device the library runs on, held until the process
 * ends; the call itself allocates nothing (it launches the same kernels as
 * bs_ws_train_step, asynchronously on stream).  Steps of at most 2048 samples:
 * BS_ERR_UNSUPPORTED beyond.  Every call on one device shares that device's
 * array, so calls that overlap on one device (two streams, two threads, or two
 * models) race: serialise them.  Other arguments and errors as
 * bs_ws_train_step. */
int bs_ws_train_step_noalloc(bs_ws_model m, int64_t n_samples, const float *feat,
                             const float *delta, const int32_t *rows, float lr, float *loss,
                             void *stream);

/* x0 = x_prev + sigma_d * y(f) for n_batch systems, features built from the
 * batch itself (one fused kernel). */
int bs_ws_infer(bs_ws_model m, int64_t n_batch, const double *values, const double *b,
                const double *x_prev, double *x0, void *stream);

/* Packed inference weights: everything the network's inference reads (BF16
 * weights, FP32 biases, FP64 scaling) in one caller-owned device buffer, so
 * that the inference below takes a plain pointer instead of a model handle.
 * bs_ws_packed_bytes(n): its size for systems of n unknowns (0 outside
 * 1..64; pure host function).  bs_ws_pack copies a model's current weights and
 * scaling into `weights` (device, at least that many bytes, 256-byte
 * aligned), asynchronously on stream.  Layout, each region 256-byte aligned:
 * W1^T, W2^T, W3^T as BF16 [256][3n rounded up to 64], [256][256], [n
 * rounded up to 32][256]; b1, b2, b3 FP32; feature means, feature deviations
 * and sigma_d FP64.  Errors: BS_ERR_INVALID_ARG (NULL, short or misaligned
 * buffer), BS_ERR_HIP. */
size_t bs_ws_packed_bytes(int32_t n);
int bs_ws_pack(bs_ws_model m, void *weights, size_t bytes, void *stream);

/* x0 = x_prev + sigma_d * y(f) for n_batch systems of n unknowns, from packed
 * weights (bs_ws_pack) and the systems' diagonals given directly:
 *   diag, b, x_prev  device [n_batch][n] FP64 (diag[s][i] = A_s[i][i])
 *   x0               device [n_batch][n] FP64, written
 * Features f = [diag, b - x_prev, x_prev] as in bs_ws_infer, which gathers the
 * diagonal out of the CSR values itself.  One kernel, asynchronous on stream.
 * Errors: BS_ERR_INVALID_ARG (NULL or misaligned pointer, n < 1, n_batch < 0),
 * BS_ERR_UNSUPPORTED (n > 64), BS_ERR_HIP.  n_batch = 0 is a no-op. */
int bs_ws_infer_packed(int64_t n_batch, int32_t n, const void *weights, const double *diag,
                       const double *b, const double *x_prev, double *x0, void *stream);

/* Text for a bs_error code; never NULL. */
const char *bs_error_string(int code);

/* Last HIP error text recorded by the library (thread-local); never NULL. */
const char *bs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BATCHSOLVE_H */
