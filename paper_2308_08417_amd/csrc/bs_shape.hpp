// Kernel shapes and launch arguments shared by the host planner and the HIP
// kernels of the fused batched solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bs {

constexpr int kWave = 64;
constexpr int kMaxRestart = 30;  // GMRES basis held in registers: m+1 vectors

// Per-team LDS scalars of GMRES: current Hessenberg column (m+2), rotated
// upper-triangular R packed by columns (m(m+1)/2), Givens c and s (m each),
// right-hand side g (m+1) and the least-squares solution y (m).  Each entry is
// written once per cycle with the same bits by every lane of the team.
constexpr int kGmresScalars = (kMaxRestart + 2) + kMaxRestart * (kMaxRestart + 1) / 2 +
                              2 * kMaxRestart + (kMaxRestart + 1) + kMaxRestart;

// Largest number of values reduced together (the LDS slot stride of the
// cross-wave stage).
constexpr int kMaxFused = 4;

// Arguments of every solver kernel (passed by value).
struct KArgs {
  int64_t n_batch;
  int n, nnz, width, fmt;      // fmt: 0 CSR, 1 ELL
  int precond, flags, max_iter, restart;
  int stage;                   // values and b prefetched into LDS (single-wave groups)
  int gmres;                   // GMRES scalars live behind the vector buffers
  int team_bytes;              // LDS bytes per team for vectors and scalars
  int stage_team_bytes;        // LDS staging bytes per team (values then b)
  int stage_vals_bytes;        // of which the values region
  int stage_offset;            // byte offset of the staging area in LDS
  int window;                  // CSR rows read through a fixed window of NZ slots
  double tol, inner_tol;
  const int* row_ptr;          // [n+1]
  const int* slot_col;         // [width][n], -1 padding
  const int* row_len;          // [n]
  const int* diag_slot;        // [n], -1 if no stored diagonal
  const double* values;
  const double* b;
  double* x;
  int* iters;
  double* resid;
  int* status;
  int* outer;
  int* sink;                   // a device word written instead of a missing status
  const double* x_alt;         // optional second initial guess [n_batch][n]
  int* alt_used;               // optional [n_batch]: 1 where x_alt was taken
  const int* layout;           // one-wave teams: lane_row[64] | lane_win[64] | col_pos[n], or null
  int nrhs;                    // right-hand sides per matrix: solve s reads matrix s / nrhs
  int block;                   // block-Jacobi block size (2, 4 or 8), 0 for scalar Jacobi / none
  int bj_offset;               // byte offset of the block-Jacobi or ILU(0) region in a team's LDS
  const int* lev;              // [n] row levels for the sweeps of multi-wave teams:
                               // lower-triangle level | upper-triangle level << 16
  int nlev_l, nlev_u;          // level counts of the lower and upper triangles
  const int* ilu_ptr;          // [n+1] start of each row's ILU(0) steps in ilu_ops
  const int* ilu_ops;          // ILU(0) schedule (header and update words, see the pattern)
  const int* sweep;            // sweep lists of multi-wave teams (see the pattern)
  int sweep_ents;              // entries in those lists
};

// Matrix of solve s (several right-hand sides per matrix: solves s*k..s*k+k-1
// share matrix s).
__host__ __device__ __forceinline__ int64_t matrix_of(const KArgs& g, int64_t s) {
  return g.nrhs == 1 ? s : s / g.nrhs;
}

// Block Jacobi: per team, the inverse rows (rows x block doubles) and a
// row-indexed exchange buffer (rows doubles).
constexpr int kMaxBlock = 8;
__host__ __device__ constexpr int bj_bytes(int rows, int block) {
  return block > 1 ? rows * (block + 1) * 8 : 0;
}

// Preconditioner kinds compiled into separate kernel instances: scalar
// Jacobi (or none: d = 1), block Jacobi, ILU(0).
constexpr int kPkScalar = 0, kPkBlock = 1, kPkIlu = 2;

// ILU(0) of a one-wave team: the factors as an n-row FP64 array, row-major,
// columns padded with zeros to a multiple of 8 plus one (an odd stride).
__host__ __device__ constexpr int ilu_stride(int n) { return ((n + 7) & ~7) + 1; }
__host__ __device__ constexpr int ilu_bytes(int n) { return ((n * ilu_stride(n) * 8) + 15) & ~15; }

// Flag bit of the absolute stop criterion (BS_FLAG_ABS_TOL).
constexpr int kFlagAbsTol = 4;

// team: lanes per system; R: rows per lane; NZ: register slots per row.
template <int TEAM_, int R_, int NZ_>
struct Shape {
  static constexpr int TEAM = TEAM_, R = R_, NZ = NZ_;
  static constexpr int WG = TEAM < kWave ? kWave : TEAM;
  static constexpr int TEAMS = WG / TEAM;  // systems per workgroup
  static constexpr int WAVES = WG / kWave;
  static constexpr int ROWS = TEAM * R;    // largest system a team holds
  // Waves per SIMD the register allocator is asked to fit: single-wave groups
  // with up to 32 slots per row are held to 3 (at most 168 VGPRs), which keeps
  // enough waves resident to hide the reductions' latency.
#ifndef BS_OCC_ONE_WAVE
#define BS_OCC_ONE_WAVE 3
#endif
  // Rows of 33..56 entries (56 slots) fit 256 registers beside the vectors:
  // two waves per SIMD, where the 64-slot shapes take 256 and more (one).
  static constexpr int OCC = (WAVES == 1 && R == 1 && NZ >= 24 && NZ <= 32) ? BS_OCC_ONE_WAVE
                             : (R == 1 && NZ == 56)                          ? 2
                                                                             : 1;
  // The mixed-precision forms hold an FP32 copy of the rows beside the FP64
  // one: at three waves per SIMD they spill, at two they do not (and a solve
  // from a close start, one inner iteration, runs 9% faster so).
#ifndef BS_OCC_ONE_WAVE_MIXED
#define BS_OCC_ONE_WAVE_MIXED 2
#endif
  static constexpr int OCC_MIXED =
      (WAVES == 1 && R == 1 && NZ >= 24 && NZ <= 32) ? BS_OCC_ONE_WAVE_MIXED : 1;
};

// Multi-wave teams copy a system's CSR values into LDS with the whole group
// (coalesced) in the shapes of at least this many register slots per row:
// there a lane's row spans many cache lines and reading it straight from HBM
// is slowest.  The copy's code costs the narrower shapes a few registers and,
// with them, a resident wave, for no gain on their short rows.
constexpr int kStageMinSlots = 32;

// Vector buffers per team (SpMV source vectors, double-buffered).  Each buffer
// holds ROWS elements plus one cell that stays zero: register slots that hold
// no entry of the lane's row gather from it.
constexpr int kVecBuffers = 2;

__host__ __device__ constexpr int round16(int b) { return (b + 15) & ~15; }
__host__ __device__ constexpr int round1k(int b) { return (b + 1023) & ~1023; }
__host__ __device__ constexpr int vec_buf_bytes(int rows) { return (rows + 1) * 8; }

// GMRES basis vectors a team keeps in LDS instead of registers.  A 1024-lane
// workgroup leaves 128 VGPRs per lane, too few for 31 FP64 basis elements next
// to the row's values and addresses: such teams keep 16 FP64 (or all 31 FP32)
// vectors in LDS, one element per lane, each lane reading only its own.
__host__ __device__ constexpr int gmres_lds_vectors(int wg, bool mixed) {
  return wg == 1024 ? (mixed ? kMaxRestart + 1 : 16) : 0;
}

// Offset of the GMRES basis region inside a team's LDS region.
__host__ __device__ constexpr int gmres_basis_offset(int rows) {
  return round16(kVecBuffers * vec_buf_bytes(rows) + kGmresScalars * 8);
}

// Bytes of a team's GMRES basis region.
__host__ __device__ constexpr int gmres_basis_bytes(int rows, int wg, bool mixed) {
  return round16(gmres_lds_vectors(wg, mixed) * rows * (mixed ? 4 : 8));
}

// LDS bytes of a team's vector buffers and solver scalars (and, for GMRES
// shapes of `wg` lanes, its basis vectors in LDS).
__host__ __device__ inline int team_vec_bytes(int rows, int solver_is_gmres, int wg = 0,
                                              bool mixed = false) {
  if (!solver_is_gmres) return round16(kVecBuffers * vec_buf_bytes(rows));
  return gmres_basis_offset(rows) + gmres_basis_bytes(rows, wg, mixed);
}

inline int red_lds_bytes(int waves) { return waves > 1 ? 2 * kMaxFused * waves * 8 : 0; }

// Staging of one team (single-wave groups): its system's values then its b,
// each copied as the 16-byte-aligned chunks that cover it, so each region
// holds up to 16 bytes more than its block; the values region also covers a
// full window of NZ slots.  With one team per wave the two regions are whole
// KiB, the span of one 16-byte-per-lane direct-to-LDS load of a wave; the
// whole staging area is always a multiple of 1 KiB.
inline int stage_vals_bytes(int teams, int stored, int nz) {
  const int b = round16((stored > nz ? stored : nz) * 8) + 16;
  return teams == 1 ? round1k(b) : b;
}
inline int stage_b_bytes(int teams, int n) {
  const int b = round16(n * 8) + 16;
  return teams == 1 ? round1k(b) : b;
}
inline int stage_total_bytes(int teams, int stored, int n, int nz) {
  return round1k(teams * (stage_vals_bytes(teams, stored, nz) + stage_b_bytes(teams, n)));
}

// ILU(0) and BatchTrsv of a multi-wave team (row i on lane i, one row per
// lane): byte offsets inside the team's region of the factor (or triangle)
// values in the pattern's CSR order (f, nnz doubles), the sweep vector (y, n
// doubles), the pivots or diagonal (d, n doubles), and the pattern's sweep
// lists: per row its list start and counts (rng, n ints), the lists (ent, at
// most nnz ints), the rows in level order (rows, 2n shorts) and the level
// starts (lvl, at most 2n+2 shorts).
struct IluMw {
  int f, y, d, rng, ent, rows, lvl, bytes;
};
__host__ __device__ constexpr IluMw ilu_mw_layout(int n, int nnz) {
  const int y = round16(nnz * 8), d = y + round16(n * 8), rng = d + round16(n * 8);
  const int ent = rng + round16(n * 4), rows = ent + round16(nnz * 4);
  const int lvl = rows + round16(n * 4);
  return IluMw{0, y, d, rng, ent, rows, lvl, lvl + round16((2 * n + 2) * 2)};
}

// LDS bytes of a team's ILU(0) or BatchTrsv region: the dense factors of a
// one-wave team, the sparse layout above for larger teams.
__host__ __device__ constexpr int tri_region_bytes(int team, int n, int nnz) {
  return team <= kWave ? ilu_bytes(n) : ilu_mw_layout(n, nnz).bytes;
}

}  // namespace bs
