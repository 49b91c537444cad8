// The fused batched Krylov solvers (paper Sec. 3.2-3.6): one kernel launch, one
// team of lanes per system, the whole solve of each system inside the kernel.
//
// Control flow.  Teams that share a wave (16- or 32-lane teams) run in lockstep
// through the same instruction stream: every cross-lane operation is executed by
// all lanes, and per-team state changes are committed under per-team
// predicates.  A team that has finished keeps executing (its results are
// discarded) until every team of its wave has finished.  Multi-wave teams make
// identical decisions in every wave because every wave reads the same reduced
// bits, so all their barriers match.
//
// Stop test.  ||r||_2 <= tol*||b||_2 on the recurrence residual, confirmed on the
// true residual b - A x; if the confirmation fails and iterations remain, the
// method restarts from the true residual.  (The paper's Alg. 1 tests |r.z|
// against a threshold; its Tab. 2 lists a relative criterion, which is used.)
#pragma once
#include <type_traits>

#include "bs_device.hpp"

namespace bs {

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Stop level on ||r||_2 (Tab. 2): tol * ||b||_2 (relative) or tol (absolute).
template <class G>
__device__ __forceinline__ double stop_limit(const G& g, double bn) {
  return (g.flags & kFlagAbsTol) ? g.tol : g.tol * bn;
}

// ------------------------------------------------------------ block Jacobi
// v of lane src of this wave (a cross-lane permute through the LDS crossbar,
// no memory access); every lane must be active.
__device__ __forceinline__ double shfl(double v, int src) {
  const int a = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Blocks of bs consecutive rows (bs = 2, 4 or 8; the last block may be
// shorter); M = the inverse of the block diagonal of A.  Per team in LDS: the
// inverse stored by columns, binv[j*rows + i] = entry (i, b0 + j) (b0 = i - i %
// bs), so that the lanes of a wave touch consecutive elements, and a
// row-indexed exchange buffer pbuf[rows].  The rows of one block always sit in
// one wave, on consecutive lanes (bs divides the rows a wave holds, and block
// Jacobi runs with row i on lane i of its team), so a wavefront-scope fence
// orders the exchanges.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// Inverse of every diagonal block by Gauss-Jordan elimination without
// pivoting: for each pivot p, row p is scaled by the pivot's reciprocal (its
// diagonal entry becoming 1/pivot), then every other row r subtracts a_rp times
// it (its entry p becoming -a_rp/pivot).  A zero or non-finite pivot, or a
// non-finite entry of the result, makes the block the identity.  The block's
// entries are scattered from the register slots (their columns found by
// gathering a vector that holds each row's own index), the elimination runs in
// registers, and the result is stored by columns.  All lanes of the workgroup
// call it together.
//
// After the gather, every LDS access stays inside the wave that owns the rows:
// a block's rows lie in one wave, and its failure flag is the exchange entry
// of its first row.  Waves of a multi-wave team may therefore leave at
// different times and go straight into bj_apply, which writes only the
// entries of its own rows.
template <class TM, class RW>
__device__ void bj_setup(TM& tm, RW& A, const KArgs& g) {
  constexpr int R = RW::R;
  const int bs = g.block, n = A.nrows(g), rows = tm.bj_rows(), per = rows / R;
  double* binv = tm.bj_region(g);
  double* pbuf = binv + (size_t)rows * bs;
  const int lane = tm.lane;
  // clear the exchange buffer (also the per-block failure flags) and the rows
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + r * per;
    pbuf[i] = 0.0;
#pragma unroll 1
    for (int j = 0; j < bs; ++j) binv[j * rows + i] = 0.0;
  }
  // each row's own index into buffer 1, then gather it through the slots
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (A.ok[r]) lds_store<double>(A.vrow[r] + RW::kBuf, (double)A.row[r]);
  tm.sync();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = A.row[r], b0 = i - (i & (bs - 1));
#pragma unroll
    for (int k0 = 0; k0 < RW::NZ; k0 += 4) {
      int col[4];
#pragma unroll
      for (int k = k0; k < k0 + 4 && k < RW::NZ; ++k)
        col[k - k0] = (int)lds_load<double>(A.c[r][k] + RW::kBuf);
#pragma unroll
      for (int k = k0; k < k0 + 4 && k < RW::NZ; ++k)
        if (A.ok[r] && A.real(r, k) && col[k - k0] >= b0 && col[k - k0] < b0 + bs)
          binv[(col[k - k0] - b0) * rows + i] = A.a[r][k];
      // four gathers in flight at a time
      __asm__ volatile("" ::: "memory");
    }
  }
  wave_lds_fence();
  // Gauss-Jordan in registers.  The rows of a block sit on consecutive lanes
  // of one wave (row i on lane i of its team: the plain layout), so each lane
  // reads the pivot row from its lane with a cross-lane permute.  Every row
  // other than p subtracts its entry p times row p scaled by one reciprocal of
  // the pivot; row p takes the scaled row.  A zero or non-finite pivot, or a
  // non-finite entry of the result, raises the block's flag (the exchange
  // entry of its first row, in the same wave) and the block becomes the
  // identity.  All lanes run every step (the permutes read every lane).
  const int me = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = A.row[r], ib = i & (bs - 1), b0 = i - ib;
    double m[kMaxBlock];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) m[j] = (A.ok[r] && j < bs) ? binv[j * rows + i] : 0.0;
#pragma unroll 1
    for (int p = 0; p < bs; ++p) {
      const int src = me - ib + p;  // lane of row b0 + p
      double q[kMaxBlock];
#pragma unroll
      for (int j = 0; j < kMaxBlock; ++j) q[j] = j < bs ? shfl(m[j], src) : 0.0;
      double piv = q[0], f = m[0];
#pragma unroll
      for (int j = 1; j < kMaxBlock; ++j) {
        piv = j == p ? q[j] : piv;
        f = j == p ? m[j] : f;
      }
      const bool act = A.ok[r] && b0 + p < n, own = ib == p;
      if (act && (piv == 0.0 || !__builtin_isfinite(piv))) bad = true;
      const double rp = 1.0 / piv;
#pragma unroll
      for (int j = 0; j < kMaxBlock; ++j) {
        const double qs = (j == p ? 1.0 : q[j]) * rp;  // row p after this step
        const double upd = own ? qs : fma(-f, qs, j == p ? 0.0 : m[j]);
        m[j] = act ? upd : m[j];
      }
    }
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) bad = bad || (j < bs && !__builtin_isfinite(m[j]));
    if (A.ok[r] && bad) pbuf[b0] = 1.0;
    wave_lds_fence();
    if (A.ok[r]) {
      const bool ident = pbuf[b0] != 0.0;
#pragma unroll
      for (int j = 0; j < kMaxBlock; ++j)
        if (j < bs) binv[j * rows + i] = ident ? (j == ib ? 1.0 : 0.0) : m[j];
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int r = 0; r < R; ++r) pbuf[lane + r * per] = 0.0;
  wave_lds_fence();
}

// z = M v for the block-Jacobi M (rows past n give 0).  All lanes of a wave call
// it together.
template <class T, class TM, class RW>
__device__ __forceinline__ void bj_apply(TM& tm, const RW& A, const KArgs& g,
                                         const T (&v)[RW::R], T (&z)[RW::R]) {
  constexpr int R = RW::R;
  const int bs = g.block, rows = tm.bj_rows();
  const double* binv = tm.bj_region(g);
  double* pbuf = tm.bj_region(g) + (size_t)rows * bs;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (A.ok[r]) pbuf[A.row[r]] = (double)v[r];
  wave_lds_fence();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T acc = (T)0;
    if (A.ok[r]) {
      const int i = A.row[r], b0 = i - (i & (bs - 1));
      // four columns of the inverse row and of the block's slice of v per
      // batch of loads
#pragma unroll
      for (int h = 0; h < kMaxBlock; h += 4) {
        if (h >= bs) break;
        double w[4], u[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          w[j] = h + j < bs ? binv[(h + j) * rows + i] : 0.0;
          u[j] = h + j < bs ? pbuf[b0 + h + j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = fma((T)w[j], (T)u[j], acc);
      }
    }
    z[r] = acc;
  }
  wave_lds_fence();
}

// ------------------------------------------------------------------ ILU(0)
// ILU(0) for one-wave teams (row i on lane i, one row per lane, n <= 64).  The
// factors live in the team's LDS region as F, row-major with an odd stride
// (the rows of a wave fall on distinct bank pairs) and zero columns padding
// each row to a multiple of 8: L strictly below the diagonal (unit diagonal
// implied), U on and above, zero off the pattern.

__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Factorization (Saad 2003, Sec. 10.3.2), right-looking: for pivot k, every row
// i > k that holds column k replaces that entry by l_ik = a_ik / u_kk (a
// division, as the IKJ form writes it) and subtracts l_ik u_kj from each of
// its entries j > k; row k's pattern (a wave-uniform bitmask read from lane k)
// bounds the columns visited, eight per batch of loads, and a row's own
// pattern mask selects which of them change, so nothing fills in (the others
// are stored back unchanged).  Each entry receives its updates in increasing
// k, as in the IKJ form.  d gets the pivot u_ii (1 on idle lanes), which the
// backward sweep divides by.  A zero pivot or a non-finite factor entry
// anywhere in the system turns M into the identity (F zero, d = 1).
template <class TM, class RW>
__device__ void ilu_setup(TM& tm, RW& A, const KArgs& g, double (&d)[RW::R]) {
  static_assert(RW::R == 1 && RW::TEAM == kWave, "ILU(0) runs on one-wave teams");
  constexpr int kB = 8;
  const int n = g.n, st = ilu_stride(n);
  double* F = tm.bj_region(g);
  const int lane = tm.lane;
  const bool ok = A.ok[0];
  const int i = ok ? A.row[0] : 0;  // rows past n address row 0 and never store
  for (int e = lane; e < n * st; e += kWave) F[e] = 0.0;
  // columns of the register slots: gather a vector holding each row's index
  if (ok) lds_store<double>(A.vrow[0] + RW::kBuf, (double)i);
  tm.sync();
  uint64_t mask = 0;
#pragma unroll
  for (int k0 = 0; k0 < RW::NZ; k0 += 4) {
    int col[4];
#pragma unroll
    for (int k = k0; k < k0 + 4 && k < RW::NZ; ++k)
      col[k - k0] = (int)lds_load<double>(A.c[0][k] + RW::kBuf);
#pragma unroll
    for (int k = k0; k < k0 + 4 && k < RW::NZ; ++k)
      if (ok && A.real(0, k)) {
        F[i * st + col[k - k0]] = A.a[0][k];
        mask |= 1ull << col[k - k0];
      }
    __asm__ volatile("" ::: "memory");
  }
  wave_lds_fence();
#pragma unroll 1
  for (int k = 0; k + 1 < n; ++k) {
    uint64_t cols = rdlane64(mask, k);
    cols = k >= 63 ? 0 : cols & (~0ull << (k + 1));
    const bool act = ok && i > k && ((mask >> k) & 1);
    const double piv = F[k * st + k];
    const double aik = F[i * st + k];
    const double l = act ? aik / piv : 0.0;
    if (act) F[i * st + k] = l;
    while (cols) {  // wave-uniform
      int j[kB];
      bool has[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        has[q] = cols != 0;
        j[q] = has[q] ? __builtin_ctzll(cols) : k;
        cols &= cols - 1;
      }
      double u[kB], f[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        u[q] = F[k * st + j[q]];
        f[q] = F[i * st + j[q]];
      }
      if (ok) {
#pragma unroll
        for (int q = 0; q < kB; ++q)
          if (has[q]) F[i * st + j[q]] = ((mask >> j[q]) & 1) ? fma(-l, u[q], f[q]) : f[q];
      }
    }
    wave_lds_fence();
  }
  // a zero pivot or a non-finite entry: the identity for the whole system
  bool bad = false;
  if (ok) {
    bad = F[i * st + i] == 0.0;
    for (int j0 = 0; j0 < n; j0 += 8) {
      double f[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = F[i * st + j0 + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) bad = bad || !__builtin_isfinite(f[q]);
    }
  }
  if (wave_any(bad)) {
    wave_lds_fence();
    for (int e = lane; e < n * st; e += kWave) F[e] = 0.0;
    d[0] = 1.0;
  } else {
    d[0] = ok ? F[i * st + i] : 1.0;
  }
  wave_lds_fence();
}

// z = (L U)^{-1} v by two column sweeps: forward, y_k (final on lane k) is
// read out and every row i > k subtracts l_ik y_k; backward, z_j = y_j / u_jj
// (a division by the pivot d of lane j) and every row i < j subtracts u_ij z_j.
// Entries off the pattern, and the padding columns (read out from idle lanes,
// whose values are zero and whose d is 1), add nothing.  The sums run in
// increasing k (forward) and decreasing j (backward).  With M the identity F
// is zero and d = 1, so z = v.
template <class T, class TM, class RW>
__device__ __forceinline__ void ilu_apply(TM& tm, const RW& A, const KArgs& g,
                                          const T (&d)[RW::R], const T (&v)[RW::R],
                                          T (&z)[RW::R]) {
  const int n = g.n, st = ilu_stride(n), n8 = st - 1;
  const double* F = tm.bj_region(g);
  const bool ok = A.ok[0];
  const int i = ok ? A.row[0] : 0;
  const int ilo = ok ? i : kWave, ihi = ok ? i : -1;  // idle lanes take no term
  const double dv = (double)d[0];
  double acc = ok ? (double)v[0] : 0.0;
  for (int k0 = 0; k0 < n8; k0 += 8) {
    double lk[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) lk[q] = F[i * st + k0 + q];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      acc = fma(ilo > k0 + q && ilo < kWave ? -lk[q] : 0.0, rdlane(acc, k0 + q), acc);
  }
  for (int j0 = n8 - 8; j0 >= 0; j0 -= 8) {
    double uj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) uj[q] = F[i * st + j0 + 7 - q];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double zj = rdlane(acc / dv, j0 + 7 - q);
      acc = fma(ihi < j0 + 7 - q && ihi >= 0 ? -uj[q] : 0.0, zj, acc);
    }
  }
  z[0] = ok ? (T)(acc / dv) : (T)0;
}

// ------------------------------------------------ ILU(0), multi-wave teams
// Teams of 2..16 waves (row i on lane i, one row per lane, up to 1024 rows)
// keep the factors sparse, in the pattern's CSR order, and run the
// factorization and both sweeps level by level (level scheduling; Saad 2003,
// Ch. 11): a row's level in the lower triangle is one more than the largest
// level among the rows its strictly lower entries name (0 if none), and its
// level in the upper triangle is defined the same way from its strictly upper
// entries.  Rows of one level depend only on earlier levels.  The
// factorization takes one level per team barrier, each lane its own row; the
// sweeps run on the team's first wave alone, whose LDS operations complete in
// issue order, so that levels follow one another without a barrier.  The
// levels, the factorization schedule and the sweep lists come with the
// pattern.

// The pattern's sweep lists into the team's region, once per kernel (they are
// the same for every system): rows in lower then upper level order and the
// level starts as 16-bit values, each row's list start and counts, the lists.
template <class TM>
__device__ __forceinline__ void sweep_lists_load(TM& tm, const KArgs& g, unsigned reg,
                                                 const IluMw& L) {
  if (tm.lists) return;
  const int n = g.n, nl = g.nlev_l + g.nlev_u + 2;
  const int* sw = g.sweep;
  for (int t = threadIdx.x; t < 2 * n; t += blockDim.x)
    lds_store<short>(reg + L.rows + t * 2, (short)sw[t]);
  for (int t = threadIdx.x; t < nl; t += blockDim.x)
    lds_store<short>(reg + L.lvl + t * 2, (short)sw[2 * n + t]);
  for (int t = threadIdx.x; t < n; t += blockDim.x)
    lds_store<int>(reg + L.rng + t * 4, sw[2 * n + nl + t]);
  for (int t = threadIdx.x; t < g.sweep_ents; t += blockDim.x)
    lds_store<int>(reg + L.ent + t * 4, sw[3 * n + nl + t]);
  tm.lists = true;
}

// One triangular sweep over the team's sweep vector y, run by the team's first
// wave: for the rows of each level in turn, lane t takes the level's t-th row r
// (then the (t+64)-th, ...) and sets y_r <- (y_r - sum_c t_rc y_c) [/ d_r] over
// the row's strictly lower (LOWER) or upper entries in increasing column, t_rc
// from the values at their CSR positions; DIV divides by d_r.  Pipelined so
// that only this level's gathers wait on the previous level: the level ends
// are read two levels ahead, the next level's first row before this level's
// list words, and that row's list range once this level's loads are out.
template <bool LOWER, bool DIV>
__device__ __forceinline__ void tri_sweep(const KArgs& g, unsigned reg, const IluMw& L) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned F = reg + L.f, Y = reg + L.y, D = reg + L.d, RNG = reg + L.rng, ENT = reg + L.ent;
  const unsigned ROWS = reg + L.rows + (LOWER ? 0 : g.n * 2);
  const unsigned LVL = reg + L.lvl + (LOWER ? 0 : (g.nlev_l + 1) * 2);
  const int nlev = LOWER ? g.nlev_l : g.nlev_u;
  // y_r update of one row from its list range gg (the list words, then the
  // values and gathers, four terms at a time)
  auto row = [&](int rr, unsigned gg) {
    const int lc = (int)((gg >> 16) & 0xffu);
    const int e0 = (int)(gg & 0xffffu) + (LOWER ? 0 : lc);
    const int e1 = e0 + (LOWER ? lc : (int)(gg >> 24));
    double acc = lds_load<double>(Y + rr * 8);
    for (int e = e0; e < e1; e += 4) {
      unsigned w[4];
      double f[4], y[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] = e + k < e1 ? lds_load<unsigned>(ENT + (e + k) * 4) : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        f[k] = e + k < e1 ? lds_load<double>(F + (w[k] & 0x7fffu) * 8) : 0.0;
        y[k] = e + k < e1 ? lds_load<double>(Y + (w[k] >> 16) * 8) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (e + k < e1) acc = fma(-f[k], y[k], acc);
    }
    if (DIV) acc = acc / lds_load<double>(D + rr * 8);
    lds_store<double>(Y + rr * 8, acc);
  };
  int qa = lds_load<short>(LVL), qb = lds_load<short>(LVL + 2);
  int qc = nlev > 1 ? lds_load<short>(LVL + 4) : qb;  // end of the next level
  int r = qa + lane < qb ? lds_load<short>(ROWS + (qa + lane) * 2) : -1;
  unsigned rg = r >= 0 ? lds_load<unsigned>(RNG + r * 4) : 0u;
  for (int l = 0; l < nlev; ++l) {
    const int qd = l + 2 < nlev ? lds_load<short>(LVL + (l + 3) * 2) : qc;
    const int nr = qb + lane < qc ? lds_load<short>(ROWS + (qb + lane) * 2) : -1;
    // This level's first row on each lane, rows of up to four terms without
    // branches: list words at clamped indices, words past the row's count (and
    // on lanes without a row) replaced by 0 (entry 0, column 0: valid
    // addresses), their terms dropped by selection.  The next row's list range
    // is read once this level's loads are out.
    const int lc = (int)((rg >> 16) & 0xffu);
    const int e0 = (int)(rg & 0xffffu) + (LOWER ? 0 : lc);
    const int ne = r >= 0 ? (LOWER ? lc : (int)(rg >> 24)) : 0;
    const int rs = r >= 0 ? r : 0;
    const int last = g.sweep_ents > 0 ? g.sweep_ents - 1 : 0;
    unsigned w[4];
    double f[4], y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned wk = lds_load<unsigned>(ENT + min(e0 + k, last) * 4);
      w[k] = k < ne ? wk : 0u;
    }
    const double y0 = lds_load<double>(Y + rs * 8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      f[k] = lds_load<double>(F + (w[k] & 0x7fffu) * 8);
      y[k] = lds_load<double>(Y + (w[k] >> 16) * 8);
    }
    const unsigned ng = nr >= 0 ? lds_load<unsigned>(RNG + nr * 4) : 0u;
    if (r >= 0) {
      if (ne <= 4) {
        double acc = y0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double t = fma(-f[k], y[k], acc);
          acc = k < ne ? t : acc;
        }
        if (DIV) acc = acc / lds_load<double>(D + r * 8);
        lds_store<double>(Y + r * 8, acc);
      } else {
        row(r, rg);
      }
    }
    for (int q = qa + kWave; q < qb; q += kWave) {  // levels of more than 64 rows
      const int rr = q + lane < qb ? lds_load<short>(ROWS + (q + lane) * 2) : -1;
      if (rr >= 0) row(rr, lds_load<unsigned>(RNG + rr * 4));
    }
    qa = qb;
    qb = qc;
    qc = qd;
    r = nr;
    rg = ng;
    __asm__ volatile("" ::: "memory");
  }
}

// Factorization, the IKJ form of the one-wave code, from the pattern's
// symbolic schedule: at its level, row i takes the columns k < i it holds in
// increasing order, replaces f_ik by f_ik / u_kk and subtracts f_ik u_kj from
// each of its entries (i,j), j > k, that row k holds; the schedule lists, per
// row, one header word per k (the positions of (i,k) and (k,k)) followed by
// one word per update (the positions of (i,j) and (k,j)).  Row k is final by
// then; row i's values are updated in place in LDS, where no other row of its
// level reads them.  Each entry so receives its updates in increasing k.  The
// row then stores its pivot.  A zero pivot or a non-finite factor entry
// anywhere in the system turns M into the identity (row values 0, pivots 1).
constexpr int kIluOpsReg = 16;  // schedule words a lane takes per pass

template <class TM, class RW>
__device__ void ilu_setup_mw(TM& tm, const RW& A, const KArgs& g) {
  static_assert(RW::R == 1 && RW::TEAM > kWave, "multi-wave ILU(0): one row per lane");
  constexpr int NZ = RW::NZ;
  const IluMw L = ilu_mw_layout(g.n, g.nnz);
  const unsigned reg = lds_addr(tm.bj_region(g));
  const unsigned F = reg + L.f, D = reg + L.d;
  sweep_lists_load(tm, g, reg, L);
  const bool ok = A.ok[0];
  int i = ok ? A.row[0] : 0;
  // opaque once per system: everything below derives from the pattern, and
  // would otherwise be loaded or formed once per kernel and pin registers
  // through the whole solve
  __asm__ volatile("" : "+v"(i));
  const int lv = ok ? g.lev[i] : 0;
  const int fb = g.fmt == 0 ? A.w[0] : g.row_ptr[i];  // CSR position of register slot 0
  const unsigned fr = F + fb * 8;
  const int o0 = g.ilu_ptr[i], o1 = ok ? g.ilu_ptr[i + 1] : o0;
  // Shapes of up to 16 slots load the row's first words before the level loop
  // (all lanes at once); wider ones, short of registers, load them when the
  // row's level comes.
  constexpr bool kEarly = NZ <= 16;
  unsigned w[kIluOpsReg];
#pragma unroll
  for (int q = 0; q < kIluOpsReg; ++q)
    w[q] = kEarly && o0 + q < o1 ? (unsigned)g.ilu_ops[o0 + q] : 0u;
  // publish the row's values
  if (ok) {
#pragma unroll
    for (int s = 0; s < NZ; ++s)
      if (A.real(0, s)) lds_store<double>(fr + s * 8, A.a[0][s]);
  }
  tm.sync();
  const int mine = ok ? (lv & 0xffff) : -1;
  for (int l = 0; l < g.nlev_l; ++l) {
    if (mine == l) {
      double lik = 0.0;
      for (int b0 = o0; b0 < o1; b0 += kIluOpsReg) {
        if (kEarly && b0 != o0) {
#pragma unroll
          for (int q = 0; q < kIluOpsReg; ++q)
            w[q] = b0 + q < o1 ? (unsigned)g.ilu_ops[b0 + q] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kIluOpsReg; ++q) {
          if (b0 + q < o1) {
            const unsigned op = kEarly ? w[q] : (unsigned)g.ilu_ops[b0 + q];
            if (op >> 31) {
              const unsigned aik = F + (op & 0x7fffu) * 8, akk = F + ((op >> 15) & 0x7fffu) * 8;
              lik = lds_load<double>(aik) / lds_load<double>(akk);
              lds_store<double>(aik, lik);
            } else {
              const unsigned aij = F + (op & 0xffffu) * 8, akj = F + (op >> 16) * 8;
              lds_store<double>(aij, fma(-lik, lds_load<double>(akj), lds_load<double>(aij)));
            }
          }
        }
      }
      lds_store<double>(D + i * 8, A.dslot[0] >= 0 ? lds_load<double>(fr + A.dslot[0] * 8) : 0.0);
    }
    tm.sync();
  }
  bool bad = false;
  if (ok) {
    bad = lds_load<double>(D + i * 8) == 0.0;
#pragma unroll
    for (int s = 0; s < NZ; ++s)
      bad = bad || (A.real(0, s) && !__builtin_isfinite(lds_load<double>(fr + s * 8)));
  }
  if (__syncthreads_or(bad)) {
    if (ok) {
#pragma unroll
      for (int s = 0; s < NZ; ++s)
        if (A.real(0, s)) lds_store<double>(fr + s * 8, 0.0);
      lds_store<double>(D + i * 8, 1.0);
    }
    tm.sync();
  }
}

// z = (L U)^{-1} v by the two row-oriented substitutions of the oracle's
// default form on the team's first wave: forward, y_i = v_i - sum_{k<i} l_ik
// y_k; backward, z_i = (y_i - sum_{j>i} u_ij z_j) / u_ii, each row's terms in
// increasing column.  With M the identity the row values are zero and the
// pivots 1, so z = v.
template <class T, class TM, class RW>
__device__ __forceinline__ void ilu_apply_mw(TM& tm, const RW& A, const KArgs& g,
                                             const T (&v)[RW::R], T (&z)[RW::R]) {
  const IluMw L = ilu_mw_layout(g.n, g.nnz);
  const unsigned reg = lds_addr(tm.bj_region(g));
  const unsigned me = reg + L.y + (unsigned)A.row[0] * 8;
  if (A.ok[0]) lds_store<double>(me, (double)v[0]);
  tm.sync();
  if (threadIdx.x < kWave) {
    tri_sweep<true, false>(g, reg, L);
    tri_sweep<false, true>(g, reg, L);
  }
  tm.sync();
  z[0] = A.ok[0] ? (T)lds_load<double>(me) : (T)0;
}

// z = M v: block Jacobi or ILU(0) in their instances, else the diagonal d
// (scalar Jacobi, or 1 without a preconditioner).
template <int PK, class T, class TM, class RW>
__device__ __forceinline__ void precond(TM& tm, const RW& A, const KArgs& g, const T (&d)[RW::R],
                                        const T (&v)[RW::R], T (&z)[RW::R]) {
  if constexpr (PK == kPkBlock) {
    bj_apply(tm, A, g, v, z);
  } else if constexpr (PK == kPkIlu) {
    if constexpr (RW::TEAM > kWave) ilu_apply_mw(tm, A, g, v, z);
    else ilu_apply(tm, A, g, d, v, z);
  } else {
#pragma unroll
    for (int r = 0; r < RW::R; ++r) z[r] = d[r] * v[r];
  }
}

// Shared epilogue: true residual for teams that do not have it, then outputs.
template <class TM, class RW>
__device__ __forceinline__ void finish(TM& tm, const RW& A, const KArgs& g,
                                       const double (&b)[RW::R], const double (&x)[RW::R], int st,
                                       int k, int outer, double bn, double rn, bool have_rn) {
  // the output addresses first: their scalar loads then overlap the residual
  // below instead of waiting one after another before each store
  double* const gx = g.x;
  int* const gi = g.iters;
  double* const gr = g.resid;
  const bool has_status = g.status != nullptr;
  int* const gs = has_status ? g.status : g.sink;
  int* const go = g.outer;
  const int flags = g.flags;
  __asm__ volatile("" ::"s"(gx), "s"(gi), "s"(gr), "s"(gs), "s"(go), "s"(flags));
  const bool need = tm.live && !have_rn;
  if (tm.any(need)) {
    double t[RW::R], q[1];
    A.template spmv<0>(tm, A.a, x, t);
    double p[RW::R];
#pragma unroll
    for (int r = 0; r < RW::R; ++r) { const double e = b[r] - t[r]; p[r] = e * e; }
    q[0] = sum_rows(p);
    tm.sum(q);
    if (need) rn = sqrt(q[0]);
  }
  if (!tm.live) return;
#pragma unroll
  for (int r = 0; r < RW::R; ++r)
    if (A.ok[r]) gx[tm.row0 + A.row[r]] = x[r];
  if (tm.lane == 0) {
    gi[tm.sys] = k;
    // the true residual, relative to ||b|| unless the criterion is absolute
    gr[tm.sys] = !finite(bn) ? bn : ((bn == 0.0 || (flags & kFlagAbsTol)) ? rn : rn / bn);
    // always one store (to the sink when no status is wanted): the persistent
    // loop counts on a fixed number of stores after each prefetch
    gs[has_status ? tm.sys : 0] = st;
    if (go) go[tm.sys] = outer;
  }
}

// Shared prologue: load the system, its Jacobi diagonal, b, x0 and the initial
// residual r0 = b - A x0 (r0 = b when x0 = 0 is promised).
template <int R>
struct Prologue {
  double b[R], x[R], r[R], d[R];
};

template <int PK, class TM, class RW>
__device__ __forceinline__ void prologue(TM& tm, RW& A, const KArgs& g, Prologue<RW::R>& P) {
  A.jacobi(g.precond, P.d);
  if constexpr (PK == kPkBlock) bj_setup(tm, A, g);
  if constexpr (PK == kPkIlu) {
    if constexpr (RW::TEAM > kWave) ilu_setup_mw(tm, A, g);
    else ilu_setup(tm, A, g, P.d);
  }
  const bool x0zero = (g.flags & 1) != 0;
#pragma unroll
  for (int r = 0; r < RW::R; ++r) {
    P.b[r] = A.bval[r];
    P.x[r] = A.xval[r];
  }
  if (!x0zero) {
    double t[RW::R];
    A.template spmv<0>(tm, A.a, P.x, t);
#pragma unroll
    for (int r = 0; r < RW::R; ++r) P.r[r] = P.b[r] - t[r];
    if (g.x_alt) {
      // Second candidate start: keep whichever has the smaller residual
      // norm (x on a tie; x_alt also when only x's norm is not a number).
      // The other buffer: lanes may still gather from buffer 0.
      double ta[RW::R], ra[RW::R], p0[RW::R], p1[RW::R];
      A.template spmv<1>(tm, A.a, A.xalt, ta);
#pragma unroll
      for (int r = 0; r < RW::R; ++r) {
        ra[r] = P.b[r] - ta[r];
        p0[r] = P.r[r] * P.r[r];
        p1[r] = ra[r] * ra[r];
      }
      double q[2] = {sum_rows(p0), sum_rows(p1)};
      tm.sum(q);
      const bool alt = q[1] < q[0] || (q[0] != q[0] && q[1] == q[1]);
#pragma unroll
      for (int r = 0; r < RW::R; ++r) {
        P.x[r] = alt ? A.xalt[r] : P.x[r];
        P.r[r] = alt ? ra[r] : P.r[r];
      }
      if (g.alt_used && tm.live && tm.lane == 0) g.alt_used[tm.sys] = alt ? 1 : 0;
    }
  } else {
#pragma unroll
    for (int r = 0; r < RW::R; ++r) P.r[r] = P.b[r];
  }
}

// =================================================================== BiCGSTAB
// Right-preconditioned BiCGSTAB (van der Vorst 1992), the solver the paper
// evaluates on all application inputs (Sec. 4.3).  Per iteration: two SpMVs and
// three fused reductions (r^.v; s.s, t.t, t.s; r.r, r^.r).  The second SpMV is
// issued before the half-step test so that ||s|| joins the t-reduction; it is
// discarded when the half step already converges.
//
// MIXED: the Krylov vectors, the FP32 copy of A and the inner reductions are
// FP32 and solve for a correction to the FP64 x, scaled by 1/||r||; the "true
// residual confirmation" becomes the FP64 outer refinement step r = b - A x,
// which also ends the inner solve when it meets inner_tol or breaks down.
template <bool MIXED, int PK, class TM, class RW>
__device__ __forceinline__ void bicgstab_system(TM& tm, RW& A, const KArgs& g) {
  using T = typename std::conditional<MIXED, float, double>::type;
  Prologue<RW::R> P;
  prologue<PK>(tm, A, g, P);
  constexpr int R = RW::R;

  // FP32 copy of the rows and of the Jacobi diagonal for the inner solve.
  using AT = typename std::conditional<MIXED, float, double>::type;
  AT a_in[R][RW::NZ];
  T d_in[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    d_in[r] = (T)P.d[r];
#pragma unroll
    for (int k = 0; k < RW::NZ; ++k) {
      // slots without an entry of the row may hold other rows' values: zero
      // them so that a value beyond FP32 range cannot meet the zero cell as Inf
      if constexpr (MIXED) a_in[r][k] = A.real(r, k) ? (AT)A.a[r][k] : (AT)0;
      else a_in[r][k] = (AT)A.a[r][k];
    }
  }

  double q2[2];
  {
    double p0[R], p1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { p0[r] = P.b[r] * P.b[r]; p1[r] = P.r[r] * P.r[r]; }
    q2[0] = sum_rows(p0);
    q2[1] = sum_rows(p1);
    tm.sum(q2);
  }
  const double bn = sqrt(q2[0]);
  double rn = sqrt(q2[1]);  // FP64 norm of the outer (or only) residual
  const double lim = stop_limit(g, bn);
  int st = tm.live ? ST_RUNNING : ST_IDLE;
  bool rtrue = true;
  if (st == ST_RUNNING) {
    if (!finite(bn)) st = ST_NONFINITE;
    else if (bn == 0.0) {
      st = ST_CONVERGED;
#pragma unroll
      for (int r = 0; r < R; ++r) P.x[r] = 0.0;
      rn = 0.0;
    }
  }
  int k = 0, outer = 0;

  // Krylov state.
  T r[R], rh[R], p[R], v[R];
  T rho, rho0, alpha, omega, rr_in;  // rr_in: squared norm of the inner residual
  double scale;  // x += scale * (inner update)
  double rn_prev = rn;
  auto restart = [&](double rtrue_norm) {
    // r_in = r / scale; r^ = r_in; p = v = 0; rho0 = alpha = omega = 1
    scale = MIXED ? rtrue_norm : 1.0;
    const double inv = MIXED ? (rtrue_norm > 0.0 ? 1.0 / rtrue_norm : 0.0) : 1.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      r[i] = (T)(MIXED ? P.r[i] * inv : P.r[i]);
      rh[i] = r[i];
      p[i] = 0;
      v[i] = 0;
    }
    rho0 = alpha = omega = (T)1;
  };
  restart(rn);
  if constexpr (MIXED) {
    T q[1];
    T pr[R];
#pragma unroll
    for (int i = 0; i < R; ++i) pr[i] = r[i] * r[i];
    q[0] = sum_rows(pr);
    tm.sum(q);
    rho = q[0];
    rr_in = q[0];
  } else {
    rho = (T)q2[1];  // r^ = r, so r^.r is the same sum as r.r
    rr_in = (T)q2[1];
  }
  // Inner stop level: absolute on the same scale as r_in.
  auto inner_lim = [&]() -> T {
    if constexpr (MIXED) {
      const double want = 0.5 * lim / (rn > 0.0 ? rn : 1.0);
      return (T)(want > g.inner_tol ? want : g.inner_tol);
    } else {
      return (T)lim;
    }
  };
  // The recurrence tests compare squared norms (no square root per test);
  // the true-residual confirmation below compares the norm itself.
  T ilim = inner_lim();
  T ilim2 = ilim * ilim;
  bool inner_end = false;  // MIXED: inner solve ended (met inner tol or broke down)

  for (;;) {
    // ---- top: convergence / budget checks, per team
    bool need_chk = false;
    if (st == ST_RUNNING) {
      if (MIXED ? !finite(rn) : !finite((double)rr_in)) {
        st = ST_NONFINITE;
      } else if (MIXED ? (rn <= lim || inner_end || rr_in <= ilim2) : (rr_in <= ilim2)) {
        if (!MIXED && rtrue) st = ST_CONVERGED;
        else if (MIXED && rtrue && rn <= lim) st = ST_CONVERGED;
        else need_chk = true;
      } else if (k >= g.max_iter) {
        st = ST_MAX_ITER;
      }
    }
    if (tm.any(need_chk)) {
      // ---- true residual (plain) / outer refinement step (mixed), FP64
      double t[R], pr[R], q[1];
      A.template spmv<0>(tm, A.a, P.x, t);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const double e = P.b[i] - t[i];
        if (need_chk) P.r[i] = e;
        pr[i] = e * e;
      }
      q[0] = sum_rows(pr);
      tm.sum(q);
      if (need_chk) {
        const double rnc = sqrt(q[0]);
        rtrue = true;
        if constexpr (MIXED) outer += 1;
        const bool stagnant = MIXED && !(rnc < rn_prev);
        rn = rnc;
        rn_prev = rnc;
        if (!finite(rnc)) st = ST_NONFINITE;
        else if (rnc <= lim) st = ST_CONVERGED;
        else if (k >= g.max_iter) st = ST_MAX_ITER;
        else if (stagnant) st = ST_BREAKDOWN;
        else {
          restart(rnc);
          inner_end = false;
          ilim = inner_lim();
          ilim2 = ilim * ilim;
        }
      }
      if constexpr (MIXED) {
        // new inner residual norm and rho for restarted teams
        T qq[1], pp[R];
#pragma unroll
        for (int i = 0; i < R; ++i) pp[i] = r[i] * r[i];
        qq[0] = sum_rows(pp);
        tm.sum(qq);
        if (need_chk && st == ST_RUNNING) { rho = qq[0]; rr_in = qq[0]; }
      } else {
        if (need_chk && st == ST_RUNNING) { rho = (T)q[0]; rr_in = (T)q[0]; }
      }
      continue;
    }
    if (!tm.any(st == ST_RUNNING)) break;

    // ---- one BiCGSTAB iteration; committed for teams still running
    bool go = st == ST_RUNNING;
    if (go) {
      k += 1;
      if (!finite((double)rho)) {
        if (MIXED) inner_end = true; else st = ST_NONFINITE;
        go = false;
      } else if (rho == (T)0) {
        if (MIXED) inner_end = true; else st = ST_BREAKDOWN;
        go = false;
      }
    }
    const T beta = (rho * alpha) / (rho0 * omega);
    T ph[R], s[R], sh[R], t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    precond<PK>(tm, A, g, d_in, p, ph);
    A.template spmv<0>(tm, a_in, ph, v);
    T q1[1];
    {
      T pr[R];
#pragma unroll
      for (int i = 0; i < R; ++i) pr[i] = rh[i] * v[i];
      q1[0] = sum_rows(pr);
    }
    tm.sum(q1);
    const T sigma = q1[0];
    if (go) {
      if (!finite((double)sigma)) { if (MIXED) inner_end = true; else st = ST_NONFINITE; go = false; }
      else if (sigma == (T)0) { if (MIXED) inner_end = true; else st = ST_BREAKDOWN; go = false; }
    }
    const T al = rho / sigma;
#pragma unroll
    for (int i = 0; i < R; ++i) s[i] = r[i] - al * v[i];
    precond<PK>(tm, A, g, d_in, s, sh);
    A.template spmv<1>(tm, a_in, sh, t);
    T q3[3];
    {
      T p0[R], p1[R], p2[R];
#pragma unroll
      for (int i = 0; i < R; ++i) { p0[i] = s[i] * s[i]; p1[i] = t[i] * t[i]; p2[i] = t[i] * s[i]; }
      q3[0] = sum_rows(p0);
      q3[1] = sum_rows(p1);
      q3[2] = sum_rows(p2);
    }
    tm.sum(q3);
    const T ss = q3[0], tt = q3[1], ts = q3[2];
    bool half = false;
    if (go) {
      if (!finite((double)ss)) { if (MIXED) inner_end = true; else st = ST_NONFINITE; go = false; }
      else if (ss <= ilim2) half = true;
      else if (!finite((double)tt) || !finite((double)ts)) {
        if (MIXED) inner_end = true; else st = ST_NONFINITE;
        go = false;
      }
    }
    const double sal = scale * (double)al;
    if (half) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        P.x[i] = fma(sal, (double)ph[i], P.x[i]);
        r[i] = s[i];
      }
      rtrue = false;
      rr_in = ss;
      go = false;
    }
    const T om = (tt == (T)0) ? (T)0 : ts / tt;
    if (go) {
      const double som = scale * (double)om;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        P.x[i] = fma(som, (double)sh[i], fma(sal, (double)ph[i], P.x[i]));
        r[i] = s[i] - om * t[i];
      }
      rtrue = false;
      rho0 = rho;
      alpha = al;
      omega = om;
    }
    T q4[2];
    {
      T p0[R], p1[R];
#pragma unroll
      for (int i = 0; i < R; ++i) { p0[i] = r[i] * r[i]; p1[i] = rh[i] * r[i]; }
      q4[0] = sum_rows(p0);
      q4[1] = sum_rows(p1);
    }
    tm.sum(q4);
    if (go) {
      rr_in = q4[0];
      rho = q4[1];
      if (om == (T)0 && !(rr_in <= ilim2)) {
        if (MIXED) inner_end = true; else st = ST_BREAKDOWN;
      }
    }
  }
  finish(tm, A, g, P.b, P.x, st, k, outer, bn, rn, st == ST_CONVERGED || st == ST_IDLE);
}

// =================================================================== Trsv
// BatchTrsv (Tab. 2): T x = b for T the lower (upper) triangle of A, diagonal
// included, one-wave teams (row i on lane i, n <= 64).  The row's register
// values outside the triangle are zeroed, so the shared epilogue's true
// residual is that of T; the triangle goes to the LDS region as for ILU(0)
// and one column sweep solves it: x_k = acc_k / t_kk (final on lane k when
// column k is reached) is read out, and every later row subtracts t_ik x_k.
// A zero diagonal entry is a breakdown (x = 0); iterations: 0.
template <bool LOWER, class TM, class RW>
__device__ __forceinline__ void trsv_system_w64(TM& tm, RW& A, const KArgs& g) {
  static_assert(RW::R == 1 && RW::TEAM == kWave, "one-wave BatchTrsv");
  const int n = g.n, st = ilu_stride(n), n8 = st - 1;
  double* F = tm.bj_region(g);
  const int lane = tm.lane;
  const bool ok = A.ok[0];
  const int i = ok ? A.row[0] : 0;
  for (int e = lane; e < n * st; e += kWave) F[e] = 0.0;
  if (ok) lds_store<double>(A.vrow[0] + RW::kBuf, (double)i);
  tm.sync();
#pragma unroll
  for (int k0 = 0; k0 < RW::NZ; k0 += 4) {
    int col[4];
#pragma unroll
    for (int k = k0; k < k0 + 4 && k < RW::NZ; ++k)
      col[k - k0] = (int)lds_load<double>(A.c[0][k] + RW::kBuf);
#pragma unroll
    for (int k = k0; k < k0 + 4 && k < RW::NZ; ++k) {
      const bool keep = ok && A.real(0, k) && (LOWER ? col[k - k0] <= i : col[k - k0] >= i);
      if (keep) F[i * st + col[k - k0]] = A.a[0][k];
      A.a[0][k] = keep ? A.a[0][k] : 0.0;
    }
    __asm__ volatile("" ::: "memory");
  }
  wave_lds_fence();
  double b[1] = {A.bval[0]}, x[1] = {A.xval[0]}, q[1] = {b[0] * b[0]};
  tm.sum(q);
  const double bn = sqrt(q[0]);
  const double tii = ok ? F[i * st + i] : 1.0;
  int stt = tm.live ? ST_CONVERGED : ST_IDLE;
  if (tm.live && !finite(bn)) {
    stt = ST_NONFINITE;
  } else if (bn == 0.0 || wave_any(tm.live && tii == 0.0)) {
    if (tm.live && bn != 0.0) stt = ST_BREAKDOWN;
    x[0] = 0.0;
  } else {
    const double dv = ok ? 1.0 / tii : 0.0;
    const int ilo = ok ? i : kWave, ihi = ok ? i : -1;  // idle lanes take no term
    double acc = ok ? b[0] : 0.0;
    if constexpr (LOWER) {
      for (int k0 = 0; k0 < n8; k0 += 8) {
        double t[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) t[p] = F[i * st + k0 + p];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const double xk = rdlane(acc * dv, k0 + p);
          acc = fma(ilo > k0 + p && ilo < kWave ? -t[p] : 0.0, xk, acc);
        }
      }
    } else {
      for (int j0 = n8 - 8; j0 >= 0; j0 -= 8) {
        double t[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) t[p] = F[i * st + j0 + 7 - p];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const double xj = rdlane(acc * dv, j0 + 7 - p);
          acc = fma(ihi < j0 + 7 - p && ihi >= 0 ? -t[p] : 0.0, xj, acc);
        }
      }
    }
    x[0] = ok ? acc * dv : 0.0;
    if (tm.live && wave_any(ok && !finite(x[0]))) stt = ST_NONFINITE;
  }
  wave_lds_fence();
  finish(tm, A, g, b, x, stt, 0, 0, bn, 0.0, false);
}

// BatchTrsv for multi-wave teams (row i on lane i, up to 1024 rows): the
// row-oriented substitution of the oracle on the team's first wave, level by
// level (the sweep of the ILU(0) form with the triangle's own diagonal):
// x_i = (b_i - sum_j t_ij x_j) / t_ii over the row's strictly lower (upper)
// entries in increasing column.  Entries outside the triangle are zeroed in
// registers as in the one-wave form, so the epilogue's residual is that of
// the triangle; a zero diagonal entry anywhere is a breakdown.
template <bool LOWER, class TM, class RW>
__device__ __forceinline__ void trsv_system_mw(TM& tm, RW& A, const KArgs& g) {
  static_assert(RW::R == 1 && RW::TEAM > kWave, "multi-wave BatchTrsv: one row per lane");
  constexpr int NZ = RW::NZ;
  const IluMw L = ilu_mw_layout(g.n, g.nnz);
  const unsigned reg = lds_addr(tm.bj_region(g));
  sweep_lists_load(tm, g, reg, L);
  const bool ok = A.ok[0];
  int i = ok ? A.row[0] : 0;
  __asm__ volatile("" : "+v"(i));  // per system: keeps the row's addresses out of the kernel-wide registers
  const unsigned fr = reg + L.f + (unsigned)(g.fmt == 0 ? A.w[0] : g.row_ptr[i]) * 8;
  const unsigned me = reg + L.y + (unsigned)i * 8;
  const double tii = ok ? A.dval[0] : 1.0;
  if (ok) {
#pragma unroll
    for (int s = 0; s < NZ; ++s)
      if (A.real(0, s)) lds_store<double>(fr + s * 8, A.a[0][s]);
    lds_store<double>(reg + L.d + (unsigned)i * 8, tii);
    lds_store<double>(me, A.bval[0]);
  }
#pragma unroll
  for (int s = 0; s < NZ; ++s) {
    const bool keep = ok && A.real(0, s) && (LOWER ? A.c[0][s] <= A.vrow[0] : A.c[0][s] >= A.vrow[0]);
    A.a[0][s] = keep ? A.a[0][s] : 0.0;
  }
  double b[1] = {A.bval[0]}, x[1] = {A.xval[0]}, q[1] = {b[0] * b[0]};
  tm.sum(q);  // also makes the stores above visible to the team
  const double bn = sqrt(q[0]);
  const bool zero_diag = __syncthreads_or(ok && tii == 0.0) != 0;
  int stt = tm.live ? ST_CONVERGED : ST_IDLE;
  if (tm.live && !finite(bn)) {
    stt = ST_NONFINITE;
  } else if (bn == 0.0 || zero_diag) {
    if (tm.live && bn != 0.0) stt = ST_BREAKDOWN;
    x[0] = 0.0;
  } else {
    if (threadIdx.x < kWave) tri_sweep<LOWER, true>(g, reg, L);
    tm.sync();
    x[0] = ok ? lds_load<double>(me) : 0.0;
    const bool nf = __syncthreads_or(ok && !finite(x[0])) != 0;
    if (tm.live && nf) stt = ST_NONFINITE;
  }
  finish(tm, A, g, b, x, stt, 0, 0, bn, 0.0, false);
}

template <bool LOWER, class TM, class RW>
__device__ __forceinline__ void trsv_system(TM& tm, RW& A, const KArgs& g) {
  if constexpr (RW::TEAM > kWave) trsv_system_mw<LOWER>(tm, A, g);
  else trsv_system_w64<LOWER>(tm, A, g);
}

// =================================================================== CG
// Preconditioned CG, Sec. 3.5 Alg. 1 step for step, with the relative-residual
// stop test.  Per iteration: one SpMV and two reductions (p.t; r.z, r.r).
template <int PK, class TM, class RW>
__device__ __forceinline__ void cg_system(TM& tm, RW& A, const KArgs& g) {
  Prologue<RW::R> P;
  prologue<PK>(tm, A, g, P);
  constexpr int R = RW::R;
  double z[R], p[R];
  precond<PK>(tm, A, g, P.d, P.r, z);
#pragma unroll
  for (int i = 0; i < R; ++i) p[i] = z[i];
  double q3[3];
  {
    double p0[R], p1[R], p2[R];
#pragma unroll
    for (int i = 0; i < R; ++i) { p0[i] = P.b[i] * P.b[i]; p1[i] = P.r[i] * P.r[i]; p2[i] = P.r[i] * z[i]; }
    q3[0] = sum_rows(p0); q3[1] = sum_rows(p1); q3[2] = sum_rows(p2);
  }
  tm.sum(q3);
  const double bn = sqrt(q3[0]);
  double rn = sqrt(q3[1]), rho = q3[2];
  double rsq = q3[1];  // squared recurrence residual (the loop compares squares)
  const double lim = stop_limit(g, bn), lim2 = lim * lim;
  int st = tm.live ? ST_RUNNING : ST_IDLE;
  if (st == ST_RUNNING) {
    if (!finite(bn)) st = ST_NONFINITE;
    else if (bn == 0.0) {
      st = ST_CONVERGED;
#pragma unroll
      for (int i = 0; i < R; ++i) P.x[i] = 0.0;
      rn = 0.0;
    }
  }
  bool rtrue = true;
  int k = 0;
  for (;;) {
    bool need_chk = false;
    if (st == ST_RUNNING) {
      if (!finite(rsq) || !finite(rho)) st = ST_NONFINITE;
      else if (rsq <= lim2) { if (rtrue) st = ST_CONVERGED; else need_chk = true; }
      else if (k >= g.max_iter) st = ST_MAX_ITER;
    }
    if (tm.any(need_chk)) {
      double t[R], rc[R], zc[R], p0[R], p1[R], q[2];
      A.template spmv<0>(tm, A.a, P.x, t);
#pragma unroll
      for (int i = 0; i < R; ++i) rc[i] = P.b[i] - t[i];
      precond<PK>(tm, A, g, P.d, rc, zc);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        p0[i] = rc[i] * rc[i];
        p1[i] = rc[i] * zc[i];
      }
      q[0] = sum_rows(p0); q[1] = sum_rows(p1);
      tm.sum(q);
      if (need_chk) {
        rn = sqrt(q[0]);
        rsq = q[0];
        rtrue = true;
        if (!finite(rn)) st = ST_NONFINITE;
        else if (rn <= lim) st = ST_CONVERGED;
        else if (k >= g.max_iter) st = ST_MAX_ITER;
        else {
#pragma unroll
          for (int i = 0; i < R; ++i) { P.r[i] = rc[i]; z[i] = zc[i]; p[i] = zc[i]; }
          rho = q[1];
        }
      }
      continue;
    }
    if (!tm.any(st == ST_RUNNING)) break;
    bool go = st == ST_RUNNING;
    if (go && rho == 0.0) { st = ST_BREAKDOWN; go = false; }
    double t[R];
    A.template spmv<0>(tm, A.a, p, t);
    double q1[1];
    {
      double pr[R];
#pragma unroll
      for (int i = 0; i < R; ++i) pr[i] = p[i] * t[i];
      q1[0] = sum_rows(pr);
    }
    tm.sum(q1);
    const double pt = q1[0];
    if (go) {
      if (!finite(pt)) { st = ST_NONFINITE; go = false; }
      else if (pt == 0.0) { st = ST_BREAKDOWN; go = false; }
    }
    const double alpha = rho / pt;
    double rr[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      rr[i] = go ? fma(-alpha, t[i], P.r[i]) : P.r[i];
      if (go) P.x[i] = fma(alpha, p[i], P.x[i]);
    }
    precond<PK>(tm, A, g, P.d, rr, z);
    double q2[2];
    {
      double p0[R], p1[R];
#pragma unroll
      for (int i = 0; i < R; ++i) { p0[i] = rr[i] * z[i]; p1[i] = rr[i] * rr[i]; }
      q2[0] = sum_rows(p0); q2[1] = sum_rows(p1);
    }
    tm.sum(q2);
    if (go) {
      const double beta = q2[0] / rho;
#pragma unroll
      for (int i = 0; i < R; ++i) { P.r[i] = rr[i]; p[i] = fma(beta, p[i], z[i]); }
      rho = q2[0];
      rsq = q2[1];
      rtrue = false;
      k += 1;
    }
  }
  finish(tm, A, g, P.b, P.x, st, k, 0, bn, rn, st == ST_CONVERGED || st == ST_IDLE);
}

// =================================================================== GMRES(m)
// Right-preconditioned restarted GMRES with Gram-Schmidt Arnoldi and Givens
// rotations (Saad 2003, Alg. 6.9 with right preconditioning): modified
// Gram-Schmidt for teams narrower than a wave, block modified Gram-Schmidt
// (blocks of four, classical inside a block) for teams of a wave or more, whose
// reductions then fuse four dots at a time.  The m+1
// basis vectors stay on chip (one element per row per lane, in registers, or
// partly in LDS for 1024-lane teams), so a cycle never touches HBM.  The Hessenberg column, the rotated triangle R, the
// rotations, g and y are per-team LDS scalars written once per cycle: every lane
// of the team computes the same bits and writes them, and reads only entries it
// has written itself, so no barrier is needed around them.  The last entry of g
// changes at every step and is kept in a register.  At the end of a cycle
// y = R^{-1} g by back substitution and x += M V y.
//
// MIXED: every cycle is an iterative-refinement step.  The cycle start forms
// the FP64 true residual r = b - A x (as the plain method does at a restart);
// the cycle's Arnoldi steps run in FP32 (basis, SpMV with an FP32 copy of A,
// dots and norms), ending when |g| <= max(inner_tol * beta, tol ||b|| / 2) or
// after m steps; the rotations and the triangular solve stay FP64 and x is
// updated in FP64.  A cycle that does not lower the FP64 residual ends the
// solve with BREAKDOWN.
// Where a team keeps the GMRES scalars (Hessenberg column, packed R, the
// rotations, g, y) and its LDS basis vectors: behind the fixed-size team's
// vector buffers.  Teams of other kernels provide their own overloads.
template <class S>
__device__ __forceinline__ double* gmres_scalar_base(const Team<S>& tm, int rows) {
  return reinterpret_cast<double*>(tm.lds + kVecBuffers * vec_buf_bytes(rows));
}
template <class S>
__device__ __forceinline__ unsigned gmres_basis_base(const Team<S>& tm, int rows) {
  return lds_addr(tm.lds) + gmres_basis_offset(rows);
}

template <bool MIXED, int PK, class TM, class RW>
__device__ __forceinline__ void gmres_system(TM& tm, RW& A, const KArgs& g) {
  static_assert(RW::R == 1, "GMRES keeps one row per lane");
  using T = typename std::conditional<MIXED, float, double>::type;
  constexpr int M = kMaxRestart;
  Prologue<RW::R> P;
  prologue<PK>(tm, A, g, P);
  const int m = g.restart;
  // LDS scalars of this team
  double* hcol = gmres_scalar_base(tm, RW::ROWS);
  double* Rt = hcol + (M + 2);               // packed by columns: R[i][j] at j(j+1)/2 + i
  double* cs = Rt + M * (M + 1) / 2;
  double* sn = cs + M;
  double* gv = sn + M;
  double* yv = gv + (M + 1);

  // the arithmetic copy of the rows (FP32 for MIXED; slots without an entry
  // zeroed so that no value beyond FP32 range meets the zero cell)
  T a_in[1][RW::NZ];
#pragma unroll
  for (int k = 0; k < RW::NZ; ++k) {
    if constexpr (MIXED) a_in[0][k] = A.real(0, k) ? (T)A.a[0][k] : (T)0;
    else a_in[0][k] = A.a[0][k];
  }

  double q1[1];
  {
    double pr[1] = {P.b[0] * P.b[0]};
    q1[0] = pr[0];
  }
  tm.sum(q1);
  const double bn = sqrt(q1[0]);
  const double lim = stop_limit(g, bn);
  int st = tm.live ? ST_RUNNING : ST_IDLE;
  double rn = 0.0;
  if (st == ST_RUNNING) {
    if (!finite(bn)) st = ST_NONFINITE;
    else if (bn == 0.0) { st = ST_CONVERGED; P.x[0] = 0.0; }
  }
  // Basis vectors 0..NL-1 live in LDS (this lane's element of vector i at
  // vb + i * ROWS * sizeof(T)), vectors NL..M in registers V[i - NL].
  constexpr int NL = gmres_lds_vectors(RW::WG, MIXED);
  constexpr int NV = M + 1 - NL;
  T V[NV > 0 ? NV : 1];
  const unsigned vb = gmres_basis_base(tm, RW::ROWS) + (unsigned)tm.lane * sizeof(T);
  constexpr unsigned vstride = RW::ROWS * sizeof(T);
#pragma unroll
  for (int i = 0; i < NV; ++i) V[i] = (T)0;
#pragma unroll
  for (int i = 0; i < NL; ++i) lds_store<T>(vb + i * vstride, (T)0);
  // basis element i of this lane (i is a compile-time index after unrolling)
  auto basis = [&](int i) -> T {
    return i < NL ? lds_load<T>(vb + i * vstride) : V[i >= NL ? i - NL : 0];
  };

  int k = 0, j = 0, cycles = 0;
  T vcur = (T)0;       // the basis vector the next Arnoldi step multiplies
  double gcur = 0.0;   // g_j, the entry the next rotation acts on
  double ilim = lim;   // the cycle's stopping level for |g|
  double beta_prev = INFINITY;
  bool start = true;   // at a cycle start (true residual due)
  const double d = P.d[0];
  const T dT = (T)d;
  for (;;) {
    // ---- cycle start: true residual, convergence, V0 = r/beta
    if (tm.any(st == ST_RUNNING && start)) {
      const bool me = st == ST_RUNNING && start;
      double t[1];
      A.template spmv<0, false>(tm, A.a, P.x, t);
      const double rc = P.b[0] - t[0];
      double q[1] = {rc * rc};
      tm.sum(q);
      if (me) {
        const double beta = sqrt(q[0]);
        rn = beta;
        if (!finite(beta)) st = ST_NONFINITE;
        else if (beta <= lim) st = ST_CONVERGED;
        else if (k >= g.max_iter) st = ST_MAX_ITER;
        else if (MIXED && !(beta < beta_prev)) st = ST_BREAKDOWN;
        else {
          vcur = (T)(rc / beta);
          if constexpr (NL > 0) lds_store<T>(vb, vcur);
          else V[0] = vcur;
          gcur = beta;
          if constexpr (MIXED) ilim = fmax(g.inner_tol * beta, 0.5 * lim);
          beta_prev = beta;
          cycles += 1;
          j = 0;
          start = false;
        }
      }
    }
    if (!tm.any(st == ST_RUNNING)) break;
    // ---- one Arnoldi step for every running team (all of them are mid-cycle)
    const bool act = st == ST_RUNNING;
    T z[1], w[1];
    {
      const T vv[1] = {vcur}, dd[1] = {dT};
      precond<PK>(tm, A, g, dd, vv, z);
    }
    A.template spmv<0, false>(tm, a_in, z, w);
    const int jmax = wave_max(act ? j : -1);
    if constexpr (RW::TEAM >= 64) {
      // Block Gram-Schmidt: blocks of four basis vectors taken in order, as
      // modified Gram-Schmidt takes single vectors; within a block the four
      // dots use the same w (classical Gram-Schmidt) and share one fused
      // reduction, then w -= V_block q.
#pragma unroll
      for (int g = 0; g < M; g += 4) {
        if (g <= jmax) {
          T vq[4], q[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            vq[t] = (g + t < M && g + t <= j) ? basis(g + t) : (T)0;
            q[t] = w[0] * vq[t];
          }
          tm.sum(q);
          if (act) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              if (g + t < M && g + t <= j) {
                w[0] = fma(-q[t], vq[t], w[0]);
                hcol[g + t] = (double)q[t];
              }
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        if (i <= jmax) {
          const T vi = basis(i);
          T q[1] = {w[0] * vi};
          tm.sum(q);
          if (act && i <= j) {
            w[0] = fma(-q[0], vi, w[0]);
            hcol[i] = (double)q[0];
          }
        }
      }
    }
    T qn[1] = {w[0] * w[0]};
    tm.sum(qn);
    bool end = false;
    if (act) {
      const double hn = sqrt((double)qn[0]);
      k += 1;
      if (!finite(hn)) {
        st = ST_NONFINITE;
      } else {
        // apply the previous rotations to column j
        double hp;
        const int cj = j * (j + 1) / 2;
        if constexpr (RW::TEAM >= 64) {
          // column j and the rotations are loaded one entry per lane (every
          // wave holds a copy): the chain reads them with readlane, not LDS loads
          const int ju = __builtin_amdgcn_readfirstlane(j);
          const int l = (int)lane_id();
          const double hreg = l <= ju ? hcol[l] : 0.0;
          const double creg = l < ju ? cs[l] : 0.0, sreg = l < ju ? sn[l] : 0.0;
          hp = rdlane(hreg, 0);
          for (int i = 0; i < ju; ++i) {
            const double hnx = rdlane(hreg, i + 1), c = rdlane(creg, i), s = rdlane(sreg, i);
            Rt[cj + i] = c * hp + s * hnx;
            hp = -s * hp + c * hnx;
          }
        } else {
          hp = hcol[0];
          for (int i = 0; i < j; ++i) {
            const double hnx = hcol[i + 1];
            const double c = cs[i], s = sn[i];
            Rt[cj + i] = c * hp + s * hnx;
            hp = -s * hp + c * hnx;
          }
        }
        const double dd = sqrt(hp * hp + hn * hn);
        if (dd == 0.0) {
          st = ST_BREAKDOWN;
        } else {
          const double c = hp / dd, s = hn / dd;
          cs[j] = c;
          sn[j] = s;
          Rt[cj + j] = dd;
          gv[j] = c * gcur;
          gcur = -s * gcur;
          end = fabs(gcur) <= ilim || hn == 0.0 || k >= g.max_iter || j == m - 1;
          if (!end) {
            const T vn = (T)((double)w[0] / hn);
            vcur = vn;
            if constexpr (NL > 0) {
              if (j + 1 < NL) lds_store<T>(vb + (unsigned)(j + 1) * vstride, vn);
            }
            // teams of a wave or more: j is the same in every lane
            const int jn = RW::TEAM >= 64 ? __builtin_amdgcn_readfirstlane(j + 1) : j + 1;
#pragma unroll
            for (int i = (NL > 1 ? NL : 1); i <= M; ++i)
              if (jn == i) V[i - NL] = vn;
            j += 1;
          }
        }
      }
    }
    // ---- cycle end: y = R^{-1} g (back substitution), x += M V y
    if (tm.any(end)) {
      const int jend = wave_max(end ? j : -1);
      double zacc = 0.0;
      if constexpr (RW::TEAM >= 64) {
        // column by column: lane l keeps g_l minus the known terms of row l;
        // y_i = (that of lane i) / R_ii, then the rows above drop R_li y_i
        if (end) {
          const int je = __builtin_amdgcn_readfirstlane(j);
          const int l = (int)lane_id();
          double acc = l <= je ? gv[l] : 0.0;
#pragma unroll
          for (int i = M - 1; i >= 0; --i) {
            if (i <= je) {
              const double yi = rdlane(acc, i) / Rt[i * (i + 1) / 2 + i];
              if (l < i) acc = fma(-Rt[i * (i + 1) / 2 + l], yi, acc);
              zacc = fma(yi, (double)basis(i), zacc);
            }
          }
        }
      } else {
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
          if (i <= jend) {
            if (end && i <= j) {
              double acc = gv[i];
              for (int l = i + 1; l <= j; ++l) acc = fma(-Rt[l * (l + 1) / 2 + i], yv[l], acc);
              const double yi = acc / Rt[i * (i + 1) / 2 + i];
              yv[i] = yi;
              zacc = fma(yi, (double)basis(i), zacc);
            }
          }
        }
      }
      // x += M V y (every lane of the wave applies M together)
      double mz[1];
      {
        const double zz[1] = {zacc}, dd[1] = {d};
        precond<PK>(tm, A, g, dd, zz, mz);
      }
      if (end) {
        if constexpr (PK != kPkScalar) P.x[0] = P.x[0] + mz[0];
        else P.x[0] = fma(d, zacc, P.x[0]);
        start = true;
      }
    }
  }
  finish(tm, A, g, P.b, P.x, st, k, MIXED ? cycles : 0, bn, rn,
         st == ST_CONVERGED || st == ST_IDLE || (st == ST_MAX_ITER && start) ||
             (MIXED && st == ST_BREAKDOWN && start));
}

// =================================================================== kernels
// Each workgroup loads the shared pattern into registers once and then walks
// over the batch: in every round the G workgroups take G consecutive slots of
// T systems (T teams each), workgroup b the slot xcd_slot(b) of the round,
// team t the system slot * T + t.  Single-wave groups prefetch the next
// round's systems into LDS while the current round is solved: wait for the
// prefetch, copy the block into registers, wait for those LDS reads, start the
// next prefetch, solve.
// Vector memory operations retire in issue order.  After the first round the
// last ones a wave issued are the previous system's four output stores (x,
// iters, resid, status), all after this round's prefetch: waiting until at most
// four are outstanding (and for LDS) means the prefetch has landed, without
// waiting for the stores to be acknowledged.  s_waitcnt vmcnt(4) expcnt(7)
// lgkmcnt(0).
constexpr int kWaitPrefetch = 0x0074;
// Multi-wave teams wait for all of their vector memory operations (their
// waves issue different numbers of output stores after the prefetch):
// s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15).
constexpr int kWaitAllVm = 0x0F70;

// Workgroups are placed on the 8 XCDs round-robin (workgroup b on XCD b mod 8),
// and each XCD has its own L2.  Slot of workgroup b in a round of the grid:
// XCD x takes the contiguous slots x*G/8 .. (x+1)*G/8-1, so
// neighbouring systems (whose values, right-hand sides and outputs share cache
// lines at their edges) are handled inside one XCD and their partial lines
// merge in one L2.  Identity when G is not a multiple of 8.
__device__ __forceinline__ unsigned xcd_slot(unsigned b, unsigned G) {
  return (G & 7u) ? b : (b & 7u) * (G >> 3) + (b >> 3);
}

// The loop body reads the arguments through ga, at an address offset by a
// zero the compiler cannot see through: otherwise it hoists every argument
// load out of the loop and keeps them all in scalar registers through the
// solve, where they spill into vector-register lanes.
#define BS_PERSISTENT_LOOP(MX, CALL)                                                \
  extern __shared__ __align__(16) char smem[];                                     \
  Team<S> tm(smem, g);                                                             \
  Rows<S, MX> A;                                                                   \
  A.load_pattern(tm, g);                                                           \
  const int64_t stride = (int64_t)gridDim.x * S::TEAMS;                            \
  const int64_t slot0 = (int64_t)xcd_slot(blockIdx.x, gridDim.x) * S::TEAMS;      \
  bool staged = false;                                                             \
  if constexpr (S::WAVES == 1) {                                                   \
    staged = g.stage != 0;                                                         \
    if (staged) A.prefetch(tm, g, slot0);                                          \
  } else if constexpr (S::NZ >= kStageMinSlots) {                                  \
    staged = g.stage == 2;                                                         \
    if (staged && slot0 < g.n_batch) A.prefetch_group(tm, g, slot0);               \
  }                                                                                \
  bool first_round = true;                                                         \
  for (int64_t base = slot0; base < g.n_batch; base += stride) {                   \
    int opaque_zero;                                                               \
    __asm__ volatile("s_mov_b32 %0, 0" : "=s"(opaque_zero));                       \
    const KArgs& ga = (&g)[opaque_zero];                                           \
    tm.sys = base + tm.tix;                                                        \
    tm.live = tm.sys < ga.n_batch;                                                 \
    tm.row0 = tm.live ? tm.sys * ga.n : 0;                                         \
    if constexpr (S::WAVES == 1) {                                                 \
      if (staged) { /* the prefetch of this round has landed */                    \
        if (first_round) __builtin_amdgcn_s_waitcnt(0);                            \
        else __builtin_amdgcn_s_waitcnt(kWaitPrefetch);                            \
        first_round = false;                                                       \
        __asm__ volatile("" ::: "memory");                                         \
      }                                                                            \
    } else {                                                                       \
      if (staged) { /* every wave's part of the prefetch has landed */             \
        __builtin_amdgcn_s_waitcnt(kWaitAllVm);                                    \
        __asm__ volatile("" ::: "memory");                                         \
        __syncthreads();                                                           \
      }                                                                            \
    }                                                                              \
    A.load_values(tm, ga);                                                         \
    if constexpr (S::WAVES == 1) {                                                 \
      if (staged && base + stride < ga.n_batch) {                                  \
        __builtin_amdgcn_s_waitcnt(0xC07F); /* staging reads done (lgkmcnt 0) */   \
        __asm__ volatile("" ::: "memory");                                         \
        A.prefetch(tm, ga, base + stride);                                         \
      }                                                                            \
    } else if constexpr (S::NZ >= kStageMinSlots) {                                \
      if (staged && base + stride < ga.n_batch) {                                  \
        __syncthreads(); /* every wave has read its rows from the block */         \
        A.prefetch_group(tm, ga, base + stride);                                   \
      }                                                                            \
    }                                                                              \
    CALL;                                                                          \
  }

// Mixed kernels keep their FP32 vectors at a 4-byte LDS stride when a team
// holds more rows than a wave: the gathers of the large systems then meet
// fewer bank conflicts (the 992-row stencil solves 8% faster), while the
// one-wave systems (54 rows) lose more to the extra address arithmetic of the
// FP64 residual SpMVs than they gain.
template <class S, bool MIXED>
constexpr bool kLds32 = MIXED && (S::ROWS > kWave);

// ILU(0) on one-wave teams: the dense factors (about 25 KB of LDS per wave
// for 54 rows) leave room for fewer than two waves per SIMD, so the register
// budget is that of two (no spills) rather than three.
template <class S, bool MIXED, int PK = kPkScalar>
__global__ __launch_bounds__(S::WG) __attribute__((amdgpu_waves_per_eu((MIXED || PK == kPkIlu) ? S::OCC_MIXED : S::OCC))) void k_bicgstab(const KArgs g) {
  BS_PERSISTENT_LOOP((kLds32<S, MIXED>), (bicgstab_system<MIXED, PK>(tm, A, ga)))
}

template <class S, bool LOWER>
__global__ __launch_bounds__(S::WG) __attribute__((amdgpu_waves_per_eu(S::OCC))) void k_trsv(const KArgs g) {
  BS_PERSISTENT_LOOP(false, (trsv_system<LOWER>(tm, A, ga)))
}

template <class S, int PK = kPkScalar>
__global__ __launch_bounds__(S::WG) __attribute__((amdgpu_waves_per_eu(S::OCC))) void k_cg(const KArgs g) {
  BS_PERSISTENT_LOOP(false, (cg_system<PK>(tm, A, ga)))
}

// GMRES keeps its basis in registers beside the row: held to three waves per
// SIMD, the one-wave shapes of 24..32 slots spill (60..148 bytes per lane),
// and their LDS (staging plus the Hessenberg scalars, about 16 KB per wave)
// leaves room for only 2.5 anyway, so they are held to two, as the mixed ones.
template <class S, bool MIXED, int PK = kPkScalar>
__global__ __launch_bounds__(S::WG) __attribute__((amdgpu_waves_per_eu(S::OCC_MIXED))) void k_gmres(const KArgs g) {
  BS_PERSISTENT_LOOP((kLds32<S, MIXED>), (gmres_system<MIXED, PK>(tm, A, ga)))
}

#undef BS_PERSISTENT_LOOP

}  // namespace bs
