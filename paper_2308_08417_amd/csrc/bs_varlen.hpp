// Uneven batches in one persistent launch: systems of different sizes (and
// patterns) share one kernel.  A workgroup of WG lanes takes tasks from an
// atomic queue; a task is up to WG/T systems of one size class, each solved by
// a team of T lanes (T a power of two in [64, WG]) that owns R rows per lane,
// rows lane, lane+T, .., lane+(R-1)T.  The largest system has WG*R rows.
//
// Teams of one wave need no workgroup barrier: when a task's teams are single
// waves, each advances on its own (wave-level fences, ballots and DPP sums)
// and the waves meet only at the next task.  Teams of several waves share the
// workgroup's barriers, so the teams of such a task advance in lockstep: any()
// is then a workgroup-wide OR and a finished team idles until the task ends.
// The solver bodies are the ones of the fixed-size kernels.
#pragma once
#include "bs_solvers.hpp"

namespace bs {

template <int WG_, int R_>
struct VarShape {
  static constexpr int WG = WG_, R = R_;
  static constexpr int WAVES = WG / kWave;
  static constexpr int MAXT = WG / kWave;  // teams per task at most (T >= 64)
  static constexpr int ROWS = WG * R;      // largest system
  // waves per SIMD that one group places (the register budget per lane);
  // asking the narrow shapes for more spills their rows to scratch
  static constexpr int OCC = WG / 256;
};

struct VTask {
  int team;   // lanes per system
  int first;  // index of the first system in the queue order
  int count;  // systems in this task (<= WG / team)
  int pad;
};

// Where a kernel finds a row's columns and the positions of its values in the
// system's value block (the source, SRC):
//   kSrcCsr      the CSR arrays themselves: row_ptr, columns, values in CSR
//                order (position = row start + k);
//   kSrcRowIdx   a row-ordered index of {column, position} pairs at the CSR
//                offsets of the pattern (the CSR walk of values in any layout);
//   kSrcSlotIdx  a slot-major index [width][rows] of {column, position} pairs,
//                column -1 for padding (the ELL walk: lanes of a team read
//                consecutive entries of one slot).
//   kSrcShared   one pattern shared by the whole batch (the fixed-size batched
//                solve, streamed kernels only): the pattern's slot-major columns
//                (-1 padding), row lengths, row starts and diagonal slots;
//                position row start + k (CSR values) or k*n + row (ELL values).
// The indexes are built on the host from validated patterns.
enum : int { kSrcCsr = 0, kSrcRowIdx = 1, kSrcSlotIdx = 2, kSrcShared = 3 };

// The batch is described by the pattern arrays (validated on the host before
// any launch): the kernel reads each row's start and length from its pattern's
// row_ptr (or a slot of the slot-major index), its columns and value
// positions, and finds the diagonal among them while loading.
struct VArgs {
  KArgs base;             // solver settings and the per-system outputs
  int64_t n_tasks;
  const VTask* tasks;
  const int* order;       // system ids in queue order
  const int* sys_rows;    // [B]
  const int* sys_pat;     // [B] pattern of each system
  const int64_t* row_off; // [B+1] first row of each system in b and x
  const int64_t* val_off; // [B+1] first value of each system (CSR order)
  const int64_t* pat_rp;  // [P] offset of the pattern's row_ptr in rowptr_all
  const int64_t* pat_col; // [P] offset of the pattern's columns in col_all
  const int* rowptr_all;  // concatenated row_ptr arrays (each starting at 0)
  const int* col_all;     // concatenated column arrays, CSR order
  const int2* idx_row;    // kSrcRowIdx: row-ordered index, pattern p at pat_col[p]
  const int2* idx_slot;   // kSrcSlotIdx: slot-major index, pattern p at pat_slot[p]
  const int64_t* pat_slot;
  const int* pat_w;       // [P] slots of each pattern's slot-major index
  int* counter;           // task counter, zero at launch
};

// Vector buffers: team t's rows at elements [t*T*R, (t+1)*T*R), then one zero
// cell per team after the ROWS elements, so the stride is a constant.
template <class VS>
constexpr unsigned var_buf_bytes() { return round16((unsigned)(VS::ROWS + VS::MAXT) * 8); }

template <class VS>
constexpr int var_lds_bytes() {
  return 2 * (int)var_buf_bytes<VS>() + 2 * kMaxFused * VS::WAVES * 8;
}

// Team of runtime size T (uniform across the workgroup for a task).
template <class VS>
struct VarTeam {
  int T;               // lanes per team
  int lane, tix;       // lane within the team, team within the workgroup
  int wpt;             // waves per team
  int lgw;             // log2(wpt)
  int64_t sys, row0;
  bool live;
  char* lds;
  double* red;         // cross-wave reduction slots
  int phase;

  __device__ void set_team(int t, char* smem) {
    T = t;
    lane = threadIdx.x & (t - 1);
    tix = threadIdx.x / t;
    wpt = t / kWave;
    lgw = __builtin_ctz((unsigned)wpt);
    lds = smem;
    red = reinterpret_cast<double*>(smem + 2 * var_buf_bytes<VS>());
  }

  // Single-wave teams: a wave's LDS operations complete in issue order, so a
  // wavefront-scope fence (for the compiler) is enough.
  __device__ __forceinline__ void sync() {
    if (wpt == 1) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
    } else {
      __syncthreads();
    }
  }

  // This team's block-Jacobi region (after the buffers and reduction slots)
  // and its row count.
  __device__ __forceinline__ double* bj_region(const KArgs& g) const {
    return reinterpret_cast<double*>(lds + var_lds_bytes<VS>()) + (size_t)tix * T * VS::R * (g.block + 1);
  }
  __device__ __forceinline__ int bj_rows() const { return T * VS::R; }

  __device__ __forceinline__ bool any(bool p) const {
    if (wpt == 1) return wave_any(p);
    return __syncthreads_or(p ? 1 : 0) != 0;
  }

  template <class V, int K>
  __device__ __forceinline__ void sum(V (&v)[K]) {
    static_assert(K <= kMaxFused && K * 16 <= 64, "too many fused values");
    wave_sums(v);
    if (wpt > 1) {
      double* buf = red + phase * (kMaxFused * VS::WAVES);
      const int w = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) buf[k * VS::WAVES + w] = (double)v[k];
      }
      __syncthreads();
      // lane l reads value l / wpt of its team's wave (l mod wpt); a butterfly
      // over aligned groups of wpt lanes leaves value k's team total in lanes
      // k*wpt .. k*wpt+wpt-1 (wpt is a power of two from 2 to 16, uniform over
      // the workgroup, and K * wpt <= 64)
      const int l = threadIdx.x & 63;
      const int vi = (l >> lgw) < K ? (l >> lgw) : 0;
      const double t = group_sum(buf[vi * VS::WAVES + tix * wpt + (l & (wpt - 1))], wpt);
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = (V)rdlane(t, k * wpt);
      phase ^= 1;
    }
  }
};

// The R rows a lane owns, their values and LDS gather addresses in registers.
// MX (the mixed-precision kernels): every team keeps a block of its own in
// each buffer, team t's T*R elements from element t*(T*R+1) with its zero cell
// behind them (teams solve independently, so no team may store into a block
// another team reads).  The addresses are kept for 4-byte elements, the FP32
// vectors' stride (consecutive elements on consecutive banks), from the block's
// start; the FP64 products of the outer residual use 2 * address - start, the
// 8-byte layout of the same block.  A slot without an entry points at the FP32
// cell behind the rows, whose FP64 image is the block's zero cell; an FP64
// vector overwrites the FP32 cell, so every FP32 product writes it again.  No
// block-Jacobi kernel takes this layout.
template <class VS, int NZ_, int SRC = kSrcCsr, bool MX = false>
struct VarRows {
  static constexpr int R = VS::R, NZ = NZ_, ROWS = VS::ROWS;
  static constexpr int OCC = VS::OCC;  // waves per SIMD the allocator is held to
  static constexpr unsigned kBuf = var_buf_bytes<VS>();
  static constexpr unsigned kElem = MX ? 4 : 8;  // bytes between elements in c and vrow
  double a[R][NZ];
  unsigned c[R][NZ];
  unsigned vrow[R];
  int row[R];
  bool ok[R];
  int dslot[R];
  unsigned zero;
  unsigned b0;  // MX: start of this team's block in buffer 0
  int n;  // rows of this team's system
  double dval[R], bval[R], xval[R], xalt[R];

  // Pattern and values of this team's system, straight from HBM.  Every load
  // is guarded: an idle lane, row or slot reads nothing.  The diagonal slot is
  // the first entry of the row whose column is the row itself.
  __device__ void load(const VarTeam<VS>& tm, const VArgs& va, unsigned lds_base) {
    const KArgs& g = va.base;
    const int s = tm.live ? (int)tm.sys : 0;
    n = tm.live ? va.sys_rows[s] : 0;
    const int p = va.sys_pat[s];
    const unsigned tr = (unsigned)(tm.T * R);  // rows of a team's block
    const unsigned tb = MX ? lds_base + (unsigned)tm.tix * (tr + 1) * 8
                           : lds_base + (unsigned)tm.tix * tr * 8;
    zero = MX ? tb + tr * 4 : lds_base + (unsigned)(ROWS + tm.tix) * 8;
    b0 = tb;
    if constexpr (MX) {
      // the block's FP64 zero cell in both buffers (the previous task may have
      // left a row value there); the first product's barrier orders these stores
      if (tm.lane == 0) {
        lds_store<double>(tb + tr * 8, 0.0);
        lds_store<double>(tb + tr * 8 + kBuf, 0.0);
      }
    }
    const int* rps = va.rowptr_all + va.pat_rp[p];
    const double* vals = g.values + va.val_off[s];
    // the pattern's index bases, read once (inside the slots' branches the
    // compiler read them again, and waited for them, at every slot)
    const int64_t pcol = SRC == kSrcSlotIdx ? va.pat_slot[p] : va.pat_col[p];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      row[r] = tm.lane + r * tm.T;
      ok[r] = row[r] < n;
      vrow[r] = tb + (unsigned)row[r] * kElem;
      const int rr = row[r];
      int len = 0, ds = -1, rp = 0;
      double dv = 0.0;
      if constexpr (SRC == kSrcSlotIdx) {
        len = ok[r] ? va.pat_w[p] : 0;
      } else if (ok[r]) {
        rp = rps[rr];
        len = rps[rr + 1] - rp;
      }
      // Every index and value load of the row first, their use after: used
      // right behind its load, each made the compiler wait for it before
      // issuing the next, one memory round trip per slot and source.  (Four
      // rows per lane keep the slot-by-slot form: there the separate phases
      // push the block-Jacobi kernels' registers into scratch.)
      if constexpr (R <= 2) {
        int colk[NZ], posk[NZ];
        bool hask[NZ];
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
          hask[k] = k < len;
          colk[k] = 0;
          posk[k] = 0;
          if (hask[k]) {
            if constexpr (SRC == kSrcCsr) {
              colk[k] = va.col_all[pcol + rp + k];
              posk[k] = rp + k;
            } else if constexpr (SRC == kSrcRowIdx) {
              const int2 e = va.idx_row[pcol + rp + k];
              colk[k] = e.x;
              posk[k] = e.y;
            } else {
              const int2 e = va.idx_slot[pcol + (int64_t)k * n + rr];
              colk[k] = e.x;
              posk[k] = e.y;
            }
          }
        }
        double vk[NZ];
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
          if constexpr (SRC == kSrcSlotIdx) hask[k] = hask[k] && colk[k] >= 0;
          vk[k] = 0.0;
          if (hask[k]) vk[k] = __builtin_nontemporal_load(vals + posk[k]);
        }
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
          const bool has = hask[k];
          const int col = colk[k];
          if (has && col == rr && ds < 0) {
            ds = k;
            dv = vk[k];
          }
          c[r][k] = has ? tb + col * kElem : zero;
          a[r][k] = vk[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
          bool has = k < len;
          int col = 0, pos = 0;
          if (has) {
            if constexpr (SRC == kSrcCsr) {
              col = va.col_all[pcol + rp + k];
              pos = rp + k;
            } else if constexpr (SRC == kSrcRowIdx) {
              const int2 e = va.idx_row[pcol + rp + k];
              col = e.x;
              pos = e.y;
            } else {
              const int2 e = va.idx_slot[pcol + (int64_t)k * n + rr];
              col = e.x;
              pos = e.y;
              has = col >= 0;
            }
          }
          double v = 0.0;
          if (has) v = __builtin_nontemporal_load(vals + pos);
          if (has && col == rr && ds < 0) {
            ds = k;
            dv = v;
          }
          c[r][k] = has ? tb + col * kElem : zero;
          a[r][k] = v;
        }
      }
      dslot[r] = ds;
      dval[r] = dv;
      bval[r] = ok[r] ? g.b[tm.row0 + rr] : 0.0;
      double xv = 0.0;
      if ((g.flags & 1) == 0 && ok[r]) xv = g.x[tm.row0 + rr];
      xval[r] = xv;
      double xa = 0.0;
      if (g.x_alt && ok[r]) xa = g.x_alt[tm.row0 + rr];
      xalt[r] = xa;
    }
  }

  __device__ __forceinline__ bool real(int r, int k) const { return c[r][k] != zero; }
  __device__ __forceinline__ int nrows(const KArgs&) const { return n; }

  __device__ void jacobi(int precond, double (&d)[R]) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double dv = dval[r];
      d[r] = !ok[r] ? 0.0 : (precond == 1 && dslot[r] >= 0 && dv != 0.0) ? 1.0 / dv : 1.0;
    }
  }

  template <int BUF, class V, class AT>
  __device__ __forceinline__ void spmv(VarTeam<VS>& tm, const AT (&av)[R][NZ], const V (&v)[R],
                                       V (&y)[R]) const {
    constexpr int kGather = 4;
    constexpr unsigned off = BUF * kBuf;
    // FP64 vectors in a mixed kernel: twice the 4-byte-element address, formed
    // at each use (the empty asm keeps a second set of addresses out of the
    // registers)
    constexpr bool kWide = MX && sizeof(V) == 8;
    auto at = [&](unsigned x) -> unsigned {
      if constexpr (kWide) {
        __asm__ volatile("" : "+v"(x));
        return 2u * x - b0;
      } else {
        return x;
      }
    };
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (ok[r]) lds_store<V>(at(vrow[r]) + off, v[r]);
    if constexpr (MX && sizeof(V) == 4) {
      if (tm.lane == 0) lds_store<float>(zero + off, 0.0f);
    }
    tm.sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      V acc[4] = {0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < NZ; k0 += kGather) {
        V xv[kGather];
#pragma unroll
        for (int k = k0; k < k0 + kGather && k < NZ; ++k) xv[k - k0] = lds_load<V>(at(c[r][k]) + off);
#pragma unroll
        for (int k = k0; k < k0 + kGather && k < NZ; ++k)
          acc[k % 4] = fma((V)av[r][k], xv[k - k0], acc[k % 4]);
        __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])::"memory");
      }
      y[r] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  }
};

// The streamed placement: a lane keeps only where its rows start; every
// product reads the columns (or index entries) and the values from memory
// again (the pattern arrays are shared by all systems of a pattern and stay in
// the caches; a system's values are re-read from L2 or HBM).  No register
// holds a row, so rows of any length fit, and the registers the row values
// would take are free for more resident waves.  Scalar Jacobi or none only.
template <class VS, int SRC>
struct VarRowsS {
  static constexpr int R = VS::R, NZ = 1, ROWS = VS::ROWS;
  // GMRES (shared-pattern streamed kernel only) runs one team per workgroup
  static constexpr int WG = VS::WG, TEAM = VS::WG;
  // without the rows in registers two workgroups fit one CU: four waves per
  // SIMD (128 registers a lane) for 512 lanes, two (256) for 256 lanes x 4 rows
  static constexpr int OCC = VS::WG >= 512 ? 4 : 2;
  static constexpr unsigned kBuf = var_buf_bytes<VS>();
  double a[R][NZ];  // not read: the products take the values from memory
  unsigned vrow[R];
  int row[R];
  bool ok[R];
  int dslot[R];     // 0 when the row stores its diagonal, else -1
  int start[R];     // row walks: first entry of the row in the pattern arrays
  int len[R];       // entries of the row (slot walk: the pattern's slot count)
  unsigned tb, zero;
  int n;
  const int* cols;   // kSrcCsr; kSrcShared: the slot-major columns
  const int2* ix;    // kSrcRowIdx, kSrcSlotIdx
  const double* vals;
  int ell;           // kSrcShared: values in the ELL layout
  double dval[R], bval[R], xval[R], xalt[R];

  // Entry k of row r: column (-1 when absent) and value position.
  __device__ __forceinline__ int2 entry(int r, int k) const {
    if constexpr (SRC == kSrcCsr) return make_int2(cols[start[r] + k], start[r] + k);
    else if constexpr (SRC == kSrcRowIdx) return ix[start[r] + k];
    else if constexpr (SRC == kSrcSlotIdx) return ix[(int64_t)k * n + row[r]];
    else return make_int2(cols[k * n + row[r]], ell ? k * n + row[r] : start[r] + k);
  }

  // kSrcShared: this team's system of a shared-pattern batch (solve tm.sys,
  // matrix tm.sys / nrhs).
  __device__ void load(const VarTeam<VS>& tm, const KArgs& g, unsigned lds_base) {
    static_assert(SRC == kSrcShared, "shared-pattern load");
    n = tm.live ? g.n : 0;
    tb = lds_base + (unsigned)(tm.tix * tm.T * R) * 8;
    zero = lds_base + (unsigned)(ROWS + tm.tix) * 8;
    cols = g.slot_col;
    ix = nullptr;
    ell = g.fmt;
    const int64_t per = g.fmt == 0 ? (int64_t)g.nnz : (int64_t)g.width * g.n;
    vals = g.values + (tm.live ? matrix_of(g, tm.sys) * per : 0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      row[r] = tm.lane + r * tm.T;
      ok[r] = row[r] < n;
      vrow[r] = tb + (unsigned)row[r] * 8;
      const int rr = row[r];
      start[r] = ok[r] ? g.row_ptr[rr] : 0;
      len[r] = ok[r] ? g.row_len[rr] : 0;
      const int ds = ok[r] ? g.diag_slot[rr] : -1;
      dslot[r] = ds >= 0 ? 0 : -1;
      dval[r] = ds >= 0 ? vals[ell ? ds * n + rr : start[r] + ds] : 0.0;
      bval[r] = ok[r] ? g.b[tm.row0 + rr] : 0.0;
      double xv = 0.0;
      if ((g.flags & 1) == 0 && ok[r]) xv = g.x[tm.row0 + rr];
      xval[r] = xv;
      double xa = 0.0;
      if (g.x_alt && ok[r]) xa = g.x_alt[tm.row0 + rr];
      xalt[r] = xa;
    }
  }

  __device__ void load(const VarTeam<VS>& tm, const VArgs& va, unsigned lds_base) {
    const KArgs& g = va.base;
    const int s = tm.live ? (int)tm.sys : 0;
    n = tm.live ? va.sys_rows[s] : 0;
    const int p = va.sys_pat[s];
    tb = lds_base + (unsigned)(tm.tix * tm.T * R) * 8;
    zero = lds_base + (unsigned)(ROWS + tm.tix) * 8;
    const int* rps = va.rowptr_all + va.pat_rp[p];
    cols = nullptr;
    ix = nullptr;
    if constexpr (SRC == kSrcCsr) cols = va.col_all + va.pat_col[p];
    else if constexpr (SRC == kSrcRowIdx) ix = va.idx_row + va.pat_col[p];
    else ix = va.idx_slot + va.pat_slot[p];
    vals = g.values + va.val_off[s];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      row[r] = tm.lane + r * tm.T;
      ok[r] = row[r] < n;
      vrow[r] = tb + (unsigned)row[r] * 8;
      const int rr = row[r];
      start[r] = 0;
      len[r] = 0;
      if (ok[r]) {
        if constexpr (SRC == kSrcSlotIdx) {
          len[r] = va.pat_w[p];
        } else {
          start[r] = rps[rr];
          len[r] = rps[rr + 1] - start[r];
        }
      }
      // the diagonal: first entry whose column is the row itself
      int ds = -1;
      double dv = 0.0;
#pragma unroll 1
      for (int k = 0; k < len[r]; ++k) {
        const int2 e = entry(r, k);
        if (e.x == rr) {
          ds = 0;
          dv = vals[e.y];
          break;
        }
      }
      dslot[r] = ds;
      dval[r] = dv;
      bval[r] = ok[r] ? g.b[tm.row0 + rr] : 0.0;
      double xv = 0.0;
      if ((g.flags & 1) == 0 && ok[r]) xv = g.x[tm.row0 + rr];
      xval[r] = xv;
      double xa = 0.0;
      if (g.x_alt && ok[r]) xa = g.x_alt[tm.row0 + rr];
      xalt[r] = xa;
    }
  }

  __device__ __forceinline__ bool real(int, int) const { return false; }
  __device__ __forceinline__ int nrows(const KArgs&) const { return n; }

  __device__ void jacobi(int precond, double (&d)[R]) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double dv = dval[r];
      d[r] = !ok[r] ? 0.0 : (precond == 1 && dslot[r] >= 0 && dv != 0.0) ? 1.0 / dv : 1.0;
    }
  }

  // Entries in groups of four: the index and value loads of a group are
  // issued together, then its LDS gathers, then the FMAs (slot k into
  // accumulator k mod 4, the order of the register placement).
  template <int BUF, bool PIPE = true, class V, class AT>
  __device__ __forceinline__ void spmv(VarTeam<VS>& tm, const AT (&)[R][NZ], const V (&v)[R],
                                       V (&y)[R]) const {
    constexpr unsigned off = BUF * kBuf;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (ok[r]) lds_store<V>(vrow[r] + off, v[r]);
    tm.sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      V acc[4] = {0, 0, 0, 0};
#pragma unroll 1
      for (int k0 = 0; k0 < len[r]; k0 += 4) {
        int2 e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] = k0 + j < len[r] ? entry(r, k0 + j) : make_int2(-1, 0);
        double av[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) av[j] = e[j].x >= 0 ? vals[e[j].y] : 0.0;
        V xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          xv[j] = lds_load<V>((e[j].x >= 0 ? tb + (unsigned)e[j].x * 8 : zero) + off);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = fma((V)av[j], xv[j], acc[j]);
      }
      y[r] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  }
};

// Per-class launches of one solve use counters counter[0..kMaxClasses), all
// cleared by k_varlen_reset (one wave; defined with the host entry points).
constexpr int kMaxClasses = 8;
__global__ void k_varlen_reset(int* counter);

// RowsT: VarRows<VS, NZ, SRC> (rows in registers) or VarRowsS<VS, SRC>.
template <class VS, class RowsT, int SOLVER, bool MIXED, bool BJ = false>
__global__ __launch_bounds__(VS::WG) __attribute__((amdgpu_waves_per_eu(RowsT::OCC)))
void k_varlen(const VArgs va) {
  static_assert(!(MIXED && BJ), "the mixed kernels' per-team blocks carry no block Jacobi");
  // buffers and reduction slots, then (BJ) the block-Jacobi region of the largest block
  __shared__ __align__(16) char smem[var_lds_bytes<VS>() + (BJ ? bj_bytes(VS::ROWS, kMaxBlock) : 0)];
  __shared__ int task_sh;
  const unsigned lds_base = lds_addr(smem);
  constexpr unsigned kBuf = var_buf_bytes<VS>();
  if (threadIdx.x < VS::MAXT * kVecBuffers) {  // zero cells of both buffers
    const int b = threadIdx.x / VS::MAXT, t = threadIdx.x % VS::MAXT;
    lds_store<double>(lds_base + b * kBuf + (VS::ROWS + t) * 8, 0.0);
  }
  VarTeam<VS> tm;
  tm.phase = 0;
  for (;;) {
    if (threadIdx.x == 0) task_sh = atomicAdd(va.counter, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(task_sh);
    __syncthreads();  // every lane has read the task before it is overwritten
    // Read the arguments at an address that depends on the task index (the
    // offset is zero: task indices are never negative).  Otherwise the compiler
    // hoists every argument load out of this loop and the ones that only the
    // loading phase needs stay live in scalar registers through the whole
    // solve, where they spill.
    const VArgs& a = (&va)[(unsigned)t >> 31];
    if (t >= a.n_tasks) break;
    const VTask task = a.tasks[t];
    tm.set_team(task.team, smem);
    tm.live = tm.tix < task.count;
    tm.sys = tm.live ? a.order[task.first + tm.tix] : 0;
    tm.row0 = tm.live ? a.row_off[tm.sys] : 0;
    RowsT A;
    A.load(tm, a, lds_base);
    if constexpr (SOLVER == 0) cg_system<BJ ? kPkBlock : kPkScalar>(tm, A, a.base);
    else bicgstab_system<MIXED, BJ ? kPkBlock : kPkScalar>(tm, A, a.base);
  }
}

// GMRES regions of a runtime-size team (one team per workgroup): behind the
// buffers and reduction slots.
template <class VS>
__device__ __forceinline__ double* gmres_scalar_base(const VarTeam<VS>& tm, int) {
  return reinterpret_cast<double*>(tm.lds + var_lds_bytes<VS>());
}
template <class VS>
__device__ __forceinline__ unsigned gmres_basis_base(const VarTeam<VS>& tm, int) {
  return lds_addr(tm.lds) + var_lds_bytes<VS>() + round16(kGmresScalars * 8);
}
template <class VS, bool MIXED>
constexpr int stream_gmres_lds_bytes() {
  return round16(kGmresScalars * 8) +
         round16(gmres_lds_vectors(VS::WG, MIXED) * VS::ROWS * (MIXED ? 4 : 8));
}

// A batch of systems that share one pattern, rows streamed (the register
// kernels cannot hold rows this long): teams of `team` lanes (a power of two,
// 64..WG) own R rows per lane; task t is the WG/team consecutive solves from
// t * WG/team, taken by the workgroups in turn (every task has the same size).
// SOLVER 2 (GMRES) takes one team of WG lanes per workgroup and one row per
// lane; its scalars and LDS basis vectors follow the buffers.
template <class VS, int SOLVER, bool MIXED>
__global__ __launch_bounds__(VS::WG)
__attribute__((amdgpu_waves_per_eu(VarRowsS<VS, kSrcShared>::OCC)))
void k_shared_stream(const KArgs g, int team) {
  __shared__ __align__(16)
      char smem[var_lds_bytes<VS>() + (SOLVER == 2 ? stream_gmres_lds_bytes<VS, MIXED>() : 0)];
  const unsigned lds_base = lds_addr(smem);
  constexpr unsigned kBuf = var_buf_bytes<VS>();
  if (threadIdx.x < VS::MAXT * kVecBuffers) {  // zero cells of both buffers
    const int b = threadIdx.x / VS::MAXT, t = threadIdx.x % VS::MAXT;
    lds_store<double>(lds_base + b * kBuf + (VS::ROWS + t) * 8, 0.0);
  }
  __syncthreads();
  VarTeam<VS> tm;
  tm.phase = 0;
  tm.set_team(team, smem);
  const int cap = VS::WG / team;
  const int64_t n_tasks = (g.n_batch + cap - 1) / cap;
  for (int64_t t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const int64_t s = t * cap + tm.tix;
    tm.live = s < g.n_batch;
    tm.sys = tm.live ? s : 0;
    tm.row0 = tm.sys * g.n;
    VarRowsS<VS, kSrcShared> A;
    A.load(tm, g, lds_base);
    if constexpr (SOLVER == 0) cg_system<kPkScalar>(tm, A, g);
    else if constexpr (SOLVER == 1) bicgstab_system<MIXED, kPkScalar>(tm, A, g);
    else gmres_system<MIXED, kPkScalar>(tm, A, g);
    __syncthreads();  // every team is done with its buffers before the next task
  }
}

// GMRES(m) for systems of more than one row per lane whose basis fits neither
// registers nor LDS (streamed rows on 1024-lane x 2-row workgroups, 1025..2048
// rows): the steps of gmres_system for teams of a wave or more (block modified
// Gram-Schmidt in blocks of four, the rotations and the back substitution
// through lane registers), every per-lane vector widened to the lane's R rows,
// and basis vector i kept in device memory at ws[i * ROWS + row].  Each lane
// reads back only the elements it wrote, so the buffer needs no barrier.
// FP64, scalar Jacobi or none.
template <class VS>
__device__ void gmres_system_wide(VarTeam<VS>& tm, VarRowsS<VS, kSrcShared>& A, const KArgs& g,
                                  double* __restrict__ ws) {
  using RW = VarRowsS<VS, kSrcShared>;
  constexpr int R = VS::R, M = kMaxRestart;
  Prologue<R> P;
  prologue<kPkScalar>(tm, A, g, P);
  const int m = g.restart;
  double* hcol = gmres_scalar_base(tm, RW::ROWS);
  double* Rt = hcol + (M + 2);  // packed by columns: R[i][j] at j(j+1)/2 + i
  double* cs = Rt + M * (M + 1) / 2;
  double* sn = cs + M;
  double* gv = sn + M;
  // this lane's element of basis vector i in row slot r
  auto at = [&](int i, int r) -> double* { return ws + (size_t)i * RW::ROWS + A.row[r]; };
  double q1[1] = {0.0};
#pragma unroll
  for (int r = 0; r < R; ++r) q1[0] += P.b[r] * P.b[r];
  tm.sum(q1);
  const double bn = sqrt(q1[0]);
  const double lim = stop_limit(g, bn);
  int st = tm.live ? ST_RUNNING : ST_IDLE;
  double rn = 0.0;
  if (st == ST_RUNNING) {
    if (!finite(bn)) {
      st = ST_NONFINITE;
    } else if (bn == 0.0) {
      st = ST_CONVERGED;
#pragma unroll
      for (int r = 0; r < R; ++r) P.x[r] = 0.0;
    }
  }
  int k = 0, j = 0;
  double vcur[R];      // the basis vector the next Arnoldi step multiplies
  double gcur = 0.0;   // g_j, the entry the next rotation acts on
  bool start = true;   // at a cycle start (true residual due)
#pragma unroll
  for (int r = 0; r < R; ++r) vcur[r] = 0.0;
  for (;;) {
    // ---- cycle start: true residual, convergence, V0 = r/beta
    if (tm.any(st == ST_RUNNING && start)) {
      const bool me = st == ST_RUNNING && start;
      double t[R], rc[R], q[1] = {0.0};
      A.template spmv<0, false>(tm, A.a, P.x, t);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        rc[r] = P.b[r] - t[r];
        q[0] += rc[r] * rc[r];
      }
      tm.sum(q);
      if (me) {
        const double beta = sqrt(q[0]);
        rn = beta;
        if (!finite(beta)) {
          st = ST_NONFINITE;
        } else if (beta <= lim) {
          st = ST_CONVERGED;
        } else if (k >= g.max_iter) {
          st = ST_MAX_ITER;
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            vcur[r] = rc[r] / beta;
            if (A.ok[r]) *at(0, r) = vcur[r];
          }
          gcur = beta;
          j = 0;
          start = false;
        }
      }
    }
    if (!tm.any(st == ST_RUNNING)) break;
    // ---- one Arnoldi step
    const bool act = st == ST_RUNNING;
    double z[R], w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = P.d[r] * vcur[r];
    A.template spmv<0, false>(tm, A.a, z, w);
    const int jmax = wave_max(act ? j : -1);
    // blocks taken in a loop (the basis is addressed, not in registers)
#pragma unroll 1
    for (int b0 = 0; b0 <= jmax && b0 < M; b0 += 4) {
      {
        double vq[4][R], q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          q[u] = 0.0;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            vq[u][r] = (b0 + u < M && b0 + u <= j && A.ok[r]) ? *at(b0 + u, r) : 0.0;
            q[u] += w[r] * vq[u][r];
          }
        }
        tm.sum(q);
        if (act) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (b0 + u < M && b0 + u <= j) {
#pragma unroll
              for (int r = 0; r < R; ++r) w[r] = fma(-q[u], vq[u][r], w[r]);
              hcol[b0 + u] = q[u];
            }
          }
        }
      }
    }
    double qn[1] = {0.0};
#pragma unroll
    for (int r = 0; r < R; ++r) qn[0] += w[r] * w[r];
    tm.sum(qn);
    bool end = false;
    if (act) {
      const double hn = sqrt(qn[0]);
      k += 1;
      if (!finite(hn)) {
        st = ST_NONFINITE;
      } else {
        // the previous rotations applied to column j, read one entry per lane
        const int cj = j * (j + 1) / 2;
        const int ju = __builtin_amdgcn_readfirstlane(j);
        const int l = (int)lane_id();
        const double hreg = l <= ju ? hcol[l] : 0.0;
        const double creg = l < ju ? cs[l] : 0.0, sreg = l < ju ? sn[l] : 0.0;
        double hp = rdlane(hreg, 0);
        for (int i = 0; i < ju; ++i) {
          const double hnx = rdlane(hreg, i + 1), c = rdlane(creg, i), s = rdlane(sreg, i);
          Rt[cj + i] = c * hp + s * hnx;
          hp = -s * hp + c * hnx;
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
          end = fabs(gcur) <= lim || hn == 0.0 || k >= g.max_iter || j == m - 1;
          if (!end) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              vcur[r] = w[r] / hn;
              if (A.ok[r]) *at(j + 1, r) = vcur[r];
            }
            j += 1;
          }
        }
      }
    }
    // ---- cycle end: y = R^{-1} g (back substitution), x += M V y
    if (tm.any(end)) {
      double zacc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) zacc[r] = 0.0;
      if (end) {
        const int je = __builtin_amdgcn_readfirstlane(j);
        const int l = (int)lane_id();
        double acc = l <= je ? gv[l] : 0.0;
        for (int i = je; i >= 0; --i) {
          const double yi = rdlane(acc, i) / Rt[i * (i + 1) / 2 + i];
          if (l < i) acc = fma(-Rt[i * (i + 1) / 2 + l], yi, acc);
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (A.ok[r]) zacc[r] = fma(yi, *at(i, r), zacc[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) P.x[r] = fma(P.d[r], zacc[r], P.x[r]);
        start = true;
      }
    }
  }
  finish(tm, A, g, P.b, P.x, st, k, 0, bn, rn,
         st == ST_CONVERGED || st == ST_IDLE || (st == ST_MAX_ITER && start));
}

// GMRES beyond 1024 rows on streamed rows: one system per workgroup of
// VS::WG lanes x VS::R rows, workgroup b keeping its basis at
// ws + b * (kMaxRestart + 1) * VS::ROWS; systems taken in turn.
template <class VS>
__global__ __launch_bounds__(VS::WG) __attribute__((amdgpu_waves_per_eu(VarRowsS<VS, kSrcShared>::OCC)))
void k_gmres_wide(const KArgs g, double* ws) {
  __shared__ __align__(16) char smem[var_lds_bytes<VS>() + round16(kGmresScalars * 8)];
  const unsigned lds_base = lds_addr(smem);
  constexpr unsigned kBuf = var_buf_bytes<VS>();
  if (threadIdx.x < VS::MAXT * kVecBuffers) {  // zero cells of both buffers
    const int b = threadIdx.x / VS::MAXT, t = threadIdx.x % VS::MAXT;
    lds_store<double>(lds_base + b * kBuf + (VS::ROWS + t) * 8, 0.0);
  }
  __syncthreads();
  VarTeam<VS> tm;
  tm.phase = 0;
  tm.set_team(VS::WG, smem);
  double* const wb = ws + (size_t)blockIdx.x * (kMaxRestart + 1) * VS::ROWS;
  for (int64_t s = blockIdx.x; s < g.n_batch; s += gridDim.x) {
    tm.live = true;
    tm.sys = s;
    tm.row0 = s * g.n;
    VarRowsS<VS, kSrcShared> A;
    A.load(tm, g, lds_base);
    gmres_system_wide(tm, A, g, wb);
    __syncthreads();  // done with the buffers before the next system
  }
}

}  // namespace bs
