// Uneven batches in one persistent launch: systems of different sizes (and
// patterns) share one kernel.  A workgroup of kVarWG lanes takes tasks from an
// atomic queue; a task is up to kVarWG/T systems of one size class, each
// solved by a team of T lanes (T a power of two in [64, kVarWG], one row per
// lane).  The teams of a workgroup advance in lockstep: every barrier and
// every branch around a barrier is decided for the whole workgroup (any() is a
// workgroup-wide OR), so a team that has finished idles until the task ends.
// The solver bodies are the ones of the fixed-size kernels.
#pragma once
#include "bs_solvers.hpp"

namespace bs {

constexpr int kVarWG = 1024;
constexpr int kVarWaves = kVarWG / kWave;
constexpr int kVarMaxTeams = kVarWG / kWave;  // teams of at least one wave

struct VTask {
  int team;   // lanes per system
  int first;  // index of the first system in the queue order
  int count;  // systems in this task (<= kVarWG / team)
  int pad;
};

struct VArgs {
  KArgs base;             // solver settings and the per-system outputs
  int64_t n_tasks;
  const VTask* tasks;
  const int* order;       // system ids in queue order
  const int* sys_rows;    // [B]
  const int* sys_pat;     // [B] pattern of each system
  const int64_t* row_off; // [B+1] first row of each system in b and x
  const int64_t* val_off; // [B+1] first value of each system (CSR order)
  const int64_t* pat_rp;  // [P] offset of the pattern's row_ptr in prow_ptr
  const int64_t* pat_row; // [P] offset of the pattern's per-row arrays
  const int64_t* pat_sc;  // [P] offset of the pattern's slot-major columns
  const int* prow_ptr;    // concatenated row_ptr arrays
  const int* prow_len;    // concatenated row lengths
  const int* pdiag;       // concatenated diagonal slots (-1 if none)
  const int* pslot_col;   // concatenated [W_p][n_p] slot-major columns
  int* counter;           // task counter, zero at launch
};

// Team of runtime size inside a kVarWG-lane workgroup.
struct VarTeam {
  int T;               // lanes per team (uniform across the workgroup)
  int lane, tix;       // lane within the team, team within the workgroup
  int wpt;             // waves per team
  int64_t sys, row0;
  bool live;
  char* lds;           // vector buffers (shared layout, see VarRows)
  double* red;         // cross-wave reduction slots
  int phase;

  __device__ void set_team(int t, char* smem) {
    T = t;
    lane = threadIdx.x & (t - 1);
    tix = threadIdx.x / t;
    wpt = t / kWave;
    lds = smem;
    red = reinterpret_cast<double*>(smem + 2 * (kVarWG + kVarMaxTeams) * 8);
  }

  __device__ __forceinline__ void sync() { __syncthreads(); }

  // Workgroup-wide: teams run in lockstep, so every branch that contains a
  // barrier must be taken by all of them.
  __device__ __forceinline__ bool any(bool p) const { return __syncthreads_or(p ? 1 : 0) != 0; }

  template <class V, int K>
  __device__ __forceinline__ void sum(V (&v)[K]) {
    static_assert(K <= kMaxFused, "too many fused values");
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = rdlane(rows_total(row16_sum(v[k])), 63);
    if (wpt > 1) {  // uniform: every team of the task has the same size
      double* buf = red + phase * (kMaxFused * kVarWaves);
      const int w = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) buf[k * kVarWaves + w] = (double)v[k];
      }
      __syncthreads();
      const int w0 = tix * wpt;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double s = buf[k * kVarWaves + w0];
        for (int i = 1; i < wpt; ++i) s += buf[k * kVarWaves + w0 + i];
        v[k] = (V)s;
      }
      phase ^= 1;
    }
  }
};

// The row a lane owns (one per lane).  Vector buffer b holds team t's row i at
// element t*T + i, and the teams' zero cells after the kVarWG rows, so the
// buffer stride is a constant whatever the team size.
template <int NZ_>
struct VarRows {
  static constexpr int R = 1, NZ = NZ_, ROWS = kVarWG;
  static constexpr unsigned kBuf = (kVarWG + kVarMaxTeams) * 8;
  double a[1][NZ];
  unsigned c[1][NZ];
  unsigned vrow[1];
  int row[1];
  bool ok[1];
  int dslot[1];
  unsigned zero;
  double dval[1], bval[1], xval[1];

  // Pattern and values of this team's system, straight from HBM.
  __device__ void load(const VarTeam& tm, const VArgs& va, unsigned lds_base) {
    const KArgs& g = va.base;
    const int s = tm.live ? (int)tm.sys : 0;
    const int n = tm.live ? va.sys_rows[s] : 0;
    const int p = va.sys_pat[s];
    row[0] = tm.lane;
    ok[0] = tm.lane < n;
    vrow[0] = lds_base + (unsigned)(tm.tix * tm.T + tm.lane) * 8;
    zero = lds_base + (unsigned)(kVarWG + tm.tix) * 8;
    const int rr = ok[0] ? row[0] : 0;
    const int64_t pr = va.pat_row[p];
    const int len = ok[0] ? va.prow_len[pr + rr] : 0;
    const int ds = ok[0] ? va.pdiag[pr + rr] : -1;
    const int rp = ok[0] ? va.prow_ptr[va.pat_rp[p] + rr] : 0;
    const int* sc = va.pslot_col + va.pat_sc[p];
    const double* vals = g.values + va.val_off[s];
    const unsigned tb = lds_base + (unsigned)(tm.tix * tm.T) * 8;
    // every load is guarded: an idle lane or slot reads nothing
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      const bool has = k < len;
      int col = 0;
      double v = 0.0;
      if (has) {
        col = sc[(size_t)k * n + rr];
        v = __builtin_nontemporal_load(vals + rp + k);
      }
      c[0][k] = has ? tb + col * 8 : zero;
      a[0][k] = v;
    }
    dslot[0] = ds;
    dval[0] = ds >= 0 ? vals[rp + ds] : 0.0;
    bval[0] = ok[0] ? g.b[tm.row0 + rr] : 0.0;
    double xv = 0.0;
    if ((g.flags & 1) == 0 && ok[0]) xv = g.x[tm.row0 + rr];
    xval[0] = xv;
  }

  __device__ __forceinline__ bool real(int, int k) const { return c[0][k] != zero; }

  __device__ void jacobi(int precond, double (&d)[1]) const {
    const double dv = dval[0];
    d[0] = !ok[0] ? 0.0 : (precond == 1 && dslot[0] >= 0 && dv != 0.0) ? 1.0 / dv : 1.0;
  }

  template <int BUF, class V, class AT>
  __device__ __forceinline__ void spmv(VarTeam& tm, const AT (&av)[1][NZ], const V (&v)[1],
                                       V (&y)[1]) const {
    constexpr int kGather = 4;
    constexpr unsigned off = BUF * kBuf;
    if (ok[0]) lds_store<V>(vrow[0] + off, v[0]);
    tm.sync();
    V acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < NZ; k0 += kGather) {
      V xv[kGather];
#pragma unroll
      for (int k = k0; k < k0 + kGather && k < NZ; ++k) xv[k - k0] = lds_load<V>(c[0][k] + off);
#pragma unroll
      for (int k = k0; k < k0 + kGather && k < NZ; ++k)
        acc[k % 4] = fma((V)av[0][k], xv[k - k0], acc[k % 4]);
      __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])::"memory");
    }
    y[0] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
};

// LDS of the uneven-batch kernel: two vector buffers, then the reduction slots.
constexpr int kVarLdsBytes = 2 * (kVarWG + kVarMaxTeams) * 8 + 2 * kMaxFused * kVarWaves * 8;

__global__ void k_varlen_reset(int* counter) { *counter = 0; }

template <int NZ, int SOLVER, bool MIXED>
__global__ __launch_bounds__(kVarWG) void k_varlen(const VArgs va) {
  __shared__ __align__(16) char smem[kVarLdsBytes];
  __shared__ int task_sh;
  const unsigned lds_base = lds_addr(smem);
  if (threadIdx.x < kVarMaxTeams * kVecBuffers) {  // zero cells of both buffers
    const int b = threadIdx.x / kVarMaxTeams, t = threadIdx.x % kVarMaxTeams;
    lds_store<double>(lds_base + b * VarRows<NZ>::kBuf + (kVarWG + t) * 8, 0.0);
  }
  VarTeam tm;
  tm.phase = 0;
  for (;;) {
    if (threadIdx.x == 0) task_sh = atomicAdd(va.counter, 1);
    __syncthreads();
    const int t = task_sh;
    __syncthreads();  // every lane has read the task before it is overwritten
    if (t >= va.n_tasks) break;
    const VTask task = va.tasks[t];
    tm.set_team(task.team, smem);
    tm.live = tm.tix < task.count;
    tm.sys = tm.live ? va.order[task.first + tm.tix] : 0;
    tm.row0 = tm.live ? va.row_off[tm.sys] : 0;
    VarRows<NZ> A;
    A.load(tm, va, lds_base);
    if constexpr (SOLVER == 0) cg_system(tm, A, va.base);
    else bicgstab_system<MIXED>(tm, A, va.base);
  }
}

}  // namespace bs
