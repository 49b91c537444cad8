// Host side of the C ABI declared in include/batchsolve.h: argument and pattern
// validation, one-time pattern preprocessing (Sec. 3.1: one pattern copy for the
// whole batch), the kernel-shape planner (Sec. 3.3 multi-level dispatch,
// Sec. 3.5 on-chip placement, Sec. 3.6 size-dependent work-group choice) and the
// launch of the fused solver kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/batchsolve.h"
#include "bs_layout.hpp"
#include "bs_registry.hpp"
#include "bs_shape.hpp"

struct bs_pattern_s {
  int n = 0, nnz = 0, width = 0, max_row = 0, device = -1;
  std::vector<int> row_ptr, col, slot_col, row_len, diag_slot;
  // level of each row in the lower and upper triangles' dependency graphs,
  // packed (lower | upper << 16), and the level counts
  std::vector<int> lev;
  int nlev_l = 0, nlev_u = 0;
  // ILU(0) schedule of the multi-wave factorization: per row (ilu_ptr), its
  // steps in increasing pivot column k, a header word
  // 1 << 31 | pos(k,k) << 15 | pos(i,k) followed by one word
  // pos(k,j) << 16 | pos(i,j) per entry (i,j), j > k, that row k holds
  // (positions in the pattern's CSR order)
  std::vector<int> ilu_ptr, ilu_ops;
  // Sweep lists of the multi-wave teams (ILU(0) substitutions, BatchTrsv):
  // rows by lower level | rows by upper level | lower level starts (nlev_l+1)
  // | upper level starts (nlev_u+1) | per row its list start (16 bits),
  // lower and upper counts (8 bits each) | per row its strictly lower then
  // strictly upper entries in increasing column, CSR position | column << 16.
  std::vector<int> sweep;
  int sweep_ents = 0;
  // bank-aware layout for one-wave teams of layout_nz register slots (0: none)
  std::vector<int> layout;
  int layout_nz = 0;
  // one allocation: row_ptr | slot_col | row_len | diag_slot | lev | ilu_ptr |
  // ilu_ops | sweep | layout
  int* d_base = nullptr;
  int *d_row_ptr = nullptr, *d_slot_col = nullptr, *d_row_len = nullptr, *d_diag = nullptr;
  int *d_lev = nullptr, *d_ilu_ptr = nullptr, *d_ilu_ops = nullptr, *d_sweep = nullptr;
  int* d_layout = nullptr;
};

namespace {
thread_local std::string g_last_error = "";
}  // namespace

namespace bs {
// The streamed placement of shared-pattern batches (bs_stream_api.hip).
int stream_plan(int n, bs_solver solver, bs_precond precond, const bs_options* o,
                bs_plan_info* info);
int stream_launch(const KArgs& a, const bs_plan_info& info, bs_solver solver, int mixed, int cus,
                  hipStream_t s);

// Shared by every translation unit of the library (bs_last_error reads it).
void set_last_error(const std::string& msg) { g_last_error = msg; }

// A device word per device that kernels may write instead of an output the
// caller did not ask for (allocated once, kept until the process ends).
int* device_sink() {
  static std::mutex mu;
  static std::vector<int*> sinks;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)sinks.size() <= dev) sinks.resize(dev + 1, nullptr);
  if (!sinks[dev]) {
    void* p = nullptr;
    if (hipMalloc(&p, 256) != hipSuccess) {
      g_last_error = "sink allocation failed";
      return nullptr;
    }
    sinks[dev] = static_cast<int*>(p);
  }
  return sinks[dev];
}
}  // namespace bs

namespace {

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return BS_ERR_HIP;
}

// Derived per-row data shared by the CSR and ELL forms.
void derive(bs_pattern_s& p) {
  const int n = p.n;
  p.row_len.resize(n);
  p.diag_slot.assign(n, -1);
  p.max_row = 0;
  for (int i = 0; i < n; ++i) {
    const int len = p.row_ptr[i + 1] - p.row_ptr[i];
    p.row_len[i] = len;
    p.max_row = std::max(p.max_row, len);
    for (int k = 0; k < len; ++k)
      if (p.col[p.row_ptr[i] + k] == i && p.diag_slot[i] < 0) p.diag_slot[i] = k;
  }
  p.width = p.max_row;
  p.slot_col.assign((size_t)p.width * n, -1);
  for (int s = 0; s < p.width; ++s)
    for (int i = 0; i < n; ++i)
      if (s < p.row_len[i]) p.slot_col[(size_t)s * n + i] = p.col[p.row_ptr[i] + s];
  // Levels for the level-scheduled sweeps (ILU(0), BatchTrsv): a row's lower
  // level is one more than the largest lower level among the columns j < i it
  // holds (0 if none), its upper level likewise over the columns j > i, taken
  // from the last row up.
  std::vector<int> lo(n, 0), up(n, 0);
  for (int i = 0; i < n; ++i)
    for (int e = p.row_ptr[i]; e < p.row_ptr[i + 1]; ++e)
      if (p.col[e] < i) lo[i] = std::max(lo[i], lo[p.col[e]] + 1);
  for (int i = n - 1; i >= 0; --i)
    for (int e = p.row_ptr[i]; e < p.row_ptr[i + 1]; ++e)
      if (p.col[e] > i) up[i] = std::max(up[i], up[p.col[e]] + 1);
  p.lev.resize(n);
  p.nlev_l = p.nlev_u = 0;
  for (int i = 0; i < n; ++i) {
    // 16 bits each: the multi-wave paths that read it take at most 1024 rows
    p.lev[i] = (int)(((unsigned)lo[i] & 0xffffu) | ((unsigned)up[i] << 16));
    p.nlev_l = std::max(p.nlev_l, lo[i] + 1);
    p.nlev_u = std::max(p.nlev_u, up[i] + 1);
  }
  // The ILU(0) schedule (symbolic factorization, the IKJ form): for row i and
  // each column k < i it holds, in increasing k, divide (i,k) by the pivot
  // (k,k), then update each (i,j), j > k, for which row k holds (k,j).  A row
  // without a stored diagonal divides by its own entry instead: the system
  // then has a zero pivot and its preconditioner is the identity anyway.  Only
  // patterns whose positions fit 15 bits get one (the multi-wave shapes hold
  // at most 16384 entries).
  p.ilu_ptr.assign(n + 1, 0);
  p.ilu_ops.clear();
  if (p.nnz < (1 << 15)) {
    std::vector<int> where(n, -1), ks;
    for (int i = 0; i < n; ++i) {
      for (int e = p.row_ptr[i]; e < p.row_ptr[i + 1]; ++e) where[p.col[e]] = e;
      ks.clear();
      for (int e = p.row_ptr[i]; e < p.row_ptr[i + 1]; ++e)
        if (p.col[e] < i) ks.push_back(p.col[e]);
      std::sort(ks.begin(), ks.end());
      for (int k : ks) {
        const int pik = where[k];
        const int pkk = p.diag_slot[k] >= 0 ? p.row_ptr[k] + p.diag_slot[k] : pik;
        p.ilu_ops.push_back((int)(0x80000000u | ((unsigned)pkk << 15) | (unsigned)pik));
        for (int e = p.row_ptr[k]; e < p.row_ptr[k + 1]; ++e) {
          const int j = p.col[e];
          if (j > k && where[j] >= 0) p.ilu_ops.push_back((e << 16) | where[j]);
        }
      }
      for (int e = p.row_ptr[i]; e < p.row_ptr[i + 1]; ++e) where[p.col[e]] = -1;
      p.ilu_ptr[i + 1] = (int)p.ilu_ops.size();
    }
  }
  // Sweep lists (same 15-bit positions; rows of up to 255 entries per triangle;
  // columns below 2^15).
  p.sweep.clear();
  p.sweep_ents = 0;
  if (p.nnz < (1 << 15) && n < (1 << 15)) {
    std::vector<int> by_l(n), by_u(n), start_l(p.nlev_l + 1, 0), start_u(p.nlev_u + 1, 0);
    for (int i = 0; i < n; ++i) {
      ++start_l[lo[i] + 1];
      ++start_u[up[i] + 1];
    }
    for (int l = 0; l < p.nlev_l; ++l) start_l[l + 1] += start_l[l];
    for (int l = 0; l < p.nlev_u; ++l) start_u[l + 1] += start_u[l];
    std::vector<int> fill_l(start_l.begin(), start_l.end() - 1), fill_u(start_u.begin(), start_u.end() - 1);
    for (int i = 0; i < n; ++i) {
      by_l[fill_l[lo[i]]++] = i;
      by_u[fill_u[up[i]]++] = i;
    }
    std::vector<int> rng(n), ent;
    std::vector<std::pair<int, int>> lw, uw;
    bool fits = true;
    for (int i = 0; i < n && fits; ++i) {
      lw.clear();
      uw.clear();
      for (int e = p.row_ptr[i]; e < p.row_ptr[i + 1]; ++e) {
        if (p.col[e] < i) lw.push_back({p.col[e], e});
        if (p.col[e] > i) uw.push_back({p.col[e], e});
      }
      std::sort(lw.begin(), lw.end());
      std::sort(uw.begin(), uw.end());
      fits = lw.size() < 256 && uw.size() < 256;
      rng[i] = (int)((unsigned)ent.size() | ((unsigned)lw.size() << 16) | ((unsigned)uw.size() << 24));
      for (const auto& q : lw) ent.push_back(q.second | (q.first << 16));
      for (const auto& q : uw) ent.push_back(q.second | (q.first << 16));
    }
    if (fits) {
      p.sweep_ents = (int)ent.size();
      p.sweep.reserve(3 * n + p.nlev_l + p.nlev_u + 2 + ent.size());
      p.sweep.insert(p.sweep.end(), by_l.begin(), by_l.end());
      p.sweep.insert(p.sweep.end(), by_u.begin(), by_u.end());
      p.sweep.insert(p.sweep.end(), start_l.begin(), start_l.end());
      p.sweep.insert(p.sweep.end(), start_u.begin(), start_u.end());
      p.sweep.insert(p.sweep.end(), rng.begin(), rng.end());
      p.sweep.insert(p.sweep.end(), ent.begin(), ent.end());
    }
  }
}

int upload(bs_pattern_s& p) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    g_last_error = "no HIP device";
    return BS_ERR_NO_DEVICE;
  }
  hipError_t e = hipGetDevice(&p.device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const size_t n_rp = p.n + 1, n_sc = std::max<size_t>((size_t)p.width * p.n, 1), n_rl = p.n;
  const size_t n_ops = std::max<size_t>(p.ilu_ops.size(), 1);
  const size_t n_sw = std::max<size_t>(p.sweep.size(), 1);
  const size_t total = n_rp + n_sc + 3 * n_rl + n_rp + n_ops + n_sw + p.layout.size();
  e = hipMalloc(&p.d_base, total * sizeof(int));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(pattern)");
  p.d_row_ptr = p.d_base;
  p.d_slot_col = p.d_row_ptr + n_rp;
  p.d_row_len = p.d_slot_col + n_sc;
  p.d_diag = p.d_row_len + n_rl;
  p.d_lev = p.d_diag + n_rl;
  p.d_ilu_ptr = p.d_lev + n_rl;
  p.d_ilu_ops = p.d_ilu_ptr + n_rp;
  p.d_sweep = p.d_ilu_ops + n_ops;
  p.d_layout = p.layout.empty() ? nullptr : p.d_sweep + n_sw;
  std::vector<int> h(total, -1);
  const size_t o_lev = n_rp + n_sc + 2 * n_rl, o_ptr = o_lev + n_rl, o_ops = o_ptr + n_rp;
  std::copy(p.lev.begin(), p.lev.end(), h.begin() + o_lev);
  std::copy(p.ilu_ptr.begin(), p.ilu_ptr.end(), h.begin() + o_ptr);
  std::copy(p.ilu_ops.begin(), p.ilu_ops.end(), h.begin() + o_ops);
  std::copy(p.sweep.begin(), p.sweep.end(), h.begin() + o_ops + n_ops);
  std::copy(p.layout.begin(), p.layout.end(), h.begin() + o_ops + n_ops + n_sw);
  std::copy(p.row_ptr.begin(), p.row_ptr.end(), h.begin());
  std::copy(p.slot_col.begin(), p.slot_col.end(), h.begin() + n_rp);
  std::copy(p.row_len.begin(), p.row_len.end(), h.begin() + n_rp + n_sc);
  std::copy(p.diag_slot.begin(), p.diag_slot.end(), h.begin() + n_rp + n_sc + n_rl);
  e = hipMemcpy(p.d_base, h.data(), total * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p.d_base);
    p.d_base = nullptr;
    return hip_fail(e, "hipMemcpy(pattern)");
  }
  return BS_OK;
}

// Columns of one row must be in range and distinct.
bool row_ok(const int* cols, int len, int n, std::vector<int>& mark, int stamp) {
  for (int k = 0; k < len; ++k) {
    const int c = cols[k];
    if (c < 0 || c >= n || mark[c] == stamp) return false;
    mark[c] = stamp;
  }
  return true;
}

// block: block-Jacobi block size (0 without); block Jacobi is FP64 only.
int variant_of(bs_solver solver, int precision, int block = 0, bool ilu = false) {
  if (solver == BS_TRSV_LOWER || solver == BS_TRSV_UPPER) {
    if (precision == BS_MIXED) return -1;
    return solver == BS_TRSV_LOWER ? bs::V_TRSV_LOWER : bs::V_TRSV_UPPER;
  }
  if (ilu) {
    if (precision == BS_MIXED) return -1;
    if (solver == BS_BICGSTAB) return bs::V_BICGSTAB_ILU;
    if (solver == BS_GMRES) return bs::V_GMRES_ILU;
    return -1;  // CG needs a symmetric preconditioner
  }
  if (block > 1) {
    if (precision == BS_MIXED) return -1;
    if (solver == BS_CG) return bs::V_CG_BJ;
    if (solver == BS_BICGSTAB) return bs::V_BICGSTAB_BJ;
    if (solver == BS_GMRES) return bs::V_GMRES_BJ;
    return -1;
  }
  if (solver == BS_CG) return precision == BS_MIXED ? -1 : bs::V_CG;
  if (solver == BS_BICGSTAB) return precision == BS_MIXED ? bs::V_BICGSTAB_MIXED : bs::V_BICGSTAB;
  if (solver == BS_GMRES) return precision == BS_MIXED ? bs::V_GMRES_MIXED : bs::V_GMRES;
  return -1;
}

bs::KernelTable table_of(int variant) {
  switch (variant) {
    case bs::V_CG: return bs::kernels_cg();
    case bs::V_BICGSTAB: return bs::kernels_bicgstab();
    case bs::V_BICGSTAB_MIXED: return bs::kernels_bicgstab_mixed();
    case bs::V_GMRES: return bs::kernels_gmres();
    case bs::V_GMRES_MIXED: return bs::kernels_gmres_mixed();
    case bs::V_CG_BJ: return bs::kernels_cg_bj();
    case bs::V_BICGSTAB_BJ: return bs::kernels_bicgstab_bj();
    case bs::V_GMRES_BJ: return bs::kernels_gmres_bj();
    case bs::V_BICGSTAB_ILU: return bs::kernels_bicgstab_ilu();
    case bs::V_GMRES_ILU: return bs::kernels_gmres_ilu();
    case bs::V_TRSV_LOWER: return bs::kernels_trsv_lower();
    case bs::V_TRSV_UPPER: return bs::kernels_trsv_upper();
    default: return {nullptr, 0};
  }
}

const bs::KernelEntry* find_kernel(int variant, int team, int r, int nz_min) {
  const bs::KernelTable t = table_of(variant);
  const bs::KernelEntry* best = nullptr;
  for (int i = 0; i < t.count; ++i) {
    const bs::KernelEntry& e = t.entries[i];
    if (e.team == team && e.r == r && e.nz >= nz_min && (!best || e.nz < best->nz)) best = &e;
  }
  return best;
}

// Rows of 33..64 entries are solved by one-wave teams (one row per lane); such a
// pattern gets its bank-aware layout for the register-slot count the planner
// takes for it.
constexpr int kLayoutSteps = 20000;

void choose_layout(bs_pattern_s& p) {
  p.layout.clear();
  p.layout_nz = 0;
  if (p.n <= 32 || p.n > bs::kLayoutLanes) return;
  const bs::KernelEntry* k = find_kernel(bs::V_BICGSTAB, bs::kWave, 1, std::max(p.max_row, 1));
  if (!k || p.nnz < k->nz) return;
  const bs::WaveLayout L =
      bs::choose_wave_layout(p.n, p.nnz, p.row_ptr.data(), p.col.data(), k->nz, kLayoutSteps);
  if (L.cost >= L.plain_cost) return;
  p.layout.reserve(2 * bs::kLayoutLanes + p.n);
  p.layout.insert(p.layout.end(), L.lane_row.begin(), L.lane_row.end());
  p.layout.insert(p.layout.end(), L.lane_win.begin(), L.lane_win.end());
  p.layout.insert(p.layout.end(), L.col_pos.begin(), L.col_pos.end());
  p.layout_nz = k->nz;
}

// Compute units of the current device (cached per device).
int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1;
    cache[dev] = v;
  }
  return cache[dev];
}

bool pow2_team(int t) { return t >= 16 && t <= 1024 && (t & (t - 1)) == 0; }

// Block-Jacobi block size of a request: 0 without block Jacobi, else 2, 4 or
// 8 (0 selects 8); -1 when the size is not one of these.
int block_of(const bs_options* o, int precond = BS_PREC_BLOCK_JACOBI) {
  if (precond != BS_PREC_BLOCK_JACOBI) return 0;
  const int b = o ? o->block_size : 0;
  if (b == 0) return 8;
  return (b == 2 || b == 4 || b == 8) ? b : -1;
}

// Staging of CSR values through LDS is used while a workgroup's staging area
// stays within this budget.
constexpr int kStageBudget = 48 * 1024;
constexpr int kLdsPerCu = 160 * 1024;

struct Plan {
  bs_plan_info info;
  const bs::KernelEntry* k;
};

// block: block-Jacobi block size (0 without block Jacobi); ilu: ILU(0).
// ILU(0) and the triangular solves take one row per lane: a one-wave team up
// to 64 rows (dense factors), else the smallest power-of-two team of at least
// n lanes, up to 1024 (sparse factors, level-scheduled sweeps); a forced team
// must hold n rows and be at least a wave.
int make_plan(bs_format fmt, int n, int nnz, int max_row, int width, bs_solver solver,
              const bs_options* o, int block, bool ilu, Plan* out) {
  const int precision = o ? o->precision : BS_FP64;
  const int variant = variant_of(solver, precision, block, ilu);
  if (variant < 0) return BS_ERR_UNSUPPORTED;
  if (n > BS_MAX_ROWS || max_row > BS_MAX_ROW_NNZ) return BS_ERR_UNSUPPORTED;
  const bool trsv = solver == BS_TRSV_LOWER || solver == BS_TRSV_UPPER;
  const bool tri = ilu || trsv;
  if (tri && (n > 1024 || (o && ((o->team != 0 && (o->team < bs::kWave || o->team < n)) ||
                                 o->rows_per_lane > 1))))
    return BS_ERR_UNSUPPORTED;
  int tri_team = bs::kWave;
  while (tri_team < n) tri_team *= 2;
  // the multi-wave schedule and sweep lists address entries with 15 bits
  if (tri && n > bs::kWave && nnz >= (1 << 15)) return BS_ERR_UNSUPPORTED;
  const int force_team = tri ? (o && o->team ? o->team : tri_team) : o ? o->team : 0,
            force_r = o ? o->rows_per_lane : 0;
  if (force_team != 0 && !pow2_team(force_team)) return BS_ERR_INVALID_ARG;
  if (force_r != 0 && force_r != 1 && force_r != 2 && force_r != 4) return BS_ERR_INVALID_ARG;
  // Sec. 3.6: at least one lane per row, rounded up to a power of two no
  // smaller than the 16-lane DPP row; systems beyond one workgroup of lanes take
  // 2 or 4 rows per lane.  Shapes are tried from the fewest rows per lane and the
  // narrowest team upwards; the first compiled shape whose register slots cover
  // the longest row is taken.
  const bs::KernelEntry* k = nullptr;
  int team = 0, r = 0;
  for (int rr = 1; rr <= 4 && !k; rr *= 2) {
    if (force_r && rr != force_r) continue;
    int t = 16;
    while (t * rr < n && t < 1024) t *= 2;
    if (force_team) t = force_team;
    for (; t <= 1024 && !k; t *= 2) {
      if (t * rr < n) break;
      k = find_kernel(variant, t, rr, std::max(max_row, 1));
      team = t;
      r = rr;
      if (force_team) break;
    }
  }
  if (!k) return BS_ERR_UNSUPPORTED;
  const int rows = team * r;
  const int wg = k->wg, teams = wg / team, waves = wg / bs::kWave;
  const bool gm = variant == bs::V_GMRES || variant == bs::V_GMRES_MIXED ||
                  variant == bs::V_GMRES_BJ || variant == bs::V_GMRES_ILU;
  const int stored = fmt == BS_CSR ? nnz : width * n;
  const bool mixed = variant == bs::V_GMRES_MIXED;
  const int vec = teams * (bs::team_vec_bytes(rows, gm, wg, mixed) + bs::bj_bytes(rows, block) +
                           (tri ? bs::tri_region_bytes(team, n, nnz) : 0)) +
                  bs::red_lds_bytes(waves);
  int stage = 0;
  // ILU(0) and the triangular solves are bound by their substitution chains,
  // not by loading the values: their LDS goes to more resident waves instead
  // of staging
  if (waves == 1 && !tri && bs::stage_total_bytes(teams, stored, n, k->nz) <= kStageBudget)
    stage = 1;
  // Multi-wave teams, CSR, rows of many slots: each system's values copied
  // into LDS by the whole group (coalesced direct-to-LDS loads issued during
  // the previous system's solve), where they fit beside the vectors; the
  // launch keeps it only where it costs no resident group.
  if (waves > 1 && fmt == BS_CSR && !tri && k->nz >= bs::kStageMinSlots &&
      vec + bs::stage_vals_bytes(teams, stored, k->nz) <= kLdsPerCu)
    stage = 2;
  out->k = k;
  out->info.team = team;
  out->info.rows_per_lane = r;
  out->info.slots = k->nz;
  out->info.group_size = wg;
  out->info.systems_per_group = teams;
  out->info.lds_bytes = vec + (stage == 1   ? bs::stage_total_bytes(teams, stored, n, k->nz)
                               : stage == 2 ? bs::stage_vals_bytes(teams, stored, k->nz)
                                            : 0);
  out->info.stage_values = stage;
  // a workgroup's LDS is at most that of a compute unit
  if (out->info.lds_bytes > kLdsPerCu) return BS_ERR_UNSUPPORTED;
  return BS_OK;
}

__global__ void k_csr_to_ell(int64_t n_batch, int n, int nnz, int width, const int* row_ptr,
                             const int* row_len, const double* src, double* dst) {
  const int64_t per = (int64_t)width * n;
  const int64_t total = n_batch * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / per;
    const int rem = (int)(e - s * per);
    const int slot = rem / n, i = rem - slot * n;
    dst[e] = slot < row_len[i] ? src[s * nnz + row_ptr[i] + slot] : 0.0;
  }
}

}  // namespace

extern "C" {

const char* bs_error_string(int code) {
  switch (code) {
    case BS_OK: return "success";
    case BS_ERR_INVALID_ARG: return "invalid argument";
    case BS_ERR_PATTERN: return "malformed sparsity pattern";
    case BS_ERR_UNSUPPORTED: return "unsupported shape or option";
    case BS_ERR_HIP: return "HIP runtime error";
    case BS_ERR_NO_DEVICE: return "no HIP device";
    default: return "unknown error";
  }
}

const char* bs_last_error(void) { return g_last_error.c_str(); }

int bs_pattern_create_csr(int32_t n_rows, int32_t nnz, const int32_t* row_ptr,
                          const int32_t* col_idx, bs_pattern* out) {
  if (!out || !row_ptr || (nnz > 0 && !col_idx) || n_rows < 1 || nnz < 0)
    return BS_ERR_INVALID_ARG;
  *out = nullptr;
  if (row_ptr[0] != 0 || row_ptr[n_rows] != nnz) return BS_ERR_PATTERN;
  for (int i = 0; i < n_rows; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return BS_ERR_PATTERN;
  std::vector<int> mark(n_rows, -1);
  for (int i = 0; i < n_rows; ++i)
    if (!row_ok(col_idx + row_ptr[i], row_ptr[i + 1] - row_ptr[i], n_rows, mark, i))
      return BS_ERR_PATTERN;
  bs_pattern_s* p = new bs_pattern_s();
  p->n = n_rows;
  p->nnz = nnz;
  p->row_ptr.assign(row_ptr, row_ptr + n_rows + 1);
  p->col.assign(col_idx, col_idx + nnz);
  derive(*p);
  choose_layout(*p);
  const int rc = upload(*p);
  if (rc != BS_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return BS_OK;
}

int bs_pattern_create_dense(int32_t n_rows, bs_pattern* out) {
  if (!out || n_rows < 1 || n_rows > 46340) return BS_ERR_INVALID_ARG;
  *out = nullptr;
  const int n = n_rows;
  std::vector<int32_t> rp(n + 1), col((size_t)n * n);
  for (int i = 0; i <= n; ++i) rp[i] = i * n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) col[(size_t)i * n + j] = j;
  return bs_pattern_create_csr(n, n * n, rp.data(), col.data(), out);
}

int bs_pattern_create_ell(int32_t n_rows, int32_t ell_width, const int32_t* ell_col,
                          bs_pattern* out) {
  if (!out || n_rows < 1 || ell_width < 0 || (ell_width > 0 && !ell_col))
    return BS_ERR_INVALID_ARG;
  *out = nullptr;
  std::vector<int> rp(n_rows + 1, 0), col;
  for (int i = 0; i < n_rows; ++i) {
    int len = 0;
    bool pad = false;
    for (int s = 0; s < ell_width; ++s) {
      const int c = ell_col[(size_t)s * n_rows + i];
      if (c == -1) {
        pad = true;
      } else {
        if (pad || c < -1 || c >= n_rows) return BS_ERR_PATTERN;
        ++len;
      }
    }
    rp[i + 1] = rp[i] + len;
  }
  col.resize(rp[n_rows]);
  for (int i = 0; i < n_rows; ++i)
    for (int s = 0; s < rp[i + 1] - rp[i]; ++s) col[rp[i] + s] = ell_col[(size_t)s * n_rows + i];
  std::vector<int> mark(n_rows, -1);
  for (int i = 0; i < n_rows; ++i)
    if (!row_ok(col.data() + rp[i], rp[i + 1] - rp[i], n_rows, mark, i)) return BS_ERR_PATTERN;
  bs_pattern_s* p = new bs_pattern_s();
  p->n = n_rows;
  p->nnz = rp[n_rows];
  p->row_ptr = std::move(rp);
  p->col = std::move(col);
  derive(*p);
  // Keep the caller's width (it may include all-padding slots).
  if (ell_width > p->width) {
    p->slot_col.resize((size_t)ell_width * n_rows, -1);
    p->width = ell_width;
  }
  choose_layout(*p);
  const int rc = upload(*p);
  if (rc != BS_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return BS_OK;
}

int bs_pattern_destroy(bs_pattern p) {
  if (!p) return BS_OK;
  if (p->d_base) (void)hipFree(p->d_base);
  delete p;
  return BS_OK;
}

int bs_wave_layout(int32_t n_rows, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                   int32_t slots, int32_t steps, int32_t* lane_row, int32_t* lane_win,
                   int32_t* col_pos, int64_t* cost) {
  if (!row_ptr || (nnz > 0 && !col_idx) || !lane_row || !lane_win || !col_pos || !cost ||
      n_rows < 1 || nnz < 0 || slots < 1 || steps < 0)
    return BS_ERR_INVALID_ARG;
  if (row_ptr[0] != 0 || row_ptr[n_rows] != nnz) return BS_ERR_PATTERN;
  int max_row = 0;
  for (int i = 0; i < n_rows; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return BS_ERR_PATTERN;
    max_row = std::max(max_row, row_ptr[i + 1] - row_ptr[i]);
  }
  std::vector<int> mark(n_rows, -1);
  for (int i = 0; i < n_rows; ++i)
    if (!row_ok(col_idx + row_ptr[i], row_ptr[i + 1] - row_ptr[i], n_rows, mark, i))
      return BS_ERR_PATTERN;
  if (n_rows <= 32 || n_rows > bs::kLayoutLanes || nnz < slots || max_row > slots)
    return BS_ERR_UNSUPPORTED;
  const bs::WaveLayout L = bs::choose_wave_layout(n_rows, nnz, row_ptr, col_idx, slots, steps);
  std::copy(L.lane_row.begin(), L.lane_row.end(), lane_row);
  std::copy(L.lane_win.begin(), L.lane_win.end(), lane_win);
  std::copy(L.col_pos.begin(), L.col_pos.end(), col_pos);
  cost[0] = L.cost;
  cost[1] = L.plain_cost;
  return BS_OK;
}

int bs_pattern_layout(bs_pattern p, int32_t* slots, int32_t* layout) {
  if (!p || !slots) return BS_ERR_INVALID_ARG;
  *slots = p->layout_nz;
  if (layout) std::copy(p->layout.begin(), p->layout.end(), layout);
  return BS_OK;
}

int bs_pattern_query(bs_pattern p, int32_t* n_rows, int32_t* nnz, int32_t* ell_width,
                     int32_t* max_row_nnz) {
  if (!p) return BS_ERR_INVALID_ARG;
  if (n_rows) *n_rows = p->n;
  if (nnz) *nnz = p->nnz;
  if (ell_width) *ell_width = p->width;
  if (max_row_nnz) *max_row_nnz = p->max_row;
  return BS_OK;
}

int bs_pattern_ell_cols(bs_pattern p, int32_t* out) {
  if (!p || (!out && p->width > 0)) return BS_ERR_INVALID_ARG;
  std::copy(p->slot_col.begin(), p->slot_col.end(), out);
  return BS_OK;
}

int bs_values_csr_to_ell(bs_pattern p, int64_t n_batch, const double* csr, double* ell,
                         void* stream) {
  if (!p || n_batch < 0) return BS_ERR_INVALID_ARG;
  if (n_batch == 0 || p->width == 0) return BS_OK;
  if (!csr || !ell) return BS_ERR_INVALID_ARG;
  const int64_t total = n_batch * (int64_t)p->width * p->n;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_csr_to_ell, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     n_batch, p->n, p->nnz, p->width, p->d_row_ptr, p->d_row_len, csr, ell);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BS_OK : hip_fail(e, "k_csr_to_ell");
}

int bs_matrix_storage(bs_format fmt, int64_t n_batch, int32_t n_rows, int32_t nnz,
                      int32_t ell_width, int64_t* value_count, int64_t* index_count) {
  if (n_batch < 0 || n_rows < 1 || nnz < 0 || ell_width < 0 || !value_count || !index_count)
    return BS_ERR_INVALID_ARG;
  if (fmt == BS_CSR) {
    *value_count = n_batch * (int64_t)nnz;
    *index_count = (int64_t)n_rows + 1 + nnz;
  } else if (fmt == BS_DENSE) {
    *value_count = n_batch * (int64_t)n_rows * n_rows;
    *index_count = 0;
  } else if (fmt == BS_ELL) {
    *value_count = n_batch * (int64_t)ell_width * n_rows;
    *index_count = (int64_t)ell_width * n_rows;
  } else {
    return BS_ERR_INVALID_ARG;
  }
  return BS_OK;
}

int bs_plan(bs_format fmt, int32_t n_rows, int32_t nnz, int32_t max_row_nnz, bs_solver solver,
            const bs_options* opts, bs_plan_info* out) {
  if (!out || n_rows < 1 || nnz < 0 || max_row_nnz < 0 ||
      (fmt != BS_CSR && fmt != BS_ELL && fmt != BS_DENSE) ||
      (solver < BS_CG || solver > BS_TRSV_UPPER))
    return BS_ERR_INVALID_ARG;
  if (fmt == BS_DENSE) {  // the full pattern in CSR order
    nnz = n_rows * n_rows;
    max_row_nnz = n_rows;
    fmt = BS_CSR;
  }
  Plan pl;
  // planned with the block-Jacobi region when opts asks for a block size
  const int block = opts && opts->block_size != 0 ? block_of(opts) : 0;
  if (block < 0) return BS_ERR_INVALID_ARG;
  const int rc =
      make_plan(fmt, n_rows, nnz, max_row_nnz, max_row_nnz, solver, opts, block, false, &pl);
  if (rc == BS_OK) *out = pl.info;
  // no register shape: the streamed placement, where the request allows it
  if (rc == BS_ERR_UNSUPPORTED && block <= 1)
    return bs::stream_plan(n_rows, solver, BS_PREC_JACOBI, opts, out);
  return rc;
}

int bs_plan_precond(bs_format fmt, int32_t n_rows, int32_t nnz, int32_t max_row_nnz,
                    bs_solver solver, bs_precond precond, const bs_options* opts,
                    bs_plan_info* out) {
  if (!out || n_rows < 1 || nnz < 0 || max_row_nnz < 0 ||
      (fmt != BS_CSR && fmt != BS_ELL && fmt != BS_DENSE) ||
      (solver < BS_CG || solver > BS_TRSV_UPPER) ||
      (precond != BS_PREC_NONE && precond != BS_PREC_JACOBI && precond != BS_PREC_BLOCK_JACOBI &&
       precond != BS_PREC_ILU))
    return BS_ERR_INVALID_ARG;
  if (fmt == BS_DENSE) {
    nnz = n_rows * n_rows;
    max_row_nnz = n_rows;
    fmt = BS_CSR;
  }
  const int block = block_of(opts, precond);
  if (block < 0) return BS_ERR_INVALID_ARG;
  Plan pl;
  const int rc = make_plan(fmt, n_rows, nnz, max_row_nnz, max_row_nnz, solver, opts, block,
                           precond == BS_PREC_ILU, &pl);
  if (rc == BS_OK) *out = pl.info;
  if (rc == BS_ERR_UNSUPPORTED) return bs::stream_plan(n_rows, solver, precond, opts, out);
  return rc;
}

size_t bs_workspace_size(bs_format fmt, int64_t n_batch, int32_t n_rows, bs_pattern pattern,
                         bs_solver solver, const bs_options* opts) {
  (void)fmt;
  (void)n_batch;
  (void)n_rows;
  (void)pattern;
  (void)solver;
  (void)opts;
  return 0;
}

int bs_batch_solve(bs_format fmt, int64_t n_batch, int32_t n_rows, bs_pattern pattern,
                   const double* values, const double* b, double* x, bs_solver solver,
                   bs_precond precond, double tol, int32_t max_iter, int32_t* iters,
                   double* resid, int32_t* status, const bs_options* opts, void* stream) {
  if (!pattern || n_batch < 0 || n_rows != pattern->n) return BS_ERR_INVALID_ARG;
  if (fmt != BS_CSR && fmt != BS_ELL && fmt != BS_DENSE) return BS_ERR_INVALID_ARG;
  // BatchDense: row-major [n][n] values are the CSR values of the full pattern
  if (fmt == BS_DENSE) {
    if ((int64_t)pattern->nnz != (int64_t)pattern->n * pattern->n) return BS_ERR_PATTERN;
    fmt = BS_CSR;
  }
  if (solver < BS_CG || solver > BS_TRSV_UPPER) return BS_ERR_INVALID_ARG;
  if (precond != BS_PREC_NONE && precond != BS_PREC_JACOBI && precond != BS_PREC_BLOCK_JACOBI &&
      precond != BS_PREC_ILU)
    return BS_ERR_INVALID_ARG;
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 0) return BS_ERR_INVALID_ARG;
  // the triangular solves take no preconditioner
  const bool trsv = solver == BS_TRSV_LOWER || solver == BS_TRSV_UPPER;
  const bool ilu = precond == BS_PREC_ILU && !trsv;
  const int block = trsv ? 0 : block_of(opts, precond);
  if (block < 0) return BS_ERR_INVALID_ARG;
  int restart = bs::kMaxRestart;
  double inner_tol = 1e-6;
  int flags = 0;
  if (opts) {
    if (opts->restart < 0 || opts->restart > bs::kMaxRestart) return BS_ERR_INVALID_ARG;
    if (opts->restart > 0) restart = opts->restart;
    if (opts->precision != BS_FP64 && opts->precision != BS_MIXED) return BS_ERR_INVALID_ARG;
    if (opts->inner_tol < 0.0 || !std::isfinite(opts->inner_tol)) return BS_ERR_INVALID_ARG;
    if (opts->inner_tol > 0.0) inner_tol = opts->inner_tol;
    flags = opts->flags;
  }
  // several right-hand sides per matrix: one solve per (matrix, right-hand side)
  const int nrhs = opts && opts->n_rhs > 0 ? opts->n_rhs : 1;
  if (opts && opts->n_rhs < 0) return BS_ERR_INVALID_ARG;
  if (n_batch > INT64_MAX / nrhs) return BS_ERR_INVALID_ARG;
  const int64_t n_solves = n_batch * nrhs;
  if (n_batch == 0) return BS_OK;
  if (!values || !b || !x || !iters || !resid) return BS_ERR_INVALID_ARG;
  Plan pl;
  int rc = make_plan(fmt, pattern->n, pattern->nnz, pattern->max_row, pattern->width, solver,
                     opts, block, ilu, &pl);
  // no register shape holds the rows: the streamed placement, if it applies
  bool streamed = false;
  if (rc == BS_ERR_UNSUPPORTED && !trsv) {
    rc = bs::stream_plan(pattern->n, solver, precond, opts, &pl.info);
    streamed = rc == BS_OK;
  }
  if (rc != BS_OK) return rc;
  // multi-wave ILU(0) and BatchTrsv need the pattern's sweep lists
  if (!streamed && (ilu || trsv) && pl.info.team > bs::kWave && pattern->sweep.empty())
    return BS_ERR_UNSUPPORTED;
  bs::KArgs a{};
  a.n_batch = n_solves;
  a.nrhs = nrhs;
  a.n = pattern->n;
  a.nnz = pattern->nnz;
  a.width = pattern->width;
  a.fmt = fmt == BS_CSR ? 0 : 1;
  a.precond = precond == BS_PREC_JACOBI ? 1 : 0;
  a.flags = flags;
  a.max_iter = max_iter;
  a.restart = restart;
  a.stage = pl.info.stage_values;
  a.gmres = solver == BS_GMRES ? 1 : 0;
  if (!streamed) {
    const int rows = pl.info.team * pl.info.rows_per_lane;
    const int teams = pl.info.systems_per_group, waves = pl.info.group_size / bs::kWave;
    const int stored = fmt == BS_CSR ? pattern->nnz : pattern->width * pattern->n;
    a.team_bytes = bs::team_vec_bytes(rows, a.gmres, pl.info.group_size,
                                      a.gmres && opts && opts->precision == BS_MIXED);
    // block Jacobi (inverse and exchange buffer) or ILU(0) (factors) after the
    // vectors
    a.block = block;
    a.bj_offset = a.team_bytes;
    a.team_bytes += bs::bj_bytes(rows, block) +
                    (ilu || trsv ? bs::tri_region_bytes(pl.info.team, pattern->n, pattern->nnz)
                                 : 0);
    a.stage_vals_bytes = bs::stage_vals_bytes(teams, stored, pl.info.slots);
    a.stage_team_bytes = a.stage_vals_bytes + bs::stage_b_bytes(teams, pattern->n);
    a.stage_offset = teams * a.team_bytes + bs::red_lds_bytes(waves);
    // CSR rows go through a fixed window when the block holds a full window
    a.window = (fmt == BS_CSR && pattern->nnz >= pl.info.slots) ? 1 : 0;
  }
  a.tol = tol;
  a.inner_tol = inner_tol;
  a.row_ptr = pattern->d_row_ptr;
  a.slot_col = pattern->d_slot_col;
  a.row_len = pattern->d_row_len;
  a.diag_slot = pattern->d_diag;
  a.lev = pattern->d_lev;
  a.nlev_l = pattern->nlev_l;
  a.nlev_u = pattern->nlev_u;
  a.ilu_ptr = pattern->d_ilu_ptr;
  a.ilu_ops = pattern->d_ilu_ops;
  a.sweep = pattern->d_sweep;
  a.sweep_ents = pattern->sweep_ents;
  a.values = values;
  a.b = b;
  a.x = x;
  a.iters = iters;
  a.resid = resid;
  a.status = status;
  a.outer = opts ? opts->outer_iters : nullptr;
  a.sink = bs::device_sink();
  if (!a.sink) return BS_ERR_HIP;
  a.x_alt = opts ? opts->x_alt : nullptr;
  a.alt_used = opts ? opts->alt_used : nullptr;
  if (a.x_alt && (flags & BS_FLAG_X0_ZERO)) return BS_ERR_INVALID_ARG;
  if (streamed) {
    a.layout = nullptr;
    a.block = 0;
    const int cus = device_cus();
    if (cus < 1) return BS_ERR_HIP;
    const int mixed = opts && opts->precision == BS_MIXED;
    const int src = bs::stream_launch(a, pl.info, solver, mixed, cus, (hipStream_t)stream);
    return src == BS_OK ? BS_OK : hip_fail(hipGetLastError(), "streamed solver launch");
  }
  a.layout = (pattern->d_layout && pl.info.team == bs::kWave && pl.info.rows_per_lane == 1 &&
              a.window && pl.k->nz == pattern->layout_nz && !(flags & BS_FLAG_PLAIN_LAYOUT) &&
              a.block <= 1 && !ilu && !trsv)  // these need row i on lane i
                 ? pattern->d_layout
                 : nullptr;
  // Persistent grid: as many workgroups as can be resident at once, each
  // walking over the batch (never more than there are systems).
  const int64_t groups = (n_solves + pl.info.systems_per_group - 1) / pl.info.systems_per_group;
  const int cus = device_cus();
  if (cus < 1) return BS_ERR_HIP;
  // Resident groups per CU, asked with 1 KiB more LDS per group than used: a
  // group count that would fill the CU's LDS to the last granule is not always
  // placed at once, and a group left over runs only after another one ends.
  int lds = pl.info.lds_bytes;
  // the group-wide copy lands in whole KiB behind the vectors: inside the launch's LDS
  if (a.stage == 2 && (a.stage_vals_bytes % 1024 != 0 || a.stage_offset + a.stage_vals_bytes > lds))
    return BS_ERR_UNSUPPORTED;
  if (a.stage == 2) {  // the group-wide copy of the values only where no group is lost to it
    const int without = lds - a.stage_vals_bytes;
    if (pl.k->occupancy((unsigned)lds + 1024) < pl.k->occupancy((unsigned)without + 1024)) {
      a.stage = 0;
      lds = without;
    }
  }
  const int64_t resident = (int64_t)pl.k->occupancy((unsigned)lds + 1024) * cus;
  const int64_t grid = std::min(groups, resident);
  const hipError_t e = pl.k->launch(a, (unsigned)grid, (unsigned)lds, (hipStream_t)stream);
  return e == hipSuccess ? BS_OK : hip_fail(e, "solver launch");
}

}  // extern "C"

namespace {
// Patterns of bs_batch_solve_dev, keyed by what identifies the caller's arrays.
struct DevPatKey {
  int device, fmt, n, nnz, width;
  const void* rp;
  const void* ci;
  int32_t generation;
  bool operator==(const DevPatKey& o) const {
    return device == o.device && fmt == o.fmt && n == o.n && nnz == o.nnz && width == o.width &&
           rp == o.rp && ci == o.ci && generation == o.generation;
  }
};
struct DevPatEntry {
  DevPatKey key;
  bs_pattern pattern = nullptr;
  uint64_t used = 0;
};
std::mutex g_dp_mu;
std::vector<DevPatEntry> g_dp_cache;
uint64_t g_dp_clock = 0;
constexpr size_t kDevPatEntries = 8;

int read_ints(std::vector<int32_t>& dst, const int32_t* src, int64_t count, hipStream_t st) {
  dst.resize((size_t)std::max<int64_t>(count, 0));
  if (count <= 0) return BS_OK;
  hipError_t e = hipMemcpyAsync(dst.data(), src, (size_t)count * sizeof(int32_t),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? BS_OK : hip_fail(e, "read pattern arrays");
}
}  // namespace

extern "C" {

int bs_batch_solve_dev(bs_format fmt, int64_t n_batch, int32_t n_rows,
                       const bs_pattern_dev* pattern, const double* values, const double* b,
                       double* x, bs_solver solver, bs_precond precond, double tol,
                       int32_t max_iter, int32_t* iters, double* resid, int32_t* status,
                       const bs_options* opts, void* workspace, size_t workspace_bytes,
                       void* stream) {
  (void)workspace;  // the solve needs none (bs_workspace_size returns 0)
  (void)workspace_bytes;
  if (n_batch < 0 || n_rows < 1) return BS_ERR_INVALID_ARG;
  if (fmt != BS_CSR && fmt != BS_ELL && fmt != BS_DENSE) return BS_ERR_INVALID_ARG;
  DevPatKey key{};
  key.fmt = fmt;
  key.n = n_rows;
  key.generation = opts ? opts->structure_generation : 0;
  if (fmt != BS_DENSE) {
    if (!pattern) return BS_ERR_INVALID_ARG;
    if (fmt == BS_CSR && (!pattern->row_ptr || pattern->nnz < 0 || (pattern->nnz > 0 && !pattern->col_idx)))
      return BS_ERR_INVALID_ARG;
    if (fmt == BS_ELL && (pattern->ell_width < 0 ||
                          (int64_t)pattern->nnz != (int64_t)pattern->ell_width * n_rows ||
                          (pattern->ell_width > 0 && !pattern->col_idx)))
      return BS_ERR_INVALID_ARG;
    key.nnz = pattern->nnz;
    key.width = fmt == BS_ELL ? pattern->ell_width : 0;
    key.rp = fmt == BS_CSR ? pattern->row_ptr : nullptr;
    key.ci = pattern->col_idx;
  }
  if (n_batch == 0) return BS_OK;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    g_last_error = "no HIP device";
    return BS_ERR_NO_DEVICE;
  }
  hipError_t e = hipGetDevice(&key.device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_dp_mu);
  DevPatEntry* ent = nullptr;
  for (DevPatEntry& d : g_dp_cache)
    if (d.key == key) ent = &d;
  if (!ent) {
    bs_pattern p = nullptr;
    int rc = BS_OK;
    if (fmt == BS_DENSE) {
      rc = bs_pattern_create_dense(n_rows, &p);
    } else if (fmt == BS_CSR) {
      std::vector<int32_t> rp, ci;
      rc = read_ints(rp, pattern->row_ptr, (int64_t)n_rows + 1, st);
      if (rc == BS_OK) rc = read_ints(ci, pattern->col_idx, pattern->nnz, st);
      if (rc == BS_OK) rc = bs_pattern_create_csr(n_rows, pattern->nnz, rp.data(), ci.data(), &p);
    } else {
      std::vector<int32_t> ci;
      rc = read_ints(ci, pattern->col_idx, (int64_t)pattern->ell_width * n_rows, st);
      if (rc == BS_OK) rc = bs_pattern_create_ell(n_rows, pattern->ell_width, ci.data(), &p);
    }
    if (rc != BS_OK) return rc;
    if (g_dp_cache.size() >= kDevPatEntries) {  // drop the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < g_dp_cache.size(); ++i)
        if (g_dp_cache[i].used < g_dp_cache[lru].used) lru = i;
      (void)bs_pattern_destroy(g_dp_cache[lru].pattern);
      g_dp_cache.erase(g_dp_cache.begin() + (long)lru);
    }
    DevPatEntry fresh;
    fresh.key = key;
    fresh.pattern = p;
    g_dp_cache.push_back(fresh);
    ent = &g_dp_cache.back();
  }
  ent->used = ++g_dp_clock;
  return bs_batch_solve(fmt, n_batch, n_rows, ent->pattern, values, b, x, solver, precond, tol,
                        max_iter, iters, resid, status, opts, stream);
}

}  // extern "C"
