// Host side of the uneven-batch entry points (bs_varbatch_*): validation and
// derivation of every distinct pattern, the task queue (size classes, largest
// first), the persistent launch, the autotuner over queue policies, and the
// captured HIP graph (counter reset + solve).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/batchsolve.h"
#include "bs_varlen.hpp"

namespace bs {
void set_last_error(const std::string& msg);
int* device_sink();
}

namespace {

int hip_err(hipError_t e, const char* what) {
  bs::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
  return BS_ERR_HIP;
}

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

typedef hipError_t (*VLaunch)(const bs::VArgs&, unsigned grid, hipStream_t);
typedef hipError_t (*VOccupancy)(int*);

template <class VS, int NZ, int SOLVER, bool MIXED, bool BJ>
hipError_t vlaunch(const bs::VArgs& a, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((bs::k_varlen<VS, NZ, SOLVER, MIXED, BJ>), dim3(grid), dim3(VS::WG), 0, s, a);
  return hipGetLastError();
}

template <class VS, int NZ, int SOLVER, bool MIXED, bool BJ>
hipError_t voccupancy(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks, reinterpret_cast<const void*>(&bs::k_varlen<VS, NZ, SOLVER, MIXED, BJ>), VS::WG, 0);
}

// Workgroup shapes (lanes, rows per lane); each holds systems of up to 1024 rows.
struct VShapeInfo {
  int wg, r;
};
constexpr VShapeInfo kVShapes[] = {{1024, 1}, {512, 2}, {256, 4}};
constexpr int kNumShapes = 3;
constexpr int kNumOrders = 3;
constexpr int kNumPolicies = kNumShapes * kNumOrders;
constexpr int kMaxVarRows = 1024;

// Compiled instances: shape x slots per row x (CG, BiCGSTAB, BiCGSTAB mixed,
// and CG and BiCGSTAB with block Jacobi).
struct VEntry {
  int wg, r, nz, solver, mixed, bj;
  VLaunch fn;
  VOccupancy occ;
};
#define VE1(W, R, NZ, SO, MX, BJ)                                                     \
  {W, R, NZ, SO, MX, BJ, &vlaunch<bs::VarShape<W, R>, NZ, SO, MX, BJ>,                 \
   &voccupancy<bs::VarShape<W, R>, NZ, SO, MX, BJ>},
#define VE(W, R, NZ)                                                                  \
  VE1(W, R, NZ, 0, false, false) VE1(W, R, NZ, 1, false, false) VE1(W, R, NZ, 1, true, false) \
  VE1(W, R, NZ, 0, false, true) VE1(W, R, NZ, 1, false, true)
#define VES(W, R) VE(W, R, 8) VE(W, R, 10) VE(W, R, 12) VE(W, R, 16)
const VEntry kVTable[] = {VES(1024, 1) VES(512, 2) VES(256, 4)};
#undef VES
#undef VE
#undef VE1

const VEntry* find_v(int wg, int r, int nz, int solver, int mixed, int bj) {
  const VEntry* best = nullptr;
  for (const VEntry& e : kVTable)
    if (e.wg == wg && e.r == r && e.solver == solver && e.mixed == mixed && e.bj == bj &&
        e.nz >= nz && (!best || e.nz < best->nz))
      best = &e;
  return best;
}

}  // namespace

struct bs_varbatch_s {
  int64_t B = 0;
  int P = 0, max_row = 0, device = -1, policy = 0;
  int policy_next = 0;  // policy of the tasks being uploaded
  std::vector<int> sys_rows, sys_pat, pat_n, pat_nnz;
  std::vector<int64_t> row_off, val_off, pat_rp, pat_row, pat_sc;
  std::vector<int> prow_ptr, prow_len, pdiag, pslot_col;
  std::vector<bs::VTask> tasks;
  std::vector<int> order;
  // device
  char* d_static = nullptr;  // everything that does not depend on the policy
  bs::VTask* d_tasks = nullptr;
  int* d_order = nullptr;
  int* d_counter = nullptr;
  bs::VArgs args{};
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
};

namespace {

// Tasks for a policy (see bs_varbatch_set_policy): workgroup shape
// policy / 3, queue order policy % 3.
void build_tasks(bs_varbatch_s& v, int policy) {
  const VShapeInfo sh = kVShapes[policy / kNumOrders];
  const int order = policy % kNumOrders;
  std::vector<int> team(v.B);
  for (int64_t s = 0; s < v.B; ++s) {
    int t = std::max(bs::kWave, next_pow2((v.sys_rows[s] + sh.r - 1) / sh.r));
    if (order == 1) t = std::min(sh.wg, 2 * t);
    team[s] = t;
  }
  std::vector<int> idx(v.B);
  for (int64_t s = 0; s < v.B; ++s) idx[s] = (int)s;
  // group by team size (largest first); inside a class, largest systems first
  // (similar sizes share a task) unless the order keeps the batch order
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (team[a] != team[b]) return team[a] > team[b];
    if (order == 2) return false;
    return v.val_off[a + 1] - v.val_off[a] > v.val_off[b + 1] - v.val_off[b];
  });
  v.order = idx;
  v.tasks.clear();
  for (int64_t i = 0; i < v.B;) {
    const int t = team[idx[i]], cap = sh.wg / t;
    int c = 0;
    while (i + c < v.B && c < cap && team[idx[i + c]] == t) ++c;
    v.tasks.push_back({t, (int)i, c, 0});
    i += c;
  }
}

int upload_tasks(bs_varbatch_s& v) {
  // what the kernel assumes of every task: a power-of-two team of at least a
  // wave that holds each of its systems, and teams that fit one workgroup
  const VShapeInfo sh = kVShapes[v.policy_next / kNumOrders];
  int64_t covered = 0;
  for (const bs::VTask& t : v.tasks) {
    if (t.team < bs::kWave || t.team > sh.wg || (t.team & (t.team - 1)) || t.count < 1 ||
        (int64_t)t.count * t.team > sh.wg || t.first != covered)
      return BS_ERR_INVALID_ARG;
    for (int i = 0; i < t.count; ++i)
      if (v.sys_rows[v.order[t.first + i]] > t.team * sh.r) return BS_ERR_INVALID_ARG;
    covered += t.count;
  }
  if (covered != v.B) return BS_ERR_INVALID_ARG;
  hipError_t e = hipMemcpy(v.d_tasks, v.tasks.data(), v.tasks.size() * sizeof(bs::VTask),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(e, "upload tasks");
  e = hipMemcpy(v.d_order, v.order.data(), v.order.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(e, "upload order");
  v.args.n_tasks = (int64_t)v.tasks.size();
  return BS_OK;
}

int launch(bs_varbatch_s& v, const double* values, const double* b, double* x, bs_solver solver,
           bs_precond precond, double tol, int max_iter, int* iters, double* resid, int* status,
           const bs_options* o, hipStream_t stream) {
  if (solver != BS_CG && solver != BS_BICGSTAB) return BS_ERR_UNSUPPORTED;
  if (precond == BS_PREC_ILU) return BS_ERR_UNSUPPORTED;  // factors of up to 1024 rows
  if (o && o->n_rhs > 1) return BS_ERR_UNSUPPORTED;        // one right-hand side per system
  if (precond != BS_PREC_NONE && precond != BS_PREC_JACOBI && precond != BS_PREC_BLOCK_JACOBI)
    return BS_ERR_INVALID_ARG;
  int block = 0;
  if (precond == BS_PREC_BLOCK_JACOBI) {
    block = o && o->block_size ? o->block_size : 8;
    if (block != 2 && block != 4 && block != 8) return BS_ERR_INVALID_ARG;
  }
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 0) return BS_ERR_INVALID_ARG;
  const int mixed = o && o->precision == BS_MIXED;
  if (o && o->precision != BS_FP64 && o->precision != BS_MIXED) return BS_ERR_INVALID_ARG;
  if (mixed && solver != BS_BICGSTAB) return BS_ERR_UNSUPPORTED;
  if (o && (o->inner_tol < 0.0 || !std::isfinite(o->inner_tol))) return BS_ERR_INVALID_ARG;
  if (v.B == 0) return BS_OK;
  if (!values || !b || !x || !iters || !resid) return BS_ERR_INVALID_ARG;
  const VShapeInfo sh = kVShapes[v.policy / kNumOrders];
  if (mixed && block > 1) return BS_ERR_UNSUPPORTED;
  const VEntry* k = find_v(sh.wg, sh.r, std::max(v.max_row, 1), solver == BS_CG ? 0 : 1, mixed,
                           block > 1 ? 1 : 0);
  if (!k) return BS_ERR_UNSUPPORTED;
  bs::VArgs a = v.args;
  bs::KArgs& g = a.base;
  g = bs::KArgs{};
  g.nrhs = 1;
  g.n_batch = v.B;
  g.precond = precond == BS_PREC_JACOBI ? 1 : 0;
  g.block = block;
  g.bj_offset = 0;  // the uneven kernel's block-Jacobi region is static
  g.flags = o ? o->flags : 0;
  g.max_iter = max_iter;
  g.restart = bs::kMaxRestart;
  g.tol = tol;
  g.inner_tol = (o && o->inner_tol > 0.0) ? o->inner_tol : 1e-6;
  g.values = values;
  g.b = b;
  g.x = x;
  g.iters = iters;
  g.resid = resid;
  g.status = status;
  g.outer = o ? o->outer_iters : nullptr;
  g.sink = bs::device_sink();
  if (!g.sink) return BS_ERR_HIP;
  g.x_alt = o ? o->x_alt : nullptr;
  g.alt_used = o ? o->alt_used : nullptr;
  if (g.x_alt && (g.flags & BS_FLAG_X0_ZERO)) return BS_ERR_INVALID_ARG;
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, v.device);
  if (e != hipSuccess) return hip_err(e, "device attribute");
  hipLaunchKernelGGL(bs::k_varlen_reset, dim3(1), dim3(1), 0, stream, v.d_counter);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "counter reset");
  int per_cu = 0;
  e = k->occ(&per_cu);
  if (e != hipSuccess) return hip_err(e, "occupancy");
  const int64_t resident = (int64_t)cus * std::max(per_cu, 1);
  const unsigned grid = (unsigned)std::min<int64_t>(resident, (int64_t)v.tasks.size());
  e = k->fn(a, grid, stream);
  return e == hipSuccess ? BS_OK : hip_err(e, "uneven-batch launch");
}

bool row_ok(const int* cols, int len, int n, std::vector<int>& mark, int stamp) {
  for (int k = 0; k < len; ++k) {
    const int c = cols[k];
    if (c < 0 || c >= n || mark[c] == stamp) return false;
    mark[c] = stamp;
  }
  return true;
}

std::string tune_key(const bs_varbatch_s& v, bs_solver solver, int mixed) {
  // histogram of team classes and the longest row
  int hist[16] = {0};
  for (int64_t s = 0; s < v.B; ++s) {
    int c = 0, t = std::max(bs::kWave, next_pow2(v.sys_rows[s]));
    while ((bs::kWave << c) < t) ++c;
    hist[c]++;
  }
  std::string k = "varbatch";
  for (int c = 0; c < 5; ++c) k += "_" + std::to_string(hist[c]);
  k += "_w" + std::to_string(v.max_row) + "_s" + std::to_string((int)solver) + "_m" +
       std::to_string(mixed);
  return k;
}

}  // namespace

extern "C" {

int bs_varbatch_create(int64_t n_batch, int32_t n_patterns, const int32_t* pat_rows,
                       const int64_t* pat_rowptr_off, const int32_t* rowptr_all,
                       const int64_t* pat_col_off, const int32_t* col_all, const int32_t* sys_pat,
                       bs_varbatch* out) {
  if (!out || n_batch < 0 || n_patterns < 0 || (n_patterns > 0 && (!pat_rows || !pat_rowptr_off ||
      !rowptr_all || !pat_col_off || !col_all)) || (n_batch > 0 && !sys_pat))
    return BS_ERR_INVALID_ARG;
  if (n_batch > 0x7fffffff) return BS_ERR_UNSUPPORTED;
  *out = nullptr;
  bs_varbatch_s* v = new bs_varbatch_s();
  v->B = n_batch;
  v->P = n_patterns;
  v->pat_n.resize(n_patterns);
  v->pat_nnz.resize(n_patterns);
  v->pat_rp.resize(n_patterns);
  v->pat_row.resize(n_patterns);
  v->pat_sc.resize(n_patterns);
  std::vector<int> mark;
  int rc = BS_OK;
  for (int p = 0; p < n_patterns && rc == BS_OK; ++p) {
    const int n = pat_rows[p];
    if (n < 1) { rc = BS_ERR_INVALID_ARG; break; }
    if (n > kMaxVarRows) { rc = BS_ERR_UNSUPPORTED; break; }
    const int32_t* rp = rowptr_all + pat_rowptr_off[p];
    const int32_t* ci = col_all + pat_col_off[p];
    if (rp[0] != 0) { rc = BS_ERR_PATTERN; break; }
    int maxr = 0;
    for (int i = 0; i < n; ++i) {
      if (rp[i + 1] < rp[i]) { rc = BS_ERR_PATTERN; break; }
      maxr = std::max(maxr, rp[i + 1] - rp[i]);
    }
    if (rc != BS_OK) break;
    if (maxr > 16) { rc = BS_ERR_UNSUPPORTED; break; }
    mark.assign(n, -1);
    for (int i = 0; i < n && rc == BS_OK; ++i)
      if (!row_ok(ci + rp[i], rp[i + 1] - rp[i], n, mark, i)) rc = BS_ERR_PATTERN;
    if (rc != BS_OK) break;
    v->max_row = std::max(v->max_row, maxr);
    v->pat_n[p] = n;
    v->pat_nnz[p] = rp[n];
    v->pat_rp[p] = (int64_t)v->prow_ptr.size();
    v->prow_ptr.insert(v->prow_ptr.end(), rp, rp + n + 1);
    v->pat_row[p] = (int64_t)v->prow_len.size();
    for (int i = 0; i < n; ++i) {
      const int len = rp[i + 1] - rp[i];
      v->prow_len.push_back(len);
      int ds = -1;
      for (int k = 0; k < len; ++k)
        if (ci[rp[i] + k] == i) { ds = k; break; }
      v->pdiag.push_back(ds);
    }
    v->pat_sc[p] = (int64_t)v->pslot_col.size();
    const size_t base = v->pslot_col.size();
    v->pslot_col.resize(base + (size_t)maxr * n + 1, -1);
    for (int s = 0; s < maxr; ++s)
      for (int i = 0; i < n; ++i)
        if (s < rp[i + 1] - rp[i]) v->pslot_col[base + (size_t)s * n + i] = ci[rp[i] + s];
  }
  if (rc == BS_OK) {
    v->sys_pat.assign(sys_pat, sys_pat + n_batch);
    v->sys_rows.resize(n_batch);
    v->row_off.assign(n_batch + 1, 0);
    v->val_off.assign(n_batch + 1, 0);
    for (int64_t s = 0; s < n_batch; ++s) {
      const int p = sys_pat[s];
      if (p < 0 || p >= n_patterns) { rc = BS_ERR_PATTERN; break; }
      v->sys_rows[s] = v->pat_n[p];
      v->row_off[s + 1] = v->row_off[s] + v->pat_n[p];
      v->val_off[s + 1] = v->val_off[s] + v->pat_nnz[p];
    }
  }
  if (rc == BS_OK) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
      (void)hipGetLastError();
      bs::set_last_error("no HIP device");
      rc = BS_ERR_NO_DEVICE;
    }
  }
  if (rc == BS_OK) {
    hipError_t e = hipGetDevice(&v->device);
    // one allocation for the policy-independent arrays
    const size_t sz = [&] {
      size_t z = 0;
      z += (v->B ? v->B : 1) * 2 * sizeof(int);                  // sys_rows, sys_pat
      z += (v->B + 1) * 2 * sizeof(int64_t);                     // row_off, val_off
      z += (v->P ? v->P : 1) * 3 * sizeof(int64_t);              // pattern offsets
      z += (v->prow_ptr.size() + v->prow_len.size() + v->pdiag.size() + v->pslot_col.size() + 4) *
           sizeof(int);
      return z + 256;
    }();
    if (e == hipSuccess) e = hipMalloc(&v->d_static, sz);
    if (e == hipSuccess) e = hipMalloc(&v->d_tasks, (size_t)(v->B + 1) * sizeof(bs::VTask));
    if (e == hipSuccess) e = hipMalloc(&v->d_order, (size_t)(v->B + 1) * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&v->d_counter, 256);
    if (e != hipSuccess) rc = hip_err(e, "varbatch allocation");
    if (rc == BS_OK) {
      std::vector<char> h(sz, 0);
      size_t off = 0;
      auto put = [&](const void* src, size_t bytes) -> size_t {
        off = (off + 15) & ~(size_t)15;
        const size_t at = off;
        if (bytes) std::memcpy(h.data() + off, src, bytes);
        off += bytes;
        return at;
      };
      const size_t o_rows = put(v->sys_rows.data(), v->B * sizeof(int));
      const size_t o_pat = put(v->sys_pat.data(), v->B * sizeof(int));
      const size_t o_roff = put(v->row_off.data(), (v->B + 1) * sizeof(int64_t));
      const size_t o_voff = put(v->val_off.data(), (v->B + 1) * sizeof(int64_t));
      const size_t o_prp = put(v->pat_rp.data(), v->P * sizeof(int64_t));
      const size_t o_prow = put(v->pat_row.data(), v->P * sizeof(int64_t));
      const size_t o_psc = put(v->pat_sc.data(), v->P * sizeof(int64_t));
      const size_t o_rp = put(v->prow_ptr.data(), v->prow_ptr.size() * sizeof(int));
      const size_t o_len = put(v->prow_len.data(), v->prow_len.size() * sizeof(int));
      const size_t o_dg = put(v->pdiag.data(), v->pdiag.size() * sizeof(int));
      const size_t o_sc = put(v->pslot_col.data(), v->pslot_col.size() * sizeof(int));
      if (off > sz) {
        rc = BS_ERR_INVALID_ARG;
      } else {
        e = hipMemcpy(v->d_static, h.data(), sz, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_err(e, "varbatch upload");
      }
      char* d = v->d_static;
      v->args.sys_rows = (const int*)(d + o_rows);
      v->args.sys_pat = (const int*)(d + o_pat);
      v->args.row_off = (const int64_t*)(d + o_roff);
      v->args.val_off = (const int64_t*)(d + o_voff);
      v->args.pat_rp = (const int64_t*)(d + o_prp);
      v->args.pat_row = (const int64_t*)(d + o_prow);
      v->args.pat_sc = (const int64_t*)(d + o_psc);
      v->args.prow_ptr = (const int*)(d + o_rp);
      v->args.prow_len = (const int*)(d + o_len);
      v->args.pdiag = (const int*)(d + o_dg);
      v->args.pslot_col = (const int*)(d + o_sc);
      v->args.tasks = v->d_tasks;
      v->args.order = v->d_order;
      v->args.counter = v->d_counter;
    }
    if (rc == BS_OK) {
      v->policy_next = 0;
      build_tasks(*v, 0);
      rc = upload_tasks(*v);
    }
  }
  if (rc != BS_OK) {
    bs_varbatch_destroy(v);
    return rc;
  }
  *out = v;
  return BS_OK;
}

int bs_varbatch_destroy(bs_varbatch v) {
  if (!v) return BS_OK;
  if (v->gexec) (void)hipGraphExecDestroy(v->gexec);
  if (v->graph) (void)hipGraphDestroy(v->graph);
  if (v->cap_stream) (void)hipStreamDestroy(v->cap_stream);
  if (v->d_static) (void)hipFree(v->d_static);
  if (v->d_tasks) (void)hipFree(v->d_tasks);
  if (v->d_order) (void)hipFree(v->d_order);
  if (v->d_counter) (void)hipFree(v->d_counter);
  delete v;
  return BS_OK;
}

int bs_varbatch_query(bs_varbatch v, int64_t* total_rows, int64_t* total_values, int32_t* n_tasks,
                      int32_t* policy) {
  if (!v) return BS_ERR_INVALID_ARG;
  if (total_rows) *total_rows = v->row_off.empty() ? 0 : v->row_off.back();
  if (total_values) *total_values = v->val_off.empty() ? 0 : v->val_off.back();
  if (n_tasks) *n_tasks = (int32_t)v->tasks.size();
  if (policy) *policy = v->policy;
  return BS_OK;
}

int bs_varbatch_set_policy(bs_varbatch v, int32_t policy) {
  if (!v || policy < 0 || policy >= kNumPolicies) return BS_ERR_INVALID_ARG;
  if (policy == v->policy) return BS_OK;
  // a captured graph holds the old task count: drop it
  if (v->gexec) { (void)hipGraphExecDestroy(v->gexec); v->gexec = nullptr; }
  if (v->graph) { (void)hipGraphDestroy(v->graph); v->graph = nullptr; }
  v->policy_next = policy;
  build_tasks(*v, policy);
  const int rc = upload_tasks(*v);
  if (rc == BS_OK) {
    v->policy = policy;
  } else {  // restore the previous tasks
    v->policy_next = v->policy;
    build_tasks(*v, v->policy);
    (void)upload_tasks(*v);
  }
  return rc;
}

int bs_varbatch_solve(bs_varbatch v, const double* values, const double* b, double* x,
                      bs_solver solver, bs_precond precond, double tol, int32_t max_iter,
                      int32_t* iters, double* resid, int32_t* status, const bs_options* opts,
                      void* stream) {
  if (!v) return BS_ERR_INVALID_ARG;
  return launch(*v, values, b, x, solver, precond, tol, max_iter, iters, resid, status, opts,
                (hipStream_t)stream);
}

int bs_varbatch_tune(bs_varbatch v, const double* values, const double* b, double* x,
                     bs_solver solver, bs_precond precond, double tol, int32_t max_iter,
                     int32_t* iters, double* resid, int32_t* status, const bs_options* opts,
                     int32_t reps, const char* cache_path, char* report, size_t report_len,
                     void* stream) {
  if (!v || reps < 1) return BS_ERR_INVALID_ARG;
  const hipStream_t st = (hipStream_t)stream;
  const int mixed = opts && opts->precision == BS_MIXED;
  const std::string key = tune_key(*v, solver, mixed);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "r");
    if (f) {
      char k[512];
      int p = -1;
      double t = 0;
      int found = -1;
      while (std::fscanf(f, "%511s %d %lf", k, &p, &t) == 3)
        if (key == k && p >= 0 && p < kNumPolicies) found = p;
      std::fclose(f);
      if (found >= 0) {
        const int rc = bs_varbatch_set_policy(v, found);
        if (rc == BS_OK && report && report_len)
          std::snprintf(report, report_len, "policy=%d cached key=%s", found, key.c_str());
        return rc;
      }
    }
  }
  double times[kNumPolicies] = {0};
  int best = 0;
  // every timed solve starts from the caller's x0 (kept in a copy) unless the
  // flags say x0 = 0; the copy back is timed for every policy alike
  const bool keep_x0 = !(opts && (opts->flags & BS_FLAG_X0_ZERO)) && v->B > 0 && x;
  const size_t xbytes = (size_t)v->row_off.back() * sizeof(double);
  double* x0 = nullptr;
  if (keep_x0) {
    hipError_t e = hipMalloc(&x0, xbytes);
    if (e == hipSuccess) e = hipMemcpyAsync(x0, x, xbytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
      if (x0) (void)hipFree(x0);
      return hip_err(e, "tune x0 copy");
    }
  }
  auto run = [&]() -> int {
    if (keep_x0) {
      const hipError_t e = hipMemcpyAsync(x, x0, xbytes, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_err(e, "tune x0 restore");
    }
    return launch(*v, values, b, x, solver, precond, tol, max_iter, iters, resid, status, opts, st);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BS_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = hip_err(hipGetLastError(), "tune events");
  for (int p = 0; p < kNumPolicies && rc == BS_OK; ++p) {
    rc = bs_varbatch_set_policy(v, p);
    if (rc != BS_OK) break;
    rc = run();
    if (rc != BS_OK) break;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps && rc == BS_OK; ++r) rc = run();
    (void)hipEventRecord(e1, st);
    hipError_t e = hipEventSynchronize(e1);
    if (e != hipSuccess) { rc = hip_err(e, "tune sync"); break; }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    times[p] = ms / reps;
    if (times[p] < times[best]) best = p;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == BS_OK) rc = bs_varbatch_set_policy(v, best);
  if (rc == BS_OK) rc = run();  // outputs of the chosen policy
  if (x0) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(x0);
  }
  if (rc != BS_OK) return rc;
  if (report && report_len) {
    std::string t;
    for (int p = 0; p < kNumPolicies; ++p) {
      char buf[32];
      std::snprintf(buf, sizeof buf, "%s%.4f", p ? "," : "", times[p]);
      t += buf;
    }
    std::snprintf(report, report_len, "policy=%d times_ms=%s key=%s", best, t.c_str(),
                  key.c_str());
  }
  if (rc == BS_OK && cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %d %.6f\n", key.c_str(), best, times[best]);
      std::fclose(f);
    }
  }
  return rc;
}

int bs_varbatch_capture(bs_varbatch v, const double* values, const double* b, double* x,
                        bs_solver solver, bs_precond precond, double tol, int32_t max_iter,
                        int32_t* iters, double* resid, int32_t* status, const bs_options* opts) {
  if (!v) return BS_ERR_INVALID_ARG;
  hipError_t e = hipSuccess;
  if (!v->cap_stream) {
    e = hipStreamCreateWithFlags(&v->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_err(e, "capture stream");
  }
  if (v->gexec) { (void)hipGraphExecDestroy(v->gexec); v->gexec = nullptr; }
  if (v->graph) { (void)hipGraphDestroy(v->graph); v->graph = nullptr; }
  e = hipStreamBeginCapture(v->cap_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_err(e, "begin capture");
  const int rc = launch(*v, values, b, x, solver, precond, tol, max_iter, iters, resid, status, opts,
                        v->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(v->cap_stream, &g);
  if (rc != BS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_err(e, "end capture");
  v->graph = g;
  e = hipGraphInstantiate(&v->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_err(e, "graph instantiate");
  return BS_OK;
}

int bs_varbatch_replay(bs_varbatch v, void* stream) {
  if (!v || !v->gexec) return BS_ERR_INVALID_ARG;
  const hipError_t e = hipGraphLaunch(v->gexec, (hipStream_t)stream);
  return e == hipSuccess ? BS_OK : hip_err(e, "graph launch");
}

}  // extern "C"
