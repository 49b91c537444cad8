// Host side of the uneven-batch entry points (bs_varbatch_*, bs_batch_solve_varlen):
// validation and derivation of every distinct pattern (CSR or ELL input), the
// task queue, the persistent launches (one for the whole batch, or one per
// size class), the autotuner over shapes, placements and walk orders, and the
// captured HIP graph (counter reset + solve).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/batchsolve.h"
#include "bs_varlen_table.hpp"

namespace bs {
void set_last_error(const std::string& msg);
int* device_sink();

__global__ void k_varlen_reset(int* counter) {
  if (threadIdx.x < kMaxClasses) counter[threadIdx.x] = 0;
}
}  // namespace bs

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

// Workgroup shapes (lanes, rows per lane); each holds systems of up to 1024 rows.
struct VShapeInfo {
  int wg, r;
};
constexpr VShapeInfo kVShapes[] = {{1024, 1}, {512, 2}, {256, 4}};
constexpr int kNumShapes = 3;
constexpr int kNumOrders = 3;
constexpr int kNumRegPolicies = kNumShapes * kNumOrders;  // rows in registers
constexpr int kNumPolicies = 2 * kNumRegPolicies;         // then the streamed placement
constexpr int kMaxVarRows = 1024;
// Size classes of the per-class plans: n <= 64, 128, 256, 512, 1024 rows.
constexpr int kNumClasses = 5;
static_assert(kNumClasses <= bs::kMaxClasses, "one task counter per class");
// A class choice: workgroup shape (code % 3), walk (code / 3 % 2: 0 the row
// order, 1 the slot-major order) and placement (code / 6: 0 registers,
// 1 streamed).
constexpr int kNumChoices = 12;

int class_of(int n) {
  int c = 0;
  while ((bs::kWave << c) < n) ++c;
  return c;
}

struct Choice {
  int shape, walk, stream;
};
Choice choice_of(int code) { return {code % kNumShapes, (code / kNumShapes) % 2, code / (2 * kNumShapes)}; }

// Kernel of (shape, slots, solver, precision, block Jacobi, source, placement):
// the registered instance with the fewest slots >= nz (any, when streamed).
const bs::VEntry* find_v(VShapeInfo sh, int nz, int solver, int mixed, int bj, int src, int stream) {
  int n = 0;
  const bs::VEntry* t = src == bs::kSrcCsr      ? bs::vtable_csr(&n)
                        : src == bs::kSrcRowIdx ? bs::vtable_row(&n)
                                                : bs::vtable_slot(&n);
  const bs::VEntry* best = nullptr;
  for (int i = 0; i < n; ++i) {
    const bs::VEntry& e = t[i];
    if (e.wg != sh.wg || e.r != sh.r || e.solver != solver || e.mixed != mixed || e.bj != bj ||
        e.src != src || e.stream != stream)
      continue;
    if (stream) return &e;
    if (e.nz >= nz && (!best || e.nz < best->nz)) best = &e;
  }
  return best;
}

}  // namespace

// Validated host description of an uneven batch: per system its row count,
// pattern and offsets; the longest row of the batch and of every size class.
struct VarDesc {
  int64_t B = 0;
  int P = 0, max_row = 0;
  int fmt = BS_CSR;  // layout of the values (BS_CSR or BS_ELL)
  std::vector<int> sys_rows, sys_pat;
  std::vector<int64_t> row_off, val_off;
  int cls_max_row[kNumClasses] = {0};
  int64_t cls_count[kNumClasses] = {0};
};

// How one solve is launched: a single persistent launch under `policy`
// (0..17), or (policy = -1) one launch per size class with the class's choice.
struct Plan {
  int policy = 0;
  int code[kNumClasses] = {0};
};

// Tasks of a plan; per-class plans keep class c's tasks at [lo[c], hi[c]).
struct TaskSet {
  std::vector<bs::VTask> tasks;
  std::vector<int> order;
  int lo[kNumClasses] = {0}, hi[kNumClasses] = {0};
};

struct bs_varbatch_s {
  VarDesc d;
  int device = -1;
  Plan plan;
  TaskSet ts;
  // the handle's pattern arrays: CSR structure, and every entry's value
  // position in its system's block as {column, position} pairs in row order
  // (idx_row, ELL input) and slot-major (idx_slot)
  std::vector<int64_t> pat_rp, pat_col, pat_slot;
  std::vector<int> pat_w, rowptr_all, col_all, idx_row, idx_slot;
  // device
  char* d_static = nullptr;  // everything that does not depend on the plan
  bs::VTask* d_tasks = nullptr;
  int* d_order = nullptr;
  int* d_counter = nullptr;
  bs::VArgs args{};
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
};

namespace {

void finish_desc(VarDesc& d, const std::vector<int>& pat_longest) {
  d.max_row = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    d.cls_max_row[c] = 0;
    d.cls_count[c] = 0;
  }
  for (int64_t s = 0; s < d.B; ++s) {
    const int c = class_of(d.sys_rows[s]), w = pat_longest[d.sys_pat[s]];
    d.cls_count[c]++;
    d.cls_max_row[c] = std::max(d.cls_max_row[c], w);
    d.max_row = std::max(d.max_row, w);
  }
}

bool row_ok(const int* cols, int len, int n, std::vector<int>& mark, int stamp) {
  for (int k = 0; k < len; ++k) {
    const int c = cols[k];
    if (c < 0 || c >= n || mark[c] == stamp) return false;
    mark[c] = stamp;
  }
  return true;
}

// Checks a CSR pattern (n rows, row_ptr rp within rp_room entries of its array,
// columns from cols within col_room entries): row_ptr starts at 0 and never
// decreases, every column lies in [0, n) and appears once per row.  Returns its
// nnz and longest row.
int check_pattern(int n, const int32_t* rp, int64_t rp_room, const int32_t* cols, int64_t col_room,
                  int* longest, int64_t* nnz, std::vector<int>& mark) {
  if (n < 1) return BS_ERR_INVALID_ARG;
  if (n > kMaxVarRows) return BS_ERR_UNSUPPORTED;
  if (rp_room < (int64_t)n + 1) return BS_ERR_PATTERN;
  if (rp[0] != 0) return BS_ERR_PATTERN;
  int maxr = 0;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return BS_ERR_PATTERN;
    maxr = std::max(maxr, rp[i + 1] - rp[i]);
  }
  if (rp[n] > col_room) return BS_ERR_PATTERN;
  mark.assign(n, -1);
  for (int i = 0; i < n; ++i)
    if (!row_ok(cols + rp[i], rp[i + 1] - rp[i], n, mark, i)) return BS_ERR_PATTERN;
  *longest = maxr;
  *nnz = rp[n];
  return BS_OK;
}

// One validated pattern: CSR structure, every entry's position in a system's
// value block, the values one system holds.
struct PatCsr {
  int n = 0, longest = 0;
  std::vector<int> rp, col, pos;
  int64_t values = 0;
};

int pattern_from_csr(int n, const int32_t* rp, const int32_t* cols, std::vector<int>& mark,
                     PatCsr& out) {
  int64_t nnz = 0;
  const int rc = check_pattern(n, rp, (int64_t)n + 1, cols, INT64_MAX, &out.longest, &nnz, mark);
  if (rc != BS_OK) return rc;
  out.n = n;
  out.rp.assign(rp, rp + n + 1);
  out.col.assign(cols, cols + nnz);
  out.pos.resize((size_t)nnz);
  for (int64_t k = 0; k < nnz; ++k) out.pos[k] = (int)k;
  out.values = nnz;
  return BS_OK;
}

// ELL pattern: slot-major columns [w][n], -1 padding after a row's entries.
int pattern_from_ell(int n, int w, const int32_t* ell, std::vector<int>& mark, PatCsr& out) {
  if (n < 1 || w < 0) return BS_ERR_INVALID_ARG;
  if (n > kMaxVarRows || w > kMaxVarRows) return BS_ERR_UNSUPPORTED;
  out.n = n;
  out.rp.assign(n + 1, 0);
  out.col.clear();
  out.pos.clear();
  out.longest = 0;
  mark.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    int len = 0;
    for (int k = 0; k < w; ++k) {
      const int c = ell[(int64_t)k * n + i];
      if (c == -1) continue;
      if (len != k) return BS_ERR_PATTERN;  // an entry after padding
      if (c < 0 || c >= n || mark[c] == i) return BS_ERR_PATTERN;
      mark[c] = i;
      out.col.push_back(c);
      out.pos.push_back(k * n + i);
      ++len;
    }
    out.rp[i + 1] = out.rp[i] + len;
    out.longest = std::max(out.longest, len);
  }
  out.values = (int64_t)w * n;
  return BS_OK;
}

// Tasks of size class `cls` (every class when cls < 0) for workgroup shape `sh`
// and queue order `ord`, appended to ts.
void append_tasks(const VarDesc& v, VShapeInfo sh, int ord, int cls, TaskSet& ts) {
  std::vector<int> idx;
  std::vector<int> team(v.B, 0);
  for (int64_t s = 0; s < v.B; ++s) {
    if (cls >= 0 && class_of(v.sys_rows[s]) != cls) continue;
    int t = std::max(bs::kWave, next_pow2((v.sys_rows[s] + sh.r - 1) / sh.r));
    if (ord == 1) t = std::min(sh.wg, 2 * t);
    team[s] = t;
    idx.push_back((int)s);
  }
  // group by team size (largest first); inside a class, largest systems first
  // (similar sizes share a task) unless the order keeps the batch order
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (team[a] != team[b]) return team[a] > team[b];
    if (ord == 2) return false;
    return v.val_off[a + 1] - v.val_off[a] > v.val_off[b + 1] - v.val_off[b];
  });
  const int base = (int)ts.order.size();
  ts.order.insert(ts.order.end(), idx.begin(), idx.end());
  for (size_t i = 0; i < idx.size();) {
    const int t = team[idx[i]], cap = sh.wg / t;
    int c = 0;
    while (i + c < idx.size() && c < cap && team[idx[i + c]] == t) ++c;
    ts.tasks.push_back({t, base + (int)i, c, 0});
    i += c;
  }
}

// Tasks of a plan.  A single launch (policy p): workgroup shape (p % 9) / 3,
// queue order p % 3.  Per-class launches: classes largest first, each with the
// shape of its choice and queue order 0.
void build_tasks(const VarDesc& v, const Plan& pl, TaskSet& ts) {
  ts.tasks.clear();
  ts.order.clear();
  if (pl.policy >= 0) {
    append_tasks(v, kVShapes[(pl.policy % kNumRegPolicies) / kNumOrders], pl.policy % kNumOrders,
                 -1, ts);
    return;
  }
  for (int c = kNumClasses - 1; c >= 0; --c) {
    ts.lo[c] = (int)ts.tasks.size();
    if (v.cls_count[c]) append_tasks(v, kVShapes[choice_of(pl.code[c]).shape], 0, c, ts);
    ts.hi[c] = (int)ts.tasks.size();
  }
}

// What the kernel assumes of every task: a power-of-two team of at least a
// wave that holds each of its systems, teams that fit one workgroup of the
// launch's shape, and the tasks covering the queue order once.
int check_range(const VarDesc& v, VShapeInfo sh, const TaskSet& ts, int lo, int hi,
                int64_t* covered) {
  for (int i = lo; i < hi; ++i) {
    const bs::VTask& t = ts.tasks[i];
    if (t.team < bs::kWave || t.team > sh.wg || (t.team & (t.team - 1)) || t.count < 1 ||
        (int64_t)t.count * t.team > sh.wg || t.first != *covered)
      return BS_ERR_INVALID_ARG;
    for (int k = 0; k < t.count; ++k)
      if (v.sys_rows[ts.order[t.first + k]] > t.team * sh.r) return BS_ERR_INVALID_ARG;
    *covered += t.count;
  }
  return BS_OK;
}

int check_tasks(const VarDesc& v, const Plan& pl, const TaskSet& ts) {
  int64_t covered = 0;
  int rc = BS_OK;
  if (pl.policy >= 0) {
    rc = check_range(v, kVShapes[(pl.policy % kNumRegPolicies) / kNumOrders], ts, 0,
                     (int)ts.tasks.size(), &covered);
  } else {
    for (int c = kNumClasses - 1; c >= 0 && rc == BS_OK; --c) {
      if (pl.code[c] < 0 || pl.code[c] >= kNumChoices) return BS_ERR_INVALID_ARG;
      rc = check_range(v, kVShapes[choice_of(pl.code[c]).shape], ts, ts.lo[c], ts.hi[c], &covered);
    }
  }
  if (rc != BS_OK) return rc;
  return covered == v.B && (int64_t)ts.order.size() == v.B ? BS_OK : BS_ERR_INVALID_ARG;
}

// One kernel launch of a solve.
struct Launch {
  const bs::VEntry* k;
  int lo, hi, counter;
};

// The kernels of a plan (one per launch).  BS_ERR_UNSUPPORTED when a launch
// has no compiled kernel (a row longer than the register placement holds, or a
// preconditioner the streamed placement does not apply).
int plan_launches(const VarDesc& v, const Plan& pl, const TaskSet& ts, int solver, int mixed, int bj,
                  int only_class, std::vector<Launch>& out) {
  out.clear();
  if (pl.policy >= 0) {
    const VShapeInfo sh = kVShapes[(pl.policy % kNumRegPolicies) / kNumOrders];
    const int stream = pl.policy >= kNumRegPolicies;
    // the walk of the input's own layout
    const int src = v.fmt == BS_ELL ? bs::kSrcSlotIdx : bs::kSrcCsr;
    const bs::VEntry* k = find_v(sh, std::max(v.max_row, 1), solver, mixed, bj, src, stream);
    if (!k) return BS_ERR_UNSUPPORTED;
    out.push_back({k, 0, (int)ts.tasks.size(), 0});
    return BS_OK;
  }
  for (int c = kNumClasses - 1; c >= 0; --c) {
    if (ts.hi[c] == ts.lo[c] || (only_class >= 0 && c != only_class)) continue;
    const Choice ch = choice_of(pl.code[c]);
    const int src = ch.walk ? bs::kSrcSlotIdx : v.fmt == BS_ELL ? bs::kSrcRowIdx : bs::kSrcCsr;
    const bs::VEntry* k = find_v(kVShapes[ch.shape], std::max(v.cls_max_row[c], 1), solver, mixed, bj,
                                 src, ch.stream);
    if (!k) return BS_ERR_UNSUPPORTED;
    out.push_back({k, ts.lo[c], ts.hi[c], c});
  }
  return BS_OK;
}

// One solve: the counter reset, then the plan's persistent launches in order on
// `stream`.  `a` holds the structure pointers; tasks/order point at the
// plan's device copy of ts; only_class >= 0 launches that class alone.
int launch(const VarDesc& v, bs::VArgs a, const Plan& pl, const TaskSet& ts, int device,
           int* counter, const double* values, const double* b, double* x, bs_solver solver,
           bs_precond precond, double tol, int max_iter, int* iters, double* resid, int* status,
           const bs_options* o, hipStream_t stream, int only_class = -1) {
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
  if (mixed && block > 1) return BS_ERR_UNSUPPORTED;
  std::vector<Launch> ls;
  int rc = plan_launches(v, pl, ts, solver == BS_CG ? 0 : 1, mixed, block > 1 ? 1 : 0, only_class,
                         ls);
  if (rc != BS_OK) return rc;
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
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return hip_err(e, "device attribute");
  hipLaunchKernelGGL(bs::k_varlen_reset, dim3(1), dim3(bs::kWave), 0, stream, counter);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "counter reset");
  const bs::VTask* tasks = a.tasks;
  for (const Launch& l : ls) {
    int per_cu = 0;
    e = l.k->occ(&per_cu);
    if (e != hipSuccess) return hip_err(e, "occupancy");
    a.tasks = tasks + l.lo;
    a.n_tasks = l.hi - l.lo;
    a.counter = counter + l.counter;
    const int64_t resident = (int64_t)cus * std::max(per_cu, 1);
    const unsigned grid = (unsigned)std::min<int64_t>(resident, a.n_tasks);
    e = l.k->fn(a, grid, stream);
    if (e != hipSuccess) return hip_err(e, "uneven-batch launch");
  }
  return BS_OK;
}

int launch(bs_varbatch_s& v, const double* values, const double* b, double* x, bs_solver solver,
           bs_precond precond, double tol, int max_iter, int* iters, double* resid, int* status,
           const bs_options* o, hipStream_t stream, int only_class = -1) {
  return launch(v.d, v.args, v.plan, v.ts, v.device, v.d_counter, values, b, x, solver, precond,
                tol, max_iter, iters, resid, status, o, stream, only_class);
}

int upload_tasks(bs_varbatch_s& v, const TaskSet& ts) {
  hipError_t e = hipSuccess;
  if (!ts.tasks.empty())
    e = hipMemcpy(v.d_tasks, ts.tasks.data(), ts.tasks.size() * sizeof(bs::VTask),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(e, "upload tasks");
  if (!ts.order.empty())
    e = hipMemcpy(v.d_order, ts.order.data(), ts.order.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(e, "upload order");
  return BS_OK;
}

void drop_graph(bs_varbatch_s& v) {
  if (v.gexec) { (void)hipGraphExecDestroy(v.gexec); v.gexec = nullptr; }
  if (v.graph) { (void)hipGraphDestroy(v.graph); v.graph = nullptr; }
}

// Switch the handle to plan `pl` (tasks built, checked and uploaded).  On
// failure the previous plan stays in force.
int apply_plan(bs_varbatch_s& v, const Plan& pl) {
  TaskSet ts;
  build_tasks(v.d, pl, ts);
  int rc = check_tasks(v.d, pl, ts);
  if (rc != BS_OK) return rc;
  drop_graph(v);  // a captured graph holds the old launches
  rc = upload_tasks(v, ts);
  if (rc != BS_OK) {
    (void)upload_tasks(v, v.ts);  // restore the previous tasks
    return rc;
  }
  v.plan = pl;
  v.ts = std::move(ts);
  return BS_OK;
}

bool same_plan(const Plan& a, const Plan& b) {
  if (a.policy != b.policy) return false;
  if (a.policy >= 0) return true;
  for (int c = 0; c < kNumClasses; ++c)
    if (a.code[c] != b.code[c]) return false;
  return true;
}

std::string plan_token(const Plan& pl) {
  if (pl.policy >= 0) return std::to_string(pl.policy);
  std::string t = "split:";
  for (int c = 0; c < kNumClasses; ++c) t += (c ? "," : "") + std::to_string(pl.code[c]);
  return t;
}

bool parse_plan(const char* tok, Plan& pl) {
  if (std::strncmp(tok, "split:", 6) == 0) {
    pl.policy = -1;
    const char* p = tok + 6;
    for (int c = 0; c < kNumClasses; ++c) {
      char* end = nullptr;
      const long v = std::strtol(p, &end, 10);
      if (end == p || v < 0 || v >= kNumChoices) return false;
      pl.code[c] = (int)v;
      p = end;
      if (c + 1 < kNumClasses) {
        if (*p != ',') return false;
        ++p;
      }
    }
    return *p == 0;
  }
  char* end = nullptr;
  const long v = std::strtol(tok, &end, 10);
  if (end == tok || *end != 0 || v < 0 || v >= kNumPolicies) return false;
  pl.policy = (int)v;
  return true;
}

std::string tune_key(const VarDesc& v, bs_solver solver, int mixed, bs_precond precond) {
  std::string k = v.fmt == BS_ELL ? "varbatch_ell" : "varbatch";
  for (int c = 0; c < kNumClasses; ++c) k += "_" + std::to_string(v.cls_count[c]);
  k += "_w";
  for (int c = 0; c < kNumClasses; ++c) k += (c ? "." : "") + std::to_string(v.cls_max_row[c]);
  k += "_s" + std::to_string((int)solver) + "_m" + std::to_string(mixed) + "_p" +
       std::to_string((int)precond);
  return k;
}

std::string choice_name(int code) {
  const Choice ch = choice_of(code);
  const VShapeInfo sh = kVShapes[ch.shape];
  return std::to_string(sh.wg) + "x" + std::to_string(sh.r) + "/" + (ch.walk ? "ell" : "csr") +
         "/" + (ch.stream ? "stream" : "reg");
}

int have_device(int* device) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    bs::set_last_error("no HIP device");
    return BS_ERR_NO_DEVICE;
  }
  const hipError_t e = hipGetDevice(device);
  return e == hipSuccess ? BS_OK : hip_err(e, "hipGetDevice");
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The handle from validated patterns: host description, the pattern arrays and
// indexes, one device allocation for them, and the tasks of the default plan.
int create_handle(int64_t n_batch, int fmt, std::vector<PatCsr>& pats, const int32_t* sys_pat,
                  bs_varbatch* out) {
  const int P = (int)pats.size();
  bs_varbatch_s* v = new bs_varbatch_s();
  VarDesc& d = v->d;
  d.B = n_batch;
  d.P = P;
  d.fmt = fmt;
  int rc = BS_OK;
  std::vector<int> longest(P, 0);
  v->pat_rp.resize(P);
  v->pat_col.resize(P);
  v->pat_slot.resize(P);
  v->pat_w.resize(P);
  for (int p = 0; p < P; ++p) {
    const PatCsr& q = pats[p];
    longest[p] = q.longest;
    v->pat_rp[p] = (int64_t)v->rowptr_all.size();
    v->rowptr_all.insert(v->rowptr_all.end(), q.rp.begin(), q.rp.end());
    v->pat_col[p] = (int64_t)v->col_all.size();
    v->col_all.insert(v->col_all.end(), q.col.begin(), q.col.end());
    if (fmt == BS_ELL)
      for (size_t k = 0; k < q.col.size(); ++k) {
        v->idx_row.push_back(q.col[k]);
        v->idx_row.push_back(q.pos[k]);
      }
    // slot-major index: width = the longest row
    const int w = q.longest;
    v->pat_w[p] = w;
    v->pat_slot[p] = (int64_t)v->idx_slot.size() / 2;
    const size_t at = v->idx_slot.size();
    v->idx_slot.resize(at + (size_t)2 * w * q.n, 0);
    for (int k = 0; k < w; ++k)
      for (int i = 0; i < q.n; ++i) {
        const int len = q.rp[i + 1] - q.rp[i];
        int* e = &v->idx_slot[at + 2 * ((size_t)k * q.n + i)];
        e[0] = k < len ? q.col[q.rp[i] + k] : -1;
        e[1] = k < len ? q.pos[q.rp[i] + k] : 0;
      }
  }
  d.sys_pat.assign(sys_pat, sys_pat + n_batch);
  d.sys_rows.resize(n_batch);
  d.row_off.assign(n_batch + 1, 0);
  d.val_off.assign(n_batch + 1, 0);
  for (int64_t s = 0; s < n_batch; ++s) {
    const int p = sys_pat[s];
    if (p < 0 || p >= P) { rc = BS_ERR_PATTERN; break; }
    d.sys_rows[s] = pats[p].n;
    d.row_off[s + 1] = d.row_off[s] + pats[p].n;
    d.val_off[s + 1] = d.val_off[s] + pats[p].values;
  }
  if (rc == BS_OK) finish_desc(d, longest);
  if (rc == BS_OK) rc = have_device(&v->device);
  if (rc == BS_OK) {
    // one allocation for the plan-independent arrays, 16-byte aligned pieces
    std::vector<char> h;
    auto put = [&](const void* src, size_t bytes) -> size_t {
      const size_t at = (h.size() + 15) & ~(size_t)15;
      h.resize(at + bytes);
      if (bytes) std::memcpy(h.data() + at, src, bytes);
      return at;
    };
    const size_t o_rows = put(d.sys_rows.data(), d.B * sizeof(int));
    const size_t o_pat = put(d.sys_pat.data(), d.B * sizeof(int));
    const size_t o_roff = put(d.row_off.data(), (d.B + 1) * sizeof(int64_t));
    const size_t o_voff = put(d.val_off.data(), (d.B + 1) * sizeof(int64_t));
    const size_t o_prp = put(v->pat_rp.data(), P * sizeof(int64_t));
    const size_t o_pco = put(v->pat_col.data(), P * sizeof(int64_t));
    const size_t o_psl = put(v->pat_slot.data(), P * sizeof(int64_t));
    const size_t o_pw = put(v->pat_w.data(), P * sizeof(int));
    const size_t o_rp = put(v->rowptr_all.data(), v->rowptr_all.size() * sizeof(int));
    const size_t o_col = put(v->col_all.data(), v->col_all.size() * sizeof(int));
    const size_t o_ir = put(v->idx_row.data(), v->idx_row.size() * sizeof(int));
    const size_t o_is = put(v->idx_slot.data(), v->idx_slot.size() * sizeof(int));
    h.resize(h.size() + 16);
    hipError_t e = hipMalloc(&v->d_static, h.size());
    if (e == hipSuccess) e = hipMalloc(&v->d_tasks, (size_t)(d.B + 1) * sizeof(bs::VTask));
    if (e == hipSuccess) e = hipMalloc(&v->d_order, (size_t)(d.B + 1) * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&v->d_counter, 256);
    if (e == hipSuccess) e = hipMemcpy(v->d_static, h.data(), h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = hip_err(e, "varbatch allocation");
    if (rc == BS_OK) {
      char* dd = v->d_static;
      v->args.sys_rows = (const int*)(dd + o_rows);
      v->args.sys_pat = (const int*)(dd + o_pat);
      v->args.row_off = (const int64_t*)(dd + o_roff);
      v->args.val_off = (const int64_t*)(dd + o_voff);
      v->args.pat_rp = (const int64_t*)(dd + o_prp);
      v->args.pat_col = (const int64_t*)(dd + o_pco);
      v->args.pat_slot = (const int64_t*)(dd + o_psl);
      v->args.pat_w = (const int*)(dd + o_pw);
      v->args.rowptr_all = (const int*)(dd + o_rp);
      v->args.col_all = (const int*)(dd + o_col);
      v->args.idx_row = (const int2*)(dd + o_ir);
      v->args.idx_slot = (const int2*)(dd + o_is);
      v->args.tasks = v->d_tasks;
      v->args.order = v->d_order;
      v->args.counter = v->d_counter;
      // default plan: one launch, 1024 lanes x 1 row, rows in registers when
      // they fit there
      Plan pl;
      pl.policy = d.max_row <= 16 ? 0 : kNumRegPolicies;
      rc = apply_plan(*v, pl);
    }
  }
  if (rc != BS_OK) {
    bs_varbatch_destroy(v);
    return rc;
  }
  *out = v;
  return BS_OK;
}

// Workspace of bs_batch_solve_varlen: the task counters, the tasks, the queue
// order.
struct WsLayout {
  size_t counter, tasks, order, total;
};
WsLayout ws_layout(int64_t B) {
  WsLayout w;
  w.counter = 0;
  w.tasks = 256;
  w.order = w.tasks + align256((size_t)(B + 1) * sizeof(bs::VTask));
  w.total = w.order + align256((size_t)(B + 1) * sizeof(int));
  return w;
}

// ---------------------------------------------------------------- caller-owned batches
// bs_batch_solve_varlen reads the caller's structure arrays once (one copy to
// the host), validates them and keeps what it derived, keyed by the arrays'
// addresses, the batch shape, the device and the caller's generation number.
struct VarKey {
  int device;
  int64_t B;
  int P;
  int32_t generation;
  const void* ptr[8];
  bool operator==(const VarKey& o) const {
    if (device != o.device || B != o.B || P != o.P || generation != o.generation) return false;
    for (int i = 0; i < 8; ++i)
      if (ptr[i] != o.ptr[i]) return false;
    return true;
  }
};

struct VarEntry {
  VarKey key;
  VarDesc d;
  Plan plan;  // plan of the tasks below
  bool built = false;
  TaskSet ts;
  const void* ws = nullptr;  // workspace that holds these tasks, or null
  Plan ws_plan;
  uint64_t used = 0;
};

std::mutex g_var_mu;
std::vector<VarEntry> g_var_cache;
uint64_t g_var_clock = 0;
constexpr size_t kVarCacheEntries = 8;

template <class T>
int d2h(std::vector<T>& dst, const T* src, int64_t count, hipStream_t st) {
  dst.resize((size_t)std::max<int64_t>(count, 0));
  if (count <= 0) return BS_OK;
  hipError_t e = hipMemcpyAsync(dst.data(), src, (size_t)count * sizeof(T), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? BS_OK : hip_err(e, "read uneven-batch structure");
}

// Reads and validates a caller-owned uneven batch (CSR).
int read_batch(VarDesc& d, int64_t B, const int32_t* sys_rows, const int64_t* row_off,
               const int64_t* val_off, int32_t P, const int32_t* pat_id,
               const int64_t* pat_rowptr_off, const int64_t* pat_col_off,
               const int32_t* rowptr_all, const int32_t* col_all, hipStream_t st) {
  d = VarDesc{};
  d.B = B;
  d.P = P;
  std::vector<int64_t> prp, pco;
  int rc = d2h(d.sys_rows, sys_rows, B, st);
  if (rc == BS_OK) rc = d2h(d.sys_pat, pat_id, B, st);
  if (rc == BS_OK) rc = d2h(d.row_off, row_off, B + 1, st);
  if (rc == BS_OK) rc = d2h(d.val_off, val_off, B + 1, st);
  if (rc == BS_OK) rc = d2h(prp, pat_rowptr_off, P, st);
  if (rc == BS_OK) rc = d2h(pco, pat_col_off, P, st);
  if (rc != BS_OK) return rc;
  // rows of each pattern: those of the systems that use it (all the same)
  std::vector<int> rows(P, 0);
  for (int64_t s = 0; s < B; ++s) {
    const int p = d.sys_pat[s];
    if (p < 0 || p >= P) return BS_ERR_PATTERN;
    const int n = d.sys_rows[s];
    if (n < 1) return BS_ERR_INVALID_ARG;
    if (n > kMaxVarRows) return BS_ERR_UNSUPPORTED;
    if (rows[p] != 0 && rows[p] != n) return BS_ERR_INVALID_ARG;
    rows[p] = n;
  }
  int64_t rp_len = 0;
  for (int p = 0; p < P; ++p)
    if (rows[p]) {
      if (prp[p] < 0 || pco[p] < 0) return BS_ERR_INVALID_ARG;
      rp_len = std::max(rp_len, prp[p] + rows[p] + 1);
    }
  std::vector<int32_t> rpa, cola;
  rc = d2h(rpa, rowptr_all, rp_len, st);
  if (rc != BS_OK) return rc;
  std::vector<int64_t> nnz(P, 0);
  int64_t col_len = 0;
  for (int p = 0; p < P; ++p)
    if (rows[p]) {
      const int32_t* rp = rpa.data() + prp[p];
      for (int i = 0; i <= rows[p]; ++i)
        if (rp[i] < 0 || (i && rp[i] < rp[i - 1])) return BS_ERR_PATTERN;
      nnz[p] = rp[rows[p]];
      col_len = std::max(col_len, pco[p] + nnz[p]);
    }
  rc = d2h(cola, col_all, col_len, st);
  if (rc != BS_OK) return rc;
  std::vector<int> mark, longest(P, 0);
  for (int p = 0; p < P; ++p)
    if (rows[p]) {
      int64_t nz = 0;
      rc = check_pattern(rows[p], rpa.data() + prp[p], rp_len - prp[p], cola.data() + pco[p],
                         col_len - pco[p], &longest[p], &nz, mark);
      if (rc != BS_OK) return rc;
    }
  // offsets: each system's rows and values follow the previous system's
  if (d.row_off[0] != 0 || d.val_off[0] != 0) return BS_ERR_INVALID_ARG;
  for (int64_t s = 0; s < B; ++s) {
    if (d.row_off[s + 1] - d.row_off[s] != d.sys_rows[s]) return BS_ERR_INVALID_ARG;
    if (d.val_off[s + 1] - d.val_off[s] != nnz[d.sys_pat[s]]) return BS_ERR_INVALID_ARG;
  }
  finish_desc(d, longest);
  return BS_OK;
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
  std::vector<PatCsr> pats(n_patterns);
  std::vector<int> mark;
  for (int p = 0; p < n_patterns; ++p) {
    const int rc = pattern_from_csr(pat_rows[p], rowptr_all + pat_rowptr_off[p],
                                    col_all + pat_col_off[p], mark, pats[p]);
    if (rc != BS_OK) return rc;
  }
  return create_handle(n_batch, BS_CSR, pats, sys_pat, out);
}

int bs_varbatch_create_ell(int64_t n_batch, int32_t n_patterns, const int32_t* pat_rows,
                           const int32_t* pat_width, const int64_t* pat_col_off,
                           const int32_t* col_all, const int32_t* sys_pat, bs_varbatch* out) {
  if (!out || n_batch < 0 || n_patterns < 0 ||
      (n_patterns > 0 && (!pat_rows || !pat_width || !pat_col_off || !col_all)) ||
      (n_batch > 0 && !sys_pat))
    return BS_ERR_INVALID_ARG;
  if (n_batch > 0x7fffffff) return BS_ERR_UNSUPPORTED;
  *out = nullptr;
  std::vector<PatCsr> pats(n_patterns);
  std::vector<int> mark;
  for (int p = 0; p < n_patterns; ++p) {
    if (pat_col_off[p] < 0) return BS_ERR_INVALID_ARG;
    const int rc = pattern_from_ell(pat_rows[p], pat_width[p], col_all + pat_col_off[p], mark, pats[p]);
    if (rc != BS_OK) return rc;
  }
  return create_handle(n_batch, BS_ELL, pats, sys_pat, out);
}

int bs_varbatch_destroy(bs_varbatch v) {
  if (!v) return BS_OK;
  drop_graph(*v);
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
  if (total_rows) *total_rows = v->d.row_off.empty() ? 0 : v->d.row_off.back();
  if (total_values) *total_values = v->d.val_off.empty() ? 0 : v->d.val_off.back();
  if (n_tasks) *n_tasks = (int32_t)v->ts.tasks.size();
  if (policy) *policy = v->plan.policy;
  return BS_OK;
}

int bs_varbatch_set_policy(bs_varbatch v, int32_t policy) {
  if (!v || policy < 0 || policy >= kNumPolicies) return BS_ERR_INVALID_ARG;
  Plan pl;
  pl.policy = policy;
  if (same_plan(pl, v->plan)) return BS_OK;
  return apply_plan(*v, pl);
}

int bs_varbatch_set_plan(bs_varbatch v, const int32_t* class_codes) {
  if (!v || !class_codes) return BS_ERR_INVALID_ARG;
  Plan pl;
  pl.policy = -1;
  for (int c = 0; c < kNumClasses; ++c) {
    if (class_codes[c] < 0 || class_codes[c] >= kNumChoices) return BS_ERR_INVALID_ARG;
    pl.code[c] = class_codes[c];
  }
  if (same_plan(pl, v->plan)) return BS_OK;
  return apply_plan(*v, pl);
}

int bs_varbatch_get_plan(bs_varbatch v, int32_t* policy, int32_t* class_codes) {
  if (!v) return BS_ERR_INVALID_ARG;
  if (policy) *policy = v->plan.policy;
  if (class_codes)
    for (int c = 0; c < kNumClasses; ++c) class_codes[c] = v->plan.policy < 0 ? v->plan.code[c] : -1;
  return BS_OK;
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
  const std::string key = tune_key(v->d, solver, mixed, precond);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "r");
    if (f) {
      char k[512], tok[128];
      double t = 0;
      Plan found;
      bool have = false;
      while (std::fscanf(f, "%511s %127s %lf", k, tok, &t) == 3) {
        Plan pl;
        if (key == k && parse_plan(tok, pl)) {
          found = pl;
          have = true;
        }
      }
      std::fclose(f);
      if (have) {
        const int rc = same_plan(found, v->plan) ? BS_OK : apply_plan(*v, found);
        if (rc == BS_OK && report && report_len)
          std::snprintf(report, report_len, "policy=%s cached key=%s", plan_token(found).c_str(),
                        key.c_str());
        return rc;
      }
    }
  }
  // the task arrays are rewritten for every candidate: nothing queued on the
  // stream may still read them
  hipError_t se = hipStreamSynchronize(st);
  if (se != hipSuccess) return hip_err(se, "tune sync");
  // every timed solve starts from the caller's x0 (kept in a copy) unless the
  // flags say x0 = 0; the copy back is timed for every candidate alike
  const bool keep_x0 = !(opts && (opts->flags & BS_FLAG_X0_ZERO)) && v->d.B > 0 && x;
  const size_t xbytes = (size_t)(v->d.row_off.empty() ? 0 : v->d.row_off.back()) * sizeof(double);
  double* x0 = nullptr;
  if (keep_x0) {
    hipError_t e = hipMalloc(&x0, xbytes);
    if (e == hipSuccess) e = hipMemcpyAsync(x0, x, xbytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
      if (x0) (void)hipFree(x0);
      return hip_err(e, "tune x0 copy");
    }
  }
  auto run = [&](int only_class) -> int {
    if (keep_x0) {
      const hipError_t e = hipMemcpyAsync(x, x0, xbytes, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_err(e, "tune x0 restore");
    }
    return launch(*v, values, b, x, solver, precond, tol, max_iter, iters, resid, status, opts, st,
                  only_class);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BS_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = hip_err(hipGetLastError(), "tune events");
  // time of the current plan (one warm-up, then reps); < 0 when unsupported
  auto time_plan = [&](int only_class, double* ms_out) -> int {
    *ms_out = -1.0;
    int r = run(only_class);
    if (r == BS_ERR_UNSUPPORTED) return BS_OK;
    if (r != BS_OK) return r;
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps && r == BS_OK; ++i) r = run(only_class);
    (void)hipEventRecord(e1, st);
    if (r != BS_OK) return r;
    const hipError_t e = hipEventSynchronize(e1);
    if (e != hipSuccess) return hip_err(e, "tune sync");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms / reps;
    return BS_OK;
  };
  // 1. single launches: every policy
  double single[kNumPolicies];
  int best_single = -1;
  for (int p = 0; p < kNumPolicies && rc == BS_OK; ++p) {
    Plan pl;
    pl.policy = p;
    rc = apply_plan(*v, pl);
    if (rc == BS_OK) rc = time_plan(-1, &single[p]);
    if (rc == BS_OK && single[p] >= 0 && (best_single < 0 || single[p] < single[best_single]))
      best_single = p;
  }
  // 2. per-class launches: every choice for every class, each class timed alone
  double cls_ms[kNumClasses][kNumChoices];
  int best_code[kNumClasses];
  for (int c = 0; c < kNumClasses; ++c) best_code[c] = -1;
  for (int code = 0; code < kNumChoices && rc == BS_OK; ++code) {
    Plan pl;
    pl.policy = -1;
    for (int c = 0; c < kNumClasses; ++c) pl.code[c] = code;
    rc = apply_plan(*v, pl);
    for (int c = 0; c < kNumClasses && rc == BS_OK; ++c) {
      cls_ms[c][code] = -1.0;
      if (!v->d.cls_count[c]) continue;
      rc = time_plan(c, &cls_ms[c][code]);
      if (rc == BS_OK && cls_ms[c][code] >= 0 &&
          (best_code[c] < 0 || cls_ms[c][code] < cls_ms[c][best_code[c]]))
        best_code[c] = code;
    }
  }
  // 3. the per-class plan as a whole against the best single launch
  Plan split;
  split.policy = -1;
  bool split_ok = rc == BS_OK && v->d.B > 0;
  for (int c = 0; c < kNumClasses; ++c) {
    if (v->d.cls_count[c] && best_code[c] < 0) split_ok = false;
    split.code[c] = best_code[c] < 0 ? 0 : best_code[c];
  }
  double split_ms = -1.0;
  if (split_ok) {
    rc = apply_plan(*v, split);
    if (rc == BS_OK) rc = time_plan(-1, &split_ms);
  }
  Plan chosen;
  double chosen_ms = -1.0;
  if (best_single >= 0) {
    chosen.policy = best_single;
    chosen_ms = single[best_single];
  }
  if (split_ms >= 0 && (chosen_ms < 0 || split_ms < chosen_ms)) {
    chosen = split;
    chosen_ms = split_ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == BS_OK && chosen_ms < 0) rc = BS_ERR_UNSUPPORTED;
  if (rc == BS_OK) rc = apply_plan(*v, chosen);
  if (rc == BS_OK) rc = run(-1);  // outputs of the chosen plan
  if (x0) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(x0);
  }
  if (rc != BS_OK) return rc;
  if (report && report_len) {
    std::string t;
    for (int p = 0; p < kNumPolicies; ++p) {
      char buf[32];
      if (single[p] >= 0) std::snprintf(buf, sizeof buf, "%s%.4f", p ? "," : "", single[p]);
      else std::snprintf(buf, sizeof buf, "%s-", p ? "," : "");
      t += buf;
    }
    std::string cl;
    for (int c = 0; c < kNumClasses; ++c) {
      if (!v->d.cls_count[c] || best_code[c] < 0) continue;
      char buf[96];
      std::snprintf(buf, sizeof buf, "%s%d:%d=%s:%.4f", cl.empty() ? "" : ",", c, best_code[c],
                    choice_name(best_code[c]).c_str(), cls_ms[c][best_code[c]]);
      cl += buf;
    }
    std::snprintf(report, report_len, "policy=%s times_ms=%s classes=%s split_ms=%.4f key=%s",
                  plan_token(chosen).c_str(), t.c_str(), cl.empty() ? "-" : cl.c_str(), split_ms,
                  key.c_str());
  }
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %s %.6f\n", key.c_str(), plan_token(chosen).c_str(), chosen_ms);
      std::fclose(f);
    }
  }
  return BS_OK;
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
  drop_graph(*v);
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

size_t bs_varlen_workspace_size(int64_t n_batch) {
  if (n_batch < 0) return 0;
  return ws_layout(n_batch).total;
}

int bs_batch_solve_varlen(int64_t n_batch, const int32_t* sys_rows, const int64_t* row_off,
                          const int64_t* val_off, int32_t n_patterns, const int32_t* pat_id,
                          const int64_t* pat_rowptr_off, const int64_t* pat_col_off,
                          const int32_t* rowptr_all, const int32_t* col_all,
                          const double* values, const double* b, double* x, bs_solver solver,
                          bs_precond precond, double tol, int32_t max_iter, int32_t* iters,
                          double* resid, int32_t* status, const bs_options* opts, void* ws,
                          size_t ws_bytes, void* stream) {
  if (n_batch < 0 || n_patterns < 0) return BS_ERR_INVALID_ARG;
  if (n_batch > 0x7fffffff) return BS_ERR_UNSUPPORTED;
  if (n_batch == 0) return BS_OK;
  if (!sys_rows || !row_off || !val_off || !pat_id || n_patterns < 1 || !pat_rowptr_off ||
      !pat_col_off || !rowptr_all || !col_all || !ws)
    return BS_ERR_INVALID_ARG;
  const WsLayout wl = ws_layout(n_batch);
  if (ws_bytes < wl.total || ((uintptr_t)ws & 255)) return BS_ERR_INVALID_ARG;
  const int vp = opts ? opts->varlen_policy : 0;
  if (vp < 0 || vp > kNumPolicies) return BS_ERR_INVALID_ARG;
  int device = -1;
  int rc = have_device(&device);
  if (rc != BS_OK) return rc;
  const hipStream_t st = (hipStream_t)stream;
  VarKey key{};
  key.device = device;
  key.B = n_batch;
  key.P = n_patterns;
  key.generation = opts ? opts->structure_generation : 0;
  const void* ptrs[8] = {sys_rows, row_off, val_off, pat_id, pat_rowptr_off, pat_col_off,
                         rowptr_all, col_all};
  for (int i = 0; i < 8; ++i) key.ptr[i] = ptrs[i];
  std::lock_guard<std::mutex> lock(g_var_mu);
  VarEntry* ent = nullptr;
  for (VarEntry& e : g_var_cache)
    if (e.key == key) ent = &e;
  if (!ent) {
    VarEntry fresh;
    fresh.key = key;
    rc = read_batch(fresh.d, n_batch, sys_rows, row_off, val_off, n_patterns, pat_id,
                    pat_rowptr_off, pat_col_off, rowptr_all, col_all, st);
    if (rc != BS_OK) return rc;
    if (g_var_cache.size() >= kVarCacheEntries) {  // drop the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < g_var_cache.size(); ++i)
        if (g_var_cache[i].used < g_var_cache[lru].used) lru = i;
      g_var_cache.erase(g_var_cache.begin() + (long)lru);
    }
    g_var_cache.push_back(std::move(fresh));
    ent = &g_var_cache.back();
  }
  ent->used = ++g_var_clock;
  // policy 0 selects 512 lanes x 2 rows, streamed when a row is longer than
  // the register placement holds
  Plan pl;
  pl.policy = vp == 0 ? (ent->d.max_row <= 16 ? 3 : kNumRegPolicies + 3) : vp - 1;
  if (!ent->built || !same_plan(ent->plan, pl)) {
    build_tasks(ent->d, pl, ent->ts);
    rc = check_tasks(ent->d, pl, ent->ts);
    if (rc != BS_OK) return rc;
    ent->plan = pl;
    ent->built = true;
    ent->ws = nullptr;
  }
  char* w = static_cast<char*>(ws);
  if (ent->ws != ws || !same_plan(ent->ws_plan, pl)) {
    // the task queue into the caller's workspace (pageable source: the copy is
    // complete when the call returns)
    hipError_t e = hipMemcpyAsync(w + wl.tasks, ent->ts.tasks.data(),
                                  ent->ts.tasks.size() * sizeof(bs::VTask), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(w + wl.order, ent->ts.order.data(), ent->ts.order.size() * sizeof(int),
                         hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_err(e, "upload uneven-batch tasks");
    // another workspace may have held this entry's tasks: now only this one does
    for (VarEntry& o : g_var_cache)
      if (o.ws == ws) o.ws = nullptr;
    ent->ws = ws;
    ent->ws_plan = pl;
  }
  bs::VArgs a{};
  a.tasks = reinterpret_cast<const bs::VTask*>(w + wl.tasks);
  a.order = reinterpret_cast<const int*>(w + wl.order);
  a.sys_rows = sys_rows;
  a.sys_pat = pat_id;
  a.row_off = row_off;
  a.val_off = val_off;
  a.pat_rp = pat_rowptr_off;
  a.pat_col = pat_col_off;
  a.rowptr_all = rowptr_all;
  a.col_all = col_all;
  return launch(ent->d, a, ent->plan, ent->ts, device, reinterpret_cast<int*>(w + wl.counter),
                values, b, x, solver, precond, tol, max_iter, iters, resid, status, opts, st);
}

int bs_varbatch_replay(bs_varbatch v, void* stream) {
  if (!v || !v->gexec) return BS_ERR_INVALID_ARG;
  const hipError_t e = hipGraphLaunch(v->gexec, (hipStream_t)stream);
  return e == hipSuccess ? BS_OK : hip_err(e, "graph launch");
}

}  // extern "C"
