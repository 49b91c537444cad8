// Host side of the learned initial guess (bs_ws_*): model object, training
// workspace, and the launches of the kernels in bs_mlp_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/batchsolve.h"
#include "bs_mlp_kernels.hpp"

namespace bs {
void set_last_error(const std::string& msg);
}

using namespace bs::mlp;

namespace {

int hip_err(hipError_t e, const char* what) {
  bs::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
  return BS_ERR_HIP;
}

constexpr int kChunk = 512;  // samples per weight-gradient partial

}  // namespace

struct bs_ws_model_s {
  int n = 0, nnz = 0, F = 0, Fp = 0, O = 0, Op = 0;
  int64_t nparam = 0;
  int step = 0;  // Adam steps taken
  std::vector<int> diag_pos;
  // device: one allocation for parameters, optimiser state, BF16 copies, scaling
  char* d_model = nullptr;
  float *master = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  uint16_t *w1t = nullptr, *w2t = nullptr, *w3t = nullptr, *w2 = nullptr, *w3 = nullptr;
  double *mu_f = nullptr, *sd_f = nullptr, *sd_d = nullptr;  // mu_f | (mu_d) ... see fit
  double* moments = nullptr;  // [2][F + O]: means then standard deviations
  int* d_diag = nullptr;
  // training workspace (grown on demand)
  char* d_ws = nullptr;
  size_t ws_bytes = 0;
  int64_t ws_Mp = 0;
};

namespace {

Net net_of(const bs_ws_model_s& m) {
  Net t;
  t.n = m.n;
  t.F = m.F;
  t.Fp = m.Fp;
  t.O = m.O;
  t.Op = m.Op;
  t.w1t = m.w1t;
  t.w2t = m.w2t;
  t.w3t = m.w3t;
  t.w2 = m.w2;
  t.w3 = m.w3;
  const int64_t o_b1 = (int64_t)m.F * kH, o_b2 = o_b1 + kH + (int64_t)kH * kH;
  const int64_t o_b3 = o_b2 + kH + (int64_t)kH * m.O;
  t.b1 = m.master + o_b1;
  t.b2 = m.master + o_b2;
  t.b3 = m.master + o_b3;
  t.mu_f = m.moments;
  t.sd_f = m.moments + (m.F + m.O);
  t.sd_d = m.moments + (m.F + m.O) + m.F;
  return t;
}

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Training workspace of a step over Mp samples (a multiple of the tile) for
// features padded to Fp and outputs padded to Op: the activations and their
// gradients feature-major, the weight-gradient partials of every 512-sample
// chunk, the bias gradients and the per-tile losses.  Every region is written
// in full by the step before it is read, so none needs clearing.
struct WorkLayout {
  size_t zT, h1, h2, d1, d2, dy, part, bg, lp, total;
  int64_t part_off[3], part_ld;
};
constexpr WorkLayout work_layout(int Fp, int Op, int64_t Mp) {
  WorkLayout w{};
  const int64_t chunks = (Mp + kChunk - 1) / kChunk;
  w.part_off[0] = 0;
  w.part_off[1] = (int64_t)Fp * kH;
  w.part_off[2] = w.part_off[1] + (int64_t)kH * kH;
  w.part_ld = w.part_off[2] + (int64_t)kH * Op;
  size_t off = 0;
  w.zT = off; off = align256(off + (size_t)Fp * Mp * 2);
  w.h1 = off; off = align256(off + (size_t)kH * Mp * 2);
  w.h2 = off; off = align256(off + (size_t)kH * Mp * 2);
  w.d1 = off; off = align256(off + (size_t)kH * Mp * 2);
  w.d2 = off; off = align256(off + (size_t)kH * Mp * 2);
  w.dy = off; off = align256(off + (size_t)Op * Mp * 2);
  w.part = off; off = align256(off + (size_t)chunks * w.part_ld * 4);
  w.bg = off; off = align256(off + (size_t)(2 * kH + Op) * 4);
  w.lp = off; off = align256(off + (size_t)(Mp / kTile) * 4);
  w.total = off;
  return w;
}

// The workspace's regions at a base address.
struct Work {
  uint16_t *zT, *h1T, *h2T, *dz1T, *dz2T, *dyT;
  float *part, *bgrad, *loss_part;
  int64_t part_ld, part_off[3];
};
Work work_at(char* base, const WorkLayout& l) {
  Work w;
  w.zT = (uint16_t*)(base + l.zT);
  w.h1T = (uint16_t*)(base + l.h1);
  w.h2T = (uint16_t*)(base + l.h2);
  w.dz1T = (uint16_t*)(base + l.d1);
  w.dz2T = (uint16_t*)(base + l.d2);
  w.dyT = (uint16_t*)(base + l.dy);
  w.part = (float*)(base + l.part);
  w.bgrad = (float*)(base + l.bg);
  w.loss_part = (float*)(base + l.lp);
  w.part_ld = l.part_ld;
  for (int L = 0; L < 3; ++L) w.part_off[L] = l.part_off[L];
  return w;
}

// The model's own workspace for M samples, grown (reallocated) on demand.
int ensure_ws(bs_ws_model_s& m, int64_t M, Work* out) {
  const int64_t Mp = (M + kTile - 1) / kTile * kTile;
  if (!m.d_ws || Mp > m.ws_Mp) {
    const WorkLayout l = work_layout(m.Fp, m.Op, Mp);
    if (m.d_ws) (void)hipFree(m.d_ws);
    m.d_ws = nullptr;
    hipError_t e = hipMalloc(&m.d_ws, l.total);
    if (e != hipSuccess) {
      m.ws_Mp = 0;
      return hip_err(e, "learned-start workspace");
    }
    m.ws_bytes = l.total;
    m.ws_Mp = Mp;
  }
  *out = work_at(m.d_ws, work_layout(m.Fp, m.Op, Mp));
  return BS_OK;
}

Apply apply_of(bs_ws_model_s& m) {
  Apply a;
  std::memset(&a, 0, sizeof a);
  a.F = m.F;
  a.Fp = m.Fp;
  a.O = m.O;
  a.Op = m.Op;
  a.nparam = m.nparam;
  a.master = m.master;
  a.m = m.adam_m;
  a.v = m.adam_v;
  a.w1t = m.w1t;
  a.w2t = m.w2t;
  a.w3t = m.w3t;
  a.w2 = m.w2;
  a.w3 = m.w3;
  return a;
}

hipError_t launch_apply(const Apply& a, hipStream_t st) {
  const unsigned grid = (unsigned)((a.nparam + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_mlp_apply, dim3(grid), dim3(kWG), 0, st, a);
  return hipGetLastError();
}

// Forward + backward over M samples and the gradient gather (and an Adam step
// if update): the shared body of bs_ws_grad and bs_ws_train_step.
int run_grad(bs_ws_model_s& m, const Work& w, int64_t M, const float* feat, const float* delta,
             const int* rows, float* grad_out, float* loss_out, int update, float lr,
             hipStream_t st) {
  const int64_t Mp = (M + kTile - 1) / kTile * kTile;
  const int tiles = (int)(Mp / kTile);
  Src src;
  std::memset(&src, 0, sizeof src);
  src.feat = feat;
  src.delta = delta;
  src.rows = rows;
  Train tr;
  tr.M = M;
  tr.Mp = Mp;
  tr.zT = w.zT;
  tr.h1T = w.h1T;
  tr.h2T = w.h2T;
  tr.dz1T = w.dz1T;
  tr.dz2T = w.dz2T;
  tr.dyT = w.dyT;
  tr.loss_part = w.loss_part;
  tr.y_out = nullptr;
  hipLaunchKernelGGL(k_mlp<kTrain>, dim3(tiles), dim3(kWG), 0, st, net_of(m), src, tr, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "learned-start forward/backward");
  WGrad g;
  g.aT[0] = w.zT;
  g.aT[1] = w.h1T;
  g.aT[2] = w.h2T;
  g.dT[0] = w.dz1T;
  g.dT[1] = w.dz2T;
  g.dT[2] = w.dyT;
  g.kin[0] = m.Fp;
  g.kin[1] = kH;
  g.kin[2] = kH;
  g.nout[0] = kH;
  g.nout[1] = kH;
  g.nout[2] = m.Op;
  int start = 0;
  for (int L = 0; L < 3; ++L) {
    g.tiles_c[L] = g.nout[L] / 32;
    g.tile_start[L] = start;
    start += (g.kin[L] / 64) * g.tiles_c[L];
  }
  g.tile_start[3] = start;
  for (int L = 0; L < 3; ++L) g.part_off[L] = w.part_off[L];
  g.part_ld = w.part_ld;
  g.Mp = Mp;
  g.chunk = kChunk;
  g.part = w.part;
  const int chunks = (int)((Mp + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(start, chunks), dim3(kWG), 0, st, g);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "learned-start weight gradients");
  BGrad bg;
  bg.dT[0] = w.dz1T;
  bg.dT[1] = w.dz2T;
  bg.dT[2] = w.dyT;
  bg.rows[0] = kH;
  bg.rows[1] = kH;
  bg.rows[2] = m.Op;
  bg.Mp = Mp;
  bg.out = w.bgrad;
  hipLaunchKernelGGL(k_mlp_bgrad, dim3(2 * kH + m.Op), dim3(kWG), 0, st, bg);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "learned-start bias gradients");
  if (loss_out) {
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(64), 0, st, w.loss_part, tiles,
                       1.0 / ((double)M * m.O), loss_out);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "learned-start loss");
  }
  Apply a = apply_of(m);
  a.part = w.part;
  a.part_ld = w.part_ld;
  for (int L = 0; L < 3; ++L) a.part_off[L] = w.part_off[L];
  a.chunks = chunks;
  a.bgrad = w.bgrad;
  a.grad_out = grad_out;
  a.update = update;
  if (update) {
    const int t = m.step + 1;
    a.lr = lr;
    a.c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
    a.c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
  }
  e = launch_apply(a, st);
  if (e != hipSuccess) return hip_err(e, "learned-start update");
  if (update) ++m.step;
  return BS_OK;
}

}  // namespace

namespace {

// Workspace of bs_ws_train_step_noalloc: a file-scope device array sized for
// the largest step it takes (2048 samples of the largest model, n = 64:
// features padded to 192, outputs to 64), about 7 MiB on every device the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel: its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int64_t kScratchSamples = 2048;
constexpr size_t kScratchBytes =
    work_layout(round_up(3 * kMaxN, 64), round_up(kMaxN, 32), kScratchSamples).total;

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// This device's address of `scratch` (looked up once per device).
int scratch_base(char** out) {
  static std::mutex mu;
  static std::vector<char*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)");
    addr[dev] = static_cast<char*>(p);
  }
  *out = addr[dev];
  return BS_OK;
}

// Packed inference weights (bs_ws_pack / bs_ws_infer_packed): for systems of
// n unknowns, regions in this order, each starting at a multiple of 256 bytes:
// W1^T BF16 [256][Fp], W2^T BF16 [256][256], W3^T BF16 [Op][256], b1 FP32
// [256], b2 FP32 [256], b3 FP32 [n], feature means FP64 [3n], feature
// deviations FP64 [3n], sigma_d FP64 [n]; Fp = 3n rounded up to 64, Op = n
// rounded up to 32 (padding entries zero).
struct Packed {
  size_t w1t, w2t, w3t, b1, b2, b3, mu, sd, sdd, total;
};
Packed packed_layout(int n) {
  const int F = 3 * n, Fp = round_up(F, 64), Op = round_up(n, 32);
  Packed p;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off = align256(off + bytes); return at; };
  p.w1t = take((size_t)kH * Fp * 2);
  p.w2t = take((size_t)kH * kH * 2);
  p.w3t = take((size_t)Op * kH * 2);
  p.b1 = take((size_t)kH * 4);
  p.b2 = take((size_t)kH * 4);
  p.b3 = take((size_t)n * 4);
  p.mu = take((size_t)F * 8);
  p.sd = take((size_t)F * 8);
  p.sdd = take((size_t)n * 8);
  p.total = off;
  return p;
}

}  // namespace

extern "C" {

int bs_ws_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                 bs_ws_model* out) {
  if (!out || n < 1 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx)) return BS_ERR_INVALID_ARG;
  *out = nullptr;
  if (n > kMaxN) return BS_ERR_UNSUPPORTED;
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return BS_ERR_PATTERN;
  std::vector<int> dpos(n, -1);
  for (int i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return BS_ERR_PATTERN;
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      if (col_idx[k] < 0 || col_idx[k] >= n) return BS_ERR_PATTERN;
      if (col_idx[k] == i) dpos[i] = k;
    }
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    bs::set_last_error("no HIP device");
    return BS_ERR_NO_DEVICE;
  }
  bs_ws_model_s* m = new bs_ws_model_s();
  m->n = n;
  m->nnz = nnz;
  m->F = 3 * n;
  m->Fp = round_up(m->F, 64);
  m->O = n;
  m->Op = round_up(n, 32);
  m->nparam = (int64_t)m->F * kH + kH + (int64_t)kH * kH + kH + (int64_t)kH * m->O + m->O;
  m->diag_pos = dpos;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off = align256(off + bytes); return at; };
  const size_t o_master = take(m->nparam * 4), o_m = take(m->nparam * 4), o_v = take(m->nparam * 4),
               o_w1t = take((size_t)kH * m->Fp * 2), o_w2t = take((size_t)kH * kH * 2),
               o_w3t = take((size_t)m->Op * kH * 2), o_w2 = take((size_t)kH * kH * 2),
               o_w3 = take((size_t)kH * m->Op * 2), o_mom = take((size_t)2 * (m->F + m->O) * 8),
               o_diag = take((size_t)n * 4);
  hipError_t e = hipMalloc(&m->d_model, off);
  if (e == hipSuccess) e = hipMemset(m->d_model, 0, off);
  if (e != hipSuccess) {
    if (m->d_model) (void)hipFree(m->d_model);
    delete m;
    return hip_err(e, "learned-start model allocation");
  }
  char* d = m->d_model;
  m->master = (float*)(d + o_master);
  m->adam_m = (float*)(d + o_m);
  m->adam_v = (float*)(d + o_v);
  m->w1t = (uint16_t*)(d + o_w1t);
  m->w2t = (uint16_t*)(d + o_w2t);
  m->w3t = (uint16_t*)(d + o_w3t);
  m->w2 = (uint16_t*)(d + o_w2);
  m->w3 = (uint16_t*)(d + o_w3);
  m->moments = (double*)(d + o_mom);
  m->d_diag = (int*)(d + o_diag);
  // unit scaling until fit: means 0, standard deviations 1
  std::vector<double> mom(2 * (m->F + m->O), 0.0);
  for (int c = 0; c < m->F + m->O; ++c) mom[m->F + m->O + c] = 1.0;
  e = hipMemcpy(m->moments, mom.data(), mom.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_diag, dpos.data(), n * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    bs_ws_destroy(m);
    return hip_err(e, "learned-start model upload");
  }
  *out = m;
  return BS_OK;
}

int bs_ws_destroy(bs_ws_model m) {
  if (!m) return BS_OK;
  if (m->d_ws) (void)hipFree(m->d_ws);
  if (m->d_model) (void)hipFree(m->d_model);
  delete m;
  return BS_OK;
}

int bs_ws_param_count(bs_ws_model m, int64_t* count) {
  if (!m || !count) return BS_ERR_INVALID_ARG;
  *count = m->nparam;
  return BS_OK;
}

int bs_ws_set_params(bs_ws_model m, const float* host) {
  if (!m || !host) return BS_ERR_INVALID_ARG;
  hipError_t e = hipMemcpy(m->master, host, m->nparam * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->adam_m, 0, m->nparam * 4);
  if (e == hipSuccess) e = hipMemset(m->adam_v, 0, m->nparam * 4);
  if (e != hipSuccess) return hip_err(e, "learned-start parameters");
  m->step = 0;
  e = launch_apply(apply_of(*m), 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start weight copies");
}

int bs_ws_get_params(bs_ws_model m, float* host) {
  if (!m || !host) return BS_ERR_INVALID_ARG;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host, m->master, m->nparam * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start parameters");
}

int bs_ws_features(bs_ws_model m, int64_t n_batch, const double* values, const double* b,
                   const double* x_prev, const double* x_next, float* feat, float* delta,
                   void* stream) {
  if (!m || n_batch < 0) return BS_ERR_INVALID_ARG;
  if (n_batch == 0) return BS_OK;
  if (!values || !b || !x_prev || !feat || (x_next && !delta)) return BS_ERR_INVALID_ARG;
  const int64_t total = n_batch * (m->F + (x_next ? m->O : 0));
  const unsigned grid = (unsigned)std::min<int64_t>((total + kWG - 1) / kWG, 65536);
  hipLaunchKernelGGL(k_mlp_features, dim3(grid), dim3(kWG), 0, (hipStream_t)stream, n_batch, m->n,
                     m->nnz, m->d_diag, values, b, x_prev, x_next, feat, delta);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start features");
}

int bs_ws_fit_scaling(bs_ws_model m, int64_t n_samples, const float* feat, const float* delta,
                      void* stream) {
  if (!m || n_samples < 1 || !feat || !delta) return BS_ERR_INVALID_ARG;
  const hipStream_t st = (hipStream_t)stream;
  const int ncol = m->F + m->O;
  const int64_t chunk = 4096;
  const int chunks = (int)((n_samples + chunk - 1) / chunk);
  double* part = nullptr;
  double* mean = nullptr;
  hipError_t e = hipMalloc(&part, (size_t)chunks * ncol * 8);
  if (e == hipSuccess) e = hipMalloc(&mean, (size_t)ncol * 8);
  if (e != hipSuccess) {
    if (part) (void)hipFree(part);
    return hip_err(e, "learned-start scaling workspace");
  }
  hipLaunchKernelGGL(k_mlp_moments, dim3(chunks), dim3(kWG), 0, st, n_samples, m->F, m->O, feat,
                     delta, (const double*)nullptr, chunk, part);
  hipLaunchKernelGGL(k_mlp_moments_final, dim3(1), dim3(kWG), 0, st, chunks, ncol, n_samples,
                     (const double*)part, 0, mean);
  hipLaunchKernelGGL(k_mlp_moments, dim3(chunks), dim3(kWG), 0, st, n_samples, m->F, m->O, feat,
                     delta, (const double*)mean, chunk, part);
  hipLaunchKernelGGL(k_mlp_moments_final, dim3(1), dim3(kWG), 0, st, chunks, ncol, n_samples,
                     (const double*)part, 1, m->moments + ncol);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->moments, mean, (size_t)ncol * 8, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  (void)hipFree(mean);
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start scaling");
}

int bs_ws_get_scaling(bs_ws_model m, double* mu_f, double* sd_f, double* sd_d) {
  if (!m) return BS_ERR_INVALID_ARG;
  std::vector<double> mom(2 * (m->F + m->O));
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(mom.data(), m->moments, mom.size() * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_err(e, "learned-start scaling");
  const int c = m->F + m->O;
  if (mu_f) std::memcpy(mu_f, mom.data(), m->F * 8);
  if (sd_f) std::memcpy(sd_f, mom.data() + c, m->F * 8);
  if (sd_d) std::memcpy(sd_d, mom.data() + c + m->F, m->O * 8);
  return BS_OK;
}

int bs_ws_set_scaling(bs_ws_model m, const double* mu_f, const double* sd_f, const double* sd_d) {
  if (!m || !mu_f || !sd_f || !sd_d) return BS_ERR_INVALID_ARG;
  const int c = m->F + m->O;
  std::vector<double> mom(2 * c, 0.0);
  for (int i = 0; i < m->F; ++i) {
    if (!(sd_f[i] > 0.0) || !std::isfinite(sd_f[i]) || !std::isfinite(mu_f[i])) return BS_ERR_INVALID_ARG;
    mom[i] = mu_f[i];
    mom[c + i] = sd_f[i];
  }
  for (int i = 0; i < m->O; ++i) {
    if (!(sd_d[i] > 0.0) || !std::isfinite(sd_d[i])) return BS_ERR_INVALID_ARG;
    mom[c + m->F + i] = sd_d[i];
  }
  const hipError_t e = hipMemcpy(m->moments, mom.data(), mom.size() * 8, hipMemcpyHostToDevice);
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start scaling");
}

int bs_ws_forward(bs_ws_model m, int64_t n_samples, const float* feat, const int32_t* rows,
                  float* y, void* stream) {
  if (!m || n_samples < 0) return BS_ERR_INVALID_ARG;
  if (n_samples == 0) return BS_OK;
  if (!feat || !y) return BS_ERR_INVALID_ARG;
  Src src;
  std::memset(&src, 0, sizeof src);
  src.feat = feat;
  src.rows = rows;
  Train tr;
  std::memset(&tr, 0, sizeof tr);
  tr.M = n_samples;
  tr.y_out = y;
  const unsigned tiles = (unsigned)((n_samples + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_mlp<kForward>, dim3(tiles), dim3(kWG), 0, (hipStream_t)stream, net_of(*m),
                     src, tr, n_samples);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start forward");
}

int bs_ws_grad(bs_ws_model m, int64_t n_samples, const float* feat, const float* delta,
               const int32_t* rows, float* grad, float* loss, void* stream) {
  if (!m || !grad) return BS_ERR_INVALID_ARG;
  if (n_samples < 1 || !feat || !delta) return BS_ERR_INVALID_ARG;
  Work w;
  const int rc = ensure_ws(*m, n_samples, &w);
  if (rc != BS_OK) return rc;
  return run_grad(*m, w, n_samples, feat, delta, rows, grad, loss, 0, 0.f, (hipStream_t)stream);
}

int bs_ws_train_step(bs_ws_model m, int64_t n_samples, const float* feat, const float* delta,
                     const int32_t* rows, float lr, float* loss, void* stream) {
  if (!m || !(lr > 0.f) || !std::isfinite(lr)) return BS_ERR_INVALID_ARG;
  if (n_samples < 1 || !feat || !delta) return BS_ERR_INVALID_ARG;
  Work w;
  const int rc = ensure_ws(*m, n_samples, &w);
  if (rc != BS_OK) return rc;
  return run_grad(*m, w, n_samples, feat, delta, rows, nullptr, loss, 1, lr, (hipStream_t)stream);
}

int bs_ws_train_step_noalloc(bs_ws_model m, int64_t n_samples, const float* feat,
                             const float* delta, const int32_t* rows, float lr, float* loss,
                             void* stream) {
  if (!m || !(lr > 0.f) || !std::isfinite(lr)) return BS_ERR_INVALID_ARG;
  if (n_samples < 1 || !feat || !delta) return BS_ERR_INVALID_ARG;
  if (n_samples > kScratchSamples) {
    bs::set_last_error("bs_ws_train_step_noalloc: more than 2048 samples");
    return BS_ERR_UNSUPPORTED;
  }
  char* base = nullptr;
  const int rc = scratch_base(&base);
  if (rc != BS_OK) return rc;
  const int64_t Mp = (n_samples + kTile - 1) / kTile * kTile;
  const WorkLayout l = work_layout(m->Fp, m->Op, Mp);
  if (l.total > kScratchBytes) return BS_ERR_UNSUPPORTED;  // cannot happen for n <= 64
  return run_grad(*m, work_at(base, l), n_samples, feat, delta, rows, nullptr, loss, 1, lr,
                  (hipStream_t)stream);
}

int bs_ws_infer(bs_ws_model m, int64_t n_batch, const double* values, const double* b,
                const double* x_prev, double* x0, void* stream) {
  if (!m || n_batch < 0) return BS_ERR_INVALID_ARG;
  if (n_batch == 0) return BS_OK;
  if (!values || !b || !x_prev || !x0) return BS_ERR_INVALID_ARG;
  Src src;
  std::memset(&src, 0, sizeof src);
  src.nnz = m->nnz;
  src.diag_pos = m->d_diag;
  src.values = values;
  src.b = b;
  src.x_prev = x_prev;
  src.x0 = x0;
  Train tr;
  std::memset(&tr, 0, sizeof tr);
  tr.M = n_batch;
  const unsigned tiles = (unsigned)((n_batch + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_mlp<kInfer>, dim3(tiles), dim3(kWG), 0, (hipStream_t)stream, net_of(*m), src,
                     tr, n_batch);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start inference");
}

size_t bs_ws_packed_bytes(int32_t n) {
  if (n < 1 || n > kMaxN) return 0;
  return packed_layout(n).total;
}

int bs_ws_pack(bs_ws_model m, void* weights, size_t bytes, void* stream) {
  if (!m || !weights) return BS_ERR_INVALID_ARG;
  const Packed p = packed_layout(m->n);
  if (bytes < p.total || ((uintptr_t)weights & 255)) return BS_ERR_INVALID_ARG;
  char* w = static_cast<char*>(weights);
  const Net t = net_of(*m);
  const hipStream_t st = (hipStream_t)stream;
  struct Piece { size_t dst; const void* src; size_t bytes; };
  const Piece pieces[] = {
      {p.w1t, t.w1t, (size_t)kH * m->Fp * 2}, {p.w2t, t.w2t, (size_t)kH * kH * 2},
      {p.w3t, t.w3t, (size_t)m->Op * kH * 2}, {p.b1, t.b1, (size_t)kH * 4},
      {p.b2, t.b2, (size_t)kH * 4},           {p.b3, t.b3, (size_t)m->O * 4},
      {p.mu, t.mu_f, (size_t)m->F * 8},       {p.sd, t.sd_f, (size_t)m->F * 8},
      {p.sdd, t.sd_d, (size_t)m->O * 8}};
  for (const Piece& q : pieces) {
    const hipError_t e = hipMemcpyAsync(w + q.dst, q.src, q.bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_err(e, "pack learned-start weights");
  }
  return BS_OK;
}

int bs_ws_infer_packed(int64_t n_batch, int32_t n, const void* weights, const double* diag,
                       const double* b, const double* x_prev, double* x0, void* stream) {
  if (n_batch < 0 || n < 1) return BS_ERR_INVALID_ARG;
  if (n > kMaxN) return BS_ERR_UNSUPPORTED;
  if (n_batch == 0) return BS_OK;
  if (!weights || !diag || !b || !x_prev || !x0 || ((uintptr_t)weights & 255))
    return BS_ERR_INVALID_ARG;
  const Packed p = packed_layout(n);
  const char* w = static_cast<const char*>(weights);
  Net t;
  std::memset(&t, 0, sizeof t);
  t.n = n;
  t.F = 3 * n;
  t.Fp = round_up(t.F, 64);
  t.O = n;
  t.Op = round_up(n, 32);
  t.w1t = reinterpret_cast<const uint16_t*>(w + p.w1t);
  t.w2t = reinterpret_cast<const uint16_t*>(w + p.w2t);
  t.w3t = reinterpret_cast<const uint16_t*>(w + p.w3t);
  t.b1 = reinterpret_cast<const float*>(w + p.b1);
  t.b2 = reinterpret_cast<const float*>(w + p.b2);
  t.b3 = reinterpret_cast<const float*>(w + p.b3);
  t.mu_f = reinterpret_cast<const double*>(w + p.mu);
  t.sd_f = reinterpret_cast<const double*>(w + p.sd);
  t.sd_d = reinterpret_cast<const double*>(w + p.sdd);
  Src src;
  std::memset(&src, 0, sizeof src);
  src.diag = diag;
  src.b = b;
  src.x_prev = x_prev;
  src.x0 = x0;
  Train tr;
  std::memset(&tr, 0, sizeof tr);
  tr.M = n_batch;
  const unsigned tiles = (unsigned)((n_batch + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_mlp<kInfer>, dim3(tiles), dim3(kWG), 0, (hipStream_t)stream, t, src, tr,
                     n_batch);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BS_OK : hip_err(e, "learned-start inference (packed weights)");
}

}  // extern "C"
