// Kernels of the learned initial guess (see bs_mlp.hpp for the layouts).
#pragma once
#include "bs_mlp.hpp"

namespace bs {
namespace mlp {

constexpr int kLdZ = 192 + kPad;   // Z tile row stride (features padded to 192 at most)
constexpr int kLdH = kH + kPad;    // hidden tile row stride
constexpr int kLdY = 64 + kPad;    // output-gradient tile row stride

enum Mode { kInfer = 0, kForward = 1, kTrain = 2 };

// LDS of the fused kernel.  Inference and forward keep two buffers (Z, later
// overwritten by H2, and H1); training keeps Z, H1, H2, dZ2 and dY.
template <int MODE>
struct Smem {
  static constexpr int kZ = MODE == kTrain ? kTile * kLdZ : kTile * kLdH;
  static constexpr int kH1 = kTile * kLdH;
  static constexpr int kH2 = MODE == kTrain ? kTile * kLdH : 0;
  static constexpr int kD = MODE == kTrain ? kTile * kLdH : 0;
  static constexpr int kDY = MODE == kTrain ? kTile * kLdY : 0;
  static constexpr int kTotal = kZ + kH1 + kH2 + kD + kDY;  // uint16 elements
};

// Four consecutive rows (4q .. 4q+3 of row block rb) of one column, packed
// for an 8-byte store into a feature-major [column][Mp] array.
__device__ __forceinline__ void store_col4(uint16_t* dstT, int64_t Mp, int col, int64_t m,
                                           const uint16_t (&h)[4]) {
  uint2 v;
  v.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
  v.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
  *reinterpret_cast<uint2*>(dstT + (size_t)col * Mp + m) = v;
}

template <int MODE>
__global__ __launch_bounds__(kWG) void k_mlp(const Net net, const Src src, const Train tr,
                                             int64_t M) {
  using S = Smem<MODE>;
  __shared__ __align__(16) uint16_t sm[S::kTotal];
  __shared__ float s_loss[kWG / 64];
  uint16_t* sZ = sm;
  uint16_t* sH1 = sm + S::kZ;
  // inference reuses the Z buffer for H2 (Z is dead after the first layer)
  uint16_t* sH2 = MODE == kTrain ? sH1 + S::kH1 : sZ;
  uint16_t* sD = sH2 + S::kH2;
  uint16_t* sDY = sD + S::kD;
  const int ldz = MODE == kTrain ? kLdZ : kLdH;

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, r16 = l & 15, q = l >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * kTile;
  const int n = net.n, F = net.F, Fp = net.Fp, O = net.O, Op = net.Op;

  // ---- normalised features of the tile -> BF16
  if constexpr (MODE == kInfer) {
    // wave w builds rows 16w .. 16w+15, lane l features l, l+64, .. (< Fp): the
    // loads of a feature's 16 rows are issued together, consecutive lanes read
    // consecutive elements, and the spread's reciprocal is taken once
    for (int f = l; f < Fp; f += 64) {
      const bool fok = f < F;
      const int kind = f < n ? 0 : f < 2 * n ? 1 : 2;
      const int j = f - kind * n;
      const double mu = fok ? net.mu_f[f] : 0.0;
      const double isd = fok ? 1.0 / net.sd_f[f] : 0.0;
      const int p = (fok && kind == 0 && !src.diag) ? src.diag_pos[f] : -1;
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t m = m0 + 16 * w + i;
        double t = 0.0;
        if (fok && m < M) {
          if (kind == 0) t = src.diag ? src.diag[m * n + j] : p >= 0 ? src.values[m * src.nnz + p] : 0.0;
          else if (kind == 1) t = src.b[m * n + j] - src.x_prev[m * n + j];
          else t = src.x_prev[m * n + j];
        }
        v[i] = t;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const bool ok = fok && m0 + 16 * w + i < M;
        sZ[(16 * w + i) * ldz + f] = to_bf16(ok ? (float)((v[i] - mu) * isd) : 0.f);
      }
    }
  } else {
    // training and forward: the raw FP32 features of the (listed) samples
    for (int idx = tid; idx < kTile * Fp; idx += kWG) {
      const int row = idx / Fp, f = idx - row * Fp;
      const int64_t m = m0 + row;
      float z = 0.f;
      if (f < F && m < M) {
        const int64_t s = src.rows ? (int64_t)src.rows[m] : m;
        const double v = (double)src.feat[s * F + f];
        z = (float)((v - net.mu_f[f]) / net.sd_f[f]);
      }
      sZ[row * ldz + f] = to_bf16(z);
    }
  }
  __syncthreads();
  if constexpr (MODE == kTrain) {  // Z feature-major for the first layer's weight gradient
    for (int idx = tid; idx < kTile * Fp; idx += kWG) {
      const int f = idx / kTile, row = idx - f * kTile;
      tr.zT[(size_t)f * tr.Mp + m0 + row] = sZ[row * ldz + f];
    }
  }

  // ---- layer 1: H1 = relu(Z W1 + b1); wave w owns columns 64w .. 64w+63
  {
    floatx4 acc[4][4];
    zero(acc);
    gemm_tile<4, 4>(acc, sZ, ldz, net.w1t, Fp, 64 * w, Fp);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int col = 64 * w + 16 * cb + r16;
        const float bias = net.b1[col];
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          h[i] = to_bf16(fmaxf(acc[rb][cb][i] + bias, 0.f));
          sH1[(16 * rb + 4 * q + i) * kLdH + col] = h[i];
        }
        if constexpr (MODE == kTrain) store_col4(tr.h1T, tr.Mp, col, m0 + 16 * rb + 4 * q, h);
      }
  }
  __syncthreads();

  // ---- layer 2: H2 = relu(H1 W2 + b2)
  {
    floatx4 acc[4][4];
    zero(acc);
    gemm_tile<4, 4>(acc, sH1, kLdH, net.w2t, kH, 64 * w, kH);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int col = 64 * w + 16 * cb + r16;
        const float bias = net.b2[col];
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          h[i] = to_bf16(fmaxf(acc[rb][cb][i] + bias, 0.f));
          sH2[(16 * rb + 4 * q + i) * kLdH + col] = h[i];
        }
        if constexpr (MODE == kTrain) store_col4(tr.h2T, tr.Mp, col, m0 + 16 * rb + 4 * q, h);
      }
  }
  __syncthreads();

  // ---- layer 3: Y = H2 W3 + b3; wave w owns columns 16w .. 16w+15 (Op <= 64)
  float sq = 0.f;
  if (16 * w < Op) {
    floatx4 acc[4][1];
    zero(acc);
    gemm_tile<4, 1>(acc, sH2, kLdH, net.w3t, kH, 16 * w, kH);
    const int col = 16 * w + r16;
    const bool cok = col < O;
    const float bias = cok ? net.b3[col] : 0.f;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      uint16_t dh[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * rb + 4 * q + i;
        const int64_t m = m0 + row;
        const bool ok = cok && m < M;
        const float y = acc[rb][0][i] + bias;
        if constexpr (MODE == kInfer) {
          if (ok) src.x0[m * n + col] = src.x_prev[m * n + col] + net.sd_d[col] * (double)y;
        } else {
          if (ok && tr.y_out) tr.y_out[m * O + col] = y;
        }
        if constexpr (MODE == kTrain) {
          float g = 0.f;
          if (ok) {
            const int64_t s = src.rows ? (int64_t)src.rows[m] : m;
            const float t = (float)((double)src.delta[s * O + col] / net.sd_d[col]);
            const float e = y - t;
            sq += e * e;
            g = 2.f * e / (float)((double)M * O);
          }
          dh[i] = to_bf16(g);
          sDY[row * kLdY + col] = dh[i];
        }
      }
      if constexpr (MODE == kTrain) store_col4(tr.dyT, tr.Mp, col, m0 + 16 * rb + 4 * q, dh);
    }
  }
  if constexpr (MODE != kTrain) return;

  // ---- loss of the tile (fixed-order sums: deterministic)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
  if (l == 0) s_loss[w] = sq;
  __syncthreads();
  if (tid == 0) tr.loss_part[blockIdx.x] = ((s_loss[0] + s_loss[1]) + (s_loss[2] + s_loss[3]));

  // ---- dZ2 = (dY W3^T) * [H2 > 0]
  {
    floatx4 acc[4][4];
    zero(acc);
    gemm_tile<4, 4>(acc, sDY, kLdY, net.w3, Op, 64 * w, Op);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int col = 64 * w + 16 * cb + r16;
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * rb + 4 * q + i;
          const bool on = from_bf16(sH2[row * kLdH + col]) > 0.f;
          h[i] = to_bf16(on ? acc[rb][cb][i] : 0.f);
          sD[row * kLdH + col] = h[i];
        }
        store_col4(tr.dz2T, tr.Mp, col, m0 + 16 * rb + 4 * q, h);
      }
  }
  __syncthreads();

  // ---- dZ1 = (dZ2 W2^T) * [H1 > 0]
  {
    floatx4 acc[4][4];
    zero(acc);
    gemm_tile<4, 4>(acc, sD, kLdH, net.w2, kH, 64 * w, kH);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int col = 64 * w + 16 * cb + r16;
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * rb + 4 * q + i;
          const bool on = from_bf16(sH1[row * kLdH + col]) > 0.f;
          h[i] = to_bf16(on ? acc[rb][cb][i] : 0.f);
        }
        store_col4(tr.dz1T, tr.Mp, col, m0 + 16 * rb + 4 * q, h);
      }
  }
}

// ---------------------------------------------------------------- weight gradients
// dW_l[k_in][n_out] = sum_m A_l[m][k_in] dZ_l[m][n_out] over one chunk of
// samples per blockIdx.y; tiles of 64 x 32 over the three layers on
// blockIdx.x.  FP32 partials per chunk, summed in order by k_mlp_apply.
struct WGrad {
  const uint16_t* aT[3];   // Z^T, H1^T, H2^T
  const uint16_t* dT[3];   // dZ1^T, dZ2^T, dY^T
  int kin[3];              // Fp, kH, kH
  int nout[3];             // kH, kH, Op
  int tiles_c[3];          // column tiles per layer
  int tile_start[4];       // first tile of each layer (prefix sums)
  int64_t part_off[3];     // offset of each layer's block in a chunk's partials
  int64_t part_ld;         // floats per chunk
  int64_t Mp;
  int chunk;               // samples per blockIdx.y (multiple of 32)
  float* part;
};

__global__ __launch_bounds__(kWG) void k_mlp_wgrad(const WGrad g) {
  const int t = blockIdx.x;
  const int layer = t < g.tile_start[1] ? 0 : (t < g.tile_start[2] ? 1 : 2);
  const int lt = t - g.tile_start[layer];
  const int tr = lt / g.tiles_c[layer], tc = lt - tr * g.tiles_c[layer];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
  const int r0 = 64 * tr + 16 * w, c0 = 32 * tc;
  const int64_t k_begin = (int64_t)blockIdx.y * g.chunk;
  const int64_t k_end = min(k_begin + g.chunk, g.Mp);
  const uint16_t* A = g.aT[layer] + (size_t)(r0 + r16) * g.Mp;
  const uint16_t* D = g.dT[layer];
  floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
  for (int64_t k0 = k_begin; k0 < k_end; k0 += 32) {
    const bf16x8 a = frag(A + k0 + 8 * q);
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const bf16x8 b = frag(D + (size_t)(c0 + 16 * cb + r16) * g.Mp + k0 + 8 * q);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
    }
  }
  float* out = g.part + (size_t)blockIdx.y * g.part_ld + g.part_off[layer];
  const int ld = g.nout[layer];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(size_t)(r0 + 4 * q + i) * ld + c0 + 16 * cb + r16] = acc[cb][i];
}

// Bias gradients: row sums of dZ^T over all samples, one workgroup per row,
// fixed summation order.
struct BGrad {
  const uint16_t* dT[3];
  int rows[3];             // kH, kH, Op
  int64_t Mp;
  float* out;              // [kH + kH + Op]
};

__global__ __launch_bounds__(kWG) void k_mlp_bgrad(const BGrad g) {
  __shared__ float red[kWG];
  int r = blockIdx.x, layer = 0;
  while (layer < 2 && r >= g.rows[layer]) r -= g.rows[layer++];
  const uint16_t* p = g.dT[layer] + (size_t)r * g.Mp;
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < g.Mp; i += kWG) s += from_bf16(p[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kWG / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) g.out[blockIdx.x] = red[0];
}

// Per parameter (flat order W1, b1, W2, b2, W3, b3): gather the gradient from
// the partials, optionally export it, optionally take an Adam step on the FP32
// master copy, and refresh the BF16 copies the products read.
struct Apply {
  int F, Fp, O, Op;
  int64_t nparam;
  float* master;
  float* m;
  float* v;
  const float* part;       // null: no gradient (refresh the BF16 copies only)
  int64_t part_ld;
  int64_t part_off[3];
  int chunks;
  const float* bgrad;      // [kH + kH + Op]
  float* grad_out;         // optional
  int update;              // take an Adam step
  float lr, c1, c2;        // c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)
  uint16_t* w1t;
  uint16_t* w2t;
  uint16_t* w3t;
  uint16_t* w2;
  uint16_t* w3;
};

__global__ __launch_bounds__(kWG) void k_mlp_apply(const Apply a) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= a.nparam) return;
  const int64_t nW1 = (int64_t)a.F * kH, nW2 = (int64_t)kH * kH;
  const int64_t o_b1 = nW1, o_W2 = o_b1 + kH, o_b2 = o_W2 + nW2, o_W3 = o_b2 + kH;
  const int64_t o_b3 = o_W3 + (int64_t)kH * a.O;
  int kind;          // 0..5 = W1, b1, W2, b2, W3, b3
  int r = 0, c = 0;  // row / column within a weight matrix (or bias index in c)
  if (i < o_b1) { kind = 0; r = (int)(i / kH); c = (int)(i % kH); }
  else if (i < o_W2) { kind = 1; c = (int)(i - o_b1); }
  else if (i < o_b2) { kind = 2; r = (int)((i - o_W2) / kH); c = (int)((i - o_W2) % kH); }
  else if (i < o_W3) { kind = 3; c = (int)(i - o_b2); }
  else if (i < o_b3) { kind = 4; r = (int)((i - o_W3) / a.O); c = (int)((i - o_W3) % a.O); }
  else { kind = 5; c = (int)(i - o_b3); }

  float theta = a.master[i];
  if (a.part) {
    float g = 0.f;
    if (kind == 1 || kind == 3 || kind == 5) {
      g = a.bgrad[(kind == 1 ? 0 : kind == 3 ? kH : 2 * kH) + c];
    } else {
      const int layer = kind / 2;
      const int ld = layer == 2 ? a.Op : kH;
      const float* p = a.part + a.part_off[layer] + (size_t)r * ld + c;
      for (int s = 0; s < a.chunks; ++s) g += p[(size_t)s * a.part_ld];
    }
    if (a.grad_out) a.grad_out[i] = g;
    if (a.update) {
      const float mm = 0.9f * a.m[i] + 0.1f * g;
      const float vv = 0.999f * a.v[i] + 0.001f * g * g;
      a.m[i] = mm;
      a.v[i] = vv;
      theta -= a.lr * (mm * a.c1) / (sqrtf(vv * a.c2) + 1e-8f);
      a.master[i] = theta;
    }
  }
  const uint16_t h = to_bf16(theta);
  if (kind == 0) a.w1t[(size_t)c * a.Fp + r] = h;
  else if (kind == 2) { a.w2t[(size_t)c * kH + r] = h; a.w2[(size_t)r * kH + c] = h; }
  else if (kind == 4) { a.w3t[(size_t)c * kH + r] = h; a.w3[(size_t)r * a.Op + c] = h; }
}

__global__ void k_mlp_loss(const float* part, int tiles, double scale, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int t = 0; t < tiles; ++t) s += part[t];
    *out = (float)(s * scale);
  }
}

// Raw training data: features [diag, b - x_prev, x_prev] (the difference in
// FP64, then rounded) and the change x_next - x_prev.
__global__ __launch_bounds__(kWG) void k_mlp_features(int64_t M, int n, int nnz, const int* diag_pos,
                                                      const double* values, const double* b,
                                                      const double* x_prev, const double* x_next,
                                                      float* feat, float* delta) {
  const int F = 3 * n, C = F + (x_next ? n : 0);
  const int64_t total = M * C;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kWG) {
    const int64_t m = i / C;
    const int c = (int)(i - m * C);
    if (c < n) {
      const int p = diag_pos[c];
      feat[m * F + c] = p >= 0 ? (float)values[m * nnz + p] : 0.f;
    } else if (c < 2 * n) {
      feat[m * F + c] = (float)(b[m * n + c - n] - x_prev[m * n + c - n]);
    } else if (c < F) {
      feat[m * F + c] = (float)x_prev[m * n + c - 2 * n];
    } else {
      const int o = c - F;
      delta[m * n + o] = (float)(x_next[m * n + o] - x_prev[m * n + o]);
    }
  }
}

// Column moments of [feat | delta] (ncol <= kWG): partial sums per chunk of
// rows, of the values (mean == null) or of squared deviations from mean.
__global__ __launch_bounds__(kWG) void k_mlp_moments(int64_t M, int F, int O, const float* feat,
                                                     const float* delta, const double* mean,
                                                     int64_t chunk, double* part) {
  const int c = threadIdx.x, ncol = F + O;
  if (c >= ncol) return;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(r0 + chunk, M);
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double v = c < F ? (double)feat[r * F + c] : (double)delta[r * O + (c - F)];
    s += mean ? (v - mean[c]) * (v - mean[c]) : v;
  }
  part[(size_t)blockIdx.x * ncol + c] = s;
}

// Sum the chunks in order: the mean (stage 0) or the standard deviation
// (stage 1, zero spread -> 1), written to out[0..ncol).
__global__ void k_mlp_moments_final(int chunks, int ncol, int64_t M, const double* part,
                                    int stage, double* out) {
  const int c = threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int g = 0; g < chunks; ++g) s += part[(size_t)g * ncol + c];
  s /= (double)M;
  if (stage == 1) {
    const double sd = sqrt(s);
    s = sd > 1e-30 ? sd : 1.0;
  }
  out[c] = s;
}

}  // namespace mlp
}  // namespace bs
