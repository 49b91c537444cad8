// Learned initial guess: a three-layer perceptron (3n -> 256 -> 256 -> n, ReLU)
// run through BF16 matrix-core products with FP32 accumulation.
//
// Layout conventions (all BF16 stored as raw 16-bit words, rounded to nearest
// with ties to even):
//  * activations of a 64-sample tile live in LDS, row-major [sample][feature]
//    with a row stride of (width + 8) elements so that the 16-byte fragment
//    reads of successive rows start in different banks;
//  * the B operand of every product is read from global memory (it stays in
//    L2: the whole network is about 240 KB) as "B transposed", row-major
//    [output column][k], so a lane's eight k values are one 16-byte load;
//  * the training kernel also writes activations and their gradients
//    feature-major [feature][sample] for the weight-gradient products, whose
//    reduction runs over samples.
//
// v_mfma_f32_16x16x32_bf16: lane l supplies row l%16 of A and column l%16 of
// B (eight k values each, the same eight for both) and receives
// C[4*(l/16) + i][l%16], i = 0..3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bs {
namespace mlp {

constexpr int kH = 256;     // hidden width
constexpr int kTile = 64;   // samples per workgroup tile
constexpr int kWG = 256;    // four waves
constexpr int kPad = 8;     // LDS row padding, elements
constexpr int kMaxN = 64;   // largest system size (3n <= 192 features)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Round to the nearest bfloat16, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 frag(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

// acc[rb][cb] += A[rb*16 .. +16][0..K) * B[0..K)[c0 + cb*16 .. +16]
// A: LDS row-major, stride lda; Bt: global row-major [column][ldb].  The B
// fragments of step k0 + 32 are loaded while the products of step k0 run (the
// weights come from L2; waiting for them at every step left the matrix cores
// idle); the products themselves run in the same order as without it.
template <int RB, int CB>
__device__ __forceinline__ void gemm_tile(floatx4 (&acc)[RB][CB], const uint16_t* A, int lda,
                                          const uint16_t* __restrict__ Bt, int ldb, int c0, int K) {
  const int l = threadIdx.x & 63, r16 = l & 15, q = l >> 4;
  bf16x8 b[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) b[cb] = frag(Bt + (size_t)(c0 + cb * 16 + r16) * ldb + 8 * q);
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a[RB], bn[CB];
    if (k0 + 32 < K) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        bn[cb] = frag(Bt + (size_t)(c0 + cb * 16 + r16) * ldb + k0 + 32 + 8 * q);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[rb] = frag(A + (rb * 16 + r16) * lda + k0 + 8 * q);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
    if (k0 + 32 < K) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b[cb] = bn[cb];
    }
  }
}

template <int RB, int CB>
__device__ __forceinline__ void zero(floatx4 (&acc)[RB][CB]) {
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// Everything a kernel needs about the network and its scaling.
struct Net {
  int n, F, Fp, O, Op;          // system size, features (3n) padded to 64, outputs padded to 32
  const uint16_t* w1t;          // [kH][Fp]   B^T of layer 1
  const uint16_t* w2t;          // [kH][kH]   B^T of layer 2
  const uint16_t* w3t;          // [Op][kH]   B^T of layer 3
  const uint16_t* w2;           // [kH][kH]   W2 itself (B^T of dH1 = dZ2 W2^T)
  const uint16_t* w3;           // [kH][Op]   W3 itself (B^T of dH2 = dY W3^T)
  const float* b1;              // [kH]
  const float* b2;              // [kH]
  const float* b3;              // [O]
  const double* mu_f;           // [F] feature means
  const double* sd_f;           // [F] feature standard deviations
  const double* sd_d;           // [O] scale of the solution change
};

// Where a tile's raw inputs come from.
struct Src {
  // training: FP32 raw features [rows][F] and changes [rows][O], optional row list
  const float* feat;
  const float* delta;
  const int* rows;
  // inference: the batch itself (FP64), CSR values with the diagonal's position,
  // or the diagonals themselves when diag is not null
  int nnz;
  const int* diag_pos;          // [n] position of A[i][i] in a system's values, -1 if none
  const double* diag;           // [rows][n] diagonal of every system, or null
  const double* values;
  const double* b;
  const double* x_prev;
  double* x0;                   // output
};

// Training outputs of the fused forward/backward kernel.
struct Train {
  int64_t M;                    // samples in the batch
  int64_t Mp;                   // padded to the tile (leading dimension of the stores)
  uint16_t* zT;                 // [Fp][Mp]
  uint16_t* h1T;                // [kH][Mp]
  uint16_t* h2T;                // [kH][Mp]
  uint16_t* dz1T;               // [kH][Mp]
  uint16_t* dz2T;               // [kH][Mp]
  uint16_t* dyT;                // [Op][Mp]
  float* loss_part;             // [tiles] sum of squared errors of each tile
  float* y_out;                 // optional [M][O] network outputs (tests)
};

}  // namespace mlp
}  // namespace bs
