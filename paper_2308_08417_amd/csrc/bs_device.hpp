// Device building blocks of the fused batched solver (paper Sec. 3.2): team
// reductions, the register-resident sparse rows with their SpMV, and the
// per-team context.  Everything here is inlined into the solver kernels.
//
// A "team" is the set of lanes that solves one system: a quarter or half of a
// wave (16/32 lanes), one wave, or a workgroup of up to 16 waves.  Each lane
// owns R rows (row = lane + r*TEAM); a row's values and column offsets stay in
// registers for the whole solve, so the matrix is read from HBM exactly once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bs_shape.hpp"

namespace bs {

enum : int {
  ST_CONVERGED = 0,
  ST_MAX_ITER = 1,
  ST_BREAKDOWN = 2,
  ST_NONFINITE = 3,
  ST_RUNNING = -1,
  ST_IDLE = -2  // team without a system (tail of the batch)
};

// ---------------------------------------------------------------- cross-lane
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ double rdlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over each row of 16 lanes by a butterfly whose every step adds a lane's
// value to its mirror partner's (quad_perm [1,0,3,2], [2,3,0,1], half-row
// mirror, row mirror).  Each pairwise sum is formed as a+b in one lane and b+a in
// the other, which IEEE addition makes bit-identical, so all 16 lanes end with
// the same bits -- the scalars of a team never diverge between its lanes.
template <class T>
__device__ __forceinline__ T row16_sum(T v) {
  v = v + dpp<0xB1>(v);
  v = v + dpp<0x4E>(v);
  v = v + dpp<0x141>(v);
  v = v + dpp<0x140>(v);
  return v;
}

__device__ __forceinline__ int row16_max(int v) {
  v = max(v, dpp<0xB1>(v));
  v = max(v, dpp<0x4E>(v));
  v = max(v, dpp<0x141>(v));
  v = max(v, dpp<0x140>(v));
  return v;
}

// Largest value over the whole wave, wave-uniform.
__device__ __forceinline__ int wave_max(int v) {
  v = row16_max(v);
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return max(max(a, b), max(c, d));
}

__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// ---------------------------------------------------------------- team context
template <class S>
struct Team {
  int lane;         // lane within the team
  int tix;          // team index within the workgroup
  int64_t sys;      // system index
  bool live;        // sys < n_batch
  char* lds;        // this team's LDS region
  double* red;      // cross-wave reduction slots (multi-wave teams)
  int phase;        // which half of `red` the next reduction uses

  __device__ Team(char* smem, const KArgs& a) {
    const int t = threadIdx.x;
    lane = S::TEAM < kWave ? (t & (S::TEAM - 1)) : t;
    tix = S::TEAM < kWave ? (t / S::TEAM) : 0;
    sys = (int64_t)blockIdx.x * S::TEAMS + tix;
    live = sys < a.n_batch;
    lds = smem + (size_t)tix * a.team_bytes;
    red = reinterpret_cast<double*>(smem + (size_t)S::TEAMS * a.team_bytes);
    phase = 0;
  }

  // Make this team's LDS writes visible to all of its lanes.
  __device__ __forceinline__ void sync() { __syncthreads(); }

  // In-place sum of K per-lane partials over the team; every lane of the team
  // receives the same bits.  All lanes of the workgroup must call it together.
  template <class T, int K>
  __device__ __forceinline__ void sum(T (&v)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = row16_sum(v[k]);
    if constexpr (S::TEAM == 32) {
      const bool hi = lane_id() >= 32;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T s0 = rdlane(v[k], 0), s1 = rdlane(v[k], 16);
        const T s2 = rdlane(v[k], 32), s3 = rdlane(v[k], 48);
        v[k] = hi ? (s2 + s3) : (s0 + s1);
      }
    } else if constexpr (S::TEAM >= 64) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T s0 = rdlane(v[k], 0), s1 = rdlane(v[k], 16);
        const T s2 = rdlane(v[k], 32), s3 = rdlane(v[k], 48);
        v[k] = (s0 + s1) + (s2 + s3);
      }
      if constexpr (S::WAVES > 1) {
        static_assert(K <= kMaxFused, "too many fused values");
        double* buf = red + phase * (kMaxFused * S::WAVES);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
          for (int k = 0; k < K; ++k) buf[k * S::WAVES + w] = (double)v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double s = buf[k * S::WAVES];
#pragma unroll
          for (int i = 1; i < S::WAVES; ++i) s += buf[k * S::WAVES + i];
          v[k] = (T)s;
        }
        phase ^= 1;
      }
    }
  }

  // Whether any team of this wave satisfies p.  For multi-wave teams every
  // wave sees the same (team-uniform) predicate.
  __device__ __forceinline__ bool any(bool p) const { return wave_any(p); }
};

// ---------------------------------------------------------------- sparse rows
// The rows a lane owns, held in registers: values a[r][k] of slot k of row
// (lane + r*TEAM), and the LDS byte offset of that slot's column inside a
// vector buffer (8 bytes per element).  `nzw` is the wave's longest row.
template <class S>
struct Rows {
  double a[S::R][S::NZ];
  int c[S::R][S::NZ];
  int row[S::R];
  bool ok[S::R];   // row < n
  int dslot[S::R];
  int nzw;

  // Load this team's system.  CSR values are either staged through the team's
  // LDS (one coalesced copy of the contiguous value block, then row reads) or
  // read straight from HBM; ELL values are read slot by slot, which is
  // coalesced across the lanes.  Syncs: the caller's whole workgroup must call.
  __device__ void load(Team<S>& tm, const KArgs& g) {
    int len[S::R];
    int lmax = 0;
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      row[r] = tm.lane + r * S::TEAM;
      ok[r] = row[r] < g.n;
      len[r] = ok[r] ? g.row_len[row[r]] : 0;
      dslot[r] = ok[r] ? g.diag_slot[row[r]] : -1;
      lmax = max(lmax, len[r]);
    }
    nzw = wave_max(lmax);
    const int64_t vbase = tm.sys * (g.fmt == 0 ? (int64_t)g.nnz : (int64_t)g.width * g.n);
    const double* vals = g.values + (tm.live ? vbase : 0);
    const double* stage = reinterpret_cast<const double*>(tm.lds);
    if (g.fmt == 0 && g.stage) {
      double* st = reinterpret_cast<double*>(tm.lds);
      if (tm.live)
        for (int e = tm.lane; e < g.nnz; e += S::TEAM) st[e] = __builtin_nontemporal_load(vals + e);
      tm.sync();
    }
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      const int rp = (ok[r] && g.fmt == 0) ? g.row_ptr[row[r]] : 0;
#pragma unroll
      for (int k = 0; k < S::NZ; ++k) {
        a[r][k] = 0.0;
        c[r][k] = 0;
        if (k < nzw) {
          const bool has = tm.live && k < len[r];
          if (has) {
            c[r][k] = g.slot_col[(size_t)k * g.n + row[r]] * 8;
            if (g.fmt == 0)
              a[r][k] = g.stage ? stage[rp + k] : __builtin_nontemporal_load(vals + rp + k);
            else
              a[r][k] = __builtin_nontemporal_load(vals + (size_t)k * g.n + row[r]);
          }
        }
      }
    }
    if (g.fmt == 0 && g.stage) tm.sync();  // staging area is reused for vectors
  }

  // Scalar Jacobi: d = 1/a_ii, 1 where the diagonal is zero or absent; 0 for
  // lanes past the last row so padded entries stay zero.
  __device__ void jacobi(int precond, double (&d)[S::R]) const {
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      double dv = 0.0;
#pragma unroll
      for (int k = 0; k < S::NZ; ++k)
        if (k == dslot[r]) dv = a[r][k];
      d[r] = !ok[r] ? 0.0 : (precond == 1 && dslot[r] >= 0 && dv != 0.0) ? 1.0 / dv : 1.0;
    }
  }

  // y = A v.  v is written to the team's vector buffer BUF, the team syncs, and
  // each lane gathers its rows' columns from LDS.  T is the arithmetic type;
  // the buffer always spaces elements 8 bytes apart.
  template <int BUF, class T, class AT>
  __device__ __forceinline__ void spmv(Team<S>& tm, const AT (&av)[S::R][S::NZ],
                                       const T (&v)[S::R], T (&y)[S::R], int rows) const {
    char* buf = tm.lds + BUF * rows * 8;
#pragma unroll
    for (int r = 0; r < S::R; ++r)
      if (ok[r]) *reinterpret_cast<T*>(buf + row[r] * 8) = v[r];
    tm.sync();
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < S::NZ; ++k)
        if (k < nzw) acc = fma((T)av[r][k], *reinterpret_cast<const T*>(buf + c[r][k]), acc);
      y[r] = acc;
    }
  }
};

template <class T, int R>
__device__ __forceinline__ T sum_rows(const T (&p)[R]) {
  T s = p[0];
#pragma unroll
  for (int r = 1; r < R; ++r) s += p[r];
  return s;
}

}  // namespace bs
