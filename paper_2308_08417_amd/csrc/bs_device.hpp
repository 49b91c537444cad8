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

// LDS gathers issued back to back in the fixed-size SpMV before their FMAs.
#ifndef BS_GATHER
#define BS_GATHER 4
#endif

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
// DPP moves with bound control: lanes whose source is outside the pattern read
// zero, so no old value has to be materialised.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
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
// the same bits.
template <class T>
__device__ __forceinline__ T row16_sum(T v) {
  v = v + dpp<0xB1>(v);
  v = v + dpp<0x4E>(v);
  v = v + dpp<0x141>(v);
  v = v + dpp<0x140>(v);
  return v;
}

// Combine the four row sums S0..S3 (all lanes of row r hold S_r): row_bcast:15
// adds the previous row's sum (row 1 then holds S1+S0, row 3 holds S3+S2);
// row_bcast:31 adds lane 31 to row 3, so lane 63 holds (S3+S2)+(S1+S0).
template <class T>
__device__ __forceinline__ T rows_pairs(T v) { return v + dpp<0x142>(v); }
template <class T>
__device__ __forceinline__ T rows_total(T v) {
  v = rows_pairs(v);
  return v + dpp<0x143>(v);
}

// Sum over aligned groups of g lanes (g = 1, 2, 4, 8 or 16, uniform): the first
// log2(g) steps of the row16_sum butterfly.  Every lane of a group ends with
// the same bits.
template <class T>
__device__ __forceinline__ T group_sum(T v, int g) {
  if (g >= 2) v = v + dpp<0xB1>(v);
  if (g >= 4) v = v + dpp<0x4E>(v);
  if (g >= 8) v = v + dpp<0x141>(v);
  if (g >= 16) v = v + dpp<0x140>(v);
  return v;
}

// gfx950 lane swaps between two registers (one instruction per 32-bit word):
//   swap32(a, b): a <- [a lanes 0-31, b lanes 0-31], b <- [a lanes 32-63, b lanes 32-63]
//   swap16(a, b): a <- [a row 0, b row 0, a row 2, b row 2],
//                 b <- [a row 1, b row 1, a row 3, b row 3]   (rows of 16 lanes)
__device__ __forceinline__ void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap32(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// Sums over the whole wave of K <= 4 values, returned wave-uniform.  Two or
// more values share the butterfly: swap32 + add leaves value 0's pair sums in
// lanes 0-31 and value 1's in lanes 32-63; swap16 + add then packs four values
// into the four rows (rows 0..3 = values 0, 2, 1, 3), and one row butterfly
// finishes all of them.  Every lane of a row ends with the same bits.
template <class T, int K>
__device__ __forceinline__ void wave_sums(T (&v)[K]) {
  static_assert(K >= 1 && K <= 4, "one to four values");
  if constexpr (K == 1) {
    v[0] = rdlane(rows_total(row16_sum(v[0])), 63);
  } else if constexpr (K == 2) {
    T a = v[0], b = v[1];
    swap32(a, b);
    const T s = rows_pairs(row16_sum(a + b));  // lane 31: rows 0+1, lane 63: rows 2+3
    v[0] = rdlane(s, 31);
    v[1] = rdlane(s, 63);
  } else {
    T a = v[0], b = v[1], c = v[2], d = (T)0;
    if constexpr (K == 4) d = v[K - 1];
    swap32(a, b);
    swap32(c, d);
    T s01 = a + b, s23 = c + d;
    swap16(s01, s23);
    const T t = row16_sum(s01 + s23);
    v[0] = rdlane(t, 0);
    v[1] = rdlane(t, 32);
    v[2] = rdlane(t, 16);
    if constexpr (K == 4) v[K - 1] = rdlane(t, 48);
  }
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

// One 16-byte-per-lane direct-to-LDS load of a wave: lane l's 16 bytes at src
// land at LDS byte lds + 16 l (lds wave-uniform, held in M0).  Issued from
// inline asm so that the compiler does not see a load in flight that writes
// LDS: it would then take the LDS counter as out of order and drain every LDS
// read of the solve with lgkmcnt(0).  The instruction has no register result
// (nothing lands in a register later); the caller waits for it with an
// explicit vmcnt before reading the LDS bytes.  Non-temporal: the values are
// read once, so they should not displace lines the outputs are merged in.
__device__ __forceinline__ void dma16(const void* src, unsigned lds) {
  __asm__ volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off nt"
                   :
                   : "v"(src), "s"(lds)
                   : "memory", "m0");
}

// 32-bit LDS addresses: gathers go through address-space-3 pointers so that a
// buffer's constant offset folds into the ds_read immediate.
typedef __attribute__((address_space(3))) char lds_char;
__device__ __forceinline__ unsigned lds_addr(const void* p) {
  return (unsigned)(uintptr_t)(const lds_char*)p;
}
template <class T>
__device__ __forceinline__ T lds_load(unsigned addr) {
  return *(const __attribute__((address_space(3))) T*)(lds_char*)(uintptr_t)addr;
}
template <class T>
__device__ __forceinline__ void lds_store(unsigned addr, T v) {
  *(__attribute__((address_space(3))) T*)(lds_char*)(uintptr_t)addr = v;
}

__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// ---------------------------------------------------------------- team context
template <class S>
struct Team {
  int lane;         // lane within the team
  int tix;          // team index within the workgroup
  int64_t sys;      // system being solved
  int64_t row0;     // offset of its first row in b and x
  bool live;        // sys < n_batch
  char* lds;        // this team's LDS region (vector buffers, solver scalars)
  char* stage_all;  // the group's staging area (single-wave groups)
  char* stage;      // this team's part of it: values, then b
  double* red;      // cross-wave reduction slots (multi-wave teams)
  int phase;        // which half of `red` the next reduction uses
  bool lists;       // the pattern's sweep lists are in LDS (multi-wave ILU(0), BatchTrsv)


  __device__ Team(char* smem, const KArgs& a) {
    const int t = threadIdx.x;
    lane = S::TEAM < kWave ? (t & (S::TEAM - 1)) : t;
    tix = S::TEAM < kWave ? (t / S::TEAM) : 0;
    sys = -1;
    row0 = 0;
    live = false;
    lds = smem + (size_t)tix * a.team_bytes;
    stage_all = smem + a.stage_offset;
    stage = stage_all + (size_t)tix * a.stage_team_bytes;
    red = reinterpret_cast<double*>(smem + (size_t)S::TEAMS * a.team_bytes);
    phase = 0;
    lists = false;
  }

  // Make this team's LDS writes visible to all of its lanes.  A single-wave
  // group needs no barrier: a wave's LDS operations complete in issue order,
  // so only the compiler must keep them in order (wavefront-scope LDS fence).
  // That also keeps the wait off the direct-to-LDS prefetch in flight, which a
  // workgroup-scope fence would have to drain.
  __device__ __forceinline__ void sync() {
    if constexpr (S::WAVES == 1) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
    } else {
      __syncthreads();
    }
  }

  // In-place sum of K per-lane partials over the team; every lane of the team
  // receives the same bits.  All lanes of the workgroup must call it together.
  template <class T, int K>
  __device__ __forceinline__ void sum(T (&v)[K]) {
    if constexpr (S::TEAM < 64) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = row16_sum(v[k]);
    }
    if constexpr (S::TEAM == 32) {
      // teams are rows {0,1} and {2,3}: their sums end in lanes 31 and 63
      const bool hi = lane_id() >= 32;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T p = rows_pairs(v[k]);
        const T s01 = rdlane(p, 31), s23 = rdlane(p, 63);
        v[k] = hi ? s23 : s01;
      }
    } else if constexpr (S::TEAM >= 64) {
      wave_sums(v);
      if constexpr (S::WAVES > 1) {
        static_assert(K <= kMaxFused && K * S::WAVES <= 64, "too many fused values");
        double* buf = red + phase * (kMaxFused * S::WAVES);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
          for (int k = 0; k < K; ++k) buf[k * S::WAVES + w] = (double)v[k];
        }
        __syncthreads();
        // lane l reads value l / WAVES of wave l mod WAVES; a butterfly over
        // aligned groups of WAVES lanes leaves value k's total in lanes
        // k*WAVES .. k*WAVES+WAVES-1, with the same bits in every wave
        const int l = threadIdx.x & 63;
        const int vi = l / S::WAVES < K ? l / S::WAVES : 0;
        const double t = group_sum(buf[vi * S::WAVES + (l & (S::WAVES - 1))], S::WAVES);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (T)rdlane(t, k * S::WAVES);
        phase ^= 1;
      }
    }
  }

  // This team's block-Jacobi region and its row count.
  __device__ __forceinline__ double* bj_region(const KArgs& a) const {
    return reinterpret_cast<double*>(lds + a.bj_offset);
  }
  static constexpr int bj_rows() { return S::ROWS; }

  // Whether any team of this wave satisfies p.  For multi-wave teams every
  // wave sees the same (team-uniform) predicate.
  __device__ __forceinline__ bool any(bool p) const { return wave_any(p); }

};

// ---------------------------------------------------------------- sparse rows
// The rows a lane owns, held in registers: values a[r][k] of register slot k
// of row (lane + r*TEAM), and the LDS address that slot gathers from in the
// team's first vector buffer (8 bytes per element).  Slots that hold no entry
// of the row gather from the buffer's zero cell, so every SpMV runs over all NZ
// slots without branches.
//
// CSR rows are read through a window: slot k holds the value at CSR position
// w + k, where w = min(row start, nnz - NZ) keeps the window inside the
// system's block.  The row's own entries sit in slots shift .. shift+len-1
// (shift = row start - w); the other slots hold neighbouring rows' values,
// which meet the zero cell.  Each slot is then one LDS read at a constant
// offset.  ELL rows use slot k for the row's k-th stored entry.
//
// MX (the mixed-precision kernels): gather addresses are kept for 4-byte
// elements, the FP32 vectors' stride (consecutive elements on consecutive
// banks), and the FP64 SpMVs of the outer residual use 2 * address - base.
// Slots without an entry point at byte 4*ROWS in the FP32 view, whose FP64
// image is the usual zero cell at 8*ROWS; an FP64 SpMV may overwrite the FP32
// zero cell, so every FP32 SpMV writes it again.
template <class S, bool MX = false>
struct Rows {
  static constexpr int R = S::R, NZ = S::NZ, ROWS = S::ROWS, WG = S::WG, TEAM = S::TEAM;
  static constexpr unsigned kElem = MX ? 4 : 8;  // bytes between elements in c and vrow
  double a[S::R][S::NZ];
  unsigned c[S::R][S::NZ];
  unsigned vrow[S::R];  // LDS address of the lane's own rows in buffer 0
  unsigned zc;          // LDS address of the zero cell in buffer 0
  unsigned b0;          // LDS address of buffer 0
  int row[S::R];
  bool ok[S::R];   // row < n
  int len[S::R];
  int dslot[S::R];  // slot of the stored diagonal, -1 if none
  int w[S::R];      // CSR: first position of the read window; ELL: the row
  double dval[S::R];  // the row's stored diagonal value (0 if none)
  double bval[S::R];  // right-hand side of the row (0 past the last row)
  double xval[S::R];  // initial guess of the row (0 when x0 = 0 is promised)
  double xalt[S::R];  // the second candidate start (when one is given)

  static constexpr unsigned kBuf = vec_buf_bytes(S::ROWS);  // bytes per vector buffer

  // The shared pattern, once per kernel: it is the same for every system.
  // Also clears the team's zero cells.
  __device__ void load_pattern(const Team<S>& tm, const KArgs& g) {
    const unsigned base = lds_addr(tm.lds);
    const unsigned zero = base + S::ROWS * kElem;
    zc = zero;
    b0 = base;
    if (tm.lane == 0) {
#pragma unroll
      for (int b = 0; b < kVecBuffers; ++b) {
        lds_store<double>(base + S::ROWS * 8 + b * kBuf, 0.0);
        if constexpr (MX) lds_store<float>(zero + b * kBuf, 0.0f);
      }
    }
    // A one-wave team may take the pattern's bank-aware layout: the row each
    // lane owns, its CSR window, and the buffer element of every x_j (64 lanes,
    // elements 0..63, the zero cell at 64).
    const int* lay = (S::TEAM == kWave && S::R == 1 && g.fmt == 0 && g.window) ? g.layout : nullptr;
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      row[r] = lay ? lay[tm.lane] : tm.lane + r * S::TEAM;
      ok[r] = row[r] >= 0 && row[r] < g.n;
      const int rr = ok[r] ? row[r] : 0;
      vrow[r] = base + (lay ? (ok[r] ? lay[2 * kWave + rr] : S::ROWS) : row[r]) * kElem;
      len[r] = ok[r] ? g.row_len[rr] : 0;
      const int ds = ok[r] ? g.diag_slot[rr] : -1;
      const int rp = g.row_ptr[rr];
      int shift = 0;
      if (g.fmt == 0) {
        w[r] = lay ? lay[kWave + tm.lane] : g.window ? max(0, min(rp, g.nnz - S::NZ)) : rp;
        shift = rp - w[r];
      } else {
        w[r] = rr;
      }
      dslot[r] = ds >= 0 ? ds + shift : -1;
#pragma unroll
      for (int k = 0; k < S::NZ; ++k) {
        const int j = k - shift;  // entry of the row held by slot k
        const bool has = j >= 0 && j < len[r];
        const int col = g.slot_col[has ? (size_t)j * g.n + rr : 0];
        const int el = lay ? lay[2 * kWave + col] : col;
        c[r][k] = has ? base + el * kElem : zero;
        // keep the full address in the register: otherwise the compiler keeps
        // col*8 and re-adds the (link-time) LDS base before every gather
        __asm__ volatile("" : "+v"(c[r][k]));
      }
      __asm__ volatile("" : "+v"(vrow[r]));
    }
  }

  // Prefetch the values and right-hand sides of the solves base..base+TEAMS-1
  // into the group's staging area with direct global-to-LDS loads of 16 bytes
  // per lane: each instruction of the wave fills 1 KiB of LDS, lane l the 16
  // bytes at offset 16l, from a source chosen per lane.  Every block is copied
  // as the 16-byte-aligned chunks that overlap it; such a chunk never crosses a
  // page, so reading all of it is safe, and its bytes outside the block land
  // outside the block's LDS range.  Single-wave groups only.
  __device__ __forceinline__ void prefetch(const Team<S>& tm, const KArgs& g, int64_t base) const {
    static_assert(S::WAVES == 1, "prefetch is for single-wave groups");
    const int per = g.fmt == 0 ? g.nnz : g.width * g.n;
    const unsigned l16 = 16u * (unsigned)lane_id();
    const unsigned vr = (unsigned)g.stage_vals_bytes;
    if constexpr (S::TEAMS == 1) {
      // one system per wave: each region is a run of whole KiB; lanes past the
      // block's last chunk fetch that chunk again
      const uintptr_t v0 = (uintptr_t)(g.values + matrix_of(g, base) * per);
      const uintptr_t va = v0 & ~(uintptr_t)15;
      const unsigned vlast = (unsigned)(((v0 + (uintptr_t)per * 8 - 1) & ~(uintptr_t)15) - va);
      for (unsigned d0 = 0; d0 < vr; d0 += 1024)
        dma16((const void*)(va + min(d0 + l16, vlast)), lds_addr(tm.stage_all + d0));
      const uintptr_t b0 = (uintptr_t)(g.b + base * g.n);
      const uintptr_t ba = b0 & ~(uintptr_t)15;
      const unsigned blast = (unsigned)(((b0 + (uintptr_t)g.n * 8 - 1) & ~(uintptr_t)15) - ba);
      const unsigned br = (unsigned)g.stage_team_bytes - vr;
      for (unsigned d0 = 0; d0 < br; d0 += 1024)
        dma16((const void*)(ba + min(d0 + l16, blast)), lds_addr(tm.stage_all + vr + d0));
    } else {
      // several teams per wave: map every lane's 16 destination bytes to its
      // team, region and chunk; lanes with nothing to fetch re-read the values
      // array's first chunk
      const unsigned ts = (unsigned)g.stage_team_bytes;
      const unsigned region = ts * S::TEAMS;
      const uintptr_t dflt = (uintptr_t)g.values & ~(uintptr_t)15;
      for (unsigned d0 = 0; d0 < region; d0 += 1024) {
        unsigned o = d0 + l16;
        int t = 0;
#pragma unroll
        for (int i = 1; i < S::TEAMS; ++i)
          if (o >= ts) { o -= ts; ++t; }
        const int64_t sy = base + t;
        uintptr_t src = dflt;
        if (d0 + l16 < region && sy < g.n_batch) {
          uintptr_t start, end;
          if (o < vr) {
            start = (uintptr_t)(g.values + matrix_of(g, sy) * per);
            end = start + (uintptr_t)per * 8;
          } else {
            o -= vr;
            start = (uintptr_t)(g.b + sy * g.n);
            end = start + (uintptr_t)g.n * 8;
          }
          const uintptr_t chunk = (start & ~(uintptr_t)15) + o;
          if (chunk < end) src = chunk;
        }
        dma16((const void*)src, lds_addr(tm.stage_all + d0));
      }
    }
  }

  // Multi-wave teams (one team per group), CSR: prefetch the values of
  // system `sys` into the group's staging area with direct global-to-LDS loads
  // of 16 bytes per lane, wave w taking the KiB chunks w, w + WAVES, ...  The
  // block is copied as the 16-byte-aligned chunks that overlap it (none
  // crosses a page); lanes past its last chunk fetch that chunk again.  The
  // area holds a whole number of KiB covering the block and 16 bytes more.
  __device__ __forceinline__ void prefetch_group(const Team<S>& tm, const KArgs& g,
                                                 int64_t sys) const {
    static_assert(S::WAVES > 1 && S::TEAMS == 1, "group prefetch is for multi-wave teams");
    const uintptr_t v0 = (uintptr_t)(g.values + matrix_of(g, sys) * g.nnz);
    const uintptr_t va = v0 & ~(uintptr_t)15;
    const unsigned vlast = (unsigned)(((v0 + (uintptr_t)g.nnz * 8 - 1) & ~(uintptr_t)15) - va);
    const unsigned l16 = 16u * (unsigned)lane_id();
    const unsigned w = (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // (wave-uniform: the destination goes to M0)
    const unsigned area = (unsigned)__builtin_amdgcn_readfirstlane(
        (int)(lds_addr(tm.lds) + (unsigned)g.stage_offset));
    const unsigned vr = (unsigned)g.stage_vals_bytes;
    for (unsigned d0 = w * 1024u; d0 < vr; d0 += (unsigned)S::WAVES * 1024u)
      dma16((const void*)(va + min(d0 + l16, vlast)), area + d0);
  }

  static __device__ __forceinline__ void settle(double& v) { __asm__ volatile("" : "+v"(v)); }

  // This team's values and right-hand side.  Staged groups read them from the
  // prefetched LDS block; other groups read HBM directly.
  __device__ void load_values(Team<S>& tm, const KArgs& g) {
    const int64_t per = g.fmt == 0 ? (int64_t)g.nnz : (int64_t)g.width * g.n;
    const double* vals = g.values + (tm.live ? matrix_of(g, tm.sys) * per : 0);
    const double* bb = g.b + (tm.live ? tm.sys * g.n : 0);
    // Per-lane offsets are passed through an empty asm once per system so the
    // compiler recomputes the per-slot addresses here instead of hoisting them
    // out of the batch loop, where they would pin registers for the whole kernel.
    int off[S::R], ln[S::R], ds[S::R], rw[S::R];
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      off[r] = w[r];
      ln[r] = tm.live ? len[r] : 0;
      ds[r] = tm.live ? dslot[r] : -1;
      rw[r] = (tm.live && ok[r]) ? row[r] : -1;
      __asm__ volatile("" : "+v"(off[r]), "+v"(ln[r]), "+v"(ds[r]), "+v"(rw[r]));
    }
    const bool win = g.fmt == 0 && g.window;
    const int step = g.fmt == 0 ? 1 : g.n;
    if constexpr (S::WAVES == 1) {
      if (g.stage) {
        // the blocks sit in LDS at their address modulo 16 (see prefetch)
        const unsigned st = lds_addr(tm.stage) + ((uintptr_t)vals & 15);
        const unsigned sb = lds_addr(tm.stage) + g.stage_vals_bytes + ((uintptr_t)bb & 15);
#pragma unroll
        for (int r = 0; r < S::R; ++r) {
          if (win) {
            const unsigned wa = st + off[r] * 8;
#pragma unroll
            for (int k = 0; k < S::NZ; ++k) a[r][k] = lds_load<double>(wa + k * 8);
          } else {
#pragma unroll
            for (int k = 0; k < S::NZ; ++k) {
              const bool has = k < ln[r];
              const double v = lds_load<double>(st + (has ? off[r] + k * step : 0) * 8);
              a[r][k] = has ? v : 0.0;
            }
          }
          const double dv = lds_load<double>(st + (ds[r] >= 0 ? off[r] + ds[r] * step : 0) * 8);
          dval[r] = ds[r] >= 0 ? dv : 0.0;
          const double bv = lds_load<double>(sb + (rw[r] >= 0 ? rw[r] : 0) * 8);
          bval[r] = rw[r] >= 0 ? bv : 0.0;
        }
        load_x0(tm, g, rw);
        return;
      }
    } else if constexpr (S::NZ >= kStageMinSlots) {
      if (g.stage == 2) {
        // Multi-wave teams, CSR: the system's values were copied into LDS by
        // the whole group (prefetch_group, coalesced direct-to-LDS loads issued
        // during the previous system's solve); each lane reads its row's window
        // from there.  Lanes reading their rows straight from HBM touch one
        // line per lane and load, which the caches serve far more slowly.  The
        // block sits at its address modulo 16, as in the one-wave staging.
        // (One team per group: its region starts the group's LDS, and the
        // staging area sits stage_offset bytes further.)
        const unsigned st = lds_addr(tm.lds) + (unsigned)g.stage_offset + ((uintptr_t)vals & 15);
#pragma unroll
        for (int r = 0; r < S::R; ++r) {
          if (win) {
            const unsigned wa = st + off[r] * 8;
#pragma unroll
            for (int k = 0; k < S::NZ; ++k) a[r][k] = lds_load<double>(wa + k * 8);
          } else {
#pragma unroll
            for (int k = 0; k < S::NZ; ++k) {
              const bool has = k < ln[r];
              const double v = lds_load<double>(st + (has ? off[r] + k : 0) * 8);
              a[r][k] = has ? v : 0.0;
            }
          }
          const double dv = lds_load<double>(st + (ds[r] >= 0 ? off[r] + ds[r] : 0) * 8);
          dval[r] = ds[r] >= 0 ? dv : 0.0;
          double bv = bb[rw[r] >= 0 ? rw[r] : 0];
          settle(bv);  // completed before the next prefetch is issued
          bval[r] = rw[r] >= 0 ? bv : 0.0;
        }
        load_x0(tm, g, rw);
        return;
      }
    }
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      if constexpr (S::WAVES > 1 && S::NZ == 56) {
        // every load of the row first, the zeros of the empty slots after: in
        // this shape the select form made the compiler wait for each load (the
        // select's condition lives in the one VCC register) before issuing
        // the next; the other shapes keep their loads in flight either way
        double v[S::NZ];
#pragma unroll
        for (int k = 0; k < S::NZ; ++k)
          v[k] = __builtin_nontemporal_load(vals + ((win || k < ln[r]) ? off[r] + k * step : 0));
#pragma unroll
        for (int k = 0; k < S::NZ; ++k) a[r][k] = (win || k < ln[r]) ? v[k] : 0.0;
      } else if (win) {
#pragma unroll
        for (int k = 0; k < S::NZ; ++k) a[r][k] = __builtin_nontemporal_load(vals + off[r] + k);
      } else {
#pragma unroll
        for (int k = 0; k < S::NZ; ++k) {
          const bool has = k < ln[r];
          const double v = __builtin_nontemporal_load(vals + (has ? off[r] + k * step : 0));
          a[r][k] = has ? v : 0.0;
        }
      }
      const double dv = vals[ds[r] >= 0 ? off[r] + ds[r] * step : 0];
      dval[r] = ds[r] >= 0 ? dv : 0.0;
      const double bv = bb[rw[r] >= 0 ? rw[r] : 0];
      bval[r] = rw[r] >= 0 ? bv : 0.0;
    }
    // Single-wave groups complete these loads here: the registers are shared
    // with the staged path, and a load left pending would make the compiler
    // wait on the in-order memory counter later, which would also drain the
    // prefetch in flight.  Wider groups have neither (and the barrier made
    // the compiler wait for each load before issuing the next): their loads
    // stay in flight together until the first product needs them.
    if constexpr (S::WAVES == 1) {
#pragma unroll
      for (int r = 0; r < S::R; ++r) {
#pragma unroll
        for (int k = 0; k < S::NZ; ++k) settle(a[r][k]);
        settle(dval[r]);
        settle(bval[r]);
      }
    }
    load_x0(tm, g, rw);
  }

  // The initial guess is read here, before the next prefetch is issued, so a
  // wait for it never waits behind that prefetch.
  __device__ __forceinline__ void load_x0(const Team<S>& tm, const KArgs& g, const int (&rw)[S::R]) {
    // Only when an initial guess is read does this wait on memory (a wait
    // here would also wait for the previous system's output stores).
    const bool zero = (g.flags & 1) != 0;
#pragma unroll
    for (int r = 0; r < S::R; ++r) xval[r] = 0.0;
    if (!zero) {
      const double* xx = g.x + (tm.live ? tm.sys * g.n : 0);
#pragma unroll
      for (int r = 0; r < S::R; ++r) {
        double xv = 0.0;
        if (rw[r] >= 0) xv = xx[rw[r]];
        settle(xv);  // completed before the next prefetch is issued
        xval[r] = xv;
      }
    }
    if (g.x_alt) {
      const double* xa = g.x_alt + (tm.live ? tm.sys * g.n : 0);
#pragma unroll
      for (int r = 0; r < S::R; ++r) {
        double xv = 0.0;
        if (rw[r] >= 0) xv = xa[rw[r]];
        settle(xv);
        xalt[r] = xv;
      }
    }
  }

  // Whether slot k of row r holds one of the row's entries (not the zero cell).
  __device__ __forceinline__ bool real(int r, int k) const { return c[r][k] != zc; }
  __device__ __forceinline__ int nrows(const KArgs& g) const { return g.n; }

  // Scalar Jacobi: d = 1/a_ii, 1 where the diagonal is zero or absent; 0 for
  // lanes past the last row so padded entries stay zero.
  __device__ void jacobi(int precond, double (&d)[S::R]) const {
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      const double dv = dval[r];
      d[r] = !ok[r] ? 0.0 : (precond == 1 && dslot[r] >= 0 && dv != 0.0) ? 1.0 / dv : 1.0;
    }
  }

  // y = A v.  v is written to the team's vector buffer BUF, the team syncs, and
  // each lane gathers its rows' columns from LDS.  T is the arithmetic type;
  // the buffer always spaces elements 8 bytes apart.  The gathers go out in
  // groups of kGather, one or two groups in flight (an empty asm that a group's
  // FMAs feed keeps later groups behind them, bounding the registers held by
  // loads in flight); four partial sums per row keep the FMA chains short.
  // Shapes with room in their register budget keep two gather groups in
  // flight; the others one.
  static constexpr bool kPipe = S::R == 1 && S::NZ <= 28;

  template <int BUF, bool PIPE = kPipe, class T, class AT>
  __device__ __forceinline__ void spmv(Team<S>& tm, const AT (&av)[S::R][S::NZ],
                                       const T (&v)[S::R], T (&y)[S::R]) const {
    constexpr int kGather = BS_GATHER;
    constexpr unsigned off = BUF * kBuf;
    // FP64 vectors in a mixed kernel: twice the 4-byte-element address, formed
    // at each use (the empty asm keeps the compiler from holding a second set
    // of addresses in registers through the solve for these rare SpMVs)
    constexpr bool kWide = MX && sizeof(T) == 8;
    auto at = [&](unsigned a) -> unsigned {
      if constexpr (kWide) {
        __asm__ volatile("" : "+v"(a));
        return 2u * a - b0;
      } else {
        return a;
      }
    };
#pragma unroll
    for (int r = 0; r < S::R; ++r)
      if (ok[r]) lds_store<T>(at(vrow[r]) + off, v[r]);
    if constexpr (MX && sizeof(T) == 4) {
      if (tm.lane == 0) lds_store<float>(zc + off, 0.0f);
    }
    tm.sync();
    constexpr int NA = S::NZ >= 4 ? 4 : S::NZ;
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      T acc[4] = {0, 0, 0, 0};
      if constexpr (PIPE) {
        // two groups in flight: the next group's gathers are issued before
        // this group's FMAs, so their LDS latency overlaps the arithmetic
        T xa[kGather], xb[kGather] = {};
#pragma unroll
        for (int k = 0; k < kGather && k < S::NZ; ++k) xa[k] = lds_load<T>(at(c[r][k]) + off);
#pragma unroll
        for (int k0 = 0; k0 < S::NZ; k0 += kGather) {
          const int k1 = k0 + kGather;
#pragma unroll
          for (int k = k1; k < k1 + kGather && k < S::NZ; ++k) xb[k - k1] = lds_load<T>(at(c[r][k]) + off);
#pragma unroll
          for (int k = k0; k < k0 + kGather && k < S::NZ; ++k)
            acc[k % NA] = fma((T)av[r][k], xa[k - k0], acc[k % NA]);
          // the group after next is issued only after this group's FMAs
          __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])::"memory");
#pragma unroll
          for (int k = 0; k < kGather; ++k) xa[k] = xb[k];
        }
      } else {
#pragma unroll
        for (int k0 = 0; k0 < S::NZ; k0 += kGather) {
          T xv[kGather];
#pragma unroll
          for (int k = k0; k < k0 + kGather && k < S::NZ; ++k) xv[k - k0] = lds_load<T>(at(c[r][k]) + off);
#pragma unroll
          for (int k = k0; k < k0 + kGather && k < S::NZ; ++k)
            acc[k % NA] = fma((T)av[r][k], xv[k - k0], acc[k % NA]);
          // finish this group's FMAs before the next group's gathers are issued
          __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])::"memory");
        }
      }
      T s = acc[0];
      if constexpr (NA == 4) s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
      else {
#pragma unroll
        for (int i = 1; i < NA; ++i) s += acc[i];
      }
      y[r] = s;
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
