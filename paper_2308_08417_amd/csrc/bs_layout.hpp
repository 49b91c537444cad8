// Host-side choice of where a one-wave team keeps its rows and vector elements
// (one system per 64-lane wave, one row per lane, CSR rows read through a
// window of NZ register slots).
//
// The sparse product gathers x[col] from LDS once per register slot: lane l
// reads the element of the column its row holds in that slot.  A 64-lane LDS
// read of 8-byte elements is served as two 32-lane halves; within a half, the
// 8-byte elements that fall on the same pair of 4-byte banks ((address / 8) mod
// 32) are served one after another, and lanes that read the same element share
// it.  With every row on the lane of its own index and x_i at element i, rows i
// and i + 32 collide on one bank pair.  The copy of the staged values into
// registers has the same structure: at slot k the lanes read CSR positions
// w_l + k, so the cost of each slot is the largest number of distinct window
// starts of one half that agree modulo 32.
//
// Three choices are free, since the pattern is shared by the whole batch and
// fixed before any solve:
//   lane_row[l]  the row that lane l owns (-1: none), a permutation of the rows
//                over the 64 lanes;
//   col_pos[j]   the element of a vector buffer that holds x_j (0..63, all
//                distinct; element 64 is the zero cell that empty slots read);
//   lane_win[l]  where lane l's CSR window starts: any w with
//                max(0, rp[i+1] - NZ) <= w <= min(rp[i], nnz - NZ) keeps row i
//                inside the window and the window inside the block.
// The cost model counts, per half and per slot, the bank pair that serves the
// most distinct elements (the unit is one such element):
//   cost = kSpmvWeight * (gathers + writes) + copy,
// kSpmvWeight SpMVs (and vector writes) per register copy of the values.  The
// search is simulated annealing from the plain layout with a fixed seed, so
// the layout, and every result computed with it, is the same on every run.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace bs {

constexpr int kLayoutLanes = 64;
constexpr int kLayoutZero = 64;     // element of the zero cell
constexpr int kSpmvWeight = 5;      // SpMVs per copy of the values into registers

struct WaveLayout {
  std::vector<int> lane_row, lane_win, col_pos;
  int64_t cost = 0, plain_cost = 0;
};

class LayoutModel {
 public:
  LayoutModel(int n, int nnz, const int* rp, const int* col, int nz)
      : n_(n), nnz_(nnz), nz_(nz), rp_(rp), col_(col) {}

  // Window limits of row i.
  int lo(int i) const { return std::max(0, rp_[i + 1] - nz_); }
  int hi(int i) const { return std::min(rp_[i], nnz_ - nz_); }

  // Element read by row i (window w) at slot k.
  int elem(int i, int w, int k, const std::vector<int>& pos) const {
    const int p = w + k;
    return (p >= rp_[i] && p < rp_[i + 1]) ? pos[col_[p]] : kLayoutZero;
  }

  // row_lane[i]: lane of row i; win[i]: window of row i; pos[j]: element of x_j.
  int64_t cost(const std::vector<int>& row_lane, const std::vector<int>& win,
               const std::vector<int>& pos) {
    int64_t gathers = 0, writes = 0, copy = 0;
    for (int h = 0; h < 2; ++h) {
      rows_.clear();
      for (int i = 0; i < n_; ++i)
        if ((row_lane[i] >> 5) == h) rows_.push_back(i);
      const bool idle = rows_.size() < 32;  // idle lanes read the zero cell
      for (int k = 0; k < nz_; ++k) {
        begin();
        if (idle) add(kLayoutZero);
        for (int i : rows_) add(elem(i, win[i], k, pos));
        gathers += peak_;
      }
      begin();
      for (int i : rows_) add(pos[i]);
      writes += peak_;
      begin();
      for (int i : rows_) add(win[i]);
      copy += (int64_t)nz_ * peak_;
    }
    return kSpmvWeight * (gathers + writes) + copy;
  }

 private:
  // distinct-element counting per bank pair
  void begin() {
    ++stamp_;
    peak_ = 0;
    std::fill(bank_, bank_ + 32, 0);
  }
  void add(int e) {
    const int key = e;  // elements: 0..64; windows: 0..nnz
    if ((int)seen_.size() <= key) seen_.resize(key + 1, 0);
    if (seen_[key] == stamp_) return;
    seen_[key] = stamp_;
    peak_ = std::max(peak_, ++bank_[e & 31]);
  }

  int n_, nnz_, nz_;
  const int *rp_, *col_;
  std::vector<int> rows_, seen_;
  int bank_[32] = {};
  int stamp_ = 0, peak_ = 0;
};

// 64-bit xorshift* generator (Vigna 2016) for the annealing moves.
struct LayoutRng {
  uint64_t s;
  explicit LayoutRng(uint64_t seed) : s(seed ? seed : 0x9E3779B97F4A7C15ull) {}
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 0x2545F4914F6CDD1Dull;
  }
  int below(int m) { return (int)((next() >> 33) % (uint64_t)m); }
  double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Requires 32 < n <= 64 (both halves hold rows), nnz >= nz, every row at most
// nz entries.  `steps` annealing moves.
inline WaveLayout choose_wave_layout(int n, int nnz, const int* rp, const int* col, int nz,
                                     int steps) {
  LayoutModel M(n, nnz, rp, col, nz);
  std::vector<int> row_lane(n), win(n), pos(n);
  for (int i = 0; i < n; ++i) {
    row_lane[i] = i;
    win[i] = M.hi(i);
    pos[i] = i;
  }
  WaveLayout out;
  out.plain_cost = M.cost(row_lane, win, pos);
  int64_t cur = out.plain_cost, best = cur;
  std::vector<int> brl = row_lane, bw = win, bp = pos;
  std::vector<int> lane_of_elem(kLayoutLanes, -1), row_of_lane(kLayoutLanes, -1);
  LayoutRng rng(0x5EEDull + (uint64_t)n * 1315423911ull + (uint64_t)nnz);
  double T = 3.0;
  for (int s = 0; s < steps; ++s) {
    std::vector<int> rl2 = row_lane, w2 = win, p2 = pos;
    const double u = rng.unit();
    if (u < 0.4) {  // move x_j to element e, swapping with its holder
      const int j = rng.below(n), e = rng.below(kLayoutLanes);
      for (int t = 0; t < n; ++t)
        if (p2[t] == e) p2[t] = p2[j];
      p2[j] = e;
    } else if (u < 0.7) {  // move row i to lane L, swapping with its owner
      const int i = rng.below(n), L = rng.below(kLayoutLanes);
      for (int t = 0; t < n; ++t)
        if (rl2[t] == L) rl2[t] = rl2[i];
      rl2[i] = L;
    } else {  // another window for row i
      const int i = rng.below(n);
      if (M.lo(i) == M.hi(i)) continue;
      w2[i] = M.lo(i) + rng.below(M.hi(i) - M.lo(i) + 1);
    }
    const int64_t c = M.cost(rl2, w2, p2);
    if (c <= cur || rng.unit() < std::exp((double)(cur - c) / T)) {
      row_lane.swap(rl2);
      win.swap(w2);
      pos.swap(p2);
      cur = c;
      if (c < best) {
        best = c;
        brl = row_lane;
        bw = win;
        bp = pos;
      }
    }
    T = std::max(0.05, T * 0.9998);
  }
  out.cost = best;
  out.lane_row.assign(kLayoutLanes, -1);
  out.lane_win.assign(kLayoutLanes, -1);
  for (int i = 0; i < n; ++i) {
    out.lane_row[brl[i]] = i;
    out.lane_win[brl[i]] = bw[i];
  }
  // an idle lane copies a window of its own half, so its reads add no element
  for (int l = 0; l < kLayoutLanes; ++l) {
    if (out.lane_row[l] >= 0) continue;
    for (int m = (l & 32); m < (l & 32) + 32; ++m)
      if (out.lane_row[m] >= 0) {
        out.lane_win[l] = out.lane_win[m];
        break;
      }
  }
  out.col_pos = bp;
  return out;
}

}  // namespace bs
