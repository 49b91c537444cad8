// The streamed placement for batches that share one pattern: the spill tier
// of the fixed-size batched solve.  When no register shape holds a row (more
// than 64 entries, BatchDense beyond 64 rows, or systems of 1025..2048 rows
// whose rows are longer than the 8 register slots of the 2-row shapes), CG and
// BiCGSTAB (FP64 or mixed) with scalar Jacobi or none run with the rows
// streamed from memory at every product, on workgroups of 512 lanes x 2 rows
// (systems of up to 1024 rows) or 1024 lanes x 2 rows (up to 2048, one system
// each); GMRES (FP64 or mixed) on workgroups of 1024 lanes x 1 row, one
// system each, with 16 FP64 (31 FP32) basis vectors in LDS and the rest in
// registers, and beyond 1024 rows (FP64) on 1024 lanes x 2 rows with the basis
// in device memory, taken from a stream-ordered allocation for the launch.  Paper Sec. 3.5 keeps on chip what fits and leaves the rest in
// global memory; here the matrix is what leaves, the Krylov vectors stay on
// chip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/batchsolve.h"
#include "bs_varlen.hpp"

namespace bs {

namespace {
using SS = VarShape<512, 2>;    // CG, BiCGSTAB
using SS2 = VarShape<1024, 2>;  // CG, BiCGSTAB beyond 1024 rows
using SG = VarShape<1024, 1>;   // GMRES: one row per lane
using SGW = VarShape<1024, 2>;  // GMRES beyond 1024 rows: basis in device memory

template <class VS, int SOLVER, bool MIXED>
hipError_t ss_launch(const KArgs& a, int team, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((k_shared_stream<VS, SOLVER, MIXED>), dim3(grid), dim3(VS::WG), 0, s, a, team);
  return hipGetLastError();
}

hipError_t gw_launch(const KArgs& a, unsigned grid, double* ws, hipStream_t s) {
  hipLaunchKernelGGL((k_gmres_wide<SGW>), dim3(grid), dim3(SGW::WG), 0, s, a, ws);
  return hipGetLastError();
}

template <class VS, int SOLVER, bool MIXED>
hipError_t ss_occupancy(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks, reinterpret_cast<const void*>(&k_shared_stream<VS, SOLVER, MIXED>), VS::WG, 0);
}

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
}  // namespace

// The streamed plan of a request, or BS_ERR_UNSUPPORTED when it has none
// (block Jacobi, ILU(0), the triangular solves, mixed GMRES beyond 1024 rows,
// more than 2048 rows, a forced team or rows per lane, mixed CG).
int stream_plan(int n, bs_solver solver, bs_precond precond, const bs_options* o,
                bs_plan_info* info) {
  if (solver != BS_CG && solver != BS_BICGSTAB && solver != BS_GMRES) return BS_ERR_UNSUPPORTED;
  if (precond != BS_PREC_NONE && precond != BS_PREC_JACOBI) return BS_ERR_UNSUPPORTED;
  if (o && (o->team != 0 || o->rows_per_lane != 0)) return BS_ERR_UNSUPPORTED;
  if (o && o->precision == BS_MIXED && solver == BS_CG) return BS_ERR_UNSUPPORTED;
  if (solver == BS_GMRES && n > SG::ROWS) {
    if (n > SGW::ROWS || (o && o->precision == BS_MIXED)) return BS_ERR_UNSUPPORTED;
    info->team = SGW::WG;
    info->rows_per_lane = SGW::R;
    info->slots = 0;
    info->group_size = SGW::WG;
    info->systems_per_group = 1;
    info->lds_bytes = var_lds_bytes<SGW>() + round16(kGmresScalars * 8);
    info->stage_values = 0;
    return BS_OK;
  }
  if (solver == BS_GMRES) {
    if (n < 1) return BS_ERR_UNSUPPORTED;
    const bool mixed = o && o->precision == BS_MIXED;
    info->team = SG::WG;
    info->rows_per_lane = 1;
    info->slots = 0;
    info->group_size = SG::WG;
    info->systems_per_group = 1;
    info->lds_bytes = var_lds_bytes<SG>() + (mixed ? stream_gmres_lds_bytes<SG, true>()
                                                   : stream_gmres_lds_bytes<SG, false>());
    info->stage_values = 0;
    return BS_OK;
  }
  if (n < 1 || n > SS2::ROWS) return BS_ERR_UNSUPPORTED;
  const bool wide = n > SS::ROWS;
  const int wg = wide ? SS2::WG : SS::WG, r = wide ? SS2::R : SS::R;
  const int team = std::max(kWave, next_pow2((n + r - 1) / r));
  info->team = team;
  info->rows_per_lane = r;
  info->slots = 0;  // streamed: no row in registers
  info->group_size = wg;
  info->systems_per_group = wg / team;
  info->lds_bytes = wide ? var_lds_bytes<SS2>() : var_lds_bytes<SS>();
  info->stage_values = 0;
  return BS_OK;
}

int stream_launch(const KArgs& a, const bs_plan_info& info, bs_solver solver, int mixed, int cus,
                  hipStream_t s) {
  if (solver == BS_GMRES && info.rows_per_lane == SGW::R) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_gmres_wide<SGW>), SGW::WG, 0) != hipSuccess)
      return BS_ERR_HIP;
    const unsigned grid =
        (unsigned)std::min<int64_t>(a.n_batch, (int64_t)std::max(per_cu, 1) * cus);
    void* ws = nullptr;
    const size_t bytes = (size_t)grid * (kMaxRestart + 1) * SGW::ROWS * sizeof(double);
    if (hipMallocAsync(&ws, bytes, s) != hipSuccess) return BS_ERR_HIP;
    const hipError_t e = gw_launch(a, grid, static_cast<double*>(ws), s);
    const hipError_t f = hipFreeAsync(ws, s);
    return (e == hipSuccess && f == hipSuccess) ? BS_OK : BS_ERR_HIP;
  }
  int per_cu = 0;
  const bool wide = solver != BS_GMRES && info.group_size == SS2::WG;
  hipError_t e = solver == BS_GMRES ? (mixed ? ss_occupancy<SG, 2, true>(&per_cu)
                                             : ss_occupancy<SG, 2, false>(&per_cu))
                 : wide ? (solver == BS_CG ? ss_occupancy<SS2, 0, false>(&per_cu)
                           : mixed        ? ss_occupancy<SS2, 1, true>(&per_cu)
                                          : ss_occupancy<SS2, 1, false>(&per_cu))
                 : solver == BS_CG ? ss_occupancy<SS, 0, false>(&per_cu)
                 : mixed           ? ss_occupancy<SS, 1, true>(&per_cu)
                                   : ss_occupancy<SS, 1, false>(&per_cu);
  if (e != hipSuccess) return BS_ERR_HIP;
  const int cap = info.systems_per_group;
  const int64_t tasks = (a.n_batch + cap - 1) / cap;
  const unsigned grid = (unsigned)std::min<int64_t>(tasks, (int64_t)std::max(per_cu, 1) * cus);
  e = solver == BS_GMRES ? (mixed ? ss_launch<SG, 2, true>(a, info.team, grid, s)
                                  : ss_launch<SG, 2, false>(a, info.team, grid, s))
      : wide ? (solver == BS_CG ? ss_launch<SS2, 0, false>(a, info.team, grid, s)
                : mixed        ? ss_launch<SS2, 1, true>(a, info.team, grid, s)
                               : ss_launch<SS2, 1, false>(a, info.team, grid, s))
      : solver == BS_CG ? ss_launch<SS, 0, false>(a, info.team, grid, s)
      : mixed           ? ss_launch<SS, 1, true>(a, info.team, grid, s)
                        : ss_launch<SS, 1, false>(a, info.team, grid, s);
  return e == hipSuccess ? BS_OK : BS_ERR_HIP;
}

}  // namespace bs
