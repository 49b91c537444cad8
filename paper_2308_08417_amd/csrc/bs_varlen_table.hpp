// Compiled instances of the uneven-batch kernel and their launch wrappers.
// Every instance is one entry of a table: workgroup shape (lanes, rows per
// lane), slots per row held in registers (0 for the streamed placement),
// solver, precision, block Jacobi, where the rows are read from (kSrc*) and
// the placement.  The tables are split over three translation units (one per
// source) so that they compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "bs_varlen.hpp"

namespace bs {

typedef hipError_t (*VLaunch)(const VArgs&, unsigned grid, hipStream_t);
typedef hipError_t (*VOccupancy)(int*);

template <class VS, class RowsT, int SOLVER, bool MIXED, bool BJ>
hipError_t vlaunch(const VArgs& a, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((k_varlen<VS, RowsT, SOLVER, MIXED, BJ>), dim3(grid), dim3(VS::WG), 0, s, a);
  return hipGetLastError();
}

template <class VS, class RowsT, int SOLVER, bool MIXED, bool BJ>
hipError_t voccupancy(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks, reinterpret_cast<const void*>(&k_varlen<VS, RowsT, SOLVER, MIXED, BJ>), VS::WG, 0);
}

struct VEntry {
  int wg, r, nz, solver, mixed, bj, src, stream;
  VLaunch fn;
  VOccupancy occ;
};

// Registers: SO = 0 CG, 1 BiCGSTAB; MX mixed; BJ block Jacobi.
#define BS_VREG(W, R, NZ, SO, MX, BJ, SRC)                                                      \
  {W, R, NZ, SO, MX, BJ, SRC, 0,                                                                \
   &bs::vlaunch<bs::VarShape<W, R>, bs::VarRows<bs::VarShape<W, R>, NZ, SRC, MX>, SO, MX, BJ>,  \
   &bs::voccupancy<bs::VarShape<W, R>, bs::VarRows<bs::VarShape<W, R>, NZ, SRC, MX>, SO, MX, BJ>},
#define BS_VSTREAM(W, R, SO, MX, SRC)                                                           \
  {W, R, 0, SO, MX, 0, SRC, 1,                                                                  \
   &bs::vlaunch<bs::VarShape<W, R>, bs::VarRowsS<bs::VarShape<W, R>, SRC>, SO, MX, false>,      \
   &bs::voccupancy<bs::VarShape<W, R>, bs::VarRowsS<bs::VarShape<W, R>, SRC>, SO, MX, false>},
// CG, BiCGSTAB, mixed BiCGSTAB; with BJ also CG and BiCGSTAB with block Jacobi
#define BS_VREG_SOLVERS(W, R, NZ, SRC)                                               \
  BS_VREG(W, R, NZ, 0, false, false, SRC) BS_VREG(W, R, NZ, 1, false, false, SRC)              \
  BS_VREG(W, R, NZ, 1, true, false, SRC)                                                        \
  BS_VREG(W, R, NZ, 0, false, true, SRC) BS_VREG(W, R, NZ, 1, false, true, SRC)
#define BS_VREG_SOLVERS_NOBJ(W, R, NZ, SRC)                                                     \
  BS_VREG(W, R, NZ, 0, false, false, SRC) BS_VREG(W, R, NZ, 1, false, false, SRC)              \
  BS_VREG(W, R, NZ, 1, true, false, SRC)
#define BS_VSTREAM_SOLVERS(W, R, SRC)                                                           \
  BS_VSTREAM(W, R, 0, false, SRC) BS_VSTREAM(W, R, 1, false, SRC) BS_VSTREAM(W, R, 1, true, SRC)

// One table per source (defined in bs_varlen_inst_*.hip).
const VEntry* vtable_csr(int* count);
const VEntry* vtable_row(int* count);
const VEntry* vtable_slot(int* count);

}  // namespace bs
