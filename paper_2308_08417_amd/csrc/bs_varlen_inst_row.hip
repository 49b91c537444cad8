// Uneven-batch kernels that walk the row-ordered index (the CSR order of
// values stored in another layout): rows in registers (8..16 slots; CG,
// BiCGSTAB, mixed BiCGSTAB) and the streamed placement.
#include "bs_varlen_table.hpp"

namespace bs {
namespace {
#define REG_NZ(W, R) BS_VREG_SOLVERS_NOBJ(W, R, 8, kSrcRowIdx) BS_VREG_SOLVERS_NOBJ(W, R, 10, kSrcRowIdx) \
  BS_VREG_SOLVERS_NOBJ(W, R, 12, kSrcRowIdx) BS_VREG_SOLVERS_NOBJ(W, R, 16, kSrcRowIdx)
const VEntry kTable[] = {REG_NZ(1024, 1) REG_NZ(512, 2) REG_NZ(256, 4)
                         BS_VSTREAM_SOLVERS(1024, 1, kSrcRowIdx)
                         BS_VSTREAM_SOLVERS(512, 2, kSrcRowIdx)
                         BS_VSTREAM_SOLVERS(256, 4, kSrcRowIdx)};
#undef REG_NZ
}  // namespace

const VEntry* vtable_row(int* count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace bs
