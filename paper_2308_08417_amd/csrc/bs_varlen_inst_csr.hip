// Uneven-batch kernels that read the CSR arrays themselves: rows in registers
// (8..16 slots, every solver form) and the streamed placement.
#include "bs_varlen_table.hpp"

namespace bs {
namespace {
#define REG_NZ(W, R) BS_VREG_SOLVERS(W, R, 8, kSrcCsr) BS_VREG_SOLVERS(W, R, 10, kSrcCsr) \
  BS_VREG_SOLVERS(W, R, 12, kSrcCsr) BS_VREG_SOLVERS(W, R, 16, kSrcCsr)
const VEntry kTable[] = {REG_NZ(1024, 1) REG_NZ(512, 2) REG_NZ(256, 4)
                         BS_VSTREAM_SOLVERS(1024, 1, kSrcCsr) BS_VSTREAM_SOLVERS(512, 2, kSrcCsr)
                         BS_VSTREAM_SOLVERS(256, 4, kSrcCsr)};
#undef REG_NZ
}  // namespace

const VEntry* vtable_csr(int* count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace bs
