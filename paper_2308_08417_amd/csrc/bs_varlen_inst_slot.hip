// Uneven-batch kernels that walk the slot-major index (the ELL order): rows in
// registers (8..16 slots, every solver form) and the streamed placement.
#include "bs_varlen_table.hpp"

namespace bs {
namespace {
#define REG_NZ(W, R) BS_VREG_SOLVERS(W, R, 8, kSrcSlotIdx) BS_VREG_SOLVERS(W, R, 10, kSrcSlotIdx) \
  BS_VREG_SOLVERS(W, R, 12, kSrcSlotIdx) BS_VREG_SOLVERS(W, R, 16, kSrcSlotIdx)
const VEntry kTable[] = {REG_NZ(1024, 1) REG_NZ(512, 2) REG_NZ(256, 4)
                         BS_VSTREAM_SOLVERS(1024, 1, kSrcSlotIdx)
                         BS_VSTREAM_SOLVERS(512, 2, kSrcSlotIdx)
                         BS_VSTREAM_SOLVERS(256, 4, kSrcSlotIdx)};
#undef REG_NZ
}  // namespace

const VEntry* vtable_slot(int* count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace bs
