// Kernel instances of the FP64 BiCGSTAB solver with the ILU(0)
// preconditioner (one row per lane).
#include "bs_registry.hpp"
#include "bs_solvers.hpp"

namespace bs {
namespace {

template <class S>
hipError_t launch(const KArgs& a, unsigned grid, unsigned lds, hipStream_t stream) {
  hipLaunchKernelGGL((k_bicgstab<S, false, kPkIlu>), dim3(grid), dim3(S::WG), lds, stream, a);
  return hipGetLastError();
}

template <class S>
int occupancy(unsigned lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_bicgstab<S, false, kPkIlu>), S::WG,
                                                   lds) != hipSuccess || n < 1)
    n = 1;
  return n;
}

#define ENTRY(T, R, NZ) {V_BICGSTAB_ILU, T, R, NZ, Shape<T, R, NZ>::WG, &launch<Shape<T, R, NZ>>, &occupancy<Shape<T, R, NZ>>},
const KernelEntry kTable[] = {BS_SHAPES_W64(ENTRY) BS_SHAPES_MW512(ENTRY) BS_SHAPES_MW1024(ENTRY)};
#undef ENTRY

}  // namespace

KernelTable kernels_bicgstab_ilu() { return {kTable, (int)(sizeof(kTable) / sizeof(kTable[0]))}; }

}  // namespace bs
