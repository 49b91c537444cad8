// Kernel instances of the FP64 GMRES solver with the block-Jacobi
// preconditioner for every compiled shape.
#include "bs_registry.hpp"
#include "bs_solvers.hpp"

namespace bs {
namespace {

template <class S>
hipError_t launch(const KArgs& a, unsigned grid, unsigned lds, hipStream_t stream) {
  hipLaunchKernelGGL((k_gmres<S, false, kPkBlock>), dim3(grid), dim3(S::WG), lds, stream, a);
  return hipGetLastError();
}

template <class S>
int occupancy(unsigned lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_gmres<S, false, kPkBlock>), S::WG,
                                                   lds) != hipSuccess || n < 1)
    n = 1;
  return n;
}

#define ENTRY(T, R, NZ) {V_GMRES_BJ, T, R, NZ, Shape<T, R, NZ>::WG, &launch<Shape<T, R, NZ>>, &occupancy<Shape<T, R, NZ>>},
const KernelEntry kTable[] = {BS_SHAPES_R1(ENTRY)};
#undef ENTRY

}  // namespace

KernelTable kernels_gmres_bj() { return {kTable, (int)(sizeof(kTable) / sizeof(kTable[0]))}; }

}  // namespace bs
