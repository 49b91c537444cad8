// Kernel instances of the batched triangular solve (lower and upper), one row
// per lane.
#include "bs_registry.hpp"
#include "bs_solvers.hpp"

namespace bs {
namespace {

template <class S, bool LOWER>
hipError_t launch(const KArgs& a, unsigned grid, unsigned lds, hipStream_t stream) {
  hipLaunchKernelGGL((k_trsv<S, LOWER>), dim3(grid), dim3(S::WG), lds, stream, a);
  return hipGetLastError();
}

template <class S, bool LOWER>
int occupancy(unsigned lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_trsv<S, LOWER>),
                                                   S::WG, lds) != hipSuccess || n < 1)
    n = 1;
  return n;
}

#define ENTRY_L(T, R, NZ) {V_TRSV_LOWER, T, R, NZ, Shape<T, R, NZ>::WG, &launch<Shape<T, R, NZ>, true>, &occupancy<Shape<T, R, NZ>, true>},
#define ENTRY_U(T, R, NZ) {V_TRSV_UPPER, T, R, NZ, Shape<T, R, NZ>::WG, &launch<Shape<T, R, NZ>, false>, &occupancy<Shape<T, R, NZ>, false>},
const KernelEntry kLower[] = {BS_SHAPES_W64(ENTRY_L) BS_SHAPES_MW512(ENTRY_L) BS_SHAPES_MW1024(ENTRY_L)};
const KernelEntry kUpper[] = {BS_SHAPES_W64(ENTRY_U) BS_SHAPES_MW512(ENTRY_U) BS_SHAPES_MW1024(ENTRY_U)};
#undef ENTRY_L
#undef ENTRY_U

}  // namespace

KernelTable kernels_trsv_lower() { return {kLower, (int)(sizeof(kLower) / sizeof(kLower[0]))}; }
KernelTable kernels_trsv_upper() { return {kUpper, (int)(sizeof(kUpper) / sizeof(kUpper[0]))}; }

}  // namespace bs
