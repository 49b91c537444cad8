// Registry of the compiled kernel instances: the host planner looks a request
// up here by (variant, team, rows per lane, slots per row).
#pragma once
#include <hip/hip_runtime.h>

#include "bs_shape.hpp"

namespace bs {

// *_BJ: the FP64 solvers with the block-Jacobi preconditioner; *_ILU: with
// ILU(0); V_TRSV_*: the triangular solves (one row per lane for both).
enum Variant {
  V_CG = 0, V_BICGSTAB = 1, V_GMRES = 2, V_BICGSTAB_MIXED = 3, V_GMRES_MIXED = 4,
  V_CG_BJ = 5, V_BICGSTAB_BJ = 6, V_GMRES_BJ = 7, V_BICGSTAB_ILU = 8, V_GMRES_ILU = 9,
  V_TRSV_LOWER = 10, V_TRSV_UPPER = 11, V_COUNT = 12
};

typedef hipError_t (*LaunchFn)(const KArgs& a, unsigned grid, unsigned lds, hipStream_t stream);
// Resident workgroups per compute unit for a given dynamic LDS size.
typedef int (*OccupancyFn)(unsigned lds);

struct KernelEntry {
  int variant, team, r, nz, wg;
  LaunchFn launch;
  OccupancyFn occupancy;
};

struct KernelTable {
  const KernelEntry* entries;
  int count;
};

KernelTable kernels_cg();
KernelTable kernels_bicgstab();
KernelTable kernels_bicgstab_mixed();
KernelTable kernels_gmres();
KernelTable kernels_gmres_mixed();
KernelTable kernels_cg_bj();
KernelTable kernels_bicgstab_bj();
KernelTable kernels_gmres_bj();
KernelTable kernels_bicgstab_ilu();
KernelTable kernels_gmres_ilu();
KernelTable kernels_trsv_lower();
KernelTable kernels_trsv_upper();

// Shapes compiled for every solver: one row per lane for teams of 16..1024
// lanes, and 2 or 4 rows per lane for the largest systems.  Slots per row are
// capped where the registers of a full workgroup would overflow.
#define BS_SHAPES_R1(X)                                                                   \
  X(16, 1, 4) X(16, 1, 8) X(16, 1, 16)                                                    \
  X(32, 1, 4) X(32, 1, 8) X(32, 1, 16) X(32, 1, 24) X(32, 1, 32)                         \
  X(64, 1, 4) X(64, 1, 8) X(64, 1, 16) X(64, 1, 24) X(64, 1, 28) X(64, 1, 32) X(64, 1, 56)  \
  X(64, 1, 64)                                                                            \
  X(128, 1, 4) X(128, 1, 8) X(128, 1, 16) X(128, 1, 32) X(128, 1, 56) X(128, 1, 64)       \
  X(256, 1, 4) X(256, 1, 8) X(256, 1, 16) X(256, 1, 32) X(256, 1, 56) X(256, 1, 64)       \
  X(512, 1, 4) X(512, 1, 8) X(512, 1, 16) X(512, 1, 32)                                   \
  X(1024, 1, 4) X(1024, 1, 8) X(1024, 1, 12) X(1024, 1, 16)
// ILU(0) and BatchTrsv shapes: one-wave teams (systems of up to 64 rows, dense
// factors) and multi-wave teams of one row per lane (65..1024 rows, sparse
// factors, level-scheduled sweeps; GMRES with ILU(0) up to 512 rows, where its
// basis stays in registers).
#define BS_SHAPES_W64(X)                                                                  \
  X(64, 1, 4) X(64, 1, 8) X(64, 1, 16) X(64, 1, 24) X(64, 1, 28) X(64, 1, 32) X(64, 1, 64)
#define BS_SHAPES_MW512(X)                                                                \
  X(128, 1, 4) X(128, 1, 8) X(128, 1, 16) X(128, 1, 32) X(128, 1, 64)                     \
  X(256, 1, 4) X(256, 1, 8) X(256, 1, 16) X(256, 1, 32) X(256, 1, 64)                     \
  X(512, 1, 4) X(512, 1, 8) X(512, 1, 16) X(512, 1, 32)
#define BS_SHAPES_MW1024(X) X(1024, 1, 4) X(1024, 1, 8) X(1024, 1, 12) X(1024, 1, 16)
#define BS_SHAPES_RN(X)                                                                   \
  X(512, 2, 8) X(512, 2, 16) X(1024, 2, 8) X(256, 4, 8) X(512, 4, 8)

}  // namespace bs
