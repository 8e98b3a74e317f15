// Host-side helpers of the team iterate kernels: class geometry, LDS sizes and launches
// (the kernels themselves are instantiated per class in gmps_team_cm*.hip).
#include "gmps_team.h"

namespace gmps {

int team_per_bundle(int cls) {
  const int tw = kWide[cls - kWideBase].TW;
  return tw < 64 ? 64 / tw : 1;
}

// every class fits the 160 KiB of LDS of a gfx950 compute unit (with the kernel's own
// bundle index and the FP64 storage type, the larger of the two)
static_assert(sizeof(TeamLds<double, 2, 16>) * 4 <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 3, 32>) * 2 <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 8, 64>) <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 17, 192>) <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 32, 256>) <= 160 * 1024 - 64, "LDS");

size_t team_lds_bytes(bool mixed, int cls) {
  switch (cls - kWideBase) {
    case 0: return (mixed ? sizeof(TeamLds<float, 2, 16>) : sizeof(TeamLds<double, 2, 16>)) * 4;
    case 1: return (mixed ? sizeof(TeamLds<float, 3, 32>) : sizeof(TeamLds<double, 3, 32>)) * 2;
    case 2: return mixed ? sizeof(TeamLds<float, 5, 64>) : sizeof(TeamLds<double, 5, 64>);
    case 3: return mixed ? sizeof(TeamLds<float, 8, 64>) : sizeof(TeamLds<double, 8, 64>);
    case 4: return mixed ? sizeof(TeamLds<float, 17, 192>) : sizeof(TeamLds<double, 17, 192>);
    case 5: return mixed ? sizeof(TeamLds<float, 32, 256>) : sizeof(TeamLds<double, 32, 256>);
  }
  return 0;
}

hipError_t launch_team(bool mixed, int cls, const IterParams& P, int grid, size_t lds, hipStream_t st) {
  switch (cls - kWideBase) {
    case 0: return launch_team_w<0>(mixed, P, grid, lds, st);
    case 1: return launch_team_w<1>(mixed, P, grid, lds, st);
    case 2: return launch_team_w<2>(mixed, P, grid, lds, st);
    case 3: return launch_team_w<3>(mixed, P, grid, lds, st);
    case 4: return launch_team_w<4>(mixed, P, grid, lds, st);
    case 5: return launch_team_w<5>(mixed, P, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

hipError_t team_occupancy(bool mixed, int cls, size_t lds, int* blocks_per_cu) {
  switch (cls - kWideBase) {
    case 0: return occupancy_team_w<0>(mixed, lds, blocks_per_cu);
    case 1: return occupancy_team_w<1>(mixed, lds, blocks_per_cu);
    case 2: return occupancy_team_w<2>(mixed, lds, blocks_per_cu);
    case 3: return occupancy_team_w<3>(mixed, lds, blocks_per_cu);
    case 4: return occupancy_team_w<4>(mixed, lds, blocks_per_cu);
    case 5: return occupancy_team_w<5>(mixed, lds, blocks_per_cu);
  }
  return hipErrorInvalidValue;
}

}  // namespace gmps
