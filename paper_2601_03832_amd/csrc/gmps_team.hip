// Host-side helpers of the team iterate kernels: class geometry, LDS sizes and launches
// (the kernels themselves are instantiated per class in gmps_team_cm*.hip).
#include "gmps_pipe.h"

namespace gmps {

int team_per_bundle(int cls) {
  const int tw = kWide[cls - kWideBase].TW;
  return tw < 64 ? 64 / tw : 1;
}

// every class fits the 160 KiB of LDS of a gfx950 compute unit (with the kernel's own
// bundle index and the FP64 storage type, the larger of the two), with the pre-contracted
// reflections' block where the class has them
static_assert((sizeof(TeamLds<double, 2, 16>) + sizeof(PcLds<2>)) * 4 <= 160 * 1024 - 64, "LDS");
static_assert((sizeof(TeamLds<double, 3, 32>) + sizeof(PcLds<3>)) * 2 <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 5, 64>) + sizeof(PcLds<5>) <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 8, 64>) + sizeof(PcLds<8>) <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 17, 192>) + sizeof(PcLds<17>) <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 32, 256>) <= 160 * 1024 - 64, "LDS");
// with the gate-level circuit block (classes up to bond 17)
static_assert((sizeof(TeamLds<double, 2, 16>) + sizeof(CircLds)) * 4 <= 160 * 1024 - 64, "LDS");
static_assert((sizeof(TeamLds<double, 3, 32>) + sizeof(CircLds)) * 2 <= 160 * 1024 - 64, "LDS");
static_assert(sizeof(TeamLds<double, 17, 192>) + sizeof(CircLds) <= 160 * 1024 - 64, "LDS");

// the pipelined kernel, with the pre-contracted reflections' overlap block
static_assert((sizeof(PipeLds<double, 2>) + sizeof(PipeOv<2>)) * 4 <= 160 * 1024 - 256, "LDS");
static_assert((sizeof(PipeLds<double, 3>) + sizeof(PipeOv<3>)) * 2 <= 160 * 1024 - 256, "LDS");
static_assert(sizeof(PipeLds<double, 5>) + sizeof(PipeOv<5>) <= 160 * 1024 - 256, "LDS");
static_assert(sizeof(PipeLds<double, 8>) + sizeof(PipeOv<8>) <= 160 * 1024 - 256, "LDS");

// the classes with a pipelined kernel (teams within one wave: bond caps 2, 3, 5 and 8)
static bool pipe_class(int w, bool, bool) { return w >= 0 && w < kNumWide && team_pipe_class(w); }

template <int W>
static size_t pipe_lds(bool mixed, bool pc) {
  constexpr int CM = kWide[W].CM, TW = kWide[W].TW;
  const size_t per = (mixed ? sizeof(PipeLds<float, CM>) : sizeof(PipeLds<double, CM>)) + (pc ? sizeof(PipeOv<CM>) : 0);
  return per * (64 / TW);
}

template <int W>
static size_t class_lds(bool mixed, bool pc) {
  constexpr int CM = kWide[W].CM, TW = kWide[W].TW;
  constexpr int teams = TeamShape<CM, TW>::TEAMS;
  size_t per = mixed ? sizeof(TeamLds<float, CM, TW>) : sizeof(TeamLds<double, CM, TW>);
  if (pc && team_pc_class(W)) per += sizeof(PcLds<CM>);
  return per * teams;
}

size_t team_lds_bytes(bool mixed, bool pc, bool pipe, int cls) {
  if (pipe && pipe_class(cls - kWideBase, mixed, pc)) {
    switch (cls - kWideBase) {
      case 0: return pipe_lds<0>(mixed, pc);
      case 1: return pipe_lds<1>(mixed, pc);
      case 2: return pipe_lds<2>(mixed, pc);
      case 3: return pipe_lds<3>(mixed, pc);
    }
  }
  switch (cls - kWideBase) {
    case 0: return class_lds<0>(mixed, pc);
    case 1: return class_lds<1>(mixed, pc);
    case 2: return class_lds<2>(mixed, pc);
    case 3: return class_lds<3>(mixed, pc);
    case 4: return class_lds<4>(mixed, pc);
    case 5: return class_lds<5>(mixed, pc);
  }
  return 0;
}

// Gate-level circuits: the sequential team kernel with the circuit block after the team blocks
// (FP64, classes with bond caps up to 17).
size_t team_circ_lds_bytes(int cls) {
  const int w = cls - kWideBase;
  size_t teams = 0, base = 0;
  switch (w) {
    case 0: base = class_lds<0>(false, false); teams = TeamShape<kWide[0].CM, kWide[0].TW>::TEAMS; break;
    case 1: base = class_lds<1>(false, false); teams = TeamShape<kWide[1].CM, kWide[1].TW>::TEAMS; break;
    case 2: base = class_lds<2>(false, false); teams = TeamShape<kWide[2].CM, kWide[2].TW>::TEAMS; break;
    case 3: base = class_lds<3>(false, false); teams = TeamShape<kWide[3].CM, kWide[3].TW>::TEAMS; break;
    case 4: base = class_lds<4>(false, false); teams = TeamShape<kWide[4].CM, kWide[4].TW>::TEAMS; break;
    default: return 0;
  }
  return base + teams * sizeof(CircLds);
}

hipError_t launch_team_circ(int cls, const IterParams& P, int grid, size_t lds, hipStream_t st) {
  switch (cls - kWideBase) {
    case 0: return launch_team_circ_w<0>(P, grid, lds, st);
    case 1: return launch_team_circ_w<1>(P, grid, lds, st);
    case 2: return launch_team_circ_w<2>(P, grid, lds, st);
    case 3: return launch_team_circ_w<3>(P, grid, lds, st);
    case 4: return launch_team_circ_w<4>(P, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

hipError_t team_circ_occupancy(int cls, size_t lds, int* blocks_per_cu) {
  switch (cls - kWideBase) {
    case 0: return occupancy_team_circ_w<0>(lds, blocks_per_cu);
    case 1: return occupancy_team_circ_w<1>(lds, blocks_per_cu);
    case 2: return occupancy_team_circ_w<2>(lds, blocks_per_cu);
    case 3: return occupancy_team_circ_w<3>(lds, blocks_per_cu);
    case 4: return occupancy_team_circ_w<4>(lds, blocks_per_cu);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_team(bool mixed, bool pc, bool pipe, int cls, const IterParams& P, int grid, size_t lds,
                       hipStream_t st) {
  const int w = cls - kWideBase;
  if (pipe && pipe_class(w, mixed, pc)) {
    switch (w) {
      case 0: return launch_pipe_w<0>(mixed, pc, P, grid, lds, st);
      case 1: return launch_pipe_w<1>(mixed, pc, P, grid, lds, st);
      case 2: return launch_pipe_w<2>(mixed, pc, P, grid, lds, st);
      case 3: return launch_pipe_w<3>(mixed, pc, P, grid, lds, st);
    }
  }
  if (pc && w >= 0 && w < kNumWide && team_pc_class(w)) {
    switch (w) {
      case 0: return launch_team_pc_w<0>(mixed, P, grid, lds, st);
      case 1: return launch_team_pc_w<1>(mixed, P, grid, lds, st);
      case 2: return launch_team_pc_w<2>(mixed, P, grid, lds, st);
      case 3: return launch_team_pc_w<3>(mixed, P, grid, lds, st);
      case 4: return launch_team_pc_w<4>(mixed, P, grid, lds, st);
    }
    return hipErrorInvalidValue;
  }
  switch (w) {
    case 0: return launch_team_w<0>(mixed, P, grid, lds, st);
    case 1: return launch_team_w<1>(mixed, P, grid, lds, st);
    case 2: return launch_team_w<2>(mixed, P, grid, lds, st);
    case 3: return launch_team_w<3>(mixed, P, grid, lds, st);
    case 4: return launch_team_w<4>(mixed, P, grid, lds, st);
    case 5: return launch_team_w<5>(mixed, P, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

hipError_t team_occupancy(bool mixed, bool pc, bool pipe, int cls, size_t lds, int* blocks_per_cu) {
  const int w = cls - kWideBase;
  if (pipe && pipe_class(w, mixed, pc)) {
    switch (w) {
      case 0: return occupancy_pipe_w<0>(mixed, pc, lds, blocks_per_cu);
      case 1: return occupancy_pipe_w<1>(mixed, pc, lds, blocks_per_cu);
      case 2: return occupancy_pipe_w<2>(mixed, pc, lds, blocks_per_cu);
      case 3: return occupancy_pipe_w<3>(mixed, pc, lds, blocks_per_cu);
    }
  }
  if (pc && w >= 0 && w < kNumWide && team_pc_class(w)) {
    switch (w) {
      case 0: return occupancy_team_pc_w<0>(mixed, lds, blocks_per_cu);
      case 1: return occupancy_team_pc_w<1>(mixed, lds, blocks_per_cu);
      case 2: return occupancy_team_pc_w<2>(mixed, lds, blocks_per_cu);
      case 3: return occupancy_team_pc_w<3>(mixed, lds, blocks_per_cu);
      case 4: return occupancy_team_pc_w<4>(mixed, lds, blocks_per_cu);
    }
    return hipErrorInvalidValue;
  }
  switch (w) {
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
