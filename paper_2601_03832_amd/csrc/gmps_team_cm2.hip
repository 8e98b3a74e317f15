// Team iterate kernel of class CM = 2 (float and double storage).
#include "gmps_team.h"

namespace gmps {
GMPS_TEAM_CLASS(0)
GMPS_TEAM_PC_CLASS(0)
GMPS_TEAM_CIRC_CLASS(0)
}  // namespace gmps
