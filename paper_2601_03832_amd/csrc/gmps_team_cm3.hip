// Team iterate kernel of class CM = 3 (float and double storage).
#include "gmps_team.h"

namespace gmps {
GMPS_TEAM_CLASS(1)
GMPS_TEAM_PC_CLASS(1)
GMPS_TEAM_CIRC_CLASS(1)
}  // namespace gmps
