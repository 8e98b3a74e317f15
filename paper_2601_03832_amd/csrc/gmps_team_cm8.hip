// Team iterate kernel of class CM = 8 (float and double storage).
#include "gmps_team.h"

namespace gmps {
GMPS_TEAM_CLASS(3)
GMPS_TEAM_PC_CLASS(3)
GMPS_TEAM_CIRC_CLASS(3)
}  // namespace gmps
