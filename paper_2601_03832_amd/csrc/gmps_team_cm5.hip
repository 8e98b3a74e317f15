// Team iterate kernel of class CM = 5 (float and double storage).
#include "gmps_team.h"

namespace gmps {
GMPS_TEAM_CLASS(2)
GMPS_TEAM_PC_CLASS(2)
GMPS_TEAM_CIRC_CLASS(2)
}  // namespace gmps
