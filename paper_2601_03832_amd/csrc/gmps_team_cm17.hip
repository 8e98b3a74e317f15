// Team iterate kernel of class CM = 17 (float and double storage).
#include "gmps_team.h"

namespace gmps {
GMPS_TEAM_CLASS(4)
GMPS_TEAM_PC_CLASS(4)
GMPS_TEAM_CIRC_CLASS(4)
}  // namespace gmps
