// Team iterate kernel of class CM = 32 (float and double storage).
#include "gmps_team.h"

namespace gmps {
GMPS_TEAM_CLASS(5)
}  // namespace gmps
