// Pipelined-reflections kernel of team class CM = 2 (float and double storage).
#include "gmps_pipe.h"

namespace gmps {
GMPS_PIPE_CLASS(0)
}  // namespace gmps
