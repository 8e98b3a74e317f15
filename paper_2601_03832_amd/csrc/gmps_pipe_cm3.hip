// Pipelined-reflections kernel of team class CM = 3 (float and double storage).
#include "gmps_pipe.h"

namespace gmps {
GMPS_PIPE_CLASS(1)
}  // namespace gmps
