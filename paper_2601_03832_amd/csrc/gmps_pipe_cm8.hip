// Pipelined-reflections kernel of team class CM = 8 (float and double storage).
#include "gmps_pipe.h"

namespace gmps {
GMPS_PIPE_CLASS(3)
}  // namespace gmps
