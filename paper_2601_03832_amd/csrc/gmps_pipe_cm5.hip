// Pipelined-reflections kernel of team class CM = 5 (float and double storage).
#include "gmps_pipe.h"

namespace gmps {
GMPS_PIPE_CLASS(2)
}  // namespace gmps
