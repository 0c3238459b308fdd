// The library's error message (lbm_last_error), shared by the 2-D and 3-D entry points.
#pragma once

#include "../../include/lbm.h"

namespace lbm {
lbm_status set_error(lbm_status st, const char *msg);
}
