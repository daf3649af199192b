// Host-side helpers shared by the runtime's translation units.
#pragma once

#include "gsr.h"

namespace gsr {

// Record `msg` as the context's last error and return `s`.
gsr_status ctx_error(gsr_ctx *c, gsr_status s, const char *msg);

// Drop the context's plan: render calls fail with NOT_PLANNED until the
// next gsr_plan.
void ctx_unplan(gsr_ctx *c);

}  // namespace gsr
