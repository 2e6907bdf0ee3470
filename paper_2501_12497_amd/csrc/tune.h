// Tile-shape autotuner of the stencil kernels.
#pragma once

#include <string>

#include "common.h"

namespace mmof {

// Times every tile-shape candidate of the plan's stencil kernels in dtype dt, keeps the fastest
// in the plan's geometry and returns a one-line report ("kernel=TWxTH(us) ...").
std::string autotune(Plan& P, int dt);
// Forces candidate `choice` of a tunable kernel (blur, grad_fwd, grad_adj, flow_fwd, flow_adj).
void set_tile(Plan& P, const std::string& kernel, int dt, int choice);

}  // namespace mmof
