#pragma once

#include "common.h"

namespace mmof {

int solve_joint(Plan& P, const double* b, double delta, const mmof_solve_params& p, double* u_io, void* v_out,
                void* vr_out, mmof_report* rep);

}  // namespace mmof
