// Host-side launchers of the HIP kernels (one translation unit per operator family).
#pragma once

#include "common.h"

namespace mmof {

// Psi and Psi^T (eq. L); weights optional.
void launch_grad_fwd(Ctx& c, Geom& g, int dt, const void* u, const void* wx, const void* wy, void* gx, void* gy);
void launch_grad_adj(Ctx& c, Geom& g, int dt, const void* gx, const void* gy, const void* wx, const void* wy,
                     void* u, bool accumulate);

// L(v) = -M-bar (direction +1) / -M-bar' (direction -1) and relatives.
void launch_flow_fwd(Ctx& c, Geom& g, int dt, int direction, int interp, const void* u, const void* v, void* r);
void launch_flow_adj(Ctx& c, Geom& g, int dt, int direction, int interp, const void* r, const void* v, void* u,
                     bool accumulate, const int32_t* d_radius /* device int: floor(max|v|)+1, or null */);
void launch_flow_dv(Ctx& c, Geom& g, int dt, int direction, int interp, const void* u, const void* v,
                    const void* w, void* gv);
// Device int *d_out = floor(max |v|) + 1 over all pairs (saturating at 1<<20, NaN -> saturate).
void launch_flow_radius(Ctx& c, Geom& g, int dt, const void* v, int32_t* d_out);

// App. C derivatives, Horn-Schunck sweeps, reverse flow.
void launch_of_derivs(Ctx& c, Geom& g, int dt, const void* u, void* I, int dr);
// n_sweeps Horn-Schunck sweeps starting from v, several per launch, ping-ponging between
// v and tmp; returns 1 when the result is in tmp, 0 when it is in v.
int launch_hs_sweeps(Ctx& c, Geom& g, int dt, const void* I, void* v, void* tmp, double gamma, int n_sweeps);
void launch_reverse_flow(Ctx& c, Geom& g, int dt, const void* v, void* vr, const int32_t* d_radius);

// Elementwise.
void launch_mm_weights(Ctx& c, int dt, int64_t n, const void* nu, double eps, void* w2);

// Forward operators.
void launch_radon_fwd(Ctx& c, Plan& p, int dt, const void* u, void* b);
void launch_radon_adj(Ctx& c, Plan& p, int dt, const void* b, void* u);
void launch_blur(Ctx& c, Plan& p, int dt, const void* in, void* out);

}  // namespace mmof
