// The wheeled carriage (section "Rigid Body Joints and Contact"): every
// segment carries two rigid wheels on hinge joints, and the wheels carry the
// ground contact with Coulomb friction at the wheel's contact point.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace snake {

// Wheel state, structure of arrays over 2N wheels; wheel 2 gb + k belongs to
// body gb (k = 0 on the body's +y side).
struct WParams {
    float* x;     // [3][2N] centres
    float* q;     // [4][2N] (w, x, y, z)
    float* v;     // [3][2N]
    float* w;     // [3][2N] angular velocity, world
    float* lam;   // [9][2N] hinge position (3), hinge axis (x, spin = 0, z),
                  // contact (normal, tangential x, tangential y)
    double mw, rw;   // wheel mass and radius
    double dw, hw;   // wheel centre at (0, +-dw, -hw) in its segment's frame
    double Ip, Ia;   // wheel inertia about a diameter and about the axle
    double relax;
};

// Wheels of every body at their hinge points, at rest, zero multipliers
// (after the chain's own initial state).
hipError_t launch_init_wheels(const KParams& P, const WParams& Wp, hipStream_t stream);

// n_steps steps of every snake with block-Jacobi iterations on the chain's
// joints and the wheels' hinge and contact blocks, in double; snakes grouped
// by lane class as for the Newton solver (list, off[9]).
hipError_t launch_carriage(const KParams& P, const NParams& Q, const WParams& Wp, const int* list, const int* off,
                           int n_steps, hipStream_t stream);

}  // namespace snake
