// The FP32 instantiation of the window kernels (the production path), shared by the FP32
// translation units; each unit sets SIM_EMIT_* before including this file.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "sim_types.h"

// DOF counts compiled as kernels of their own: torque models (CartPole, Ant, Humanoid), muscle
// models (the humanoid skeleton), and the compact layout (small models, 16 / 32 / 64 lanes per
// environment)
#define SIM_NV_LIST(X) X(2) X(14) X(27)
#define SIM_NV_LIST_MTU(X) X(27)
#define SIM_COMPACT 1
#define SIM_NV_LIST_SMALL(X) X(2) X(14)

namespace sim_f32 {
typedef float real;
#include "sim_math.h"
#include "sim_dynamics.h"
#include "sim_task.h"
#include "sim_kernels.h"
#if SIM_EMIT_MAIN
#include "sim_gemm.h"
#endif
}  // namespace sim_f32
