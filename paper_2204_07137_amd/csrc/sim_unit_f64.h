// The FP64 instantiation of the window kernels (reference-precision path on the GPU), shared by
// the FP64 translation units; each unit sets SIM_EMIT_* before including this file.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "sim_types.h"

// DOF counts compiled as kernels of their own: the humanoid's 27, for torque and muscle models,
// so that the FP64 parity runs cover the DOF-specialised kernel of the production path; every
// other model runs the padded 32-DOF kernel.  No compact layout in FP64 (the FP32 compact
// kernels are checked bitwise against the full ones).
#define SIM_NV_LIST(X) X(27)
#define SIM_NV_LIST_MTU(X) X(27)
#define SIM_COMPACT 0
#define SIM_NV_LIST_SMALL(X)

namespace sim_f64 {
typedef double real;
#include "sim_math.h"
#include "sim_dynamics.h"
#include "sim_task.h"
#include "sim_kernels.h"
#if SIM_EMIT_MAIN
#include "sim_gemm.h"
#endif
}  // namespace sim_f64
