// FP64 instantiation of the window kernels (reference-precision path on the GPU).
#include <hip/hip_runtime.h>
#include <math.h>
#include "sim_types.h"

// FP64 path: every model runs the padded 32-DOF kernel
// DOF counts of muscle-driven models with a kernel of their own (the humanoid skeleton)
#define SIM_NV_LIST_MTU(X)
#define SIM_NV_LIST(X)

namespace sim_f64 {
typedef double real;
#include "sim_math.h"
#include "sim_dynamics.h"
#include "sim_task.h"
#include "sim_kernels.h"
#include "sim_gemm.h"
}  // namespace sim_f64
