// FP32 instantiation of the window kernels (the production path).
#include <hip/hip_runtime.h>
#include <math.h>
#include "sim_types.h"

// DOF counts compiled as kernels of their own (CartPole, Ant, Humanoid)
// DOF counts of muscle-driven models with a kernel of their own (the humanoid skeleton)
#define SIM_NV_LIST_MTU(X) X(27)
#define SIM_NV_LIST(X) X(2) X(14) X(27)

namespace sim_f32 {
typedef float real;
#include "sim_math.h"
#include "sim_dynamics.h"
#include "sim_task.h"
#include "sim_kernels.h"
#include "sim_gemm.h"
}  // namespace sim_f32
