// The learning-episode update kernels (actor and critic Adam, TD-lambda, critic fit, target
// critic), in FP32 and FP64.  A translation unit of its own, with its own instance of the
// row-contraction GEMMs.
#include <hip/hip_runtime.h>
#include <math.h>
#include "sim_types.h"

namespace sim_l32 {
typedef float real;
#include "sim_math.h"
#include "sim_gemm.h"
#include "sim_learn.h"
}  // namespace sim_l32

namespace sim_l64 {
typedef double real;
#include "sim_math.h"
#include "sim_gemm.h"
#include "sim_learn.h"
}  // namespace sim_l64
