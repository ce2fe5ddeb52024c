// FP64 window kernels: full and muscle layouts, plain per-substep path, MLP weight preparation,
// window loss and the policy-parameter gradient.
#define SIM_EMIT_MAIN 1
#include "sim_unit_f64.h"
