// FP32 window kernels of the compact layout (small models, 16 / 32 / 64 lanes per environment).
#define SIM_EMIT_COMPACT 1
#include "sim_unit_f32.h"
