// FP32 mixed-morphology group kernel, adjoint (every layout in one launch).
#define SIM_EMIT_GROUP_ADJ 1
#include "sim_unit_f32.h"
