// FP64 mixed-morphology group kernel, forward (every layout in one launch).
#define SIM_EMIT_GROUP_FWD 1
#include "sim_unit_f64.h"
