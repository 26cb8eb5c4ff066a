// Five-step solve of grids with a different number of points per axis, FP32
// arithmetic and storage; the kernels live in psn_general.h.
#include "psn_general.h"
#include "psn_general_launch.h"

PSN_DEFINE_GENERAL(float, float, f32)
