// Five-step solve of grids with a different number of points per axis, FP64
// arithmetic and storage (also used by split-precision plans on such grids);
// the kernels live in psn_general.h.
#include "psn_general.h"
#include "psn_general_launch.h"

PSN_DEFINE_GENERAL(double, double, f64)
