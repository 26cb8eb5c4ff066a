// Pass kernels and launchers instantiated for one precision (split); the
// templates live in psn_passes.h.
#include "psn_passes.h"

PSN_DEFINE_PRECISION(psn::DT_SPLIT, split)
