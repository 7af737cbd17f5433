// Patch-solve kernels instantiated for double (one translation unit per precision so the
// two compile in parallel).
#include "patch_kernels.h"

VSR_INSTANTIATE_PATCH(double)
