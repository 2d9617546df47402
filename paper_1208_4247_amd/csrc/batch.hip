// batch.hip -- placeholder until the batched kernels land.
#include "gmg_internal.h"
