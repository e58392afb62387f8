// Level-operator kernels of degree 3 (see op_kernel.h).
#define HH_OP_DEGREE 3
#include "op_kernel.h"
