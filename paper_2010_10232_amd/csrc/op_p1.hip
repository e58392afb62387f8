// Level-operator kernels of degree 1 (see op_kernel.h).
#define HH_OP_DEGREE 1
#include "op_kernel.h"
