// Level-operator kernels of degree 4 (see op_kernel.h).
#define HH_OP_DEGREE 4
#include "op_kernel.h"
