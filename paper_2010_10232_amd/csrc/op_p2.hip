// Level-operator kernels of degree 2 (see op_kernel.h).
#define HH_OP_DEGREE 2
#include "op_kernel.h"
