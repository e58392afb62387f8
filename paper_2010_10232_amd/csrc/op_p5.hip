// Level-operator kernels of degree 5 (see op_kernel.h).
#define HH_OP_DEGREE 5
#include "op_kernel.h"
