// Evaluation kernels for form vectors of 1 word (32 forms per word).
#include "eval_kernels.h"

INSTANTIATE_EVAL_W(1)
