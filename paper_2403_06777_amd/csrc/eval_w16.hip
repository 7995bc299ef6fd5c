// Evaluation kernels for form vectors of 16 words (32 forms per word).
#include "eval_kernels.h"

INSTANTIATE_EVAL_W(16)
