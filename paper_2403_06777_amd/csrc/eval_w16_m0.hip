// Evaluation kernels for form vectors of 16 words (32 forms per word), programs
// without variable monomials.
#include "eval_kernels.h"

INSTANTIATE_EVAL_WM(16, false)
