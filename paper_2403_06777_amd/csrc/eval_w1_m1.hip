// Evaluation kernels for form vectors of 1 word (32 forms per word), programs
// with variable monomials.
#include "eval_kernels.h"

INSTANTIATE_EVAL_WM(1, true)
