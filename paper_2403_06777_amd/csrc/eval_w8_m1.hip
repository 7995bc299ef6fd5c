// Evaluation kernels for form vectors of 8 words (32 forms per word), programs
// with variable monomials.
#include "eval_kernels.h"

INSTANTIATE_EVAL_WM(8, true)
