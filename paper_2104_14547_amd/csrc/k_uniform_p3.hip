// Uniform-batch kernels, degree 3 in u.
#define ND_P 3
#include "k_uniform.inc"
