// Uniform-batch kernels, degree 2 in u.
#define ND_P 2
#include "k_uniform.inc"
