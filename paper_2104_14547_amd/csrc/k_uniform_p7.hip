// Uniform-batch kernels, degree 7 in u.
#define ND_P 7
#include "k_uniform.inc"
