// Uniform-batch kernels, degree 1 in u.
#define ND_P 1
#include "k_uniform.inc"
