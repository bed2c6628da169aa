// Uniform-batch kernels, degree 5 in u.
#define ND_P 5
#include "k_uniform.inc"
