// Uniform-batch kernels, degree 4 in u.
#define ND_P 4
#include "k_uniform.inc"
