// Uniform-batch kernels, degree 6 in u.
#define ND_P 6
#include "k_uniform.inc"
