// Persistent ragged-batch bwd kernel, degrees <= 7.
#define ND_MAXD 7
#define ND_KIND 1
#include "k_plan.inc"
