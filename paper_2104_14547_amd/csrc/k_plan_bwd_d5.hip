// Persistent ragged-batch bwd kernel, degrees <= 5.
#define ND_MAXD 5
#define ND_KIND 1
#include "k_plan.inc"
