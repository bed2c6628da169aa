// Persistent ragged-batch fwd kernel, degrees <= 7.
#define ND_MAXD 7
#define ND_KIND 0
#include "k_plan.inc"
