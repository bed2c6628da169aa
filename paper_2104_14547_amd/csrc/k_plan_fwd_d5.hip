// Persistent ragged-batch fwd kernel, degrees <= 5.
#define ND_MAXD 5
#define ND_KIND 0
#include "k_plan.inc"
