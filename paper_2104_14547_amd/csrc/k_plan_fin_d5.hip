// Persistent ragged-batch fin kernel, degrees <= 5.
#define ND_MAXD 5
#define ND_KIND 2
#include "k_plan.inc"
