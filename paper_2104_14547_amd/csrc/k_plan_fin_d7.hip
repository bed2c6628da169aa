// Persistent ragged-batch fin kernel, degrees <= 7.
#define ND_MAXD 7
#define ND_KIND 2
#include "k_plan.inc"
