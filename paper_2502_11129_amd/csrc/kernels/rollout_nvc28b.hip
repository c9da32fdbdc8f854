// Rollout kernel instantiations: (nv capacity, body slots, contacts in registers).
#define SIMK_FAMILY(X) X(28, 2, 4) X(28, 2, 12)
#include "../rollout_inst.inc"
