// Rollout kernel instantiations: (nv capacity, body slots, contacts in registers).
#define SIMK_FAMILY(X) X(8, 1, 16) X(8, 1, 2)
#include "../rollout_inst.inc"
