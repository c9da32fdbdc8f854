// Rollout kernel instantiations: (nv capacity, body slots, contacts in registers).
#define SIMK_FAMILY(X) X(12, 1, 16) X(12, 1, 2)
#include "../rollout_inst.inc"
