// Rollout kernel instantiations: (nv capacity, body slots, contacts in registers).
#define SIMK_FAMILY(X) X(20, 1, 8) X(20, 2, 8) X(20, 1, 2) X(20, 1, 4)
#include "../rollout_inst.inc"
