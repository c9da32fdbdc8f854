// Rollout kernel instantiations: (nv capacity, body slots, contacts in registers).
#define SIMK_FAMILY(X) X(24, 1, 8) X(24, 2, 8) X(24, 2, 2) X(24, 1, 2)
#include "../rollout_inst.inc"
