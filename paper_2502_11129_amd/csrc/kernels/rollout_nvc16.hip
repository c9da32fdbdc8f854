// Rollout kernel instantiations: (nv capacity, body slots, contacts in registers).
#define SIMK_FAMILY(X) X(16, 1, 16) X(16, 2, 16) X(16, 1, 2) X(16, 2, 8) X(16, 1, 8)
#include "../rollout_inst.inc"
