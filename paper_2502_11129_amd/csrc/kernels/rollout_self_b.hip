// Rollout kernel instantiations with self-collision: (nv capacity, body slots, contacts in registers).
#define SIMK_SELF_FAMILY(X) X(20, 1, 8) X(24, 1, 8)
#include "../rollout_inst.inc"
