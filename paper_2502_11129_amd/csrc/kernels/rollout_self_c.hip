// Rollout kernel instantiations with self-collision: (nv capacity, body slots, contacts in registers).
#define SIMK_SELF_FAMILY(X) X(24, 2, 8) X(28, 2, 8)
#include "../rollout_inst.inc"
