// Rollout kernel instantiations with self-collision: (nv capacity, body slots, contacts in registers).
#define SIMK_SELF_FAMILY(X) X(12, 1, 8) X(12, 1, 2) X(16, 1, 8)
#include "../rollout_inst.inc"
