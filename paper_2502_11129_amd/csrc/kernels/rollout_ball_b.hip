// Rollout kernel instantiations for variants with a ball: (nv capacity, body slots, contacts in registers).
#define SIMK_BALL_FAMILY(X) X(20, 1, 8) X(24, 1, 8)
#include "../rollout_inst.inc"
