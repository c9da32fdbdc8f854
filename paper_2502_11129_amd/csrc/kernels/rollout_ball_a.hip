// Rollout kernel instantiations for variants with a ball: (nv capacity, body slots, contacts in registers).
#define SIMK_BALL_FAMILY(X) X(12, 1, 8) X(12, 1, 2) X(16, 1, 8)
#include "../rollout_inst.inc"
