// Rollout kernel instantiations with the tree-sparse factorisation of M~:
// (nv capacity, body slots, contacts in registers).
#define SIMK_TREE_FAMILY(X) X(24, 2, 8)
#include "../rollout_inst.inc"
