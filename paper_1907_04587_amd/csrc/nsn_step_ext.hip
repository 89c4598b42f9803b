// The extended instantiation of the Newton kernel (linear tets, islands): the same
// source as nsn_step.hip, built with a larger basic-block budget for the inliner so
// that every function taking the per-env context is inlined (see the launchers there).
#define NSN_STEP_EXT_TU 1
#include "nsn_step.hip"
