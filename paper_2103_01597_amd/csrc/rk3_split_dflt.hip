// The split fused kernel's FP64 instantiation for stencil radius 4, built
// with the default instruction scheduler (rk3_split.hip itself is built with
// the iterative ILP scheduler, which measured slower for it).
#define MHD_DEFAULT_SCHED 1
#include "rk3_split.hip"
