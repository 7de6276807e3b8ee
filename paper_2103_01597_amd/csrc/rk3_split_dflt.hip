// The split fused kernel's FP64 instantiation for stencil radius 4, built
// with the default instruction scheduler (rk3_split.hip itself is built with
// the iterative ILP scheduler, which measured slower for it).
// Its physics constants are read with vector loads (MHD_SPLIT_PHYS_SMEM 0),
// which measured faster for it than scalar loads.
#define MHD_DEFAULT_SCHED 1
#define MHD_SPLIT_PHYS_SMEM 0
#include "rk3_split.hip"
