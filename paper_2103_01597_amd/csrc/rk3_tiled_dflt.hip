// The tiled fused kernel's instantiations for stencil radii 1 and 4, built
// with the default instruction scheduler (rk3_tiled.hip itself is built with
// the iterative ILP scheduler, which measured slower for these radii).
#define MHD_DEFAULT_SCHED 1
#include "rk3_tiled.hip"
