// The split fused kernel's FP64 instantiation for stencil radius 3 (sixth
// order, the default), built with the plane step as a lambda the plane loop
// calls (rk3_split.hip has the measurements behind that choice).
#define MHD_SPLIT_F64R3 1
#define MHD_SPLIT_BODY_LAMBDA 1
#include "rk3_split.hip"
