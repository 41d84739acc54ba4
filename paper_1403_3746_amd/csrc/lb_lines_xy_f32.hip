// Fused x + y macroscopic line passes in float.
#define LB_T float
#define LB_FN(name) name##_f32
#include "lb_lines_xy.inc"
