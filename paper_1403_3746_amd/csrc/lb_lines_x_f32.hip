// Line passes along x in float.
#define LB_T float
#define LB_DIR 0
#define LB_FN(name) name##_x_f32
#include "lb_lines.inc"
