// Line passes along y in float.
#define LB_T float
#define LB_DIR 1
#define LB_FN(name) name##_y_f32
#include "lb_lines.inc"
