// Line passes along x in double.
#define LB_T double
#define LB_DIR 0
#define LB_FN(name) name##_x_f64
#include "lb_lines.inc"
