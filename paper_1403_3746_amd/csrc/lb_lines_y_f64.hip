// Line passes along y in double.
#define LB_T double
#define LB_DIR 1
#define LB_FN(name) name##_y_f64
#include "lb_lines.inc"
