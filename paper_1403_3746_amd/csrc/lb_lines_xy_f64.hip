// Fused x + y macroscopic line passes in double.
#define LB_T double
#define LB_FN(name) name##_f64
#include "lb_lines_xy.inc"
