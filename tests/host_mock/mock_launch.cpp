// No-op stand-ins for the kernel launch functions, with argument checks (CPU check of the host
// runtime).
#include "lb_launch.h"
#include <cassert>
namespace lbfft {
static void chk(const LaunchSet& L) { assert(L.insts && L.ilist && L.ninst > 0 && L.nx > 0 && L.ny > 0); }
#define M(name, T) hipError_t name(const LaunchSet& L, const JobDesc* j, int n) { chk(L); assert(j && n > 0); return hipSuccess; }
M(macro_x_f64, double) M(macro_y_f64, double) M(macro_x_f32, float) M(macro_y_f32, float)
#define MXY(name) hipError_t name(const LaunchSet& L, const JobDesc* a, int na, const JobDesc* b, int nb) { chk(L); assert(L.nx == L.ny && a && b && na > 0 && nb > 0); return hipSuccess; }
MXY(macro_xy_f64) MXY(macro_xy_f32)
#define P(name, T) hipError_t name(const LaunchSet& L, const DvmConst<T>* d, const DvmConst<double>* d64, const int* p, int n, StageArgs) { chk(L); assert(d && d64 && p && n > 0); return hipSuccess; }
P(pop_x_f64, double) P(pop_y_f64, double) P(pop_x_f32, float) P(pop_y_f32, float)
int variants_y_f64(int) { return 0; }
int variants_y_f32(int n) { return n >= 1024 ? (1 << YV_WIDE) | (1 << YV_LONG) : 0; }
int variants_x_f64(int) { return 0; }
int variants_x_f32(int n) { return (n == 128 || n == 256 || n == 512) ? 1 << XV_R4 : 0; }
template <typename T> hipError_t launch_moments(const LaunchSet& L, const DvmConst<double>*, int) { chk(L); return hipSuccess; }
template <typename T> hipError_t launch_stress(const LaunchSet& L) { chk(L); return hipSuccess; }
template <typename T> hipError_t launch_finalize(const LaunchSet& L) { chk(L); return hipSuccess; }
template <typename T> hipError_t launch_init(const LaunchSet& L, const DvmConst<double>*) { chk(L); return hipSuccess; }
template <typename T> hipError_t launch_tables(const InstDesc*, int, int, int, hipStream_t) { return hipSuccess; }
template <typename T> hipError_t launch_conserve(const LaunchSet& L, int) { chk(L); return hipSuccess; }
template <typename T> hipError_t launch_to_f64(const void*, double*, int64_t, hipStream_t) { return hipSuccess; }
template <typename T> hipError_t launch_from_f64(const double*, void*, int64_t, hipStream_t) { return hipSuccess; }
#define I(T) template hipError_t launch_moments<T>(const LaunchSet&, const DvmConst<double>*, int); \
 template hipError_t launch_stress<T>(const LaunchSet&); template hipError_t launch_finalize<T>(const LaunchSet&); \
 template hipError_t launch_init<T>(const LaunchSet&, const DvmConst<double>*); \
 template hipError_t launch_tables<T>(const InstDesc*, int, int, int, hipStream_t); \
 template hipError_t launch_conserve<T>(const LaunchSet&, int); \
 template hipError_t launch_to_f64<T>(const void*, double*, int64_t, hipStream_t); \
 template hipError_t launch_from_f64<T>(const double*, void*, int64_t, hipStream_t);
I(double) I(float)
}
