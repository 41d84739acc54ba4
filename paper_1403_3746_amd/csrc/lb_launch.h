// Internal launch interface between the host runtime and the kernel units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "lb_types.h"

namespace lbfft {

// One launch covers `ninst` instances of the same grid size, listed (as indices into `insts`)
// in device array `ilist`.
struct LaunchSet {
    const InstDesc* insts;
    const int* ilist;
    int ninst;
    int nx, ny;
    hipStream_t stream;
    // when set, the launch timestamps its own start and end into these events
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    int ppb = 1;   // populations per block of the x population pass (tuned per size class)
    // launch-plan variants (YVariant) of the population y pass and of the macroscopic y (or fused
    // x + y) passes, tuned per size class; used where they exist, else the default plan
    int ypop_var = 0, ymac_var = 0;
    int xpop_var = 0;   // XVariant of the population x pass
};

// Launch through hipExtLaunchKernelGGL when the set carries timing events.
#define LB_LAUNCH(L, kernel, grid, block, ...)                                                  \
    do {                                                                                        \
        if ((L).ev_start)                                                                       \
            hipExtLaunchKernelGGL(kernel, grid, block, 0, (L).stream, (L).ev_start, (L).ev_stop, \
                                  0, __VA_ARGS__);                                              \
        else                                                                                    \
            hipLaunchKernelGGL(kernel, grid, block, 0, (L).stream, __VA_ARGS__);                \
    } while (0)

// Set the calling thread's error message (lb_last_error) and return `status`.
int set_error(int status, const char* msg);

// Line passes (lb_lines_<dir>_<prec>.hip).
hipError_t macro_x_f64(const LaunchSet& L, const JobDesc* jobs, int njobs);
hipError_t macro_y_f64(const LaunchSet& L, const JobDesc* jobs, int njobs);
hipError_t macro_x_f32(const LaunchSet& L, const JobDesc* jobs, int njobs);
hipError_t macro_y_f32(const LaunchSet& L, const JobDesc* jobs, int njobs);
// Population passes: dvm64 is the float64 velocity set the x pass forms the equilibrium with
// (unused by the y pass); pops/npops list the y populations (y pass), or npops is the populations
// per block of the x pass.
hipError_t pop_x_f64(const LaunchSet& L, const DvmConst<double>* dvm, const DvmConst<double>* dvm64,
                     const int* pops, int npops, StageArgs st);
hipError_t pop_y_f64(const LaunchSet& L, const DvmConst<double>* dvm, const DvmConst<double>* dvm64,
                     const int* pops, int npops, StageArgs st);
hipError_t pop_x_f32(const LaunchSet& L, const DvmConst<float>* dvm, const DvmConst<double>* dvm64,
                     const int* pops, int npops, StageArgs st);
hipError_t pop_y_f32(const LaunchSet& L, const DvmConst<float>* dvm, const DvmConst<double>* dvm64,
                     const int* pops, int npops, StageArgs st);

// Bit set (1 << YVariant) of the launch-plan variants the y passes have for y lines of n points
// (lb_lines_y_<prec>.hip): YV_WIDE for the population pass, YV_LONG for both.
int variants_y_f64(int n);
int variants_y_f32(int n);
// Bit mask of the XVariant plans of the population x pass that exist for x lines of n points
// (lb_lines_x_<prec>.hip): XV_R4.
int variants_x_f64(int n);
int variants_x_f32(int n);

// Fused x + y macroscopic passes of square grids (lb_lines_xy_<prec>.hip).
hipError_t macro_xy_f64(const LaunchSet& L, const JobDesc* jx, int njx, const JobDesc* jy, int njy);
hipError_t macro_xy_f32(const LaunchSet& L, const JobDesc* jx, int njx, const JobDesc* jy, int njy);

// Pointwise kernels (lb_pointwise.hip).
template <typename T>
hipError_t launch_moments(const LaunchSet& L, const DvmConst<double>* dvm, int f_field);
template <typename T>
hipError_t launch_stress(const LaunchSet& L);
template <typename T>
hipError_t launch_finalize(const LaunchSet& L);
template <typename T>
hipError_t launch_init(const LaunchSet& L, const DvmConst<double>* dvm);
template <typename T>
hipError_t launch_tables(const InstDesc* insts, int inst, int nx, int ny, hipStream_t s);
// Conservation sums of the instances of L (needs moments and d_x rho, d_y rho of the state).
template <typename T>
hipError_t launch_conserve(const LaunchSet& L, int record);
template <typename T>
hipError_t launch_to_f64(const void* src, double* dst, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_from_f64(const double* src, void* dst, int64_t n, hipStream_t s);

}  // namespace lbfft
