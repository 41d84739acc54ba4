// Windowed-FFT derivative (Eq. 3) of a caller's device field without any device allocation: the
// descriptor, the job, the float64-generated tables and the two staging fields the line pass
// works on live in one static device array (`scratch`), which each GPU the library runs on
// holds until the process ends.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "lbfft.h"
#include "lb_launch.h"
#include "lb_types.h"

using namespace lbfft;

namespace {

// Layout of the array: descriptor, job, instance list, tables (kx, ky, twx, twy: at most
// 6 * 2048 words), then the input and output fields of LB_NOALLOC_MAX_CELLS words each.
constexpr size_t OFF_DESC = 0;
constexpr size_t OFF_JOB = 256;
constexpr size_t OFF_ILIST = 512;
constexpr size_t OFF_TABLES = 1024;
constexpr size_t TABLE_BYTES = 6 * 2048 * 8 + 4 * 256;
constexpr size_t OFF_ARENA = (OFF_TABLES + TABLE_BYTES + 255) / 256 * 256;
constexpr size_t SCRATCH_BYTES = OFF_ARENA + 2 * (size_t)LB_NOALLOC_MAX_CELLS * 8;

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

// The descriptor and job arrive as kernel arguments (copied at launch), so no host buffer has to
// outlive the call.
__global__ void __launch_bounds__(64) put_descriptor(InstDesc d, JobDesc j, unsigned char* base) {
    if (threadIdx.x == 0) {
        *reinterpret_cast<InstDesc*>(base + OFF_DESC) = d;
        *reinterpret_cast<JobDesc*>(base + OFF_JOB) = j;
        *reinterpret_cast<int*>(base + OFF_ILIST) = 0;
    }
}

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_scratch[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up once per device.
hipError_t scratch_of_current_device(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

lb_status err(lb_status s, const char* fmt, long long a = 0, long long b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), fmt, a, b);
    return static_cast<lb_status>(set_error(s, buf));
}

lb_status hip_err(hipError_t e, const char* what) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s failed: %s", what, hipGetErrorString(e));
    return static_cast<lb_status>(set_error(LB_E_HIP, buf));
}

}  // namespace

extern "C" lb_status lb_derivative_noalloc(int nx, int ny, double dx, lb_precision prec, int axis,
                                           int order, const double* d_g, double* d_out,
                                           void* hip_stream) {
    set_error(LB_OK, "");
    if (!d_g || !d_out) return err(LB_E_ARG, "null field pointer");
    if (!(dx > 0)) return err(LB_E_ARG, "dx must be positive");
    if ((axis != 0 && axis != 1) || (order != 1 && order != 2))
        return err(LB_E_ARG, "axis must be 0/1 and order 1/2");
    if (prec != LB_FP64 && prec != LB_FP32) return err(LB_E_ARG, "bad precision");
    if (!grid_ok(nx, ny))
        return err(LB_E_SIZE, "unsupported grid %lldx%lld (each side 2^a or 3*2^a in [8,2048]; ny "
                   "may also be 1 or 2)", nx, ny);
    const int64_t nc = (int64_t)nx * ny;
    if (nc > LB_NOALLOC_MAX_CELLS)
        return err(LB_E_SIZE, "grid of %lld cells exceeds the static scratch limit of %lld cells",
                   nc, (long long)LB_NOALLOC_MAX_CELLS);
    unsigned char* base = nullptr;
    hipError_t e = scratch_of_current_device(&base);
    if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t w = prec == LB_FP64 ? 8 : 4;

    InstDesc I{};
    I.nx = nx;
    I.ny = ny;
    I.ncell = nc;
    I.dx = dx;
    size_t t = OFF_TABLES;
    I.kx = base + t;  t = up256(t + w * nx);
    I.ky = base + t;  t = up256(t + w * ny);
    I.twx = base + t; t = up256(t + 2 * w * nx);
    I.twy = base + t;
    I.base = base + OFF_ARENA;   // field 0: the input, field 1: the derivative
    JobDesc J{};
    J.in = 0;
    J.out[0] = 1;
    J.out[1] = -1;
    J.mult[0] = order == 1 ? M_D : M_DD;
    J.mult[1] = M_NONE;
    const InstDesc* d_desc = reinterpret_cast<const InstDesc*>(base + OFF_DESC);
    const JobDesc* d_job = reinterpret_cast<const JobDesc*>(base + OFF_JOB);
    const int* d_ilist = reinterpret_cast<const int*>(base + OFF_ILIST);
    unsigned char* in = base + OFF_ARENA;
    unsigned char* outf = in + (size_t)nc * w;

    hipLaunchKernelGGL(put_descriptor, dim3(1), dim3(64), 0, s, I, J, base);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "descriptor launch");
    e = prec == LB_FP64 ? launch_tables<double>(d_desc, 0, nx, ny, s) : launch_tables<float>(d_desc, 0, nx, ny, s);
    if (e != hipSuccess) return hip_err(e, "table kernel");
    if (prec == LB_FP64)
        e = hipMemcpyAsync(in, d_g, (size_t)nc * 8, hipMemcpyDeviceToDevice, s);
    else
        e = launch_from_f64<float>(d_g, in, nc, s);
    if (e != hipSuccess) return hip_err(e, "input staging");
    LaunchSet L{d_desc, d_ilist, 1, nx, ny, s};
    if (prec == LB_FP64)
        e = axis == 0 ? macro_x_f64(L, d_job, 1) : macro_y_f64(L, d_job, 1);
    else
        e = axis == 0 ? macro_x_f32(L, d_job, 1) : macro_y_f32(L, d_job, 1);
    if (e != hipSuccess) return hip_err(e, "line pass");
    if (prec == LB_FP64)
        e = hipMemcpyAsync(d_out, outf, (size_t)nc * 8, hipMemcpyDeviceToDevice, s);
    else
        e = launch_to_f64<float>(outf, d_out, nc, s);
    if (e != hipSuccess) return hip_err(e, "output staging");
    return LB_OK;
}
