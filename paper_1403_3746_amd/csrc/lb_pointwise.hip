// Pointwise kernels (moments, stress, initial equilibrium, float64 tables, conservation
// partial sums, precision conversion) and their launches, for both precisions.
#include "lb_kernels.h"
#include "lb_launch.h"

namespace lbfft {

namespace {

inline dim3 cell_grid(int64_t ncell, int ninst) {
    return dim3((unsigned)((ncell + 255) / 256), (unsigned)ninst);
}

// Wavenumber k(m) of Eq. (3) and forward twiddles exp(-2 pi i m/N), generated in float64 and
// rounded to the working precision.  k(m) = (2/dx) S(sin(pi m'/N)), S the arcsin series
// truncated after phi^15, m' the signed index; the Nyquist mode of an even N gets 0.
template <typename T>
__global__ void __launch_bounds__(256)
tables_kernel(const InstDesc* __restrict__ insts, int inst) {
    const InstDesc& I = insts[inst];
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const double coef[8] = {1.0, 1.0 / 6.0, 3.0 / 40.0, 5.0 / 112.0, 35.0 / 1152.0,
                            63.0 / 2816.0, 231.0 / 13312.0, 143.0 / 10240.0};
#pragma unroll
    for (int axis = 0; axis < 2; ++axis) {
        const int n = axis == 0 ? I.nx : I.ny;
        if (m >= n) continue;
        const int ms = (2 * m < n) ? m : m - n;
        double k = 0.0;
        if (!(n % 2 == 0 && 2 * m == n)) {
            const double phi = sinpi((double)ms / (double)n);
            const double p2 = phi * phi;
            double s = coef[7];
            for (int j = 6; j >= 0; --j) s = s * p2 + coef[j];
            k = (2.0 / I.dx) * phi * s;
        }
        double sn, cs;
        sincospi(2.0 * (double)m / (double)n, &sn, &cs);
        T* kap = reinterpret_cast<T*>(const_cast<void*>(axis == 0 ? I.kx : I.ky));
        cpx<T>* tw = reinterpret_cast<cpx<T>*>(const_cast<void*>(axis == 0 ? I.twx : I.twy));
        kap[m] = T(k);
        tw[m] = {T(cs), T(-sn)};
    }
}

// Final sum of the block partials in a fixed order (one block per instance): each thread adds
// RED_BLOCKS / 256 partials of each quantity, then a pairwise tree in LDS -- the same order in every
// call, so the sums are reproducible.  cons = sums times dx^2 (the non-finite count unscaled); with
// record != 0 the four integrals are also appended to the history ring buffer.
constexpr int FINAL_THREADS = 256;
static_assert(RED_BLOCKS % FINAL_THREADS == 0, "partials per thread");

__global__ void __launch_bounds__(FINAL_THREADS)
conserve_final(const InstDesc* __restrict__ insts, const int* __restrict__ ilist, int record) {
    const InstDesc& I = insts[ilist[blockIdx.x]];
    const int t = threadIdx.x;
    __shared__ double sh[5][FINAL_THREADS];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = t; b < I.red_blocks; b += FINAL_THREADS) {
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += I.red[b * 5 + k];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k][t] = acc[k];
    __syncthreads();
    for (int s = FINAL_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sh[k][t] += sh[k][t + s];
        }
        __syncthreads();
    }
    const double area = I.dx * I.dx;
    if (t < 5) I.cons[t] = t < 4 ? sh[t][0] * area : sh[t][0];
    if (record && I.hist_len > 0) {
        const unsigned long long n = *I.hist_count;
        __syncthreads();   // every thread has read the count before thread 0 advances it
        if (t < 4) I.hist[(n % (unsigned long long)I.hist_len) * 4 + t] = sh[t][0] * area;
        if (t == 0) *I.hist_count = n + 1;
    }
}

}  // namespace

template <typename T>
hipError_t launch_moments(const LaunchSet& L, const DvmConst<double>* dvm, int f_field) {
    const int64_t nc = (int64_t)L.nx * L.ny;
    LB_LAUNCH(L, (moments_kernel<T>), cell_grid(nc, L.ninst), dim3(256), L.insts, L.ilist, dvm,
              f_field);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stress(const LaunchSet& L) {
    const int64_t nc = (int64_t)L.nx * L.ny;
    LB_LAUNCH(L, (stress_kernel<T>), cell_grid(nc, L.ninst), dim3(256), L.insts, L.ilist);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const LaunchSet& L) {
    const int64_t nc = (int64_t)L.nx * L.ny;
    LB_LAUNCH(L, (finalize_kernel<T>), cell_grid(nc, L.ninst), dim3(256), L.insts, L.ilist);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const LaunchSet& L, const DvmConst<double>* dvm) {
    const int64_t nc = (int64_t)L.nx * L.ny;
    hipLaunchKernelGGL((init_kernel<T>), cell_grid(nc, L.ninst), dim3(256), 0, L.stream,
                       L.insts, L.ilist, dvm);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tables(const InstDesc* insts, int inst, int nx, int ny, hipStream_t s) {
    const int n = nx > ny ? nx : ny;
    hipLaunchKernelGGL((tables_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, s, insts, inst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_conserve(const LaunchSet& L, int record) {
    hipLaunchKernelGGL((conserve_partial<T>), dim3(RED_BLOCKS, L.ninst), dim3(256), 0, L.stream,
                       L.insts, L.ilist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(conserve_final, dim3(L.ninst), dim3(FINAL_THREADS), 0, L.stream, L.insts, L.ilist, record);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_to_f64(const void* src, double* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((to_f64<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const T*>(src), dst, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_from_f64(const double* src, void* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((from_f64<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                       reinterpret_cast<T*>(dst), n);
    return hipGetLastError();
}

#define LB_INST(T)                                                                         \
    template hipError_t launch_moments<T>(const LaunchSet&, const DvmConst<double>*, int); \
    template hipError_t launch_stress<T>(const LaunchSet&);                                \
    template hipError_t launch_finalize<T>(const LaunchSet&);                              \
    template hipError_t launch_init<T>(const LaunchSet&, const DvmConst<double>*);         \
    template hipError_t launch_tables<T>(const InstDesc*, int, int, int, hipStream_t);     \
    template hipError_t launch_conserve<T>(const LaunchSet&, int);                         \
    template hipError_t launch_to_f64<T>(const void*, double*, int64_t, hipStream_t);      \
    template hipError_t launch_from_f64<T>(const double*, void*, int64_t, hipStream_t);
LB_INST(double)
LB_INST(float)
#undef LB_INST

}  // namespace lbfft
