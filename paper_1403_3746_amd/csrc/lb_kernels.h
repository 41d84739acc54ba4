// Kernel templates of the lbfft library (gfx950).  Instantiated per precision and line length
// in lb_lines_*.hip and lb_pointwise.hip.
//
// One Runge-Kutta stage R(f) (Eq. 1, Sec. 2.3) runs as:
//   moments      pointwise   f -> rho, u, T                              (Sec. 2.1)
//   macro X1|Y1  x, y lines  first and second derivatives of rho, T, u   (Eq. 3) (independent:
//                            one fused launch on square grids)
//   stress       pointwise   S, div u, q rho T grad T, most of C         (Eq. 2, Sec. 2.2)
//   macro X2|Y2  x, y lines  derivatives of S, div u, Q                  (Eq. 3) (likewise)
//   finalize     pointwise   B = div S/(rho T), C + C_q                  (Eq. 2)
//   pop X        x lines     per population: v_x d_x f, f^eq, I_i, BGK, RK axpy -> final (axis-x
//                            populations) or partial (the rest)
//   pop Y        y lines     per population: add -c v_y d_y f to the partial -> final
// Line passes pack two real lines (rows 2l, 2l+1 or columns 2l, 2l+1) into one complex line,
// which is exact because every spectral multiplier used is Hermitian (m(-k) = conj m(k)).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lb_decode.h"
#include "lb_fft.h"
#include "lb_types.h"

#ifndef LB_YSEG
#define LB_YSEG 128      // bytes of each row a y-pass tile covers (2 * lines per block * word)
#endif
#ifndef LB_YMAX_THREADS
#define LB_YMAX_THREADS 512  // threads per y-pass block at most
#endif
#ifndef LB_YMAX_THREADS_WIDE
#define LB_YMAX_THREADS_WIDE 1024  // the same for the wide y-tile variant the tuner may pick
#endif
#define LB_LDS_BYTES 163840      // LDS of one CU
#ifndef LB_POPX_WAVES
#define LB_POPX_WAVES 3  // waves per SIMD the single-population FP32 x pass must fit (register budget)
#endif
#ifndef LB_POPX_BATCH_LDS
#define LB_POPX_BATCH_LDS 40960  // LDS bytes up to which the x pass transforms its P lines together
#endif
#ifndef LB_POPX_FOLD_BASE
#define LB_POPX_FOLD_BASE 1  // first stage: fold the base f^n into the x pass's multiplier
#endif
#ifndef LB_POPX_WAVES_F64
#define LB_POPX_WAVES_F64 3  // the same for FP64 (fewer: its epilogue holds twice the registers)
#endif
#ifndef LB_FP32_EQ64
#define LB_FP32_EQ64 1   // FP32 state: form the equilibrium in float64 arithmetic (see EqType)
#endif

namespace lbfft {

// ---------------------------------------------------------------------------------------
// Launch geometry of the line passes.  Small tiles keep many blocks in flight for a single grid;
// y tiles span LPW column pairs (2*LPW*sizeof(T) bytes of each row), and neighbouring tiles of one
// field run together on the same XCD (decode_block_jm) so partially used cache lines are reused
// from L2.
// LDS: x blocks (lanes of one line adjacent) store each line contiguously; y blocks (lanes of
// neighbouring lines adjacent) interleave their lines word by word (LS = LPW).
template <typename T, int N, int DIR, int LPW_OVERRIDE = 0, int MAXT = LB_YMAX_THREADS, int RR = 0>
struct LineCfg {
    static constexpr int R = RR ? RR : default_R(N);   // elements per thread
    static constexpr int TPL = N / R;
    static constexpr int CB = 2 * (int)sizeof(T);  // bytes of one complex word
    static constexpr int at_least(int l, int lo) { return l < lo ? lo : l; }
    // x: one line per block unless lines are short (then fill one wave)
    static constexpr int lpw_x() { return at_least(64 / TPL, 1); }
    // y: LB_YSEG-byte row segments, at least one wave per block, at most MAXT threads and the
    // LDS of one CU (long lines get fewer column pairs)
    static constexpr int lpw_y() {
        int l = at_least(at_least(LB_YSEG / CB, 64 / TPL), 1);
        while (l > 1 && (l * TPL > MAXT || l * lds_line(N) * CB > LB_LDS_BYTES)) l /= 2;
        return l;
    }
    static constexpr int LPW = LPW_OVERRIDE > 0 ? LPW_OVERRIDE : (DIR == 0 ? lpw_x() : lpw_y());
    static constexpr int WG = LPW * TPL;
    static constexpr int LS = DIR == 0 ? 1 : LPW;
    static constexpr int LDS = LPW * lds_line(N);   // complex words
    // LDS base of line l of the block
    __device__ __forceinline__ static int lds_base(int l) { return DIR == 0 ? l * lds_line(N) : l; }
};

// Launch-plan variants of the y passes that the tuner may pick per size class (FP32 only: a
// 1024-thread block leaves 128 registers per thread, which the FP64 passes exceed):
//   wide: the population y pass in blocks of up to LB_YMAX_THREADS_WIDE threads, where that holds
//         more column pairs than the default (the macroscopic passes would spill);
//   long radix: lines of 1024 and 2048 points held 16 elements per thread (radix-16 passes), and
//         lines of 3 * 2^a points from 96 to 384 held 24 (a radix-24 pass, then radix 8): fewer
//         threads per line, so a block of up to 512 threads holds more column pairs, and fewer
//         passes through LDS.
template <typename T, int N>
constexpr bool pop_y_wide_exists() {
    // lines of 3 * 2^a points hold 12 elements per thread and would spill at 1024 threads
    return sizeof(T) == 4 && default_R(N) == 8 &&
           LineCfg<T, N, 1, 0, LB_YMAX_THREADS_WIDE>::LPW != LineCfg<T, N, 1, 0, LB_YMAX_THREADS>::LPW;
}
template <typename T, int N>
constexpr bool long_exists() {
    return sizeof(T) == 4 && (N == 1024 || N == 2048 || (N % 3 == 0 && N >= 96 && N <= 384));
}
// elements per thread of that plan
constexpr int long_R(int N) { return N % 3 == 0 ? 24 : 16; }
// and of the population x pass: FP32 lines of 128 to 512 points held 4 elements per thread (twice
// the threads per line: full 128-byte row segments per load instruction and half the registers
// per line, for more passes through LDS)
template <typename T, int N>
constexpr bool popx_r4_exists() { return sizeof(T) == 4 && (N == 128 || N == 256 || N == 512); }

__device__ __forceinline__ BlockWork decode_block(int ngroups, int ntiles, int njobs) {
    return decode_block_at(blockIdx.x, ngroups, ntiles, njobs);
}

#ifndef LB_WAVE_SYNC_X
#define LB_WAVE_SYNC_X 1  // x macroscopic blocks of one-wave lines: per-wave LDS ordering
#endif
#ifndef LB_JOBMAJOR_X
#define LB_JOBMAJOR_X 1   // x macroscopic passes: job-major block order
#endif
#ifndef LB_JOBMAJOR_Y
#define LB_JOBMAJOR_Y 1   // y macroscopic and population passes: job-major block order
#endif

// Spectral multiplier kind MK applied to coefficient x of wavenumber k, including the 1/N of the
// inverse transform:  M_D -> i (k/N) x,  M_DD -> -(k^2/N) x,  M_NONE -> 0.  The kind is a template
// argument so that a line's R coefficients are scaled without a branch per element.
template <int MK, typename T>
__device__ __forceinline__ cpx<T> spectral_mult(T k, T invN, cpx<T> x) {
    if constexpr (MK == M_D) {
        const T a = k * invN;
        return {-a * x.im, a * x.re};
    } else if constexpr (MK == M_DD) {
        const T a = -k * k * invN;
        return {a * x.re, a * x.im};
    } else {
        return {T(0), T(0)};
    }
}

template <typename T>
struct vec2 {
    T a, b;
};

// Field `id` of an instance as a global-memory pointer (cells indexed by 32-bit offsets).
template <typename T>
__device__ __forceinline__ LB_GLOBAL T* fieldp(const InstDesc& I, int id) {
    return gcast(reinterpret_cast<T*>(I.base) + (int64_t)id * I.ncell);
}

// The instance's field arena through one buffer resource (an SGPR descriptor).  A field is a
// uniform 32-bit byte offset (soffset) and a cell a per-lane 32-bit byte offset (voffset), so an
// access needs no 64-bit address arithmetic and a field costs one SGPR instead of four.  The
// runtime keeps the arena (NFIELDS * ncell * sizeof(T) bytes) below 2^32 bytes.
struct Arena {
    __amdgpu_buffer_rsrc_t r;
};

template <typename T>
__device__ __forceinline__ Arena arena(const InstDesc& I) {
    const uint32_t bytes = (uint32_t)NFIELDS * (uint32_t)I.ncell * (uint32_t)sizeof(T);
    return Arena{__builtin_amdgcn_make_buffer_rsrc(I.base, 0, (int)bytes, 0x00020000)};
}
template <typename T>
__device__ __forceinline__ uint32_t fofs(const InstDesc& I, int id) {
    return (uint32_t)id * (uint32_t)I.ncell * (uint32_t)sizeof(T);
}

__device__ __forceinline__ double bload(Arena a, uint32_t fo, uint32_t e, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(a.r, e * 8u, fo, 0));
}
__device__ __forceinline__ float bload(Arena a, uint32_t fo, uint32_t e, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(a.r, e * 4u, fo, 0));
}
__device__ __forceinline__ void bstore(Arena a, uint32_t fo, uint32_t e, double v) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(a.r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), a.r, e * 8u, fo, 0);
}
__device__ __forceinline__ void bstore(Arena a, uint32_t fo, uint32_t e, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), a.r, e * 4u, fo, 0);
}

// Addressing of the two real lines packed into complex line `line` at position p.
template <int DIR>
struct LineAddr {
    // cell index of the real part (re) and imaginary part (im) of position p
    __device__ __forceinline__ static uint32_t re(int line, int p, int nx) {
        return DIR == 0 ? (uint32_t)(2 * line) * nx + p : (uint32_t)p * nx + 2 * line;
    }
    __device__ __forceinline__ static uint32_t im(int line, int p, int nx) {
        return DIR == 0 ? (uint32_t)(2 * line + 1) * nx + p : (uint32_t)p * nx + 2 * line + 1;
    }
};

template <typename T, int DIR, int R, int TPL>
__device__ __forceinline__ void load_line(const LB_GLOBAL T* g, cpx<T> (&v)[R], int line, int t,
                                          int nx, int ny, bool active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int p = t + m * TPL;
        cpx<T> z = {T(0), T(0)};
        if (active) {
            if constexpr (DIR == 0) {
                z.re = g[LineAddr<0>::re(line, p, nx)];
                if (2 * line + 1 < ny) z.im = g[LineAddr<0>::im(line, p, nx)];
            } else {
                const LB_GLOBAL vec2<T>* w = reinterpret_cast<const LB_GLOBAL vec2<T>*>(g + LineAddr<1>::re(line, p, nx));
                z.re = w->a;
                z.im = w->b;
            }
        }
        v[m] = z;
    }
}

// The wavenumbers k[t + m*TPL] of a thread's R line elements: requested up front and kept in
// registers for R <= 8; lines of 3 * 2^a points (R = 12) read them where they are used.
#ifndef LB_WAVENUM_PRE
#define LB_WAVENUM_PRE 8
#endif
template <typename T, int R, int TPL>
struct Wavenum {
    static constexpr bool PRE = R <= LB_WAVENUM_PRE;
    T k[PRE ? R : 1];
    const LB_GLOBAL T* kap;
    int t;
    __device__ __forceinline__ void load(const LB_GLOBAL T* table, int thread) {
        kap = table;
        t = thread;
        if constexpr (PRE) {
#pragma unroll
            for (int m = 0; m < R; ++m) k[m] = kap[t + m * TPL];
        }
    }
    __device__ __forceinline__ T operator[](int m) const {
        if constexpr (PRE) return k[m];
        else return kap[t + m * TPL];
    }
};

// ---------------------------------------------------------------------------------------
// Macroscopic line pass driven by a job table: the work of block b (LPW lines per block, Q jobs
// of the job table per block).  With Q > 1 the lines of all Q jobs are requested before the first
// transform, so the later jobs' loads (and the earlier jobs' stores) overlap the transforms.
#ifndef LB_MACRO_JOBS_F64
#define LB_MACRO_JOBS_F64 1   // jobs per block of the FP64 macroscopic line passes
#endif
#ifndef LB_MACRO_JOBS_F32
#define LB_MACRO_JOBS_F32 1   // the same in FP32
#endif
template <typename T>
__host__ __device__ constexpr int macro_jobs() { return sizeof(T) == 8 ? LB_MACRO_JOBS_F64 : LB_MACRO_JOBS_F32; }
__host__ __device__ constexpr int job_slots(int njobs, int Q) { return (njobs + Q - 1) / Q; }

template <typename T, int N, int DIR, int LPW_, int RR = 0, int Q = macro_jobs<T>()>
__device__ __forceinline__ void macro_body(int b, const InstDesc* __restrict__ insts,
                                           const int* __restrict__ ilist, int ngroups, int ntiles,
                                           const JobDesc* __restrict__ jobs, int njobs,
                                           cpx<T>* lds_all) {
    using C = LineCfg<T, N, DIR, LPW_, LB_YMAX_THREADS, RR>;
    // x blocks whose lines fit in a wave synchronise per wave (line_sync)
    constexpr bool WAVE = DIR == 0 && C::TPL <= 64 && LB_WAVE_SYNC_X;
    using FFT = LineFFT<T, N, C::R, false, C::LS, WAVE>;
    using IFFT = LineFFT<T, N, C::R, true, C::LS, WAVE>;
    constexpr int R = C::R, TPL = C::TPL, LPW = C::LPW;
    constexpr bool JM = DIR == 0 ? LB_JOBMAJOR_X : LB_JOBMAJOR_Y;
    const int nslots = job_slots(njobs, Q);
    const BlockWork w = JM ? decode_block_jm(b, ngroups, ntiles, nslots) : decode_block_at(b, ngroups, ntiles, nslots);
    if (!w.valid) return;
    const InstDesc& I = insts[ilist[w.inst_local]];
    // the block's jobs (uniform over the block): a slot past the table's end, or a q-flux job of
    // an instance with q = 0, does nothing
    JobDesc J[Q];
    bool run[Q];
    bool any = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int jq = w.job * Q + q;
        run[q] = jq < njobs;
        J[q] = jobs[run[q] ? jq : 0];
        if (J[q].flag_q && I.q == 0.0) run[q] = false;
        any = any || run[q];
    }
    if (!any) return;

    const int tid = threadIdx.x;
    const int l = DIR == 0 ? tid / TPL : tid % LPW;
    const int t = DIR == 0 ? tid % TPL : tid / LPW;
    const int line = w.tile * LPW + l;
    const int nx = I.nx, ny = I.ny;
    const int nlines = DIR == 0 ? (ny + 1) / 2 : nx / 2;
    const bool active = line < nlines;
    cpx<T>* lds = lds_all + C::lds_base(l);
    const LB_GLOBAL T* kap = gcast(reinterpret_cast<const T*>(DIR == 0 ? I.kx : I.ky));
    const twptr<T> tw = gcast(reinterpret_cast<const cpx<T>*>(DIR == 0 ? I.twx : I.twy));

    cpx<T> X[Q][R], Y[R];
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (run[q]) load_line<T, DIR, R, TPL>(fieldp<T>(I, J[q].in), X[q], line, t, nx, ny, active);
    // twiddles and wavenumbers are shared by the forward and inverse transforms of every job
    typename FFT::Tw tws;
    tws.load(tw, t);
    Wavenum<T, R, TPL> kv;
    kv.load(kap, t);
    const T invN = T(1.0 / N);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!run[q]) continue;
        FFT::run(X[q], lds, t, tws);
#pragma unroll 1
        for (int o = 0; o < 2; ++o) {
            // select the job slot without runtime indexing (which would go through scratch)
            const int outf = o == 0 ? J[q].out[0] : J[q].out[1];
            if (outf < 0) continue;
            const int mk = o == 0 ? J[q].mult[0] : J[q].mult[1];
            // one uniform branch per output, outside the element loop
            if (mk == M_D) {
#pragma unroll
                for (int m = 0; m < R; ++m) Y[m] = spectral_mult<M_D>(kv[m], invN, X[q][m]);
            } else if (mk == M_DD) {
#pragma unroll
                for (int m = 0; m < R; ++m) Y[m] = spectral_mult<M_DD>(kv[m], invN, X[q][m]);
            } else {
#pragma unroll
                for (int m = 0; m < R; ++m) Y[m] = spectral_mult<M_NONE>(kv[m], invN, X[q][m]);
            }
            IFFT::run(Y, lds, t, tws);
            if (!active) continue;
            LB_GLOBAL T* out = fieldp<T>(I, outf);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int p = t + m * TPL;
                if constexpr (DIR == 0) {
                    out[LineAddr<0>::re(line, p, nx)] = Y[m].re;
                    if (2 * line + 1 < ny) out[LineAddr<0>::im(line, p, nx)] = Y[m].im;
                } else {
                    LB_GLOBAL vec2<T>* o2 = reinterpret_cast<LB_GLOBAL vec2<T>*>(out + LineAddr<1>::re(line, p, nx));
                    o2->a = Y[m].re;
                    o2->b = Y[m].im;
                }
            }
        }
    }
}

template <typename T, int N, int DIR, int RR = 0>
__global__ void __launch_bounds__((LineCfg<T, N, DIR, 0, LB_YMAX_THREADS, RR>::WG))
macro_pass(const InstDesc* __restrict__ insts, const int* __restrict__ ilist, int ngroups,
           int ntiles, const JobDesc* __restrict__ jobs, int njobs) {
    using C = LineCfg<T, N, DIR, 0, LB_YMAX_THREADS, RR>;
    __shared__ cpx<T> lds_all[C::LDS];
    macro_body<T, N, DIR, C::LPW, RR>(blockIdx.x, insts, ilist, ngroups, ntiles, jobs, njobs, lds_all);
}

// The x and y macroscopic passes of one stage of a square grid in one launch: the two read the
// same moments and write different fields, so their blocks can run side by side.  Blocks below
// nbx take x tiles, the rest y tiles; both use the y pass's block shape (x tiles of as many lines).
template <typename T, int N, int RR = 0>
struct MacroXY {
    using Y = LineCfg<T, N, 1, 0, LB_YMAX_THREADS, RR>;
    using X = LineCfg<T, N, 0, Y::LPW, LB_YMAX_THREADS, RR>;
    static constexpr int LPW = Y::LPW;
    static constexpr int WG = Y::WG;
    static constexpr int LDS = Y::LDS;
    static_assert(X::WG == WG && X::LDS == LDS, "x and y tiles of the fused pass must have one block shape");
};

template <typename T, int N, int RR = 0>
__global__ void __launch_bounds__((MacroXY<T, N, RR>::WG))
macro_xy_pass(const InstDesc* __restrict__ insts, const int* __restrict__ ilist, int nbx,
              int ngroups_x, int ntiles_x, const JobDesc* __restrict__ jobs_x, int njobs_x,
              int ngroups_y, int ntiles_y, const JobDesc* __restrict__ jobs_y, int njobs_y) {
    using M = MacroXY<T, N, RR>;
    __shared__ cpx<T> lds_all[M::LDS];
    const int b = blockIdx.x;
    if (b < nbx)
        macro_body<T, N, 0, M::LPW, RR>(b, insts, ilist, ngroups_x, ntiles_x, jobs_x, njobs_x, lds_all);
    else
        macro_body<T, N, 1, M::LPW, RR>(b - nbx, insts, ilist, ngroups_y, ntiles_y, jobs_y, njobs_y, lds_all);
}

// ---------------------------------------------------------------------------------------
// Arithmetic type of the equilibrium in the population x pass.  With an FP32 state it is float64:
// in a nearly uniform state every cell rounds the same FP32 dot products of the same moments the
// same way, so their rounding (and that of the FP32 inverse moment matrix, whose columns then do
// not sum to the exact mass row) does not average out but biases sum_i f_i^eq against rho in every
// cell alike -- a systematic mass drift of ~1e-9 per step.  float64 FMAs issue at the float32 rate
// here (packed FP32 is not used), and the result is rounded once.
template <typename T>
struct EqType {
    using type = T;
};
template <>
struct EqType<float> {
    using type = typename std::conditional<LB_FP32_EQ64 != 0, double, float>::type;
};
template <typename T>
using EqT = typename EqType<T>::type;

template <typename T>
__device__ __forceinline__ const DvmConst<EqT<T>>& eq_table(const DvmConst<T>* d, const DvmConst<double>* d64) {
    if constexpr (std::is_same<EqT<T>, T>::value)
        return *d;
    else
        return *d64;
}

// Equilibrium f_i^eq of the seven kinetic moments: f^eq = C^{-1} M^eq(rho, u, T).
// meq_unit fills m[j] = M^eq_j / rho (the Maxwellian moments per unit density, Sec. 2.2).
template <typename T>
__device__ __forceinline__ void meq_unit(T ux, T uy, T Tm, T b, T (&m)[16]) {
    const T u2 = ux * ux + uy * uy;
    const T h2 = (b + T(2)) * Tm + u2;
    const T h4 = (b + T(4)) * Tm + u2;
    m[0] = T(1);
    m[1] = ux;
    m[2] = uy;
    m[3] = b * Tm + u2;
    m[4] = Tm + ux * ux;
    m[5] = ux * uy;
    m[6] = Tm + uy * uy;
    m[7] = ux * h2;
    m[8] = uy * h2;
    m[9] = T(3) * Tm * ux + ux * ux * ux;
    m[10] = Tm * uy + ux * ux * uy;
    m[11] = Tm * ux + ux * uy * uy;
    m[12] = T(3) * Tm * uy + uy * uy * uy;
    m[13] = h2 * Tm + h4 * ux * ux;
    m[14] = h4 * ux * uy;
    m[15] = h2 * Tm + h4 * uy * uy;
}

// f^eq_i from row c = (C^{-1})_i
template <typename T>
__device__ __forceinline__ T feq_row(const T (&c)[16], T rho, const T (&m)[16]) {
    T s = T(0);
#pragma unroll
    for (int j = 0; j < 16; ++j) s += c[j] * m[j];
    return rho * s;
}
template <typename T>
__device__ __forceinline__ T feq_dot(const DvmConst<T>& D, int i, T rho, const T (&m)[16]) {
    return feq_row(D.cinv[i], rho, m);
}

// Equilibria of a mirror pair (i0, i1) from row c = (C^{-1})_i0: i1 is i0 reflected in x (AX = 0)
// or y (AX = 1), so row i1 of C^{-1} is row i0 with the sign of the moments odd in v_x (resp. v_y)
// flipped.  With E, O the even and odd parts of row i0's dot product, f^eq_i0 = rho (E + O) and
// f^eq_i1 = rho (E - O).  Odd moments in the row order of meq_unit: v_x -> 1, 5, 7, 9, 11, 14;
// v_y -> 2, 5, 8, 10, 12, 14.
template <typename T, int AX>
__device__ __forceinline__ void feq_mirror_row(const T (&c)[16], T rho, const T (&m)[16], T& fe0, T& fe1) {
    constexpr unsigned ODD = AX == 0 ? ((1u << 1) | (1u << 5) | (1u << 7) | (1u << 9) | (1u << 11) | (1u << 14))
                                     : ((1u << 2) | (1u << 5) | (1u << 8) | (1u << 10) | (1u << 12) | (1u << 14));
    T e = T(0), o = T(0);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if ((ODD >> j) & 1u)
            o += c[j] * m[j];
        else
            e += c[j] * m[j];
    }
    fe0 = rho * (e + o);
    fe1 = rho * (e - o);
}

template <typename T>
__device__ __forceinline__ T feq_pop(const DvmConst<T>& D, int i, T rho, T ux, T uy, T Tm, T b) {
    T m[16];
    meq_unit(ux, uy, Tm, b, m);
    return feq_dot(D, i, rho, m);
}

// ---------------------------------------------------------------------------------------
// Epilogue of the population x pass for one thread: its R positions of the block's two rows,
// cell k = 2 m + h (position m, row h).  Per cell it reads the seven macroscopic inputs (rho, u_x,
// u_y, T, B_x, B_y, C) and the P base values, and writes P results.  The cells run in groups of
// LB_EPI_CELLS_F64 / _F32 whose reads are issued one group ahead of the group being computed and stored, so a
// thread has the next group's loads in flight instead of waiting on each cell's loads in turn.
#ifndef LB_EPI_EARLY_F64
#define LB_EPI_EARLY_F64 1
#endif
#ifndef LB_EPI_EARLY_F32
#define LB_EPI_EARLY_F32 0
#endif
#ifndef LB_EPI_CELLS_F64
#define LB_EPI_CELLS_F64 2
#endif
#ifndef LB_EPI_CELLS_F32
#define LB_EPI_CELLS_F32 2
#endif
template <typename T, int R, int TPL, int P>
struct PopXEpi {
    using E = EqT<T>;
    static constexpr int NV = 7 + P;   // values read per cell
    static constexpr int G = sizeof(T) == 8 ? LB_EPI_CELLS_F64 : LB_EPI_CELLS_F32;
    static constexpr int NG = 2 * R / G;
    static_assert((2 * R) % G == 0, "cells per group must divide the cells per thread");
    const DvmConst<T>& D;
    const DvmConst<E>& DE;        // the inverse moment matrix in the equilibrium's arithmetic
    const int (&pop)[P];
    Arena a;
    const uint32_t (&cf)[7];      // field offsets of rho, u_x, u_y, T, B_x, B_y, C
    const uint32_t (&basep)[P];
    const uint32_t (&outp)[P];
    bool has_base;
    int line, t, nx;
    bool row1;   // the block's second row exists (odd ny leaves the last pair with one row)
    E b;
    T c, ct;     // c = alpha dt; ct = c / tau, the same value as in the spectral loss term
    const E (&fref)[P];   // reference populations of the block's P populations (the state is f - fref)
    E Tref;      // reference temperature (the temperature field holds T - Tref)

    __device__ __forceinline__ uint32_t cell(int k) const {
        const int m = k >> 1, h = k & 1;
        // the missing second row of an odd grid reads row 0's cell and stores nothing
        return (uint32_t)(2 * line + (h & (int)row1)) * nx + t + m * TPL;
    }
    __device__ __forceinline__ void load(int g, T (&v)[G][NV]) const {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint32_t e = cell(g * G + j);
#pragma unroll
            for (int f = 0; f < 7; ++f) v[j][f] = bload(a, cf[f], e, T());
#pragma unroll
            for (int q = 0; q < P; ++q) v[j][7 + q] = has_base ? bload(a, basep[q], e, T()) : T(0);
        }
    }
    // rotu: the block's pairs are y mirrors (v_x = 0); their equilibria are those of the x-mirror
    // pairs rot(i) at the turned velocity (u_y, -u_x).  v[0] holds the first group's inputs
    // (requested by the caller with load(0, v[0]), possibly before the transforms).
    __device__ __forceinline__ void run(const cpx<T> (&X)[P][R], bool rotu, T (&v)[2][G][NV]) const {
        // The block's constants, read once into registers: read through D inside the cell loop,
        // they would be fetched again after every store (a buffer store may alias any memory).
        constexpr int NR = P == 1 ? 1 : P / 2;
        E crow[NR][16];   // C^{-1} row of the population, or of each pair's first population
        T pvx[P], pvy[P], pwe[P];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = P == 1 ? pop[0] : (rotu ? D.rot[pop[2 * r]] : pop[2 * r]);
#pragma unroll
            for (int j = 0; j < 16; ++j) crow[r][j] = DE.cinv[i][j];
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            pvx[q] = D.vx[pop[q]];
            pvy[q] = D.vy[pop[q]];
            pwe[q] = D.w[pop[q]] - D.eta2[pop[q]];
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (g + 1 < NG) load(g + 1, v[(g + 1) & 1]);
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int k = g * G + j, m = k >> 1, h = k & 1;
                const T* x = v[g & 1][j];
                const T rho = x[0], ux = x[1], uy = x[2], Bx = x[4], By = x[5], Dc = x[6];
                const E TmE = Tref + E(x[3]);
                const T Tm = T(TmE);
                E mq[16];
                // BGK gain and forcing: f^eq/tau + I = f^eq [1/tau - A - B.(v - u) - D |v - u|^2]
                // with A = -2 D T; the force part expanded in v: h0 + hx v_x + hy v_y + hv |v|^2.
                // The gain's 1/tau part is applied with the coefficient ct of the loss term
                // -(c/tau) f in the spectral multiplier, so that the two cancel in the mass.
                const T h0 = T(2) * Dc * Tm + Bx * ux + By * uy - Dc * (ux * ux + uy * uy);
                const T hx = T(2) * Dc * ux - Bx, hy = T(2) * Dc * uy - By, hv = -Dc;
                E fe[P];
                if constexpr (P == 1) {
                    meq_unit<E>(E(ux), E(uy), TmE, b, mq);
                    fe[0] = feq_row(crow[0], E(rho), mq);
                } else {
                    meq_unit<E>(E(rotu ? uy : ux), E(rotu ? -ux : uy), TmE, b, mq);
#pragma unroll
                    for (int q = 0; q < P; q += 2) feq_mirror_row<E, 0>(crow[q / 2], E(rho), mq, fe[q], fe[q + 1]);
                }
                const uint32_t e = cell(k);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    // relaxation towards f^eq of the deviation from the reference: the loss of
                    // the reference itself, -ct fref, joins the gain ct f^eq
                    const T feq = T(fe[q]);
                    const T dfeq = T(fe[q] - fref[q]);
                    const T gq = h0 + hx * pvx[q] + hy * pvy[q] + hv * pwe[q];
                    const T lin = h == 0 ? X[q][m].re : X[q][m].im;
                    const T base = has_base ? x[7 + q] : T(0);
                    const T out = base + lin + ct * dfeq + c * (feq * gq);
                    if (h == 0 || row1) bstore(a, outp[q], e, out);
                }
            }
        }
    }
};

// Minimum waves per SIMD the population x pass is compiled for: the register budget.  Lines of
// 3 * 2^a points hold 12 elements per thread instead of 8 and get one wave less.
template <typename T>
constexpr int popx_waves(int N, int P) {
    const int w = (sizeof(T) == 8 ? LB_POPX_WAVES_F64 : LB_POPX_WAVES) / P - (default_R(N) == 12 ? 1 : 0);
    return w > 1 ? w : 1;
}

// ---------------------------------------------------------------------------------------
// Population x pass: one block = (instance, tile of row pairs, P populations).  For each
// population i of the block (D.xorder[job*P + q]):
//   out = base + c [ -v_x D_x f - (f - f^eq)/tau + I ]
// to out_field + i if v_y = 0 (final) or to the partial block F_P + i otherwise.  Fields hold
// g = f - fref with fref uniform, so D_x f = D_x g and the terms linear in g, -c v_x D_x g -
// (c/tau) g, are one spectral multiplier (-c/tau + i (-c v_x k))/N, while the reference's own loss
// -(c/tau) fref joins the gain: (c/tau)(f^eq - fref).  The equilibrium moments and the coefficient
// loads of a cell are shared by the P populations.
template <typename T, int N, int P, int RR = 0>
__global__ void __launch_bounds__((LineCfg<T, N, 0, 0, LB_YMAX_THREADS, RR>::WG))
__attribute__((amdgpu_waves_per_eu(popx_waves<T>(N, P))))
pop_x_pass(const InstDesc* __restrict__ insts, const int* __restrict__ ilist, int ngroups,
           int ntiles, const DvmConst<T>* __restrict__ dvm, const DvmConst<double>* __restrict__ dvm64,
           StageArgs st) {
    using C = LineCfg<T, N, 0, 0, LB_YMAX_THREADS, RR>;
    constexpr int R = C::R, TPL = C::TPL;
    // the block's P lines are transformed together when their LDS fits the budget
    constexpr bool BATCH = P > 1 && P * C::LDS * (int)sizeof(cpx<T>) <= LB_POPX_BATCH_LDS;
    __shared__ cpx<T> lds_all[BATCH ? P * C::LDS : C::LDS];
    const BlockWork w = decode_block(ngroups, ntiles, 16 / P);
    if (!w.valid) return;
    const InstDesc& I = insts[ilist[w.inst_local]];
    const DvmConst<T>& D = *dvm;
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid % TPL;
    const int line = w.tile * C::LPW + l;
    const int nx = I.nx, ny = I.ny;
    const bool active = line < (ny + 1) / 2;
    cpx<T>* lds = lds_all + C::lds_base(l);
    const T c = T(st.use_dt ? st.alpha * I.dt : st.alpha);
    const T inv_tau = T(1.0 / I.tau);
    const T ct = c * inv_tau;
    const twptr<T> tw = gcast(reinterpret_cast<const cpx<T>*>(I.twx));
    const LB_GLOBAL T* kap = gcast(reinterpret_cast<const T*>(I.kx));
    const T invN = T(1.0 / N);

    int pop[P];
#pragma unroll
    for (int q = 0; q < P; ++q) pop[q] = D.xorder[w.job * P + q];
    // first stage: the base is the transformed field itself, so it joins the spectral multiplier
    // (1 - c/tau instead of -c/tau) and is not read a second time per cell
    const bool fold = LB_POPX_FOLD_BASE && st.base_field == st.f_field;
    const bool has_base = st.base_field >= 0 && !fold;
    const T ct1 = fold ? ct - T(1) : ct;   // the multiplier's real part is -ct1
    const uint32_t cf[7] = {fofs<T>(I, RHO), fofs<T>(I, UX), fofs<T>(I, UY), fofs<T>(I, TT),
                            fofs<T>(I, BX), fofs<T>(I, BY), fofs<T>(I, CT)};
    uint32_t basep[P], outp[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        // without a base (folded, or the bare right-hand side) nothing is read for it
        basep[q] = fofs<T>(I, has_base ? st.base_field + pop[q] : F_P + pop[q]);
        // out may equal the base block (second stage writes f^{n+1} over f^n per cell)
        outp[q] = fofs<T>(I, (D.vy[pop[q]] == T(0) ? st.out_field : F_P) + pop[q]);
    }
    const bool row1 = 2 * line + 1 < ny;
    EqT<T> fref[P];
#pragma unroll
    for (int q = 0; q < P; ++q) fref[q] = EqT<T>(I.fref[pop[q]]);
    const PopXEpi<T, R, TPL, P> epi{D, eq_table(dvm, dvm64), pop, arena<T>(I), cf, basep, outp, has_base,
                                    line, t, nx, row1, EqT<T>(I.b), c, ct, fref, EqT<T>(I.T_ref)};
    using Epi = PopXEpi<T, R, TPL, P>;
    T ev[2][Epi::G][Epi::NV];
    // FP64, P > 1: the first group of epilogue inputs is requested before the transforms (its latency
    // then hides behind them; the registers are free at the occupancy FP64 blocks run at)
    constexpr bool EARLY = P > 1 && (sizeof(T) == 8 ? LB_EPI_EARLY_F64 : LB_EPI_EARLY_F32);
    if constexpr (EARLY) {
        if (active) epi.load(0, ev[0]);
    }
    // X[q] <- -c v_x D_x f_i - (c/tau) f_i on the block's two rows; all P lines are loaded
    // before the first transform so their memory latencies overlap
    cpx<T> X[P][R];
#pragma unroll
    for (int q = 0; q < P; ++q)
        load_line<T, 0, R, TPL>(fieldp<T>(I, st.f_field + D.xorder[w.job * P + q]), X[q], line, t,
                                nx, ny, active);
    // twiddles and wavenumbers are shared by the block's 2P transforms
    typename LineFFT<T, N, R, false>::Tw tws;
    tws.load(tw, t);
    Wavenum<T, R, TPL> kv;
    kv.load(kap, t);
    if constexpr (BATCH) {
        // the block's populations all have v_x != 0 or all v_x = 0 (pairs in x-pass order)
        const T vx0 = D.vx[D.xorder[w.job * P]];
        if (vx0 != T(0)) {
            LineFFT<T, N, R, false>::template run_n<P>(X, lds, C::LDS, t, tws);
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const T s = -c * D.vx[D.xorder[w.job * P + q]] * invN, mr = -ct1 * invN;
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    const T mi = s * kv[m];
                    const cpx<T> x = X[q][m];
                    X[q][m] = {mr * x.re - mi * x.im, mr * x.im + mi * x.re};
                }
            }
            LineFFT<T, N, R, true>::template run_n<P>(X, lds, C::LDS, t, tws);
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q)
#pragma unroll
                for (int m = 0; m < R; ++m) X[q][m] = {-ct1 * X[q][m].re, -ct1 * X[q][m].im};
        }
    }
#pragma unroll
    for (int q = 0; q < (BATCH ? 0 : P); ++q) {
        const int i = D.xorder[w.job * P + q];
        const T vx = D.vx[i];
        if (vx != T(0)) {
            LineFFT<T, N, R, false>::run(X[q], lds, t, tws);
            const T s = -c * vx * invN, mr = -ct1 * invN;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const T mi = s * kv[m];
                const cpx<T> x = X[q][m];
                X[q][m] = {mr * x.re - mi * x.im, mr * x.im + mi * x.re};
            }
            LineFFT<T, N, R, true>::run(X[q], lds, t, tws);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) X[q][m] = {-ct1 * X[q][m].re, -ct1 * X[q][m].im};
        }
    }
    if (!active) return;
    // keep the (other) epilogue loads out of the transforms above: their registers would be
    // live there
    asm volatile("" ::: "memory");
    if constexpr (!EARLY) epi.load(0, ev[0]);
    // pairs of populations with v_x != 0 are x mirrors, the others y mirrors (uniform per block)
    epi.run(X, P > 1 && D.vx[pop[0]] == T(0), ev);
}

// Population y pass: one block = (instance, tile of column pairs, population i with v_y != 0).
//   out = partial - c v_y D_y f
template <typename T, int N, int MAXT = LB_YMAX_THREADS, int RR = 0>
__global__ void __launch_bounds__((LineCfg<T, N, 1, 0, MAXT, RR>::WG))
pop_y_pass(const InstDesc* __restrict__ insts, const int* __restrict__ ilist, int ngroups,
           int ntiles, const DvmConst<T>* __restrict__ dvm, const int* __restrict__ pops, int npops,
           StageArgs st) {
    using C = LineCfg<T, N, 1, 0, MAXT, RR>;
    constexpr int R = C::R, TPL = C::TPL, LPW = C::LPW;
    __shared__ cpx<T> lds_all[C::LDS];
    const BlockWork w = LB_JOBMAJOR_Y ? decode_block_jm(blockIdx.x, ngroups, ntiles, npops)
                                      : decode_block(ngroups, ntiles, npops);
    if (!w.valid) return;
    const InstDesc& I = insts[ilist[w.inst_local]];
    const int i = pops[w.job];
    const int tid = threadIdx.x;
    const int l = tid % LPW, t = tid / LPW;
    const int line = w.tile * LPW + l;
    const int nx = I.nx, ny = I.ny;
    const bool active = line < nx / 2;
    cpx<T>* lds = lds_all + C::lds_base(l);
    const T vy = dvm->vy[i];
    const twptr<T> tw = gcast(reinterpret_cast<const cpx<T>*>(I.twy));

    // the line, the twiddles and the wavenumbers (and in FP32 the partial sums the result is
    // added to) are requested before the transforms so that their latencies overlap; in FP64 the
    // partial sums are read after the transforms, all before the first store, to spare registers.
    // The FP32 long-radix plans (16 or 24 elements per thread) spare registers the same way and
    // read each pass's twiddles when the pass runs: at 1024 and 2048 points that leaves them 121
    // registers instead of 164-177, four waves per SIMD instead of two or three.
    constexpr bool LONG = sizeof(T) == 4 && R >= 16;
    constexpr bool EARLY = sizeof(T) == 4 && !LONG;
    constexpr int PL = LONG ? 0 : tw_preload_limit<T>();
    using FFT = LineFFT<T, N, R, false, C::LS, false, PL>;
    using IFFT = LineFFT<T, N, R, true, C::LS, false, PL>;
    cpx<T> X[R];
    load_line<T, 1, R, TPL>(fieldp<T>(I, st.f_field + i), X, line, t, nx, ny, active);
    cpx<T> Pv[R];
    if constexpr (EARLY) load_line<T, 1, R, TPL>(fieldp<T>(I, F_P + i), Pv, line, t, nx, ny, active);
    typename FFT::Tw tws;
    tws.load(tw, t);
    const LB_GLOBAL T* kap = gcast(reinterpret_cast<const T*>(I.ky));
    Wavenum<T, R, TPL> kv;
    kv.load(kap, t);
    FFT::run(X, lds, t, tws);
    const T s = -T(st.use_dt ? st.alpha * I.dt : st.alpha) * vy * T(1.0 / N);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const T a = s * kv[m];
        const cpx<T> x = X[m];
        X[m] = {-a * x.im, a * x.re};
    }
    IFFT::run(X, lds, t, tws);
    if (!active) return;
    if constexpr (!EARLY) load_line<T, 1, R, TPL>(fieldp<T>(I, F_P + i), Pv, line, t, nx, ny, true);
    LB_GLOBAL T* out = fieldp<T>(I, st.out_field + i);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int p = t + m * TPL;
        LB_GLOBAL vec2<T>* o = reinterpret_cast<LB_GLOBAL vec2<T>*>(out + LineAddr<1>::re(line, p, nx));
        o->a = Pv[m].re + X[m].re;
        o->b = Pv[m].im + X[m].im;
    }
}

// ---------------------------------------------------------------------------------------
// Pointwise kernels: grid = (cell chunks, instances in the launch).
#define LB_POINTWISE_PROLOGUE                                        \
    const InstDesc& I = insts[ilist[blockIdx.y]];                    \
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;        \
    if (e >= (uint32_t)I.ncell) return;

// Moments of Sec. 2.1: rho = sum f, rho u = sum f v, rho (b T + u^2) = sum f (v^2 + eta^2).
template <typename T>
__global__ void __launch_bounds__(256)
moments_kernel(const InstDesc* __restrict__ insts, const int* __restrict__ ilist,
               const DvmConst<double>* __restrict__ dvm, int f_field) {
    LB_POINTWISE_PROLOGUE
    const DvmConst<double>& D = *dvm;
    // The stored state is f - fref: its moments plus those of the reference, which is at rest
    // with density rho_ref and energy moment e_ref = rho_ref b T_ref.  The deviations' own moments
    // r, jx, jy, en are summed in the working precision (their rounding scales with the
    // deviation); the rest is formed in float64 and rounded once on store.  The temperature is
    // stored as T - T_ref = ((E - rho b T_ref) / rho - |u|^2) / b, where E - rho b T_ref =
    // en - r b T_ref.
    T r = 0, jx = 0, jy = 0, en = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const T f = fieldp<T>(I, f_field + i)[e];
        r += f;
        jx += f * T(D.vx[i]);
        jy += f * T(D.vy[i]);
        en += f * T(D.w[i]);
    }
    const double rho = I.rho_ref + double(r);
    const double ux = double(jx) / rho, uy = double(jy) / rho;
    fieldp<T>(I, RHO)[e] = T(rho);
    fieldp<T>(I, UX)[e] = T(ux);
    fieldp<T>(I, UY)[e] = T(uy);
    fieldp<T>(I, TT)[e] = T(((double(en) - double(r) * I.bT_ref) / rho - ux * ux - uy * uy) / I.b);
}

// Stress S = (P^w - rho T) I + Lambda - zeta (div u) I, div u, Q = q rho T grad T and the part
// C0 of Eq. (2)'s C that needs no second pass (everything but -K rho grad rho . grad(div u);
// C_q is added in finalize_kernel) (Sec. 2.2).
template <typename T>
__global__ void __launch_bounds__(256)
stress_kernel(const InstDesc* __restrict__ insts, const int* __restrict__ ilist) {
    LB_POINTWISE_PROLOGUE
    const T rho = fieldp<T>(I, RHO)[e], Tm = T(I.T_ref) + fieldp<T>(I, TT)[e];   // field: T - T_ref
    const T rx = fieldp<T>(I, RX)[e], ry = fieldp<T>(I, RY)[e];
    const T lap = fieldp<T>(I, RXX)[e] + fieldp<T>(I, RYY)[e];
    const T Tx = fieldp<T>(I, TX)[e], Ty = fieldp<T>(I, TY)[e];
    const T uxx = fieldp<T>(I, UXX)[e], uxy = fieldp<T>(I, UXY)[e];   // d_x u_x, d_y u_x
    const T uyx = fieldp<T>(I, UYX)[e], uyy = fieldp<T>(I, UYY)[e];   // d_x u_y, d_y u_y
    const T K = T(I.K), H = T(I.H), zeta = T(I.zeta), a = T(I.a), bw = T(I.bw);

    const T div = uxx + uyy;
    const T rT = rho * Tm;
    const T Pw = rT / (T(1) - bw * rho) - a * rho * rho;
    const T M = K + H * Tm;
    const T g2 = rx * rx + ry * ry;
    const T iT2 = T(1) / (Tm * Tm);
    const T mtx = -K * Tx * iT2, mty = -K * Ty * iT2;   // grad(M/T), H constant
    const T iso = -M * (rho * lap + T(0.5) * g2) - rT * (rx * mtx + ry * mty);
    const T Lxx = M * rx * rx + iso, Lxy = M * rx * ry, Lyy = M * ry * ry + iso;
    const T pn = Pw - rT;
    fieldp<T>(I, SXX)[e] = pn + Lxx - zeta * div;
    fieldp<T>(I, SXY)[e] = Lxy;
    fieldp<T>(I, SYY)[e] = pn + Lyy - zeta * div;
    fieldp<T>(I, DIV)[e] = div;
    const T lam_du = Lxx * uxx + Lxy * uyx + Lxy * uxy + Lyy * uyy;
    const T rgr = rx * (uxx * rx + uyx * ry) + ry * (uxy * rx + uyy * ry);
    const T num = pn * div + lam_du - zeta * div * div + a * rho * rho * div +
                  K * (T(-0.5) * g2 * div - rgr);
    fieldp<T>(I, C0)[e] = num / (T(2) * rT * Tm);
    if (I.q != 0.0) {
        const T qrt = T(I.q) * rT;
        fieldp<T>(I, QX)[e] = qrt * Tx;
        fieldp<T>(I, QY)[e] = qrt * Ty;
    }
}

// B = div S / (rho T) and C + C_q of Eq. (2) from the second derivative passes:
//   C = C0 - K rho grad rho . grad(div u) / (2 rho T^2),  C_q = div Q / (rho T^2).
template <typename T>
__global__ void __launch_bounds__(256)
finalize_kernel(const InstDesc* __restrict__ insts, const int* __restrict__ ilist) {
    LB_POINTWISE_PROLOGUE
    const T rho = fieldp<T>(I, RHO)[e], Tm = T(I.T_ref) + fieldp<T>(I, TT)[e];   // field: T - T_ref
    const T rT = rho * Tm;
    fieldp<T>(I, BX)[e] = (fieldp<T>(I, DSXX)[e] + fieldp<T>(I, DYSXY)[e]) / rT;
    fieldp<T>(I, BY)[e] = (fieldp<T>(I, DSXY)[e] + fieldp<T>(I, DYSYY)[e]) / rT;
    const T rx = fieldp<T>(I, RX)[e], ry = fieldp<T>(I, RY)[e];
    const T gdx = fieldp<T>(I, GDX)[e], gdy = fieldp<T>(I, GDY)[e];
    T c = fieldp<T>(I, C0)[e] - T(I.K) * rho * (rx * gdx + ry * gdy) / (T(2) * rT * Tm);
    if (I.q != 0.0) c += (fieldp<T>(I, DQX)[e] + fieldp<T>(I, DYQY)[e]) / (rT * Tm);
    fieldp<T>(I, CT)[e] = c;
}

// Initial populations f = f^eq(rho0, u0, T0), computed in float64 from float64 inputs staged in
// the F_B block (4 double fields), stored as f - fref in the working precision into F_A.
template <typename T>
__global__ void __launch_bounds__(256)
init_kernel(const InstDesc* __restrict__ insts, const int* __restrict__ ilist,
            const DvmConst<double>* __restrict__ dvm) {
    LB_POINTWISE_PROLOGUE
    const int64_t nc = I.ncell;
    const LB_GLOBAL double* stage = gcast(reinterpret_cast<const double*>(reinterpret_cast<const T*>(I.base) + F_B * nc));
    const double rho = stage[e], ux = stage[nc + e], uy = stage[2 * nc + e], Tm = stage[3 * nc + e];
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = feq_pop<double>(*dvm, i, rho, ux, uy, Tm, I.b);
#pragma unroll
    for (int i = 0; i < 16; ++i) fieldp<T>(I, F_A + i)[e] = T(f[i] - I.fref[i]);
}

// Per-cell conserved densities, summed per block in float64 (grid: red_blocks x instances):
//   mass rho, momentum rho u, energy rho (b T + u^2)/2 - a rho^2 + K |grad rho|^2 / 2 (Sec. 2.2),
// and a count of non-finite cells.  Block partials go to I.red[block * 5 + k].
template <typename T>
__global__ void __launch_bounds__(256)
conserve_partial(const InstDesc* __restrict__ insts, const int* __restrict__ ilist) {
    const InstDesc& I = insts[ilist[blockIdx.y]];
    const uint32_t nc = (uint32_t)I.ncell;
    double acc[5] = {0, 0, 0, 0, 0};
    const LB_GLOBAL T* rp = fieldp<T>(I, RHO);
    const LB_GLOBAL T* xp = fieldp<T>(I, UX);
    const LB_GLOBAL T* yp = fieldp<T>(I, UY);
    const LB_GLOBAL T* tp = fieldp<T>(I, TT);
    const LB_GLOBAL T* gxp = fieldp<T>(I, RX);
    const LB_GLOBAL T* gyp = fieldp<T>(I, RY);
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += I.red_blocks * blockDim.x) {
        const double rho = rp[e], ux = xp[e], uy = yp[e], Tm = I.T_ref + tp[e], rx = gxp[e], ry = gyp[e];
        const double en = 0.5 * rho * (I.b * Tm + ux * ux + uy * uy) - I.a * rho * rho +
                          0.5 * I.K * (rx * rx + ry * ry);
        acc[0] += rho;
        acc[1] += rho * ux;
        acc[2] += rho * uy;
        acc[3] += en;
        acc[4] += (isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(Tm)) ? 0.0 : 1.0;
    }
    __shared__ double sh[5][256];
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) I.red[blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

// Convert between the working precision and float64 (host transfers of non-hot calls).
template <typename T>
__global__ void __launch_bounds__(256) to_f64(const T* __restrict__ src, double* __restrict__ dst, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = double(src[e]);
}
template <typename T>
__global__ void __launch_bounds__(256) from_f64(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = T(src[e]);
}

}  // namespace lbfft
