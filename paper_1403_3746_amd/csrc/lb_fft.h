// Line FFT engine for gfx950: Stockham autosort mixed-radix (2, 3, 4, 8, 12, 16, 24) transforms of complex
// lines of length N held R elements per thread, exchanged through LDS between passes.
//
// A line is processed by N/R consecutive "line threads"; thread t holds elements t + m*(N/R),
// m = 0..R-1 ("natural" order) on entry and the transform coefficients X[t + m*(N/R)] on exit.
// Passes whose radix equals R read (first pass) or write (last pass) registers directly; all
// other passes go through the line's LDS region of N complex words.  Twiddles come from a
// float64-generated table exp(-2 pi i k/N), k = 0..N-1, rounded to the working precision.
#pragma once
#include <hip/hip_runtime.h>

// Global-memory pointers: pointers read out of descriptors are otherwise generic (flat), and flat
// accesses also hold the LDS wait counter, which stalls the FFT's LDS exchanges on field loads.
#define LB_GLOBAL __attribute__((address_space(1)))

namespace lbfft {

template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ const LB_GLOBAL T* gcast(const T* p) {
    return (const LB_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ LB_GLOBAL T* gcast(T* p) {
    return (LB_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> rot90(cpx<T> a) {
    if (INV) return {-a.im, a.re};
    return {a.im, -a.re};
}

// In-register DFT of size r, outputs in natural order.  Forward kernel exp(-2 pi i pq/r),
// inverse exp(+2 pi i pq/r).
template <typename T, int r, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T, bool INV>
struct Dft<T, 3, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        const T h = T(0.86602540378443864676);  // sqrt(3)/2
        cpx<T> s = cadd(v[1], v[2]);
        cpx<T> d = csub(v[1], v[2]);
        cpx<T> x0 = v[0];
        cpx<T> t = {x0.re - T(0.5) * s.re, x0.im - T(0.5) * s.im};
        cpx<T> rd = rot90<T, INV>(d);   // -i d (forward), +i d (inverse)
        v[0] = cadd(x0, s);
        v[1] = {t.re + h * rd.re, t.im + h * rd.im};
        v[2] = {t.re - h * rd.re, t.im - h * rd.im};
    }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        cpx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        cpx<T> a2 = cadd(v[1], v[3]), a3 = rot90<T, INV>(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        const T s = T(0.70710678118654752440);
        // split into even/odd halves of the decimation-in-frequency step
        cpx<T> a[4], b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = cadd(v[k], v[k + 4]);
            b[k] = csub(v[k], v[k + 4]);
        }
        // b[k] *= w8^k, w8 = exp(-+ i pi/4)
        {
            cpx<T> x = b[1];
            // forward: (1 - i)/sqrt2 ; inverse: (1 + i)/sqrt2
            b[1] = INV ? cpx<T>{s * (x.re - x.im), s * (x.re + x.im)}
                       : cpx<T>{s * (x.re + x.im), s * (x.im - x.re)};
            b[2] = rot90<T, INV>(b[2]);
            x = b[3];
            // forward: (-1 - i)/sqrt2 ; inverse: (-1 + i)/sqrt2
            b[3] = INV ? cpx<T>{s * (-x.re - x.im), s * (x.re - x.im)}
                       : cpx<T>{s * (x.im - x.re), s * (-x.re - x.im)};
        }
        Dft<T, 4, INV>::run(a);
        Dft<T, 4, INV>::run(b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = a[k];
            v[2 * k + 1] = b[k];
        }
    }
};

// 12-point DFT by the Good-Thomas (prime-factor) split 12 = 3 x 4: with the input index
// n = (4 n1 + 3 n2) mod 12 and the output index k = (4 k1 + 9 k2) mod 12 (both bijections, by the
// Chinese remainder theorem) the kernel factors as W12^(nk) = W3^(n1 k1) W4^(n2 k2), so four
// 3-point DFTs over n1 followed by three 4-point DFTs over n2 need no twiddles between them.
template <typename T, bool INV>
struct Dft<T, 12, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        cpx<T> y[4][3];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 3; ++n1) y[n2][n1] = v[(4 * n1 + 3 * n2) % 12];
            Dft<T, 3, INV>::run(y[n2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            cpx<T> c[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            Dft<T, 4, INV>::run(c);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[(4 * k1 + 9 * k2) % 12] = c[k2];
        }
    }
};

// 24-point DFT by the Good-Thomas split 24 = 3 x 8: input index n = (8 n1 + 3 n2) mod 24, output
// index k = (16 k1 + 9 k2) mod 24, so W24^(nk) = W3^(n1 k1) W8^(n2 k2): eight 3-point DFTs over n1,
// then three 8-point DFTs over n2, no twiddles between them.
template <typename T, bool INV>
struct Dft<T, 24, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        cpx<T> y[8][3];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 3; ++n1) y[n2][n1] = v[(8 * n1 + 3 * n2) % 24];
            Dft<T, 3, INV>::run(y[n2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            cpx<T> c[8];
#pragma unroll
            for (int n2 = 0; n2 < 8; ++n2) c[n2] = y[n2][k1];
            Dft<T, 8, INV>::run(c);
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) v[(16 * k1 + 9 * k2) % 24] = c[k2];
        }
    }
};

// a * W16^m, W16 = exp(-+ 2 pi i / 16) (forward / inverse), for the internal twiddles of the
// 16-point DFT (m = n2 k1 <= 9); m is a constant after unrolling, so the switch folds away and the
// eighth and quarter turns cost no general product.
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> w16(cpx<T> a, int m) {
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    const T h = T(0.70710678118654752440);
    // forward W16^m = (cos t, -sin t), t = pi m / 8; the inverse conjugates
    auto mul = [](cpx<T> x, T c, T sn) -> cpx<T> {
        const T si = INV ? -sn : sn;   // multiply by (c, -si)
        return {x.re * c + x.im * si, x.im * c - x.re * si};
    };
    switch (m) {
        case 0: return a;
        case 1: return mul(a, c1, s1);
        case 2: return INV ? cpx<T>{h * (a.re - a.im), h * (a.re + a.im)} : cpx<T>{h * (a.re + a.im), h * (a.im - a.re)};
        case 3: return mul(a, s1, c1);
        case 4: return rot90<T, INV>(a);
        case 6: return INV ? cpx<T>{h * (-a.re - a.im), h * (a.re - a.im)} : cpx<T>{h * (a.im - a.re), h * (-a.re - a.im)};
        case 9: return mul(a, -c1, -s1);
        default: return mul(a, T(0), T(0));   // not reached: m = n2 k1 takes the values above
    }
}

// 16-point DFT as 4 x 4: element n = 4 n1 + n2, output k = k1 + 4 k2; 4-point DFTs over n1, the
// internal twiddles W16^(n2 k1), 4-point DFTs over n2.
template <typename T, bool INV>
struct Dft<T, 16, INV> {
    __device__ __forceinline__ static void run(cpx<T>* v) {
        cpx<T> b[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) b[n2][n1] = v[4 * n1 + n2];
            Dft<T, 4, INV>::run(b[n2]);
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) b[n2][k1] = w16<T, INV>(b[n2][k1], n2 * k1);
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cpx<T> c[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
            Dft<T, 4, INV>::run(c);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = c[k2];
        }
    }
};

// ---------------------------------------------------------------------------------------
// Radix plans.  R (elements per thread) and the pass radices are compile-time functions of N.
// Supported N: 1, 2 and 2^a, 3*2^a for 8 <= N <= 2048.
constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

constexpr int default_R(int N) {
    return N <= 2 ? N : (N % 3 == 0 ? 12 : (N == 16 || N == 32 ? 4 : 8));
}

struct Plan {
    int np;
    int r[12];
};

constexpr Plan make_plan(int N, int R) {
    Plan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    if (N <= 1) return p;
    if (N == 2) {
        p.np = 1;
        p.r[0] = 2;
        return p;
    }
    if (R == 24) {
        // lines of 3 * 2^a points held 24 elements per thread: one radix-24 pass from the
        // registers, then N/24 = 2^b in radix-8 passes, a radix-2 or radix-4 pass first where b is
        // not a multiple of 3
        p.r[p.np++] = 24;
        int q = N / 24;
        const int rem = 1 << (ilog2c(q) % 3);
        if (rem > 1) {
            p.r[p.np++] = rem;
            q /= rem;
        }
        for (; q > 1; q /= 8) p.r[p.np++] = 8;
        return p;
    }
    if (R == 12) {
        // lines of 3 * 2^a points: one radix-12 pass straight from the registers, then the power
        // of two N/12 in radix-4 passes (a radix-2 pass first when the exponent is odd)
        p.r[p.np++] = 12;
        int q = N / 12;
        if (q > 1 && (ilog2c(q) & 1)) {
            p.r[p.np++] = 2;
            q /= 2;
        }
        for (; q > 1; q /= 4) p.r[p.np++] = 4;
        return p;
    }
    int three = (N % 3 == 0) ? 1 : 0;
    int pow2 = three ? N / 3 : N;
    int big = R;
    int nbig = 0;
    while (pow2 >= big && pow2 % big == 0) {
        pow2 /= big;
        ++nbig;
    }
    int rem = pow2;  // 1, 2, 4 (or 8 with radix-16 passes)
    // first a big radix, then the odd factors, then the remaining big radices
    if (nbig > 0) {
        p.r[p.np++] = big;
        --nbig;
    }
    if (three) p.r[p.np++] = 3;
    if (rem > 1) p.r[p.np++] = rem;
    while (nbig-- > 0) p.r[p.np++] = big;
    return p;
}

constexpr int plan_ns(const Plan& p, int s) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= p.r[i];
    return ns;
}

// LDS index of line element i: one padding word after every 8 elements, so the stride-r writes of
// a Stockham pass (r = 2..8 complex words apart in consecutive lanes) spread over the banks.
constexpr int LDS_PAD_SHIFT = 3;
__host__ __device__ constexpr int lds_idx(int i) { return i + (i >> LDS_PAD_SHIFT); }
// LDS words reserved per line of length N.
__host__ __device__ constexpr int lds_line(int N) { return N + (N >> LDS_PAD_SHIFT) + 1; }

template <typename T>
using twptr = const LB_GLOBAL cpx<T>*;

// Bytes a table read may address: the longest line's table (2048 complex float64 words).
constexpr int TABLE_MAX_BYTES = 2048 * 16;

// Table entry idx as one load of the whole complex word (a 16-byte buffer load in float64, 8 bytes
// in float32).  Read member by member, the two halves were separate loads that the code generator
// pairs up again afterwards, and hipcc of ROCm 7.2 (AMD clang 22) paired them wrongly in the
// 96-point float64 x passes: the imaginary half of one twiddle was taken from another entry's
// load (the optimised IR was right; the emitted code was not).  One intrinsic load per entry
// leaves nothing to pair.
template <typename T>
__device__ __forceinline__ cpx<T> ldc(twptr<T> p, int idx) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, TABLE_MAX_BYTES, 0x00020000);
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (unsigned)idx * 16u, 0, 0));
    else
        return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, (unsigned)idx * 8u, 0, 0));
}

// Barrier between the LDS exchanges of a transform.  WAVE: every line the block holds belongs to
// one wave (x blocks of lines of at most 64 threads), so only the wave's own LDS accesses need
// ordering: a wave's LDS instructions execute in issue order, and the fences keep the compiler
// from moving accesses across; the block's waves then run their transforms independently.
template <bool WAVE>
__device__ __forceinline__ void line_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Number of twiddles a radix-r butterfly reads: radix 16 reads w, w^2, w^4, w^8 and forms the rest
// by at most two products; radix 8 reads w, w^2, w^4 and forms the rest by at most two products;
// radix 4 reads w, w^2; radix 2 and 3 read w^q, q = 1..r-1, directly.
constexpr int tw_reads(int r) { return r == 16 ? 4 : (r == 8 ? 3 : (r == 4 ? 2 : r - 1)); }

// Twiddles w^q, q = 1..r-1, of one butterfly from its tw_reads(r) loaded values.
template <typename T, int r>
__device__ __forceinline__ void twiddle_powers(const cpx<T>* b, cpx<T>* w) {
    if constexpr (r == 16) {
        w[1] = b[0];
        w[2] = b[1];
        w[4] = b[2];
        w[8] = b[3];
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
#pragma unroll
        for (int q = 1; q < 8; ++q) w[8 + q] = cmul(w[8], w[q]);
    } else if constexpr (r == 8) {
        w[1] = b[0];
        w[2] = b[1];
        w[4] = b[2];
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    } else if constexpr (r == 4) {
        w[1] = b[0];
        w[2] = b[1];
        w[3] = cmul(w[1], w[2]);
    } else {
#pragma unroll
        for (int q = 1; q < r; ++q) w[q] = b[q - 1];
    }
}

// The tw_reads(r) table values of a butterfly with base index `step`.
template <typename T, int r>
__device__ __forceinline__ void tw_fetch(twptr<T> table, int step, cpx<T>* d) {
    if constexpr (r == 16) {
        d[0] = ldc(table, step);
        d[1] = ldc(table, 2 * step);
        d[2] = ldc(table, 4 * step);
        d[3] = ldc(table, 8 * step);
    } else if constexpr (r == 8) {
        d[0] = ldc(table, step);
        d[1] = ldc(table, 2 * step);
        d[2] = ldc(table, 4 * step);
    } else if constexpr (r == 4) {
        d[0] = ldc(table, step);
        d[1] = ldc(table, 2 * step);
    } else {
#pragma unroll
        for (int q = 1; q < r; ++q) d[q - 1] = ldc(table, q * step);
    }
}

// The twiddles one thread reads over all passes of a line transform (passes after the first).
// Pass s with Ns = r_0...r_{s-1} gives butterfly b of thread t (element j = t + b*TPL,
// k = j mod Ns) the powers of tw[k*N/(Ns*r)].  When they fit in a few registers (COUNT complex
// values, at most LB_TW_PRELOAD / LB_TW_PRELOAD_F32) they are loaded together up front, so their
// latencies overlap,
// and shared by the forward and inverse transforms of the line (the inverse multiplies by their
// conjugates); otherwise each pass loads its own from the table.
#ifndef LB_TW_PRELOAD
#define LB_TW_PRELOAD 12      // float64: at most 12 complex values (48 registers)
#endif
#ifndef LB_TW_PRELOAD_F32
#define LB_TW_PRELOAD_F32 18  // float32: at most 18 (36 registers; the 384- and 768-point plans)
#endif
template <typename T>
constexpr int tw_preload_limit() { return sizeof(T) == 4 ? LB_TW_PRELOAD_F32 : LB_TW_PRELOAD; }
// PL: the preload limit, which a kernel may lower to spare registers
template <typename T, int N, int R, int PL = tw_preload_limit<T>()>
struct TwSet {
    static constexpr Plan P = make_plan(N, R);
    static constexpr int TPL = N / R;
    static constexpr int offset(int s) {
        int o = 0;
        for (int i = 0; i < s; ++i)
            if (plan_ns(P, i) > 1) o += (R / P.r[i]) * tw_reads(P.r[i]);
        return o;
    }
    static constexpr int COUNT = offset(P.np);
    static constexpr bool PRE = COUNT <= PL;
    cpx<T> w[PRE && COUNT > 0 ? COUNT : 1];
    twptr<T> table;
    int t;

    // pass s's twiddles, read with the index the pass itself uses (stockham_pass)
    template <int s>
    __device__ __forceinline__ void load_pass() {
        if constexpr (s < P.np) {
            constexpr int r = P.r[s], Ns = plan_ns(P, s), NB = R / r, OFF = offset(s);
            if constexpr (Ns > 1) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int j = t + b * TPL;
                    const int k = j % Ns;
                    tw_fetch<T, r>(table, k * (N / (Ns * r)), w + OFF + b * tw_reads(r));
                }
            }
            load_pass<s + 1>();
        }
    }
    __device__ __forceinline__ void load(twptr<T> tab, int thread) {
        table = tab;
        t = thread;
        if constexpr (PRE) load_pass<0>();
    }
    // the preloaded tw_reads(r) values of butterfly b of pass s
    template <int s>
    __device__ __forceinline__ void get(int b, cpx<T>* d) const {
        constexpr int r = P.r[s], OFF = offset(s);
#pragma unroll
        for (int i = 0; i < tw_reads(r); ++i) d[i] = w[OFF + b * tw_reads(r) + i];
    }
};

// Pass S of the plan: one Stockham pass of radix r = P.r[S] with Ns = product of the previous radices.
// LDS element i of the line lives at lds[lds_idx(i) * LS]: LS = 1 for line-contiguous storage,
// LS = lines per block for lines interleaved word by word (lanes of neighbouring lines adjacent).
template <typename T, int N, int R, int S, bool INV, bool FROM_REG, bool TO_REG, int LS, bool WAVE = false, int PL = 0>
__device__ __forceinline__ void stockham_pass(cpx<T> (&v)[R], cpx<T>* lds, int t, const TwSet<T, N, R, PL>& tw) {
    using TW = TwSet<T, N, R, PL>;
    constexpr int r = TW::P.r[S];
    constexpr int Ns = plan_ns(TW::P, S);
    constexpr int TPL = N / R;
    constexpr int NB = R / r;
    static_assert(R % r == 0, "radix must divide R");
    cpx<T> a[R];
    if constexpr (FROM_REG) {
        static_assert(NB == 1, "register-direct pass needs r == R");
#pragma unroll
        for (int q = 0; q < r; ++q) a[q] = v[q];
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + b * TPL;
#pragma unroll
            for (int q = 0; q < r; ++q) a[b * r + q] = lds[lds_idx(j + q * (N / r)) * LS];
        }
        line_sync<WAVE>();
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * TPL;
        const int k = j % Ns;
        if constexpr (Ns > 1) {
            cpx<T> tb[tw_reads(r)], w[r];
            if constexpr (TW::PRE)
                tw.template get<S>(b, tb);
            else
                tw_fetch<T, r>(tw.table, k * (N / (Ns * r)), tb);
            twiddle_powers<T, r>(tb, w);
#pragma unroll
            for (int q = 1; q < r; ++q) a[b * r + q] = INV ? cmulc(a[b * r + q], w[q]) : cmul(a[b * r + q], w[q]);
        }
        Dft<T, r, INV>::run(&a[b * r]);
        if constexpr (TO_REG) {
            static_assert(NB == 1, "register-direct pass needs r == R");
#pragma unroll
            for (int q = 0; q < r; ++q) v[q] = a[q];
        } else {
            const int base = (j / Ns) * Ns * r + k;
#pragma unroll
            for (int q = 0; q < r; ++q) lds[lds_idx(base + q * Ns) * LS] = a[b * r + q];
        }
    }
    if constexpr (!TO_REG) line_sync<WAVE>();
}

// Pass S for Q lines at once (line q's LDS region starts `stride` complex words after line
// q-1's): one LDS round trip and one pair of barriers for all Q lines, the butterflies' twiddle
// powers formed once and applied to every line, and Q independent butterflies per twiddle set for
// the scheduler to interleave.
template <typename T, int N, int R, int S, bool INV, bool FROM_REG, bool TO_REG, int LS, int Q,
          bool WAVE = false, int PL = 0>
__device__ __forceinline__ void stockham_pass_n(cpx<T> (&v)[Q][R], cpx<T>* lds, int stride, int t,
                                                const TwSet<T, N, R, PL>& tw) {
    using TW = TwSet<T, N, R, PL>;
    constexpr int r = TW::P.r[S];
    constexpr int Ns = plan_ns(TW::P, S);
    constexpr int TPL = N / R;
    constexpr int NB = R / r;
    static_assert(R % r == 0, "radix must divide R");
    cpx<T> a[Q][R];
    if constexpr (FROM_REG) {
        static_assert(NB == 1, "register-direct pass needs r == R");
#pragma unroll
        for (int l = 0; l < Q; ++l)
#pragma unroll
            for (int q = 0; q < r; ++q) a[l][q] = v[l][q];
    } else {
#pragma unroll
        for (int l = 0; l < Q; ++l)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = t + b * TPL;
#pragma unroll
                for (int q = 0; q < r; ++q) a[l][b * r + q] = lds[l * stride + lds_idx(j + q * (N / r)) * LS];
            }
        line_sync<WAVE>();
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * TPL;
        const int k = j % Ns;
        if constexpr (Ns > 1) {
            cpx<T> tb[tw_reads(r)], w[r];
            if constexpr (TW::PRE)
                tw.template get<S>(b, tb);
            else
                tw_fetch<T, r>(tw.table, k * (N / (Ns * r)), tb);
            twiddle_powers<T, r>(tb, w);
#pragma unroll
            for (int l = 0; l < Q; ++l)
#pragma unroll
                for (int q = 1; q < r; ++q)
                    a[l][b * r + q] = INV ? cmulc(a[l][b * r + q], w[q]) : cmul(a[l][b * r + q], w[q]);
        }
#pragma unroll
        for (int l = 0; l < Q; ++l) Dft<T, r, INV>::run(&a[l][b * r]);
        if constexpr (TO_REG) {
            static_assert(NB == 1, "register-direct pass needs r == R");
#pragma unroll
            for (int l = 0; l < Q; ++l)
#pragma unroll
                for (int q = 0; q < r; ++q) v[l][q] = a[l][q];
        } else {
            const int base = (j / Ns) * Ns * r + k;
#pragma unroll
            for (int l = 0; l < Q; ++l)
#pragma unroll
                for (int q = 0; q < r; ++q) lds[l * stride + lds_idx(base + q * Ns) * LS] = a[l][b * r + q];
        }
    }
    if constexpr (!TO_REG) line_sync<WAVE>();
}

template <typename T, int N, int R, bool INV, int LS = 1, bool WAVE = false, int PL = tw_preload_limit<T>()>
struct LineFFT {
    static constexpr Plan P = make_plan(N, R);
    static constexpr int TPL = N / R;
    using Tw = TwSet<T, N, R, PL>;

    template <int s>
    __device__ __forceinline__ static void passes(cpx<T> (&v)[R], cpx<T>* lds, int t, const Tw& tw) {
        if constexpr (s < P.np) {
            constexpr int r = P.r[s];
            constexpr bool first = (s == 0);
            constexpr bool last = (s == P.np - 1);
            constexpr bool from_reg = first && (r == R);
            constexpr bool to_reg = last && (r == R);
            stockham_pass<T, N, R, s, INV, from_reg, to_reg, LS, WAVE>(v, lds, t, tw);
            passes<s + 1>(v, lds, t, tw);
        }
    }

    // Transform the line in place: v[m] = x[t + m*TPL] on entry, X[t + m*TPL] on exit, with the
    // thread's twiddles already loaded.  All threads of the workgroup (of the wave, with WAVE) must
    // call this together (it contains barriers).
    __device__ __forceinline__ static void run(cpx<T> (&v)[R], cpx<T>* lds, int t, const Tw& tw) {
        if constexpr (P.np == 0) {
            return;
        } else {
            constexpr bool first_reg = (P.r[0] == R);
            constexpr bool last_reg = (P.r[P.np - 1] == R);
            if constexpr (!first_reg) {
#pragma unroll
                for (int m = 0; m < R; ++m) lds[lds_idx(t + m * TPL) * LS] = v[m];
                line_sync<WAVE>();
            }
            passes<0>(v, lds, t, tw);
            if constexpr (!last_reg) {
#pragma unroll
                for (int m = 0; m < R; ++m) v[m] = lds[lds_idx(t + m * TPL) * LS];
            }
            // the next transform may write LDS that slower threads are still reading
            if constexpr (!(P.np == 1 && first_reg && last_reg)) line_sync<WAVE>();
        }
    }

    template <int s, int Q>
    __device__ __forceinline__ static void passes_n(cpx<T> (&v)[Q][R], cpx<T>* lds, int stride, int t,
                                                    const Tw& tw) {
        if constexpr (s < P.np) {
            constexpr int r = P.r[s];
            constexpr bool from_reg = (s == 0) && (r == R);
            constexpr bool to_reg = (s == P.np - 1) && (r == R);
            stockham_pass_n<T, N, R, s, INV, from_reg, to_reg, LS, Q, WAVE>(v, lds, stride, t, tw);
            passes_n<s + 1, Q>(v, lds, stride, t, tw);
        }
    }

    // Transform Q lines together (line l's LDS region at lds + l*stride); same contract as run.
    template <int Q>
    __device__ __forceinline__ static void run_n(cpx<T> (&v)[Q][R], cpx<T>* lds, int stride, int t,
                                                 const Tw& tw) {
        if constexpr (P.np == 0) {
            return;
        } else {
            constexpr bool first_reg = (P.r[0] == R);
            constexpr bool last_reg = (P.r[P.np - 1] == R);
            if constexpr (!first_reg) {
#pragma unroll
                for (int l = 0; l < Q; ++l)
#pragma unroll
                    for (int m = 0; m < R; ++m) lds[l * stride + lds_idx(t + m * TPL) * LS] = v[l][m];
                line_sync<WAVE>();
            }
            passes_n<0, Q>(v, lds, stride, t, tw);
            if constexpr (!last_reg) {
#pragma unroll
                for (int l = 0; l < Q; ++l)
#pragma unroll
                    for (int m = 0; m < R; ++m) v[l][m] = lds[l * stride + lds_idx(t + m * TPL) * LS];
            }
            if constexpr (!(P.np == 1 && first_reg && last_reg)) line_sync<WAVE>();
        }
    }

    // The same, loading the twiddles from the table first.
    __device__ __forceinline__ static void run(cpx<T> (&v)[R], cpx<T>* lds, int t, twptr<T> table) {
        Tw tw;
        tw.load(table, t);
        run(v, lds, t, tw);
    }
};

}  // namespace lbfft
