// Shared host/device data structures of the lbfft library: instance descriptors, field ids of
// the per-instance arena and the job descriptors that drive the line-FFT passes.
#pragma once
#include <stdint.h>

namespace lbfft {

// Field ids inside one instance's arena.  Every field is nx*ny words of the working precision,
// row-major [ny][nx].  Population blocks are 16 consecutive fields.
enum FieldId : int {
    F_A = 0,     // state f^n (and f^{n+1} after the step), 16 fields
    F_B = 16,    // midpoint state f^{n+1/2}, 16 fields (also the rhs output of lb_rhs)
    F_P = 32,    // per-population partial updates between the x and y passes, 16 fields
    RHO = 48, UX, UY, TT,                        // moments (Sec. 2.1)
    RX, RXX, TX, UXX, UYX,                       // x pass 1: d_x rho, d_xx rho, d_x T, d_x u_x, d_x u_y
    RY, RYY, TY, UXY, UYY,                       // y pass 1: d_y rho, d_yy rho, d_y T, d_y u_x, d_y u_y
    SXX, SXY, SYY, DIV, C0, QX, QY,              // stress S, div u, C without the grad(div u) and
                                                 // C_q terms, Q = q rho T grad T
    DSXX, DSXY, GDX, DQX,                        // x pass 2: d_x of S_xx, S_xy, div u, Q_x
    DYSXY, DYSYY, GDY, DYQY,                     // y pass 2: d_y of S_xy, S_yy, div u, Q_y
    BX, BY, CT,                                  // B and C + C_q of Eq. (2)
    SCR0, SCR1,                                  // scratch for lb_derivative
    NFIELDS
};

// Spectral multiplier kinds of a job.
enum MultKind : int8_t { M_NONE = 0, M_D = 1, M_DD = 2 };

// One job of a macroscopic line pass: out[o] = IFFT(mult[o] * FFT(in)) along the pass direction,
// o = 0, 1 (out[1] = -1 when unused).  flag_q: the job only runs for instances with q != 0.
struct JobDesc {
    int16_t in;
    int16_t out[2];
    int8_t mult[2];
    int8_t flag_q;
    int8_t pad;
};

// Per-instance descriptor, stored in device memory.
struct InstDesc {
    int32_t nx, ny;
    int64_t ncell;
    void* base;            // field arena (NFIELDS * ncell words)
    const void* kx;        // wavenumber k(m) of Eq. (3) along x, nx words
    const void* ky;        // along y, ny words
    const void* twx;       // forward twiddles exp(-2 pi i m / nx), nx complex words
    const void* twy;       // ny complex words
    double* red;           // conservation partial sums of this instance: RED_BLOCKS x 5 (float64)
    double* cons;          // last conservation result: mass, momentum x, y, energy, non-finite cells
    double* hist;          // conservation history ring buffer, hist_len x 4 (float64)
    unsigned long long* hist_count;   // history entries written so far
    int32_t red_blocks;    // blocks of the partial-sum kernel
    int32_t hist_len;      // ring-buffer length (0: no per-step history)
    double dx, dt, tau, K, H, zeta, q, b, a, bw;
    // Reference populations of the stored state: the arena holds f - fref (FP32 contexts: fref =
    // f^eq(rho_ref, 0, T_ref) of the instance's mean initial density and temperature, so that the
    // stored deviations are small and their rounding too; FP64 contexts: fref = 0, the plain f).
    // rho_ref and e_ref are the density and energy moments sum fref and sum fref (v^2 + eta^2);
    // rho_ref is exactly representable in float32.  T_ref = e_ref / (b rho_ref) is the reference's
    // temperature, bT_ref = b T_ref: the temperature field holds T - T_ref (FP64 contexts: both 0).
    double fref[16];
    double rho_ref, e_ref, T_ref, bT_ref;
};

// Line lengths of the transforms: 2^a and 3 * 2^a from 8 to 2048.  A grid takes them along x,
// and along y also 1 or 2 (quasi-1-D: the y-derivative vanishes).
inline constexpr bool line_ok(int n) {
    for (int p = 8; p <= 2048; p *= 2)
        if (n == p || (n == 3 * p / 2 && n <= 1536)) return true;
    return false;
}
inline constexpr bool grid_ok(int nx, int ny) { return line_ok(nx) && (line_ok(ny) || ny == 1 || ny == 2); }

// Launch-plan variants of the y passes (lb_kernels.h): the default plan, wide population y
// tiles, and the long-radix plan (YV_LONG: 16 elements per thread for 2^a lines, 24 for 3 * 2^a
// lines).
enum YVariant : int { YV_DEFAULT = 0, YV_WIDE = 1, YV_LONG = 2 };
// Launch-plan variants of the population x pass: the default plan, 4 elements per thread.
enum XVariant : int { XV_DEFAULT = 0, XV_R4 = 1 };

// Conservation partial-sum blocks per instance (each block strides over the grid).
constexpr int RED_BLOCKS = 512;

// Context-wide constants (velocity set and the inverse moment matrix), stored in device
// memory in both precisions.
template <typename T>
struct DvmConst {
    T vx[16], vy[16], w[16];   // w = v^2 + eta^2
    T eta2[16];                // eta^2
    T cinv[16][16];            // inverse of the 16x16 moment matrix of the seven kinetic moments
    int xorder[16];            // population order of the x pass: populations with v_x != 0 first,
                               // grouped so that a block of P consecutive entries shares its FFT load
    int rot[16];               // population whose velocity is v_i turned by -90 degrees, (v_y, -v_x)
};

// Stage description for the population passes.
struct StageArgs {
    int f_field;      // population block read (F_A or F_B)
    int base_field;   // base population block of the Runge-Kutta axpy (-1: zero base)
    int out_field;    // destination population block
    double alpha;     // stage fraction: 1/2 (first stage) or 1 (second stage)
    int use_dt;       // 1: the axpy coefficient is alpha * dt; 0: it is alpha (rhs diagnostic)
};

}  // namespace lbfft
