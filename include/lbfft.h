/*
 * lbfft.h -- C ABI of the MI355X (gfx950) D2V16 windowed-FFT thermal liquid-vapour lattice
 * Boltzmann library.
 *
 * The library evolves Eq. (1) of Gan, Xu, Zhang, Wang, Yu, Yang, "Lattice Boltzmann kinetic
 * modeling and simulation of thermal liquid-vapor system" (arXiv 1403.3746):
 *
 *   d f_i/dt + v_i . grad f_i = -(f_i - f_i^eq)/tau + I_i,        i = 1..16   (Eq. 1)
 *
 * on periodic nx x ny grids with the D2V16 velocity set and its seven-moment equilibrium
 * (Sec. 2.1), the van der Waals / interfacial forcing term I_i of Eq. (2) (Sec. 2.2), spatial
 * derivatives by the windowed FFT with the 16th-order wavenumber of Eq. (3) and the two-stage
 * Runge-Kutta scheme (Sec. 2.3).  Many independent simulations ("instances", possibly of
 * different sizes) are advanced together.
 *
 * Conventions shared by every entry point:
 *  - Fields are row-major [ny][nx] (x fastest), x_j = j*dx.  Population arrays are
 *    [16][ny][nx]; population index 0..15 is the paper's i = 1..16.  Ring 1 (0..3) lies on the
 *    axes and is the only ring with eta = eta0; ring 2 (4..7) on the diagonals; ring 3 (8..11)
 *    on the axes; ring 4 (12..15) on the diagonals.  Member k of a ring is member 0 rotated by
 *    k*90 degrees.
 *  - Host arrays are float64 and owned by the caller.  Device memory is one caller-owned
 *    workspace (e.g. a torch uint8 tensor) of at least lb_workspace_bytes(); the library never
 *    allocates device memory in lb_step.
 *  - All GPU work is enqueued on the caller's HIP stream.  lb_step is asynchronous; errors of
 *    asynchronous work are reported by the next synchronising call (lb_moments, lb_get_f,
 *    lb_conservation, lb_sync).
 *  - Functions return lb_status; on error lb_last_error() gives a thread-local message.  No
 *    C++ exception crosses this boundary.
 */
#ifndef LBFFT_H
#define LBFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx lb_ctx; /* opaque; created by lb_init, released by lb_free */

typedef enum {
    LB_OK = 0,
    LB_E_ARG = -1,       /* invalid argument (null pointer, bad index, non-physical parameter)  */
    LB_E_SIZE = -2,      /* unsupported grid size or workspace too small                         */
    LB_E_NOMEM = -3,     /* host allocation failed                                              */
    LB_E_HIP = -4,       /* a HIP runtime call failed                                           */
    LB_E_NONFINITE = -5, /* the state holds NaN or Inf                                          */
    LB_E_STATE = -6      /* call not valid in the context's current state                       */
} lb_status;

typedef enum { LB_FP64 = 0, LB_FP32 = 1 } lb_precision;

/* Per-instance parameters.  Sec. 2.2: B, C, C_q, Lambda (M = K + H T), zeta, q, the van der
 * Waals pressure P^w = rho T/(1 - vdw_b rho) - vdw_a rho^2 (the paper's 3 rho T/(3 - rho) -
 * 9/8 rho^2 is vdw_a = 9/8, vdw_b = 1/3); Sec. 2.1: b_dof = b; Sec. 2.3: dx = dy, dt. */
typedef struct {
    int32_t nx, ny;   /* nx in {8,12,16,24,...,1536,2048} (2^a or 3*2^a, 8..2048);
                         ny likewise, or ny in {1,2} (quasi-1D: the y-derivative vanishes)     */
    double dx;        /* grid spacing, dx = dy > 0                                             */
    double dt;        /* time step > 0                                                         */
    double tau;       /* relaxation time > 0                                                   */
    double K, H;      /* interfacial coefficients, M = K + H T                                 */
    double zeta;      /* bulk viscosity                                                        */
    double q;         /* heat-flux coefficient of C_q                                          */
    double b_dof;     /* total degrees of freedom b (> 0)                                      */
    double vdw_a, vdw_b; /* van der Waals a and b_w                                            */
    int32_t hist_len; /* steps of per-step float64 conservation history kept (ring buffer);
                         0 = none.  See lb_conservation_history.                                */
} lb_params;

/* D2V16 ring speeds (Sec. 2.1; the paper defers the values to Kataoka and Tsutahara).  Axis
 * rings: (+-va,0),(0,+-va) and (+-vc,0),(0,+-vc); diagonal rings: (+-vb,+-vb) and (+-vd,+-vd)
 * (vb, vd are the component magnitudes).  eta0 is eta_i of ring 1 (2.5 in the paper). */
typedef struct {
    double va, vb, vc, vd, eta0;
} lb_dvm;

/* Device workspace, in bytes, that lb_init needs for n_inst instances with parameters p[0..n_inst-1]
 * at precision prec.  Returns 0 if an argument is invalid. */
size_t lb_workspace_bytes(int n_inst, const lb_params* p, lb_precision prec);

/* Create a context for n_inst instances and set f_i = f_i^eq(rho0, u0, T0) in every cell.
 *  p[k]             parameters of instance k (copied).
 *  dvm              velocity set; NULL selects (va, vb, vc, vd, eta0) = (1, 0.5, 2, 1, 2.5).
 *  rho0[k] ... T0[k] host float64 arrays [ny][nx] of instance k (read during the call only).
 *  d_workspace      device memory of ws_bytes >= lb_workspace_bytes(n_inst, p, prec), 256-byte
 *                   aligned, owned by the caller and kept alive until lb_free.
 *  hip_stream       hipStream_t on which all work is enqueued (NULL = the null stream).
 * Errors: LB_E_ARG (null pointers, tau/dt/dx <= 0, rho0 <= 0, T0 <= 0 or 1 - vdw_b rho0 <= 0 in
 * any cell), LB_E_SIZE (grid size unsupported or workspace too small), LB_E_NOMEM, LB_E_HIP.
 * On error *out is NULL. */
lb_status lb_init(lb_ctx** out, int n_inst, const lb_params* p, const lb_dvm* dvm,
                  lb_precision prec, const double* const* rho0, const double* const* ux0,
                  const double* const* uy0, const double* const* T0, void* d_workspace,
                  size_t ws_bytes, void* hip_stream);

/* Enqueue n_steps >= 0 Runge-Kutta steps (Sec. 2.3) of every instance on the stream:
 *   f^{n+1/2} = f^n + dt/2 R(f^n),  f^{n+1} = f^n + dt R(f^{n+1/2}),
 *   R(f) = -v_i . grad f_i - (f_i - f_i^eq)/tau + I_i.
 * Steps are replayed from captured HIP graphs: one step per replay, and a graph of 16
 * consecutive steps (LBFFT_GRAPH_STEPS in the environment at lb_init: 1..64) used while at least
 * that many steps remain.  In both, the size classes of a batch are parallel branches that join
 * only at the end of the graph.  Asynchronous. */
lb_status lb_step(lb_ctx* ctx, int n_steps);

/* Block until all enqueued work is done; reports asynchronous HIP errors. */
lb_status lb_sync(lb_ctx* ctx);

/* Copy the moments (Sec. 2.1) rho = sum f, rho u = sum f v, rho (b T + u^2) = sum f (v^2 + eta^2)
 * of instance inst into host arrays [ny][nx] (any pointer may be NULL).  They are formed in
 * float64 from the stored state; an FP32 context stores them rounded to float32 (T as its
 * deviation from the instance's reference temperature, added back here).  Synchronises. */
lb_status lb_moments(lb_ctx* ctx, int inst, double* rho, double* ux, double* uy, double* T);

/* Grid integrals (sum over cells times dx^2), accumulated in float64 in both precisions:
 * out[0] mass, out[1..2] momentum, out[3] total energy e_T = sum f (v^2+eta^2)/2 - a rho^2 +
 * K |grad rho|^2/2 (Sec. 2.2; rho T - a rho^2 + K|grad rho|^2/2 + rho u^2/2 at b = 2), gradients
 * by the windowed FFT.  Synchronises.  Returns LB_E_NONFINITE if the state holds NaN/Inf. */
lb_status lb_conservation(lb_ctx* ctx, int inst, double out[4]);

/* Per-step conservation history (instances with hist_len > 0).  Every lb_step records, on the
 * GPU inside the captured step and in float64 in both precisions, the four integrals of
 * lb_conservation for the state at the start of the step (step index 0, 1, 2, ...; the first
 * stage's moments and d_x rho, d_y rho are reused, so nothing is recomputed).  This copies the
 * latest min(recorded, hist_len, max_entries) entries, oldest first, into out[n][4], sets *n_out
 * and *first_step (step index of out[0]).  Synchronises.  LB_E_STATE if hist_len = 0,
 * LB_E_NONFINITE if an entry is NaN/Inf. */
lb_status lb_conservation_history(lb_ctx* ctx, int inst, int max_entries, double* out, int* n_out,
                                  long long* first_step);

/* Copy the populations of instance inst to / from a host float64 array [16][ny][nx]
 * (checkpoint and restart).  In FP32 mode the device holds the deviation f - fref from a fixed
 * reference equilibrium (at rest, the mean initial density and temperature; float64), so that its
 * rounding scales with the deviation instead of f: lb_get_f returns fref + the float32 deviation,
 * lb_set_f stores the deviation rounded to float32.  Synchronise. */
lb_status lb_get_f(lb_ctx* ctx, int inst, double* f);
lb_status lb_set_f(lb_ctx* ctx, int inst, const double* f);

/* Replace the state of instance inst by the equilibrium of the given macroscopic fields:
 * f = f^eq(rho, u, T) of the seven kinetic moments (Sec. 2.1), as lb_init does for the initial
 * condition.  rho, ux, uy, T: host float64 arrays [ny][nx], read only.  Used to restart a run
 * at another temperature (the coexistence runs of Sec. 3.1 lower T once the phases have
 * settled).  LB_E_ARG if a pointer is NULL or a cell has rho <= 0, T <= 0, 1 - vdw_b rho <= 0
 * or a non-finite value (the state is then unchanged).  Synchronises. */
lb_status lb_set_moments(lb_ctx* ctx, int inst, const double* rho, const double* ux,
                         const double* uy, const double* T);

/* Diagnostics on the current state of instance inst, each computed with the same kernels as
 * lb_step and copied to host arrays [ny][nx]; they synchronise and leave the state unchanged.
 *  lb_force_coefficients: B_x, B_y and C + C_q of Eq. (2) from the moments of the current f.
 *  lb_rhs: R(f) of Eq. (1) for all 16 populations, [16][ny][nx].                          */
lb_status lb_force_coefficients(lb_ctx* ctx, int inst, double* Bx, double* By, double* C);
lb_status lb_rhs(lb_ctx* ctx, int inst, double* R);

/* Windowed-FFT derivative (Sec. 2.3, Eq. 3) of a host field g[ny][nx] of instance inst's grid:
 * axis 0 = x, 1 = y; order 1 = D, 2 = D D.  out[ny][nx] on the host.  Uses the library's
 * line-FFT kernels through the instance's scratch fields; synchronises. */
lb_status lb_derivative(lb_ctx* ctx, int inst, int axis, int order, const double* g, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the windowed-FFT derivative of lb_derivative without a
 * context or workspace.  d_g and d_out are float64 device arrays [ny][nx] (caller-owned; d_out may
 * not alias d_g); the line pass runs in precision prec on the stream hip_stream of the current
 * device.  Every buffer the kernels need (descriptor, tables, staging fields) lives in one static
 * device array of the library that each GPU it runs on holds until the process ends; nothing is
 * allocated.  Calls on one GPU share that array, so calls that overlap on one GPU (several streams
 * or threads) race; it keeps the last call's contents, and each call writes everything it reads.
 * Asynchronous.  Errors: LB_E_ARG (null pointer, dx <= 0, axis/order/prec invalid), LB_E_SIZE (grid
 * not supported as in lb_params, or nx * ny > LB_NOALLOC_MAX_CELLS), LB_E_HIP. */
#define LB_NOALLOC_MAX_CELLS (1 << 20)
lb_status lb_derivative_noalloc(int nx, int ny, double dx, lb_precision prec, int axis, int order,
                                const double* d_g, double* d_out, void* hip_stream);

/* Pass kinds of one Runge-Kutta stage, in launch order (index into lb_step_timed's output).
 * The x and y passes of each macroscopic pair are independent and run concurrently in the
 * captured step. */
enum {
    LB_PASS_MOMENTS = 0,   /* moments of f (Sec. 2.1)                                  */
    LB_PASS_MACRO_X1 = 1,  /* x derivatives of rho, T, u (Eq. 3)                       */
    LB_PASS_MACRO_Y1 = 2,  /* y derivatives of rho, T, u                               */
    LB_PASS_STRESS = 3,    /* stress S, div u and most of C (Eq. 2)                    */
    LB_PASS_MACRO_X2 = 4,  /* x derivatives of S, div u (and q rho T grad T)           */
    LB_PASS_MACRO_Y2 = 5,  /* y derivatives of S, div u (and q rho T grad T)           */
    LB_PASS_FINALIZE = 6,  /* B and C + C_q (Eq. 2)                                    */
    LB_PASS_POP_X = 7,     /* population x pass: equilibrium, forcing, BGK, RK axpy    */
    LB_PASS_POP_Y = 8,     /* population y pass                                        */
    LB_NPASS = 9
};

/* Enqueue n_steps Runge-Kutta steps exactly as lb_step does but with direct kernel launches, each
 * timestamping its own start and end into a HIP event pair (hipExtLaunchKernelGGL); waits
 * for completion and writes the mean duration in milliseconds of one launch of each pass kind
 * (over both stages of all steps and all size classes) to ms[LB_NPASS].  Advances the state like
 * lb_step.  For measurement only. */
lb_status lb_step_timed(lb_ctx* ctx, int n_steps, double ms[LB_NPASS]);

/* Launch plan chosen for instance inst's size class at lb_init (measured on the class's data
 * unless the environment sets LBFFT_TUNE=0; LBFFT_PPB, LBFFT_YPOP, LBFFT_YMAC and LBFFT_XPOP fix a
 * choice):
 *  out[0] = populations per block of the x population pass (1, 2 or 4),
 *  out[1] = size classes in the context,
 *  out[2] = plan of the population y pass: 0 default, 1 wide tiles (blocks of up to 1024
 *           threads, twice the column pairs of long columns), 2 long radix (16 elements per
 *           thread for 1024 and 2048 points, 24 for 96, 192 and 384 points: fewer threads per
 *           line, more column pairs per 512-thread block, fewer passes through LDS),
 *  out[3] = plan of the macroscopic y (or fused x + y) pass: 0 default, 2 long radix,
 *  out[4] = plan of the population x pass: 0 default, 1 four elements per thread (twice the
 *           threads per line).
 * The variants exist in FP32, the wide tiles for y lines limited by the default 512-thread block,
 * the long radix for lines of 96, 192, 384, 1024 and 2048 points, four elements per thread for x
 * lines of 128, 256 and 512 points; elsewhere the entry is 0.
 * n = length of out (>= 2; entries beyond min(n, 5) are not written). */
lb_status lb_plan_info(lb_ctx* ctx, int inst, int* out, int n);

/* Release the context (not the caller's workspace).  NULL is ignored. */
void lb_free(lb_ctx* ctx);

/* Thread-local message describing the last error of this thread ("" if none). */
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBFFT_H */
