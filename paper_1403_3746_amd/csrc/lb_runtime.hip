// Host runtime of the lbfft C ABI: argument checks, workspace carving, float64 tables and the
// inverse moment matrix, stage sequencing, HIP graph capture of one Runge-Kutta step, and the
// synchronising diagnostics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbfft.h"
#include "lb_launch.h"
#include "lb_types.h"

#ifndef LB_GRAPH_STEPS
#define LB_GRAPH_STEPS 16  // steps per replay of the multi-step graph
#endif

using namespace lbfft;

namespace {

thread_local std::string g_err;

lb_status fail(lb_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define LB_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LB_E_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                                 \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// The kernels address an instance's field arena through one buffer descriptor with 32-bit byte
// offsets, so the largest arena (2048 x 2048 cells in FP64) must stay below 2^32 bytes.
static_assert((unsigned long long)NFIELDS * 2048 * 2048 * 8 < (1ull << 32),
              "field arena of the largest grid exceeds 32-bit buffer offsets");

size_t word_bytes(lb_precision p) { return p == LB_FP64 ? 8 : 4; }

// Workspace layout.  Header: InstDesc[n], DvmConst<double>, DvmConst<float>, job tables,
// population list, instance index lists, reduction partials.  Then per instance: tables
// (kx, ky, twx, twy) and the field arena.
struct Layout {
    size_t insts, dvm64, dvm32, jobs, pops, ilist, header;
    std::vector<size_t> tables, red, arena;
    size_t total;
};

constexpr int MAX_JOBS = 32;

Layout make_layout(int n, const lb_params* p, lb_precision prec) {
    Layout L;
    size_t off = 0;
    L.insts = off; off = align_up(off + sizeof(InstDesc) * n);
    L.dvm64 = off; off = align_up(off + sizeof(DvmConst<double>));
    L.dvm32 = off; off = align_up(off + sizeof(DvmConst<float>));
    L.jobs = off;  off = align_up(off + sizeof(JobDesc) * MAX_JOBS);
    L.pops = off;  off = align_up(off + sizeof(int) * 16);
    L.ilist = off; off = align_up(off + sizeof(int) * 2 * n);
    L.header = off;
    const size_t w = word_bytes(prec);
    for (int k = 0; k < n; ++k) {
        const size_t nc = (size_t)p[k].nx * p[k].ny;
        L.tables.push_back(off);
        off = align_up(off + w * (p[k].nx + p[k].ny) + 2 * w * (p[k].nx + p[k].ny) + 4 * ALIGN);
        // conservation: partials, last result (8 doubles), history counter, history ring
        L.red.push_back(off);
        off = align_up(off + sizeof(double) * (5 * RED_BLOCKS + 8 + 1 + 4 * (size_t)p[k].hist_len));
        L.arena.push_back(off);
        off = align_up(off + w * nc * NFIELDS);
    }
    L.total = off;
    return L;
}

// Gauss-Jordan inverse with partial pivoting (float64).  Returns false if singular.
bool invert16(const double A[16][16], double X[16][16]) {
    double M[16][32];
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 32; ++j) M[i][j] = j < 16 ? A[i][j] : (j - 16 == i ? 1.0 : 0.0);
    for (int c = 0; c < 16; ++c) {
        int piv = c;
        for (int r = c + 1; r < 16; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (std::fabs(M[piv][c]) < 1e-300) return false;
        if (piv != c)
            for (int j = 0; j < 32; ++j) std::swap(M[c][j], M[piv][j]);
        const double d = M[c][c];
        for (int j = 0; j < 32; ++j) M[c][j] /= d;
        for (int r = 0; r < 16; ++r) {
            if (r == c) continue;
            const double f = M[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 32; ++j) M[r][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j) X[i][j] = M[i][16 + j];
    return true;
}

// D2V16 velocities (population order of the header) and the inverse of the moment matrix whose
// rows are the seven kinetic moments [1, vx, vy, w, vx^2, vx vy, vy^2, w vx, w vy, vx^3,
// vx^2 vy, vx vy^2, vy^3, w vx^2, w vx vy, w vy^2], w = v^2 + eta^2 (Sec. 2.1, 2.2).
bool build_dvm(const lb_dvm& d, DvmConst<double>& D) {
    const double ax[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    const double dg[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    const double speed[4] = {d.va, d.vb, d.vc, d.vd};
    for (int ring = 0; ring < 4; ++ring)
        for (int k = 0; k < 4; ++k) {
            const int i = ring * 4 + k;
            const double(*u)[2] = (ring % 2 == 0) ? ax : dg;
            D.vx[i] = speed[ring] * u[k][0];
            D.vy[i] = speed[ring] * u[k][1];
            const double eta = ring == 0 ? d.eta0 : 0.0;
            D.w[i] = D.vx[i] * D.vx[i] + D.vy[i] * D.vy[i] + eta * eta;
            D.eta2[i] = eta * eta;
        }
    double A[16][16];
    for (int i = 0; i < 16; ++i) {
        const double x = D.vx[i], y = D.vy[i], w = D.w[i];
        const double row[16] = {1, x, y, w, x * x, x * y, y * y, w * x, w * y,
                                x * x * x, x * x * y, x * y * y, y * y * y,
                                w * x * x, w * x * y, w * y * y};
        for (int j = 0; j < 16; ++j) A[j][i] = row[j];
    }
    return invert16(A, D.cinv);
}

}  // namespace

// The thread's error message, set by the other host unit of the library.
int lbfft::set_error(int status, const char* msg) {
    g_err = msg;
    return status;
}

struct lb_ctx {
    int n = 0;
    lb_precision prec = LB_FP64;
    std::vector<lb_params> p;
    lb_dvm dvm{};
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    Layout lay;
    std::vector<InstDesc> hinst;
    // host copies uploaded at init (kept alive for the asynchronous copies)
    DvmConst<double> dvm64{};
    DvmConst<float> dvm32{};
    std::vector<JobDesc> jobs;
    std::vector<int> ilist_h;
    int pops_h[16] = {0};
    int npops = 0;
    // job table slices
    int j_x1 = 0, n_x1 = 0, j_y1 = 0, n_y1 = 0, j_x2 = 0, n_x2 = 0, j_y2 = 0, n_y2 = 0;
    int j_dx = 0, j_dxx = 0, j_dy = 0, j_dyy = 0;   // single-job tables of lb_derivative
    // size classes: instances sharing (nx, ny), as a slice [start, start+count) of ilist
    struct Class {
        int nx, ny, start, count;
        int ppb = 1;   // tuned populations per block of the x population pass
        int ypop_var = 0, ymac_var = 0;   // tuned y-pass plan variants (YVariant) where they exist
        int xpop_var = 0;                 // tuned x population pass plan (XVariant) where it exists
        bool hist = false;   // some instance keeps a per-step conservation history
    };
    std::vector<Class> classes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // a graph of graph_steps consecutive steps (fewer replays while enough steps remain)
    hipGraph_t graph_k = nullptr;
    hipGraphExec_t exec_k = nullptr;
    int graph_steps = LB_GRAPH_STEPS;
    bool use_graph = true;
    int ppb_override = 0;   // populations per x-pass block forced by LBFFT_PPB (1, 2 or 4), else tuned
    int ypop_override = -1;   // population y pass variant forced by LBFFT_YPOP (0, 1, 2), else tuned
    int ymac_override = -1;   // macroscopic y pass variant forced by LBFFT_YMAC (0, 2), else tuned
    int xpop_override = -1;   // population x pass variant forced by LBFFT_XPOP (0, 1), else tuned
    bool fuse_xy = true;    // square grids: x and y macroscopic passes in one launch (LBFFT_FUSE_XY=0: off)

    template <typename Q>
    Q* dev(size_t off) const { return reinterpret_cast<Q*>(ws + off); }
    const InstDesc* d_insts() const { return dev<InstDesc>(lay.insts); }
    const JobDesc* d_jobs(int j) const { return dev<JobDesc>(lay.jobs) + j; }
    const int* d_ilist(int k) const { return dev<int>(lay.ilist) + k; }
    size_t wbytes() const { return word_bytes(prec); }
};

namespace {

JobDesc job(int in, int out0, int m0, int out1 = -1, int m1 = M_NONE, int flag_q = 0) {
    JobDesc j;
    std::memset(&j, 0, sizeof(j));
    j.in = (int16_t)in;
    j.out[0] = (int16_t)out0;
    j.out[1] = (int16_t)out1;
    j.mult[0] = (int8_t)m0;
    j.mult[1] = (int8_t)m1;
    j.flag_q = (int8_t)flag_q;
    return j;
}

// Job tables of the four macroscopic line passes of one stage.  Every job is one input; the
// first and second derivatives of rho share a job (one forward transform, two inverse).
void build_jobs(lb_ctx& c) {
    auto& J = c.jobs;
    J.clear();
    // X1 / Y1: first (and for rho second) derivatives of the moments
    c.j_x1 = (int)J.size();
    J.push_back(job(RHO, RX, M_D, RXX, M_DD));
    J.push_back(job(TT, TX, M_D));
    J.push_back(job(UX, UXX, M_D));
    J.push_back(job(UY, UYX, M_D));
    c.n_x1 = (int)J.size() - c.j_x1;
    c.j_y1 = (int)J.size();
    J.push_back(job(RHO, RY, M_D, RYY, M_DD));
    J.push_back(job(TT, TY, M_D));
    J.push_back(job(UX, UXY, M_D));
    J.push_back(job(UY, UYY, M_D));
    c.n_y1 = (int)J.size() - c.j_y1;
    // X2 / Y2: derivatives of the stress, of div u and of Q = q rho T grad T (q != 0 only)
    c.j_x2 = (int)J.size();
    J.push_back(job(SXX, DSXX, M_D));
    J.push_back(job(SXY, DSXY, M_D));
    J.push_back(job(DIV, GDX, M_D));
    J.push_back(job(QX, DQX, M_D, -1, M_NONE, 1));
    c.n_x2 = (int)J.size() - c.j_x2;
    c.j_y2 = (int)J.size();
    J.push_back(job(SXY, DYSXY, M_D));
    J.push_back(job(SYY, DYSYY, M_D));
    J.push_back(job(DIV, GDY, M_D));
    J.push_back(job(QY, DYQY, M_D, -1, M_NONE, 1));
    c.n_y2 = (int)J.size() - c.j_y2;
    // lb_derivative: SCR0 -> SCR1
    c.j_dx = (int)J.size();
    J.push_back(job(SCR0, SCR1, M_D));
    c.j_dxx = (int)J.size();
    J.push_back(job(SCR0, SCR1, M_DD));
    c.j_dy = c.j_dx;
    c.j_dyy = c.j_dxx;
}

void apply_plan(const lb_ctx& c, const lb_ctx::Class& k, LaunchSet& L) {
    L.ppb = c.ppb_override ? c.ppb_override : k.ppb;
    L.ypop_var = c.ypop_override >= 0 ? c.ypop_override : k.ypop_var;
    L.ymac_var = c.ymac_override >= 0 ? c.ymac_override : k.ymac_var;
    L.xpop_var = c.xpop_override >= 0 ? c.xpop_override : k.xpop_var;
}

LaunchSet set_of(const lb_ctx& c, const lb_ctx::Class& k) {
    LaunchSet L{c.d_insts(), c.d_ilist(k.start), k.count, k.nx, k.ny, c.stream};
    apply_plan(c, k, L);
    return L;
}

LaunchSet set_one(const lb_ctx& c, int inst, hipStream_t s) {
    // the second half of ilist is the identity map
    LaunchSet L{c.d_insts(), c.d_ilist(c.n + inst), 1, c.p[inst].nx, c.p[inst].ny, s};
    for (const auto& k : c.classes)
        if (k.nx == L.nx && k.ny == L.ny) apply_plan(c, k, L);
    return L;
}

// Bit set (1 << YVariant) of the y-pass plan variants the class's y lines have.
int class_variants(const lb_ctx& c, int ny) {
    return c.prec == LB_FP64 ? variants_y_f64(ny) : variants_y_f32(ny);
}
// Bit set (1 << XVariant) of the x population pass plans the class's x lines have.
int class_variants_x(const lb_ctx& c, int nx) {
    return c.prec == LB_FP64 ? variants_x_f64(nx) : variants_x_f32(nx);
}

// The x and y macroscopic passes of a square grid run as one fused launch, issued in the x slot.
bool fused_xy(const lb_ctx& c, const LaunchSet& L) { return c.fuse_xy && L.nx == L.ny; }

hipError_t macro_xy(const lb_ctx& c, const LaunchSet& L, int jx, int njx, int jy, int njy) {
    if (c.prec == LB_FP64) return macro_xy_f64(L, c.d_jobs(jx), njx, c.d_jobs(jy), njy);
    return macro_xy_f32(L, c.d_jobs(jx), njx, c.d_jobs(jy), njy);
}

hipError_t macro(const lb_ctx& c, const LaunchSet& L, int dir, int j0, int nj) {
    const JobDesc* jt = c.d_jobs(j0);
    if (c.prec == LB_FP64) return dir == 0 ? macro_x_f64(L, jt, nj) : macro_y_f64(L, jt, nj);
    return dir == 0 ? macro_x_f32(L, jt, nj) : macro_y_f32(L, jt, nj);
}

hipError_t moments(const lb_ctx& c, const LaunchSet& L, int f_field) {
    const DvmConst<double>* d64 = c.dev<DvmConst<double>>(c.lay.dvm64);
    return c.prec == LB_FP64 ? launch_moments<double>(L, d64, f_field) : launch_moments<float>(L, d64, f_field);
}

hipError_t stress(const lb_ctx& c, const LaunchSet& L) {
    return c.prec == LB_FP64 ? launch_stress<double>(L) : launch_stress<float>(L);
}

hipError_t finalize(const lb_ctx& c, const LaunchSet& L) {
    return c.prec == LB_FP64 ? launch_finalize<double>(L) : launch_finalize<float>(L);
}

// Optional timing hook: supplies a start/stop event pair for every launch of a pass.
struct PassHook {
    virtual bool events(int pass, hipEvent_t* start, hipEvent_t* stop) = 0;
    virtual ~PassHook() = default;
};

hipError_t pop_x(const lb_ctx& c, const LaunchSet& L, StageArgs st) {
    const int* pops = c.dev<int>(c.lay.pops);
    const int ppb = L.ppb;
    const DvmConst<double>* d64 = c.dev<DvmConst<double>>(c.lay.dvm64);
    if (c.prec == LB_FP64) return pop_x_f64(L, d64, d64, pops, ppb, st);
    return pop_x_f32(L, c.dev<DvmConst<float>>(c.lay.dvm32), d64, pops, ppb, st);
}

hipError_t pop_y(const lb_ctx& c, const LaunchSet& L, StageArgs st) {
    const int* pops = c.dev<int>(c.lay.pops);
    const DvmConst<double>* d64 = c.dev<DvmConst<double>>(c.lay.dvm64);
    if (c.prec == LB_FP64) return pop_y_f64(L, d64, d64, pops, c.npops, st);
    return pop_y_f32(L, c.dev<DvmConst<float>>(c.lay.dvm32), d64, pops, c.npops, st);
}

// Launch pass `kind` of one stage for the instances of L.
hipError_t run_pass(const lb_ctx& c, const LaunchSet& L, int kind, StageArgs st) {
    switch (kind) {
        case LB_PASS_MOMENTS: return moments(c, L, st.f_field);
        case LB_PASS_MACRO_X1:
            if (fused_xy(c, L)) return macro_xy(c, L, c.j_x1, c.n_x1, c.j_y1, c.n_y1);
            return macro(c, L, 0, c.j_x1, c.n_x1);
        case LB_PASS_MACRO_Y1:
            if (fused_xy(c, L)) return hipSuccess;   // done by the fused launch in the x slot
            return macro(c, L, 1, c.j_y1, c.n_y1);
        case LB_PASS_STRESS: return stress(c, L);
        case LB_PASS_MACRO_X2:
            if (fused_xy(c, L)) return macro_xy(c, L, c.j_x2, c.n_x2, c.j_y2, c.n_y2);
            return macro(c, L, 0, c.j_x2, c.n_x2);
        case LB_PASS_MACRO_Y2:
            if (fused_xy(c, L)) return hipSuccess;
            return macro(c, L, 1, c.j_y2, c.n_y2);
        case LB_PASS_FINALIZE: return finalize(c, L);
        case LB_PASS_POP_X: return pop_x(c, L, st);
        case LB_PASS_POP_Y: return pop_y(c, L, st);
    }
    return hipErrorInvalidValue;
}

// Moments and the force coefficients B, C (+ C_q) of the population block f_field.
hipError_t force_passes(const lb_ctx& c, const LaunchSet& L, int f_field) {
    StageArgs st{f_field, -1, -1, 0.0, 0};
    for (int k = LB_PASS_MOMENTS; k <= LB_PASS_FINALIZE; ++k) {
        hipError_t e = run_pass(c, L, k, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t pop_passes(const lb_ctx& c, const LaunchSet& L, StageArgs st) {
    hipError_t e = pop_x(c, L, st);
    if (e != hipSuccess) return e;
    return pop_y(c, L, st);
}

hipError_t launch_pass(const lb_ctx& c, const lb_ctx::Class& cl, hipStream_t s, int k,
                       StageArgs st, PassHook* hook) {
    LaunchSet L = set_of(c, cl);
    L.stream = s;
    // a y pass fused into its x launch launches nothing (and takes no timing events)
    if ((k == LB_PASS_MACRO_Y1 || k == LB_PASS_MACRO_Y2) && fused_xy(c, L)) return hipSuccess;
    if (hook && !hook->events(k, &L.ev_start, &L.ev_stop)) return hipErrorInvalidValue;
    return run_pass(c, L, k, st);
}

// One Runge-Kutta stage of the instances of one size class on stream s:
//   moments -> X1 -> Y1 -> stress -> X2 -> Y2 -> finalize -> pop x -> pop y.
// (X1/Y1 and X2/Y2 are independent: one fused launch each on square grids, else in order.)
hipError_t enqueue_class_stage(const lb_ctx& c, const lb_ctx::Class& cl, hipStream_t s,
                               StageArgs st, PassHook* hook) {
    for (int k = 0; k < LB_NPASS; ++k) {
        hipError_t e = launch_pass(c, cl, s, k, st, hook);
        if (e != hipSuccess) return e;
        // per-step FP64 conservation of the state f^n: its moments and d_x rho, d_y rho exist
        // after the first stage's y derivative pass
        if (k == LB_PASS_MACRO_Y1 && cl.hist && st.f_field == F_A && st.use_dt) {
            LaunchSet L = set_of(c, cl);
            L.stream = s;
            e = c.prec == LB_FP64 ? launch_conserve<double>(L, 1) : launch_conserve<float>(L, 1);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// f^{n+1/2} = f^n + dt/2 R(f^n) into F_B;  f^{n+1} = f^n + dt R(f^{n+1/2}) into F_A, for one
// size class.
hipError_t enqueue_class_step(const lb_ctx& c, const lb_ctx::Class& cl, hipStream_t s,
                              PassHook* hook = nullptr) {
    StageArgs s1{F_A, F_A, F_B, 0.5, 1};
    StageArgs s2{F_B, F_A, F_A, 1.0, 1};
    hipError_t e = enqueue_class_stage(c, cl, s, s1, hook);
    if (e != hipSuccess) return e;
    return enqueue_class_stage(c, cl, s, s2, hook);
}

// One step of every instance on stream s, size classes one after the other, all on s.
hipError_t enqueue_step(const lb_ctx& c, hipStream_t s, PassHook* hook = nullptr) {
    for (const auto& cl : c.classes) {
        hipError_t e = enqueue_class_step(c, cl, s, hook);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// `nsteps` steps of every instance captured as one graph.  With several size classes the capture
// stream forks once to one stream per class (default priority); each branch runs its class's steps
// in order and the branches join once at the end, so classes never wait for each other between
// steps and every fork/join event is recorded exactly once in the capture.
hipError_t capture_steps(const lb_ctx& c, hipStream_t cs, std::vector<hipStream_t>& br,
                         std::vector<hipEvent_t>& ev, int nsteps) {
    if (c.classes.size() <= 1) {
        for (int s = 0; s < nsteps; ++s) {
            hipError_t e = enqueue_step(c, cs);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t e = hipEventRecord(ev[0], cs);
    for (size_t k = 0; e == hipSuccess && k < c.classes.size(); ++k) {
        e = hipStreamWaitEvent(br[k], ev[0], 0);
        for (int s = 0; e == hipSuccess && s < nsteps; ++s) e = enqueue_class_step(c, c.classes[k], br[k]);
        if (e == hipSuccess) e = hipEventRecord(ev[k + 1], br[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev[k + 1], 0);
    }
    return e;
}

// Capture `nsteps` steps on private streams with fresh fork/join events, instantiate and upload the
// graph (so that its first replay costs no more than later ones).
hipError_t build_graph(const lb_ctx& c, int nsteps, hipGraph_t* graph, hipGraphExec_t* exec) {
    const size_t nb = c.classes.size();
    std::vector<hipStream_t> br(nb, nullptr);
    std::vector<hipEvent_t> ev(nb + 1, nullptr);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (size_t k = 0; e == hipSuccess && k < nb; ++k) e = hipStreamCreateWithFlags(&br[k], hipStreamNonBlocking);
    for (size_t k = 0; e == hipSuccess && k <= nb; ++k) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = capture_steps(c, cs, br, ev, nsteps);
            e = hipStreamEndCapture(cs, graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphUpload(*exec, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    }
    for (auto x : ev)
        if (x) (void)hipEventDestroy(x);
    for (auto x : br)
        if (x) (void)hipStreamDestroy(x);
    if (cs) (void)hipStreamDestroy(cs);
    return e;
}

// Best-of-rounds timing of launch candidates on the stream: every round launches each candidate
// once (interleaved, so clock and cache drift touch all of them); the first round only warms up.
// Returns the index of the fastest candidate in *best.
template <typename Launch>
hipError_t time_candidates(const lb_ctx& c, int ncand, Launch launch, float* best_ms, int* best) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    for (int k = 0; k < ncand; ++k) best_ms[k] = 1e30f;
    for (int round = 0; round < 7 && e == hipSuccess; ++round)
        for (int k = 0; k < ncand && e == hipSuccess; ++k) {
            e = hipEventRecord(a, c.stream);
            if (e == hipSuccess) e = launch(k);
            if (e == hipSuccess) e = hipEventRecord(b, c.stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
            if (e == hipSuccess && round > 0 && t < best_ms[k]) best_ms[k] = t;
        }
    *best = 0;
    for (int k = 1; k < ncand; ++k)
        if (best_ms[k] < best_ms[*best]) *best = k;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
}

// Launch plan of one size class, measured on the class's own data with arguments that leave the
// state untouched: the x population pass in both stages' forms (populations per block 1, 2, 4 and,
// where it exists, the 4-elements-per-thread plan, chosen together), then, with stage-1 arguments --
// where the class's y lines have them -- the plan variants of the population y pass (default,
// wide tiles, long radix) and of the macroscopic y or fused x + y pass (default, long radix).  Fixed
// choices (LBFFT_PPB, LBFFT_YPOP, LBFFT_YMAC, LBFFT_XPOP) are not re-tuned.
hipError_t tune_class(lb_ctx& c, lb_ctx::Class& cl) {
    const bool verbose = std::getenv("LBFFT_VERBOSE") != nullptr;
    LaunchSet L = set_of(c, cl);
    hipError_t e = force_passes(c, L, F_A);
    if (e != hipSuccess) return e;
    const StageArgs st{F_A, F_A, F_B, 0.5, 1};
    float ms[6];
    int best = 0;
    // the x population pass: populations per block (1, 2, 4) and, where the class's x lines have
    // it, the 4-elements-per-thread plan, chosen together
    const bool x_r4 = (class_variants_x(c, cl.nx) & (1 << XV_R4)) != 0;
    int pc[6], vc[6], nxc = 0;
    for (int v : {XV_DEFAULT, XV_R4}) {
        if ((v == XV_R4 && !x_r4) || (c.xpop_override >= 0 && v != c.xpop_override)) continue;
        for (int p : {1, 2, 4}) {
            if (c.ppb_override && p != c.ppb_override) continue;
            pc[nxc] = p;
            vc[nxc++] = v;
        }
    }
    if (nxc > 1) {
        // both stages' forms: the first folds the base into the transform, the second reads it per
        // cell (here from F_B, written in place, so the state in F_A stays untouched)
        const StageArgs st2{F_A, F_B, F_B, 1.0, 1};
        e = time_candidates(c, nxc, [&](int k) {
                L.ppb = pc[k];
                L.xpop_var = vc[k];
                hipError_t r = pop_x(c, L, st);
                return r == hipSuccess ? pop_x(c, L, st2) : r;
            }, ms, &best);
        if (e != hipSuccess) return e;
        cl.ppb = pc[best];
        cl.xpop_var = vc[best];
        if (verbose)
            for (int k = 0; k < nxc; ++k)
                std::fprintf(stderr, "lbfft tune: class %dx%d x%d  pops/block %d  x variant %d  %.4f ms\n",
                             cl.nx, cl.ny, cl.count, pc[k], vc[k], ms[k]);
    }
    L = set_of(c, cl);
    if ((e = pop_x(c, L, st)) != hipSuccess) return e;   // the partial sums the y pass adds to
    const int have = class_variants(c, cl.ny);
    int cand[3] = {YV_DEFAULT, 0, 0}, nc = 1;
    for (int v : {YV_WIDE, YV_LONG})
        if (have & (1 << v)) cand[nc++] = v;
    if (c.ypop_override < 0 && nc > 1) {
        e = time_candidates(c, nc, [&](int k) { L.ypop_var = cand[k]; return pop_y(c, L, st); }, ms, &best);
        if (e != hipSuccess) return e;
        cl.ypop_var = cand[best];
        if (verbose)
            for (int k = 0; k < nc; ++k)
                std::fprintf(stderr, "lbfft tune: class %dx%d  pop y variant %d  %.4f ms\n", cl.nx, cl.ny,
                             cand[k], ms[k]);
    }
    L.ypop_var = cl.ypop_var;
    if (c.ymac_override < 0 && (have & (1 << YV_LONG))) {
        const int mc[2] = {YV_DEFAULT, YV_LONG};
        const int kind = fused_xy(c, L) ? LB_PASS_MACRO_X1 : LB_PASS_MACRO_Y1;
        e = time_candidates(c, 2, [&](int k) { L.ymac_var = mc[k]; return run_pass(c, L, kind, st); }, ms, &best);
        if (e != hipSuccess) return e;
        cl.ymac_var = mc[best];
        if (verbose)
            for (int k = 0; k < 2; ++k)
                std::fprintf(stderr, "lbfft tune: class %dx%d  macro y variant %d  %.4f ms\n", cl.nx, cl.ny,
                             mc[k], ms[k]);
    }
    return hipSuccess;
}

lb_status check_inst(const lb_ctx* c, int inst) {
    if (!c) return fail(LB_E_ARG, "null context");
    if (inst < 0 || inst >= c->n) return fail(LB_E_ARG, "instance %d out of range [0,%d)", inst, c->n);
    return LB_OK;
}

// Reference populations of an FP32 instance (the arena stores f - fref): the equilibrium at rest of
// the mean initial temperature and of the mean initial density rounded to float32 (so that the
// moment kernel adds an exact rho_ref), in float64 (Sec. 2.1, seven kinetic moments at u = 0); and
// the reference's own temperature, from which the temperature field is stored as a deviation.
void set_reference(const DvmConst<double>& D, const lb_params& q, const double* rho0, const double* T0,
                   InstDesc& I) {
    const int64_t nc = (int64_t)q.nx * q.ny;
    double sr = 0.0, st = 0.0;
    for (int64_t e = 0; e < nc; ++e) {
        sr += rho0[e];
        st += T0[e];
    }
    const double rho = (double)(float)(sr / nc), T = st / nc, b = q.b_dof;
    // Maxwellian moments per unit density at u = 0 in the row order of the moment matrix
    const double h2 = (b + 2.0) * T;
    const double m[16] = {1, 0, 0, b * T, T, 0, T, 0, 0, 0, 0, 0, 0, h2 * T, 0, h2 * T};
    I.rho_ref = rho;
    I.e_ref = 0.0;
    for (int i = 0; i < 16; ++i) {
        double s = 0.0;
        for (int j = 0; j < 16; ++j) s += D.cinv[i][j] * m[j];
        I.fref[i] = rho * s;
        I.e_ref += I.fref[i] * D.w[i];
    }
    I.bT_ref = I.e_ref / rho;
    I.T_ref = I.bT_ref / b;
}

// Copy field `fid` of instance inst (nc words of the working precision) to host float64.
lb_status field_to_host(lb_ctx* c, int inst, int fid, double* dst, int64_t nfields = 1) {
    const InstDesc& I = c->hinst[inst];
    const int64_t n = I.ncell * nfields;
    unsigned char* src = reinterpret_cast<unsigned char*>(I.base) + (size_t)fid * I.ncell * c->wbytes();
    if (c->prec == LB_FP64) {
        LB_HIP(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, c->stream));
        LB_HIP(hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(n);
        LB_HIP(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, c->stream));
        LB_HIP(hipStreamSynchronize(c->stream));
        for (int64_t k = 0; k < n; ++k) dst[k] = tmp[k];
    }
    return LB_OK;
}

lb_status field_from_host(lb_ctx* c, int inst, int fid, const double* src, int64_t nfields = 1) {
    const InstDesc& I = c->hinst[inst];
    const int64_t n = I.ncell * nfields;
    unsigned char* dst = reinterpret_cast<unsigned char*>(I.base) + (size_t)fid * I.ncell * c->wbytes();
    if (c->prec == LB_FP64) {
        LB_HIP(hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, c->stream));
        LB_HIP(hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(n);
        for (int64_t k = 0; k < n; ++k) tmp[k] = (float)src[k];
        LB_HIP(hipMemcpyAsync(dst, tmp.data(), n * 4, hipMemcpyHostToDevice, c->stream));
        LB_HIP(hipStreamSynchronize(c->stream));
    }
    return LB_OK;
}

// Host (rho, u_x, u_y, T) fields of an instance: present, finite, rho > 0, T > 0, 1 - b_w rho > 0.
lb_status check_moment_fields(const lb_params& q, int k, const double* rho, const double* ux,
                              const double* uy, const double* T) {
    if (!rho || !ux || !uy || !T) return fail(LB_E_ARG, "instance %d: null field", k);
    const int64_t nc = (int64_t)q.nx * q.ny;
    for (int64_t e = 0; e < nc; ++e) {
        const double r = rho[e], t = T[e];
        if (!(r > 0) || !(t > 0) || !(1.0 - q.vdw_b * r > 0) || !std::isfinite(ux[e]) ||
            !std::isfinite(uy[e]) || !std::isfinite(r) || !std::isfinite(t))
            return fail(LB_E_ARG, "instance %d cell %lld: need rho > 0, T > 0, 1 - vdw_b rho > 0 "
                        "and finite u", k, (long long)e);
    }
    return LB_OK;
}

lb_status validate_params(const lb_params& q, int k) {
    if (!grid_ok(q.nx, q.ny))
        return fail(LB_E_SIZE, "instance %d: unsupported grid %dx%d (each side 2^a or 3*2^a in "
                    "[8,2048]; ny may also be 1 or 2)", k, q.nx, q.ny);
    if (!(q.dx > 0) || !(q.dt > 0) || !(q.tau > 0) || !(q.b_dof > 0))
        return fail(LB_E_ARG, "instance %d: dx, dt, tau and b must be positive", k);
    const double v[] = {q.K, q.H, q.zeta, q.q, q.vdw_a, q.vdw_b};
    for (double x : v)
        if (!std::isfinite(x)) return fail(LB_E_ARG, "instance %d: non-finite parameter", k);
    if (q.vdw_b < 0) return fail(LB_E_ARG, "instance %d: vdw_b must be >= 0", k);
    if (q.hist_len < 0 || q.hist_len > (1 << 24))
        return fail(LB_E_ARG, "instance %d: hist_len must be in [0, 2^24]", k);
    return LB_OK;
}

// Stage host (rho, u_x, u_y, T) as float64 in the F_B block of instance k, then set
// f = f^eq(rho, u, T) in F_A (Sec. 2.1).  Fields already checked.  Synchronous.
lb_status state_from_moments(lb_ctx* c, int k, const double* rho, const double* ux, const double* uy,
                             const double* T) {
    const InstDesc& I = c->hinst[k];
    unsigned char* stage = reinterpret_cast<unsigned char*>(I.base) + (size_t)F_B * I.ncell * c->wbytes();
    const double* src[4] = {rho, ux, uy, T};
    for (int f = 0; f < 4; ++f)
        LB_HIP(hipMemcpyAsync(stage + (size_t)f * I.ncell * 8, src[f], I.ncell * 8,
                              hipMemcpyHostToDevice, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    const LaunchSet L = set_one(*c, k, c->stream);
    if (c->prec == LB_FP64)
        LB_HIP(launch_init<double>(L, c->dev<DvmConst<double>>(c->lay.dvm64)));
    else
        LB_HIP(launch_init<float>(L, c->dev<DvmConst<double>>(c->lay.dvm64)));
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

size_t lb_workspace_bytes(int n_inst, const lb_params* p, lb_precision prec) {
    if (n_inst <= 0 || !p || (prec != LB_FP64 && prec != LB_FP32)) return 0;
    for (int k = 0; k < n_inst; ++k)
        if (validate_params(p[k], k) != LB_OK) return 0;
    return make_layout(n_inst, p, prec).total;
}

lb_status lb_init(lb_ctx** out, int n_inst, const lb_params* p, const lb_dvm* dvm,
                  lb_precision prec, const double* const* rho0, const double* const* ux0,
                  const double* const* uy0, const double* const* T0, void* d_workspace,
                  size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    if (!out) return fail(LB_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_inst <= 0 || !p || !rho0 || !ux0 || !uy0 || !T0 || !d_workspace)
        return fail(LB_E_ARG, "null argument or n_inst <= 0");
    if (prec != LB_FP64 && prec != LB_FP32) return fail(LB_E_ARG, "bad precision");
    if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN)
        return fail(LB_E_ARG, "workspace must be %zu-byte aligned", ALIGN);
    for (int k = 0; k < n_inst; ++k) {
        lb_status s = validate_params(p[k], k);
        if (s != LB_OK) return s;
        s = check_moment_fields(p[k], k, rho0[k], ux0[k], uy0[k], T0[k]);
        if (s != LB_OK) return s;
    }
    Layout lay = make_layout(n_inst, p, prec);
    if (ws_bytes < lay.total)
        return fail(LB_E_SIZE, "workspace of %zu bytes < %zu required", ws_bytes, lay.total);

    lb_ctx* c = new (std::nothrow) lb_ctx();
    if (!c) return fail(LB_E_NOMEM, "host allocation failed");
    c->n = n_inst;
    c->prec = prec;
    c->p.assign(p, p + n_inst);
    c->dvm = dvm ? *dvm : lb_dvm{1.0, 0.5, 2.0, 1.0, 2.5};
    c->ws = reinterpret_cast<unsigned char*>(d_workspace);
    c->ws_bytes = ws_bytes;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->lay = lay;
    if (const char* g = std::getenv("LBFFT_NO_GRAPH")) c->use_graph = !(g[0] == '1');
    if (const char* g = std::getenv("LBFFT_GRAPH_STEPS")) {
        const int k = std::atoi(g);
        if (k >= 1 && k <= 64) c->graph_steps = k;
    }
    if (const char* g = std::getenv("LBFFT_FUSE_XY")) c->fuse_xy = !(g[0] == '0');
    if (const char* g = std::getenv("LBFFT_PPB")) {
        const int v = std::atoi(g);
        if (v == 1 || v == 2 || v == 4) c->ppb_override = v;
    }
    if (const char* g = std::getenv("LBFFT_YPOP")) {
        if (g[0] >= '0' && g[0] <= '2') c->ypop_override = g[0] - '0';
    }
    if (const char* g = std::getenv("LBFFT_YMAC")) {
        if (g[0] == '0' || g[0] == '2') c->ymac_override = g[0] - '0';
    }
    if (const char* g = std::getenv("LBFFT_XPOP")) {
        if (g[0] == '0' || g[0] == '1') c->xpop_override = g[0] - '0';
    }

    if (!build_dvm(c->dvm, c->dvm64)) {
        delete c;
        return fail(LB_E_ARG, "the velocity set gives a singular moment matrix");
    }
    for (int i = 0; i < 16; ++i) {
        c->dvm32.vx[i] = (float)c->dvm64.vx[i];
        c->dvm32.vy[i] = (float)c->dvm64.vy[i];
        c->dvm32.w[i] = (float)c->dvm64.w[i];
        c->dvm32.eta2[i] = (float)c->dvm64.eta2[i];
        for (int j = 0; j < 16; ++j) c->dvm32.cinv[i][j] = (float)c->dvm64.cinv[i][j];
    }
    for (int i = 0; i < 16; ++i)
        if (c->dvm64.vy[i] != 0.0) c->pops_h[c->npops++] = i;
    // x-pass order: mirror pairs -- populations with v_x != 0 paired with their x mirror, then the
    // v_x = 0 ones paired with their y mirror (the kernel forms both equilibria of a pair from one
    // split dot product).  Every ring of the D2V16 set is closed under both mirrors.
    {
        int k = 0;
        bool used[16] = {false};
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < 16; ++i) {
                if (used[i] || ((c->dvm64.vx[i] != 0.0) != (pass == 0))) continue;
                int j = -1;
                for (int m = 0; m < 16; ++m) {
                    const bool xm = c->dvm64.vx[m] == -c->dvm64.vx[i] && c->dvm64.vy[m] == c->dvm64.vy[i];
                    const bool ym = c->dvm64.vx[m] == c->dvm64.vx[i] && c->dvm64.vy[m] == -c->dvm64.vy[i];
                    if (m != i && !used[m] && (pass == 0 ? xm : ym)) j = m;
                }
                if (j < 0) {
                    delete c;
                    return fail(LB_E_ARG, "velocity set is not closed under mirror reflections");
                }
                used[i] = used[j] = true;
                c->dvm64.xorder[k++] = i;
                c->dvm64.xorder[k++] = j;
            }
        for (int i = 0; i < 16; ++i) c->dvm32.xorder[i] = c->dvm64.xorder[i];
    }
    // quarter-turn partner of each population: f^eq_i(u) = f^eq_rot(i)(u_y, -u_x) on a velocity
    // set closed under quarter turns, which lets the x pass form the equilibria of a y-mirror pair
    // with the x-mirror split of the turned pair
    for (int i = 0; i < 16; ++i) {
        int j = -1;
        for (int m = 0; m < 16; ++m)
            if (c->dvm64.vx[m] == c->dvm64.vy[i] && c->dvm64.vy[m] == -c->dvm64.vx[i] &&
                c->dvm64.eta2[m] == c->dvm64.eta2[i])
                j = m;
        if (j < 0) {
            delete c;
            return fail(LB_E_ARG, "velocity set is not closed under quarter turns");
        }
        c->dvm64.rot[i] = c->dvm32.rot[i] = j;
    }
    build_jobs(*c);

    // instance descriptors and size classes
    const size_t w = word_bytes(prec);
    c->hinst.resize(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        InstDesc& I = c->hinst[k];
        std::memset(&I, 0, sizeof(I));
        I.nx = p[k].nx;
        I.ny = p[k].ny;
        I.ncell = (int64_t)p[k].nx * p[k].ny;
        I.base = c->ws + lay.arena[k];
        size_t t = lay.tables[k];
        I.kx = c->ws + t;  t = align_up(t + w * I.nx);
        I.ky = c->ws + t;  t = align_up(t + w * I.ny);
        I.twx = c->ws + t; t = align_up(t + 2 * w * I.nx);
        I.twy = c->ws + t;
        double* red = c->dev<double>(lay.red[k]);
        I.red = red;
        I.cons = red + 5 * RED_BLOCKS;
        I.hist_count = reinterpret_cast<unsigned long long*>(red + 5 * RED_BLOCKS + 8);
        I.hist = red + 5 * RED_BLOCKS + 9;
        I.red_blocks = RED_BLOCKS;
        I.hist_len = p[k].hist_len;
        I.dx = p[k].dx; I.dt = p[k].dt; I.tau = p[k].tau; I.K = p[k].K; I.H = p[k].H;
        I.zeta = p[k].zeta; I.q = p[k].q; I.b = p[k].b_dof; I.a = p[k].vdw_a; I.bw = p[k].vdw_b;
        // FP64 stores f itself (fref = 0); FP32 stores the deviation from a reference equilibrium
        if (prec == LB_FP32) set_reference(c->dvm64, p[k], rho0[k], T0[k], I);
    }
    std::vector<int> order;
    for (int k = 0; k < n_inst; ++k) {
        bool found = false;
        for (auto& cl : c->classes)
            if (cl.nx == p[k].nx && cl.ny == p[k].ny) found = true;
        if (found) continue;
        lb_ctx::Class cl{p[k].nx, p[k].ny, (int)order.size(), 0};
        for (int j = 0; j < n_inst; ++j)
            if (p[j].nx == cl.nx && p[j].ny == cl.ny) {
                order.push_back(j);
                ++cl.count;
                if (p[j].hist_len > 0) cl.hist = true;
            }
        c->classes.push_back(cl);
    }
    c->ilist_h = order;
    for (int k = 0; k < n_inst; ++k) c->ilist_h.push_back(k);

    lb_status st = LB_OK;
    auto up = [&](size_t off, const void* src, size_t bytes) -> bool {
        hipError_t e = hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            st = fail(LB_E_HIP, "upload failed: %s", hipGetErrorString(e));
            return false;
        }
        return true;
    };
    bool ok = up(lay.insts, c->hinst.data(), sizeof(InstDesc) * n_inst) &&
              up(lay.dvm64, &c->dvm64, sizeof(c->dvm64)) && up(lay.dvm32, &c->dvm32, sizeof(c->dvm32)) &&
              up(lay.jobs, c->jobs.data(), sizeof(JobDesc) * c->jobs.size()) &&
              up(lay.pops, c->pops_h, sizeof(int) * 16) &&
              up(lay.ilist, c->ilist_h.data(), sizeof(int) * c->ilist_h.size());
    if (ok) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            ok = false;
            st = fail(LB_E_HIP, "sync failed: %s", hipGetErrorString(e));
        }
    }
    // conservation partials, last result, history counter and ring start at zero (the caller's
    // workspace is uninitialised); done at init, outside any captured graph
    for (int k = 0; ok && k < n_inst; ++k) {
        const size_t bytes = sizeof(double) * (5 * RED_BLOCKS + 8 + 1 + 4 * (size_t)p[k].hist_len);
        hipError_t e = hipMemsetAsync(c->hinst[k].red, 0, bytes, c->stream);
        if (e != hipSuccess) {
            ok = false;
            st = fail(LB_E_HIP, "clearing conservation buffers: %s", hipGetErrorString(e));
        }
    }
    // tables in float64, rounded to the working precision
    for (int k = 0; ok && k < n_inst; ++k) {
        hipError_t e = prec == LB_FP64 ? launch_tables<double>(c->d_insts(), k, p[k].nx, p[k].ny, c->stream)
                                       : launch_tables<float>(c->d_insts(), k, p[k].nx, p[k].ny, c->stream);
        if (e != hipSuccess) {
            ok = false;
            st = fail(LB_E_HIP, "table kernel: %s", hipGetErrorString(e));
        }
    }
    // initial condition: f = f^eq(rho0, u0, T0)
    for (int k = 0; ok && k < n_inst; ++k) {
        st = state_from_moments(c, k, rho0[k], ux0[k], uy0[k], T0[k]);
        ok = st == LB_OK;
    }
    if (ok) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            ok = false;
            st = fail(LB_E_HIP, "init sync: %s", hipGetErrorString(e));
        }
    }
    // tune the launch variants of each size class on its own data (unless disabled)
    const char* tune_env = std::getenv("LBFFT_TUNE");
    const bool tune = !(tune_env && tune_env[0] == '0');
    for (auto& cl : c->classes) {
        if (!ok) break;
        const int64_t cells = (int64_t)cl.nx * cl.ny * cl.count;
        cl.ppb = cells >= (1 << 20) ? 2 : 1;   // default without tuning
        if (tune && (!c->ppb_override || c->ypop_override < 0 || c->ymac_override < 0 || c->xpop_override < 0)) {
            hipError_t e = tune_class(*c, cl);
            if (e != hipSuccess) {
                ok = false;
                st = fail(LB_E_HIP, "tuning: %s", hipGetErrorString(e));
            }
        }
    }
    // capture one Runge-Kutta step into a graph, and graph_steps consecutive steps into a second
    // one (fewer replays): private streams of default priority, one branch per size class
    if (ok && c->use_graph) {
        hipError_t e = build_graph(*c, 1, &c->graph, &c->exec);
        if (e == hipSuccess && c->graph_steps > 1) e = build_graph(*c, c->graph_steps, &c->graph_k, &c->exec_k);
        if (e != hipSuccess) {
            ok = false;
            st = fail(LB_E_HIP, "graph capture: %s", hipGetErrorString(e));
        }
    }
    if (!ok) {
        lb_free(c);
        return st;
    }
    *out = c;
    return LB_OK;
}

lb_status lb_step(lb_ctx* c, int n_steps) {
    if (!c) return fail(LB_E_ARG, "null context");
    if (n_steps < 0) return fail(LB_E_ARG, "n_steps < 0");
    int s = 0;
    if (c->exec_k)
        for (; s + c->graph_steps <= n_steps; s += c->graph_steps) LB_HIP(hipGraphLaunch(c->exec_k, c->stream));
    for (; s < n_steps; ++s) {
        if (c->exec) {
            LB_HIP(hipGraphLaunch(c->exec, c->stream));
        } else {
            LB_HIP(enqueue_step(*c, c->stream));
        }
    }
    return LB_OK;
}

namespace {
// One start/stop event pair per launch, tagged with its pass kind.
struct EventHook : PassHook {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t next = 0;
    bool events(int pass, hipEvent_t* start, hipEvent_t* stop) override {
        if (2 * next + 1 >= ev.size()) return false;
        kind[next] = pass;
        *start = ev[2 * next];
        *stop = ev[2 * next + 1];
        ++next;
        return true;
    }
};
}  // namespace

lb_status lb_step_timed(lb_ctx* c, int n_steps, double ms[LB_NPASS]) {
    if (!c) return fail(LB_E_ARG, "null context");
    if (n_steps <= 0 || !ms) return fail(LB_E_ARG, "need n_steps > 0 and an output array");
    EventHook h;
    const size_t nlaunch = (size_t)n_steps * 2 * LB_NPASS * c->classes.size();
    h.ev.resize(2 * nlaunch, nullptr);
    h.kind.resize(nlaunch, -1);
    lb_status st = LB_OK;
    for (size_t k = 0; k < h.ev.size() && st == LB_OK; ++k)
        if (hipEventCreate(&h.ev[k]) != hipSuccess) st = fail(LB_E_HIP, "hipEventCreate failed");
    for (int s = 0; s < n_steps && st == LB_OK; ++s) {
        hipError_t e = enqueue_step(*c, c->stream, &h);
        if (e != hipSuccess) st = fail(LB_E_HIP, "step launch: %s", hipGetErrorString(e));
    }
    if (st == LB_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = fail(LB_E_HIP, "sync failed");
    double sum[LB_NPASS] = {0};
    int cnt[LB_NPASS] = {0};
    for (size_t k = 0; st == LB_OK && k < h.next; ++k) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, h.ev[2 * k], h.ev[2 * k + 1]) != hipSuccess) {
            st = fail(LB_E_HIP, "hipEventElapsedTime failed");
            break;
        }
        sum[h.kind[k]] += t;
        cnt[h.kind[k]] += 1;
    }
    for (int k = 0; k < LB_NPASS; ++k) ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
    for (auto e : h.ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

lb_status lb_sync(lb_ctx* c) {
    if (!c) return fail(LB_E_ARG, "null context");
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

lb_status lb_moments(lb_ctx* c, int inst, double* rho, double* ux, double* uy, double* T) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    LB_HIP(moments(*c, set_one(*c, inst, c->stream), F_A));
    double* dst[4] = {rho, ux, uy, T};
    for (int f = 0; f < 4; ++f)
        if (dst[f] && (s = field_to_host(c, inst, RHO + f, dst[f])) != LB_OK) return s;
    // the temperature field holds T - T_ref
    const double Tref = c->hinst[inst].T_ref;
    if (T && Tref != 0.0)
        for (int64_t e = 0; e < c->hinst[inst].ncell; ++e) T[e] += Tref;
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

lb_status lb_conservation(lb_ctx* c, int inst, double out[4]) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!out) return fail(LB_E_ARG, "out is NULL");
    const LaunchSet L = set_one(*c, inst, c->stream);
    // the same passes (fused or not) as the step, so the on-demand sums equal the recorded ones
    const StageArgs st{F_A, -1, -1, 0.0, 0};
    LB_HIP(run_pass(*c, L, LB_PASS_MOMENTS, st));
    LB_HIP(run_pass(*c, L, LB_PASS_MACRO_X1, st));
    LB_HIP(run_pass(*c, L, LB_PASS_MACRO_Y1, st));
    LB_HIP(c->prec == LB_FP64 ? launch_conserve<double>(L, 0) : launch_conserve<float>(L, 0));
    double r[5];
    LB_HIP(hipMemcpyAsync(r, c->hinst[inst].cons, sizeof(r), hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    for (int k = 0; k < 4; ++k) out[k] = r[k];
    if (r[4] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[3]))
        return fail(LB_E_NONFINITE, "instance %d holds %g non-finite cells", inst, r[4]);
    return LB_OK;
}

lb_status lb_conservation_history(lb_ctx* c, int inst, int max_entries, double* out, int* n_out,
                                  long long* first_step) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!out || !n_out || max_entries < 0) return fail(LB_E_ARG, "null output or max_entries < 0");
    const InstDesc& I = c->hinst[inst];
    *n_out = 0;
    if (first_step) *first_step = 0;
    if (I.hist_len <= 0) return fail(LB_E_STATE, "instance %d keeps no history (hist_len = 0)", inst);
    unsigned long long count = 0;
    std::vector<double> ring(4 * (size_t)I.hist_len);
    LB_HIP(hipMemcpyAsync(&count, I.hist_count, sizeof(count), hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipMemcpyAsync(ring.data(), I.hist, ring.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    const unsigned long long have = count < (unsigned long long)I.hist_len ? count : (unsigned long long)I.hist_len;
    const unsigned long long take = have < (unsigned long long)max_entries ? have : (unsigned long long)max_entries;
    const unsigned long long first = count - take;
    for (unsigned long long t = 0; t < take; ++t) {
        const unsigned long long slot = (first + t) % (unsigned long long)I.hist_len;
        for (int k = 0; k < 4; ++k) out[4 * t + k] = ring[4 * slot + k];
    }
    *n_out = (int)take;
    if (first_step) *first_step = (long long)first;
    for (unsigned long long t = 0; t < take; ++t)
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(out[4 * t + k]))
                return fail(LB_E_NONFINITE, "instance %d: non-finite conservation history", inst);
    return LB_OK;
}

lb_status lb_get_f(lb_ctx* c, int inst, double* f) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!f) return fail(LB_E_ARG, "f is NULL");
    if ((s = field_to_host(c, inst, F_A, f, 16)) != LB_OK) return s;
    // the arena holds f - fref (fref = 0 in FP64)
    const InstDesc& I = c->hinst[inst];
    if (c->prec == LB_FP32)
        for (int i = 0; i < 16; ++i)
            for (int64_t e = 0; e < I.ncell; ++e) f[i * I.ncell + e] += I.fref[i];
    return LB_OK;
}

lb_status lb_set_f(lb_ctx* c, int inst, const double* f) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!f) return fail(LB_E_ARG, "f is NULL");
    const InstDesc& I = c->hinst[inst];
    if (c->prec == LB_FP64) return field_from_host(c, inst, F_A, f, 16);
    std::vector<double> g((size_t)16 * I.ncell);
    for (int i = 0; i < 16; ++i)
        for (int64_t e = 0; e < I.ncell; ++e) g[i * I.ncell + e] = f[i * I.ncell + e] - I.fref[i];
    return field_from_host(c, inst, F_A, g.data(), 16);
}

lb_status lb_set_moments(lb_ctx* c, int inst, const double* rho, const double* ux, const double* uy,
                         const double* T) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if ((s = check_moment_fields(c->p[inst], inst, rho, ux, uy, T)) != LB_OK) return s;
    return state_from_moments(c, inst, rho, ux, uy, T);
}

lb_status lb_force_coefficients(lb_ctx* c, int inst, double* Bx, double* By, double* C) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    LB_HIP(force_passes(*c, set_one(*c, inst, c->stream), F_A));
    if (Bx && (s = field_to_host(c, inst, BX, Bx)) != LB_OK) return s;
    if (By && (s = field_to_host(c, inst, BY, By)) != LB_OK) return s;
    if (C && (s = field_to_host(c, inst, CT, C)) != LB_OK) return s;
    return LB_OK;
}

lb_status lb_rhs(lb_ctx* c, int inst, double* R) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!R) return fail(LB_E_ARG, "R is NULL");
    const LaunchSet L = set_one(*c, inst, c->stream);
    LB_HIP(force_passes(*c, L, F_A));
    StageArgs st{F_A, -1, F_B, 1.0, 0};
    LB_HIP(pop_passes(*c, L, st));
    return field_to_host(c, inst, F_B, R, 16);
}

lb_status lb_derivative(lb_ctx* c, int inst, int axis, int order, const double* g, double* out) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!g || !out) return fail(LB_E_ARG, "null field");
    if ((axis != 0 && axis != 1) || (order != 1 && order != 2))
        return fail(LB_E_ARG, "axis must be 0/1 and order 1/2");
    if ((s = field_from_host(c, inst, SCR0, g)) != LB_OK) return s;
    const int j = axis == 0 ? (order == 1 ? c->j_dx : c->j_dxx) : (order == 1 ? c->j_dy : c->j_dyy);
    LB_HIP(macro(*c, set_one(*c, inst, c->stream), axis, j, 1));
    return field_to_host(c, inst, SCR1, out);
}

lb_status lb_plan_info(lb_ctx* c, int inst, int* out, int n) {
    lb_status s = check_inst(c, inst);
    if (s != LB_OK) return s;
    if (!out || n < 2) return fail(LB_E_ARG, "need an output array of length >= 2");
    const LaunchSet L = set_one(*c, inst, c->stream);
    // the variant a launch actually runs: the chosen one where it exists for the class's lines
    const int have = class_variants(*c, L.ny), have_x = class_variants_x(*c, L.nx);
    const int v[5] = {L.ppb, (int)c->classes.size(), (have >> L.ypop_var) & 1 ? L.ypop_var : 0,
                      (have >> L.ymac_var) & 1 ? L.ymac_var : 0, (have_x >> L.xpop_var) & 1 ? L.xpop_var : 0};
    for (int k = 0; k < n && k < 5; ++k) out[k] = v[k];
    return LB_OK;
}

void lb_free(lb_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->exec_k) (void)hipGraphExecDestroy(c->exec_k);
    if (c->graph_k) (void)hipGraphDestroy(c->graph_k);
    delete c;
}

}  // extern "C"
