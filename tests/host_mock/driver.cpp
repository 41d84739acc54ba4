// Host-runtime driver for the CPU check: a 512^2 FP64 context and a mixed-size FP32 batch with
// conservation history, each initialised, stepped (graph and timed paths) and freed.
#include "lbfft.h"
#include <cstdio>
#include <cstdlib>
#include <vector>
int main() {
    const int n = 512;
    lb_params p{n, n, 1.0, 1e-3, 1e-2, 1e-2, 0, 0, 0, 2.0, 9.0 / 49, 2.0 / 21, 0};
    std::vector<double> rho(n * n, 3.5), ux(n * n, 0), uy(n * n, 0), T(n * n, 0.514);
    size_t ws = lb_workspace_bytes(1, &p, LB_FP64);
    printf("ws %zu\n", ws);
    void* mem = aligned_alloc(256, ws);
    const double* r[1] = {rho.data()}; const double* x[1] = {ux.data()}; const double* y[1] = {uy.data()}; const double* t[1] = {T.data()};
    lb_ctx* c = nullptr;
    int st = lb_init(&c, 1, &p, nullptr, LB_FP64, r, x, y, t, mem, ws, nullptr);
    printf("init %d %s\n", st, lb_last_error());
    st = lb_step(c, 3); printf("step %d\n", st);
    double ms[LB_NPASS]; st = lb_step_timed(c, 2, ms); printf("timed %d\n", st);
    double out[4]; st = lb_conservation(c, 0, out); printf("cons %d\n", st);
    std::vector<double> T2(n * n, 0.5);
    st = lb_set_moments(c, 0, rho.data(), ux.data(), uy.data(), T2.data()); printf("setmom %d\n", st);
    T2[7] = -1.0;
    st = lb_set_moments(c, 0, rho.data(), ux.data(), uy.data(), T2.data()); printf("setmom_bad %d\n", st);
    lb_free(c); free(mem);
    // batch of two classes with history
    lb_params q[3] = {p, p, p}; q[1].nx = 96; q[1].ny = 96; q[2].hist_len = 8;
    std::vector<double> r2(96 * 96, 3.5), z2(96 * 96, 0), t2(96 * 96, 0.514);
    const double* rr[3] = {rho.data(), r2.data(), rho.data()}; const double* xx[3] = {ux.data(), z2.data(), ux.data()};
    const double* tt[3] = {T.data(), t2.data(), T.data()};
    ws = lb_workspace_bytes(3, q, LB_FP32); mem = aligned_alloc(256, ws);
    st = lb_init(&c, 3, q, nullptr, LB_FP32, rr, xx, xx, tt, mem, ws, nullptr);
    printf("init2 %d %s\n", st, lb_last_error());
    lb_step(c, 2); lb_free(c); free(mem);
    // long columns: a class whose population y pass has a wide variant to tune
    lb_params w = p; w.nx = 24; w.ny = 1024;
    std::vector<double> r3(24 * 1024, 3.5), z3(24 * 1024, 0), t3(24 * 1024, 0.514);
    const double* r3p[1] = {r3.data()}; const double* z3p[1] = {z3.data()}; const double* t3p[1] = {t3.data()};
    ws = lb_workspace_bytes(1, &w, LB_FP32); mem = aligned_alloc(256, ws);
    st = lb_init(&c, 1, &w, nullptr, LB_FP32, r3p, z3p, z3p, t3p, mem, ws, nullptr);
    int plan[4] = {0, 0, -1, -1};
    printf("init3 %d %d\n", st, lb_plan_info(c, 0, plan, 4));
    lb_step(c, 1); lb_free(c); free(mem);
    printf("done\n");
    return 0;
}
