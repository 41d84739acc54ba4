// CPU emulation of the line FFT engine (lb_fft.h): one std::thread per lane of a workgroup, a
// std::barrier for the workgroup barrier, the LDS as a shared array.  For each case it transforms
// every line of a block forward (checked against a naive DFT) and back (checked against the
// input), with the block shapes the kernels use: x blocks (lines contiguous in LDS, LS = 1) and
// y blocks (lines interleaved word by word, LS = lines per block), one line at a time (run) and
// Q lines together (run_n), and x blocks of one-wave lines with per-wave ordering (WAVE).  Prints one line per case: precision N layout Q fwd_err rt_err.
#include <cmath>
#include <complex>
#include <cstdio>
#include <memory>
#include <thread>
#include <vector>

#include "lb_fft.h"

thread_local std::barrier<>* host_workgroup_barrier;
thread_local std::barrier<>* host_wave_barrier;

// One barrier per 64-lane wave of a workgroup of wg threads.
static std::vector<std::unique_ptr<std::barrier<>>> wave_barriers(int wg) {
    std::vector<std::unique_ptr<std::barrier<>>> w;
    for (int b = 0; b < wg; b += 64) w.emplace_back(new std::barrier<>(std::min(64, wg - b)));
    return w;
}

using namespace lbfft;

template <typename T, int N, int LS, int LINES, int Q, bool WAVE = false, int RR = 0>
void run_case(const char* layout) {
    constexpr int R = RR ? RR : default_R(N), TPL = N / R, WG = LINES * TPL;
    // LDS: x blocks give line l the region l*lds_line(N) (element i at lds_idx(i)); y blocks
    // interleave the lines (element i of line l at lds_idx(i)*LINES + l)
    constexpr int STRIDE = LINES * lds_line(N);
    std::vector<cpx<T>> tab(N), lds(Q * STRIDE + 1), x(Q * LINES * N), y(x.size()), z(x.size());
    for (int k = 0; k < N; ++k) tab[k] = {T(std::cos(-2 * M_PI * k / N)), T(std::sin(-2 * M_PI * k / N))};
    for (size_t k = 0; k < x.size(); ++k)
        x[k] = {T(std::sin(0.37 * double(k * k % 1013) + 1.0)), T(std::cos(0.71 * double(k % 997)))};
    std::barrier<> bar(WG);
    auto wbar = wave_barriers(WG);
    std::vector<std::thread> th;
    for (int tid = 0; tid < WG; ++tid)
        th.emplace_back([&, tid] {
            host_workgroup_barrier = &bar;
            host_wave_barrier = wbar[tid / 64].get();
            const int l = LS == 1 ? tid / TPL : tid % LINES;
            const int t = LS == 1 ? tid % TPL : tid / LINES;
            cpx<T>* ld = lds.data() + (LS == 1 ? l * lds_line(N) : l);
            typename LineFFT<T, N, R, false, LS, WAVE>::Tw tw;
            tw.load(tab.data(), t);
            cpx<T> v[Q][R];
            for (int q = 0; q < Q; ++q)
                for (int m = 0; m < R; ++m) v[q][m] = x[(q * LINES + l) * N + t + m * TPL];
            if constexpr (Q == 1) {
                LineFFT<T, N, R, false, LS, WAVE>::run(v[0], ld, t, tw);
            } else {
                LineFFT<T, N, R, false, LS, WAVE>::template run_n<Q>(v, ld, STRIDE, t, tw);
            }
            for (int q = 0; q < Q; ++q)
                for (int m = 0; m < R; ++m) {
                    y[(q * LINES + l) * N + t + m * TPL] = v[q][m];
                    v[q][m].re *= T(1.0 / N);
                    v[q][m].im *= T(1.0 / N);
                }
            if constexpr (Q == 1) {
                LineFFT<T, N, R, true, LS, WAVE>::run(v[0], ld, t, tw);
            } else {
                LineFFT<T, N, R, true, LS, WAVE>::template run_n<Q>(v, ld, STRIDE, t, tw);
            }
            for (int q = 0; q < Q; ++q)
                for (int m = 0; m < R; ++m) z[(q * LINES + l) * N + t + m * TPL] = v[q][m];
        });
    for (auto& h : th) h.join();
    double ef = 0, nf = 0, er = 0, nr = 0;
    for (int line = 0; line < Q * LINES; ++line) {
        const cpx<T>* xi = &x[line * N];
        for (int k = 0; k < N; ++k) {
            std::complex<double> s = 0;
            for (int n = 0; n < N; ++n)
                s += std::complex<double>(xi[n].re, xi[n].im) * std::polar(1.0, -2 * M_PI * double((long)k * n % N) / N);
            const cpx<T>& Y = y[line * N + k];
            ef = std::max(ef, std::abs(s - std::complex<double>(Y.re, Y.im)));
            nf = std::max(nf, std::abs(s));
            const cpx<T>& Z = z[line * N + k];
            er = std::max(er, std::abs(std::complex<double>(double(xi[k].re) - Z.re, double(xi[k].im) - Z.im)));
            nr = std::max(nr, std::abs(std::complex<double>(xi[k].re, xi[k].im)));
        }
    }
    std::printf("%s %d %s%s %d %.3e %.3e\n", sizeof(T) == 8 ? "f64" : "f32", N, layout,
                RR == 16 ? "16" : (RR == 4 ? "4" : (RR == 24 ? "24" : "")), Q,
                ef / nf, er / nr);
}

template <typename T>
void all_sizes() {
    // x blocks: one line (several for short lines, as the kernels fill a wave), one at a time
    run_case<T, 8, 1, 8, 1>("x");
    run_case<T, 12, 1, 4, 1>("x");
    run_case<T, 16, 1, 4, 1>("x");
    run_case<T, 24, 1, 2, 1>("x");
    run_case<T, 32, 1, 2, 1>("x");
    run_case<T, 48, 1, 2, 1>("x");
    run_case<T, 64, 1, 2, 1>("x");
    run_case<T, 96, 1, 2, 1>("x");
    run_case<T, 128, 1, 1, 1>("x");
    run_case<T, 192, 1, 1, 1>("x");
    run_case<T, 256, 1, 1, 1>("x");
    run_case<T, 384, 1, 1, 1>("x");
    run_case<T, 512, 1, 1, 1>("x");
    run_case<T, 768, 1, 1, 1>("x");
    run_case<T, 1024, 1, 1, 1>("x");
    run_case<T, 1536, 1, 1, 1>("x");
    run_case<T, 2048, 1, 1, 1>("x");
    // several lines transformed together
    run_case<T, 16, 1, 2, 4>("x");
    run_case<T, 96, 1, 2, 2>("x");
    run_case<T, 128, 1, 1, 4>("x");
    run_case<T, 512, 1, 1, 2>("x");
    run_case<T, 2048, 1, 1, 2>("x");
    // y blocks: lines interleaved word by word
    run_case<T, 8, 4, 4, 1>("y");
    run_case<T, 48, 4, 4, 1>("y");
    run_case<T, 128, 8, 8, 1>("y");
    run_case<T, 384, 2, 2, 1>("y");
    run_case<T, 2048, 2, 2, 1>("y");
    // x blocks of several one-wave lines ordered per wave (line_sync<true>): only the threads of
    // one emulated wave synchronise, so a pass touching another wave's line would race
    run_case<T, 96, 1, 8, 1, true>("xw");
    run_case<T, 256, 1, 4, 1, true>("xw");
    run_case<T, 512, 1, 8, 1, true>("xw");
    run_case<T, 768, 1, 2, 1, true>("xw");
    // 16 elements per thread (radix-16 passes), the long lines' alternative plan
    run_case<T, 512, 1, 1, 1, false, 16>("x");
    run_case<T, 1024, 1, 1, 1, false, 16>("x");
    run_case<T, 2048, 1, 1, 1, false, 16>("x");
    run_case<T, 1024, 4, 4, 1, false, 16>("y");
    run_case<T, 2048, 2, 2, 1, false, 16>("y");
    run_case<T, 1024, 1, 2, 1, true, 16>("xw");
    // 4 elements per thread for x lines of 128-512 points (the population x pass's alternative
    // plan): two one-wave lines per wave, one line per wave, a line of two waves
    run_case<T, 128, 1, 2, 1, true, 4>("xw");
    run_case<T, 128, 1, 2, 2, false, 4>("x");
    run_case<T, 256, 1, 1, 2, true, 4>("xw");
    run_case<T, 512, 1, 1, 2, false, 4>("x");
    // 24 elements per thread for lines of 3 * 2^a points (the long-radix y and fused plans)
    run_case<T, 96, 16, 16, 1, false, 24>("y");
    run_case<T, 384, 16, 16, 1, false, 24>("y");
    run_case<T, 192, 1, 8, 1, true, 24>("xw");
    run_case<T, 384, 1, 16, 1, true, 24>("xw");
}

int main() {
    all_sizes<double>();
    all_sizes<float>();
    return 0;
}
