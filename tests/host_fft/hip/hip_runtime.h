// Host stand-in for the few HIP names the line FFT header uses: device qualifiers become plain
// inline functions and the workgroup barrier becomes a C++20 barrier shared by the threads that
// emulate one workgroup's lanes.
#pragma once
#include <barrier>
#include <cstring>
#define __device__
#define __host__
#define __forceinline__ inline
extern thread_local std::barrier<>* host_workgroup_barrier;
inline void __syncthreads() { host_workgroup_barrier->arrive_and_wait(); }
// The per-wave ordering of the FFT's LDS exchanges (line_sync<true>): a barrier over the threads
// emulating the lanes of one 64-lane wave (the lanes of a wave run in lockstep on the GPU).
extern thread_local std::barrier<>* host_wave_barrier;
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_wave_barrier() host_wave_barrier->arrive_and_wait()
// Buffer loads of the twiddle table: a resource is the base pointer, a load copies the bytes at
// the given offset.
struct host_buffer_rsrc {
    const char* p;
};
template <int B>
struct host_bytes {
    unsigned char b[B];
};
template <int B>
inline host_bytes<B> host_buffer_load(host_buffer_rsrc r, unsigned off) {
    host_bytes<B> x;
    std::memcpy(x.b, r.p + off, B);
    return x;
}
#define __amdgpu_buffer_rsrc_t host_buffer_rsrc
#define __builtin_amdgcn_make_buffer_rsrc(p, stride, num, flags) host_buffer_rsrc{(const char*)(p)}
#define __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, aux) host_buffer_load<16>((r), (voff) + (soff))
#define __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, aux) host_buffer_load<8>((r), (voff) + (soff))
