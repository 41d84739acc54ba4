// Host stand-in for the few HIP names the line FFT header uses: device qualifiers become plain
// inline functions and the workgroup barrier becomes a C++20 barrier shared by the threads that
// emulate one workgroup's lanes.
#pragma once
#include <barrier>
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
