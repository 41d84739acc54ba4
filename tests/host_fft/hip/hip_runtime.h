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
