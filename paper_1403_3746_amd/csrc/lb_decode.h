// Block-index decoding of the line passes (host and device: the host tests enumerate it).
#pragma once
#include <hip/hip_runtime.h>

namespace lbfft {

// Decode the flat block index into (instance, tile, job).  Workgroups are dealt to the 8 XCDs
// round-robin (block b runs on XCD b mod 8); each XCD gets a contiguous range of (instance, tile)
// groups and runs all jobs of a group back to back, so the inputs a group's jobs share (the
// coefficient fields of the population x pass) stay in that XCD's L2.  A launch has
// 8 * groups_per_xcd(ngroups) * njobs blocks; the decoded (group, job) pairs of its valid blocks
// are all pairs, each once.
struct BlockWork {
    int inst_local, tile, job;
    bool valid;
};

__host__ __device__ constexpr int groups_per_xcd(int ngroups) { return (ngroups + 7) / 8; }

__host__ __device__ inline BlockWork decode_block_at(int b, int ngroups, int ntiles, int njobs) {
    const int xcd = b & 7;
    const int slot = b >> 3;
    const int gpx = groups_per_xcd(ngroups);
    const int g_local = slot / njobs;
    const int group = xcd * gpx + g_local;
    BlockWork w;
    w.job = slot % njobs;
    w.valid = g_local < gpx && group < ngroups;
    w.inst_local = group / ntiles;
    w.tile = group % ntiles;
    return w;
}

// The same split over XCDs for passes whose jobs share no input (one field per job): each XCD runs
// its range of groups tile after tile for one job, then the next job, so the tiles in flight on an
// XCD are neighbours in the same field -- the cache lines and DRAM pages that neighbouring column
// tiles split are then requested together -- and the XCD's working set is one field's strip.
__host__ __device__ inline BlockWork decode_block_jm(int b, int ngroups, int ntiles, int njobs) {
    const int xcd = b & 7;
    const int slot = b >> 3;
    const int gpx = groups_per_xcd(ngroups);
    const int g_local = slot % gpx;
    const int group = xcd * gpx + g_local;
    BlockWork w;
    w.job = slot / gpx;
    w.valid = w.job < njobs && group < ngroups;
    w.inst_local = group / ntiles;
    w.tile = group % ntiles;
    return w;
}

}  // namespace lbfft
