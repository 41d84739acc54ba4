// Host check of the line passes' block decoding (paper_1403_3746_amd/csrc/lb_decode.h): for a
// range of launch shapes, every (instance, tile, job) is decoded by exactly one valid block, every
// block of XCD x takes a group in x's contiguous range, and in the job-major order the consecutive
// blocks of one XCD take consecutive tiles of one job.  Prints one line per order and exits 1 on the
// first failure.
#include <cstdio>
#include <vector>

#include "lb_decode.h"

using namespace lbfft;

template <typename F>
static bool check(const char* name, F decode, bool job_major) {
    long cases = 0;
    for (int ninst = 1; ninst <= 5; ++ninst)
        for (int ntiles = 1; ntiles <= 40; ntiles += (ntiles < 10 ? 1 : 7))
            for (int njobs = 1; njobs <= 16; ++njobs) {
                const int ngroups = ninst * ntiles, gpx = groups_per_xcd(ngroups);
                const int nblocks = 8 * gpx * njobs;
                std::vector<int> seen(ngroups * njobs, 0);
                std::vector<int> last_group(8, -1), last_job(8, -1);
                for (int b = 0; b < nblocks; ++b) {
                    const BlockWork w = decode(b, ngroups, ntiles, njobs);
                    const int xcd = b & 7;
                    if (!w.valid) continue;
                    const int group = w.inst_local * ntiles + w.tile;
                    if (w.inst_local < 0 || w.inst_local >= ninst || w.tile < 0 || w.tile >= ntiles ||
                        w.job < 0 || w.job >= njobs || group / gpx != xcd) {
                        std::printf("%s FAIL range b=%d ninst=%d ntiles=%d njobs=%d\n", name, b, ninst,
                                    ntiles, njobs);
                        return false;
                    }
                    ++seen[group * njobs + w.job];
                    if (job_major && last_job[xcd] == w.job && group != last_group[xcd] + 1) {
                        std::printf("%s FAIL order b=%d\n", name, b);
                        return false;
                    }
                    last_group[xcd] = group;
                    last_job[xcd] = w.job;
                }
                for (int s : seen)
                    if (s != 1) {
                        std::printf("%s FAIL cover ninst=%d ntiles=%d njobs=%d\n", name, ninst, ntiles,
                                    njobs);
                        return false;
                    }
                ++cases;
            }
    std::printf("%s ok %ld\n", name, cases);
    return true;
}

int main() {
    const bool a = check("group_major", decode_block_at, false);
    const bool b = check("job_major", decode_block_jm, true);
    return a && b ? 0 : 1;
}
