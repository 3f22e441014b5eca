// Host-build check of merged launches (test infrastructure only): a kernel
// written with MJ_KERNEL, launched merged over njobs argument structs with
// uneven grids, must see in every workgroup its own launch's argument
// struct, block index and grid size -- for launch counts on both sides of
// one and two rounds of the wave's search, and for workgroups of one full
// wave, several waves and a partial last wave.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "mj_device.h"

namespace {

struct ProbeArgs {
    uint32_t job;          // this launch's index
    uint32_t* seen;        // [blocks of the merged grid] (job << 16 | bid), by first block of the launch
    uint32_t first;        // first block of this launch in the merged grid
    uint32_t* nblk_seen;   // [njobs]
};

MJ_KERNEL(k_probe_multi, 256, ProbeArgs) {
    if (threadIdx.x == 0) {
        A.seen[A.first + vg.bid] = (A.job << 16) | vg.bid;
        A.nblk_seen[A.job] = vg.nblk;
    }
}

int fails = 0;

void run(uint32_t njobs, uint32_t block, std::mt19937& g) {
    std::vector<ProbeArgs> args(njobs);
    std::vector<uint32_t> base(njobs + 1, 0), grid(njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        grid[j] = 1 + g() % (j % 7 == 0 ? 9 : 2);
        base[j + 1] = base[j] + grid[j];
    }
    const uint32_t total = base[njobs];
    std::vector<uint32_t> seen(total, 0xFFFFFFFFu), nblk(njobs, 0);
    for (uint32_t j = 0; j < njobs; ++j) args[j] = ProbeArgs{j, seen.data(), base[j], nblk.data()};
    mj::MultiGrid M{args.data(), base.data(), njobs};
    hipLaunchKernelGGL(k_probe_multi_multi, dim3(total), dim3(block), 0, nullptr, M);
    bool ok = true;
    for (uint32_t j = 0; j < njobs && ok; ++j) {
        ok = nblk[j] == grid[j];
        for (uint32_t b = 0; b < grid[j] && ok; ++b) ok = seen[base[j] + b] == ((j << 16) | b);
    }
    std::printf("[multi] %5u launches, %4u threads a workgroup: %s\n", njobs, block, ok ? "ok" : "FAILED");
    if (!ok) ++fails;
}

}  // namespace

int main() {
    std::mt19937 g(12345);
    for (uint32_t njobs : {1u, 2u, 3u, 63u, 64u, 65u, 100u, 129u, 512u, 4095u, 4096u, 4097u, 6000u})
        for (uint32_t block : {64u, 96u, 256u})
            run(njobs, block, g);
    std::printf("[multi] %s\n", fails ? "FAILED" : "all checks passed");
    return fails ? 1 : 0;
}
