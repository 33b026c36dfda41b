// tuned_blocks.h — candidate block sizes measured by paper_2601_01405_amd/autotune.py
// on no device: the untuned defaults: the fastest B of each (n, d) bucket for single builds and for
// batches of same-bucket clouds (clustered clouds, a singleton-ball radius and a
// radius inside the clusters).  Generated; rerun the tuner to refresh.
#pragma once
#include <stdint.h>

namespace bm {

struct TunedBlock {
    int64_t n_min;      // the bucket holds n >= n_min (up to the next row's n_min)
    int32_t d_max;      // and d <= d_max (above the previous row's d_max)
    int32_t single;     // B for one build
    int32_t batch;      // B for each chain of a batch
};

constexpr TunedBlock kTunedBlocks[] = {
    {0, 8, 64, 256},
    {0, 16, 64, 256},
    {0, 32, 64, 256},
    {0, 64, 64, 256},
    {0, 128, 64, 256},
    {0, 256, 64, 256},
    {2048, 8, 64, 256},
    {2048, 16, 64, 256},
    {2048, 32, 64, 256},
    {2048, 64, 64, 256},
    {2048, 128, 64, 256},
    {2048, 256, 64, 256},
    {8192, 8, 256, 1024},
    {8192, 16, 256, 1024},
    {8192, 32, 256, 1024},
    {8192, 64, 256, 1024},
    {8192, 128, 256, 1024},
    {8192, 256, 256, 1024},
    {32768, 8, 256, 2048},
    {32768, 16, 256, 2048},
    {32768, 32, 256, 2048},
    {32768, 64, 256, 2048},
    {32768, 128, 256, 2048},
    {32768, 256, 256, 2048},
    {131072, 8, 8192, 4096},
    {131072, 16, 8192, 4096},
    {131072, 32, 8192, 4096},
    {131072, 64, 8192, 4096},
    {131072, 128, 8192, 4096},
    {131072, 256, 8192, 4096},
};

} // namespace bm
