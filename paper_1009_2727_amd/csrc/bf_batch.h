// bf_batch.h -- launches of one step of several runs, gathered per phase, so that a batch of
// independent runs executes Faraday, the electron push and Ampere as one persistent launch each
// over a device work queue (the other phases run as the runs' own launches, in phase order).
#pragma once
#include <functional>
#include <utility>
#include <vector>
#include "bf_kernels.h"

namespace bf {

// phases of a step in execution order
enum {
    SLOT_FARADAY, SLOT_STATIONS, SLOT_PUSH, SLOT_IONS, SLOT_ANTENNA, SLOT_FILTER, SLOT_AMPERE,
    SLOT_WINDOW, SLOT_SORT, SLOT_COUNT
};

struct BatchRec {
    std::vector<FaradayDesc<float>> faraday;
    std::vector<AmpereDesc<float>> ampere;
    std::vector<GpdDesc<float>> gpd;
    // work items of each descriptor (cell blocks or particle segments)
    std::vector<int> n_faraday, n_ampere, n_gpd;
    // each run's own launches by phase slot, with the run's index in the batch
    std::vector<std::pair<int, std::function<void(hipStream_t)>>> slots[SLOT_COUNT];

    void clear()
    {
        faraday.clear(); ampere.clear(); gpd.clear();
        n_faraday.clear(); n_ampere.clear(); n_gpd.clear();
        for (auto& v : slots) v.clear();
    }
};

}  // namespace bf
