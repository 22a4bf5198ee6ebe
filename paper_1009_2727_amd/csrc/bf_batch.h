// bf_batch.h -- launches of one step of several runs, gathered per phase, so that a batch of
// independent runs executes each heavy phase as one persistent launch over a device work queue
// (the light phases run as the runs' own launches, in phase order).
#pragma once
#include <functional>
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
    std::vector<FilterDesc<float>> filter;
    std::vector<GpdDesc<float>> gpd;
    std::vector<IonDesc<float>> ion;
    // work items of each descriptor (blocks, tiles or particle segments)
    std::vector<int> n_faraday, n_ampere, n_filter, n_gpd, n_ion;
    int max_halo = 0;
    std::vector<std::function<void(hipStream_t)>> slots[SLOT_COUNT];

    void clear()
    {
        faraday.clear(); ampere.clear(); filter.clear(); gpd.clear(); ion.clear();
        n_faraday.clear(); n_ampere.clear(); n_filter.clear(); n_gpd.clear(); n_ion.clear();
        max_halo = 0;
        for (auto& v : slots) v.clear();
    }
};

}  // namespace bf
