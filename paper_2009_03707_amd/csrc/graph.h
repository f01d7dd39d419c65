// Host-side input of the MS-complex graph (graph.cpp): the critical list and
// the six arc matrices of one result, copied to host memory by ms_graph_build
// (api.hip).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/msc.h"

namespace msc {

struct HostCsr {
    int64_t nrows = 0, ncols = 0;
    std::vector<int64_t> rowptr;  // nrows + 1
    std::vector<uint32_t> col;
    std::vector<uint64_t> val;
};

struct GraphInput {
    int64_t dims[3] = {0, 0, 0};
    int64_t count[4] = {0, 0, 0, 0};
    std::vector<uint32_t> id, vmax;
    std::vector<uint8_t> index;
    std::vector<float> value;
    // down and up arcs of every index: M10, M10^T, M21, M21^T, M32, M32^T
    HostCsr m10, m10t, m21, m21t, m32, m32t;
};

// Builds the graph (one worker per range of nodes and direction); returns
// null and sets *err on failure (e.g. an inconsistent input).
ms_graph* graph_from_host(GraphInput& in, int nthreads, std::string* err);

}  // namespace msc
