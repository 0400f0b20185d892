// Captured iteration chunk of the flexible CG, cached per network: a network
// alternating with others on one lattice keeps its own graph.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace hisq {

struct FcgGraphCache {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string key;   // every launch argument the chunk holds by value
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
};

}  // namespace hisq
