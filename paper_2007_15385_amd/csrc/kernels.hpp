// Host-side launchers of the HIP kernels (private to the library).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace pipdev {

enum TestKind : int { K_VORONOI = 0, K_SOO = 1, K_RAY = 2, K_PLAIN = 3, K_MARGIN = 4 };

struct StreamLaunch {
    int kind;             // TestKind
    const double* V;      // device [n][2]
    int n;
    const void* Q;        // device [m][2], float32 or binary64
    int qdt;              // 0 float32, 1 binary64
    int64_t m;
    uint32_t* labels;     // device [ceil(m/32)]
    float* margin;        // device [m] (margin kernel only)
    int32_t* status;      // device [1] or null
    int max_blocks;       // upper bound on the persistent grid
    hipStream_t stream;
};

hipError_t launch_stream(const StreamLaunch& L);
hipError_t launch_generators_one(const double* V, int n, double* P, int32_t* status,
                                 hipStream_t stream);
hipError_t stream_max_blocks_per_cu(int kind, int qdt, int* out);

}  // namespace pipdev
