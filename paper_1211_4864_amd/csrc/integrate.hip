// Kick and stream maps of the symmetric stream-kick-stream subcycle
// (Habib et al. 2012, Sec. II, Eq. 6), in float64, and the kick's adjoint.
// Memory-bound elementwise updates over the 3n components.
#include "common.h"

namespace hsr {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t m) {
    const int64_t b = (m + kBlock - 1) / kBlock;
    return (int)(b < 65536 ? b : 65536);
}

__global__ __launch_bounds__(kBlock) void k_kick(double* __restrict__ vel,
                                                 const float* __restrict__ acc,
                                                 int64_t m, double dt) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * kBlock)
        vel[k] = __builtin_fma(dt, (double)acc[k], vel[k]);
}

__global__ __launch_bounds__(kBlock) void k_stream(double* __restrict__ pos,
                                                   const double* __restrict__ vel,
                                                   int64_t m, double dt,
                                                   double box) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * kBlock) {
        double x = __builtin_fma(dt, vel[k], pos[k]);
        if (box > 0.0) {
            x = x - box * floor(x / box);
            if (x >= box) x -= box;
        }
        pos[k] = x;
    }
}

__global__ __launch_bounds__(kBlock) void k_kick_adjoint(
    const double* __restrict__ gv, float* __restrict__ ga, int64_t m, double dt) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * kBlock)
        ga[k] = (float)(dt * gv[k]);
}

}  // namespace

hipError_t launch_kick(double* vel, const float* acc, int64_t m, double dt,
                       hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick, dim3(grid_for(m)), dim3(kBlock), 0, st, vel, acc,
                       m, dt);
    return hipGetLastError();
}

hipError_t launch_stream(double* pos, const double* vel, int64_t m, double dt,
                         double box, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream, dim3(grid_for(m)), dim3(kBlock), 0, st, pos,
                       vel, m, dt, box);
    return hipGetLastError();
}

hipError_t launch_kick_adjoint(const double* gv, float* ga, int64_t m,
                               double dt, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_adjoint, dim3(grid_for(m)), dim3(kBlock), 0, st,
                       gv, ga, m, dt);
    return hipGetLastError();
}

}  // namespace hsr
