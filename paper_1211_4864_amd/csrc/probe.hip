// Instruction-rate probes of the float32 vector ALU, for measurement only
// (not on the force path).  They give the peak that the pair kernels are
// held to at the clock the chip actually sustains under a VALU load:
//
//   kind 0: float32 fused multiply-add, 16 independent chains per lane;
//   kind 1: float32 reciprocal square root (v_rsq_f32), 16 chains;
//   kind 2: the forward pair term's mix, 1 reciprocal square root per
//           18 float32 FMAs, 16 interleaved chains;
//   kind 3: float32 FMA accumulating into its destination (v_fmac_f32, the
//           short encoding), 16 chains.
//
// A launch puts W waves on every SIMD (4 W one-wave workgroups per compute
// unit).  Every wave reads the shader-clock counter and the constant-rate
// wall clock around its loop, so the host gets the instruction rate, the
// shader clock during the run and the cycles between one wave's
// instructions.  Operands live in vector registers (a VALU instruction may
// read one scalar register only), the chains are independent so that issue
// rather than latency sets the rate, and the build disables packed float32,
// so every FMA is a plain v_fma_f32.
#include "common.h"

namespace hsr {

namespace {

constexpr int kProbeBlock = 64;     // one wave per workgroup
constexpr int kMaxProbeWaves = 8 * 1024;
constexpr int kChains = 16;

__device__ __forceinline__ float vreg(float s) {
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

template <int KIND>
__global__ __launch_bounds__(kProbeBlock) void k_valu_probe(
    int iters, float a_s, float b_s, float* __restrict__ sink,
    unsigned long long* __restrict__ clocks) {
    const float a = vreg(a_s), b = vreg(b_s);
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = 1.0f + 1e-3f * (float)(threadIdx.x + c);
    __syncthreads();
    const unsigned long long c0 = clock64();
    const unsigned long long w0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (KIND == 0) {
                x[c] = __builtin_fmaf(x[c], a, b);          // v_fma_f32 (VOP3)
            } else if (KIND == 1) {
                x[c] = __builtin_amdgcn_rsqf(x[c]);
            } else if (KIND == 3) {
                x[c] = __builtin_fmaf(a, b, x[c]);          // v_fmac_f32 (VOP2)
            }
        }
        if (KIND == 2) {
            // 1 rsq + 18 FMA per chain, the chains interleaved: the forward
            // pair term's instruction mix without its loads
#pragma unroll
            for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_rsqf(x[c]);
#pragma unroll
            for (int q = 0; q < 18; ++q)
#pragma unroll
                for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
        }
    }
    const unsigned long long c1 = clock64();
    const unsigned long long w1 = wall_clock64();
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    sink[blockIdx.x * kProbeBlock + threadIdx.x] = s;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int w = blockIdx.x * (kProbeBlock / kWave) + threadIdx.x / kWave;
        clocks[2 * w] = c1 - c0;
        clocks[2 * w + 1] = w1 - w0;
    }
}

}  // namespace

size_t probe_scratch_bytes() {
    return sizeof(float) * (size_t)kMaxProbeWaves * kWave +
           sizeof(unsigned long long) * 2 * (size_t)kMaxProbeWaves;
}

size_t probe_clock_offset() { return sizeof(float) * (size_t)kMaxProbeWaves * kWave; }

int probe_ops_per_iter(int kind) {
    return kind == 2 ? kChains * 19 : kChains;
}

hipError_t launch_valu_probe(int kind, int waves, int iters, void* scratch,
                             hipStream_t st) {
    if (waves <= 0 || waves > kMaxProbeWaves) return hipErrorInvalidValue;
    float* sink = reinterpret_cast<float*>(scratch);
    unsigned long long* clocks = reinterpret_cast<unsigned long long*>(
        reinterpret_cast<char*>(scratch) + probe_clock_offset());
    const float a = 0.999f, b = 1e-3f;
    switch (kind) {
        case 0:
            hipLaunchKernelGGL(k_valu_probe<0>, dim3(waves), dim3(kProbeBlock),
                               0, st, iters, a, b, sink, clocks);
            break;
        case 1:
            hipLaunchKernelGGL(k_valu_probe<1>, dim3(waves), dim3(kProbeBlock),
                               0, st, iters, a, b, sink, clocks);
            break;
        case 2:
            hipLaunchKernelGGL(k_valu_probe<2>, dim3(waves), dim3(kProbeBlock),
                               0, st, iters, a, b, sink, clocks);
            break;
        case 3:
            hipLaunchKernelGGL(k_valu_probe<3>, dim3(waves), dim3(kProbeBlock),
                               0, st, iters, a, b, sink, clocks);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hsr
