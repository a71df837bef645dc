// Plain float32 kernels, kept for comparison with the tiled pair kernels at
// the same accuracy: one thread per target particle, sources read straight
// from global memory over the 27-cell stencil, the cut-off as a branch, and
// sums in float64 (the simple way to reach the accuracy that the tiled
// kernels get from compensated float32 sums).  The pair arithmetic is the
// tiled kernels' float32 formula, with the grid polynomial in the same
// well-conditioned basis.  No LDS staging, source culling, work list or
// lane splitting.  They compute the same operation (Habib et al. 2012,
// Sec. III, Eq. 7, and its vector-Jacobian product) on the same binned
// records; they are not on the library's main path.
#include "common.h"

// A plain implementation lets the compiler fuse multiply-adds as it likes.
#pragma clang fp contract(fast)

namespace hsr {

namespace {

constexpr int kBlock = 256;

struct Stencil {
    int key[27];
    float sx[27], sy[27], sz[27];
    int m;
};

// Stencil cells of a cell and the shift that moves their records into the
// cell's frame (periodic wrap or open-domain clipping).
__device__ __forceinline__ void stencil(int cell, const Geom& g, Stencil* S) {
    const int N = g.N;
    const int cz = cell % N, cy = (cell / N) % N, cx = cell / (N * N);
    S->m = 0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                int x = cx + a, y = cy + b, z = cz + c;
                if (g.periodic) {
                    x = (x + N) % N;
                    y = (y + N) % N;
                    z = (z + N) % N;
                } else if (x < 0 || x >= N || y < 0 || y >= N || z < 0 || z >= N) {
                    continue;
                }
                S->key[S->m] = (x * N + y) * N + z;
                S->sx[S->m] = (float)a * g.Lc_f;
                S->sy[S->m] = (float)b * g.Lc_f;
                S->sz[S->m] = (float)c * g.Lc_f;
                ++S->m;
            }
}

__global__ __launch_bounds__(kBlock) void k_force_plain(
    const float4* __restrict__ rec, const int* __restrict__ keys,
    const int* __restrict__ cs, const int* __restrict__ perm, int n, Geom g,
    PairParams P, float* __restrict__ out) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    Stencil S;
    stencil(keys[k] >> g.sbits, g, &S);
    const float4 xi = rec[k];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int q = 0; q < S.m; ++q) {
        const int end = cs[S.key[q] + 1];
        for (int j = cs[S.key[q]]; j < end; ++j) {
            const float4 pj = rec[j];
            const float dx = (pj.x + S.sx[q]) - xi.x;
            const float dy = (pj.y + S.sy[q]) - xi.y;
            const float dz = (pj.z + S.sz[q]) - xi.z;
            const float u = dx * dx + dy * dy + dz * dz + P.eps;
            if (u < P.rc2e) {
                const float y = rsqrtf(u);
                const float t = u * P.alpha + P.beta;
                const float p =
                    ((((P.b[5] * t + P.b[4]) * t + P.b[3]) * t + P.b[2]) * t + P.b[1]) * t + P.b[0];
                const float mf = pj.w * (y * y * y - p);
                ax += (double)(mf * dx);
                ay += (double)(mf * dy);
                az += (double)(mf * dz);
            }
        }
    }
    const int64_t o = 3 * (int64_t)perm[k];
    out[o] = (float)ax;
    out[o + 1] = (float)ay;
    out[o + 2] = (float)az;
}

__global__ __launch_bounds__(kBlock) void k_vjp_plain(
    const float4* __restrict__ rec, const float4* __restrict__ gs,
    const int* __restrict__ keys, const int* __restrict__ cs,
    const int* __restrict__ perm, int n, Geom g, PairParams P,
    double* __restrict__ out) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    Stencil S;
    stencil(keys[k] >> g.sbits, g, &S);
    const float4 xk = rec[k];
    const float4 gk = gs[k];
    double ox = 0.0, oy = 0.0, oz = 0.0;
    for (int q = 0; q < S.m; ++q) {
        const int end = cs[S.key[q] + 1];
        for (int j = cs[S.key[q]]; j < end; ++j) {
            const float4 pj = rec[j];
            const float4 gj = gs[j];
            const float dx = (pj.x + S.sx[q]) - xk.x;
            const float dy = (pj.y + S.sy[q]) - xk.y;
            const float dz = (pj.z + S.sz[q]) - xk.z;
            const float u = dx * dx + dy * dy + dz * dz + P.eps;
            if (u < P.rc2e) {
                const float y = rsqrtf(u);
                const float y3 = y * y * y;
                const float t = u * P.alpha + P.beta;
                const float p =
                    ((((P.b[5] * t + P.b[4]) * t + P.b[3]) * t + P.b[2]) * t + P.b[1]) * t + P.b[0];
                // 2 f'(s) = -3 y^5 - 2 poly'(s)
                const float dp2 =
                    (((P.db2[4] * t + P.db2[3]) * t + P.db2[2]) * t + P.db2[1]) * t + P.db2[0];
                const float f = y3 - p;
                const float f2 = -3.0f * y3 * y * y - dp2;
                const float wx = xk.w * gj.x - pj.w * gk.x;
                const float wy = xk.w * gj.y - pj.w * gk.y;
                const float wz = xk.w * gj.z - pj.w * gk.z;
                const float c = f2 * (dx * wx + dy * wy + dz * wz);
                ox += (double)(f * wx + c * dx);
                oy += (double)(f * wy + c * dy);
                oz += (double)(f * wz + c * dz);
            }
        }
    }
    const int64_t o = 3 * (int64_t)perm[k];
    out[o] = ox;
    out[o + 1] = oy;
    out[o + 2] = oz;
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_force_plain(const float4* rec, const int* keys_sorted,
                              const int* cell_start, const int* perm, int n,
                              Geom g, PairParams p, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_force_plain, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                       0, st, rec, keys_sorted, cell_start, perm, n, g, p, out);
    return hipGetLastError();
}

hipError_t launch_vjp_plain(const float4* rec, const float4* gsorted,
                            const int* keys_sorted, const int* cell_start,
                            const int* perm, int n, Geom g, PairParams p,
                            double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vjp_plain, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                       0, st, rec, gsorted, keys_sorted, cell_start, perm, n, g,
                       p, out);
    return hipGetLastError();
}

}  // namespace hsr
