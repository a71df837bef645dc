// Long-range spectral particle-mesh (PM) force (Habib et al. 2012, Sec. II):
// Cloud-In-Cell deposit of the masses on a periodic ng^3 grid, a forward
// 3-D FFT, the isotropising filter of Eq. 5 times the sixth-order periodic
// influence function, fourth-order spectral differencing of the potential
// (one inverse FFT per component), and CIC interpolation back to the
// particles.
//
// Readings where the paper names an operator only by its order: the
// influence function is the inverse of the Fourier symbol of the
// sixth-order central-difference Laplacian,
//   K6(k) = sum_a [6 sin^2(k_a D/2) - 0.6 sin^2(k_a D) + (2/45) sin^2(3 k_a D/2)] / D^2
// (the same polynomial in cos(k_a D) as 49/18 - 3 cos + 3/10 cos 2 - 1/45
// cos 3, written without its cancelling constant); the gradient symbol is
// that of the fourth-order central difference, (4/3 sin(k_a D) -
// 1/6 sin(2 k_a D)) / D; the filter's sinc is read as
// [sin(k D/2) / (k D/2)]^n_s with k = |k|, sigma in grid cells.
//
// Layout and precision: the grid is complex float32 (ng^3 float2, z
// fastest).  The deposit accumulates fixed-point int64 (2^62 / (n max|m|)
// per unit mass), so the density does not depend on the order of the
// atomic additions and the whole solve is bitwise reproducible.  The FFT is
// radix 2, one axis per pass: a workgroup loads a tile of lines into LDS
// (lines adjacent in memory, so that the loads of the strided axes are
// coalesced), bit-reverses on the way in, runs log2(ng) butterfly stages
// with twiddles from a float32 table, and writes the tile back.
#include <algorithm>

#include "common.h"

namespace hsr {

namespace {

constexpr int kPB = 256;
constexpr float kPi = 3.14159265358979323846f;

// ---- deposit

// Largest |mass|, as the bit pattern of a non-negative float (ordered like
// an unsigned integer), for the fixed-point scale.
__global__ __launch_bounds__(kPB) void k_pm_mass_max(const float* __restrict__ mass, int n,
                                                     unsigned* __restrict__ out) {
    const int i = blockIdx.x * kPB + threadIdx.x;
    unsigned v = i < n ? __float_as_uint(fabsf(mass[i])) : 0u;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v = max(v, (unsigned)__shfl_xor((int)v, o));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, v);
}

// Lower grid index and the CIC fraction of a coordinate (grid point g at
// g D, periodic).
__device__ __forceinline__ int cic_axis(double x, double inv_d, int ng, double* frac) {
    double u = x * inv_d;
    u -= (double)ng * floor(u / (double)ng);
    double fl = floor(u);
    int i = (int)fl;
    double f = u - fl;
    if (i >= ng) { i -= ng; }
    if (i < 0) { i = 0; f = 0.0; }        // non-finite positions
    *frac = f;
    return i;
}

__global__ __launch_bounds__(kPB) void k_pm_deposit(const double* __restrict__ pos,
                                                    const float* __restrict__ mass, int n,
                                                    int ng, double inv_d,
                                                    const unsigned* __restrict__ mmax_bits,
                                                    unsigned long long* __restrict__ grid) {
    const int i = blockIdx.x * kPB + threadIdx.x;
    if (i >= n) return;
    const double mmax = (double)__uint_as_float(*mmax_bits);
    if (!(mmax > 0.0)) return;
    const double scale = 4611686018427387904.0 / ((double)n * mmax);   // 2^62
    double f[3];
    int g0[3];
    for (int a = 0; a < 3; ++a) g0[a] = cic_axis(pos[3 * (int64_t)i + a], inv_d, ng, &f[a]);
    const double m = (double)mass[i] * scale;
    for (int c = 0; c < 8; ++c) {
        const int bx = c >> 2, by = (c >> 1) & 1, bz = c & 1;
        const double w = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) *
                         (bz ? f[2] : 1.0 - f[2]);
        const int x = g0[0] + bx == ng ? 0 : g0[0] + bx;
        const int y = g0[1] + by == ng ? 0 : g0[1] + by;
        const int z = g0[2] + bz == ng ? 0 : g0[2] + bz;
        const long long q = llrint(m * w);
        atomicAdd(&grid[((int64_t)x * ng + y) * ng + z], (unsigned long long)q);
    }
}

// Fixed-point mass to complex density (mass / D^3), imaginary part zero.
__global__ __launch_bounds__(kPB) void k_pm_density(const unsigned long long* __restrict__ q,
                                                    int64_t cells, int n,
                                                    const unsigned* __restrict__ mmax_bits,
                                                    double inv_vol, float2* __restrict__ rho) {
    const int64_t c = blockIdx.x * (int64_t)kPB + threadIdx.x;
    if (c >= cells) return;
    const double mmax = (double)__uint_as_float(*mmax_bits);
    const double unit = mmax > 0.0 ? ((double)n * mmax) / 4611686018427387904.0 : 0.0;
    rho[c] = make_float2((float)((double)(long long)q[c] * unit * inv_vol), 0.0f);
}

// ---- FFT

// tw[k] = exp(-2 pi i k / ng), k < ng / 2.
__global__ __launch_bounds__(kPB) void k_twiddles(int ng, float2* __restrict__ tw) {
    const int k = blockIdx.x * kPB + threadIdx.x;
    if (k >= ng / 2) return;
    float s, c;
    sincospif(2.0f * (float)k / (float)ng, &s, &c);
    tw[k] = make_float2(c, -s);
}

// One radix-2 FFT pass along `axis` (0: x, stride ng^2; 1: y, stride ng;
// 2: z, contiguous) over tiles of tl lines.  sign -1: forward, +1: inverse
// (unnormalised).
__global__ __launch_bounds__(kPB) void k_fft_pass(float2* __restrict__ data, int ng, int lg,
                                                  int axis, int tl, int sign,
                                                  const float2* __restrict__ tw) {
    extern __shared__ float2 sm[];
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t ng2 = (int64_t)ng * ng;
    int64_t base0, lstride, estride;       // line t of the tile: base0 + t lstride
    if (axis == 2) {
        base0 = (int64_t)g * tl * ng;
        lstride = ng;
        estride = 1;
    } else {
        const int per = ng / tl;           // tiles per row of lines
        const int outer = g / per, z0 = (g % per) * tl;
        base0 = axis == 1 ? (int64_t)outer * ng2 + z0 : (int64_t)outer * ng + z0;
        lstride = 1;
        estride = axis == 1 ? ng : ng2;
    }
    const int tot = tl * ng;
    for (int idx = tid; idx < tot; idx += kPB) {
        int t, j;
        if (axis == 2) { t = idx / ng; j = idx - t * ng; }
        else { j = idx / tl; t = idx - j * tl; }
        const float2 v = data[base0 + t * lstride + j * estride];
        const int r = (int)(__brev((unsigned)j) >> (32 - lg));
        sm[t * ng + r] = v;
    }
    __syncthreads();
    const int nb = tot / 2;                // butterflies per stage
    for (int half = 1, tstep = ng / 2; half < ng; half <<= 1, tstep >>= 1) {
        for (int b = tid; b < nb; b += kPB) {
            const int t = b / (ng / 2);
            const int q = b - t * (ng / 2);
            const int grp = q / half, p = q - grp * half;
            const int i0 = t * ng + grp * 2 * half + p, i1 = i0 + half;
            float2 w = tw[p * tstep];
            if (sign > 0) w.y = -w.y;
            const float2 a = sm[i0], x = sm[i1];
            const float2 m = make_float2(w.x * x.x - w.y * x.y, w.x * x.y + w.y * x.x);
            sm[i0] = make_float2(a.x + m.x, a.y + m.y);
            sm[i1] = make_float2(a.x - m.x, a.y - m.y);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < tot; idx += kPB) {
        int t, j;
        if (axis == 2) { t = idx / ng; j = idx - t * ng; }
        else { j = idx / tl; t = idx - j * tl; }
        data[base0 + t * lstride + j * estride] = sm[t * ng + j];
    }
}

// ---- k space

__device__ __forceinline__ int freq(int m, int ng) { return m < ng / 2 ? m : m - ng; }

// phi(k) = -4 pi S(k) rho(k) / K6(k), in place; phi(0) = 0.
__global__ __launch_bounds__(kPB) void k_pm_potential(float2* __restrict__ a, int ng,
                                                      float d, float sigma, int n_s) {
    const int64_t c = blockIdx.x * (int64_t)kPB + threadIdx.x;
    const int64_t cells = (int64_t)ng * ng * ng;
    if (c >= cells) return;
    const int mz = (int)(c % ng), my = (int)((c / ng) % ng), mx = (int)(c / ((int64_t)ng * ng));
    if (mx == 0 && my == 0 && mz == 0) {
        a[c] = make_float2(0.0f, 0.0f);
        return;
    }
    const int f[3] = {freq(mx, ng), freq(my, ng), freq(mz, ng)};
    float k6 = 0.0f, k2 = 0.0f;
    for (int q = 0; q < 3; ++q) {
        const float th = (float)f[q] / (float)ng;      // k_q D / (2 pi)
        const float s1 = sinpif(th), s2 = sinpif(2.0f * th), s3 = sinpif(3.0f * th);
        k6 += 6.0f * s1 * s1 - 0.6f * s2 * s2 + (2.0f / 45.0f) * s3 * s3;
        const float kq = 2.0f * kPi * th / d;
        k2 += kq * kq;
    }
    k6 /= d * d;
    const float kmag = sqrtf(k2);
    const float x = 0.5f * kmag * d;
    const float sinc = sinf(x) / x;
    float S = expf(-0.25f * k2 * sigma * sigma * d * d);
    for (int q = 0; q < n_s; ++q) S *= sinc;
    const float g = -4.0f * kPi * S / k6;
    const float2 v = a[c];
    a[c] = make_float2(g * v.x, g * v.y);
}

// out(k) = -i D_axis(k) phi(k).
__global__ __launch_bounds__(kPB) void k_pm_gradient(const float2* __restrict__ phi,
                                                     float2* __restrict__ out, int ng,
                                                     float d, int axis) {
    const int64_t c = blockIdx.x * (int64_t)kPB + threadIdx.x;
    const int64_t cells = (int64_t)ng * ng * ng;
    if (c >= cells) return;
    const int m = axis == 2 ? (int)(c % ng)
                            : (axis == 1 ? (int)((c / ng) % ng) : (int)(c / ((int64_t)ng * ng)));
    const float th = (float)freq(m, ng) / (float)ng;
    const float dk = ((4.0f / 3.0f) * sinpif(2.0f * th) - (1.0f / 6.0f) * sinpif(4.0f * th)) / d;
    const float2 v = phi[c];
    // -i dk (x + i y) = dk y - i dk x
    out[c] = make_float2(dk * v.y, -dk * v.x);
}

// Acceleration component at the particles: CIC interpolation of the real
// part of the inverse transform, scaled by 1 / ng^3.
__global__ __launch_bounds__(kPB) void k_pm_interp(const double* __restrict__ pos, int n,
                                                   int ng, double inv_d,
                                                   const float2* __restrict__ grid, float norm,
                                                   int axis, float* __restrict__ out) {
    const int i = blockIdx.x * kPB + threadIdx.x;
    if (i >= n) return;
    double f[3];
    int g0[3];
    for (int a = 0; a < 3; ++a) g0[a] = cic_axis(pos[3 * (int64_t)i + a], inv_d, ng, &f[a]);
    float acc = 0.0f;
    for (int c = 0; c < 8; ++c) {
        const int bx = c >> 2, by = (c >> 1) & 1, bz = c & 1;
        const float w = (float)((bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) *
                                (bz ? f[2] : 1.0 - f[2]));
        const int x = g0[0] + bx == ng ? 0 : g0[0] + bx;
        const int y = g0[1] + by == ng ? 0 : g0[1] + by;
        const int z = g0[2] + bz == ng ? 0 : g0[2] + bz;
        acc = __builtin_fmaf(w, grid[((int64_t)x * ng + y) * ng + z].x, acc);
    }
    out[3 * (int64_t)i + axis] = acc * norm;
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

size_t pm_workspace_bytes(int ng) {
    const size_t cells = (size_t)ng * ng * ng;
    // two complex grids, the twiddles, the mass maximum; the fixed-point
    // deposit reuses the second complex grid (8 bytes per cell)
    return 2 * (cells * sizeof(float2) + 256) + ((size_t)ng / 2 * sizeof(float2) + 256) + 256;
}

hipError_t launch_pm_accel(const double* pos, const float* mass, int n, double box, int ng,
                           float sigma, int n_s, void* ws, float* out_acc, hipStream_t st) {
    const int64_t cells = (int64_t)ng * ng * ng;
    int lg = 0;
    while ((1 << lg) < ng) ++lg;
    auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* p = reinterpret_cast<char*>(ws);
    float2* A = reinterpret_cast<float2*>(p);
    p += align(cells * sizeof(float2));
    float2* B = reinterpret_cast<float2*>(p);
    unsigned long long* Q = reinterpret_cast<unsigned long long*>(B);
    p += align(cells * sizeof(float2));
    float2* tw = reinterpret_cast<float2*>(p);
    p += align((size_t)ng / 2 * sizeof(float2));
    unsigned* mmax = reinterpret_cast<unsigned*>(p);
    const double d = box / ng;
    const double inv_d = (double)ng / box;
    hipError_t e = launch_fill_i32(reinterpret_cast<int*>(mmax), 1, 0, st);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(reinterpret_cast<int*>(Q), (int)(2 * cells), 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_twiddles, dim3(blocks_for(ng / 2, kPB)), dim3(kPB), 0, st, ng, tw);
    if (n > 0) {
        hipLaunchKernelGGL(k_pm_mass_max, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st, mass, n,
                           mmax);
        hipLaunchKernelGGL(k_pm_deposit, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st, pos,
                           mass, n, ng, inv_d, (const unsigned*)mmax, Q);
    }
    hipLaunchKernelGGL(k_pm_density, dim3(blocks_for(cells, kPB)), dim3(kPB), 0, st,
                       (const unsigned long long*)Q, cells, n, (const unsigned*)mmax,
                       1.0 / (d * d * d), A);
    const int tl = std::max(1, std::min(std::min(16, ng), 4096 / ng));
    const size_t shm = (size_t)tl * ng * sizeof(float2);
    const int tiles = (int)(((int64_t)ng * ng) / tl);
    auto fft = [&](float2* g, int sign) {
        for (int axis = 2; axis >= 0; --axis)
            hipLaunchKernelGGL(k_fft_pass, dim3(tiles), dim3(kPB), shm, st, g, ng, lg, axis,
                               tl, sign, (const float2*)tw);
    };
    fft(A, -1);
    hipLaunchKernelGGL(k_pm_potential, dim3(blocks_for(cells, kPB)), dim3(kPB), 0, st, A, ng,
                       (float)d, sigma, n_s);
    const float norm = (float)(1.0 / (double)cells);
    for (int axis = 0; axis < 3; ++axis) {
        hipLaunchKernelGGL(k_pm_gradient, dim3(blocks_for(cells, kPB)), dim3(kPB), 0, st,
                           (const float2*)A, B, ng, (float)d, axis);
        fft(B, +1);
        if (n > 0)
            hipLaunchKernelGGL(k_pm_interp, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st, pos, n,
                               ng, inv_d, (const float2*)B, norm, axis, out_acc);
    }
    return hipGetLastError();
}

}  // namespace hsr
