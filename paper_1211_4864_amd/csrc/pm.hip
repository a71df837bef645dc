// Long-range spectral particle-mesh (PM) force (Habib et al. 2012, Sec. II):
// Cloud-In-Cell deposit of the masses on a periodic ng^3 grid, a forward
// 3-D FFT, the isotropising filter of Eq. 5 times the sixth-order periodic
// influence function, fourth-order spectral differencing of the potential,
// inverse FFTs and CIC interpolation back to the particles.
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
// Layout and order of work (grids complex float32, ng^3 float2, z fastest):
//  - One pass over the particles writes the grid cell of each particle's
//    lower CIC corner and a record (the three CIC fractions and the mass,
//    float32).  The particles are sorted by that cell (a stable LSD radix sort
//    of the cell index) and their records gathered into that order, so that
//    the deposit and the interpolation read the records contiguously and
//    touch the grid locally.
//  - Deposit: each particle adds m w 2^62 / (n max|m|), rounded to int64, to
//    its 8 corners.  A wave first sums the contributions of its particles
//    that share a cell (a segmented scan over the sorted keys), so only one
//    atomic per cell and wave reaches memory.  Integer sums do not depend on
//    the order of the additions: the whole solve is bitwise reproducible.
//  - FFT: one kernel per axis.  A workgroup transforms L lines of ng points
//    as ng = R1 x R2 (the four-step method): each thread does a length-R1
//    DFT in registers, multiplies by the twiddles of the length-ng transform
//    and passes its values through LDS to the threads of a length-R2 DFT.
//    For the strided axes the L lines are adjacent in memory, so that the
//    loads and stores of a wave are contiguous over the lines.
//  - The first forward pass reads the fixed-point deposit.  The last forward
//    pass (x) applies the potential's and the gradient's symbols to its
//    lines in registers and runs the inverse x pass of the two output grids
//    at once: B = (D_y - i D_x) phi (its inverse is a_x + i a_y, both real)
//    and A = -i D_z phi (its inverse has a_z as real part).  The inverse y
//    and z passes take both grids in one launch, and one interpolation
//    kernel reads a_x, a_y and a_z at the 8 corners.  1 / ng^3 is folded
//    into the potential.
#include <algorithm>

#include "common.h"

namespace hsr {

namespace {

constexpr int kPB = 256;
constexpr float kPi = 3.14159265358979323846f;

// ---- mass maximum, for the fixed-point scale

constexpr int kMaxBlocks = 1024;

// Largest |mass| as the bit pattern of a non-negative float (ordered like
// an unsigned integer): a grid-stride maximum per thread, reduced over the
// workgroup, one atomic per workgroup.
__global__ __launch_bounds__(kPB) void k_pm_mass_max(const float* __restrict__ mass, int n,
                                                     unsigned* __restrict__ out) {
    __shared__ unsigned part[kPB / kWave];
    unsigned v = 0u;
    for (int i = blockIdx.x * kPB + threadIdx.x; i < n; i += gridDim.x * kPB)
        v = max(v, __float_as_uint(fabsf(mass[i])));
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v = max(v, (unsigned)__shfl_xor((int)v, o));
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = part[0];
        for (int w = 1; w < kPB / kWave; ++w) m = max(m, part[w]);
        atomicMax(out, m);
    }
}

// ---- sort by cell

// Lower grid index and the CIC fraction of a coordinate (grid point g at
// g D, periodic).
__device__ __forceinline__ int cic_axis(double x, double inv_d, int ng, double* frac) {
    double u = x * inv_d;
    u -= (double)ng * floor(u / (double)ng);
    double fl = floor(u);
    int i = (int)fl;
    double f = u - fl;
    if (i >= ng) { i -= ng; }
    if (i < 0 || !(f >= 0.0 && f < 1.0)) { i = 0; f = 0.0; }   // non-finite positions
    *frac = f;
    return i;
}

__device__ __forceinline__ void cic_point(const double* __restrict__ pos, int i, double inv_d,
                                          int ng, int g0[3], double f[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) g0[a] = cic_axis(pos[3 * (int64_t)i + a], inv_d, ng, &f[a]);
}

__global__ __launch_bounds__(kPB) void k_pm_keys(const double* __restrict__ pos,
                                                 const float* __restrict__ mass, int n, int ng,
                                                 double inv_d, int* __restrict__ keys,
                                                 int* __restrict__ vals,
                                                 float4* __restrict__ rec) {
    const int i = blockIdx.x * kPB + threadIdx.x;
    if (i >= n) return;
    int g0[3];
    double f[3];
    cic_point(pos, i, inv_d, ng, g0, f);
    keys[i] = (g0[0] * ng + g0[1]) * ng + g0[2];
    vals[i] = i;
    rec[i] = make_float4((float)f[0], (float)f[1], (float)f[2], mass[i]);
}

__global__ __launch_bounds__(kPB) void k_pm_gather(const int* __restrict__ perm,
                                                   const float4* __restrict__ rec_in, int n,
                                                   float4* __restrict__ rec) {
    const int k = blockIdx.x * kPB + threadIdx.x;
    if (k >= n) return;
    rec[k] = rec_in[perm[k]];
}

// Lower corner of a cell key and the fractions of a record.
__device__ __forceinline__ void cic_record(int key, float4 r, int ng, int g0[3], double f[3]) {
    g0[2] = key % ng;
    g0[1] = (key / ng) % ng;
    g0[0] = key / (ng * ng);
    f[0] = (double)r.x;
    f[1] = (double)r.y;
    f[2] = (double)r.z;
}

// ---- deposit

__device__ __forceinline__ int64_t corner_index(const int g0[3], int c, int ng) {
    const int bx = c >> 2, by = (c >> 1) & 1, bz = c & 1;
    const int x = g0[0] + bx == ng ? 0 : g0[0] + bx;
    const int y = g0[1] + by == ng ? 0 : g0[1] + by;
    const int z = g0[2] + bz == ng ? 0 : g0[2] + bz;
    return ((int64_t)x * ng + y) * ng + z;
}

__device__ __forceinline__ double corner_weight(const double f[3], int c) {
    const int bx = c >> 2, by = (c >> 1) & 1, bz = c & 1;
    return (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
}

// Lane k of the grid takes the k-th particle in cell order.  Lanes of a wave
// with the same key form a segment; for each corner a segmented inclusive
// scan leaves the segment's sum in its last lane, which adds it to the grid.
__global__ __launch_bounds__(kPB) void k_pm_deposit(const int* __restrict__ keys,
                                                    const float4* __restrict__ rec, int n,
                                                    int ng,
                                                    const unsigned* __restrict__ mmax_bits,
                                                    unsigned long long* __restrict__ grid) {
    const double mmax = (double)__uint_as_float(*mmax_bits);
    if (!(mmax > 0.0)) return;                       // uniform: nothing to deposit
    const double scale = 4611686018427387904.0 / ((double)n * mmax);   // 2^62
    const int k = blockIdx.x * kPB + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const bool live = k < n;
    const int key = live ? keys[k] : -1 - lane;      // padding lanes: own segments
    int g0[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    double m = 0.0;
    if (live) {
        const float4 r = rec[k];
        cic_record(key, r, ng, g0, f);
        m = (double)r.w * scale;
    }
    const int prev = __shfl_up(key, 1);
    const int next = __shfl_down(key, 1);
    const bool head = lane == 0 || prev != key;
    const bool tail = lane == kWave - 1 || next != key;
    const unsigned long long heads = __ballot(head);
    if (heads == ~0ull) {                            // no shared cells in this wave
        if (!live) return;
        for (int c = 0; c < 8; ++c) {
            const long long q = llrint(m * corner_weight(f, c));
            atomicAdd(&grid[corner_index(g0, c, ng)], (unsigned long long)q);
        }
        return;
    }
    const unsigned long long upto = (2ull << lane) - 1ull;   // lanes 0..lane
    const int sstart = 63 - __clzll(heads & upto);
    for (int c = 0; c < 8; ++c) {
        long long v = live ? llrint(m * corner_weight(f, c)) : 0ll;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const long long t = __shfl_up(v, off);
            if (lane - off >= sstart) v += t;
        }
        if (tail && live)
            atomicAdd(&grid[corner_index(g0, c, ng)], (unsigned long long)v);
    }
}

// ---- FFT

// cos(2 pi j / 32), j = 0..8
__device__ constexpr float kCos32[9] = {1.0f,         0.980785251f, 0.923879504f,
                                        0.831469595f, 0.707106769f, 0.555570245f,
                                        0.382683426f, 0.195090324f, 0.0f};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// b * exp(SIGN 2 pi i j / 32), 0 <= j < 16, j a compile-time constant after
// unrolling (so the multiplications by 1 and by +-i fold away).
template <int SIGN>
__device__ __forceinline__ float2 rot32(float2 b, int j) {
    if (j == 0) return b;
    if (j == 8) return SIGN < 0 ? make_float2(b.y, -b.x) : make_float2(-b.y, b.x);
    const float c = j <= 8 ? kCos32[j] : -kCos32[16 - j];
    const float s = j <= 8 ? kCos32[8 - j] : kCos32[j - 8];
    return cmul(b, make_float2(c, SIGN < 0 ? -s : s));
}

template <int R>
__device__ constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// In-register DFT of length R (2..32), natural order in and out:
// v[k] <- sum_j v[j] exp(SIGN 2 pi i j k / R).  Radix-2 decimation in time.
template <int SIGN, int R>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = v[bitrev<R>(i)];
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int g = 0; g < R; g += 2 * h) {
#pragma unroll
            for (int p = 0; p < h; ++p) {
                const float2 a = t[g + p];
                const float2 b = rot32<SIGN>(t[g + p + h], p * (16 / h));
                t[g + p] = make_float2(a.x + b.x, a.y + b.y);
                t[g + p + h] = make_float2(a.x - b.x, a.y - b.y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

template <int NG>
struct Shape {
    static constexpr int R1 = NG == 8 ? 2 : NG == 16 ? 4 : NG == 32 ? 4 : NG == 64 ? 8
                            : NG == 128 ? 8 : NG == 256 ? 16 : 32;
    static constexpr int R2 = NG / R1;
    static constexpr int TPL = R1 > R2 ? R1 : R2;          // threads per line
    static constexpr int L = NG < kPB / TPL ? NG : kPB / TPL;   // lines per workgroup
    static constexpr int P = R2 + 1;                       // LDS row pitch
    static constexpr int THREADS = L * TPL;
    static constexpr int TILES = NG * NG / L;
};

enum { kPlain = 0, kFromFixed = 1, kFusedX = 2 };

struct FftArgs {
    float2* a;                         // first grid
    float2* b;                         // second grid (two-grid passes, fused output)
    const unsigned long long* q;       // fixed-point deposit (first pass)
    const float2* tw;                  // tw[k] = exp(-2 pi i k / ng)
    const float4* sym;                 // per-axis symbol terms at index m
    const unsigned* mmax_bits;
    double unit;                       // density per fixed-point unit and max|m|
    float d, sigma;
    int n_s;
};

__device__ __forceinline__ int freq(int m, int ng) { return m < ng / 2 ? m : m - ng; }

// Per-axis terms of the symbols at index m: the K6 term (times D^2), k_a^2
// and the gradient symbol D_a.
__device__ __forceinline__ float4 axis_symbol(int m, int ng, float d) {
    const float th = (float)freq(m, ng) / (float)ng;        // k_a D / (2 pi)
    const float s1 = sinpif(th), s2 = sinpif(2.0f * th), s3 = sinpif(3.0f * th);
    const float k6 = 6.0f * s1 * s1 - 0.6f * s2 * s2 + (2.0f / 45.0f) * s3 * s3;
    const float kq = 2.0f * kPi * th / d;
    const float dk = ((4.0f / 3.0f) * s2 - (1.0f / 6.0f) * sinpif(4.0f * th)) / d;
    return make_float4(k6, kq * kq, dk, 0.0f);
}

// One pass along AXIS (0: x, stride ng^2; 1: y, stride ng; 2: z,
// contiguous) over the L lines of workgroup blockIdx.x.  kPlain transforms
// grid a (blockIdx.y == 0) or b (blockIdx.y == 1) in place with sign SIGN;
// kFromFixed reads the fixed-point deposit and writes the forward transform
// of the density into a; kFusedX (AXIS 0) does the forward x transform of
// a, the symbols and the inverse x transforms into b and a.
template <int NG, int AXIS, int MODE, int SIGN>
__global__ __launch_bounds__(kPB) void k_fft(FftArgs A) {
    using S = Shape<NG>;
    constexpr int R1 = S::R1, R2 = S::R2, TPL = S::TPL, L = S::L, P = S::P;
    __shared__ float2 sm[L * R1 * P];
    const int tid = threadIdx.x;
    const int line = AXIS == 2 ? tid / TPL : tid % L;
    const int r = AXIS == 2 ? tid % TPL : tid / L;
    const int g = blockIdx.x;
    int64_t base, es;
    int ly = 0, lz = 0;                                     // the line's y and z (AXIS 0)
    if (AXIS == 2) {
        base = ((int64_t)g * L + line) * NG;
        es = 1;
    } else {
        const int outer = g / (NG / L);
        const int z = (g % (NG / L)) * L + line;
        base = AXIS == 1 ? (int64_t)outer * NG * NG + z : (int64_t)outer * NG + z;
        es = AXIS == 1 ? NG : (int64_t)NG * NG;
        ly = outer;
        lz = z;
    }
    auto li = [&](int k1, int n2) {
        return AXIS == 2 ? line * (R1 * P) + k1 * P + n2 : line + L * (k1 * P + n2);
    };
    float2* data = (MODE == kPlain && blockIdx.y == 1) ? A.b : A.a;
    double unit = 0.0;
    if (MODE == kFromFixed) unit = A.unit * (double)__uint_as_float(*A.mmax_bits);

    // stage 1: thread n2 = r, DFT over n1 of x[n2 + R2 n1], twiddle, to LDS
    constexpr int FS = MODE == kFusedX ? -1 : SIGN;
    float2 v[R1];
    if (r < R2) {
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) {
            const int64_t at = base + (int64_t)(r + R2 * n1) * es;
            if (MODE == kFromFixed)
                v[n1] = make_float2((float)((double)(long long)A.q[at] * unit), 0.0f);
            else
                v[n1] = data[at];
        }
        dft<FS, R1>(v);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            float2 w = A.tw[(r * k1) & (NG - 1)];
            if (FS > 0) w.y = -w.y;
            sm[li(k1, r)] = cmul(v[k1], w);
        }
    }
    __syncthreads();
    // stage 2: thread k1 = r, DFT over n2; u[k2] = X[k1 + R1 k2]
    float2 u[R2];
    if (r < R1) {
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) u[n2] = sm[li(r, n2)];
        dft<FS, R2>(u);
    }
    if (MODE != kFusedX) {
        if (r < R1) {
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) data[base + (int64_t)(r + R1 * k2) * es] = u[k2];
        }
        return;
    }
    // symbols: phi = -4 pi S(k) / K6(k) / ng^3 times the density's transform
    float2 bv[R2];
    if (r < R1) {
        const float4 sy = A.sym[ly], sz = A.sym[lz];
        const float norm = 1.0f / ((float)NG * (float)NG * (float)NG);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            const int mx = r + R1 * k2;
            const float4 sx = A.sym[mx];
            const float dkx = sx.z, dky = sy.z, dkz = sz.z;
            float gk = 0.0f;
            if (mx != 0 || ly != 0 || lz != 0) {
                const float k6 = (sx.x + sy.x + sz.x) / (A.d * A.d);
                const float ksq = sx.y + sy.y + sz.y;
                const float xh = 0.5f * sqrtf(ksq) * A.d;
                const float sinc = sinf(xh) / xh;
                float Sk = expf(-0.25f * ksq * A.sigma * A.sigma * A.d * A.d);
                for (int q = 0; q < A.n_s; ++q) Sk *= sinc;
                gk = -4.0f * kPi * Sk / k6 * norm;
            }
            const float2 ph = make_float2(gk * u[k2].x, gk * u[k2].y);
            bv[k2] = make_float2(dky * ph.x + dkx * ph.y, dky * ph.y - dkx * ph.x);
            u[k2] = make_float2(dkz * ph.y, -dkz * ph.x);
        }
    }
    // inverse x transforms: thread k1 = r holds X[k1 + R1 k2]; a length-R2
    // DFT over k2, the twiddles, LDS, a length-R1 DFT over k1 by thread n2
#pragma unroll
    for (int out = 0; out < 2; ++out) {
        float2* dst = out == 0 ? A.b : A.a;
        __syncthreads();                                    // LDS reads above are done
        if (r < R1) {
            if (out == 0) dft<+1, R2>(bv);
            else dft<+1, R2>(u);
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) {
                float2 w = A.tw[(n2 * r) & (NG - 1)];
                w.y = -w.y;
                sm[li(r, n2)] = cmul(out == 0 ? bv[n2] : u[n2], w);
            }
        }
        __syncthreads();
        if (r < R2) {
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) v[k1] = sm[li(k1, r)];
            dft<+1, R1>(v);
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) dst[base + (int64_t)(r + R2 * n1) * es] = v[n1];
        }
    }
}

// tw[k] = exp(-2 pi i k / ng) and the per-axis symbol terms, k < ng.
__global__ __launch_bounds__(kPB) void k_tables(int ng, float d, float2* __restrict__ tw,
                                                float4* __restrict__ sym) {
    const int k = blockIdx.x * kPB + threadIdx.x;
    if (k >= ng) return;
    float s, c;
    sincospif(2.0f * (float)k / (float)ng, &s, &c);
    tw[k] = make_float2(c, -s);
    sym[k] = axis_symbol(k, ng, d);
}

// ---- interpolation

// Lane k takes the k-th particle in cell order: a_x, a_y from the real and
// imaginary parts of grid b, a_z from the real part of grid a.
__global__ __launch_bounds__(kPB) void k_pm_interp(const int* __restrict__ perm,
                                                   const int* __restrict__ keys,
                                                   const float4* __restrict__ rec, int n,
                                                   int ng,
                                                   const float2* __restrict__ gxy,
                                                   const float2* __restrict__ gz,
                                                   float* __restrict__ out) {
    const int k = blockIdx.x * kPB + threadIdx.x;
    if (k >= n) return;
    const int i = perm[k];
    int g0[3];
    double f[3];
    cic_record(keys[k], rec[k], ng, g0, f);
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    for (int c = 0; c < 8; ++c) {
        const float w = (float)corner_weight(f, c);
        const int64_t at = corner_index(g0, c, ng);
        const float2 xy = gxy[at];
        ax = __builtin_fmaf(w, xy.x, ax);
        ay = __builtin_fmaf(w, xy.y, ay);
        az = __builtin_fmaf(w, gz[at].x, az);
    }
    out[3 * (int64_t)i + 0] = ax;
    out[3 * (int64_t)i + 1] = ay;
    out[3 * (int64_t)i + 2] = az;
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

template <int NG>
void launch_fft_all(const FftArgs& a, hipStream_t st) {
    using S = Shape<NG>;
    const dim3 blk(S::THREADS);
    hipLaunchKernelGGL((k_fft<NG, 2, kFromFixed, -1>), dim3(S::TILES), blk, 0, st, a);
    hipLaunchKernelGGL((k_fft<NG, 1, kPlain, -1>), dim3(S::TILES, 1), blk, 0, st, a);
    hipLaunchKernelGGL((k_fft<NG, 0, kFusedX, -1>), dim3(S::TILES), blk, 0, st, a);
    hipLaunchKernelGGL((k_fft<NG, 1, kPlain, +1>), dim3(S::TILES, 2), blk, 0, st, a);
    hipLaunchKernelGGL((k_fft<NG, 2, kPlain, +1>), dim3(S::TILES, 2), blk, 0, st, a);
}

// Radix sort of the cell keys: bits = 3 log2(ng), at most three passes of
// 8..10-bit digits.
void pm_sort_shape(int ng, int* passes, int* digit_bits) {
    int lg = 0;
    while ((1 << lg) < ng) ++lg;
    const int bits = 3 * lg;
    const int p = (bits + 9) / 10;
    *passes = p;
    *digit_bits = std::max(8, (bits + p - 1) / p);
}

struct PmLayout {
    size_t a, b, tw, sym, mmax, keys_a, vals_a, keys_b, vals_b, rec_in, rec, hist, scan_tmp,
        total;
};

PmLayout pm_layout(int ng, int64_t n) {
    PmLayout L{};
    const size_t cells = (size_t)ng * ng * ng;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    int passes, db;
    pm_sort_shape(ng, &passes, &db);
    const int nn = (int)std::max<int64_t>(n, 1);
    const size_t hist_n = ((size_t)1 << db) * (size_t)radix_blocks(nn);
    const size_t ni = sizeof(int) * (size_t)nn;
    L.a = take(cells * sizeof(float2));
    L.b = take(cells * sizeof(float2));      // also the fixed-point deposit
    L.tw = take((size_t)ng * sizeof(float2));
    L.sym = take((size_t)ng * sizeof(float4));
    L.mmax = take(sizeof(unsigned));
    L.keys_a = take(ni);
    L.vals_a = take(ni);
    L.keys_b = take(ni);
    L.vals_b = take(ni);
    L.rec_in = take(sizeof(float4) * (size_t)nn);
    L.rec = take(sizeof(float4) * (size_t)nn);
    L.hist = take(sizeof(int) * hist_n);
    L.scan_tmp = take(sizeof(int) * scan_tmp_ints((int)hist_n));
    L.total = off;
    return L;
}

}  // namespace

size_t pm_workspace_bytes(int ng, int64_t n) { return pm_layout(ng, n).total; }

hipError_t launch_pm_accel(const double* pos, const float* mass, int n, double box, int ng,
                           float sigma, int n_s, void* ws, float* out_acc, hipStream_t st) {
    const int64_t cells = (int64_t)ng * ng * ng;
    const PmLayout PL = pm_layout(ng, n);
    char* base = reinterpret_cast<char*>(ws);
    float2* A = reinterpret_cast<float2*>(base + PL.a);
    float2* B = reinterpret_cast<float2*>(base + PL.b);
    unsigned long long* Q = reinterpret_cast<unsigned long long*>(B);
    float2* tw = reinterpret_cast<float2*>(base + PL.tw);
    float4* sym = reinterpret_cast<float4*>(base + PL.sym);
    unsigned* mmax = reinterpret_cast<unsigned*>(base + PL.mmax);
    int* ka = reinterpret_cast<int*>(base + PL.keys_a);
    int* va = reinterpret_cast<int*>(base + PL.vals_a);
    int* kb = reinterpret_cast<int*>(base + PL.keys_b);
    int* vb = reinterpret_cast<int*>(base + PL.vals_b);
    float4* rec_in = reinterpret_cast<float4*>(base + PL.rec_in);
    float4* rec = reinterpret_cast<float4*>(base + PL.rec);
    int* hist = reinterpret_cast<int*>(base + PL.hist);
    int* tmp = reinterpret_cast<int*>(base + PL.scan_tmp);
    const double d = box / ng;
    const double inv_d = (double)ng / box;
    hipError_t e = launch_fill_i32(reinterpret_cast<int*>(mmax), 1, 0, st);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(reinterpret_cast<int*>(Q), (int)(2 * cells), 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tables, dim3(blocks_for(ng, kPB)), dim3(kPB), 0, st, ng, (float)d,
                       tw, sym);
    if (n > 0) {
        hipLaunchKernelGGL(k_pm_mass_max, dim3(std::min(kMaxBlocks, blocks_for(n, kPB))),
                           dim3(kPB), 0, st, mass, n, mmax);
        hipLaunchKernelGGL(k_pm_keys, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st, pos, mass,
                           n, ng, inv_d, ka, va, rec_in);
        int passes, db;
        pm_sort_shape(ng, &passes, &db);
        for (int p = 0; p < passes; ++p) {
            e = launch_radix_pass(ka, va, kb, vb, n, db * p, db, hist, tmp, st);
            if (e != hipSuccess) return e;
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        hipLaunchKernelGGL(k_pm_gather, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st,
                           (const int*)va, (const float4*)rec_in, n, rec);
        hipLaunchKernelGGL(k_pm_deposit, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st,
                           (const int*)ka, (const float4*)rec, n, ng, (const unsigned*)mmax, Q);
    }
    FftArgs fa{};
    fa.a = A;
    fa.b = B;
    fa.q = Q;
    fa.tw = tw;
    fa.sym = sym;
    fa.mmax_bits = mmax;
    // density = q (n max|m| / 2^62) / D^3; k_fft multiplies by max|m|
    fa.unit = (double)n / 4611686018427387904.0 / (d * d * d);
    fa.d = (float)d;
    fa.sigma = sigma;
    fa.n_s = n_s;
    switch (ng) {
        case 8: launch_fft_all<8>(fa, st); break;
        case 16: launch_fft_all<16>(fa, st); break;
        case 32: launch_fft_all<32>(fa, st); break;
        case 64: launch_fft_all<64>(fa, st); break;
        case 128: launch_fft_all<128>(fa, st); break;
        case 256: launch_fft_all<256>(fa, st); break;
        case 512: launch_fft_all<512>(fa, st); break;
        default: return hipErrorInvalidValue;
    }
    if (n > 0)
        hipLaunchKernelGGL(k_pm_interp, dim3(blocks_for(n, kPB)), dim3(kPB), 0, st,
                           (const int*)va, (const int*)ka, (const float4*)rec, n, ng,
                           (const float2*)B, (const float2*)A, out_acc);
    return hipGetLastError();
}

}  // namespace hsr
