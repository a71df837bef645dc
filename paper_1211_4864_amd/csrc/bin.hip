// Chaining-mesh binning: cell keys and cell-relative float32 records,
// stable LSD radix passes (each block orders its tile of keys in LDS and
// writes each digit's keys out as one run), the occupancy histogram of the
// sorted keys (wave-aggregated atomics: sorted keys arrive in runs), its
// exclusive prefix scan (cell_start), and the gather of the records into
// sorted order.  The sort key is the cell index followed by the Morton code
// of the particle's sub-cell (4^3 per cell when the key has room), so a
// cell's particles are grouped spatially and, within a sub-cell, keep their
// input order: the binning is deterministic.
//
// The chaining mesh is the cell list of the particle-particle part of a
// P^3M code (Habib et al. 2012, Sec. II); cells are at least r_cut wide so
// that all short-range partners of a particle lie in the 27 adjacent cells.
#include "common.h"

namespace hsr {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;   // 4096 elements per block

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Lanes of the wave holding the same BITS-bit value (a match over ballots).
template <int BITS>
__device__ __forceinline__ uint64_t peers(unsigned v, bool active) {
    uint64_t m = __ballot(active);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (v >> b) & 1u;
        const uint64_t bl = __ballot(bit && active);
        m &= bit ? bl : ~bl;
    }
    return active ? m : 0ull;
}

// Wrapped (periodic) or raw (open) coordinate and its cell index on one
// axis.  x == box after the wrap maps to 0; a non-finite coordinate lands in
// cell 0 (its record then carries the NaN and so do its accelerations).
__device__ __forceinline__ int axis_cell(double x, const Geom& g, double* xw) {
    double v = x;
    if (g.periodic) {
        v = x - g.box * floor(x / g.box);
        if (v >= g.box) v -= g.box;
    }
    const double k = floor(v / g.Lc);
    int c;
    if (!(k >= 0.0)) c = 0;
    else if (!(k <= (double)(g.N - 1))) c = g.N - 1;
    else c = (int)k;
    *xw = v;
    return c;
}

// Sub-cell index along one axis, 0..S-1, of a coordinate in its cell.
__device__ __forceinline__ int axis_sub(double xw, int c, const Geom& g, int S) {
    const double t = floor((xw - (double)c * g.Lc) / g.Lc * (double)S);
    if (!(t >= 0.0)) return 0;
    if (!(t <= (double)(S - 1))) return S - 1;
    return (int)t;
}

// Sort key (cell index, then the sub-cell Morton code) and the float32
// record (position relative to the cell's lower corner, mass) of every
// particle, in input order.
__global__ __launch_bounds__(kBlock) void k_cell_keys(
    const double* __restrict__ pos, const float* __restrict__ mass, int n,
    Geom g, int* __restrict__ keys, int* __restrict__ vals,
    float4* __restrict__ rec) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double xw, yw, zw;
    const int cx = axis_cell(pos[3 * (int64_t)i], g, &xw);
    const int cy = axis_cell(pos[3 * (int64_t)i + 1], g, &yw);
    const int cz = axis_cell(pos[3 * (int64_t)i + 2], g, &zw);
    const int key = (cx * g.N + cy) * g.N + cz;
    int code = 0;
    const int levels = g.sbits / 3;
    if (levels > 0) {
        const int S = 1 << levels;
        const int sx = axis_sub(xw, cx, g, S);
        const int sy = axis_sub(yw, cy, g, S);
        const int sz = axis_sub(zw, cz, g, S);
        for (int b = 0; b < levels; ++b)
            code |= (((sx >> b) & 1) << (3 * b + 2)) |
                    (((sy >> b) & 1) << (3 * b + 1)) | (((sz >> b) & 1) << (3 * b));
    }
    keys[i] = (key << g.sbits) | code;
    vals[i] = i;
    float4 r;
    r.x = (float)(xw - (double)cx * g.Lc);
    r.y = (float)(yw - (double)cy * g.Lc);
    r.z = (float)(zw - (double)cz * g.Lc);
    r.w = mass ? mass[i] : 0.0f;
    rec[i] = r;
}

// Occupancy of every cell from the sorted keys.  Consecutive entries share
// cells, so each wave adds one count per distinct cell it holds.
__global__ __launch_bounds__(kBlock) void k_cell_hist(
    const int* __restrict__ keys, int n, int sbits, int* __restrict__ counts) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    bool pending = k < n;
    const int cell = pending ? keys[k] >> sbits : 0;
    uint64_t left = __ballot(pending);
    while (left) {
        const int lead = __shfl(cell, __ffsll((unsigned long long)left) - 1);
        const uint64_t same = __ballot(pending && cell == lead);
        if (pending && cell == lead && (same & lanemask_lt()) == 0ull)
            atomicAdd(&counts[cell], __popcll(same));
        if (cell == lead) pending = false;
        left &= ~same;
    }
}

// ---------------------------------------------------------------- scan
// Exclusive prefix sum of int32 in three passes: per-block sums, a single
// block scan of those sums, per-block scan plus carry.

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(v, d);
        if (lane_id() >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total.
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[kBlock / kWave];
    const int incl = wave_incl_scan(v);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; ++q) {
        const int s = wsum[q];
        if (q < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(
    const int* __restrict__ in, int n, int* __restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int s = 0;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t e = base + it * kBlock + threadIdx.x;
        if (e < n) s += in[e];
    }
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block scans an array of any length in chunks, carrying the total.
__global__ __launch_bounds__(kBlock) void k_scan_single(int* __restrict__ a,
                                                        int n) {
    int carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += kTile) {
        int v[kItems];
        int s = 0;
        const int64_t b = c0 + (int64_t)threadIdx.x * kItems;
#pragma unroll
        for (int q = 0; q < kItems; ++q) {
            v[q] = (b + q < n) ? a[b + q] : 0;
            s += v[q];
        }
        int tot;
        int pre = block_excl_scan(s, &tot) + carry;
#pragma unroll
        for (int q = 0; q < kItems; ++q) {
            if (b + q < n) a[b + q] = pre;
            pre += v[q];
        }
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(
    const int* in, int* out, int n, const int* __restrict__ bsum) {
    const int64_t b = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
        v[q] = (b + q < n) ? in[b + q] : 0;
        s += v[q];
    }
    int tot;
    int pre = block_excl_scan(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
        if (b + q < n) out[b + q] = pre;
        pre += v[q];
    }
}

// ---------------------------------------------------------------- radix
// One stable counting-sort pass on a DB-bit digit of the sort key: per
// block digit histograms, their scan (digit-major over the blocks), then the
// scatter.  This direct scatter writes each element as it is ranked; it
// serves digits of 11 bits, whose LDS-staged variant below would not fit.

template <int DB>
__global__ __launch_bounds__(kBlock) void k_radix_hist(
    const int* __restrict__ keys, int n, int shift, int* __restrict__ hist,
    int nblocks) {
    constexpr int R = 1 << DB;
    __shared__ int h[R];
    for (int q = threadIdx.x; q < R; q += kBlock) h[q] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int it = 0; it < kItems; ++it) {
        const int64_t e = base + it * kBlock + threadIdx.x;
        const bool active = e < n;
        const unsigned d = active ? ((unsigned)keys[e] >> shift) & (unsigned)(R - 1) : 0u;
        const uint64_t pm = peers<DB>(d, active);
        if (active && (pm & lanemask_lt()) == 0ull) atomicAdd(&h[d], __popcll(pm));
    }
    __syncthreads();
    for (int q = threadIdx.x; q < R; q += kBlock)
        hist[(int64_t)q * nblocks + blockIdx.x] = h[q];
}

template <int DB>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const int* __restrict__ kin, const int* __restrict__ vin,
    int* __restrict__ kout, int* __restrict__ vout, int n, int shift,
    const int* __restrict__ offs, int nblocks) {
    constexpr int R = 1 << DB;
    constexpr int kW = kBlock / kWave;
    __shared__ int base_d[R];     // global offset of this block's digit d
    __shared__ int run_d[R];      // digit d entries already placed by this block
    __shared__ int wcnt[kW][R];
    for (int q = threadIdx.x; q < R; q += kBlock) {
        base_d[q] = offs[(int64_t)q * nblocks + blockIdx.x];
        run_d[q] = 0;
    }
    const int w = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int it = 0; it < kItems; ++it) {
        for (int q = threadIdx.x; q < R; q += kBlock)
#pragma unroll
            for (int v = 0; v < kW; ++v) wcnt[v][q] = 0;
        __syncthreads();
        const int64_t e = base + it * kBlock + threadIdx.x;
        const bool active = e < n;
        const int key = active ? kin[e] : 0;
        const int val = active ? vin[e] : 0;
        const unsigned d = ((unsigned)key >> shift) & (unsigned)(R - 1);
        const uint64_t pm = peers<DB>(d, active);
        const int rank = __popcll(pm & lanemask_lt());
        if (active && rank == 0) wcnt[w][d] = __popcll(pm);
        __syncthreads();
        // each digit: exclusive prefix over the waves for these 256 keys
        for (int t = threadIdx.x; t < R; t += kBlock) {
            int acc = run_d[t];
#pragma unroll
            for (int v = 0; v < kW; ++v) {
                const int c = wcnt[v][t];
                wcnt[v][t] = acc;
                acc += c;
            }
            run_d[t] = acc;
        }
        __syncthreads();
        if (active) {
            const int dst = base_d[d] + wcnt[w][d] + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
    }
}

// The same pass with the block's keys first placed in LDS in their sorted
// order (a stable local counting sort of the 4096-key tile), then written
// out in that order: each digit's keys of the block go to consecutive
// global slots, so the writes are runs instead of one scattered element per
// lane.  Wave w ranks the keys w * 1024 .. w * 1024 + 1023 of the tile, 64 at
// a time, against its own digit counters; one prefix over the waves then
// places every key.  Needs 2^DB * (2 + 2 * kW) + 2 * 4096 ints of LDS; used
// for DB <= 10.
template <int DB>
__global__ __launch_bounds__(kBlock) void k_radix_scatter_staged(
    const int* __restrict__ kin, const int* __restrict__ vin,
    int* __restrict__ kout, int* __restrict__ vout, int n, int shift,
    const int* __restrict__ offs, int nblocks) {
    constexpr int R = 1 << DB;
    constexpr int kW = kBlock / kWave;
    constexpr int kPerW = kTile / kW / kWave;   // keys per lane
    constexpr int kPerT = R / kBlock;           // digits per thread
    static_assert(kPerT >= 1, "at least one digit per thread");
    __shared__ int base_d[R];     // global offset of this block's digit d
    __shared__ int loc_d[R];      // first tile slot of digit d in this block
    __shared__ int cw[kW][R];     // per wave: digit counts, then their prefix
    __shared__ int part[kBlock];
    __shared__ int skey[kTile];
    __shared__ int sval[kTile];
    // This block's count of each digit follows from the scanned offsets
    // (digit-major over the blocks); a block scan gives the tile slots.
    const int64_t flat = (int64_t)R * nblocks;
    int cnt[kPerT];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        const int d = threadIdx.x * kPerT + j;
        const int64_t idx = (int64_t)d * nblocks + blockIdx.x;
        const int o = offs[idx];
        const int nx = idx + 1 < flat ? offs[idx + 1] : n;
        base_d[d] = o;
        cnt[j] = nx - o;
        sum += cnt[j];
#pragma unroll
        for (int v = 0; v < kW; ++v) cw[v][d] = 0;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int s = 1; s < kBlock; s <<= 1) {      // inclusive scan of the sums
        const int v = threadIdx.x >= s ? part[threadIdx.x - s] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int acc = part[threadIdx.x] - sum;
#pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        loc_d[threadIdx.x * kPerT + j] = acc;
        acc += cnt[j];
    }
    // rank of each key among the equal digits before it in this wave's keys
    const int w = threadIdx.x / kWave;
    const int64_t first = (int64_t)blockIdx.x * kTile + (int64_t)w * (kPerW * kWave) +
                          lane_id();
    int key[kPerW], val[kPerW], rk[kPerW];
#pragma unroll
    for (int r = 0; r < kPerW; ++r) {
        const int64_t e = first + r * kWave;
        const bool active = e < n;
        key[r] = active ? kin[e] : 0;
        val[r] = active ? vin[e] : 0;
    }
#pragma unroll
    for (int r = 0; r < kPerW; ++r) {
        const bool active = first + r * kWave < n;
        const unsigned d = ((unsigned)key[r] >> shift) & (unsigned)(R - 1);
        const uint64_t pm = peers<DB>(d, active);
        const int rank = __popcll(pm & lanemask_lt());
        rk[r] = active ? cw[w][d] + rank : 0;
        // A wave's LDS accesses complete in program order; the barriers keep
        // the compiler from moving the counter update across the reads.
        __builtin_amdgcn_wave_barrier();
        if (active && rank == 0) cw[w][d] += __popcll(pm);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves
    for (int d = threadIdx.x; d < R; d += kBlock) {
        int a = 0;
#pragma unroll
        for (int v = 0; v < kW; ++v) {
            const int c = cw[v][d];
            cw[v][d] = a;
            a += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerW; ++r) {
        if (first + r * kWave < n) {
            const unsigned d = ((unsigned)key[r] >> shift) & (unsigned)(R - 1);
            const int slot = loc_d[d] + cw[w][d] + rk[r];
            skey[slot] = key[r];
            sval[slot] = val[r];
        }
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int m = (int)min((int64_t)kTile, (int64_t)n - base);
    for (int i = threadIdx.x; i < m; i += kBlock) {
        const int k = skey[i];
        const unsigned d = ((unsigned)k >> shift) & (unsigned)(R - 1);
        const int dst = base_d[d] + (i - loc_d[d]);
        kout[dst] = k;
        vout[dst] = sval[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_records(
    const float4* __restrict__ rec_in, const int* __restrict__ perm, int n,
    float4* __restrict__ rec) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    rec[k] = rec_in[perm[k]];
}

__global__ __launch_bounds__(kBlock) void k_gather_vec3(
    const float* __restrict__ v, const int* __restrict__ perm, int n,
    float4* __restrict__ out) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t i = perm[k];
    out[k] = make_float4(v[3 * i], v[3 * i + 1], v[3 * i + 2], 0.0f);
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int* p, int n, int value) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k < n) p[k] = value;
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_cell_keys(const double* pos, const float* mass, int n,
                            Geom g, int* keys, int* vals, float4* rec,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                       0, st, pos, mass, n, g, keys, vals, rec);
    return hipGetLastError();
}

hipError_t launch_cell_hist(const int* keys_sorted, int n, int sbits,
                            int* counts, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_hist, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                       0, st, keys_sorted, n, sbits, counts);
    return hipGetLastError();
}

size_t scan_tmp_ints(int n) { return (size_t)blocks_for(n, kTile) + 1; }

hipError_t launch_scan_exclusive(const int* in, int* out, int n, int* tmp,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nb = blocks_for(n, kTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kBlock), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, st, in, out, n,
                       (const int*)tmp);
    return hipGetLastError();
}

int radix_blocks(int n) { return blocks_for(n, kTile); }

namespace {
template <int DB>
hipError_t radix_pass(const int* kin, const int* vin, int* kout, int* vout,
                      int n, int shift, int* hist, int* scan_tmp,
                      hipStream_t st) {
    const int nb = radix_blocks(n);
    hipLaunchKernelGGL(k_radix_hist<DB>, dim3(nb), dim3(kBlock), 0, st, kin, n,
                       shift, hist, nb);
    hipError_t e = launch_scan_exclusive(hist, hist, (1 << DB) * nb, scan_tmp, st);
    if (e != hipSuccess) return e;
    if constexpr (DB <= 10)
        hipLaunchKernelGGL(k_radix_scatter_staged<DB>, dim3(nb), dim3(kBlock), 0, st,
                           kin, vin, kout, vout, n, shift, (const int*)hist, nb);
    else
        hipLaunchKernelGGL(k_radix_scatter<DB>, dim3(nb), dim3(kBlock), 0, st, kin,
                           vin, kout, vout, n, shift, (const int*)hist, nb);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_radix_pass(const int* kin, const int* vin, int* kout,
                             int* vout, int n, int shift, int digit_bits,
                             int* hist, int* scan_tmp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    switch (digit_bits) {
        case 8: return radix_pass<8>(kin, vin, kout, vout, n, shift, hist, scan_tmp, st);
        case 9: return radix_pass<9>(kin, vin, kout, vout, n, shift, hist, scan_tmp, st);
        case 10: return radix_pass<10>(kin, vin, kout, vout, n, shift, hist, scan_tmp, st);
        case 11: return radix_pass<11>(kin, vin, kout, vout, n, shift, hist, scan_tmp, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_records(const float4* rec_in, const int* perm, int n,
                                 float4* rec, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_records, dim3(blocks_for(n, kBlock)),
                       dim3(kBlock), 0, st, rec_in, perm, n, rec);
    return hipGetLastError();
}

hipError_t launch_gather_vec3(const float* v, const int* perm, int n,
                              float4* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_vec3, dim3(blocks_for(n, kBlock)), dim3(kBlock),
                       0, st, v, perm, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int n, int value, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0,
                       st, p, n, value);
    return hipGetLastError();
}

}  // namespace hsr
