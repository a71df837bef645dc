// Work list for the pair kernels.  One item is one wave's worth of target
// particles from a single chaining cell; its sources are the cell's 27-cell
// stencil.  A cell of c targets yields floor(c/64) items of 64 targets (one
// per lane) and at most two items for the remainder r = c mod 64: the largest
// power of two p <= r, and r - p.  An item of T targets runs with k =
// floor_pow2(64 / T) lanes per target, each lane taking every k-th source,
// so a power-of-two item keeps all 64 lanes busy whatever its size.  Items
// are ordered by decreasing cost so that the longest ones start first.
//
// This replaces the tree walk that gathers leaf interaction lists in the
// paper's BG/Q code (Habib et al. 2012, Sec. III, walk minimisation and the
// paragraph on neighbour lists after Eq. 7).
#include "common.h"

namespace hsr {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int floor_pow2(int v) {
    return v <= 0 ? 0 : (1 << (31 - __clz(v)));
}

// Calls emit(i_offset, count, ksplit) for the items of a cell of c targets.
template <typename Emit>
__device__ void cell_items(int c, Emit emit) {
    int o = 0;
    for (; o + kItemI <= c; o += kItemI) emit(o, kItemI, 1);
    int r = c - o;
    if (r > 0) {
        const int p = floor_pow2(r);
        emit(o, p, kItemI / p);
        o += p;
        r -= p;
    }
    if (r > 0) emit(o, r, floor_pow2(kItemI / r));
}

__global__ __launch_bounds__(kBlock) void k_items_count(
    const int* __restrict__ cs, int ncell, int* __restrict__ cell_items_out) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    int cnt = 0;
    cell_items(cs[c + 1] - cs[c], [&](int, int, int) { ++cnt; });
    cell_items_out[c] = cnt;
}

__global__ __launch_bounds__(kBlock) void k_items_write(
    const int* __restrict__ cs, int ncell, const int* __restrict__ cell_off,
    WorkItem* __restrict__ items) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    int k = cell_off[c];
    const int start = cs[c];
    cell_items(cs[c + 1] - start, [&](int o, int cnt, int ks) {
        WorkItem it;
        it.i_begin = start + o;
        it.i_count = cnt;
        it.key = c;
        it.ksplit = ks;
        items[k++] = it;
    });
}

// Number of source particles in the 27-cell stencil of a cell.
__device__ int window_sources(int key, const int* cs, const Geom& g) {
    const int N = g.N;
    const int cz = key % N, cy = (key / N) % N, cx = key / (N * N);
    int total = 0;
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
                const int kk = (x * N + y) * N + z;
                total += cs[kk + 1] - cs[kk];
            }
    return total;
}

// Quarter-octave buckets of the per-lane source count (the wave's running
// time), 0 = cheapest.
__device__ __forceinline__ int cost_bucket(int sources, int ksplit) {
    const float l = log2f(fmaxf((float)sources / (float)ksplit, 1.0f));
    return min(kCostBuckets - 1, (int)(4.0f * l));
}

// Per-block histogram of buckets; each block then reserves one range per
// bucket (one global atomic per bucket and block) in k_items_scatter.
__global__ __launch_bounds__(kBlock) void k_items_bucket(
    const WorkItem* __restrict__ items, const int* __restrict__ n_items_dev,
    const int* __restrict__ cs, Geom g, int* __restrict__ bucket_of,
    int* __restrict__ bucket_count) {
    __shared__ int h[kCostBuckets];
    for (int q = threadIdx.x; q < kCostBuckets; q += kBlock) h[q] = 0;
    __syncthreads();
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const int n_items = *n_items_dev;
    if (k < n_items) {
        const WorkItem it = items[k];
        const int b = cost_bucket(window_sources(it.key, cs, g), it.ksplit);
        bucket_of[k] = b;
        atomicAdd(&h[b], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kCostBuckets; q += kBlock)
        if (h[q]) atomicAdd(&bucket_count[q], h[q]);
}

// Offsets in decreasing-cost order.
__global__ void k_items_bucket_scan(const int* __restrict__ bucket_count,
                                    int* __restrict__ bucket_off) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int acc = 0;
    for (int b = kCostBuckets - 1; b >= 0; --b) {
        bucket_off[b] = acc;
        acc += bucket_count[b];
    }
}

__global__ __launch_bounds__(kBlock) void k_items_scatter(
    const WorkItem* __restrict__ items, const int* __restrict__ n_items_dev,
    const int* __restrict__ bucket_of, int* __restrict__ bucket_off,
    WorkItem* __restrict__ out) {
    __shared__ int h[kCostBuckets];
    __shared__ int base[kCostBuckets];
    for (int q = threadIdx.x; q < kCostBuckets; q += kBlock) h[q] = 0;
    __syncthreads();
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const bool active = k < *n_items_dev;
    const int b = active ? bucket_of[k] : 0;
    // Order inside a bucket is arbitrary; results do not depend on it
    // because every item writes only its own targets.
    const int local = active ? atomicAdd(&h[b], 1) : 0;
    __syncthreads();
    for (int q = threadIdx.x; q < kCostBuckets; q += kBlock)
        base[q] = h[q] ? atomicAdd(&bucket_off[q], h[q]) : 0;
    __syncthreads();
    if (active) out[base[b] + local] = items[k];
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_items_count(const int* cell_start, Geom g, int* cell_items,
                              hipStream_t st) {
    const int ncell = g.N * g.N * g.N;
    hipLaunchKernelGGL(k_items_count, dim3(blocks_for(ncell, kBlock)),
                       dim3(kBlock), 0, st, cell_start, ncell, cell_items);
    return hipGetLastError();
}

hipError_t launch_items_write(const int* cell_start, Geom g,
                              const int* cell_off, WorkItem* items,
                              hipStream_t st) {
    const int ncell = g.N * g.N * g.N;
    hipLaunchKernelGGL(k_items_write, dim3(blocks_for(ncell, kBlock)),
                       dim3(kBlock), 0, st, cell_start, ncell, cell_off, items);
    return hipGetLastError();
}

hipError_t launch_items_order(const WorkItem* items, const int* n_items_dev,
                              int max_items, const int* cell_start, Geom g,
                              int* bucket_of, int* bucket_count,
                              int* bucket_off, WorkItem* items_sorted,
                              hipStream_t st) {
    hipError_t e = launch_fill_i32(bucket_count, kCostBuckets, 0, st);
    if (e != hipSuccess) return e;
    const int nb = blocks_for(max_items, kBlock);
    hipLaunchKernelGGL(k_items_bucket, dim3(nb), dim3(kBlock), 0, st, items,
                       n_items_dev, cell_start, g, bucket_of, bucket_count);
    hipLaunchKernelGGL(k_items_bucket_scan, dim3(1), dim3(64), 0, st,
                       (const int*)bucket_count, bucket_off);
    hipLaunchKernelGGL(k_items_scatter, dim3(nb), dim3(kBlock), 0, st, items,
                       n_items_dev, (const int*)bucket_of, bucket_off,
                       items_sorted);
    return hipGetLastError();
}

}  // namespace hsr
