// Work list for the pair kernels.  Each item is one wave's worth of target
// particles (at most kItemI) taken from a run of consecutive cells along z
// in one (x, y) column; its sources are the 9 neighbouring columns over the
// run's z range widened by one cell at each end, i.e. the 27-cell stencil of
// every cell in the run.  Dense cells are split into several items; sparse
// cells are merged so that a wave's lanes stay busy.  Items are ordered by
// decreasing source count so that the longest ones start first.
//
// This replaces the tree walk that gathers leaf interaction lists in the
// paper's BG/Q code (Habib et al. 2012, Sec. III, walk minimisation and the
// paragraph on neighbour lists after Eq. 7).
#include "common.h"

namespace hsr {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int cell_count(const int* cs, int key) {
    return cs[key + 1] - cs[key];
}

// Walks the cells of one column and calls emit(z0, nz, i_begin, i_count) for
// every item, in increasing z.  Identical in the counting and writing passes.
template <typename Emit>
__device__ void walk_column(const int* cs, int col, int N, int zmax, Emit emit) {
    const int kbase = col * N;
    bool open = false;
    int z0 = 0, zlast = 0, run_n = 0;
    for (int z = 0; z < N; ++z) {
        const int c = cell_count(cs, kbase + z);
        if (c == 0) continue;
        if (c > kItemI) {
            if (open) {
                emit(z0, zlast - z0 + 1, cs[kbase + z0], run_n);
                open = false;
            }
            const int start = cs[kbase + z];
            for (int o = 0; o < c; o += kItemI)
                emit(z, 1, start + o, min(kItemI, c - o));
            continue;
        }
        if (open && run_n + c <= kItemI && z - z0 + 1 <= zmax) {
            run_n += c;
            zlast = z;
        } else {
            if (open) emit(z0, zlast - z0 + 1, cs[kbase + z0], run_n);
            open = true;
            z0 = z;
            zlast = z;
            run_n = c;
        }
    }
    if (open) emit(z0, zlast - z0 + 1, cs[kbase + z0], run_n);
}

__global__ __launch_bounds__(kBlock) void k_items_count(
    const int* __restrict__ cs, int N, int zmax, int* __restrict__ col_items) {
    const int col = blockIdx.x * kBlock + threadIdx.x;
    if (col >= N * N) return;
    int cnt = 0;
    walk_column(cs, col, N, zmax, [&](int, int, int, int) { ++cnt; });
    col_items[col] = cnt;
}

__global__ __launch_bounds__(kBlock) void k_items_write(
    const int* __restrict__ cs, int N, int zmax, const int* __restrict__ col_off,
    WorkItem* __restrict__ items) {
    const int col = blockIdx.x * kBlock + threadIdx.x;
    if (col >= N * N) return;
    int k = col_off[col];
    walk_column(cs, col, N, zmax, [&](int z0, int nz, int ib, int ic) {
        WorkItem it;
        it.i_begin = ib;
        it.i_count = ic;
        it.key0 = col * N + z0;
        it.nz = nz;
        items[k++] = it;
    });
}

// Number of source particles in an item's stencil window.
__device__ int window_sources(const WorkItem& it, const int* cs, const Geom& g) {
    const int N = g.N;
    const int z0 = it.key0 % N;
    const int col = it.key0 / N;
    const int cx = col / N, cy = col % N;
    int total = 0;
    for (int a = -1; a <= 1; ++a) {
        for (int b = -1; b <= 1; ++b) {
            int x = cx + a, y = cy + b;
            if (g.periodic) {
                x = (x + N) % N;
                y = (y + N) % N;
            } else if (x < 0 || x >= N || y < 0 || y >= N) {
                continue;
            }
            const int kb = (x * N + y) * N;
            int lo = z0 - 1, hi = z0 + it.nz;   // inclusive
            if (g.periodic) {
                if (lo < 0) {
                    total += cs[kb + N] - cs[kb + N - 1];
                    lo = 0;
                }
                if (hi >= N) {
                    total += cs[kb + 1] - cs[kb];
                    hi = N - 1;
                }
            } else {
                lo = max(lo, 0);
                hi = min(hi, N - 1);
            }
            total += cs[kb + hi + 1] - cs[kb + lo];
        }
    }
    return total;
}

__device__ __forceinline__ int cost_bucket(int j) {
    // quarter-octave buckets of the source count, 0 = cheapest
    const float l = log2f((float)max(j, 1));
    return min(kCostBuckets - 1, (int)(4.0f * l));
}

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
        const int b = cost_bucket(window_sources(items[k], cs, g));
        bucket_of[k] = b;
        atomicAdd(&h[b], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kCostBuckets; q += kBlock)
        if (h[q]) atomicAdd(&bucket_count[q], h[q]);
}

// Offsets in decreasing-cost order; also resets the placement cursors.
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
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= *n_items_dev) return;
    // Order inside a bucket is arbitrary; results do not depend on it
    // because every item writes only its own targets.
    const int dst = atomicAdd(&bucket_off[bucket_of[k]], 1);
    out[dst] = items[k];
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_items_count(const int* cell_start, Geom g, int zmax,
                              int* col_items, hipStream_t st) {
    const int ncol = g.N * g.N;
    hipLaunchKernelGGL(k_items_count, dim3(blocks_for(ncol, kBlock)),
                       dim3(kBlock), 0, st, cell_start, g.N, zmax, col_items);
    return hipGetLastError();
}

hipError_t launch_items_write(const int* cell_start, Geom g, int zmax,
                              const int* col_off, WorkItem* items,
                              hipStream_t st) {
    const int ncol = g.N * g.N;
    hipLaunchKernelGGL(k_items_write, dim3(blocks_for(ncol, kBlock)),
                       dim3(kBlock), 0, st, cell_start, g.N, zmax, col_off,
                       items);
    return hipGetLastError();
}

hipError_t launch_items_order(const WorkItem* items, const int* n_items_dev,
                              int max_items, const int* cell_start, Geom g,
                              int* bucket_of, int* bucket_count,
                              int* bucket_off, WorkItem* items_sorted,
                              int* /*scan_tmp*/, hipStream_t st) {
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
