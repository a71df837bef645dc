// Work list for the pair kernels.  One item is one wave's worth of target
// particles from one run of cells: a single chaining cell, or an aligned
// pair of cells along z that holds at most 64 targets (the run rule is in
// run_of).  Its sources are the run's 3 x 3 x (zlen + 2) stencil cells.  A
// run of c targets yields floor(c/64) items of 64 targets (one per lane) and
// at most two items for the remainder r = c mod 64: the largest power of two
// p <= r, and r - p.  An item of T targets runs with k = floor_pow2(64 / T)
// lanes per target, each lane taking every k-th source, so a power-of-two
// item keeps all 64 lanes busy whatever its size.
//
// Order of the items.  The chip has 8 XCDs, each with its own L2, and a
// kernel's workgroup k runs on XCD k mod 8.  The cells are split into 8
// spatially contiguous ranges of equal cost (columns of cells in key order),
// one per XCD, and XCD x receives the items of its range at workgroups
// x, x + 8, x + 16, ..., in decreasing cost so that the longest items start
// first.  The items of a dense cell and of its neighbours then share one L2,
// which holds their common source window.  Items beyond the shortest XCD
// list follow at the end in plain decreasing cost.
//
// This replaces the tree walk that gathers leaf interaction lists in the
// paper's BG/Q code (Habib et al. 2012, Sec. III, walk minimisation and the
// paragraph on neighbour lists after Eq. 7).
#include "common.h"

namespace hsr {

namespace {

constexpr int kBlock = 256;
constexpr int kXcd = kXcds;

__device__ __forceinline__ int floor_pow2(int v) {
    return v <= 0 ? 0 : (1 << (31 - __clz(v)));
}

// Run of cells that cell c belongs to.  The cells of a column are grouped in
// aligned blocks of kZRun along z; a block whose cells hold at most kItemI
// targets in all is one run (its first cell is the head), otherwise each
// cell is a run of its own.  In a periodic box a run leaves at least two
// cells of the column outside it, so its window of zlen + 2 cells along z
// has no cell twice.
struct Run {
    bool head;     // c starts a run (and emits its items)
    int zlen;      // cells in the run
    int count;     // targets in the run
};

__device__ __forceinline__ Run run_of(int c, const int* __restrict__ cs,
                                      const Geom& g) {
    const int N = g.N;
    const int cz = c % N;
    const int z0 = cz - cz % kZRun;
    int zl = min(kZRun, N - z0);
    if (g.periodic) zl = min(zl, N - 2);
    if (zl >= 2 && cz < z0 + zl) {
        const int first = c - (cz - z0);
        const int total = cs[first + zl] - cs[first];
        if (total <= kItemI) return Run{cz == z0, zl, total};
    }
    return Run{true, 1, cs[c + 1] - cs[c]};
}

// Calls emit(i_offset, count, ksplit) for the items of a run of c targets.
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
                    x = x < 0 ? x + N : (x >= N ? x - N : x);
                    y = y < 0 ? y + N : (y >= N ? y - N : y);
                    z = z < 0 ? z + N : (z >= N ? z - N : z);
                } else if (x < 0 || x >= N || y < 0 || y >= N || z < 0 || z >= N) {
                    continue;
                }
                const int kk = (x * N + y) * N + z;
                total += cs[kk + 1] - cs[kk];
            }
    return total;
}

// Per cell: number of items, window size, and the cell's pair work
// (targets x window) added to its column (cx, cy).
__global__ __launch_bounds__(kBlock) void k_items_count(
    const int* __restrict__ cs, Geom g, int* __restrict__ cell_items_out,
    int* __restrict__ cell_window, unsigned long long* __restrict__ col_cost) {
    const int ncell = g.N * g.N * g.N;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    const int occ = cs[c + 1] - cs[c];
    const Run run = run_of(c, cs, g);
    int cnt = 0;
    if (run.head) cell_items(run.count, [&](int, int, int) { ++cnt; });
    cell_items_out[c] = cnt;
    const int w = window_sources(c, cs, g);
    cell_window[c] = w;
    if (occ > 0)
        atomicAdd(&col_cost[c / g.N], (unsigned long long)occ * (unsigned long long)w);
}

// XCD of each column of cells: the columns in key order are cut into kXcd
// ranges of equal total work.  One block; the columns are split into
// contiguous chunks per thread.
__global__ __launch_bounds__(1024) void k_column_xcd(
    const unsigned long long* __restrict__ col_cost, int ncol,
    int* __restrict__ col_xcd) {
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const int per = (ncol + 1023) / 1024;
    const int a = min(ncol, t * per), b = min(ncol, a + per);
    unsigned long long sum = 0;
    for (int q = a; q < b; ++q) sum += col_cost[q];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {       // inclusive scan of the chunks
        const unsigned long long v = t >= d ? part[t - d] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const unsigned long long total = part[1023];
    unsigned long long run = part[t] - sum;
    for (int q = a; q < b; ++q) {
        // the column goes to the XCD that holds the midpoint of its work
        const double mid = (double)run + 0.5 * (double)col_cost[q];
        int x = total ? (int)(mid * kXcd / (double)total) : 0;
        col_xcd[q] = min(kXcd - 1, max(0, x));
        run += col_cost[q];
    }
}

__global__ __launch_bounds__(kBlock) void k_items_write(
    const int* __restrict__ cs, Geom g, const int* __restrict__ cell_off,
    WorkItem* __restrict__ items) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.N * g.N * g.N) return;
    const Run run = run_of(c, cs, g);
    if (!run.head) return;
    int k = cell_off[c];
    const int start = cs[c];
    cell_items(run.count, [&](int o, int cnt, int ks) {
        WorkItem it;
        it.i_begin = start + o;
        it.i_count = cnt;
        it.key = c;
        it.ksplit = (short)ks;
        it.zlen = (short)run.zlen;
        items[k++] = it;
    });
}


// Quarter-octave buckets of the per-lane source count (the wave's running
// time), 0 = cheapest.
__device__ __forceinline__ int cost_bucket(int sources, int ksplit) {
    const float l = log2f(fmaxf((float)sources / (float)ksplit, 1.0f));
    return min(kCostBuckets - 1, (int)(4.0f * l));
}

// Bucket of an item: its XCD's list, then its cost bucket.
constexpr int kOrderBuckets = kXcd * kCostBuckets;

// Per-block histogram of buckets; each block then reserves one range per
// bucket (one global atomic per bucket and block) in k_items_scatter.
__global__ __launch_bounds__(kBlock) void k_items_bucket(
    const WorkItem* __restrict__ items, const int* __restrict__ n_items_dev,
    const int* __restrict__ cell_window, const int* __restrict__ col_xcd, Geom g,
    int* __restrict__ bucket_of, int* __restrict__ bucket_count) {
    __shared__ int h[kOrderBuckets];
    for (int q = threadIdx.x; q < kOrderBuckets; q += kBlock) h[q] = 0;
    __syncthreads();
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const int n_items = *n_items_dev;
    if (k < n_items) {
        const WorkItem it = items[k];
        // a run's window spans zlen + 2 cells along z instead of 3
        const int window = cell_window[it.key] * (it.zlen + 2) / 3;
        const int b = col_xcd[it.key / g.N] * kCostBuckets +
                      cost_bucket(window, it.ksplit);
        bucket_of[k] = b;
        atomicAdd(&h[b], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kOrderBuckets; q += kBlock)
        if (h[q]) atomicAdd(&bucket_count[q], h[q]);
}

// Rank offsets inside each XCD's list (decreasing cost), and the layout of
// the lists: meta[x] = length of list x, meta[kXcd + x] = offset of its
// items beyond the shortest list in the tail, meta[2 kXcd] = shortest
// length.
__global__ void k_items_bucket_scan(const int* __restrict__ bucket_count,
                                    int* __restrict__ bucket_off,
                                    int* __restrict__ meta) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int shortest = 0x7fffffff;
    for (int x = 0; x < kXcd; ++x) {
        int acc = 0;
        for (int b = kCostBuckets - 1; b >= 0; --b) {
            bucket_off[x * kCostBuckets + b] = acc;
            acc += bucket_count[x * kCostBuckets + b];
        }
        meta[x] = acc;
        shortest = min(shortest, acc);
    }
    int tail = 0;
    for (int x = 0; x < kXcd; ++x) {
        meta[kXcd + x] = tail;
        tail += meta[x] - shortest;
    }
    meta[2 * kXcd] = shortest;
}

// Final position of rank r of XCD x's list: workgroup r * kXcd + x while
// every list still has items, then the remaining items of each list in turn.
__device__ __forceinline__ int xcd_slot(int x, int r, const int* meta) {
    const int shortest = meta[2 * kXcd];
    if (r < shortest) return r * kXcd + x;
    return kXcd * shortest + meta[kXcd + x] + (r - shortest);
}

__global__ __launch_bounds__(kBlock) void k_items_scatter(
    const WorkItem* __restrict__ items, const int* __restrict__ n_items_dev,
    const int* __restrict__ bucket_of, int* __restrict__ bucket_off,
    const int* __restrict__ meta, WorkItem* __restrict__ out) {
    __shared__ int h[kOrderBuckets];
    __shared__ int base[kOrderBuckets];
    for (int q = threadIdx.x; q < kOrderBuckets; q += kBlock) h[q] = 0;
    __syncthreads();
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const bool active = k < *n_items_dev;
    const int b = active ? bucket_of[k] : 0;
    // Order inside a bucket is arbitrary; results do not depend on it
    // because every item writes only its own targets.
    const int local = active ? atomicAdd(&h[b], 1) : 0;
    __syncthreads();
    for (int q = threadIdx.x; q < kOrderBuckets; q += kBlock)
        base[q] = h[q] ? atomicAdd(&bucket_off[q], h[q]) : 0;
    __syncthreads();
    if (active) out[xcd_slot(b / kCostBuckets, base[b] + local, meta)] = items[k];
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_items_count(const int* cell_start, Geom g, int* cell_items,
                              int* cell_window, unsigned long long* col_cost,
                              int* col_xcd, hipStream_t st) {
    const int ncell = g.N * g.N * g.N;
    const int ncol = g.N * g.N;
    hipError_t e = launch_fill_i32(reinterpret_cast<int*>(col_cost), 2 * ncol, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_items_count, dim3(blocks_for(ncell, kBlock)),
                       dim3(kBlock), 0, st, cell_start, g, cell_items,
                       cell_window, col_cost);
    hipLaunchKernelGGL(k_column_xcd, dim3(1), dim3(1024), 0, st,
                       (const unsigned long long*)col_cost, ncol, col_xcd);
    return hipGetLastError();
}

hipError_t launch_items_write(const int* cell_start, Geom g,
                              const int* cell_off, WorkItem* items,
                              hipStream_t st) {
    const int ncell = g.N * g.N * g.N;
    hipLaunchKernelGGL(k_items_write, dim3(blocks_for(ncell, kBlock)),
                       dim3(kBlock), 0, st, cell_start, g, cell_off, items);
    return hipGetLastError();
}

hipError_t launch_items_order(const WorkItem* items, const int* n_items_dev,
                              int max_items, const int* cell_window,
                              const int* col_xcd, Geom g, int* bucket_of,
                              int* buckets, WorkItem* items_sorted,
                              hipStream_t st) {
    int* bucket_count = buckets;
    int* bucket_off = buckets + kOrderBuckets;
    int* meta = buckets + 2 * kOrderBuckets;
    hipError_t e = launch_fill_i32(bucket_count, kOrderBuckets, 0, st);
    if (e != hipSuccess) return e;
    const int nb = blocks_for(max_items, kBlock);
    hipLaunchKernelGGL(k_items_bucket, dim3(nb), dim3(kBlock), 0, st, items,
                       n_items_dev, cell_window, col_xcd, g, bucket_of,
                       bucket_count);
    hipLaunchKernelGGL(k_items_bucket_scan, dim3(1), dim3(64), 0, st,
                       (const int*)bucket_count, bucket_off, meta);
    hipLaunchKernelGGL(k_items_scatter, dim3(nb), dim3(kBlock), 0, st, items,
                       n_items_dev, (const int*)bucket_of, bucket_off,
                       (const int*)meta, items_sorted);
    return hipGetLastError();
}

}  // namespace hsr
