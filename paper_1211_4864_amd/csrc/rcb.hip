// Recursive coordinate bisection (RCB) of the chaining cells into fat leaves,
// the organisation of the short-range solver in the paper's BG/Q code
// (Habib et al. 2012, Sec. III: an RCB tree whose nodes are split at the
// centre of mass along the longest side of their bounding box, particles
// partitioned into disjoint child ranges, and leaves of a few hundred
// particles at most that share one interaction list).
//
// Here the chaining mesh remains the coarse level: every cell is at least
// r_cut wide, so a leaf's interaction list is drawn from its cell's 27
// neighbours.  Inside each cell holding more than leaf_max particles one
// workgroup builds the cell's tree:
//
//   - a node is reduced (bounding box, mass-weighted centre) over its
//     contiguous range of sorted records;
//   - it is split at the centre of mass along the longest side: a stable
//     three-phase partition (count the left side, block-scan the flags,
//     scatter both sides into a scratch buffer) writes the two children into
//     disjoint contiguous ranges, then the range is copied back;
//   - a child with at most leaf_max particles is a leaf, otherwise it is
//     split in turn.  The larger child is pushed on a stack and the smaller
//     one processed first, so the stack never holds more than log2(n)
//     entries;
//   - if every particle falls on one side (all coordinates on the longest
//     axis equal, i.e. coincident particles), the node is cut in two by
//     index without moving anything (recorded as axis 3).
//
// Records carry positions relative to their cell, so all the arithmetic is
// float32.  Partitions are stable and the reductions have a fixed order, so
// the tree is bitwise reproducible.  Leaves never cross cells.
#include <algorithm>

#include "common.h"

namespace hsr {

namespace {

constexpr int kRB = 256;                  // threads of an RCB workgroup
constexpr int kRW = kRB / kWave;          // its waves
constexpr int kStack = 40;                // > log2(2^31)

__device__ __forceinline__ uint64_t lanemask_lt_r() {
    const int l = threadIdx.x & (kWave - 1);
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ float axis_of(float4 r, int a) {
    return a == 0 ? r.x : (a == 1 ? r.y : r.z);
}

// Cells with more than leaf_max particles, appended in any order (each is
// processed on its own, so the order does not change the result); cells
// with 1..leaf_max particles are leaves as they stand.
__global__ __launch_bounds__(kRB) void k_rcb_select(const int* __restrict__ cs,
                                                    int ncell, int leaf_max,
                                                    int* __restrict__ list,
                                                    int* __restrict__ n_list,
                                                    int* __restrict__ leafmark) {
    const int c = blockIdx.x * kRB + threadIdx.x;
    if (c >= ncell) return;
    const int b = cs[c], cnt = cs[c + 1] - b;
    if (cnt > leaf_max) {
        list[atomicAdd(n_list, 1)] = c;
    } else if (cnt > 0) {
        leafmark[b] = 1;
    }
}

// Block-wide reduction of 10 floats: min of v[0..2], max of v[3..5], sum of
// v[6..9].  Every thread receives the result.
__device__ void block_reduce10(float* v, float (*red)[10]) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = fminf(v[q], __shfl_xor(v[q], o));
#pragma unroll
        for (int q = 3; q < 6; ++q) v[q] = fmaxf(v[q], __shfl_xor(v[q], o));
#pragma unroll
        for (int q = 6; q < 10; ++q) v[q] += __shfl_xor(v[q], o);
    }
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 10; ++q) red[w][q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 10; ++q) v[q] = red[0][q];
    for (int k = 1; k < kRW; ++k) {
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = fminf(v[q], red[k][q]);
#pragma unroll
        for (int q = 3; q < 6; ++q) v[q] = fmaxf(v[q], red[k][q]);
#pragma unroll
        for (int q = 6; q < 10; ++q) v[q] += red[k][q];
    }
    __syncthreads();
}

__device__ int block_sum(int v, int* redi) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
    if (lane == 0) redi[w] = v;
    __syncthreads();
    int t = 0;
    for (int k = 0; k < kRW; ++k) t += redi[k];
    __syncthreads();
    return t;
}

// One workgroup per listed cell: builds the cell's RCB tree in place in the
// sorted records and permutation, marks the first entry of every leaf, and
// (when nodes is not null) records every internal node as (begin, count,
// left count, axis) with its split coordinate.
__global__ __launch_bounds__(kRB) void k_rcb_cells(
    const int* __restrict__ cs, const int* __restrict__ list,
    const int* __restrict__ n_list, int leaf_max, float4* __restrict__ rec,
    int* __restrict__ perm, float4* __restrict__ rec_tmp, int* __restrict__ perm_tmp,
    int* __restrict__ leafmark, int4* __restrict__ nodes, float* __restrict__ split_out,
    int* __restrict__ n_nodes) {
    __shared__ float red[kRW][10];
    __shared__ int redi[kRW];
    __shared__ int wcnt[kRW];
    __shared__ int st_b[kStack], st_c[kStack];
    if ((int)blockIdx.x >= *n_list) return;
    const int cell = list[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    int sp = 0;                      // stack depth (the same in every thread)
    int b = cs[cell], c = cs[cell + 1] - b;
    const float inf = __builtin_huge_valf();
    while (true) {
        // ---- phase 0: bounding box and centre of mass of [b, b + c)
        float v[10] = {inf, inf, inf, -inf, -inf, -inf, 0.f, 0.f, 0.f, 0.f};
        for (int e = tid; e < c; e += kRB) {
            const float4 r = rec[b + e];
            v[0] = fminf(v[0], r.x); v[1] = fminf(v[1], r.y); v[2] = fminf(v[2], r.z);
            v[3] = fmaxf(v[3], r.x); v[4] = fmaxf(v[4], r.y); v[5] = fmaxf(v[5], r.z);
            v[6] = __builtin_fmaf(r.w, r.x, v[6]);
            v[7] = __builtin_fmaf(r.w, r.y, v[7]);
            v[8] = __builtin_fmaf(r.w, r.z, v[8]);
            v[9] += r.w;
        }
        block_reduce10(v, red);
        int axis = 0;
        float ext = v[3] - v[0];
        if (v[4] - v[1] > ext) { axis = 1; ext = v[4] - v[1]; }
        if (v[5] - v[2] > ext) { axis = 2; }
        // centre of mass along the axis; the box centre if the masses sum
        // to zero
        const float lo = axis == 0 ? v[0] : (axis == 1 ? v[1] : v[2]);
        const float hi = axis == 0 ? v[3] : (axis == 1 ? v[4] : v[5]);
        const float mx = axis == 0 ? v[6] : (axis == 1 ? v[7] : v[8]);
        const float split = v[9] > 0.0f ? mx / v[9] : 0.5f * (lo + hi);
        // ---- phase 1: size of the left side
        int mine = 0;
        for (int e = tid; e < c; e += kRB) mine += axis_of(rec[b + e], axis) < split ? 1 : 0;
        int nl = block_sum(mine, redi);
        if (nl == 0 || nl == c) {
            // every particle on one side: cut by index, nothing moves
            axis = 3;
            nl = c / 2;
        } else {
            // ---- phase 2: stable scatter of both sides into the scratch range
            int lbase = 0, rbase = nl;
            for (int t0 = 0; t0 < c; t0 += kRB) {
                const int e = t0 + tid;
                const bool act = e < c;
                const float4 r = act ? rec[b + e] : make_float4(0.f, 0.f, 0.f, 0.f);
                const int pv = act ? perm[b + e] : 0;
                const bool left = act && axis_of(r, axis) < split;
                const uint64_t m = __ballot(left);
                const int before_w = __popcll(m & lanemask_lt_r());
                if (lane == 0) wcnt[w] = __popcll(m);
                __syncthreads();
                int wpre = 0, tile_left = 0;
                for (int k = 0; k < kRW; ++k) {
                    if (k < w) wpre += wcnt[k];
                    tile_left += wcnt[k];
                }
                __syncthreads();
                const int lefts_before = wpre + before_w;
                if (act) {
                    const int dst = left ? lbase + lefts_before
                                         : rbase + (tid - lefts_before);
                    rec_tmp[b + dst] = r;
                    perm_tmp[b + dst] = pv;
                }
                const int tile_n = min(kRB, c - t0);
                lbase += tile_left;
                rbase += tile_n - tile_left;
            }
            __syncthreads();
            // ---- phase 3: copy the partitioned range back
            for (int e = tid; e < c; e += kRB) {
                rec[b + e] = rec_tmp[b + e];
                perm[b + e] = perm_tmp[b + e];
            }
            __syncthreads();
        }
        if (nodes != nullptr && tid == 0) {
            const int k = atomicAdd(n_nodes, 1);
            nodes[k] = make_int4(b, c, nl, axis);
            split_out[k] = split;
        }
        // ---- children
        const int lb = b, lc = nl, rb = b + nl, rc = c - nl;
        if (tid == 0) {
            if (lc <= leaf_max) leafmark[lb] = 1;
            if (rc <= leaf_max) leafmark[rb] = 1;
        }
        const bool lin = lc > leaf_max, rin = rc > leaf_max;
        if (lin && rin) {
            // push the larger, continue with the smaller
            const bool lsmall = lc <= rc;
            if (tid == 0) {
                st_b[sp] = lsmall ? rb : lb;
                st_c[sp] = lsmall ? rc : lc;
            }
            ++sp;
            b = lsmall ? lb : rb;
            c = lsmall ? lc : rc;
        } else if (lin || rin) {
            b = lin ? lb : rb;
            c = lin ? lc : rc;
        } else {
            if (sp == 0) break;
            __syncthreads();
            --sp;
            b = st_b[sp];
            c = st_c[sp];
        }
        __syncthreads();
    }
}

// Leaf table: the sorted entries marked as the first of a leaf, in order.
// leafidx is the exclusive scan of leafmark (n + 1 entries).
__global__ __launch_bounds__(kRB) void k_leaf_compact(const int* __restrict__ leafmark,
                                                      const int* __restrict__ leafidx,
                                                      int n, int* __restrict__ leaf_start) {
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i < n && leafmark[i]) leaf_start[leafidx[i]] = i;
    if (i == n) leaf_start[leafidx[n]] = n;
}

__device__ __forceinline__ int floor_pow2_r(int v) {
    return v <= 0 ? 0 : (1 << (31 - __clz(v)));
}

// Items of a leaf of c particles: floor(c / 64) full ones, then at most two
// for the remainder (the largest power of two, then the rest), as for the
// cells of the chaining-mesh work list.
template <typename Emit>
__device__ void for_leaf_items(int c, Emit emit) {
    int o = 0;
    for (; o + kItemI <= c; o += kItemI) emit(o, kItemI, 1);
    int r = c - o;
    if (r > 0) {
        const int p = floor_pow2_r(r);
        emit(o, p, kItemI / p);
        o += p;
        r -= p;
    }
    if (r > 0) emit(o, r, floor_pow2_r(kItemI / r));
}

__global__ __launch_bounds__(kRB) void k_leaf_items_count(
    const int* __restrict__ leaf_start, const int* __restrict__ n_leaves_dev,
    int max_leaves, int* __restrict__ leaf_items) {
    const int l = blockIdx.x * kRB + threadIdx.x;
    const int nl = *n_leaves_dev;
    if (l > max_leaves) return;
    if (l >= nl) {
        leaf_items[l] = 0;
        return;
    }
    int cnt = 0;
    for_leaf_items(leaf_start[l + 1] - leaf_start[l], [&](int, int, int) { ++cnt; });
    leaf_items[l] = cnt;
}

__global__ __launch_bounds__(kRB) void k_leaf_items_write(
    const int* __restrict__ leaf_start, const int* __restrict__ n_leaves_dev,
    const int* __restrict__ item_off, const int* __restrict__ keys_sorted, int sbits,
    WorkItem* __restrict__ items) {
    const int l = blockIdx.x * kRB + threadIdx.x;
    if (l >= *n_leaves_dev) return;
    const int b = leaf_start[l];
    const int cell = keys_sorted[b] >> sbits;
    int k = item_off[l];
    for_leaf_items(leaf_start[l + 1] - b, [&](int o, int cnt, int ks) {
        WorkItem it;
        it.i_begin = b + o;
        it.i_count = cnt;
        it.key = cell;
        it.ksplit = (short)ks;
        it.zlen = 1;
        items[k++] = it;
    });
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_rcb(const int* cell_start, int ncell, int n, int leaf_max,
                      int* cell_list, int* counters, float4* rec, int* perm,
                      float4* rec_tmp, int* perm_tmp, int* leafmark,
                      int4* nodes, float* split, hipStream_t st) {
    // counters[0]: listed cells, counters[1]: recorded nodes
    hipError_t e = launch_fill_i32(counters, 2, 0, st);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(leafmark, n + 1, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rcb_select, dim3(blocks_for(ncell, kRB)), dim3(kRB), 0, st,
                       cell_start, ncell, leaf_max, cell_list, counters, leafmark);
    // at most min(ncell, n / (leaf_max + 1)) cells hold more than leaf_max
    const int64_t most = std::min<int64_t>(ncell, (int64_t)n / ((int64_t)leaf_max + 1));
    if (most > 0)
        hipLaunchKernelGGL(k_rcb_cells, dim3((int)most), dim3(kRB), 0, st, cell_start,
                           (const int*)cell_list, (const int*)counters, leaf_max, rec,
                           perm, rec_tmp, perm_tmp, leafmark, nodes, split, counters + 1);
    return hipGetLastError();
}

hipError_t launch_leaf_table(const int* leafmark, int* leafidx, int n, int* scan_tmp,
                             int* leaf_start, hipStream_t st) {
    hipError_t e = launch_scan_exclusive(leafmark, leafidx, n + 1, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_leaf_compact, dim3(blocks_for(n + 1, kRB)), dim3(kRB), 0, st,
                       leafmark, (const int*)leafidx, n, leaf_start);
    return hipGetLastError();
}

hipError_t launch_leaf_items(const int* leaf_start, const int* n_leaves_dev,
                             int max_leaves, const int* keys_sorted, int sbits,
                             int* leaf_items, int* scan_tmp, WorkItem* items,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_leaf_items_count, dim3(blocks_for(max_leaves + 1, kRB)), dim3(kRB),
                       0, st, leaf_start, n_leaves_dev, max_leaves, leaf_items);
    hipError_t e = launch_scan_exclusive(leaf_items, leaf_items, max_leaves + 1, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_leaf_items_write, dim3(blocks_for(max_leaves, kRB)), dim3(kRB), 0,
                       st, leaf_start, n_leaves_dev, (const int*)leaf_items, keys_sorted,
                       sbits, items);
    return hipGetLastError();
}

}  // namespace hsr
