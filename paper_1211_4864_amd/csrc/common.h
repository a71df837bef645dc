// Internal definitions shared by the HIP translation units of libhacc_sr.
// Not part of the public interface (include/hacc_sr.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsr {

constexpr int kWave = 64;

// Chaining-mesh geometry: N^3 cells of side Lc = |box| / N >= r_cut.
struct Geom {
    int N;            // cells per axis
    int periodic;     // 1: periodic cube [0, box); 0: open domain [0, box)
    double box;       // |box|
    double Lc;        // cell side, float64
    float Lc_f;       // cell side rounded to float32 (frame shifts)
    int sbits;        // sub-cell bits of the sort key: 6 (4^3 sub-cells), 3 or 0
};

// Pair-kernel constants derived on the host from (r_cut, eps, poly).
// The grid-force polynomial is evaluated in t = alpha * (s + eps) + beta,
// which maps s in [0, r_cut^2] onto [-1, 1]; b[] are its coefficients in t
// db2[] those of 2 d(poly)/ds, also in t, and dq3[] = db2[] / 3.
struct PairParams {
    float alpha, beta;
    float eps;
    float rc2e;       // float32(r_cut^2 + eps): cut-off test on s + eps
    float cull2;      // float32(r_cut^2 (1 + 2^-12)): staging drops sources
                      // at least this far (squared) from the target box
    float b[6];
    float db2[5];
    float dq3[5];
};

// One unit of pair-kernel work: T = i_count target particles of one cell,
// processed by one wave with ksplit lanes per target (T * ksplit <= 64).
struct WorkItem {
    int i_begin;      // first sorted entry of the targets
    int i_count;      // number of targets T (1..kItemI)
    int key;          // first cell of the item's run of cells
    short ksplit;     // lanes per target, a power of two
    short zlen;       // cells in the run: key, key + 1, ... along z
};

// Small cells are merged into runs of up to kZRun cells along z (one item,
// one source window of 3 x 3 x (zlen + 2) cells) when a whole aligned block
// holds at most kItemI targets.
constexpr int kZRun = 2;
constexpr int kMaxSegments = 9 * (kZRun + 2);   // stencil cells of a run

constexpr int kItemI = 64;     // lanes of a wave

// ---- launch wrappers (each defined in the translation unit of its kernels)

// binning (bin.hip)
hipError_t launch_cell_keys(const double* pos, const float* mass, int n,
                            Geom g, int* keys, int* vals, float4* rec,
                            hipStream_t st);
hipError_t launch_cell_hist(const int* keys_sorted, int n, int sbits,
                            int* counts, hipStream_t st);
size_t scan_tmp_ints(int n);
hipError_t launch_scan_exclusive(const int* in, int* out, int n, int* tmp,
                                 hipStream_t st);
int radix_blocks(int n);
constexpr int kMaxDigitBits = 11;
hipError_t launch_radix_pass(const int* kin, const int* vin, int* kout,
                             int* vout, int n, int shift, int digit_bits,
                             int* hist, int* scan_tmp, hipStream_t st);
hipError_t launch_gather_records(const float4* rec_in, const int* perm, int n,
                                 float4* rec, hipStream_t st);
hipError_t launch_gather_vec3(const float* v, const int* perm, int n,
                              float4* out, hipStream_t st);
hipError_t launch_fill_i32(int* p, int n, int value, hipStream_t st);

// work list (worklist.hip)
constexpr int kCostBuckets = 128;
constexpr int kXcds = 8;            // XCDs of an MI355X
// Ints of the ordering buffer: counts and offsets of kXcds * kCostBuckets
// buckets, then 2 kXcds + 1 list-layout entries.
constexpr int kOrderInts = 2 * kXcds * kCostBuckets + 2 * kXcds + 1;
hipError_t launch_items_count(const int* cell_start, Geom g, int* cell_items,
                              int* cell_window, unsigned long long* col_cost,
                              int* col_xcd, hipStream_t st);
hipError_t launch_items_write(const int* cell_start, Geom g,
                              const int* cell_off, WorkItem* items,
                              hipStream_t st);
hipError_t launch_items_order(const WorkItem* items, const int* n_items_dev,
                              int max_items, const int* cell_window,
                              const int* col_xcd, Geom g, int* bucket_of,
                              int* buckets, WorkItem* items_sorted,
                              hipStream_t st);

// pair kernels (pair.hip)
hipError_t launch_pair_force(const WorkItem* items, int max_items,
                             const int* n_items_dev, const float4* rec,
                             const int* cell_start, const int* perm, Geom g,
                             PairParams p, float* out_acc, hipStream_t st);
hipError_t launch_pair_count(const WorkItem* items, int max_items,
                             const int* n_items_dev, const float4* rec,
                             const int* cell_start, Geom g, PairParams p,
                             unsigned long long* counts, hipStream_t st);
hipError_t launch_pair_vjp(const WorkItem* items, int max_items,
                           const int* n_items_dev, const float4* rec,
                           const float4* gsorted, const int* cell_start,
                           const int* perm, Geom g, PairParams p,
                           double* out_grad, hipStream_t st);

// RCB fat leaves inside the chaining cells (rcb.hip)
hipError_t launch_rcb(const int* cell_start, int ncell, int n, int leaf_max,
                      int* cell_list, int* counters, float4* rec, int* perm,
                      float4* rec_tmp, int* perm_tmp, int* leafmark,
                      int4* nodes, float* split, hipStream_t st);
hipError_t launch_leaf_table(const int* leafmark, int* leafidx, int n, int* scan_tmp,
                             int* leaf_start, hipStream_t st);
hipError_t launch_leaf_items(const int* leaf_start, const int* n_leaves_dev,
                             int max_leaves, const int* keys_sorted, int sbits,
                             int* leaf_items, int* scan_tmp, WorkItem* items,
                             hipStream_t st);

// plain reference kernels (plain.hip)
hipError_t launch_force_plain(const float4* rec, const int* keys_sorted,
                              const int* cell_start, const int* perm, int n,
                              Geom g, PairParams p, float* out, hipStream_t st);
hipError_t launch_vjp_plain(const float4* rec, const float4* gsorted,
                            const int* keys_sorted, const int* cell_start,
                            const int* perm, int n, Geom g, PairParams p,
                            double* out, hipStream_t st);

// float32 VALU rate probes (probe.hip), measurement only
size_t probe_scratch_bytes();
size_t probe_clock_offset();
int probe_ops_per_iter(int kind);
hipError_t launch_valu_probe(int kind, int waves, int iters, void* scratch,
                             hipStream_t st);

// long-range spectral PM force (pm.hip)
size_t pm_workspace_bytes(int ng, int64_t n);
hipError_t launch_pm_accel(const double* pos, const float* mass, int n, double box, int ng,
                           float sigma, int n_s, void* ws, float* out_acc, hipStream_t st);

// kick / stream (integrate.hip)
hipError_t launch_kick(double* vel, const float* acc, int64_t m, double dt,
                       hipStream_t st);
hipError_t launch_stream(double* pos, const double* vel, int64_t m, double dt,
                         double box, hipStream_t st);
hipError_t launch_kick_adjoint(const double* gv, float* ga, int64_t m,
                               double dt, hipStream_t st);

}  // namespace hsr
