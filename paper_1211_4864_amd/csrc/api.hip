// C-ABI entry points of libhacc_sr (declared in include/hacc_sr.h): host-side
// argument validation, workspace layout, and the launch sequence of each
// operation on the registered stream.
#include <hacc_sr.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"

using namespace hsr;

namespace {

hipStream_t g_stream = nullptr;
void* g_ws = nullptr;
size_t g_ws_bytes = 0;

// The binning (sorted records, permutation, cell table and ordered work list)
// that the last hacc_sr_force or hacc_sr_force_vjp left in the workspace,
// named by a token for hacc_sr_force_vjp_binned.  Every other call that
// writes the workspace, and any change of workspace or stream, retires it.
struct KeptBinning {
    uint64_t token;          // 0: none
    int64_t n;
    double box;
    float r_cut;
    const void* ws;
    hipStream_t stream;
    int* perm;
};
KeptBinning g_kept{};
uint64_t g_kept_serial = 0;

void retire_binning() { g_kept.token = 0; }
char g_err[256] = "";

constexpr int kTimers = 8;
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events[kTimers];

int hip_fail(hipError_t e) {
    std::snprintf(g_err, sizeof(g_err), "HIP error %d: %s", (int)e,
                  hipGetErrorString(e));
    return HACC_SR_EHIP;
}

#define HIP_TRY(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_);       \
    } while (0)

// Records an event pair around the launches made by `body`, when timing is on.
template <typename F>
int timed(int which, F body) {
    hipEvent_t a = nullptr, b = nullptr;
    if (g_timing) {
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        HIP_TRY(hipEventRecord(a, g_stream));
    }
    const int rc = body();
    if (g_timing) {
        HIP_TRY(hipEventRecord(b, g_stream));
        g_events[which].emplace_back(a, b);
    }
    return rc;
}

bool is_fin(double v) { return std::isfinite(v); }

int key_bits(int64_t ncell) {
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < ncell) ++bits;
    return bits;
}


// Validates (n, box, r_cut) and derives the chaining-mesh geometry.
int make_geom(int64_t n, double box, float r_cut, Geom* g) {
    if (n < 0 || !is_fin(box) || box == 0.0 || !is_fin(r_cut) || !(r_cut > 0.0f))
        return HACC_SR_EINVAL;
    if (n >= (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    const double b = std::fabs(box);
    double Nd = std::floor(b / (double)r_cut);
    if (Nd < 1.0) Nd = 1.0;
    if (box > 0.0 && Nd < 3.0) return HACC_SR_EDOMAIN;   // 27 distinct neighbours
    if (Nd > 1290.0) return HACC_SR_EDOMAIN;             // N^3 + 1 < 2^31
    int N = (int)Nd;
    while (N > 1 && b / N < (double)r_cut) --N;
    if (box > 0.0 && N < 3) return HACC_SR_EDOMAIN;
    // the work list's capacity (see layout_for) must fit an int
    const int64_t ncell = (int64_t)N * N * N;
    if (2 * std::min<int64_t>(n, ncell) + n / kItemI + 1 > (int64_t)INT32_MAX)
        return HACC_SR_EDOMAIN;
    g->N = N;
    g->periodic = box > 0.0 ? 1 : 0;
    g->box = b;
    g->Lc = b / N;
    g->Lc_f = (float)g->Lc;
    const int cb = key_bits((int64_t)N * N * N);
    g->sbits = cb + 6 <= 31 ? 6 : (cb + 3 <= 31 ? 3 : 0);
    return HACC_SR_OK;
}

int make_params(float r_cut, float eps, const float* poly, PairParams* P) {
    if (!poly || !is_fin(eps) || !(eps > 0.0f)) return HACC_SR_EINVAL;
    for (int k = 0; k < 6; ++k)
        if (!is_fin(poly[k])) return HACC_SR_EINVAL;
    const double rc2 = (double)r_cut * (double)r_cut;
    const float alpha = (float)(2.0 / rc2);
    const float beta = (float)(-1.0 - (double)alpha * (double)eps);
    if (!is_fin(alpha) || !is_fin(beta)) return HACC_SR_EINVAL;
    // s as a function of t: s = (t - beta) / alpha - eps = u0 + u1 t, exact
    // for the float32 alpha and beta the kernel uses.  Compose poly(s(t)).
    const double u1 = 1.0 / (double)alpha;
    const double u0 = -(double)beta / (double)alpha - (double)eps;
    double b[6] = {0, 0, 0, 0, 0, 0};
    double pw[6] = {1, 0, 0, 0, 0, 0};   // coefficients of (u0 + u1 t)^k
    for (int k = 0; k < 6; ++k) {
        for (int m = 0; m <= k; ++m) b[m] += (double)poly[k] * pw[m];
        double nx[6] = {0, 0, 0, 0, 0, 0};
        for (int m = 0; m <= k && m < 5; ++m) {
            nx[m] += u0 * pw[m];
            nx[m + 1] += u1 * pw[m];
        }
        std::memcpy(pw, nx, sizeof(pw));
    }
    P->alpha = alpha;
    P->beta = beta;
    P->eps = eps;
    P->rc2e = (float)(rc2 + (double)eps);
    // A margin far above float32 rounding: a culled source fails the
    // kernel's own cut-off test against every target of the item.
    P->cull2 = (float)(rc2 * (1.0 + 1.0 / 4096.0));
    for (int m = 0; m < 6; ++m) P->b[m] = (float)b[m];
    // 2 d(poly)/ds = 2 alpha d(poly)/dt
    for (int m = 1; m < 6; ++m) {
        P->db2[m - 1] = (float)(2.0 * (double)alpha * m * b[m]);
        P->dq3[m - 1] = (float)(2.0 * (double)alpha * m * b[m] / 3.0);
    }
    for (int m = 0; m < 6; ++m)
        if (!is_fin(P->b[m])) return HACC_SR_EINVAL;
    for (int m = 0; m < 5; ++m)
        if (!is_fin(P->db2[m]) || !is_fin(P->dq3[m])) return HACC_SR_EINVAL;
    return HACC_SR_OK;
}

// ---------------------------------------------------------------- workspace

struct Layout {
    size_t keys_a, vals_a, keys_b, vals_b, counts, hist, scan_tmp, rec,
        gsorted, cell_items, items, items_sorted, bucket_of, buckets,
        cell_window, col_cost, col_xcd;
    // RCB fat leaves only
    size_t leafmark, leafidx, leaf_start, leaf_items, cell_list, rcb_counters;
    bool rcb;
    size_t total;
    int64_t ncell;
    int max_items;
    int radix_nb;
    int digit_bits;   // radix digit width (8..11)
    int passes;       // radix passes over the sort key
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Work items of the RCB work list: a leaf of c particles gives floor(c / 64)
// full items and at most two more, and there are at most n leaves.
int64_t rcb_item_bound(int64_t n) { return 2 * n + n / kItemI + 1; }

Layout layout_for(int64_t n, const Geom& g, bool rcb = false) {
    Layout L{};
    const int nn = (int)n;
    L.rcb = rcb;
    L.ncell = (int64_t)g.N * g.N * g.N;
    // a cell of c targets gives floor(c / 64) full items and at most two more
    L.max_items = (int)(2 * std::min<int64_t>(n, L.ncell) + n / kItemI + 1);
    if (rcb) L.max_items = (int)std::max<int64_t>(L.max_items, rcb_item_bound(n));
    L.radix_nb = radix_blocks(nn > 0 ? nn : 1);
    // at most three stable passes: digits of ceil(bits / 3) bits, 8 to 11
    const int bits = key_bits(L.ncell) + g.sbits;
    L.digit_bits = std::min(kMaxDigitBits, std::max(8, (bits + 2) / 3));
    L.passes = (bits + L.digit_bits - 1) / L.digit_bits;
    const int64_t hist_n = ((int64_t)1 << L.digit_bits) * L.radix_nb;
    int64_t scan_n = std::max<int64_t>(hist_n, L.ncell + 1);
    if (rcb) scan_n = std::max<int64_t>(scan_n, n + 2);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const size_t ni = sizeof(int) * (size_t)std::max<int64_t>(n, 1);
    L.keys_a = take(ni);
    L.vals_a = take(ni);
    L.keys_b = take(ni);
    L.vals_b = take(ni);
    L.counts = take(sizeof(int) * (size_t)(L.ncell + 1));
    L.hist = take(sizeof(int) * (size_t)hist_n);
    L.scan_tmp = take(sizeof(int) * scan_tmp_ints((int)scan_n));
    L.rec = take(sizeof(float4) * (size_t)std::max<int64_t>(n, 1));
    // also holds the records in input order during binning (the sorted
    // cotangents are gathered only after the records)
    L.gsorted = take(sizeof(float4) * (size_t)std::max<int64_t>(n, 1));
    L.cell_items = take(sizeof(int) * (size_t)(L.ncell + 1));
    L.items = take(sizeof(WorkItem) * (size_t)L.max_items);
    L.items_sorted = take(sizeof(WorkItem) * (size_t)L.max_items);
    L.bucket_of = take(sizeof(int) * (size_t)L.max_items);
    L.buckets = take(sizeof(int) * kOrderInts);
    L.cell_window = take(sizeof(int) * (size_t)L.ncell);
    L.col_cost = take(sizeof(unsigned long long) * (size_t)(g.N) * (size_t)g.N);
    L.col_xcd = take(sizeof(int) * (size_t)(g.N) * (size_t)g.N);
    if (rcb) {
        const size_t n2 = sizeof(int) * (size_t)(n + 2);
        L.leafmark = take(n2);
        L.leafidx = take(n2);
        L.leaf_start = take(n2);
        L.leaf_items = take(n2);
        L.cell_list = take(sizeof(int) * (size_t)L.ncell);
        L.rcb_counters = take(sizeof(int) * 4);
    }
    L.total = off + 256;   // slack for aligning the base pointer
    return L;
}

template <typename T>
T* ws_at(size_t off) {
    const uintptr_t base = ((uintptr_t)g_ws + 255) & ~(uintptr_t)255;
    return reinterpret_cast<T*>(base + off);
}

int check_ws(const Layout& L) {
    if (!g_ws || g_ws_bytes < L.total) return HACC_SR_ENOSPACE;
    return HACC_SR_OK;
}


// Bins into the workspace; returns (through the pointers) where cell_start,
// the permutation and the sorted records ended up.
int bin_impl(const double* pos, const float* mass, int64_t n, const Geom& g,
             const Layout& L, int* cell_start, int** perm_out, float4* rec,
             int* perm_user, int** keys_out = nullptr, int** spare_out = nullptr) {
    const int nn = (int)n;
    int* ka = ws_at<int>(L.keys_a);
    int* va = ws_at<int>(L.vals_a);
    int* kb = ws_at<int>(L.keys_b);
    int* vb = ws_at<int>(L.vals_b);
    int* hist = ws_at<int>(L.hist);
    int* tmp = ws_at<int>(L.scan_tmp);
    float4* rec_in = ws_at<float4>(L.gsorted);
    const int ncp = (int)(L.ncell + 1);
    HIP_TRY(launch_cell_keys(pos, mass, nn, g, ka, va, rec_in, g_stream));
    for (int p = 0; p < L.passes; ++p) {
        HIP_TRY(launch_radix_pass(ka, va, kb, vb, nn, L.digit_bits * p,
                                  L.digit_bits, hist, tmp, g_stream));
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    HIP_TRY(launch_fill_i32(cell_start, ncp, 0, g_stream));
    HIP_TRY(launch_cell_hist(ka, nn, g.sbits, cell_start, g_stream));
    HIP_TRY(launch_scan_exclusive(cell_start, cell_start, ncp, tmp, g_stream));
    HIP_TRY(launch_gather_records(rec_in, va, nn, rec, g_stream));
    if (perm_user) {
        HIP_TRY(hipMemcpyAsync(perm_user, va, sizeof(int) * (size_t)nn,
                               hipMemcpyDeviceToDevice, g_stream));
    }
    *perm_out = va;
    if (keys_out) *keys_out = ka;
    if (spare_out) *spare_out = vb;
    return HACC_SR_OK;
}

// Builds the RCB fat leaves inside the cells of a binning made by bin_impl
// (reordering the sorted records and permutation within each cell) and the
// leaf table.  Returns the device count of leaves.
int rcb_impl(int64_t n, const Geom& g, const Layout& L, const int* cell_start,
             float4* rec, int* perm, int* spare, int leaf_max, int4* nodes,
             float* split, const int** n_leaves_dev) {
    int* leafmark = ws_at<int>(L.leafmark);
    int* leafidx = ws_at<int>(L.leafidx);
    int* counters = ws_at<int>(L.rcb_counters);
    HIP_TRY(launch_rcb(cell_start, (int)L.ncell, (int)n, leaf_max,
                       ws_at<int>(L.cell_list), counters, rec, perm,
                       ws_at<float4>(L.gsorted), spare, leafmark, nodes, split,
                       g_stream));
    HIP_TRY(launch_leaf_table(leafmark, leafidx, (int)n, ws_at<int>(L.scan_tmp),
                              ws_at<int>(L.leaf_start), g_stream));
    *n_leaves_dev = leafidx + n;
    return HACC_SR_OK;
}

// Work list of the RCB leaves, cost-ordered like the chaining-mesh one.
// Reads the number of leaves back to the host (one stream synchronisation)
// to size the launch.
int worklist_rcb_impl(int64_t n, const int* cell_start, const int* keys_sorted,
                      const Geom& g, const Layout& L, const int* n_leaves_dev,
                      const WorkItem** items_out, const int** n_items_dev,
                      int* grid_items) {
    int nleaves = 0;
    HIP_TRY(hipMemcpyAsync(&nleaves, n_leaves_dev, sizeof(int), hipMemcpyDeviceToHost,
                           g_stream));
    HIP_TRY(hipStreamSynchronize(g_stream));
    int* li = ws_at<int>(L.leaf_items);
    WorkItem* items = ws_at<WorkItem>(L.items);
    WorkItem* sorted = ws_at<WorkItem>(L.items_sorted);
    int* tmp = ws_at<int>(L.scan_tmp);
    HIP_TRY(launch_leaf_items(ws_at<int>(L.leaf_start), n_leaves_dev, nleaves, keys_sorted,
                              g.sbits, li, tmp, items, g_stream));
    const int64_t bound = n / kItemI + 2 * (int64_t)nleaves + 1;
    // cell windows and the XCD of each column of cells, for the cost order
    int* cw = ws_at<int>(L.cell_window);
    int* cx = ws_at<int>(L.col_xcd);
    HIP_TRY(launch_items_count(cell_start, g, ws_at<int>(L.cell_items), cw,
                               ws_at<unsigned long long>(L.col_cost), cx, g_stream));
    HIP_TRY(launch_items_order(items, li + nleaves, (int)bound, cw, cx, g,
                               ws_at<int>(L.bucket_of), ws_at<int>(L.buckets), sorted,
                               g_stream));
    *items_out = sorted;
    *n_items_dev = li + nleaves;
    *grid_items = (int)bound;
    return HACC_SR_OK;
}

int check_leaf_max(int32_t leaf_max) {
    return (leaf_max >= 1 && leaf_max <= (1 << 20)) ? HACC_SR_OK : HACC_SR_EINVAL;
}


// Builds the cost-ordered work list; returns the device counter of items.
int worklist_impl(const int* cell_start, const Geom& g, const Layout& L,
                  const WorkItem** items_out, const int** n_items_dev) {
    int* ci = ws_at<int>(L.cell_items);
    WorkItem* items = ws_at<WorkItem>(L.items);
    WorkItem* sorted = ws_at<WorkItem>(L.items_sorted);
    int* bof = ws_at<int>(L.bucket_of);
    int* bc = ws_at<int>(L.buckets);
    int* tmp = ws_at<int>(L.scan_tmp);
    const int nc = (int)L.ncell;
    HIP_TRY(launch_fill_i32(ci + nc, 1, 0, g_stream));
    int* cw = ws_at<int>(L.cell_window);
    int* cx = ws_at<int>(L.col_xcd);
    HIP_TRY(launch_items_count(cell_start, g, ci, cw,
                               ws_at<unsigned long long>(L.col_cost), cx,
                               g_stream));
    HIP_TRY(launch_scan_exclusive(ci, ci, nc + 1, tmp, g_stream));
    HIP_TRY(launch_items_write(cell_start, g, ci, items, g_stream));
    HIP_TRY(launch_items_order(items, ci + nc, L.max_items, cw, cx, g, bof, bc,
                               sorted, g_stream));
    *items_out = sorted;
    *n_items_dev = ci + nc;
    return HACC_SR_OK;
}

// Shared by the RCB force and VJP: binning, RCB leaves, leaf work list.
int rcb_prepare(const double* pos, const float* mass, int64_t n, const Geom& g,
                const Layout& L, int leaf_max, const float* grad_acc, int** perm_out,
                const WorkItem** items, const int** nitems, int* grid) {
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    int *perm = nullptr, *keys = nullptr, *spare = nullptr;
    const int* nl_dev = nullptr;
    int rc = timed(2, [&] {
        int r = bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr, &keys, &spare);
        if (r != HACC_SR_OK) return r;
        return HACC_SR_OK;
    });
    if (rc != HACC_SR_OK) return rc;
    rc = timed(6, [&] {
        return rcb_impl(n, g, L, cs, rec, perm, spare, leaf_max, nullptr, nullptr, &nl_dev);
    });
    if (rc != HACC_SR_OK) return rc;
    if (grad_acc) {
        // the cotangents follow the final (RCB) order
        HIP_TRY(launch_gather_vec3(grad_acc, perm, (int)n, ws_at<float4>(L.gsorted),
                                   g_stream));
    }
    rc = timed(3, [&] {
        return worklist_rcb_impl(n, cs, keys, g, L, nl_dev, items, nitems, grid);
    });
    *perm_out = perm;
    return rc;
}

int pm_check(double box, int32_t ng, float sigma, int32_t n_s) {
    if (!is_fin(box) || !(box > 0.0)) return HACC_SR_EINVAL;
    if (ng < 8 || ng > 512 || (ng & (ng - 1))) return HACC_SR_EINVAL;
    if (!is_fin(sigma) || sigma < 0.0f || n_s < 0 || n_s > 16) return HACC_SR_EINVAL;
    return HACC_SR_OK;
}

// The short-range force of hacc_sr_force on a validated call: binning, work
// list and the pair kernel, into out_acc.
int force_into(const double* pos, const float* mass, int64_t n, const Geom& g,
               const PairParams& P, const Layout& L, float* out_acc, int** perm_out = nullptr) {
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    int* perm = nullptr;
    int rc = timed(2, [&] { return bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr); });
    if (rc != HACC_SR_OK) return rc;
    const WorkItem* items;
    const int* nitems;
    rc = timed(3, [&] { return worklist_impl(cs, g, L, &items, &nitems); });
    if (rc != HACC_SR_OK) return rc;
    if (perm_out) *perm_out = perm;
    return timed(0, [&] {
        HIP_TRY(launch_pair_force(items, L.max_items, nitems, rec, cs, perm, g,
                                  P, out_acc, g_stream));
        return HACC_SR_OK;
    });
}

void keep_binning(int64_t n, double box, float r_cut, int* perm) {
    g_kept = KeptBinning{++g_kept_serial, n, box, r_cut, g_ws, g_stream, perm};
}

// ---------------------------------------------------------------- no-alloc

// Scratch memory of hacc_sr_force_noalloc, for callers that cannot allocate:
// a file-scope device array that every GPU the library runs on holds until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory, so its device address is taken once per device with
// hipGetSymbolAddress and only that address is used.
constexpr size_t kNoAllocBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return HACC_SR_EDOMAIN;
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HACC_SR_OK;
}

// Points the workspace at the scratch array for the duration of one call.
struct WorkspaceSwap {
    void* ws;
    size_t bytes;
    WorkspaceSwap(void* p, size_t b) : ws(g_ws), bytes(g_ws_bytes) {
        g_ws = p;
        g_ws_bytes = b;
    }
    ~WorkspaceSwap() {
        g_ws = ws;
        g_ws_bytes = bytes;
    }
};

}  // namespace

extern "C" {

int hacc_sr_force_noalloc(const double* pos, const float* mass, int64_t n, double box,
                          float r_cut, float eps, const float* poly, float* out_acc) {
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (n > 0 && (!pos || !mass || !out_acc)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g);
    if (L.total > kNoAllocBytes) return HACC_SR_ENOSPACE;
    void* base = nullptr;
    if ((rc = scratch_for_current_device(&base)) != HACC_SR_OK) return rc;
    WorkspaceSwap swap(base, kNoAllocBytes);
    // the same kernels as hacc_sr_force; every buffer that must start at
    // zero is cleared by a fill kernel, so earlier contents do not matter
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    int* perm = nullptr;
    if ((rc = bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr)) != HACC_SR_OK) return rc;
    const WorkItem* items;
    const int* nitems;
    if ((rc = worklist_impl(cs, g, L, &items, &nitems)) != HACC_SR_OK) return rc;
    HIP_TRY(launch_pair_force(items, L.max_items, nitems, rec, cs, perm, g, P, out_acc,
                              g_stream));
    return HACC_SR_OK;
}


#ifndef HSR_SOURCE_SHA256
#error "build with -DHSR_SOURCE_SHA256=<sha256 of the sources> (paper_1211_4864_amd/build.py)"
#endif

int hacc_sr_version(void) { return 201; }

const char* hacc_sr_source_hash(void) { return HSR_SOURCE_SHA256; }

const char* hacc_sr_strerror(int code) {
    switch (code) {
        case HACC_SR_OK: return "ok";
        case HACC_SR_EINVAL: return "invalid argument";
        case HACC_SR_EDOMAIN: return "unsupported domain: periodic box below 3 r_cut, n >= 2^31, too many cells or work items";
        case HACC_SR_ENOSPACE: return "workspace unset or too small";
        case HACC_SR_EHIP: return g_err[0] ? g_err : "HIP runtime error";
        case HACC_SR_ESTALE: return "the binning named by the token is no longer in the workspace";
        default: return "unknown error code";
    }
}

int hacc_sr_set_stream(void* stream) {
    if ((hipStream_t)stream != g_stream) retire_binning();
    g_stream = (hipStream_t)stream;
    return HACC_SR_OK;
}

int hacc_sr_grid_dim(double box, float r_cut, int32_t* cells_per_axis) {
    if (!cells_per_axis) return HACC_SR_EINVAL;
    Geom g;
    const int rc = make_geom(0, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    *cells_per_axis = g.N;
    return HACC_SR_OK;
}

int hacc_sr_workspace_bytes(int64_t n, double box, float r_cut, size_t* bytes) {
    if (!bytes) return HACC_SR_EINVAL;
    Geom g;
    const int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    *bytes = layout_for(n, g).total;
    return HACC_SR_OK;
}

int hacc_sr_set_workspace(void* dev_ptr, size_t bytes) {
    if (!dev_ptr && bytes) return HACC_SR_EINVAL;
    if (dev_ptr != g_ws || (dev_ptr ? bytes : 0) != g_ws_bytes) retire_binning();
    g_ws = dev_ptr;
    g_ws_bytes = dev_ptr ? bytes : 0;
    return HACC_SR_OK;
}

int hacc_sr_bin(const double* pos, const float* mass, int64_t n, double box,
                float r_cut, int32_t* cell_start, int32_t* perm,
                float* sorted_rec) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    if (!cell_start) return HACC_SR_EINVAL;
    if (n > 0 && (!pos || !mass || !perm || !sorted_rec)) return HACC_SR_EINVAL;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    return timed(2, [&] {
        if (n == 0) {
            HIP_TRY(launch_fill_i32(cell_start, (int)(L.ncell + 1), 0, g_stream));
            return HACC_SR_OK;
        }
        int* p;
        return bin_impl(pos, mass, n, g, L, cell_start, &p,
                        reinterpret_cast<float4*>(sorted_rec), perm);
    });
}

int hacc_sr_force(const double* pos, const float* mass, int64_t n, double box,
                  float r_cut, float eps, const float* poly, float* out_acc) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (n > 0 && (!pos || !mass || !out_acc)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* perm = nullptr;
    if ((rc = force_into(pos, mass, n, g, P, L, out_acc, &perm)) != HACC_SR_OK) return rc;
    keep_binning(n, box, r_cut, perm);
    return HACC_SR_OK;
}

int hacc_sr_full_step(double* pos, double* vel, const float* mass, int64_t n, double box,
                      int32_t ng, float sigma, int32_t n_s, float r_cut, float eps,
                      const float* poly, double dt, int32_t n_c, float* acc_scratch) {
    retire_binning();
    int rc = pm_check(box, ng, sigma, n_s);
    if (rc != HACC_SR_OK) return rc;
    Geom g;
    if ((rc = make_geom(n, box, r_cut, &g)) != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (!is_fin(dt) || n_c < 1 || n_c > 1000000) return HACC_SR_EINVAL;
    if (n > 0 && (!pos || !vel || !mass || !acc_scratch)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g);
    if (!g_ws || g_ws_bytes < std::max(L.total, pm_workspace_bytes(ng, n) + 256))
        return HACC_SR_ENOSPACE;
    const int64_t m = 3 * n;
    auto pm_kick = [&](double t) {
        int r = timed(7, [&] {
            HIP_TRY(launch_pm_accel(pos, mass, (int)n, box, ng, sigma, n_s, ws_at<char>(0),
                                    acc_scratch, g_stream));
            return HACC_SR_OK;
        });
        if (r != HACC_SR_OK) return r;
        HIP_TRY(launch_kick(vel, acc_scratch, m, t, g_stream));
        return HACC_SR_OK;
    };
    // M_lr(t/2) (M_sr(t/n_c))^n_c M_lr(t/2)
    if ((rc = pm_kick(0.5 * dt)) != HACC_SR_OK) return rc;
    const double h = dt / n_c;
    for (int c = 0; c < n_c; ++c) {
        HIP_TRY(launch_stream(pos, vel, m, 0.5 * h, box, g_stream));
        if ((rc = force_into(pos, mass, n, g, P, L, acc_scratch)) != HACC_SR_OK) return rc;
        HIP_TRY(launch_kick(vel, acc_scratch, m, h, g_stream));
        HIP_TRY(launch_stream(pos, vel, m, 0.5 * h, box, g_stream));
    }
    return pm_kick(0.5 * dt);
}

int hacc_sr_force_vjp(const double* pos, const float* mass, int64_t n,
                      double box, float r_cut, float eps, const float* poly,
                      const float* grad_acc, double* out_grad_pos) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (n > 0 && (!pos || !mass || !grad_acc || !out_grad_pos))
        return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    float4* gs = ws_at<float4>(L.gsorted);
    int* perm = nullptr;
    rc = timed(2, [&] {
        const int r = bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr);
        if (r != HACC_SR_OK) return r;
        HIP_TRY(launch_gather_vec3(grad_acc, perm, (int)n, gs, g_stream));
        return HACC_SR_OK;
    });
    if (rc != HACC_SR_OK) return rc;
    const WorkItem* items;
    const int* nitems;
    rc = timed(3, [&] { return worklist_impl(cs, g, L, &items, &nitems); });
    if (rc != HACC_SR_OK) return rc;
    rc = timed(1, [&] {
        HIP_TRY(launch_pair_vjp(items, L.max_items, nitems, rec, gs, cs, perm, g,
                                P, out_grad_pos, g_stream));
        return HACC_SR_OK;
    });
    if (rc == HACC_SR_OK) keep_binning(n, box, r_cut, perm);
    return rc;
}

int hacc_sr_binning_token(uint64_t* token) {
    if (!token) return HACC_SR_EINVAL;
    *token = g_kept.token;
    return HACC_SR_OK;
}

int hacc_sr_force_vjp_binned(uint64_t token, int64_t n, double box, float r_cut, float eps,
                             const float* poly, const float* grad_acc,
                             double* out_grad_pos) {
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (n > 0 && (!grad_acc || !out_grad_pos)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    if (token == 0 || token != g_kept.token || n != g_kept.n || box != g_kept.box ||
        r_cut != g_kept.r_cut || g_ws != g_kept.ws || g_stream != g_kept.stream)
        return HACC_SR_ESTALE;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    float4* gs = ws_at<float4>(L.gsorted);
    int* perm = g_kept.perm;
    const WorkItem* items = ws_at<WorkItem>(L.items_sorted);
    const int* nitems = ws_at<int>(L.cell_items) + L.ncell;
    rc = timed(2, [&] {
        HIP_TRY(launch_gather_vec3(grad_acc, perm, (int)n, gs, g_stream));
        return HACC_SR_OK;
    });
    if (rc != HACC_SR_OK) return rc;
    return timed(1, [&] {
        HIP_TRY(launch_pair_vjp(items, L.max_items, nitems, rec, gs, cs, perm, g,
                                P, out_grad_pos, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_workspace_bytes_rcb(int64_t n, double box, float r_cut, size_t* bytes) {
    if (!bytes) return HACC_SR_EINVAL;
    Geom g;
    const int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    if (rcb_item_bound(n) > (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    *bytes = layout_for(n, g, true).total;
    return HACC_SR_OK;
}

int hacc_sr_rcb_bin(const double* pos, const float* mass, int64_t n, double box,
                    float r_cut, int32_t leaf_max, int32_t* cell_start, int32_t* perm,
                    float* sorted_rec, int32_t* leaf_start, int32_t* n_leaves,
                    int32_t* nodes, float* node_split, int32_t* n_nodes) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    if ((rc = check_leaf_max(leaf_max)) != HACC_SR_OK) return rc;
    if (rcb_item_bound(n) > (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    if (!cell_start || !leaf_start || !n_leaves) return HACC_SR_EINVAL;
    if (n > 0 && (!pos || !mass || !perm || !sorted_rec)) return HACC_SR_EINVAL;
    const bool want_nodes = nodes || node_split || n_nodes;
    if (want_nodes && !(nodes && node_split && n_nodes)) return HACC_SR_EINVAL;
    const Layout L = layout_for(n, g, true);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    return timed(2, [&] {
        if (n == 0) {
            HIP_TRY(launch_fill_i32(cell_start, (int)(L.ncell + 1), 0, g_stream));
            HIP_TRY(launch_fill_i32(leaf_start, 1, 0, g_stream));
            HIP_TRY(launch_fill_i32(n_leaves, 1, 0, g_stream));
            if (want_nodes) HIP_TRY(launch_fill_i32(n_nodes, 1, 0, g_stream));
            return HACC_SR_OK;
        }
        int* cs = ws_at<int>(L.counts);
        float4* rec = ws_at<float4>(L.rec);
        int *p = nullptr, *spare = nullptr;
        int r = bin_impl(pos, mass, n, g, L, cs, &p, rec, nullptr, nullptr, &spare);
        if (r != HACC_SR_OK) return r;
        const int* nl_dev = nullptr;
        r = rcb_impl(n, g, L, cs, rec, p, spare, leaf_max,
                     want_nodes ? reinterpret_cast<int4*>(nodes) : nullptr, node_split,
                     &nl_dev);
        if (r != HACC_SR_OK) return r;
        const int nn = (int)n;
        HIP_TRY(hipMemcpyAsync(cell_start, cs, sizeof(int) * (size_t)(L.ncell + 1),
                               hipMemcpyDeviceToDevice, g_stream));
        HIP_TRY(hipMemcpyAsync(perm, p, sizeof(int) * (size_t)nn, hipMemcpyDeviceToDevice,
                               g_stream));
        HIP_TRY(hipMemcpyAsync(sorted_rec, rec, sizeof(float4) * (size_t)nn,
                               hipMemcpyDeviceToDevice, g_stream));
        HIP_TRY(hipMemcpyAsync(n_leaves, nl_dev, sizeof(int), hipMemcpyDeviceToDevice,
                               g_stream));
        // leaves + 1 entries; the caller's array holds n + 1
        HIP_TRY(hipMemcpyAsync(leaf_start, ws_at<int>(L.leaf_start),
                               sizeof(int) * (size_t)(nn + 1), hipMemcpyDeviceToDevice,
                               g_stream));
        if (want_nodes)
            HIP_TRY(hipMemcpyAsync(n_nodes, ws_at<int>(L.rcb_counters) + 1, sizeof(int),
                                   hipMemcpyDeviceToDevice, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_force_rcb(const double* pos, const float* mass, int64_t n, double box,
                      float r_cut, float eps, const float* poly, int32_t leaf_max,
                      float* out_acc) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if ((rc = check_leaf_max(leaf_max)) != HACC_SR_OK) return rc;
    if (rcb_item_bound(n) > (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    if (n > 0 && (!pos || !mass || !out_acc)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g, true);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* perm = nullptr;
    const WorkItem* items;
    const int* nitems;
    int grid = 0;
    rc = rcb_prepare(pos, mass, n, g, L, leaf_max, nullptr, &perm, &items, &nitems, &grid);
    if (rc != HACC_SR_OK) return rc;
    return timed(0, [&] {
        HIP_TRY(launch_pair_force(items, grid, nitems, ws_at<float4>(L.rec),
                                  ws_at<int>(L.counts), perm, g, P, out_acc, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_force_vjp_rcb(const double* pos, const float* mass, int64_t n, double box,
                          float r_cut, float eps, const float* poly, int32_t leaf_max,
                          const float* grad_acc, double* out_grad_pos) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if ((rc = check_leaf_max(leaf_max)) != HACC_SR_OK) return rc;
    if (rcb_item_bound(n) > (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    if (n > 0 && (!pos || !mass || !grad_acc || !out_grad_pos)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g, true);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* perm = nullptr;
    const WorkItem* items;
    const int* nitems;
    int grid = 0;
    rc = rcb_prepare(pos, mass, n, g, L, leaf_max, grad_acc, &perm, &items, &nitems, &grid);
    if (rc != HACC_SR_OK) return rc;
    return timed(1, [&] {
        HIP_TRY(launch_pair_vjp(items, grid, nitems, ws_at<float4>(L.rec),
                                ws_at<float4>(L.gsorted), ws_at<int>(L.counts), perm, g, P,
                                out_grad_pos, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_force_plain(const double* pos, const float* mass, int64_t n,
                        double box, float r_cut, float eps, const float* poly,
                        float* out_acc) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (n > 0 && (!pos || !mass || !out_acc)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    int *perm = nullptr, *keys = nullptr;
    rc = bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr, &keys);
    if (rc != HACC_SR_OK) return rc;
    return timed(4, [&] {
        HIP_TRY(launch_force_plain(rec, keys, cs, perm, (int)n, g,
                                   P, out_acc,
                                   g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_force_vjp_plain(const double* pos, const float* mass, int64_t n,
                            double box, float r_cut, float eps,
                            const float* poly, const float* grad_acc,
                            double* out_grad_pos) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    PairParams P;
    if ((rc = make_params(r_cut, eps, poly, &P)) != HACC_SR_OK) return rc;
    if (n > 0 && (!pos || !mass || !grad_acc || !out_grad_pos))
        return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    float4* gs = ws_at<float4>(L.gsorted);
    int *perm = nullptr, *keys = nullptr;
    rc = bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr, &keys);
    if (rc != HACC_SR_OK) return rc;
    HIP_TRY(launch_gather_vec3(grad_acc, perm, (int)n, gs, g_stream));
    return timed(5, [&] {
        HIP_TRY(launch_vjp_plain(rec, gs, keys, cs, perm, (int)n, g,
                                 P, out_grad_pos,
                                 g_stream));
        return HACC_SR_OK;
    });
}


int hacc_sr_pm_workspace_bytes(int32_t ng, int64_t n, size_t* bytes) {
    if (!bytes || ng < 8 || ng > 512 || (ng & (ng - 1)) || n < 0) return HACC_SR_EINVAL;
    if (n >= (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    *bytes = pm_workspace_bytes(ng, n) + 256;
    return HACC_SR_OK;
}

int hacc_sr_pm_accel(const double* pos, const float* mass, int64_t n, double box,
                     int32_t ng, float sigma, int32_t n_s, float* out_acc) {
    retire_binning();
    int rc = pm_check(box, ng, sigma, n_s);
    if (rc != HACC_SR_OK) return rc;
    if (n < 0) return HACC_SR_EINVAL;
    if (n >= (int64_t)INT32_MAX) return HACC_SR_EDOMAIN;
    if (n > 0 && (!pos || !mass || !out_acc)) return HACC_SR_EINVAL;
    if (n == 0) return HACC_SR_OK;
    if (!g_ws || g_ws_bytes < pm_workspace_bytes(ng, n) + 256) return HACC_SR_ENOSPACE;
    return timed(7, [&] {
        HIP_TRY(launch_pm_accel(pos, mass, (int)n, box, ng, sigma, n_s, ws_at<char>(0),
                                out_acc, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_kick(double* vel, const float* acc, int64_t n, double dt) {
    if (n < 0 || !is_fin(dt)) return HACC_SR_EINVAL;
    if (n > 0 && (!vel || !acc)) return HACC_SR_EINVAL;
    HIP_TRY(launch_kick(vel, acc, 3 * n, dt, g_stream));
    return HACC_SR_OK;
}

int hacc_sr_stream(double* pos, const double* vel, int64_t n, double dt,
                   double box) {
    if (n < 0 || !is_fin(dt) || !is_fin(box)) return HACC_SR_EINVAL;
    if (n > 0 && (!pos || !vel)) return HACC_SR_EINVAL;
    HIP_TRY(launch_stream(pos, vel, 3 * n, dt, box, g_stream));
    return HACC_SR_OK;
}

int hacc_sr_kick_adjoint(const double* grad_vel, float* grad_acc, int64_t n,
                         double dt) {
    if (n < 0 || !is_fin(dt)) return HACC_SR_EINVAL;
    if (n > 0 && (!grad_vel || !grad_acc)) return HACC_SR_EINVAL;
    HIP_TRY(launch_kick_adjoint(grad_vel, grad_acc, 3 * n, dt, g_stream));
    return HACC_SR_OK;
}

int hacc_sr_count_pairs(const double* pos, int64_t n, double box, float r_cut,
                        float eps, int64_t* out_counts) {
    retire_binning();
    Geom g;
    int rc = make_geom(n, box, r_cut, &g);
    if (rc != HACC_SR_OK) return rc;
    if (!is_fin(eps) || !(eps > 0.0f) || !out_counts) return HACC_SR_EINVAL;
    if (n > 0 && !pos) return HACC_SR_EINVAL;
    const float zero_poly[6] = {0, 0, 0, 0, 0, 0};
    PairParams P;
    if ((rc = make_params(r_cut, eps, zero_poly, &P)) != HACC_SR_OK) return rc;
    const Layout L = layout_for(n, g);
    if ((rc = check_ws(L)) != HACC_SR_OK) return rc;
    HIP_TRY(launch_fill_i32(reinterpret_cast<int*>(out_counts), 4, 0, g_stream));
    if (n == 0) return HACC_SR_OK;
    int* cs = ws_at<int>(L.counts);
    float4* rec = ws_at<float4>(L.rec);
    int* perm = nullptr;
    rc = bin_impl(pos, nullptr, n, g, L, cs, &perm, rec, nullptr);
    if (rc != HACC_SR_OK) return rc;
    const WorkItem* items;
    const int* nitems;
    if ((rc = worklist_impl(cs, g, L, &items, &nitems)) != HACC_SR_OK) return rc;
    HIP_TRY(launch_pair_count(items, L.max_items, nitems, rec, cs, g, P,
                              reinterpret_cast<unsigned long long*>(out_counts),
                              g_stream));
    return HACC_SR_OK;
}

int hacc_sr_valu_probe(int kind, int waves_per_simd, double* out) {
    retire_binning();
    if (kind < 0 || kind > 3 || waves_per_simd < 1 || waves_per_simd > 8 || !out)
        return HACC_SR_EINVAL;
    const size_t need = probe_scratch_bytes();
    if (!g_ws || g_ws_bytes < need + 256) return HACC_SR_ENOSPACE;
    void* scratch = ws_at<char>(0);
    int dev = 0, wall_khz = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int simds = 4 * ncu;
    const int waves = simds * waves_per_simd;
    // a few milliseconds per launch at 8 waves per SIMD
    const int base = kind == 1 ? 8192 : (kind == 2 ? 2048 : 32768);
    const int iters = base * 8 / waves_per_simd;
    const int reps = 5;
    HIP_TRY(launch_valu_probe(kind, waves, 64, scratch, g_stream));   // warm-up
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(a, g_stream));
    for (int r = 0; r < reps; ++r)
        HIP_TRY(launch_valu_probe(kind, waves, iters, scratch, g_stream));
    HIP_TRY(hipEventRecord(b, g_stream));
    HIP_TRY(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    // per-wave loop clocks of the last launch
    std::vector<unsigned long long> clk(2 * (size_t)waves);
    HIP_TRY(hipMemcpyAsync(clk.data(), ws_at<char>(probe_clock_offset()),
                           clk.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, g_stream));
    HIP_TRY(hipStreamSynchronize(g_stream));
    double cyc = 0.0, wall = 0.0;
    for (int w = 0; w < waves; ++w) {
        cyc += (double)clk[2 * w];
        wall += (double)clk[2 * w + 1];
    }
    cyc /= waves;
    wall /= waves;
    const double ops_wave = (double)iters * probe_ops_per_iter(kind);
    const double per_launch_s = 1e-3 * (double)ms / reps;
    out[0] = ops_wave * waves * kWave / per_launch_s;       // lane operations / s
    out[1] = wall > 0.0 ? cyc / (wall / ((double)wall_khz * 1e3)) / 1e9 : 0.0;   // GHz
    out[2] = cyc / ops_wave;                                // cycles between a wave's instructions
    out[3] = 1e3 * per_launch_s;
    return HACC_SR_OK;
}

int hacc_sr_timing_enable(int enable) {
    for (auto& v : g_events) {
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        v.clear();
    }
    g_timing = enable != 0;
    return HACC_SR_OK;
}

int hacc_sr_timing_read(int kernel, int64_t* launches, double* total_ms) {
    if (kernel < 0 || kernel >= kTimers || !launches || !total_ms)
        return HACC_SR_EINVAL;
    double tot = 0.0;
    for (auto& pr : g_events[kernel]) {
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
    }
    *launches = (int64_t)g_events[kernel].size();
    *total_ms = tot;
    return HACC_SR_OK;
}

}  // extern "C"
