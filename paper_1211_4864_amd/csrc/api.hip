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
char g_err[256] = "";

constexpr int kTimers = 6;
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
    for (int m = 1; m < 6; ++m) P->db2[m - 1] = (float)(2.0 * (double)alpha * m * b[m]);
    for (int m = 0; m < 6; ++m)
        if (!is_fin(P->b[m])) return HACC_SR_EINVAL;
    for (int m = 0; m < 5; ++m)
        if (!is_fin(P->db2[m])) return HACC_SR_EINVAL;
    return HACC_SR_OK;
}

// ---------------------------------------------------------------- workspace

struct Layout {
    size_t keys_a, vals_a, keys_b, vals_b, counts, hist, scan_tmp, rec,
        gsorted, cell_items, items, items_sorted, bucket_of, buckets,
        cell_window, col_cost, col_xcd;
    size_t total;
    int64_t ncell;
    int max_items;
    int radix_nb;
    int digit_bits;   // radix digit width (8..11)
    int passes;       // radix passes over the sort key
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout_for(int64_t n, const Geom& g) {
    Layout L{};
    const int nn = (int)n;
    L.ncell = (int64_t)g.N * g.N * g.N;
    // a cell of c targets gives floor(c / 64) full items and at most two more
    L.max_items = (int)(2 * std::min<int64_t>(n, L.ncell) + n / kItemI + 1);
    L.radix_nb = radix_blocks(nn > 0 ? nn : 1);
    // at most three stable passes: digits of ceil(bits / 3) bits, 8 to 11
    const int bits = key_bits(L.ncell) + g.sbits;
    L.digit_bits = std::min(kMaxDigitBits, std::max(8, (bits + 2) / 3));
    L.passes = (bits + L.digit_bits - 1) / L.digit_bits;
    const int64_t hist_n = ((int64_t)1 << L.digit_bits) * L.radix_nb;
    const int64_t scan_n = std::max<int64_t>(hist_n, L.ncell + 1);
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
             int* perm_user, int** keys_out = nullptr) {
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
    return HACC_SR_OK;
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

}  // namespace

extern "C" {

int hacc_sr_version(void) { return 100; }

const char* hacc_sr_strerror(int code) {
    switch (code) {
        case HACC_SR_OK: return "ok";
        case HACC_SR_EINVAL: return "invalid argument";
        case HACC_SR_EDOMAIN: return "unsupported domain: periodic box below 3 r_cut, n >= 2^31, too many cells or work items";
        case HACC_SR_ENOSPACE: return "workspace unset or too small";
        case HACC_SR_EHIP: return g_err[0] ? g_err : "HIP runtime error";
        default: return "unknown error code";
    }
}

int hacc_sr_set_stream(void* stream) {
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
    g_ws = dev_ptr;
    g_ws_bytes = dev_ptr ? bytes : 0;
    return HACC_SR_OK;
}

int hacc_sr_bin(const double* pos, const float* mass, int64_t n, double box,
                float r_cut, int32_t* cell_start, int32_t* perm,
                float* sorted_rec) {
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
    int* perm = nullptr;
    rc = timed(2, [&] { return bin_impl(pos, mass, n, g, L, cs, &perm, rec, nullptr); });
    if (rc != HACC_SR_OK) return rc;
    const WorkItem* items;
    const int* nitems;
    rc = timed(3, [&] { return worklist_impl(cs, g, L, &items, &nitems); });
    if (rc != HACC_SR_OK) return rc;
    return timed(0, [&] {
        HIP_TRY(launch_pair_force(items, L.max_items, nitems, rec, cs, perm, g,
                                  P, out_acc, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_force_vjp(const double* pos, const float* mass, int64_t n,
                      double box, float r_cut, float eps, const float* poly,
                      const float* grad_acc, double* out_grad_pos) {
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
    return timed(1, [&] {
        HIP_TRY(launch_pair_vjp(items, L.max_items, nitems, rec, gs, cs, perm, g,
                                P, out_grad_pos, g_stream));
        return HACC_SR_OK;
    });
}

int hacc_sr_force_plain(const double* pos, const float* mass, int64_t n,
                        double box, float r_cut, float eps, const float* poly,
                        float* out_acc) {
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
