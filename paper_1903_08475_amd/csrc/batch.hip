// Batched solve of many independent fields with different plans (grid
// sizes, lmax).  Split forms: one persistent kernel takes the items of
// every stage (input split, moment contraction, radial scans, expansion)
// of every field from one queue, in an order fixed on the host
// (batch_order.h) so that each item's producers come before it; per-field
// counters make an item wait for its field's previous stage, so fields
// finish one after another instead of all at the end.  FP64: one persistent
// work-queue kernel per stage, each queue holding the tiles of every field,
// longest first.  The launches and a counter reset are captured once in a
// hipGraph per plan list and dtype and replayed; a call only refreshes the
// fields' rho/phi pointers (kept in device memory, read by the kernels) and
// launches the graph on the caller's stream.  Per-field completion times
// inside one batched call are stamped on the device and can be read back.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "mpg_internal.h"

namespace mpg {
namespace {

// Start of a batched solve: clears the queue heads (and the fused
// kernel's counters and status word, n_heads of them in all) and the
// per-field completion stamps, and stamps the start time (stamps[n]).
__global__ void k_batch_start(int *heads, int n_heads, unsigned long long *stamps, int n) {
    for (int t = threadIdx.x; t < n_heads || t < n + 2; t += blockDim.x) {
        if (t < n_heads) heads[t] = 0;
        if (t < n + 2 && t != n) stamps[t] = 0;
    }
    if (threadIdx.x == 0) stamps[n] = wall_clock64();
}

struct Batch {
    std::vector<const Plan *> plans;
    std::vector<int> epochs;  // the plans' tuning epochs when the batch was built
    int dtype = MPG_F64, precision = MPG_FP64;
    int n1 = 0, ns = 0, n2 = 0;
    std::vector<SplitArgs> sa;
    std::vector<F64Args> fa;
    std::vector<ScanArgs> sc;
    void *args_dev = nullptr;
    ScanArgs *scan_dev = nullptr;
    BatchItem *items_dev = nullptr;
    int *heads = nullptr;        // fused: [0] queue head, [1] status, [2 ..] finished items per field and stage
    int *need = nullptr;         // fused: items per field and stage
    FusedItem *fitems = nullptr;
    unsigned long long *stamps = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~Batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (args_dev) (void)hipFree(args_dev);
        if (scan_dev) (void)hipFree(scan_dev);
        if (items_dev) (void)hipFree(items_dev);
        if (heads) (void)hipFree(heads);
        if (need) (void)hipFree(need);
        if (fitems) (void)hipFree(fitems);
        if (stamps) (void)hipFree(stamps);
    }
};

std::mutex g_mu;
std::vector<Batch *> g_batches;

int cu_count() {
    static int n = 0;
    if (!n) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            n = prop.multiProcessorCount;
        if (n <= 0) n = 256;
    }
    return n;
}

#define CHECK(x)                                  \
    do {                                          \
        hipError_t e_ = (x);                      \
        if (e_ != hipSuccess) return e_;          \
    } while (0)

// Work of one field (one field of the plan) in the fused kernel's units,
// with the plan's block shapes and scan chunks.
FieldShape field_shape(const Plan &plan) {
    Plan p = plan;
    p.gemm1_rows = p.gemm1_rows_batch;  // a batch's moment shape
    FieldShape sh;
    const int rt = (p.n_r + kSplitTile - 1) / kSplitTile;
    const int nb1 = p.gemm1_rows == 2 ? 1 : 2;  // column tiles per moment block
    sh.split_units = (int)(split_input_threads(p, 1) / 2048);
    sh.rows1 = p.gemm1_rows == 2 ? (rt + 1) / 2 : rt;
    sh.units_e = (p.tiles_e() + nb1 - 1) / nb1;
    sh.units_o = (p.tiles_o() + nb1 - 1) / nb1;
    sh.six_e = six_units(p.six_e, sh.units_e, nb1);
    sh.six_o = p.fold ? six_units(p.six_o, sh.units_o, nb1) : 0;
    sh.kang = p.kang();
    sh.splitk_max = p.splitk;
    // a single solve's K split choice fills the chip with one field's tiles;
    // in a batch the other fields fill it, so only the item length counts
    sh.splitk_min = 1;
    sh.scan_blocks = (p.np + 63) / 64;
    sh.n_r = p.n_r;
    sh.chunks = scan_args(p, 1, true).chunks;
    const int at = p.n2() / kSplitTile;
    sh.rows2 = p.gemm2_rows == 2 ? (rt + 1) / 2 : rt;
    sh.cols2 = p.gemm2_rows == 2 ? at : (at + 1) / 2;
    if (p.fold) {
        const int ne = p.ne_p / kSlabK, no = p.no_p / kSlabK;
        const int e3 = three_slabs(ne, p.six_e / kSlabK), o3 = three_slabs(no, p.six_o / kSlabK);
        sh.k2_three = e3 + o3;
        sh.k2_six = (ne - e3) + (no - o3);
    } else {
        const int ns = p.kq() / kSlabK, n3 = three_slabs(ns, p.six_e / kSlabK);
        sh.k2_three = n3;
        sh.k2_six = ns - n3;
    }
    return sh;
}

// polls of a stage wait before it gives up (about 4 s; MPG_BATCH_SPIN_LIMIT
// overrides it when the batch is built, to exercise the give-up path)
int spin_limit() {
    const char *v = getenv("MPG_BATCH_SPIN_LIMIT");
    const long x = v ? strtol(v, nullptr, 10) : 0;
    return x > 0 && x < (1L << 30) ? (int)x : (1 << 24);
}

// Split forms: every stage of every field in one persistent kernel (one
// block per CU), items in the order of batch_order.h; each field's K split
// as fused_splitk chooses.
hipError_t build_fused(Batch &b, const std::vector<const Plan *> &plans, int dtype) {
    b.plans = plans;
    for (const Plan *p : plans) b.epochs.push_back(p->tune_epoch);
    b.dtype = dtype;
    b.precision = plans[0]->precision;
    const int n = (int)plans.size();
    const int cus = cu_count();
    std::vector<FieldShape> shapes(n);
    for (int f = 0; f < n; ++f) shapes[f] = field_shape(*plans[f]);
    const std::vector<FusedItem> items = fused_items(shapes, cus);
    std::vector<int> need(n * kFusedStages, 0);
    for (const FusedItem &it : items) ++need[it.f * kFusedStages + it.st];
    for (int f = 0; f < n; ++f) {
        Plan q = *plans[f];
        q.splitk = fused_splitk(shapes[f]);
        q.gemm1_rows = q.gemm1_rows_batch;
        b.sa.push_back(split_args(q, 1, nullptr, nullptr, dtype));
        b.sc.push_back(scan_args(q, 1, true));
    }
    b.n1 = (int)items.size();
    const int n_counters = 2 + n * kFusedStages;
    CHECK(hipMalloc(&b.args_dev, sizeof(SplitArgs) * n));
    CHECK(hipMalloc(&b.scan_dev, sizeof(ScanArgs) * n));
    CHECK(hipMalloc(&b.fitems, sizeof(FusedItem) * items.size()));
    CHECK(hipMalloc(&b.heads, sizeof(int) * n_counters));
    CHECK(hipMalloc(&b.need, sizeof(int) * n * kFusedStages));
    CHECK(hipMalloc(&b.stamps, sizeof(unsigned long long) * (n + 2)));
    CHECK(hipMemset(b.stamps, 0, sizeof(unsigned long long) * (n + 2)));
    CHECK(hipMemset(b.heads, 0, sizeof(int) * n_counters));
    CHECK(hipMemcpy(b.scan_dev, b.sc.data(), sizeof(ScanArgs) * n, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(b.fitems, items.data(), sizeof(FusedItem) * items.size(), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(b.need, need.data(), sizeof(int) * n * kFusedStages, hipMemcpyHostToDevice));
    FusedCtl ctl{b.heads, b.heads + 2, b.need, b.heads + 1, b.stamps, n, spin_limit()};

    // capture: counter reset and start stamp (a kernel, not a memset), then
    // the fused kernel
    CHECK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    CHECK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(256), 0, b.cap, b.heads, n_counters, b.stamps, n);
    hipError_t e = batch_fused_bf16((const SplitArgs *)b.args_dev, b.scan_dev, b.fitems, b.n1, ctl, dtype, cus, b.cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b.cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    CHECK(e2);
    b.graph = g;
    CHECK(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    return hipSuccess;
}

// FP64: one persistent work-queue kernel per stage (moments, radial scans,
// expansion), each queue holding the tiles of every field, longest first.
hipError_t build_staged(Batch &b, const std::vector<const Plan *> &plans, int dtype) {
    b.plans = plans;
    for (const Plan *p : plans) b.epochs.push_back(p->tune_epoch);
    b.dtype = dtype;
    b.precision = plans[0]->precision;
    const int n = (int)plans.size();
    const int T2 = kF64Tile2;  // tile side of the expansion

    // work items per stage, longest first
    std::vector<int> order(n);
    for (int f = 0; f < n; ++f) order[f] = f;
    std::vector<BatchItem> i1, is, i2;
    std::vector<Plan> q(n);
    for (int f = 0; f < n; ++f) {
        q[f] = *plans[f];
        q[f].splitk = choose_splitk(q[f], 1);
        q[f].gemm1_rows = q[f].gemm1_rows_batch;
        b.fa.push_back(f64_args(q[f], 1, nullptr, nullptr, dtype));
        b.sc.push_back(scan_args(q[f], 1, false));
    }
    // moment items, longest K first
    std::vector<std::pair<long long, BatchItem>> c1;
    for (int f = 0; f < n; ++f) {
        const Plan &p = q[f];
        const int t1 = b.fa[f].t1;  // the plan's moment tile side
        const int rt = (p.n_r + t1 - 1) / t1, ct = b.fa[f].tiles_e + b.fa[f].tiles_o;
        for (int z = 0; z < p.splitk; ++z)
            for (int m = 0; m < rt; ++m)
                for (int c = 0; c < ct; ++c) c1.push_back({(long long)b.fa[f].kchunk, BatchItem{f, c, m, z}});
    }
    std::stable_sort(c1.begin(), c1.end(), [](const std::pair<long long, BatchItem> &a,
                                              const std::pair<long long, BatchItem> &b) { return a.first > b.first; });
    for (const auto &it : c1) i1.push_back(it.second);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return q[a].n_r * q[a].splitk > q[c].n_r * q[c].splitk; });
    for (int f : order)
        for (int x = 0; x < b.sc[f].col_blocks; ++x) is.push_back({f, x, 0, 0});
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return q[a].np > q[c].np; });
    for (int f : order) {
        const Plan &p = q[f];
        const int rt = (p.n_r + T2 - 1) / T2, at = p.n2() / T2;
        for (int a = 0; a < at; ++a)
            for (int m = 0; m < rt; ++m) i2.push_back({f, m, a, 0});
    }
    b.n1 = (int)i1.size();
    b.ns = (int)is.size();
    b.n2 = (int)i2.size();
    std::vector<BatchItem> all;
    all.reserve(i1.size() + is.size() + i2.size());
    all.insert(all.end(), i1.begin(), i1.end());
    all.insert(all.end(), is.begin(), is.end());
    all.insert(all.end(), i2.begin(), i2.end());

    CHECK(hipMalloc(&b.args_dev, sizeof(F64Args) * n));
    CHECK(hipMalloc(&b.scan_dev, sizeof(ScanArgs) * n));
    CHECK(hipMalloc(&b.items_dev, sizeof(BatchItem) * all.size()));
    CHECK(hipMalloc(&b.heads, sizeof(int) * 4));
    CHECK(hipMalloc(&b.stamps, sizeof(unsigned long long) * (n + 2)));
    CHECK(hipMemset(b.stamps, 0, sizeof(unsigned long long) * (n + 2)));
    const BatchTrack track{b.stamps, n};
    CHECK(hipMemcpy(b.scan_dev, b.sc.data(), sizeof(ScanArgs) * n, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(b.items_dev, all.data(), sizeof(BatchItem) * all.size(), hipMemcpyHostToDevice));

    // capture: counter reset and start stamp (a kernel, not a memset) and the
    // three stages
    CHECK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    CHECK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    const int cus = cu_count();
    hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(256), 0, b.cap, b.heads, 4, b.stamps, n);
    const BatchItem *it1 = b.items_dev, *its = b.items_dev + b.n1, *it2 = b.items_dev + b.n1 + b.ns;
    hipError_t e = batch_gemm1_f64((const F64Args *)b.args_dev, it1, b.n1, b.heads + 0, dtype, 4 * cus, b.cap);
    if (e == hipSuccess) e = batch_scan(b.scan_dev, its, b.ns, b.heads + 1, 2 * cus, b.cap);
    if (e == hipSuccess)
        e = batch_gemm2_f64((const F64Args *)b.args_dev, it2, b.n2, b.heads + 2, dtype, 4 * cus, track, b.cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b.cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    CHECK(e2);
    b.graph = g;
    CHECK(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    return hipSuccess;
}

Batch *find(const std::vector<const Plan *> &plans, int dtype) {
    for (Batch *b : g_batches)
        if (b->dtype == dtype && b->plans == plans) return b;
    return nullptr;
}

// whether a plan's tuning changed since the batch captured its launches
bool stale(const Batch &b) {
    for (size_t f = 0; f < b.plans.size(); ++f)
        if (b.plans[f]->tune_epoch != b.epochs[f]) return true;
    return false;
}

}  // namespace

hipError_t potential_batch(const std::vector<const Plan *> &plans, const void *const *rho, void *const *phi,
                           int dtype, hipStream_t stream) {
    std::lock_guard<std::mutex> lock(g_mu);
    Batch *b = find(plans, dtype);
    if (b && stale(*b)) {
        // captured with older tuning choices: rebuild (after its last replay)
        CHECK(hipStreamSynchronize(stream));
        g_batches.erase(std::find(g_batches.begin(), g_batches.end(), b));
        delete b;
        b = nullptr;
    }
    if (!b) {
        b = new (std::nothrow) Batch();
        if (!b) return hipErrorOutOfMemory;
        hipError_t e = plans[0]->split() ? build_fused(*b, plans, dtype) : build_staged(*b, plans, dtype);
        if (e != hipSuccess) {
            delete b;
            return e;
        }
        g_batches.push_back(b);
    }
    const int n = (int)plans.size();
    if (b->precision != MPG_FP64) {
        for (int f = 0; f < n; ++f) {
            b->sa[f].rho = rho[f];
            b->sa[f].phi = phi[f];
        }
        CHECK(hipMemcpyAsync(b->args_dev, b->sa.data(), sizeof(SplitArgs) * n, hipMemcpyHostToDevice, stream));
    } else {
        for (int f = 0; f < n; ++f) {
            b->fa[f].rho = rho[f];
            b->fa[f].phi = phi[f];
        }
        CHECK(hipMemcpyAsync(b->args_dev, b->fa.data(), sizeof(F64Args) * n, hipMemcpyHostToDevice, stream));
    }
    return hipGraphLaunch(b->exec, stream);
}

BatchChoice batch_choice(const Plan &p) {
    BatchChoice c;
    c.chunks = scan_args(p, 1, true).chunks;
    c.gemm1_rows = p.gemm1_rows_batch;
    if (p.split()) {
        c.splitk = fused_splitk(field_shape(p));
        c.gemm2_rows = p.gemm2_rows;
    } else {
        c.splitk = choose_splitk(p, 1);
        c.gemm2_rows = 1;
    }
    return c;
}

hipError_t batch_field_times(const std::vector<const Plan *> &plans, int dtype, double *ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    Batch *b = find(plans, dtype);
    if (!b) return hipErrorNotFound;
    const int n = (int)plans.size();
    CHECK(hipStreamSynchronize(plans[0]->stream));
    std::vector<unsigned long long> st(n + 2);
    CHECK(hipMemcpy(st.data(), b->stamps, sizeof(unsigned long long) * (n + 2), hipMemcpyDeviceToHost));
    if (b->fitems) {
        int status = 0;
        CHECK(hipMemcpy(&status, b->heads + 1, sizeof(int), hipMemcpyDeviceToHost));
        if (status) return hipErrorLaunchTimeOut;  // a stage wait gave up: the results are incomplete
    }
    int khz = 0;
    CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, plans[0]->device));
    if (khz <= 0) return hipErrorInvalidValue;
    for (int f = 0; f < n; ++f) ms[f] = st[f] > st[n] ? (double)(st[f] - st[n]) / khz : -1.0;
    return hipSuccess;
}

void forget_plan(const Plan *p) {
    std::lock_guard<std::mutex> lock(g_mu);
    for (size_t k = 0; k < g_batches.size();) {
        Batch *b = g_batches[k];
        if (std::find(b->plans.begin(), b->plans.end(), p) != b->plans.end()) {
            (void)hipDeviceSynchronize();
            delete b;
            g_batches.erase(g_batches.begin() + k);
        } else {
            ++k;
        }
    }
}

}  // namespace mpg
