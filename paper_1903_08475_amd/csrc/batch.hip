// Batched solve of many independent fields with different plans (grid
// sizes, lmax) through persistent work-queue kernels, one per stage
// (moment contraction, radial scans, expansion).  Each stage's queue holds
// the tiles of every field, ordered longest first; the persistent blocks
// pull tiles until the queue is empty.  The three launches, the counter
// reset and (split forms) one launch that splits the inputs of every field
// are captured once in a hipGraph and replayed; a call only refreshes
// the fields' rho/phi pointers (kept in device memory, read by the kernels)
// and launches the graph on the caller's stream.  The expansion kernels also
// stamp the device wall clock when the last tile of a field is done, so the
// per-field completion times inside one batched call can be read back.
#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "mpg_internal.h"

namespace mpg {
namespace {

// Start of a batched solve: clears the queue heads and the per-field
// completion stamps and stamps the start time (stamps[n]).
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
    size_t *split_offs = nullptr;  // input split: first thread of each field, and the total
    int *heads = nullptr;
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
        if (split_offs) (void)hipFree(split_offs);
        if (heads) (void)hipFree(heads);
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

hipError_t build(Batch &b, const std::vector<const Plan *> &plans, int dtype) {
    b.plans = plans;
    for (const Plan *p : plans) b.epochs.push_back(p->tune_epoch);
    b.dtype = dtype;
    b.precision = plans[0]->precision;
    const int n = (int)plans.size();
    const bool split = b.precision != MPG_FP64;
    // tile sides of the moment contraction (rows) and the expansion
    const int T1 = split ? kSplitTile : kF64Tile1, T2 = split ? kSplitTile : kF64Tile2;

    // work items per stage, longest first
    std::vector<int> order(n);
    for (int f = 0; f < n; ++f) order[f] = f;
    std::vector<BatchItem> i1, is, i2;
    std::vector<int> kchunk(n), tiles_e(n), tiles_o(n);
    std::vector<Plan> q(n);
    for (int f = 0; f < n; ++f) {
        q[f] = *plans[f];
        q[f].splitk = choose_splitk(q[f], 1);
        const Plan &p = q[f];
        if (split) {
            SplitArgs g = split_args(p, 1, nullptr, nullptr, dtype);
            b.sa.push_back(g);
            kchunk[f] = g.kchunk;
            tiles_e[f] = g.tiles_e;
            tiles_o[f] = g.tiles_o;
        } else {
            F64Args g = f64_args(p, 1, nullptr, nullptr, dtype);
            b.fa.push_back(g);
            kchunk[f] = g.kchunk;
            tiles_e[f] = g.tiles_e;
            tiles_o[f] = g.tiles_o;
        }
        b.sc.push_back(scan_args(p, 1, split));
    }
    // GEMM1 items, longest first: K per item, times the products per
    // product of the split forms (six, or three off the tier's column pairs)
    std::vector<std::pair<long long, BatchItem>> c1;
    for (int f = 0; f < n; ++f) {
        const Plan &p = q[f];
        const int rt = (p.n_r + T1 - 1) / T1;
        // the split GEMM1 takes column tiles in pairs (per parity block)
        const int pe = (tiles_e[f] + 1) / 2, po = (tiles_o[f] + 1) / 2;
        const int ct = split ? pe + po : tiles_e[f] + tiles_o[f];
        for (int z = 0; z < p.splitk; ++z)
            for (int m = 0; m < rt; ++m)
                for (int c = 0; c < ct; ++c) {
                    bool six = true;
                    if (split) six = c < pe ? c < six_pairs(p.six_e, pe) : c - pe < six_pairs(p.six_o, po);
                    c1.push_back({(long long)kchunk[f] * (six ? 6 : 3), BatchItem{f, c, m, z}});
                }
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
        // the split GEMM2 takes angular tiles in pairs
        const int rt = (p.n_r + T2 - 1) / T2;
        const int at = split ? (p.n2() / T2 + 1) / 2 : p.n2() / T2;
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

    const size_t asz = split ? sizeof(SplitArgs) * n : sizeof(F64Args) * n;
    CHECK(hipMalloc(&b.args_dev, asz));
    CHECK(hipMalloc(&b.scan_dev, sizeof(ScanArgs) * n));
    CHECK(hipMalloc(&b.items_dev, sizeof(BatchItem) * all.size()));
    CHECK(hipMalloc(&b.heads, sizeof(int) * 4));
    CHECK(hipMalloc(&b.stamps, sizeof(unsigned long long) * (n + 2)));
    CHECK(hipMemset(b.stamps, 0, sizeof(unsigned long long) * (n + 2)));
    const BatchTrack track{b.stamps, n};
    CHECK(hipMemcpy(b.scan_dev, b.sc.data(), sizeof(ScanArgs) * n, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(b.items_dev, all.data(), sizeof(BatchItem) * all.size(), hipMemcpyHostToDevice));
    std::vector<size_t> offs(n + 1, 0);
    for (int f = 0; f < n; ++f) offs[f + 1] = offs[f] + (split ? split_input_threads(q[f], 1) : 0);
    if (split) {
        CHECK(hipMalloc(&b.split_offs, sizeof(size_t) * (n + 1)));
        CHECK(hipMemcpy(b.split_offs, offs.data(), sizeof(size_t) * (n + 1), hipMemcpyHostToDevice));
    }

    // capture: counter reset and start stamp (a kernel, not a memset), the input
    // split of every field (split forms) and the three stages
    CHECK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    CHECK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    const int cus = cu_count();
    hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(256), 0, b.cap, b.heads, 4, b.stamps, n);
    const BatchItem *it1 = b.items_dev, *its = b.items_dev + b.n1, *it2 = b.items_dev + b.n1 + b.ns;
    hipError_t e;
    e = hipSuccess;
    if (split) {
        e = batch_split_input_bf16((const SplitArgs *)b.args_dev, b.split_offs, n, offs[n], dtype, b.cap);
        if (e == hipSuccess)
            e = batch_gemm1_bf16((const SplitArgs *)b.args_dev, it1, b.n1, b.heads + 0, dtype, cus, b.cap);
        if (e == hipSuccess) e = batch_scan(b.scan_dev, its, b.ns, b.heads + 1, 2 * cus, b.cap);
        if (e == hipSuccess)
            e = batch_gemm2_bf16((const SplitArgs *)b.args_dev, it2, b.n2, b.heads + 2, dtype, cus, track, b.cap);
    } else {
        e = batch_gemm1_f64((const F64Args *)b.args_dev, it1, b.n1, b.heads + 0, dtype, 4 * cus, b.cap);
        if (e == hipSuccess) e = batch_scan(b.scan_dev, its, b.ns, b.heads + 1, 2 * cus, b.cap);
        if (e == hipSuccess)
            e = batch_gemm2_f64((const F64Args *)b.args_dev, it2, b.n2, b.heads + 2, dtype, 4 * cus, track, b.cap);
    }
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
        hipError_t e = build(*b, plans, dtype);
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

hipError_t batch_field_times(const std::vector<const Plan *> &plans, int dtype, double *ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    Batch *b = find(plans, dtype);
    if (!b) return hipErrorNotFound;
    const int n = (int)plans.size();
    CHECK(hipStreamSynchronize(plans[0]->stream));
    std::vector<unsigned long long> st(n + 2);
    CHECK(hipMemcpy(st.data(), b->stamps, sizeof(unsigned long long) * (n + 2), hipMemcpyDeviceToHost));
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
