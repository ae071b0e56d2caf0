// xrt_batch.cpp -- batches of x-ray transform problems (include/xrt_batch.h):
// per-problem plans and buffers, the work lists of the persistent forward and
// adjoint launches, HIP graph capture and the run-time autotuner.  The
// arithmetic is in xrt_kernels.hip; this file only builds tables and
// sequences launches.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "xrt.h"
#include "xrt_batch.h"
#include "xrt_internal.h"

namespace {

constexpr uint64_t kBatchMagic = 0x58525442'41544348ull;  // "XRTBATCH"

}  // namespace

struct xrt_batch {
    uint64_t magic;
    int count;
    std::vector<xrt_plan*> plans;
    std::vector<float*> coeffs, sino, back;   // device addresses inside `buf`
    float* buf = nullptr;
    float* spart = nullptr;                   // per-strip forward partial sums of all problems
    void* probs = nullptr;                    // device table of launch records
    int2* items_f = nullptr;
    int2* items_a = nullptr;                  // adjoint, vertical lines
    int2* items_ah = nullptr;                 // adjoint, horizontal lines
    int nitems_f = 0, nitems_a = 0, nitems_ah = 0;
    unsigned int* counters = nullptr;         // [0] forward, [1] adjoint vertical, [2] adjoint horizontal
    int64_t total_lines = 0;
    int cus = 0;
    xrt_batch_config cfg;
    std::vector<int> order_f, order_a;        // problems by decreasing work
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph = nullptr;
};

namespace {

thread_local char g_err[256] = "";

xrt_status hip_fail(const char* what, hipError_t e)
{
    snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
    xrt::set_last_error(g_err);
    return XRT_EHIP;
}

#define XB_CHECK(call, what)                             \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(what, e_); \
    } while (0)

bool batch_ok(const xrt_batch* b) { return b && b->magic == kBatchMagic; }

bool config_ok(const xrt_batch_config& c)
{
    const bool lines = c.lines_per_item == 256 || c.lines_per_item == 512 || c.lines_per_item == 1024 ||
                       c.lines_per_item == 2048;
    return lines && c.fwd_blocks_per_cu >= 1 && c.fwd_blocks_per_cu <= 32 && c.adj_blocks_per_cu >= 1 &&
           c.adj_blocks_per_cu <= 32;
}

// adjoint tiles of a plan: kTileI x kTileJ for the vertical lines, the
// transposed kTileJ x kTileI for the horizontal ones
int tiles_of(const xrt_plan* p, bool horizontal = false)
{
    const int ti = horizontal ? xrt::kTileJ : xrt::kTileI, tj = horizontal ? xrt::kTileI : xrt::kTileJ;
    return ((p->g.nx + ti - 1) / ti) * ((p->g.ny + tj - 1) / tj);
}

// forward list: every block of lines of every problem, largest problem first
xrt_status build_forward_items(xrt_batch* b)
{
    std::vector<int2> it;
    for (int p : b->order_f) {
        const int64_t m = b->plans[p]->m;
        const int64_t nb = (m + b->cfg.lines_per_item - 1) / b->cfg.lines_per_item;
        const int ns = xrt::batch_strips(b->plans[p]);
        for (int st = 0; st < ns; ++st)
            for (int64_t k = 0; k < nb; ++k) it.push_back(make_int2(p, (int)(st * nb + k)));
    }
    if (b->items_f) (void)hipFree(b->items_f);
    b->items_f = nullptr;
    b->nitems_f = (int)it.size();
    if (it.empty()) return XRT_OK;
    XB_CHECK(hipMalloc((void**)&b->items_f, it.size() * sizeof(int2)), "hipMalloc");
    XB_CHECK(hipMemcpy(b->items_f, it.data(), it.size() * sizeof(int2), hipMemcpyHostToDevice), "hipMemcpy");
    return XRT_OK;
}

// adjoint lists: every tile of every problem, largest problem first, one
// list per orientation
xrt_status build_adjoint_items(xrt_batch* b)
{
    for (int h = 0; h < 2; ++h) {
        std::vector<int2> it;
        for (int p : b->order_a)
            for (int t = 0; t < tiles_of(b->plans[p], h == 1); ++t) it.push_back(make_int2(p, t));
        int2** dst = h ? &b->items_ah : &b->items_a;
        (h ? b->nitems_ah : b->nitems_a) = (int)it.size();
        XB_CHECK(hipMalloc((void**)dst, std::max<size_t>(1, it.size()) * sizeof(int2)), "hipMalloc");
        if (!it.empty())
            XB_CHECK(hipMemcpy(*dst, it.data(), it.size() * sizeof(int2), hipMemcpyHostToDevice), "hipMemcpy");
    }
    return XRT_OK;
}

void release(xrt_batch* b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    for (xrt_plan* p : b->plans) xrt_plan_destroy(p);
    void* ptrs[] = {b->buf, b->spart, b->probs, b->items_f, b->items_a, b->items_ah, b->counters};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    b->magic = 0;
}

hipError_t enqueue_forward(xrt_batch* b, hipStream_t s)
{
    for (int p = 0; p < b->count; ++p) {
        hipError_t e = xrt::launch_layouts(b->plans[p], b->coeffs[p], s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = xrt::launch_reset_counters(b->counters, 3, s);
    if (e == hipSuccess && b->nitems_f > 0)
        e = xrt::launch_batch_forward(b->probs, b->items_f, b->nitems_f, b->counters, b->cfg.lines_per_item,
                                      b->cus * b->cfg.fwd_blocks_per_cu, s);
    for (int p = 0; p < b->count && e == hipSuccess; ++p)
        e = xrt::launch_batch_fwd_reduce(b->probs, p, b->plans[p]->m, s);
    return e;
}

hipError_t enqueue_adjoint(xrt_batch* b, hipStream_t s)
{
    for (int p = 0; p < b->count; ++p) {
        hipError_t e = xrt::launch_sort_sino(b->plans[p], b->sino[p], s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = xrt::launch_reset_counters(b->counters, 3, s);
    if (e != hipSuccess || b->nitems_a == 0) return e;
    // the horizontal lines add into the images the vertical launch wrote
    e = xrt::launch_batch_adjoint(b->probs, b->items_a, b->nitems_a, b->counters + 1,
                                  b->cus * b->cfg.adj_blocks_per_cu, 0, s);
    if (e != hipSuccess) return e;
    e = xrt::launch_batch_adjoint(b->probs, b->items_ah, b->nitems_ah, b->counters + 2,
                                  b->cus * b->cfg.adj_blocks_per_cu, 1, s);
    if (e != hipSuccess) return e;
    int64_t max_m = 0;
    for (xrt_plan* p : b->plans) max_m = std::max<int64_t>(max_m, p->m);
    return xrt::launch_batch_nonfinite(b->probs, b->count, max_m, s);
}

void drop_graph(xrt_batch* b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

}  // namespace

extern "C" {

xrt_status xrt_batch_create(const xrt_problem* problems, int32_t count, void* stream, xrt_batch** out)
{
    if (!problems || !out || count < 1) return XRT_EINVAL;
    *out = nullptr;
    for (int p = 0; p < count; ++p)
        if (!xrt::valid_basis(problems[p].degree)) return XRT_EDEGREE;
    hipStream_t s = (hipStream_t)stream;
    xrt_batch* b = new xrt_batch();
    b->magic = kBatchMagic;
    b->count = count;
    b->cfg.fwd_blocks_per_cu = 4;
    b->cfg.lines_per_item = 256;
    b->cfg.adj_blocks_per_cu = 2;
    b->cfg.pad = 0;
    for (int p = 0; p < count; ++p) {
        xrt_plan* pl = nullptr;
        xrt_status st = xrt::plan_create(problems[p].grid, problems[p].degree, &problems[p].lines, stream, false, &pl);
        if (st != XRT_OK) {
            release(b);
            delete b;
            return st;
        }
        b->plans.push_back(pl);
    }
    // buffers: per problem coefficients, sinogram, back-projection
    int64_t total = 0;
    std::vector<int64_t> oc(count), os(count), ob(count), op(count);
    int64_t spart_total = 0;
    for (int p = 0; p < count; ++p) {
        const int64_t npix = (int64_t)b->plans[p]->g.nx * b->plans[p]->g.ny, m = b->plans[p]->m;
        oc[p] = total;
        total += (npix + 63) / 64 * 64;
        os[p] = total;
        total += (std::max<int64_t>(m, 1) + 63) / 64 * 64;
        ob[p] = total;
        total += (npix + 63) / 64 * 64;
        b->total_lines += m;
        op[p] = spart_total;
        spart_total += (int64_t)xrt::batch_strips(b->plans[p]) * ((m + 63) / 64 * 64);
    }
    hipError_t e = hipMalloc((void**)&b->buf, total * sizeof(float));
    if (e == hipSuccess) e = hipMemsetAsync(b->buf, 0, total * sizeof(float), s);
    if (e == hipSuccess) e = hipMalloc((void**)&b->spart, std::max<int64_t>(spart_total, 1) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&b->counters, 3 * sizeof(unsigned int));
    if (e == hipSuccess) e = hipMalloc(&b->probs, (size_t)count * xrt::batch_prob_size());
    if (e != hipSuccess) {
        xrt_status st = e == hipErrorOutOfMemory ? XRT_ENOMEM : hip_fail("xrt_batch_create", e);
        release(b);
        delete b;
        return st;
    }
    std::vector<unsigned char> table((size_t)count * xrt::batch_prob_size());
    for (int p = 0; p < count; ++p) {
        b->coeffs.push_back(b->buf + oc[p]);
        b->sino.push_back(b->buf + os[p]);
        b->back.push_back(b->buf + ob[p]);
        xrt::batch_fill(b->plans[p], b->sino[p], b->back[p], b->spart + op[p],
                        table.data() + (size_t)p * xrt::batch_prob_size());
    }
    e = hipMemcpy(b->probs, table.data(), table.size(), hipMemcpyHostToDevice);
    // order problems by decreasing work: lines x rows for the forward, per-tile work for the adjoint
    std::vector<double> wf(count), wa(count);
    for (int p = 0; p < count; ++p) {
        const xrt_plan* pl = b->plans[p];
        wf[p] = (double)pl->m_valid * std::max(pl->g.nx, pl->g.ny);
        wa[p] = wf[p] / tiles_of(pl);
    }
    b->order_f.resize(count);
    b->order_a.resize(count);
    std::iota(b->order_f.begin(), b->order_f.end(), 0);
    std::iota(b->order_a.begin(), b->order_a.end(), 0);
    std::stable_sort(b->order_f.begin(), b->order_f.end(), [&](int x, int y) { return wf[x] > wf[y]; });
    std::stable_sort(b->order_a.begin(), b->order_a.end(), [&](int x, int y) { return wa[x] > wa[y]; });
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    xrt_status st = e == hipSuccess ? XRT_OK : hip_fail("xrt_batch_create", e);
    if (st == XRT_OK) st = build_forward_items(b);
    if (st == XRT_OK) st = build_adjoint_items(b);
    if (st == XRT_OK && hipStreamSynchronize(s) != hipSuccess) st = hip_fail("hipStreamSynchronize", hipGetLastError());
    if (st != XRT_OK) {
        release(b);
        delete b;
        return st;
    }
    *out = b;
    return XRT_OK;
}

void xrt_batch_destroy(xrt_batch* b)
{
    if (!batch_ok(b)) return;
    (void)hipDeviceSynchronize();
    release(b);
    delete b;
}

xrt_status xrt_batch_buffers(const xrt_batch* b, int32_t p, float** coeffs, float** sino, float** back)
{
    if (!batch_ok(b) || p < 0 || p >= b->count) return XRT_EINVAL;
    if (coeffs) *coeffs = b->coeffs[p];
    if (sino) *sino = b->sino[p];
    if (back) *back = b->back[p];
    return XRT_OK;
}

xrt_status xrt_batch_info(const xrt_batch* b, int64_t* total_lines, int32_t* fwd_items, int32_t* adj_items)
{
    if (!batch_ok(b)) return XRT_EINVAL;
    if (total_lines) *total_lines = b->total_lines;
    if (fwd_items) *fwd_items = b->nitems_f;
    if (adj_items) *adj_items = b->nitems_a + b->nitems_ah;
    return XRT_OK;
}

xrt_status xrt_batch_forward(xrt_batch* b, void* stream)
{
    if (!batch_ok(b)) return XRT_EINVAL;
    XB_CHECK(enqueue_forward(b, (hipStream_t)stream), "batch forward");
    return XRT_OK;
}

xrt_status xrt_batch_adjoint(xrt_batch* b, void* stream)
{
    if (!batch_ok(b)) return XRT_EINVAL;
    XB_CHECK(enqueue_adjoint(b, (hipStream_t)stream), "batch adjoint");
    return XRT_OK;
}

xrt_status xrt_batch_run(xrt_batch* b, int32_t use_graph, void* stream)
{
    if (!batch_ok(b)) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        XB_CHECK(enqueue_forward(b, s), "batch forward");
        XB_CHECK(enqueue_adjoint(b, s), "batch adjoint");
        return XRT_OK;
    }
    if (!b->graph) {
        // capture on the batch's own stream (the caller's may be the null
        // stream, which cannot be captured); the graph is replayed on `stream`
        hipGraph_t g = nullptr;
        XB_CHECK(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t e = enqueue_forward(b, b->capture_stream);
        if (e == hipSuccess) e = enqueue_adjoint(b, b->capture_stream);
        hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->graph = nullptr;
            return hip_fail("graph capture", e);
        }
    }
    XB_CHECK(hipGraphLaunch(b->graph, s), "hipGraphLaunch");
    return XRT_OK;
}

xrt_status xrt_batch_get_config(const xrt_batch* b, xrt_batch_config* cfg)
{
    if (!batch_ok(b) || !cfg) return XRT_EINVAL;
    *cfg = b->cfg;
    return XRT_OK;
}

xrt_status xrt_batch_set_config(xrt_batch* b, const xrt_batch_config* cfg)
{
    if (!batch_ok(b) || !cfg || !config_ok(*cfg)) return XRT_EINVAL;
    XB_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");   // the old work list may be in use
    const bool relist = cfg->lines_per_item != b->cfg.lines_per_item;
    b->cfg = *cfg;
    b->cfg.pad = 0;
    drop_graph(b);
    if (relist) return build_forward_items(b);
    return XRT_OK;
}

xrt_status xrt_batch_autotune(xrt_batch* b, int32_t reps, xrt_batch_config* best, void* stream)
{
    if (!batch_ok(b) || reps < 1) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    XB_CHECK(hipEventCreate(&e0), "hipEventCreate");
    XB_CHECK(hipEventCreate(&e1), "hipEventCreate");
    auto time_it = [&](bool fwd, float* ms) -> xrt_status {
        XB_CHECK(fwd ? enqueue_forward(b, s) : enqueue_adjoint(b, s), "autotune warm-up");
        XB_CHECK(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < reps; ++r) XB_CHECK(fwd ? enqueue_forward(b, s) : enqueue_adjoint(b, s), "autotune run");
        XB_CHECK(hipEventRecord(e1, s), "hipEventRecord");
        XB_CHECK(hipEventSynchronize(e1), "hipEventSynchronize");
        XB_CHECK(hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime");
        return XRT_OK;
    };
    xrt_batch_config c = b->cfg, win = b->cfg;
    float best_f = 1e30f, best_a = 1e30f;
    xrt_status st = XRT_OK;
    const int bpc[] = {1, 2, 4, 8, 16};
    const int lpi[] = {256, 512, 1024, 2048};
    for (int L : lpi) {
        for (int k : bpc) {
            c.fwd_blocks_per_cu = k;
            c.lines_per_item = L;
            if ((st = xrt_batch_set_config(b, &c)) != XRT_OK) break;
            float ms = 0.f;
            if ((st = time_it(true, &ms)) != XRT_OK) break;
            if (ms < best_f) {
                best_f = ms;
                win.fwd_blocks_per_cu = k;
                win.lines_per_item = L;
            }
        }
        if (st != XRT_OK) break;
    }
    if (st == XRT_OK) {
        c = win;
        for (int k : {1, 2, 4, 8}) {
            c.adj_blocks_per_cu = k;
            if ((st = xrt_batch_set_config(b, &c)) != XRT_OK) break;
            float ms = 0.f;
            if ((st = time_it(false, &ms)) != XRT_OK) break;
            if (ms < best_a) {
                best_a = ms;
                win.adj_blocks_per_cu = k;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != XRT_OK) return st;
    st = xrt_batch_set_config(b, &win);
    if (st == XRT_OK && best) *best = b->cfg;
    return st;
}

}  // extern "C"
