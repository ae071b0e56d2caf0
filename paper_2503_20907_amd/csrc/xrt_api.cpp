// Host side of libxrt.so: argument checks, plan construction, dispatch, and
// the FP64 construction of the knot-transition table used by the kernels.
#include <algorithm>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>


#include "xrt_internal.h"

using namespace xrt;

namespace {

constexpr uint64_t kPlanMagic = 0x58525450'4c414e31ull;  // "XRTPLAN1"
constexpr int kMaxGrid = 32768;
// persistent forward: at most this many bytes of per-strip line sums, and
// workgroups per compute unit (measured on the 2048^2 benchmark: 8 per CU and
// 512 lines per item beat 2, 4 or 16 per CU and 256-2048 lines)
constexpr size_t kMaxStripSums = (size_t)4 << 30;
constexpr int kFwdBlocksPerCU = 8;
// adjoint workgroups per orientation pass that the tile split aims at
constexpr int64_t kAdjUnits = 12288;
// resident adjoint workgroups per CU: the kernels' waves per SIMD (XRT_ADJ_WAVES)
constexpr int64_t kAdjWavesPerSimd = 5;

thread_local char g_last_error[256] = "";

void set_error(const char* what, hipError_t e)
{
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
}

bool finite_grid(const xrt_grid& g)
{
    return isfinite(g.spacing) && isfinite(g.cx) && isfinite(g.cy);
}

xrt_status check_grid(const xrt_grid& g)
{
    if (g.nx <= 0 || g.ny <= 0 || !(g.spacing > 0.0) || !finite_grid(g)) return XRT_EINVAL;
    if (g.nx > kMaxGrid || g.ny > kMaxGrid) return XRT_ESIZE;
    return XRT_OK;
}

xrt_status check_lines(const xrt_lines* L)
{
    if (!L) return XRT_EINVAL;
    if (L->n < 0) return XRT_EINVAL;
    if (L->n >= (int64_t)0x7fffffff) return XRT_ESIZE;
    if (L->kind == XRT_LINES_THETA_Y) {
        if (L->n > 0 && (!L->theta || !L->y)) return XRT_EINVAL;
    } else if (L->kind == XRT_LINES_ENDPOINTS) {
        if (L->n > 0 && !L->endpoints) return XRT_EINVAL;
    } else {
        return XRT_EINVAL;
    }
    return XRT_OK;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Allocs {
    hipStream_t s;
    bool failed = false;
    hipError_t err = hipSuccess;
    template <class T>
    T* get(size_t count)
    {
        if (failed) return nullptr;
        void* p = nullptr;
        size_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 256;
        hipError_t e = hipMallocAsync(&p, bytes, s);
        if (e != hipSuccess) {
            failed = true;
            err = e;
            (void)hipGetLastError();
            return nullptr;
        }
        return (T*)p;
    }
};

void free_plan_memory(xrt_plan* p, hipStream_t s)
{
    void* ptrs[] = {p->xc, p->kap, p->idx, p->off, p->hdr,
                    p->cv, p->dv, p->ch, p->dh, p->sw, p->part, p->spart, p->fctr, p->adj_part};
    for (void* q : ptrs)
        if (q) (void)hipFreeAsync(q, s);
}

}  // namespace

namespace xrt {
void set_last_error(const char* msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

}  // namespace xrt

extern "C" {

const char* xrt_version(void) { return "0.1.0"; }

const char* xrt_status_string(xrt_status st)
{
    switch (st) {
    case XRT_OK: return "ok";
    case XRT_EINVAL: return "invalid argument";
    case XRT_EDEGREE: return "degree must be 0, 1, 2, 3 or XRT_BOX3";
    case XRT_ESIZE: return "size out of the supported range";
    case XRT_ENOMEM: return "device memory allocation failed";
    case XRT_EHIP: return "HIP runtime error";
    case XRT_EPLAN: return "invalid plan";
    default: return "unknown status";
    }
}

const char* xrt_last_error(void) { return g_last_error; }

xrt_status xrt_plan_create(xrt_grid g, int degree, const xrt_lines* lines, void* stream,
                           xrt_plan** out)
{
    return xrt::plan_create(g, degree, lines, stream, true, out);
}

}  // extern "C"

namespace xrt {
xrt_status plan_check(xrt_grid g, int degree, const xrt_lines* lines)
{
    if (!valid_basis(degree)) return XRT_EDEGREE;
    xrt_status st = check_grid(g);
    if (st != XRT_OK) return st;
    return check_lines(lines);
}

void plan_init(xrt_plan* p, xrt_grid g, int degree, int64_t m, bool split_tiles)
{
    memset(p, 0, sizeof(*p));
    p->magic = kPlanMagic;
    p->g.nx = g.nx;
    p->g.ny = g.ny;
    p->g.h = g.spacing;
    p->g.cx = g.cx;
    p->g.cy = g.cy;
    p->degree = degree;
    p->m = m;
    // crossing buckets: floor(Xc) + boff in [0, nbk) for every line that
    // reaches the grid (|Xc| <= nmin + nmaj/2 + (n+1))
    p->boff_v = (g.ny + 1) / 2 + 8;
    p->boff_h = (g.nx + 1) / 2 + 8;
    p->nbk_v = g.nx + g.ny + 24;
    p->nbk_h = g.nx + g.ny + 24;
    const int64_t per_v = (int64_t)kSlopeBins * p->nbk_v, per_h = (int64_t)kSlopeBins * p->nbk_h;
    p->key_space = per_v + per_h + 1;
    p->pitch_v = round_up(g.nx + 2 * kPad, 16);
    p->pitch_h = round_up(g.ny + 2 * kPad, 16);
    p->strips_v = (g.ny + kStrip - 1) / kStrip;
    p->strips_h = (g.nx + kStrip - 1) / kStrip;
    p->fwd_sub = 1;
    // split each adjoint tile's candidate lines over up to 8 workgroups
    // (partial images, summed in a fixed order), aiming at kAdjUnits
    // workgroups per pass: with few units per compute unit the tiles that
    // finish last leave it partly idle (2048^2: 2048 tiles per pass, cubic
    // adjoint 27.9 ms unsplit, 25.4 ms split 6 ways)
    const int64_t tiles = (int64_t)((g.nx + kTileI - 1) / kTileI) * ((g.ny + kTileJ - 1) / kTileJ);
    p->adj_split = split_tiles ? (int)std::min<int64_t>(8, (kAdjUnits + tiles - 1) / tiles) : 1;
    // both passes in one launch when one pass's workgroups would not fill the
    // GPU's resident slots (kAdjWavesPerSimd workgroups of 4 waves per CU)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    p->adj_merge = p->adj_split > 1 && tiles * p->adj_split < (int64_t)cus * kAdjWavesPerSimd ? 1 : 0;
}

hipError_t plan_build(const xrt_plan* p, const xrt_lines* lines, const PlanTemps& t, hipStream_t s,
                      const char** what)
{
    hipError_t e = hipSuccess;
#define XRT_TRY(call, label)                   \
    do {                                       \
        if (e == hipSuccess) {                 \
            e = (call);                        \
            if (e != hipSuccess) *what = label; \
        }                                      \
    } while (0)
    const int64_t per_v = (int64_t)kSlopeBins * p->nbk_v, per_h = (int64_t)kSlopeBins * p->nbk_h;
    // cleared by a kernel (no memset node if a caller captures the stream)
    XRT_TRY(launch_fill_u32(t.count, p->key_space, 0u, s), "clear");
    XRT_TRY(launch_fill_u32((uint32_t*)p->hdr, sizeof(PlanHeader) / 4, 0u, s), "clear");
    CanonArgs ca;
    ca.L.kind = lines->kind;
    ca.L.theta = lines->theta;
    ca.L.y = lines->y;
    ca.L.ep = lines->endpoints;
    ca.m = p->m;
    ca.g = p->g;
    ca.degree = geom_degree(p->degree);
    ca.nbk_v = p->nbk_v;
    ca.nbk_h = p->nbk_h;
    ca.boff_v = p->boff_v;
    ca.boff_h = p->boff_h;
    ca.key = t.key;
    ca.xc = t.xc_in;
    ca.kap = t.kap_in;
    ca.count = t.count;
    ca.hdr = p->hdr;
    XRT_TRY(launch_canon(ca, s), "canonicalize");
    XRT_TRY(launch_scan(t.count, p->off, p->key_space, t.scan_tmp, s), "scan");
    SortArgs sa;
    sa.m = p->m;
    sa.max_key = (uint32_t)(p->key_space - 1);
    sa.key = t.key;
    sa.tmp = t.sort_tmp;
    sa.xc_in = t.xc_in;
    sa.kap_in = t.kap_in;
    sa.xc = p->xc;
    sa.kap = p->kap;
    sa.idx = p->idx;
    XRT_TRY(launch_radix_sort(sa, s), "sort");
    XRT_TRY(launch_header(p->hdr, p->off, per_v, per_v + per_h, s), "header");
#undef XRT_TRY
    return e;
}

xrt_status plan_create(xrt_grid g, int degree, const xrt_lines* lines, void* stream, bool own_buffers,
                       xrt_plan** out)
{
    if (!out) return XRT_EINVAL;
    *out = nullptr;
    xrt_status st = plan_check(g, degree, lines);
    if (st != XRT_OK) return st;

    hipStream_t s = (hipStream_t)stream;
    xrt_plan* p = new (std::nothrow) xrt_plan;
    if (!p) return XRT_ENOMEM;
    // test hook: XRT_SCHEDULE=plain selects the schedules otherwise kept
    // for very large problems (one forward launch per strip, unsplit
    // adjoint tiles), so that tests can compare them with the defaults
    const char* sched = getenv("XRT_SCHEDULE");
    const bool plain = sched && strcmp(sched, "plain") == 0;
    plan_init(p, g, degree, lines->n, own_buffers && !plain);

    const int64_t m = p->m;
    Allocs al{s};
    p->xc = al.get<double>(m);
    p->kap = al.get<double>(m);
    p->idx = al.get<int32_t>(m);
    p->off = al.get<uint32_t>(p->key_space + 1);
    p->hdr = al.get<PlanHeader>(1);
    p->cv = al.get<float>((size_t)g.ny * p->pitch_v);
    p->dv = al.get<float>((size_t)g.ny * p->pitch_v);
    p->ch = al.get<float>((size_t)g.nx * p->pitch_h);
    p->dh = al.get<float>((size_t)g.nx * p->pitch_h);
    p->sw = al.get<float>(m);
    // The forward runs as one persistent launch with a sum per line and strip
    // (summed in strip order afterwards) while those sums take at most
    // kMaxStripSums bytes; beyond that, one launch per strip adds into one
    // running sum per line.  Plans inside a batch need neither (the batch
    // has its own forward and adjoint launches).
    {
        const int ns = std::max(p->strips_v, p->strips_h);
        const size_t sums = (size_t)ns * (size_t)m * sizeof(float);
        p->fwd_persist = own_buffers && !plain && sums <= kMaxStripSums ? 1 : 0;
        if (own_buffers) {
            int dev = 0, cus = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
                cus = 256;
            p->fwd_grid = cus * kFwdBlocksPerCU;
            // two lines per thread and item, unless that leaves fewer than
            // four items per workgroup (small problems: one line per thread)
            p->fwd_lpi = (int64_t)ns * (m / (2 * kBlock)) >= 4 * (int64_t)p->fwd_grid ? 2 * kBlock : kBlock;
            // small problems: items of a half or a quarter strip while there
            // are fewer than two items per workgroup, so that the last round
            // of items is short (512^2 cubic, 138,240 lines: 2,160 whole-strip
            // items for 2,048 workgroups took two full rounds, 0.139 ms per
            // forward call; half strips 0.125 ms; quarter strips, with each
            // line's setup repeated per part, 0.139 ms again).  The launches
            // per strip use the same parts, so both schedules add the same
            // partial sums in the same order.
            const int64_t items = (int64_t)ns * ((m + p->fwd_lpi - 1) / p->fwd_lpi);
            while (p->fwd_sub < 4 && items * p->fwd_sub < 2 * (int64_t)p->fwd_grid &&
                   sums * (size_t)(2 * p->fwd_sub) <= kMaxStripSums)
                p->fwd_sub *= 2;
        }
        if (p->fwd_persist) {
            p->spart = al.get<float>((size_t)ns * (size_t)p->fwd_sub * (size_t)m);
            p->fctr = al.get<unsigned int>(1);
        } else if (own_buffers) {
            p->part = al.get<double>((size_t)m);
        }
        p->adj_part = p->adj_split > 1
                          ? al.get<float>((size_t)(p->adj_merge ? 2 : 1) * p->adj_split * g.nx * g.ny)
                          : nullptr;
    }
    // temporaries
    PlanTemps t;
    t.key = al.get<uint32_t>(m);
    t.xc_in = al.get<double>(m);
    t.kap_in = al.get<double>(m);
    t.count = al.get<uint32_t>(p->key_space);
    t.scan_tmp = al.get<uint32_t>(scan_tmp_words(p->key_space));
    t.sort_tmp = al.get<uint32_t>(radix_tmp_words(m, p->key_space - 1));
    auto free_tmp = [&]() {
        void* q[] = {t.key, t.xc_in, t.kap_in, t.count, t.scan_tmp, t.sort_tmp};
        for (void* v : q)
            if (v) (void)hipFreeAsync(v, s);
    };
    if (al.failed) {
        set_error("hipMallocAsync", al.err);
        free_tmp();
        free_plan_memory(p, s);
        (void)hipStreamSynchronize(s);
        delete p;
        return XRT_ENOMEM;
    }

    const char* what = "plan";
    hipError_t e = plan_build(p, lines, t, s, &what);
    PlanHeader h;
    memset(&h, 0, sizeof(h));
    if (e == hipSuccess) {
        e = hipMemcpyAsync(&h, p->hdr, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) what = "header read";
    }
    free_tmp();
    if (e == hipSuccess) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) what = "synchronize";
    }
    if (e != hipSuccess) {
        set_error(what, e);
        free_plan_memory(p, s);
        (void)hipStreamSynchronize(s);
        delete p;
        return XRT_EHIP;
    }
    if (h.error) {
        free_plan_memory(p, s);
        (void)hipStreamSynchronize(s);
        delete p;
        return XRT_EINVAL;
    }
    p->m_vert = h.m_vert;
    p->m_valid = h.m_valid;
    *out = p;
    return XRT_OK;
}
}  // namespace xrt

extern "C" {

static bool plan_ok(const xrt_plan* p) { return p && p->magic == kPlanMagic; }

xrt_status xrt_plan_info(const xrt_plan* p, int64_t* n_lines, int64_t* n_crossing)
{
    if (!plan_ok(p)) return XRT_EPLAN;
    if (n_lines) *n_lines = p->m;
    if (n_crossing) *n_crossing = p->m_valid;
    return XRT_OK;
}

xrt_status xrt_plan_forward(const xrt_plan* p, const float* coeffs, float* sino, void* stream)
{
    if (!plan_ok(p)) return XRT_EPLAN;
    if (!coeffs || (!sino && p->m > 0)) return XRT_EINVAL;
    hipError_t e = launch_forward(p, coeffs, sino, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("forward launch", e);
        return XRT_EHIP;
    }
    return XRT_OK;
}

xrt_status xrt_plan_adjoint(const xrt_plan* p, const float* sino, float* coeffs_out, void* stream)
{
    if (!plan_ok(p)) return XRT_EPLAN;
    if (!coeffs_out || (!sino && p->m > 0)) return XRT_EINVAL;
    hipError_t e = launch_adjoint(p, sino, coeffs_out, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("adjoint launch", e);
        return XRT_EHIP;
    }
    return XRT_OK;
}

xrt_status xrt_plan_nnz(const xrt_plan* p, int64_t* nnz, void* stream)
{
    if (!plan_ok(p)) return XRT_EPLAN;
    if (!nnz) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d = nullptr;
    hipError_t e = hipMallocAsync((void**)&d, sizeof(*d), s);
    if (e != hipSuccess) {
        set_error("hipMallocAsync", e);
        return XRT_ENOMEM;
    }
    unsigned long long hcount = 0;
    e = hipMemsetAsync(d, 0, sizeof(*d), s);
    if (e == hipSuccess) e = launch_nnz(p, d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hcount, d, sizeof(hcount), hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(d, s);
    hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        set_error("nnz", e);
        return XRT_EHIP;
    }
    *nnz = (int64_t)hcount;
    return XRT_OK;
}

void xrt_plan_destroy(xrt_plan* p)
{
    if (!plan_ok(p)) return;
    (void)hipDeviceSynchronize();
    free_plan_memory(p, nullptr);
    (void)hipDeviceSynchronize();
    p->magic = 0;
    delete p;
}

xrt_status xrt_forward(const float* coeffs, xrt_grid g, int degree, const xrt_lines* lines,
                       float* sino, void* stream)
{
    if (!coeffs || !lines) return XRT_EINVAL;
    if (!valid_basis(degree)) return XRT_EDEGREE;
    xrt_status st = check_grid(g);
    if (st != XRT_OK) return st;
    st = check_lines(lines);
    if (st != XRT_OK) return st;
    if (lines->n > 0 && !sino) return XRT_EINVAL;
    xrt_plan* p = nullptr;
    st = xrt_plan_create(g, degree, lines, stream, &p);
    if (st != XRT_OK) return st;
    st = xrt_plan_forward(p, coeffs, sino, stream);
    // stream-ordered frees: the memory is released once the launches above
    // have run, without waiting here
    free_plan_memory(p, (hipStream_t)stream);
    p->magic = 0;
    delete p;
    return st;
}

xrt_status xrt_adjoint(const float* sino, const xrt_lines* lines, int degree, xrt_grid g,
                       float* coeffs_out, void* stream)
{
    if (!coeffs_out || !lines) return XRT_EINVAL;
    if (!valid_basis(degree)) return XRT_EDEGREE;
    xrt_status st = check_grid(g);
    if (st != XRT_OK) return st;
    st = check_lines(lines);
    if (st != XRT_OK) return st;
    if (lines->n > 0 && !sino) return XRT_EINVAL;
    xrt_plan* p = nullptr;
    st = xrt_plan_create(g, degree, lines, stream, &p);
    if (st != XRT_OK) return st;
    st = xrt_plan_adjoint(p, sino, coeffs_out, stream);
    // stream-ordered frees: the memory is released once the launches above
    // have run, without waiting here
    free_plan_memory(p, (hipStream_t)stream);
    p->magic = 0;
    delete p;
    return st;
}

}  // extern "C"
