// xrt_adjoint_noalloc: the plan-less adjoint without any device allocation.
//
// xrt_adjoint builds a temporary plan in memory it allocates (line records,
// bucket offsets, sort temporaries, the sorted sinogram and the split tiles'
// partial images) and frees it again.  This variant carves the same buffers
// out of one file-scope device array, `scratch`, of kNoAllocBytes, so that
// callers that cannot allocate device memory can still back-project an
// arbitrary line list.  The plan is built with the same kernels
// (plan_build) and the adjoint runs the same launches (launch_adjoint), so
// the result equals xrt_adjoint's bit for bit.
//
// Each GPU holds its own copy of `scratch` (at its own address) from the
// first use until the process ends.  Host code never names the array in a
// kernel argument: at the first call on a device the library looks up that
// device's address with hipGetSymbolAddress; every later use goes through
// that address.  All calls
// on one GPU share its array: calls that overlap on one GPU (on different
// streams, or from different threads) race and must be serialised by the
// caller.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "xrt_internal.h"

namespace xrt {

// 64 MiB: a 512^2 grid with about 700,000 lines, or 128^2 with about 1.1M.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

struct DevScratch {
    std::once_flag once;
    hipError_t err = hipSuccess;
    unsigned char* ptr = nullptr;
};
DevScratch g_dev[kMaxDevices];

void setup_device(DevScratch& d)
{
    void* ptr = nullptr;
    d.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (d.err == hipSuccess) d.ptr = (unsigned char*)ptr;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sequential carving of the array.
struct Carve {
    unsigned char* base;
    size_t used;
    template <class T>
    T* take(size_t count)
    {
        T* p = (T*)(base + used);
        used = align_up(used + count * sizeof(T));
        return p;
    }
};

}  // namespace
}  // namespace xrt

using namespace xrt;

extern "C" xrt_status xrt_adjoint_noalloc(const float* sino, const xrt_lines* lines, int degree, xrt_grid g,
                                          float* coeffs_out, void* stream)
{
    if (!coeffs_out || !lines) return XRT_EINVAL;
    xrt_status st = plan_check(g, degree, lines);
    if (st != XRT_OK) return st;
    if (lines->n > 0 && !sino) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t npix = (int64_t)g.nx * g.ny;
    if (lines->n == 0) {
        const hipError_t e = launch_fill_u32((uint32_t*)coeffs_out, npix, 0u, s);
        if (e != hipSuccess) {
            set_last_error("adjoint (no allocation): clear");
            return XRT_EHIP;
        }
        return XRT_OK;
    }

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_last_error("adjoint (no allocation): no usable current device");
        return XRT_EHIP;
    }
    DevScratch& d = g_dev[dev];
    std::call_once(d.once, setup_device, std::ref(d));
    if (d.err != hipSuccess || !d.ptr) {
        char msg[200];
        snprintf(msg, sizeof(msg), "adjoint (no allocation): scratch set-up: %s", hipGetErrorString(d.err));
        set_last_error(msg);
        return XRT_EHIP;
    }

    xrt_plan p;
    plan_init(&p, g, degree, lines->n, true);
    const int64_t m = p.m;
    // persistent part: line records, bucket offsets, header, sorted sinogram,
    // partial images
    Carve c{d.ptr, 0};
    p.hdr = c.take<PlanHeader>(1);
    p.xc = c.take<double>(m);
    p.kap = c.take<double>(m);
    p.idx = c.take<int32_t>(m);
    p.off = c.take<uint32_t>(p.key_space + 1);
    // the build's temporaries are dead once the sort has run; the sorted
    // sinogram and the partial images are written only after it, so they
    // share the same bytes
    const size_t shared_at = c.used;
    PlanTemps t;
    t.key = c.take<uint32_t>(m);
    t.xc_in = c.take<double>(m);
    t.kap_in = c.take<double>(m);
    t.count = c.take<uint32_t>(p.key_space);
    t.scan_tmp = c.take<uint32_t>(scan_tmp_words(p.key_space));
    t.sort_tmp = c.take<uint32_t>(radix_tmp_words(m, p.key_space - 1));
    const size_t temps_end = c.used;
    c.used = shared_at;
    p.sw = c.take<float>(m);
    p.adj_part = p.adj_split > 1 ? c.take<float>((size_t)(p.adj_merge ? 2 : 1) * p.adj_split * npix) : nullptr;
    const size_t need = std::max(temps_end, c.used);
    if (need > kNoAllocBytes) {
        char msg[200];
        snprintf(msg, sizeof(msg),
                 "adjoint (no allocation): %lld lines on %d x %d need %zu bytes of scratch, the maximum is %zu",
                 (long long)m, g.nx, g.ny, need, kNoAllocBytes);
        set_last_error(msg);
        return XRT_ESIZE;
    }

    const char* what = "plan";
    hipError_t e = plan_build(&p, lines, t, s, &what);
    if (e == hipSuccess) {
        e = launch_adjoint(&p, sino, coeffs_out, s);
        what = "adjoint launch";
    }
    if (e != hipSuccess) {
        char msg[200];
        snprintf(msg, sizeof(msg), "adjoint (no allocation): %s: %s", what, hipGetErrorString(e));
        set_last_error(msg);
        return XRT_EHIP;
    }
    return XRT_OK;
}
