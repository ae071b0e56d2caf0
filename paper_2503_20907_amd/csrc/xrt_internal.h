// Internal definitions shared by the translation units of libxrt.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xrt.h"
#include "xrt_geom.h"

namespace xrt {

// Padding (in cells) on both sides of every row of the coefficient layouts;
// large enough for every tap and knot slot a line touches in a row it visits.
constexpr int kPad = 8;
// Slope bins of the plan (the slope kappa of a line lies in [-1, 1]).
constexpr int kSlopeBins = 512;
constexpr int kBlock = 256;
// Rows per strip of the forward's strip-major schedule (one strip of the
// coefficient layouts, about 2 MB at 2048 columns, stays in an XCD's L2).
constexpr int kStrip = 128;

// Number of knot-transition slots per row for degree n.
__host__ __device__ constexpr int n_slots(int n) { return n + 1; }

// Device-resident plan header, written by the plan builder.
struct PlanHeader {
    int64_t m_vert;   // sorted lines [0, m_vert) are "vertical" (|sin| >= |cos|)
    int64_t m_valid;  // sorted lines [m_vert, m_valid) are "horizontal"; the rest miss the grid
    int64_t error;    // non-zero: a line was degenerate or non-finite
    int64_t pad;
};



struct LineIn {
    int kind;
    const float* theta;
    const float* y;
    const float* ep;
};

struct CanonArgs {
    LineIn L;
    int64_t m;
    GridGeom g;
    int degree;
    int nbk_v, nbk_h, boff_v, boff_h;
    uint32_t* key;
    double* xc;
    double* kap;
    uint32_t* count;  // [key_space]
    xrt::PlanHeader* hdr;
};

// Stable sort of the plan's lines by key (LSD radix sort, 8 bits per pass).
struct SortArgs {
    int64_t m;
    uint32_t max_key;      // largest key value (sets the number of passes)
    uint32_t* key;         // [m] keys; overwritten (used as a ping-pong buffer)
    uint32_t* tmp;         // radix_tmp_words(m, max_key) words
    const double* xc_in;   // [m] line records in input order
    const double* kap_in;
    double* xc;            // [m] line records in sorted order
    double* kap;
    int32_t* idx;          // [m] input position of each sorted line
};

struct RadixArgs {
    const uint32_t* key_in;
    const uint32_t* val_in;  // null: the element's own index
    uint32_t* key_out;
    uint32_t* val_out;
    int64_t m;
    int shift;
    const uint32_t* hoff;    // [256][nblk] first output position of every (digit, workgroup)
    int nblk;
};

// Lines with a non-finite sinogram value (k_adj_nonfinite).
struct NonFiniteArgs {
    int64_t m;
    const PlanHeader* hdr;
    const double* xc;
    const double* kap;
    const float* sw;   // [m] sinogram in sorted order (scaled)
    int nx, ny;
    int degree;        // B-spline degree (geometry degree for the box spline)
    int box;           // 1: the box spline's support
    float* out;
};

// Launchers (xrt_kernels.hip).  All enqueue on `s` and return the launch status.
hipError_t launch_canon(const CanonArgs& a, hipStream_t s);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s);
int64_t scan_tmp_words(int64_t n);
int64_t radix_tmp_words(int64_t m, int64_t max_key);
hipError_t launch_radix_sort(const SortArgs& a, hipStream_t s);
hipError_t launch_header(PlanHeader* hdr, const uint32_t* off, int64_t vert_end, int64_t valid_end,
                         hipStream_t s);
hipError_t launch_forward(const xrt_plan* p, const float* coeffs, float* sino, hipStream_t s);
hipError_t launch_adjoint(const xrt_plan* p, const float* sino, float* out, hipStream_t s);
// NaN into every pixel of the support of each line whose value in sw (a
// plan's sorted, scaled sinogram) is NaN or infinite
hipError_t launch_adj_nonfinite(const xrt_plan* p, const float* sw, float* out, hipStream_t s);
hipError_t launch_nnz(const xrt_plan* p, unsigned long long* out, hipStream_t s);

// Temporaries of a plan build (device memory, released after it).
struct PlanTemps {
    uint32_t* key;       // [m]
    double* xc_in;       // [m]
    double* kap_in;      // [m]
    uint32_t* count;     // [key_space]
    uint32_t* scan_tmp;  // scan_tmp_words(key_space)
    uint32_t* sort_tmp;  // radix_tmp_words(m, key_space - 1)
};
// argument checks of a plan (or plan-less call)
xrt_status plan_check(xrt_grid g, int degree, const xrt_lines* lines);
// sizes, bucket layout and tile split of a plan of m lines (no memory)
void plan_init(xrt_plan* p, xrt_grid g, int degree, int64_t m, bool split_tiles);
// enqueues the build of a plan whose buffers (xc, kap, idx, off, hdr) are
// set: clears, canonicalisation, key counts and offsets, stable sort,
// header.  Does not synchronise; *what names the failing step.
hipError_t plan_build(const xrt_plan* p, const xrt_lines* lines, const PlanTemps& t, hipStream_t s,
                      const char** what);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// xrt_plan_create; own_buffers = false leaves out the buffers that only the
// plan's own forward and adjoint use (persistent forward sums, split-tile
// partial images): plans inside a batch, which has its own launches
xrt_status plan_create(xrt_grid g, int degree, const xrt_lines* lines, void* stream, bool own_buffers,
                       xrt_plan** out);

// batches of plans (persistent launches; see xrt_batch.cpp)
size_t batch_prob_size();
// strips of the forward schedule of a plan (per-strip partial sums: strips x lines floats)
int batch_strips(const xrt_plan* p);
// writes the per-problem launch record (batch_prob_size() bytes) to dst (host memory)
void batch_fill(const xrt_plan* p, float* sino, float* back, float* spart, void* dst);
hipError_t launch_batch_fwd_reduce(const void* probs, int p, int64_t m, hipStream_t s);
hipError_t launch_layouts(const xrt_plan* p, const float* coeffs, hipStream_t s);
hipError_t launch_sort_sino(const xrt_plan* p, const float* sino, hipStream_t s);
hipError_t launch_reset_counters(unsigned int* c, int n, hipStream_t s);
// non-finite sinogram values of every problem (after both adjoint launches)
hipError_t launch_batch_nonfinite(const void* probs, int count, int64_t max_m, hipStream_t s);
hipError_t launch_batch_forward(const void* probs, const int2* items, int nitems, unsigned int* counter,
                                int lines_per_item, int grid, hipStream_t s);
// horizontal = 0: the vertical lines on kTileI x kTileJ tiles (writes the
// images); 1: the horizontal lines on the transposed tiles (adds into them)
hipError_t launch_batch_adjoint(const void* probs, const int2* items, int nitems, unsigned int* counter, int grid,
                                int horizontal, hipStream_t s);

}  // namespace xrt

namespace xrt {
// basis code of the 3-directional box spline (Section III-C); plans of it use
// the degree-1 margins for canonicalisation and binning (its row window,
// 1 + |kappa| columns, is within the degree-1 one)
constexpr int kBox3 = 16;
inline bool valid_basis(int d) { return (d >= 0 && d <= 3) || d == kBox3; }
inline int geom_degree(int d) { return d == kBox3 ? 1 : d; }
// message returned by xrt_last_error() on this thread
void set_last_error(const char* msg);
}  // namespace xrt

struct xrt_plan;
struct xrt_plan {
    uint64_t magic;
    xrt::GridGeom g;
    int degree;
    int64_t m;          // number of lines
    int64_t m_vert, m_valid;
    int nbk_v, nbk_h;   // crossing buckets per slope bin, per orientation
    int boff_v, boff_h; // bucket offset, per orientation
    int64_t key_space;  // number of keys (2 * bins * buckets + 1)
    // sorted line records
    double* xc;         // crossing of the centre major line
    double* kap;        // slope d(minor)/d(major)
    int32_t* idx;       // original position of the line
    uint32_t* off;      // [key_space + 1] start of every key in sorted order
    xrt::PlanHeader* hdr;
    // workspace
    int pitch_v, pitch_h;
    float *cv, *dv, *ch, *dh;  // coefficient / difference layouts
    float* sw;                 // sinogram in sorted order, scaled
    int strips_v, strips_h;    // strips of kStrip rows, per orientation
    int fwd_persist;           // 1: one persistent forward launch (spart); 0: one launch per strip part (part)
    int fwd_grid;              // workgroups of the persistent launch
    int fwd_lpi;               // lines per work item of the persistent launch
    int fwd_sub;               // parts per strip of the persistent launch's items (1, 2, 4)
    double* part;              // [m] running sums over the strips (fwd_persist = 0)
    float* spart;              // [max strips][m] per-strip sums (fwd_persist = 1)
    unsigned int* fctr;        // work counter of the persistent launch
    int adj_split;             // workgroups sharing one adjoint tile's candidate lines
    float* adj_part;           // [adj_split][ny][nx] partial images (adj_split > 1), twice that with adj_merge
    int adj_merge;             // 1: both adjoint passes in one launch (grids too small to fill the GPU per pass)
};
