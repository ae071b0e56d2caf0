// HIP kernels of libxrt.so (gfx950): plan building, coefficient layouts,
// forward projection and tile-binned adjoint of the B-spline x-ray transform.
//
// The footprint of a line with |sin t| >= |cos t| ("vertical"; the other case
// swaps x1 and x2, the case split of Section II-B) is evaluated row by row.
// In row j the line crosses the row's centre line at minor coordinate
// X(j) = X0 + kappa j (kappa = cot t), and the row contributes
//     (h/|sin t|) sum_i c_ij psi_r(X(j) - i),   r = |kappa| <= 1,
// where psi_r = beta^n * beta^n_r is the footprint of Proposition 1 / eq. (6)
// written in units of the row (phi_theta(u) = psi_r(u/|sin t|)/|sin t|).
//
// psi_r is split exactly (an identity derived from eq. (6)) as
//     psi_r(v) = S_r(v) + sum_k delta_k r^n E((v - kappa_k)/r),
//     S_r = beta^n + [n >= 2] r^2 (mu_2/2) beta^n'',
//     delta_k = (-1)^k C(n+1, k),  kappa_k = k - (n+1)/2 (knots of beta^n),
// where mu_2 = (n+1)/12 is the second moment of beta^n and E is one fixed
// function of compact support (-(n+1)/2, (n+1)/2) per degree (the (n+1)-fold
// integral of beta^n minus its polynomial tail).  Summed over a row this gives
//     sum_i c_i psi_r(X - i) = sum_d W_d(t) c_{J-d}
//                            + r^n sum_K E((X + (n+1)/2 - K)/r) D_K,
// with J = floor(X + (n+1)/2), t its fraction, W_d the n+1 B-spline weights
// (plus the r^2 beta'' term), and D_K = sum_l delta_l c_{K-l} the (n+1)-th
// backward difference of the row at knot K.  At most n+1 knots K lie within
// (n+1) r / 2 of X, so a row costs n+1 taps plus n+1 knot slots whatever r
// is.  E is a cubic-per-interval table (16 intervals per unit) built in FP64
// on the host and copied to LDS; the adjoint reads part of its entries from
// the global copy instead (adj_mem_slots).  Line geometry (crossings, floors)
// is FP64; the row arithmetic is FP32 in local coordinates t in [0, 1).
//
// The adjoint applies the transpose of exactly the same row arithmetic:
// every line adds W_d s to the cells J-d and r^n E(.) s to the knots K of an
// LDS tile, and the tile's output is A + Delta^T K.  One launch takes the
// vertical lines and writes the image, a second one the horizontal lines and
// adds into it (on grids too small to fill the GPU per pass, one launch runs
// both).  A tile's candidate lines are shared by up to 8 workgroups (every
// split-th chunk each), whose partial images k_adj_reduce adds in a fixed
// order.
//
// The forward is one persistent launch: workgroups take (orientation, strip,
// run of lines) items in strip order, and each line's strip sums are added
// in strip order afterwards (k_fwd_reduce).  On small problems an item covers
// a half or a quarter strip, and the parts' sums are added in the same way.
//
// The 3-directional box spline (basis code kBox3) uses the same schedules
// with its own row arithmetic (box_row, box_F): a telescoped row sum over two
// or four columns instead of taps and knots.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "xrt_internal.h"

namespace xrt {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

// ---------------------------------------------------------------- geometry

// Line (theta, y) of eq. (1) in world coordinates -> index space of the grid,
// then to the crossing form minor = X0 + kappa * major.
__device__ inline Canon canonicalize(const LineIn& L, int64_t m, const GridGeom& g, int degree)
{
    int bad = 0;
    double c, s, yw;
    if (L.kind == XRT_LINES_ENDPOINTS) {
        double px = L.ep[4 * m + 0], py = L.ep[4 * m + 1];
        double qx = L.ep[4 * m + 2], qy = L.ep[4 * m + 3];
        double dx = qx - px, dy = qy - py;
        double len = sqrt(dx * dx + dy * dy);
        if (!(len > 0.0) || !isfinite(len) || !isfinite(px) || !isfinite(py)) {
            bad = 1;
            len = 1.0;
            dx = 1.0;
            dy = 0.0;
        }
        c = dx / len;
        s = dy / len;
        yw = px * s - py * c;
    } else {
        double t = (double)L.theta[m];
        yw = (double)L.y[m];
        if (!isfinite(t) || !isfinite(yw)) {
            bad = 1;
            t = 0.0;
            yw = 0.0;
        }
        sincos(t, &s, &c);
    }
    return canon_core(c, s, yw, g, degree, bad);
}

__device__ inline int slope_bin(double kap)
{
    int b = (int)floor((kap + 1.0) * (0.5 * kSlopeBins));
    return b < 0 ? 0 : (b >= kSlopeBins ? kSlopeBins - 1 : b);
}

// ---------------------------------------------------------------- plan build

__global__ void __launch_bounds__(kBlock) k_canon(CanonArgs A)
{
    int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= A.m) return;
    Canon o = canonicalize(A.L, m, A.g, A.degree);
    uint32_t key;
    const uint32_t per_cls_v = (uint32_t)kSlopeBins * (uint32_t)A.nbk_v;
    const uint32_t per_cls_h = (uint32_t)kSlopeBins * (uint32_t)A.nbk_h;
    if (o.cls == 2) {
        key = per_cls_v + per_cls_h;
    } else {
        const int nbk = o.cls == 0 ? A.nbk_v : A.nbk_h;
        const int boff = o.cls == 0 ? A.boff_v : A.boff_h;
        double fb = floor(o.xc) + boff;
        int bk = (int)fmin(fmax(fb, 0.0), (double)(nbk - 1));
        key = (o.cls == 0 ? 0u : per_cls_v) + (uint32_t)slope_bin(o.kap) * (uint32_t)nbk + (uint32_t)bk;
    }
    if (o.bad) atomicOr((unsigned long long*)&A.hdr->error, 1ull);
    A.key[m] = key;
    A.xc[m] = o.xc;
    A.kap[m] = o.kap;
    atomicAdd(&A.count[key], 1u);
}

// Exclusive scan of n uint32 (block-local part): every block scans
// kBlock * 8 elements and writes its total to part[blockIdx.x].
constexpr int kScanPer = 8;
constexpr int kScanTile = kBlock * kScanPer;

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    // Hillis-Steele over the block in LDS
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        uint32_t x = tid >= d ? sh[tid - d] : 0u;
        __syncthreads();
        sh[tid] += x;
        __syncthreads();
    }
    uint32_t incl = sh[tid];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_tile(const uint32_t* in, uint32_t* out,
                                                    uint32_t* part, int64_t n)
{
    __shared__ uint32_t sh[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        v[e] = base + e < n ? in[base + e] : 0u;
        sum += v[e];
    }
    uint32_t total;
    uint32_t pre = block_excl_scan(sum, sh, &total);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        if (base + e < n) out[base + e] = pre;
        pre += v[e];
    }
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) k_scan_add(uint32_t* out, const uint32_t* part, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const uint32_t add = part[blockIdx.x];
    for (int e = threadIdx.x; e < kScanTile; e += kBlock) {
        int64_t i = base + e;
        if (i < n) out[i] += add;
    }
}


// Stable LSD radix sort of the plan keys, 8 bits per pass: the lines of one
// key keep their input order, so a plan (and every result computed with it)
// depends only on the line list.  Each workgroup owns kRsTile consecutive
// elements; k_rs_hist counts its digits, an exclusive scan of the
// digit-major table [digit][workgroup] gives every (digit, workgroup) its
// first output position, and k_rs_scatter places the elements in input
// order: rounds of kBlock elements, ranks within a wave from a match of the
// 8 digit bits over ballots, then the counts of the earlier waves.
constexpr int kRsPer = 16;
constexpr int kRsTile = kBlock * kRsPer;
static_assert(kBlock == 256, "one digit per thread");

__global__ void __launch_bounds__(kBlock) k_rs_hist(const uint32_t* __restrict__ key, int64_t m, int shift,
                                                  uint32_t* __restrict__ hist, int nblk)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsPer; ++r) {
        const int64_t i = base + r * kBlock + threadIdx.x;
        if (i < m) atomicAdd(&cnt[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) k_rs_scatter(RadixArgs A)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    run[tid] = A.hoff[(int64_t)tid * A.nblk + blockIdx.x];
#pragma unroll
    for (int v = 0; v < 4; ++v) wc[v][tid] = 0;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsPer; ++r) {
        const int64_t i = base + r * kBlock + tid;
        const bool valid = i < A.m;
        uint32_t k = 0, v = 0, d = 0;
        if (valid) {
            k = A.key_in[i];
            v = A.val_in ? A.val_in[i] : (uint32_t)i;
            d = (k >> A.shift) & 255u;
        }
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int u = 0; u < w; ++u) pos += wc[u][d];
            A.key_out[pos] = k;
            A.val_out[pos] = v;
        }
        __syncthreads();
        run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
#pragma unroll
        for (int u = 0; u < 4; ++u) wc[u][tid] = 0;
        __syncthreads();
    }
}

// sorted position -> line records of the line it holds
__global__ void __launch_bounds__(kBlock) k_rs_gather(const uint32_t* __restrict__ val,
                                                    const double* __restrict__ xc_in,
                                                    const double* __restrict__ kap_in, double* __restrict__ xc,
                                                    double* __restrict__ kap, int32_t* __restrict__ idx, int64_t m)
{
    const int64_t pos = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pos >= m) return;
    const uint32_t l = val[pos];
    xc[pos] = xc_in[l];
    kap[pos] = kap_in[l];
    idx[pos] = (int32_t)l;
}

__global__ void k_header(PlanHeader* hdr, const uint32_t* off, int64_t vert_end, int64_t valid_end)
{
    hdr->m_vert = off[vert_end];
    hdr->m_valid = off[valid_end];
}

// ---------------------------------------------------------------- layouts
// Backward (n+1)-th difference weights delta_l = (-1)^l C(n+1, l).
template <int N>
__device__ inline float delta_w(int l)
{
    constexpr float d0[2] = {1.f, -1.f};
    constexpr float d1[3] = {1.f, -2.f, 1.f};
    constexpr float d2[4] = {1.f, -3.f, 3.f, -1.f};
    constexpr float d3[5] = {1.f, -4.f, 6.f, -4.f, 1.f};
    return N == 0 ? d0[l] : N == 1 ? d1[l] : N == 2 ? d2[l] : d3[l];
}

// Rows of C along x1 (for vertical lines): cv[j][p] = c[j][p - kPad],
// dv[j][p] = sum_l delta_l c[j][p - kPad - l] (zero outside the grid).
template <int N>
__global__ void __launch_bounds__(kBlock) k_layout_v(const float* __restrict__ c, int nx, int ny,
                                                     int pitch, float* __restrict__ cv,
                                                     float* __restrict__ dv)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const int j = blockIdx.y;
    if (p >= pitch) return;
    const float* row = c + (int64_t)j * nx;
    const int i = p - kPad;
    float cc = (i >= 0 && i < nx) ? row[i] : 0.f;
    float d = 0.f;
#pragma unroll
    for (int l = 0; l <= N + 1; ++l) {
        int ii = i - l;
        float v = (ii >= 0 && ii < nx) ? row[ii] : 0.f;
        d += delta_w<N>(l) * v;
    }
    cv[(int64_t)j * pitch + p] = cc;
    dv[(int64_t)j * pitch + p] = d;
}

// Columns of C (for horizontal lines), transposed through LDS:
// ch[i][p] = c[p - kPad][i], dh[i][p] = sum_l delta_l c[p - kPad - l][i].
constexpr int kTr = 32;
template <int N>
__global__ void __launch_bounds__(kBlock) k_layout_h(const float* __restrict__ c, int nx, int ny,
                                                     int pitch, float* __restrict__ ch,
                                                     float* __restrict__ dh)
{
    __shared__ float sh[kTr + 4][kTr + 1];
    const int p0 = blockIdx.x * kTr;  // padded position along x2 (output minor)
    const int i0 = blockIdx.y * kTr;  // column index (output major)
    const int tx = threadIdx.x % kTr, ty = threadIdx.x / kTr;  // 32 x 8
    // rows j = p0 - kPad - (N+1) + r for r in [0, kTr + N + 1)
    for (int r = ty; r < kTr + N + 1; r += kBlock / kTr) {
        int j = p0 - kPad - (N + 1) + r;
        int i = i0 + tx;
        sh[r][tx] = (j >= 0 && j < ny && i < nx) ? c[(int64_t)j * nx + i] : 0.f;
    }
    __syncthreads();
    for (int r = ty; r < kTr; r += kBlock / kTr) {
        int i = i0 + r;      // output row (major)
        int p = p0 + tx;     // output position
        if (i >= nx || p >= pitch) continue;
        float cc = sh[tx + N + 1][r];
        float d = 0.f;
#pragma unroll
        for (int l = 0; l <= N + 1; ++l) d += delta_w<N>(l) * sh[tx + N + 1 - l][r];
        ch[(int64_t)i * pitch + p] = cc;
        dh[(int64_t)i * pitch + p] = d;
    }
}

// ---------------------------------------------------------------- row math
// Constants of one line: ka = 1/(A r) with A = (n+1)/2 (the knot argument's
// scale), r^n, the beta'' weight rho, and the number of knot slots
// S = ceil((n+1) r) (at most n+1) that can be non-zero in a row: only knots
// within (n+1) r / 2 of the crossing matter.
struct LineConst {
    float ka, rn, rho;
    int slots;
};

template <int N>
__device__ inline LineConst line_const(double kap)
{
    LineConst k;
    const float r = (float)fabs(kap);
    k.ka = 2.f / ((float)(N + 1) * fmaxf(r, 1e-30f));
    float rn = 1.f;
#pragma unroll
    for (int e = 0; e < N; ++e) rn *= r;
    k.rn = rn;
    // (r^2/2) * mu_2 with mu_2 = (n+1)/12; the term exists for n >= 2
    k.rho = N >= 2 ? r * r * (float)(N + 1) / 24.0f : 0.f;
    const int sl = (int)ceilf((float)(N + 1) * r);
    k.slots = sl < 1 ? 1 : (sl > N + 1 ? N + 1 : sl);
    return k;
}

// Slot count shared by the active lanes of a wave (the largest one).
template <int N>
__device__ inline int wave_slots(int mine)
{
    int S = 1;
#pragma unroll
    for (int v = 2; v <= N + 1; ++v)
        if (__ballot(mine >= v) != 0) S = v;
    return S;
}

// The knot-transition function E in closed form.  E(z) = g(|z|) with the
// parity of E (even for odd n; for even n it changes sign at 0), and on
// [0, A], A = (n+1)/2, only the knots kappa_l < 0 of G's truncated-power sum
// reach g(zeta) = G(-zeta):
//   n = 0: (1/2 - zeta)_+
//   n = 1: (1 - zeta)_+^3 / 6
//   n = 2: ((3/2 - zeta)_+^5 - 3 (1/2 - zeta)_+^5) / 120
//   n = 3: ((2 - zeta)_+^7 - 4 (1 - zeta)_+^7) / 5040.
// With w = clamp(1 - zeta/A, 0, 1) and v = clamp(A w - 1, 0, 1) =
// (A - 1 - zeta)_+ (the inner term, n >= 2): g = knot_scale x with
// x = w^(2n+1) - knot_inner v^(2n+1).  A knot slot is then VALU work only.
// A table of E (cubic pieces, 16 per unit, 16-byte entries) was read before:
// its loads queued on the LDS behind the adjoint's accumulator atomics and
// on the vector L1, and every row waited for them.  2048^2 cubic: adjoint
// 24.6 -> 22.0 ms, forward 13.7 -> 13.2 ms, although the adjoint's four-slot
// row grew from 66 to 70 VALU instructions.  In FP32 the closed form is also
// closer to E than the table was (2.7e-8 absolute for n = 3).
//
// For even n, E jumps at 0 (by P(0): 1 for n = 0, 1/8 for n = 2), and the
// jump cancels the one of the taps at the same knot.  Which side of the knot
// the row lies on must therefore be the side the taps take, J = floor(q) in
// FP64: it comes from the slot's integer offset (knots at or left of J take
// the sign of z >= 0), not from the sign of the FP32 argument, which rounds
// to 0 when q lies within ~1e-8 below the knot (the fraction of q then
// rounds to 1.0f).
template <int N>
__device__ constexpr float knot_scale()
{
    return N == 0 ? 0.5f : N == 1 ? 1.f / 6.f : N == 2 ? 7.59375f / 120.f : 128.f / 5040.f;
}

template <int N>
__device__ constexpr float knot_inner()
{
    return N == 2 ? 3.f / 7.59375f : N == 3 ? 1.f / 32.f : 0.f;
}

template <int P>
__device__ inline float ipow(float w)
{
    if constexpr (P == 1) return w;
    else if constexpr (P == 3) return (w * w) * w;
    else if constexpr (P == 5) {
        const float w2 = w * w;
        return (w2 * w2) * w;
    } else {
        const float w2 = w * w;
        return (w2 * w2) * (w2 * w);
    }
}

__device__ inline float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 1.f); }

// x of the knot at distance zeta = A |u| from q.  A knot at least one cell
// from q (the outer slots: zeta >= 1 since r <= 1) has no inner term.
template <int N, bool INNER>
__device__ inline float knot_x(float u)
{
    const float w = clamp01(1.f - fabsf(u));
    float x = ipow<2 * N + 1>(w);
    if constexpr (INNER && N >= 2) {
        const float v = clamp01(fmaf(w, 0.5f * (N + 1), -1.f));
        x = fmaf(ipow<2 * N + 1>(v), -knot_inner<N>(), x);
    }
    return x;
}

// The S knots nearest to q of a row, K = J + c, and the arguments
// u_c = (t - c) ka, so that zeta = A |u_c| = |q - K|/r (ka = 1/(A r)):
//   S = 4: c = -1 .. 2;  S = 3: c = 0, 1, and 2 (t >= 1/2) or -1;
//   S = 2: c = 0, 1;     S = 1: c = 1 (t >= 1/2) or 0
// (the slots of knot_o).  The knots with c in {0, 1} are the near ones; the
// others lie at least one cell from q, so zeta >= 1 (r <= 1) and their inner
// term vanishes.

// Knots the forward loads per row, and the first one's offset from J.
template <int S>
__device__ constexpr int fwd_run() { return S == 3 ? 4 : S; }
template <int S>
__device__ constexpr int fwd_run_o(bool up) { return S == 3 ? -1 : knot_o<S>(up); }

// Forward: sum over the row's knots of E((q - K)/r) D_K / knot_scale.  dv
// holds D_K for K = J + knot_o<S>(up) + s, s < S, except for S = 3, where it
// holds the four knots c = -1 .. 2 (fwd_run) so that only the far knot's
// value is chosen by t >= 1/2.
template <int N, int S>
__device__ inline float fwd_knots(float t, bool up, float ka, const float* dv)
{
    constexpr bool even = N % 2 == 0;
    const float u0 = t * ka;
    if constexpr (S == 1) {
        const float x = knot_x<N, true>(up ? u0 - ka : u0);
        return (even ? (up ? x : -x) : x) * dv[0];
    } else {
        const float x0 = knot_x<N, true>(u0), x1 = knot_x<N, true>(u0 - ka);
        if constexpr (S == 2) {
            return fmaf(x1, dv[1], (even ? -x0 : x0) * dv[0]);
        } else if constexpr (S == 3) {
            const float xf = knot_x<N, false>(up ? fmaf(-2.f, ka, u0) : u0 + ka);
            return fmaf(even ? (up ? xf : -xf) : xf, up ? dv[3] : dv[0], fmaf(x1, dv[2], (even ? -x0 : x0) * dv[1]));
        } else {
            const float xm = knot_x<N, false>(u0 + ka), x2 = knot_x<N, false>(fmaf(-2.f, ka, u0));
            return fmaf(x2, dv[3], fmaf(x1, dv[2], fmaf(even ? -x0 : x0, dv[1], (even ? -xm : xm) * dv[0])));
        }
    }
}

// sum_d w_d(t) c_{J-d} written in powers of t, times kTapScale<N> (c[0] is
// c_{J-N}, c[N] is c_J).  For n = 3:
//   6 S = (c0 + 4c1 + c2) + 3t (c2 - c0) + 3(t^2 + 2 rho)(c0 - 2c1 + c2)
//         + t (t^2 + 6 rho)(c3 - c0 + 3(c1 - c2)).
template <int N>
__device__ constexpr float tap_scale() { return N == 3 ? 6.f : 1.f; }

template <int N>
__device__ inline float tap_sum(float t, float rho, const float* c)
{
    if constexpr (N == 0) {
        return c[0];
    } else if constexpr (N == 1) {
        return fmaf(t, c[1] - c[0], c[0]);
    } else if constexpr (N == 2) {
        // (c0 + c1)/2 + t (c1 - c0) + (t^2/2 + rho)(c0 - 2 c1 + c2)
        const float d2 = fmaf(-2.f, c[1], c[0] + c[2]);
        return fmaf(fmaf(0.5f * t, t, rho), d2, fmaf(t, c[1] - c[0], 0.5f * (c[0] + c[1])));
    } else {
        const float e0 = c[0] + c[2];
        const float a0 = fmaf(4.f, c[1], e0);
        const float a2 = fmaf(-2.f, c[1], e0);
        const float a3 = fmaf(3.f, c[1] - c[2], c[3] - c[0]);
        const float t3 = 3.f * t;
        const float p2 = fmaf(t3, t, 6.f * rho);
        const float p3 = t * fmaf(t, t, 6.f * rho);
        return fmaf(a3, p3, fmaf(a2, p2, fmaf(c[2] - c[0], t3, a0)));
    }
}

// Loads of C consecutive floats (pointer at the first).
template <int C>
__device__ inline void load_run(const float* __restrict__ p, float* v)
{
    if constexpr (C == 1) {
        v[0] = p[0];
    } else if constexpr (C == 2) {
        f2u a = *(const f2u*)p;
        v[0] = a.x;
        v[1] = a.y;
    } else {
        f4u a = *(const f4u*)p;  // C = 3 reads one float of padding
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        if constexpr (C == 4) v[3] = a.w;
    }
}

__device__ inline int xcd_logical(int bid, int nblk_pad)
{
    // blocks are dispatched round-robin over the 8 XCDs; give every XCD one
    // contiguous range of logical blocks so that its L2 sees neighbouring work
    const int per = nblk_pad / 8;
    return (bid % 8) * per + bid / 8;
}

// ---------------------------------------------------------------- box spline
// Footprint of the 3-directional box spline (directions e1, e2, e1+e2): by
// Proposition 1 the convolution of three centred unit-mass boxes of widths
// |<theta_perp, u_d>| = |sin|, |cos|, |sin - cos|.  Measured along a row in
// minor cells (distance = offset * A, A = 1/sqrt(1+kappa^2), kappa the slope
// minor per major) the widths become 1, |kappa| and 1 - kappa (kappa >= 0) or
// 1 + |kappa| (kappa < 0), and the footprint of a centre at offset v is
// psi(v) / A with psi = box_1 * R, R the trapezoid density of the two other
// widths a <= b (a + b = 1 for kappa >= 0, a = |kappa|, b = 1 + |kappa|
// otherwise).  Since box_1 * R (v) = F(v + 1/2) - F(v - 1/2) with F the
// distribution function of R, a row sum telescopes (summation by parts):
//   sum_i c_i psi(X - i) = c_{i0-1} + sum_{d=0..2} F_d (c_{i0+d} - c_{i0+d-1}),
// i0 = floor(X), t = X - i0, F_d = F at t + 1 + a' - d measured from the left
// end of R's support, a' = |kappa| for kappa < 0 and 0 otherwise.  For
// kappa >= 0 only F_1 = F(t) lies strictly between 0 and 1:
// c_{i0} + F(t) (c_{i0+1} - c_{i0}), a two-tap row like linear interpolation.
// The row sums then take the B-spline scaling h sqrt(1 + kappa^2).
//
// R's density ramps up on [0, a], is flat (1/b) on [a, b] and ramps down on
// [b, a + b].  With p = (a - t)_+ and q = (t + a - 1)_+ (the same
// expressions for both signs):
//   kappa >= 0 (b = 1 - a):  F(t) = (t - a/2)/b + (p^2 - q^2)/(2ab);
//   kappa <  0 (b = 1 + a):  F_0 = 1 - p^2/(2ab) (ramp down),
//                            F_1 = (t + a/2)/b (flat part),
//                            F_2 = q^2/(2ab) (ramp up).
// Both fit F_0 = 1 - k0 p^2, F_1 = t/b + c1 + k1 (p^2 - q^2), F_2 = k2 q^2
// with per-line constants (kappa >= 0: k0 = k2 = 0; kappa < 0: k1 = 0).
// For a -> 0 the p and q terms are O(a): nothing large is formed.
struct BoxRow {
    float a, am1;         // a, a - 1
    float invb, c1;       // 1/b, -+a/(2b)
    float k0, k1, k2;     // 1/(2ab) or 0 (see above)
    int neg;              // kappa < 0: four columns per row
};

__device__ inline BoxRow box_row(double kap)
{
    BoxRow k;
    double a, b;
    k.neg = kap < 0.0 ? 1 : 0;
    if (!k.neg) {
        a = fmin(kap, 1.0 - kap);
        b = 1.0 - a;
    } else {
        a = -kap;
        b = 1.0 - kap;
    }
    if (!(a > 1e-30)) a = 0.0;  // a term below 1e-30 is dropped
    const float inv2ab = a > 0.0 ? (float)(0.5 / (a * b)) : 0.f;
    k.a = (float)a;
    k.am1 = (float)(a - 1.0);
    k.invb = (float)(1.0 / b);
    k.c1 = (float)((k.neg ? 0.5 : -0.5) * a / b);
    k.k0 = k.neg ? inv2ab : 0.f;
    k.k1 = k.neg ? 0.f : inv2ab;
    k.k2 = k.neg ? inv2ab : 0.f;
    return k;
}

// F_0, F_1, F_2 at fraction t (valid for either sign of kappa)
__device__ inline void box_F(float t, const BoxRow& k, float& F0, float& F1, float& F2)
{
    const float p = fmaxf(k.a - t, 0.f), q = fmaxf(t + k.am1, 0.f);
    F0 = fmaf(-k.k0 * p, p, 1.f);
    F2 = (k.k2 * q) * q;
    F1 = fmaf((p - q) * (p + q), k.k1, fmaf(t, k.invb, k.c1));
}

// F(t) of a line with kappa >= 0
__device__ inline float box_F1(float t, const BoxRow& k)
{
    const float p = fmaxf(k.a - t, 0.f), q = fmaxf(t + k.am1, 0.f);
    return fmaf((p - q) * (p + q), k.k1, fmaf(t, k.invb, k.c1));
}

// ---------------------------------------------------------------- forward
struct FwdArgs {
    int64_t m;
    const PlanHeader* hdr;
    const double* xc;
    const double* kap;
    const int32_t* idx;
    const float* cv;
    const float* dv;
    const float* ch;
    const float* dh;
    int pitch_v, pitch_h;
    int nx, ny;
    double h;
    float* sino;
    double* part;            // [m] sums over the strip parts done so far (one launch per part)
    float* spart;            // [strips * sub][m] per-part sums (persistent launch)
    unsigned int* counter;   // work counter of the persistent launch
    int persist;             // 1: persistent launch (spart), 0: one launch per strip part (part)
    int lines_per_item;      // persistent launch: lines per work item (a multiple of kBlock)
    int sub;                 // persistent launch: parts of kStrip / sub rows per strip (1, 2, 4)
    int strips_v, strips_h;
    int strip;     // strip of this launch (one launch per strip part)
    int q;         // part of the strip (of sub) of this launch
    int nblk, nblk_pad;
};


// Sum over the rows [ja, jb] of one line (times tap_scale<N>).  C and D are
// the layout bases (uniform) at row 0 of the row numbers ja, jb; element
// (row j, minor i) sits at j * pitch + kPad + i, and q is X + (n+1)/2 + kPad
// at row ja (the padded column coordinate, positive on every row a line
// reaches).
template <int N, int S>
__device__ inline float fwd_walk(double q, double kap, int ja, int jb, const LineConst& lc,
                                 const float* __restrict__ C, const float* __restrict__ D, int pitch)
{
    const float rho = lc.rho;
    const float ernk = tap_scale<N>() * lc.rn * knot_scale<N>();
    // byte offsets (within one strip), so that the loads take the uniform
    // base plus a 32-bit offset
    const char* __restrict__ Cb = (const char*)C;
    // the knot run's first knot lies at a fixed offset from J for S >= 2
    // (fwd_run_o), folded into the uniform base
    constexpr int kFixedRun = S >= 2 ? (fwd_run_o<S>(false) + N) * 4 : 0;
    const char* __restrict__ Db = (const char*)D + kFixedRun;
    uint32_t off = (uint32_t)ja * (uint32_t)pitch * 4u;
    const uint32_t step = (uint32_t)pitch * 4u;
    // the row offset ends the walk (ja <= jb here)
    const uint32_t off_end = off + (uint32_t)(jb - ja + 1) * step;
    float part = 0.f;
    // walk q - N: its floor is the first tap J - N, so that the taps and the
    // knot slots (at J - N + N + o) share one offset register.  The walk is
    // in 32.32 fixed point, as the adjoint's (adj_fix): the fraction in the
    // low word, the column in the high word, one add with carry per row.
    const int64_t Q0 = (int64_t)rint((q - (double)N) * 4294967296.0);
    const int64_t Kq = (int64_t)rint(kap * 4294967296.0);
    const uint32_t Kf = (uint32_t)Kq;
    const int Ki = (int)(Kq >> 32);
    uint32_t tf = (uint32_t)Q0;
    int J = (int)(Q0 >> 32);
    do {
        const float t = (float)tf * 0x1p-32f;
        const bool up = t >= 0.5f;
        float cv[N + 1], dv[fwd_run<S>()];
        const uint32_t o = off + (uint32_t)J * 4u;
        load_run<N + 1>((const float*)(Cb + o), cv);
        if constexpr (S >= 2) load_run<fwd_run<S>()>((const float*)(Db + o), dv);
        else load_run<1>((const float*)(Db + (o + (uint32_t)(fwd_run_o<S>(up) + N) * 4u)), dv);
        part += fmaf(ernk, fwd_knots<N, S>(t, up, lc.ka, dv), tap_sum<N>(t, rho, cv));
        const uint32_t tn = tf + Kf;
        J += Ki + (tn < tf ? 1 : 0);
        tf = tn;
        off += step;
    } while (off != off_end);
    return part;
}

// Box-spline row sums over the rows [ja, jb] (q = X at row ja): two columns
// per row, or four when the wave holds a line of negative slope (the
// four-column form is exact for both signs).
template <bool NEG>
__device__ inline float fwd_walk_box(double q, double kap, int ja, int jb, const BoxRow& bk,
                                     const float* __restrict__ C, int pitch)
{
    // q = X + kPad at row ja (padded column coordinate, positive); walked in
    // 32.32 fixed point (fraction in the low word, column in the high word)
    const char* __restrict__ Cb = (const char*)C;
    uint32_t off = (uint32_t)ja * (uint32_t)pitch * 4u;
    const uint32_t step = (uint32_t)pitch * 4u;
    float part = 0.f;
    const int64_t Q0 = (int64_t)rint(q * 4294967296.0);
    const int64_t Kq = (int64_t)rint(kap * 4294967296.0);
    const uint32_t Kf = (uint32_t)Kq;
    const uint32_t Ki = (uint32_t)(int32_t)(Kq >> 32);
    uint32_t tf = (uint32_t)Q0;
    uint32_t i0 = (uint32_t)(int32_t)(Q0 >> 32);
    for (int j = ja; j <= jb; ++j) {
        const float t = (float)tf * 0x1p-32f;
        if constexpr (NEG) {
            float c[4];
            load_run<4>((const float*)(Cb + (off + (i0 - 1u) * 4u)), c);
            float F0, F1, F2;
            box_F(t, bk, F0, F1, F2);
            part += fmaf(F2, c[3] - c[2], fmaf(F1, c[2] - c[1], fmaf(F0, c[1] - c[0], c[0])));
        } else {
            float c[2];
            load_run<2>((const float*)(Cb + (off + i0 * 4u)), c);
            part += fmaf(box_F1(t, bk), c[1] - c[0], c[0]);
        }
        const uint32_t tn = tf + Kf;
        i0 += Ki + (tn < tf ? 1u : 0u);
        tf = tn;
        off += step;
    }
    return part;
}

// Sum of line k over the rows of strip `st` that it reaches (times
// tap_scale<N>); [*ja, *jb] is that row range (empty when *ja > *jb).  The
// lanes of a wave that call it together share the knot-slot count.
// Line k's sum over the rows of part q (of nsub) of strip st: rows
// [st kStrip + q kStrip / nsub, st kStrip + (q + 1) kStrip / nsub).
template <int N, bool VERT>
__device__ inline float fwd_strip_sum(const FwdArgs& A, int64_t k, int st, int* ja_out, int* jb_out, int q = 0,
                                      int nsub = 1)
{
    const int strip = st;
    const int rlo = strip * kStrip + q * (kStrip / nsub), rhi = rlo + kStrip / nsub - 1;
    const double xc = A.xc[k], kap = A.kap[k];
    const int nmaj = VERT ? A.ny : A.nx, nmin = VERT ? A.nx : A.ny;
    const int pitch = VERT ? A.pitch_v : A.pitch_h;
    // layout bases at the strip's first row, so that the walks' 32-bit byte
    // offsets stay within one strip (a whole layout can exceed 4 GiB)
    const int r0 = strip * kStrip;
    const float* __restrict__ C = (VERT ? A.cv : A.ch) + (size_t)r0 * (size_t)pitch;
    const float* __restrict__ D = (VERT ? A.dv : A.dh) + (size_t)r0 * (size_t)pitch;
    const double x0 = xc - kap * (0.5 * (nmaj - 1));
    float acc = 0.f;
    int ja, jb;
    if constexpr (N == kBox3) {
        // the footprint reaches 1 (kappa >= 0) or 1 + |kappa| minor cells
        int jlo, jhi;
        row_range(x0, kap, 1.0 / kap, kap >= 0.0 ? 1.0 : 1.0 - kap, nmaj, nmin, &jlo, &jhi);
        ja = max(jlo, rlo);
        jb = min(jhi, rhi);
        const BoxRow bk = box_row(kap);
        const bool neg = __ballot(ja <= jb && bk.neg) != 0ull;
        if (ja <= jb) {
            const double q0 = x0 + kap * (double)ja + (double)kPad;
            acc = neg ? fwd_walk_box<true>(q0, kap, ja - r0, jb - r0, bk, C, pitch)
                      : fwd_walk_box<false>(q0, kap, ja - r0, jb - r0, bk, C, pitch);
        }
    } else {
        const double H = 0.5 * (N + 1);
        int jlo, jhi;
        row_range(x0, kap, 1.0 / kap, H * (1.0 + fabs(kap)), nmaj, nmin, &jlo, &jhi);
        ja = max(jlo, rlo);
        jb = min(jhi, rhi);
        const LineConst lc = line_const<N>(kap);
        const int S = wave_slots<N>(ja <= jb ? lc.slots : 1);
        if (ja <= jb) {
            const double q0 = x0 + kap * (double)ja + H + (double)kPad;
            if (S == 1) acc = fwd_walk<N, 1>(q0, kap, ja - r0, jb - r0, lc, C, D, pitch);
            else if (S == 2) acc = fwd_walk<N, (N >= 1 ? 2 : 1)>(q0, kap, ja - r0, jb - r0, lc, C, D, pitch);
            else if (S == 3) acc = fwd_walk<N, (N >= 2 ? 3 : 1)>(q0, kap, ja - r0, jb - r0, lc, C, D, pitch);
            else acc = fwd_walk<N, (N >= 3 ? 4 : 1)>(q0, kap, ja - r0, jb - r0, lc, C, D, pitch);
        }
    }
    *ja_out = ja;
    *jb_out = jb;
    return acc;
}

// Forward, one launch per (orientation, strip of kStrip rows, part of it):
// the blocks in flight at any time read one strip of the layout, which stays
// in L2.  The launches of one orientation run in strip order and each adds
// its partial sums into part[k] (the first one writes), so the sum is
// deterministic and equals the persistent launch's; k_fwd_reduce scales and
// scatters.  Used when the persistent launch's per-part sums would take too
// much memory.
template <int N, bool VERT>
__global__ void __launch_bounds__(kBlock) k_forward(FwdArgs A)
{
    const int strip = A.strip;
    const int bid = blockIdx.x;
    const int64_t m_vert = A.hdr->m_vert, m_valid = A.hdr->m_valid;
    // vertical lines are the sorted range [0, m_vert), horizontal ones
    // [m_vert, m_valid).  The grid covers all m lines; the blocks of this
    // launch's range are spread evenly over the XCDs and the rest return.
    const int64_t first = VERT ? 0 : m_vert, end = VERT ? m_vert : m_valid;
    const int nb = (int)((end - first + kBlock - 1) / kBlock);
    const int nb_pad = (nb + 7) / 8 * 8;
    if (bid >= nb_pad) return;
    const int lb = xcd_logical(bid, nb_pad);
    if (lb >= nb) return;
    const int64_t k = first + (int64_t)lb * kBlock + threadIdx.x;
    if (k >= end) return;
    int ja, jb;
    const float acc = fwd_strip_sum<N, VERT>(A, k, strip, &ja, &jb, A.q, A.sub);
    if (strip == 0 && A.q == 0) A.part[k] = (double)acc;
    else if (ja <= jb) A.part[k] += (double)acc;
}

__device__ inline int next_item(unsigned int* counter, int* s_item)
{
    __syncthreads();   // everyone is done with the previous item (and with *s_item)
    if (threadIdx.x == 0) *s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    return *s_item;
}

// Forward as one persistent launch: workgroups take items (orientation,
// strip, run of lines_per_item lines) from a counter, the vertical lines'
// strips first, each orientation's strips in order, so that the workgroups
// in flight read about one strip of the layouts (as with one launch per
// strip, without a launch's tail per strip).  Line k's sum over strip st goes
// to spart[st][k]; k_fwd_reduce adds the strips in order.  The counter starts
// at zero; every workgroup leaves once the items are used up.
template <int N>
__global__ void __launch_bounds__(kBlock) k_forward_persist(FwdArgs A)
{
    __shared__ int s_item;
    const int64_t m_vert = A.hdr->m_vert, m_valid = A.hdr->m_valid;
    const int lpi = A.lines_per_item, nsub = A.sub;
    const int64_t nbv = (m_vert + lpi - 1) / lpi;
    const int64_t nbh = (m_valid - m_vert + lpi - 1) / lpi;
    const int64_t items_v = nbv * A.strips_v * nsub, items = items_v + nbh * A.strips_h * nsub;
    for (;;) {
        const int it = next_item(A.counter, &s_item);
        if (it >= items) break;
        const bool vert = it < items_v;   // uniform over the workgroup
        const int64_t li = vert ? it : it - items_v;
        const int64_t nb = vert ? nbv : nbh;
        // item li: strip part sq = st nsub + q, then the run of lines; a
        // strip's parts follow each other, so the items in flight share it
        const int sq = (int)(li / nb), st = sq / nsub, q = sq - st * nsub;
        const int64_t first = (vert ? 0 : m_vert) + (li - (int64_t)sq * nb) * lpi;
        const int64_t end = vert ? m_vert : m_valid;
        for (int sub = 0; sub < lpi; sub += kBlock) {
            const int64_t k = first + sub + threadIdx.x;
            if (k < end) {
                int ja, jb;
                const float acc = vert ? fwd_strip_sum<N, true>(A, k, st, &ja, &jb, q, nsub)
                                       : fwd_strip_sum<N, false>(A, k, st, &ja, &jb, q, nsub);
                A.spart[(int64_t)sq * A.m + k] = acc;
            }
        }
    }
}

// sino[idx[k]] = (sum over strips of part[s][k]) * h / max(|cos|,|sin|);
// lines that miss the grid get 0.
template <int N>
__global__ void __launch_bounds__(kBlock) k_fwd_reduce(FwdArgs A)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= A.m) return;
    const int64_t m_valid = A.hdr->m_valid;
    float v = 0.f;
    if (k < m_valid) {
        double acc;
        if (A.persist) {
            // the strip (part) sums in strip order, as the launches per strip add them
            const int ns = (k < A.hdr->m_vert ? A.strips_v : A.strips_h) * A.sub;
            acc = (double)A.spart[k];
            for (int st = 1; st < ns; ++st) acc += (double)A.spart[(int64_t)st * A.m + k];
        } else {
            acc = A.part[k];
        }
        const double kap = A.kap[k];
        v = (float)(acc * A.h * sqrt(1.0 + kap * kap) / (double)tap_scale<N>());
    }
    A.sino[A.idx[k]] = v;
}

// ---------------------------------------------------------------- adjoint
// Sinogram in sorted order, times h / max(|cos|, |sin|).
struct SortSinoArgs {
    int64_t m;
    const PlanHeader* hdr;
    const double* kap;
    const int32_t* idx;
    const float* sino;
    double h;
    float* sw;
};

__global__ void __launch_bounds__(kBlock) k_sort_sino(SortSinoArgs A)
{
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= A.m) return;
    if (k >= A.hdr->m_valid) {
        A.sw[k] = 0.f;
        return;
    }
    double kap = A.kap[k];
    A.sw[k] = (float)((double)A.sino[A.idx[k]] * A.h * sqrt(1.0 + kap * kap));
}

struct AdjArgs {
    const double* xc;
    const double* kap;
    const float* sw;
    const uint32_t* off;
    int nx, ny;
    int nbk_v, nbk_h, boff_v, boff_h;
    int tiles_i, tiles_j;
    int ntiles, ntiles_pad;
    int split;     // workgroups per tile (blockIdx.y): chunk c goes to workgroup c % split
    float* part;   // [split][ny][nx] partial images when split > 1
    float* out;
    int accumulate;  // 1: out += this launch's image (the second pass of a plan's adjoint)
};

// accumulator rows are padded to an odd pitch so that the rows the lanes of a
// wave update fall into different LDS banks; an accumulator holds the
// tile's kTileJ rows along the lines, each kTileI wide across them, plus
// halos
constexpr int kAccWords = kTileJ * kAccPitch;
constexpr int kPix = kTileI * kTileJ / kBlock;
// every thread flushes kPix whole pixels, and the candidate scan takes the
// slope bins two per thread
static_assert(kTileI * kTileJ % kBlock == 0, "a tile must hold a whole number of pixels per thread");
static_assert(kSlopeBins == 2 * kBlock, "the candidate scan assumes two slope bins per thread");

// The LDS accumulators are int32 fixed point: float atomic adds to LDS are an
// order of magnitude slower than integer ones on gfx950.  Lines are taken in
// chunks of 2 kBlock (two per thread; 8 kBlock for the box spline); a chunk
// scales the tap contributions by 2^e with e = 21 - exponent(max |s| over the
// chunk) (19 - for 8 kBlock lines), so each of them (|s w| <= |s|, since
// |w| <= 1) is below 2^21 (2^19) in magnitude and the at most 2 kBlock
// (8 kBlock) contributions a chunk makes to one accumulator word (one per
// line) stay below 2^30.  The knot contributions r^n E s are bounded by G(0) |s|
// (G(0) = 1/2, 1/6, 1/16, 0.0246 for n = 0..3) and get 2^kKnotShift more
// resolution under the same bound.  After each chunk the integers are
// converted back (scaled exactly by powers of two) into per-thread FP32
// outputs and cleared.  The rounding to integers is at most 2^-22 max|s| per
// contribution, about an FP32 rounding, and the integer sums do not depend on
// the order of the atomics.
template <int N>
__device__ constexpr int knot_shift() { return N == 0 ? 1 : N == 1 ? 2 : N == 2 ? 4 : 5; }
// Lines per thread and chunk, and the scale exponent's bound that keeps a
// chunk's adj_lpt kBlock contributions to one word below 2^30.  The box
// spline's rows are cheap, so the per-chunk work (candidate search, maximum,
// flush) weighs more: 8 lines per thread took its 2048^2 adjoint from 12.6 to
// 11.6 ms; the cubic spline is fastest at 2 (24.9 ms; 25.1 at 4, 25.5 at 8).
template <int N>
__device__ constexpr int adj_lpt() { return N == kBox3 ? 8 : 2; }
template <int N>
__device__ constexpr int adj_scale_bits() { return adj_lpt<N>() == 2 ? 21 : adj_lpt<N>() == 4 ? 20 : 19; }
constexpr int kAdjLptMax = 8;

// Round-to-nearest integer of a float below 2^22 in magnitude: adding
// 1.5 * 2^23 leaves exactly the rounded value in the mantissa.
constexpr float kRoundMagic = 12582912.0f;
constexpr int kRoundMagicBits = 0x4B400000;

__device__ inline int fixed_round(float a, float b)
{
    return __float_as_int(fmaf(a, b, kRoundMagic)) - kRoundMagicBits;
}

// The weights of the taps J - d: beta^n(t + d - (n+1)/2), plus the
// r^2 (mu_2/2) beta^n'' term (rho) for n >= 2.  Degree 1: t, 1 - t.
// Degree 2: t^2/2 + rho, 3/4 - 2 rho - (t - 1/2)^2, (1 - t)^2/2 + rho.
// Degree 3, with h2 = (t^2 + 2 rho)/2 and h3 = t (t^2 + 6 rho)/6:
//   w0 = h3, w3 = 1/6 - t/2 + h2 - h3, w1 = 1/6 + t/2 + h2 - 3 h3,
//   w2 = 2/3 - 2 h2 + 3 h3.
// The adjoint needs them times a line constant sigma, rounded to
// integers as fixed_round does: the round-to-nearest-even constant
// kRoundMagic is carried in per-line coefficients (and in the last
// multiply-add of each weight), and sigma is folded into the coefficients,
// so that a weight costs about what the unscaled one does.  Sums that pass
// through kRoundMagic are rounded to integers on the way (at most three
// roundings per weight, each to nearest even, so unbiased).
template <int N>
struct TapScaled {
    float a, b, c, d, e, f;
};

template <int N>
__device__ inline TapScaled<N> tap_scaled(float sigma, float rho)
{
    TapScaled<N> k;
    k.a = k.b = k.c = k.d = k.e = k.f = 0.f;
    if constexpr (N == 0) {
        k.a = sigma + kRoundMagic;
    } else if constexpr (N == 1) {
        k.a = sigma;
        k.b = sigma + kRoundMagic;
    } else if constexpr (N == 2) {
        k.a = sigma;
        k.b = fmaf(sigma, rho, kRoundMagic);
        k.c = fmaf(sigma, 0.75f - 2.f * rho, kRoundMagic);
        k.d = 0.5f * sigma;
    } else {
        k.a = 0.5f * sigma;
        k.b = sigma * rho;
        k.c = sigma * (1.f / 6.f);
        k.d = 6.f * rho;
        k.e = fmaf(sigma, 2.f / 3.f, kRoundMagic);
        k.f = fmaf(sigma, 1.f / 6.f, kRoundMagic);
    }
    return k;
}

__device__ inline int magic_int(float x) { return __float_as_int(x) - kRoundMagicBits; }

// round(sigma * w[d]) for the taps J - d (d = 0..N)
template <int N>
__device__ inline void tap_fixed(float t, const TapScaled<N>& k, int* wi)
{
    if constexpr (N == 0) {
        wi[0] = magic_int(k.a);
    } else if constexpr (N == 1) {
        wi[0] = magic_int(fmaf(k.a, t, kRoundMagic));
        wi[1] = magic_int(fmaf(-k.a, t, k.b));
    } else if constexpr (N == 2) {
        // sigma (t^2/2 + rho), sigma (3/4 - 2 rho - (t - 1/2)^2), sigma ((1-t)^2/2 + rho)
        const float u = t - 0.5f, s = 1.f - t;
        wi[0] = magic_int(fmaf(k.d * t, t, k.b));
        wi[1] = magic_int(fmaf(-k.a * u, u, k.c));
        wi[2] = magic_int(fmaf(k.d * s, s, k.b));
    } else {
        // every term times sigma: h2 = sigma (t^2 + 2 rho)/2,
        // h3 = sigma t (t^2 + 6 rho)/6, u = sigma/6 + h2 - h3
        const float ct = k.c * t, p = fmaf(t, t, k.d);
        const float h3 = ct * p;
        const float h2 = fmaf(k.a * t, t, k.b);
        const float um = (k.f + h2) - h3;  // u + kRoundMagic
        wi[0] = magic_int(fmaf(ct, p, kRoundMagic));
        wi[3] = magic_int(fmaf(-k.a, t, um));
        wi[1] = magic_int(fmaf(k.a, t, fmaf(-2.f, h3, um)));
        wi[2] = magic_int(fmaf(3.f, h3, fmaf(-2.f, h2, k.e)));
    }
}

// One knot atomic: sc is the line's scale (2^e s r^n kKnotScale), negated
// for the knots at or left of q when n is even (E's parity), and carries the
// rounding to an integer.
__device__ inline void knot_add(int* a, float sc, float x) { atomicAdd(a, fixed_round(sc, x)); }

// Adjoint: the row's knot atomics (the slots of fwd_knots), into the knot
// accumulator at kj (knot J).  For even n the knots with c <= 0 take -sc.
template <int N, int S>
__device__ inline void adj_knots(float t, bool up, float ka, float sc, int* kj)
{
    constexpr bool even = N % 2 == 0;
    const float u0 = t * ka;
    if constexpr (S == 1) {
        const float u = up ? u0 - ka : u0;
        knot_add(kj + (up ? 1 : 0), even ? (up ? sc : -sc) : sc, knot_x<N, true>(u));
    } else {
        knot_add(kj, even ? -sc : sc, knot_x<N, true>(u0));
        knot_add(kj + 1, sc, knot_x<N, true>(u0 - ka));
        if constexpr (S == 3) {
            knot_add(kj + (up ? 2 : -1), even ? (up ? sc : -sc) : sc,
                     knot_x<N, false>(up ? fmaf(-2.f, ka, u0) : u0 + ka));
        } else if constexpr (S == 4) {
            knot_add(kj - 1, even ? -sc : sc, knot_x<N, false>(u0 + ka));
            knot_add(kj + 2, sc, knot_x<N, false>(fmaf(-2.f, ka, u0)));
        }
    }
}

template <int N, int S>
__device__ inline void adj_row(AdjStep st, float sck, float ka, const TapScaled<N>& tk, int* s_a, int* s_k)
{
    // (float) of the low word rounds to nearest and can give t = 1.0 just
    // below a knot: the taps then take the left cell's polynomial at its right
    // end and the knots their integer side, which agree
    const float t = (float)st.tf * 0x1p-32f;
    const bool up = t >= 0.5f;
    int wi[N + 1];
    tap_fixed<N>(t, tk, wi);
    int* ar = s_a + st.base;  // taps J-N .. J, ascending
#pragma unroll
    for (int d = 0; d <= N; ++d) atomicAdd(ar + d, wi[N - d]);
    adj_knots<N, S>(t, up, ka, sck, s_k + st.base + N);
}

template <int N, int S>
__device__ inline void adj_walk(double q0, double kap, int cnt, int row0, float svs, float svk,
                                const LineConst& lc, int W, int* s_a, int* s_k)
{
    // start each lane at a different row (adj_start_row)
    const int jj0 = adj_start_row<kAdjSpread>(threadIdx.x, cnt);
    const float sck = svk * lc.rn * knot_scale<N>();
    const TapScaled<N> tk = tap_scaled<N>(svs, lc.rho);
    // walk q - N (exact): its floor is the first tap J - N (at least 0: the
    // halo covers the footprint), which is the base address of the row; the
    // knot slots share it (at J + o, adj_knot_offset).  Rows jj0 .. cnt-1,
    // then (back to row 0) 0 .. jj0-1, in one loop: every lane of a wave then
    // takes cnt steps (two loops would take up to twice as many, since the
    // lanes' start rows are spread).  The address grows by at least W - 1
    // per row, so it marks the wrap and the end.
    const AdjFix F = adj_fix(q0 - (double)N, kap, row0, W);
    AdjStep st = adj_fix_at(F, jj0);
    const AdjStep st0 = adj_fix_at(F, 0);
    const uint32_t mid = st.base, end = adj_fix_at(F, cnt).base;
    do {
        adj_row<N, S>(st, sck, lc.ka, tk, s_a, s_k);
        adj_fix_next(F, st);
        if (st.base == end) st = st0;
    } while (st.base != mid);
}

// Box spline: the row weights psi(X - i) = F_{i-i0} - F_{i-i0+1} of the
// telescoped row sum (F_{-1} = 1, F_3 = 0) into the fixed-point LDS
// accumulator: columns i0 and i0+1 for kappa >= 0, i0-1 .. i0+2 otherwise.
template <bool NEG>
__device__ inline void adj_walk_box(double q0, double kap, int cnt, int row0, float svs, const BoxRow& bk,
                                    int W, int* s_a)
{
    // start row spread and fixed-point walk as in adj_walk, on q - 1: its
    // floor is the first column floor(q) - 1 (columns floor(q) - 1 ..
    // floor(q) + 2)
    const int jj0 = adj_start_row<kAdjSpread>(threadIdx.x, cnt);
    const AdjFix F = adj_fix(q0 - 1.0, kap, row0, W);
    AdjStep st = adj_fix_at(F, jj0);
    const AdjStep st0 = adj_fix_at(F, 0);
    const uint32_t mid = st.base, end = adj_fix_at(F, cnt).base;
    do {
        const float t = (float)st.tf * 0x1p-32f;
        int* ar = s_a + st.base;
        if constexpr (NEG) {
            // kappa < 0: 1 - F_0 = k0 p^2 is formed directly
            const float p = fmaxf(bk.a - t, 0.f), qq = fmaxf(t + bk.am1, 0.f);
            const float w0 = (bk.k0 * p) * p, F2 = (bk.k2 * qq) * qq;
            const float F1 = fmaf(t, bk.invb, bk.c1);
            atomicAdd(ar, fixed_round(svs, w0));
            atomicAdd(ar + 1, fixed_round(svs, (1.f - w0) - F1));
            atomicAdd(ar + 2, fixed_round(svs, F1 - F2));
            atomicAdd(ar + 3, fixed_round(svs, F2));
        } else {
            const float F = box_F1(t, bk);
            atomicAdd(ar + 1, fixed_round(svs, 1.f - F));
            atomicAdd(ar + 2, fixed_round(svs, F));
        }
        adj_fix_next(F, st);
        if (st.base == end) st = st0;
    } while (st.base != mid);
}

__device__ inline void adj_line_box(const AdjArgs& A, double xck, double kap, bool active, float sv, int e, bool vert,
                                    int maj0, int min0, int TM, int TN, int nmaj, int W, double jc, double marg, int* s_a)
{
    if (!active) return;
    const int nmin = vert ? A.nx : A.ny;
    // rows whose crossing lies within the footprint's half-width (1 for
    // kappa >= 0, 1 + |kappa| otherwise; at most marg) of the tile
    const double ml = kap >= 0.0 ? 1.0 : 1.0 - kap;
    const AdjRows rr = adj_rows(xck, kap, jc, ml, nmaj, nmin, maj0, min0, TM, TN);
    const int ra = rr.ra, rb = rr.rb;
    const double x0 = rr.x0;
    (void)marg;
    if (ra > rb) return;
    const BoxRow bk = box_row(kap);
    const double q0 = adj_q0(x0, kap, ra, min0, 0.0);
    if (bk.neg) adj_walk_box<true>(q0, kap, rb - ra + 1, ra - maj0, ldexpf(sv, e), bk, W, s_a);
    else adj_walk_box<false>(q0, kap, rb - ra + 1, ra - maj0, ldexpf(sv, e), bk, W, s_a);
}

template <int N>
__device__ inline void adj_line(const AdjArgs& A, double xck, double kapk, bool active, float sv, int e,
                                bool vert, int maj0, int min0, int TM, int TN, int nmaj, int W,
                                double jc, double marg, int* s_a, int* s_k)
{
    const double H = 0.5 * (N + 1);
    int ra = 0, rb = -1;
    double kap = 0.0, x0 = 0.0;
    if (active) {
        kap = kapk;
        const int nmin = vert ? A.nx : A.ny;
        // rows whose crossing lies within the footprint's half-width
        // H (1 + |kappa|) of the tile (at most marg)
        const AdjRows rr = adj_rows(xck, kap, jc, H * (1.0 + fabs(kap)), nmaj, nmin, maj0, min0, TM, TN);
        ra = rr.ra;
        rb = rr.rb;
        x0 = rr.x0;
    }
    (void)marg;
    const bool work = active && ra <= rb;
    const LineConst lc = line_const<N>(kap);
    const int S = wave_slots<N>(work ? lc.slots : 1);
    if (!work) return;
    const float svs = ldexpf(sv, e);
    const float svk = ldexpf(sv, e + knot_shift<N>());
    // local q: column index within the LDS row (halo included)
    const double q0 = adj_q0(x0, kap, ra, min0, H);
    const int cnt = rb - ra + 1, row0 = ra - maj0;
    if (S == 1) adj_walk<N, 1>(q0, kap, cnt, row0, svs, svk, lc, W, s_a, s_k);
    else if (S == 2) adj_walk<N, (N >= 1 ? 2 : 1)>(q0, kap, cnt, row0, svs, svk, lc, W, s_a, s_k);
    else if (S == 3) adj_walk<N, (N >= 2 ? 3 : 1)>(q0, kap, cnt, row0, svs, svk, lc, W, s_a, s_k);
    else adj_walk<N, (N >= 3 ? 4 : 1)>(q0, kap, cnt, row0, svs, svk, lc, W, s_a, s_k);
}

__device__ inline float block_max(float v, float* red)
{
    // wave-level then block-level maximum (kBlock = 4 waves of 64)
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// 5 waves per SIMD (95 VGPRs, 29 KB of LDS per workgroup)
#ifndef XRT_ADJ_WAVES
#define XRT_ADJ_WAVES 5
#endif
#define XRT_ADJ_ATTR __attribute__((amdgpu_waves_per_eu(XRT_ADJ_WAVES, XRT_ADJ_WAVES)))
// LDS of one adjoint workgroup
struct AdjShared {
    int a[kAccWords];
    int k[kAccWords];
    uint32_t start[kSlopeBins];
    uint32_t pre[kSlopeBins + 1];
    uint32_t scan[kBlock];
    uint32_t run[8 * kAdjLptMax];  // slope bins of the first and last item of each run of 64 items of a chunk
    float red[4];
};

// Which lines a launch takes: the vertical lines on kTileI x kTileJ tiles,
// or the horizontal lines on the transposed kTileJ x kTileI tiles (adding
// into the image the first launch wrote).  A tile is thus always kTileI
// pixels across the lines it takes, so a line rarely leaves the tile's rows
// early and idles its lane for the rest of the wave's walk.
enum AdjMode { kAdjVert = 1, kAdjHoriz = 2 };

template <int MODE>
__device__ constexpr int adj_ti() { return MODE == kAdjHoriz ? kTileJ : kTileI; }
template <int MODE>
__device__ constexpr int adj_tj() { return MODE == kAdjHoriz ? kTileI : kTileJ; }

// One pixel tile of the adjoint; `kpart` selects this workgroup's share of
// the candidate chunks when A.split > 1.
template <int N, int MODE>
__device__ __forceinline__ void adj_tile(const AdjArgs& A, int tile, int kpart, AdjShared& sh)
{
    constexpr int TI = adj_ti<MODE>(), TJ = adj_tj<MODE>();
    int* s_a = sh.a;
    int* s_k = sh.k;
    uint32_t* s_start = sh.start;
    uint32_t* s_pre = sh.pre;
    uint32_t* s_scan = sh.scan;
    float* s_red = sh.red;
    const int tid = threadIdx.x;
    // consecutive tiles (one XCD's range, sharing its L2) run along the
    // lines: down a column of tiles for vertical lines, along a row for
    // horizontal ones
    constexpr bool kColMajor = MODE == kAdjVert;
    const int ti = kColMajor ? tile / A.tiles_j : tile % A.tiles_i;
    const int tj = kColMajor ? tile % A.tiles_j : tile / A.tiles_i;
    const int i0 = ti * TI, j0 = tj * TJ;
    // a row whose crossing X lies outside (min0 - (n+1), min0 + TN + n) adds
    // nothing to the tile's outputs: its taps J-d (J = floor(X + (n+1)/2))
    // miss [min0, min0 + TN) and its knots (within (n+1)/2 of X + (n+1)/2)
    // miss [min0, min0 + TN + n].  Box spline: columns floor(X)-1 .. floor(X)+2.
    const double marg = N == kBox3 ? 2.0 : (double)N + 1.0;

    float o[kPix];
#pragma unroll
    for (int e = 0; e < kPix; ++e) o[e] = 0.f;

    {
        constexpr bool vert = MODE == kAdjVert;
        // tile in (major, minor) coordinates of this orientation
        const int maj0 = vert ? j0 : i0, min0 = vert ? i0 : j0;
        const int TM = vert ? TJ : TI, TN = vert ? TI : TJ;
        const int nmaj = vert ? A.ny : A.nx;
        const int W = TN + 2 * kHalo + 1;  // odd pitch (kAccPitch)
        static_assert(adj_ti<MODE>() == kTileI || adj_tj<MODE>() == kTileI, "kTileI across the lines");
        const int nbk = vert ? A.nbk_v : A.nbk_h;
        const int boff = vert ? A.boff_v : A.boff_h;
        const uint32_t cls_base = vert ? 0u : (uint32_t)kSlopeBins * (uint32_t)A.nbk_v;
        const double jc = 0.5 * (nmaj - 1);

        for (int e = tid; e < TM * W; e += kBlock) {
            s_a[e] = 0;
            if constexpr (N != kBox3) s_k[e] = 0;
        }
        // candidate range of every slope bin: lines whose crossing of some
        // tile row falls within [min0 - marg, min0 + TN - 1 + marg]
        uint32_t cnt_local[kSlopeBins / kBlock];
#pragma unroll
        for (int u = 0; u < kSlopeBins / kBlock; ++u) {
            const int b = tid + u * kBlock;
            const double klo = -1.0 + 2.0 * b / kSlopeBins, khi = -1.0 + 2.0 * (b + 1) / kSlopeBins;
            const double da = maj0 - jc, db = maj0 + TM - 1 - jc;
            const double e1 = klo * da, e2 = klo * db, e3 = khi * da, e4 = khi * db;
            const double mx = fmax(fmax(e1, e2), fmax(e3, e4));
            const double mn = fmin(fmin(e1, e2), fmin(e3, e4));
            const double xlo = min0 - marg - mx, xhi = min0 + TN - 1 + marg - mn;
            int blo = (int)fmin(fmax(floor(xlo) + boff, 0.0), (double)(nbk - 1));
            int bhi = (int)fmin(fmax(floor(xhi) + boff, 0.0), (double)(nbk - 1));
            const uint32_t base = cls_base + (uint32_t)b * (uint32_t)nbk;
            const uint32_t st = A.off[base + blo], en = A.off[base + bhi + 1];
            s_start[b] = st;
            cnt_local[u] = en - st;
        }
        // exclusive scan of the counts (bins tid and tid + kBlock)
        {
            uint32_t tot;
            uint32_t p0 = block_excl_scan(cnt_local[0], s_scan, &tot);
            const uint32_t tot0 = tot;
            uint32_t p1 = block_excl_scan(cnt_local[1], s_scan, &tot);
            s_pre[tid] = p0;
            s_pre[tid + kBlock] = tot0 + p1;
            if (tid == 0) s_pre[kSlopeBins] = tot0 + tot;
        }
        __syncthreads();
        const uint32_t total = s_pre[kSlopeBins];

        constexpr int kAdjLpt = adj_lpt<N>();
        static_assert(kAdjLpt <= kAdjLptMax, "run table too small");
        constexpr uint32_t kChunk = (uint32_t)kAdjLpt * kBlock;
        for (uint32_t base = (uint32_t)kpart * kChunk; base < total; base += (uint32_t)A.split * kChunk) {
            // item -> slope bin b with s_pre[b] <= item < s_pre[b+1].  Each
            // wave takes runs of 64 consecutive items; 16 threads first find
            // the bins of every run's first and last item, so that a lane
            // then searches only the few bins its run spans.
            if (tid < 8 * kAdjLpt) {
                const uint32_t first = base + (uint32_t)((tid >> 3) * kBlock + ((tid >> 1) & 3) * 64);
                uint32_t it = first;
                if (tid & 1) it = min(first + 63u, total - 1u);
                int lo = 0, hi = kSlopeBins;
                if (first < total) {
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= it) lo = mid;
                        else hi = mid;
                    }
                }
                sh.run[tid] = (uint32_t)lo;
            }
            __syncthreads();
            uint32_t kk[kAdjLpt];
            float svv[kAdjLpt];
            double xcv[kAdjLpt], kpv[kAdjLpt];
            float amax = 0.f;
#pragma unroll
            for (int u = 0; u < kAdjLpt; ++u) {
                kk[u] = 0;
                svv[u] = 0.f;
                xcv[u] = 0.0;
                kpv[u] = 0.0;
                const uint32_t item = base + (uint32_t)(u * kBlock + tid);
                if (item < total) {
                    const int r = (u << 3) | ((tid >> 6) << 1);
                    int lo = (int)sh.run[r], hi = (int)sh.run[r + 1] + 1;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= item) lo = mid;
                        else hi = mid;
                    }
                    kk[u] = s_start[lo] + (item - s_pre[lo]);
                    svv[u] = A.sw[kk[u]];
                    // the line records are loaded with the value (one
                    // latency instead of two before the walk)
                    xcv[u] = A.xc[kk[u]];
                    kpv[u] = A.kap[kk[u]];
                }
                // a NaN or infinite value is left out here (it would break
                // the chunk's scale); k_adj_nonfinite marks its pixels
                if (!(fabsf(svv[u]) <= FLT_MAX)) svv[u] = 0.f;
                amax = fmaxf(amax, fabsf(svv[u]));
            }
            const float mx = block_max(amax, s_red);
            if (!(mx > 0.f)) continue;  // uniform: nothing to add in this chunk
            int em;
            (void)frexpf(mx, &em);
            // |s| 2^e < 2^adj_scale_bits (every row weight is at most 1)
            const int e = adj_scale_bits<N>() - em;
            const double kscale = ldexp(1.0, -e - knot_shift<N>());
#pragma unroll
            for (int u = 0; u < kAdjLpt; ++u) {
                if constexpr (N == kBox3)
                    adj_line_box(A, xcv[u], kpv[u], svv[u] != 0.f, svv[u], e, vert, maj0, min0, TM, TN, nmaj, W, jc, marg,
                                 s_a);
                else
                    adj_line<N>(A, xcv[u], kpv[u], svv[u] != 0.f, svv[u], e, vert, maj0, min0, TM, TN, nmaj, W,
                                jc, marg, s_a, s_k);
            }
            __syncthreads();
            // flush: output += (A + Delta^T K) 2^-e  (forward difference of K)
#pragma unroll
            for (int q = 0; q < kPix; ++q) {
                const int p = tid + q * kBlock;
                const int pj = p / TI, pi = p % TI;  // pixel (row, column) in the tile
                const int lmaj = vert ? pj : pi, lmin = vert ? pi : pj;
                const int* ar = s_a + lmaj * W + kHalo + lmin;
                if constexpr (N == kBox3) {
                    o[q] += ldexpf((float)ar[0], -e);
                } else {
                    const int* kr = s_k + lmaj * W + kHalo + lmin;
                    // the (n+1)-th difference of integers below 2^30 (at most
                    // 2^35 in magnitude) is exact in FP64; scaled by a power of
                    // two, then rounded once to FP32
                    double v = 0.0;
#pragma unroll
                    for (int l = 0; l <= N + 1; ++l) v = fma((double)delta_w<N>(l), (double)kr[l], v);
                    o[q] += ldexpf((float)ar[0], -e) + (float)(v * kscale);
                }
            }
            __syncthreads();
            for (int z = tid; z < TM * W; z += kBlock) {
                s_a[z] = 0;
                if constexpr (N != kBox3) s_k[z] = 0;
            }
            // the next chunk's block_max synchronises before its atomics
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kPix; ++e) {
        const int p = tid + e * kBlock;
        const int pj = p / TI, pi = p % TI;
        const int i = i0 + pi, j = j0 + pj;
        if (i < A.nx && j < A.ny) {
            if (A.split > 1) A.part[((int64_t)kpart * A.ny + j) * A.nx + i] = o[e];
            else if (A.accumulate) A.out[(int64_t)j * A.nx + i] += o[e];
            else A.out[(int64_t)j * A.nx + i] = o[e];
        }
    }
}

template <int N, int MODE>
__global__ void __launch_bounds__(kBlock) XRT_ADJ_ATTR k_adjoint(AdjArgs A)
{
    __shared__ AdjShared sh;
    const int tile = xcd_logical(blockIdx.x, A.ntiles_pad);
    if (tile >= A.ntiles) return;  // uniform per block
    adj_tile<N, MODE>(A, tile, (int)blockIdx.y, sh);
}

// Both passes in one launch (small grids, where one pass's workgroups do
// not fill the GPU): blockIdx.y < split runs the vertical lines' tile parts,
// the rest the horizontal lines' on the transposed tiles; every part writes
// its own partial image (V.part, then H.part), which one reduction adds in
// order.
template <int N>
__global__ void __launch_bounds__(kBlock) XRT_ADJ_ATTR k_adjoint_both(AdjArgs V, AdjArgs H)
{
    __shared__ AdjShared sh;
    const bool vert = (int)blockIdx.y < V.split;   // uniform per block
    const AdjArgs& A = vert ? V : H;
    if ((int)blockIdx.x >= A.ntiles_pad) return;
    const int tile = xcd_logical(blockIdx.x, A.ntiles_pad);
    if (tile >= A.ntiles) return;
    if (vert) adj_tile<N, kAdjVert>(V, tile, (int)blockIdx.y, sh);
    else adj_tile<N, kAdjHoriz>(H, tile, (int)blockIdx.y - V.split, sh);
}

// Lines whose (sorted, scaled) sinogram value is NaN or infinite: the
// adjoint's fixed-point sums leave them out, and every pixel inside the
// line's footprint support, |X(j) - i| < W in each row j it reaches, is set
// to NaN here, after both passes.  W is the support half-width in minor
// cells: (n+1)(1 + |kappa|)/2 for the B-splines, 1 (kappa >= 0) or
// 1 + |kappa| for the box spline.
__device__ inline void adj_nonfinite_line(const NonFiniteArgs& A, int64_t k)
{
    if (k >= A.m) return;
    if (fabsf(A.sw[k]) <= FLT_MAX) return;
    if (k >= A.hdr->m_valid) return;
    const bool vert = k < A.hdr->m_vert;
    const int nmaj = vert ? A.ny : A.nx, nmin = vert ? A.nx : A.ny;
    const double kap = A.kap[k];
    const double x0 = A.xc[k] - kap * (0.5 * (nmaj - 1));
    const double W = A.box ? (kap >= 0.0 ? 1.0 : 1.0 - kap) : 0.5 * (A.degree + 1) * (1.0 + fabs(kap));
    int jlo, jhi;
    row_range(x0, kap, 1.0 / kap, W, nmaj, nmin, &jlo, &jhi);
    const float nan = __int_as_float(0x7fc00000);
    for (int j = jlo; j <= jhi; ++j) {
        const double X = x0 + kap * (double)j;
        const int lo = (int)fmax(floor(X - W) + 1.0, 0.0);
        const int hi = (int)fmin(ceil(X + W) - 1.0, (double)(nmin - 1));
        for (int i = lo; i <= hi; ++i) {
            const int64_t pix = vert ? (int64_t)j * A.nx + i : (int64_t)i * A.nx + j;
            A.out[pix] = nan;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_adj_nonfinite(NonFiniteArgs A)
{
    adj_nonfinite_line(A, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// out (+)= sum over the split workgroups' partial images, in a fixed order
__global__ void __launch_bounds__(kBlock) k_adj_reduce(const float* part, int split, int64_t npix, int accumulate,
                                                       float* out)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= npix) return;
    float v = part[k];
    for (int g = 1; g < split; ++g) v += part[(int64_t)g * npix + k];
    if (accumulate) v += out[k];
    out[k] = v;
}

// ---------------------------------------------------------------- batch
struct BatchProb {
    FwdArgs f;      // forward of this problem (sino = its sinogram buffer)
    AdjArgs a;      // adjoint, vertical lines (split 1, out = its image buffer)
    AdjArgs ah;     // adjoint, horizontal lines on transposed tiles (adds into out)
    int degree;
    int nstrip;     // strips of kStrip rows (the larger of the two orientations)
    int64_t m_vert, m_valid;
    float* spart;   // [nstrip][m] per-strip line sums (unscaled)
    NonFiniteArgs nf;  // lines with a non-finite sinogram value (after the adjoint)
};
struct BatchArgs {
    const BatchProb* probs;
    const int2* items;   // (problem, line block or tile)
    int nitems;
    unsigned int* counter;
    int lines_per_item;  // forward: lines per item, a multiple of kBlock
};

// Many problems (each with its own plan) in persistent launches: one for the
// forward, two for the adjoint (one per orientation).  Work items (problem,
// block of lines) for the forward and (problem, tile) for the adjoint are
// listed largest problem first; every workgroup takes the next item from its
// launch's atomic counter until the list is exhausted (the only atomics on
// global memory: the adjoint of an item is the gather of one tile, whose
// pixels only that workgroup writes in that launch).
// Line k over the rows of strip `st` (unscaled sum into spart[st][k]).
template <int N, bool VERT>
__device__ inline void fwd_line_strip(const BatchProb& P, int64_t k, int st)
{
    int ja, jb;
    P.spart[(int64_t)st * P.f.m + k] = fwd_strip_sum<N, VERT>(P.f, k, st, &ja, &jb);
}

template <int N>
__device__ inline void fwd_block_any(const BatchProb& P, int64_t k0, int st)
{
    const int64_t k = k0 + threadIdx.x;
    if (k < P.m_vert) fwd_line_strip<N, true>(P, k, st);
    else if (k < P.m_valid) fwd_line_strip<N, false>(P, k, st);
}

// items (problem, strip * blocks + block): the items of one problem are
// listed strip by strip, so the workgroups in flight share one strip of its
// layouts (as in the single-problem schedule)
__global__ void __launch_bounds__(kBlock) k_batch_forward(BatchArgs B)
{
    __shared__ int s_item;
    for (;;) {
        const int it = next_item(B.counter, &s_item);
        if (it >= B.nitems) break;
        const int2 w = B.items[it];
        const BatchProb& P = B.probs[w.x];
        const int deg = P.degree;
        const int nb = (int)((P.f.m + B.lines_per_item - 1) / B.lines_per_item);
        const int st = w.y / nb, blk = w.y - st * nb;
        const int64_t base = (int64_t)blk * B.lines_per_item;
        for (int sub = 0; sub < B.lines_per_item; sub += kBlock) {
            const int64_t k0 = base + sub;
            if (k0 >= P.f.m) break;
            switch (deg) {
            case 0: fwd_block_any<0>(P, k0, st); break;
            case 1: fwd_block_any<1>(P, k0, st); break;
            case 2: fwd_block_any<2>(P, k0, st); break;
            case 3: fwd_block_any<3>(P, k0, st); break;
            default: fwd_block_any<kBox3>(P, k0, st); break;
            }
        }
    }
}

// sino[idx[k]] = (sum of the strips' sums of line k) * h / max(|cos|,|sin|),
// 0 for lines that miss the grid; one launch per problem
__global__ void __launch_bounds__(kBlock) k_batch_fwd_reduce(const BatchProb* probs, int p)
{
    const BatchProb& P = probs[p];
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= P.f.m) return;
    float v = 0.f;
    if (k < P.m_valid) {
        const int ns = k < P.m_vert ? P.f.strips_v : P.f.strips_h;
        double acc = 0.0;
        for (int st = 0; st < ns; ++st) acc += (double)P.spart[(int64_t)st * P.f.m + k];
        const double kap = P.f.kap[k];
        const int n = P.degree;  // the box spline's row sums are unscaled, as degrees 0..2
        const double ts = n == 3 ? (double)tap_scale<3>() : n == 2 ? (double)tap_scale<2>()
                        : n == 1 ? (double)tap_scale<1>() : (double)tap_scale<0>();
        v = (float)(acc * P.f.h * sqrt(1.0 + kap * kap) / ts);
    }
    P.f.sino[P.f.idx[k]] = v;
}

// One orientation of the adjoint of every problem: the vertical lines on
// kTileI x kTileJ tiles, or (a second launch, adding into the images) the
// horizontal lines on the transposed tiles.
template <int MODE>
__global__ void __launch_bounds__(kBlock) XRT_ADJ_ATTR k_batch_adjoint(BatchArgs B)
{
    __shared__ AdjShared sh;
    __shared__ int s_item;
    for (;;) {
        const int it = next_item(B.counter, &s_item);
        if (it >= B.nitems) break;
        const int2 w = B.items[it];
        const BatchProb& P = B.probs[w.x];
        const AdjArgs& A = MODE == kAdjVert ? P.a : P.ah;
        switch (P.degree) {
        case 0: adj_tile<0, MODE>(A, w.y, 0, sh); break;
        case 1: adj_tile<1, MODE>(A, w.y, 0, sh); break;
        case 2: adj_tile<2, MODE>(A, w.y, 0, sh); break;
        case 3: adj_tile<3, MODE>(A, w.y, 0, sh); break;
        default: adj_tile<kBox3, MODE>(A, w.y, 0, sh); break;
        }
    }
}

__global__ void k_reset_counter(unsigned int* c) { c[threadIdx.x] = 0u; }

// ---------------------------------------------------------------- nnz
struct NnzArgs {
    int64_t m;
    const PlanHeader* hdr;
    const double* xc;
    const double* kap;
    int nx, ny, degree;
    unsigned long long* out;
};

__global__ void __launch_bounds__(kBlock) k_nnz(NnzArgs A)
{
    __shared__ unsigned long long sh[kBlock];
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long cnt = 0;
    if (k < A.m && k < A.hdr->m_valid) {
        const bool vert = k < A.hdr->m_vert;
        const int nmaj = vert ? A.ny : A.nx, nmin = vert ? A.nx : A.ny;
        const double kap = A.kap[k];
        const double x0 = A.xc[k] - kap * (0.5 * (nmaj - 1));
        // support half-width in minor cells: (n+1)(1 + |kappa|)/2 for B-splines;
        // the box spline: 1 (kappa >= 0) or 1 + |kappa| (kappa < 0)
        const double W = A.degree == kBox3 ? (kap >= 0.0 ? 1.0 : 1.0 + fabs(kap))
                                           : 0.5 * (A.degree + 1) * (1.0 + fabs(kap));
        int jlo, jhi;
        row_range(x0, kap, 1.0 / kap, W, nmaj, nmin, &jlo, &jhi);
        for (int j = jlo; j <= jhi; ++j) {
            const double X = x0 + kap * (double)j;
            // integers i in (X - W, X + W) within [0, nmin - 1]
            double lo = fmax(floor(X - W) + 1.0, 0.0);
            double hi = fmin(ceil(X + W) - 1.0, (double)(nmin - 1));
            if (hi >= lo) cnt += (unsigned long long)(hi - lo + 1.0);
        }
    }
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(A.out, sh[0]);
}

// ---------------------------------------------------------------- launchers
hipError_t launch_canon(const CanonArgs& a, hipStream_t s)
{
    if (a.m == 0) return hipSuccess;
    dim3 grid((unsigned)((a.m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_canon, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Exclusive scan of n counts into out[0..n] (out[n] = total); tmp needs
// room for the per-block partials of every level.
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s)
{
    const int64_t nblk = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nblk), dim3(kBlock), 0, s, in, out, tmp, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nblk > 1) {
        // scan the block totals (in place into tmp + nblk), then add
        e = launch_scan(tmp, tmp + nblk, nblk, tmp + nblk + nblk + 1, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nblk), dim3(kBlock), 0, s, out,
                           (const uint32_t*)(tmp + nblk), n);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // total = scanned last partial + last block total
        return hipMemcpyAsync(out + n, tmp + nblk + nblk, sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, s);
    }
    return hipMemcpyAsync(out + n, tmp, sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
}

int64_t scan_tmp_words(int64_t n)
{
    int64_t w = 0;
    while (true) {
        int64_t nblk = (n + kScanTile - 1) / kScanTile;
        w += nblk + nblk + 1;
        if (nblk <= 1) break;
        n = nblk;
    }
    return w + 16;
}

int64_t radix_tmp_words(int64_t m, int64_t max_key)
{
    const int64_t nblk = (m + kRsTile - 1) / kRsTile;
    const int64_t nh = 256 * nblk;
    (void)max_key;
    // key and value ping-pong buffers, the digit table and its scan
    return 3 * m + 2 * nh + 1 + scan_tmp_words(nh);
}

hipError_t launch_radix_sort(const SortArgs& a, hipStream_t s)
{
    if (a.m == 0) return hipSuccess;
    int bits = 0;
    while (bits < 32 && (a.max_key >> bits) != 0) ++bits;
    const int passes = bits <= 8 ? 1 : (bits + 7) / 8;
    const int64_t nblk = (a.m + kRsTile - 1) / kRsTile;
    const int64_t nh = 256 * nblk;
    uint32_t* key2 = a.tmp;
    uint32_t* val1 = key2 + a.m;
    uint32_t* val2 = val1 + a.m;
    uint32_t* hist = val2 + a.m;
    uint32_t* hoff = hist + nh;
    uint32_t* stmp = hoff + nh + 1;
    const uint32_t* kin = a.key;
    const uint32_t* vin = nullptr;  // the first pass numbers the lines itself
    uint32_t* kout = key2;
    uint32_t* vout = val1;
    uint32_t* kspare = a.key;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(kBlock), 0, s, kin, a.m, 8 * p, hist, (int)nblk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_scan(hist, hoff, nh, stmp, s);
        if (e != hipSuccess) return e;
        RadixArgs ra;
        ra.key_in = kin;
        ra.val_in = vin;
        ra.key_out = kout;
        ra.val_out = vout;
        ra.m = a.m;
        ra.shift = 8 * p;
        ra.hoff = hoff;
        ra.nblk = (int)nblk;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, s, ra);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // the output becomes the next input; the old input's buffers take the next output
        uint32_t* knext = kspare;
        kspare = kout;
        kin = kout;
        kout = knext;
        vin = vout;
        vout = vout == val1 ? val2 : val1;
    }
    dim3 grid((unsigned)((a.m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_rs_gather, grid, dim3(kBlock), 0, s, vin, a.xc_in, a.kap_in, a.xc, a.kap, a.idx, a.m);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_header(PlanHeader* hdr, const uint32_t* off, int64_t vert_end, int64_t valid_end,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_header, dim3(1), dim3(1), 0, s, hdr, off, vert_end, valid_end);
    return hipGetLastError();
}

template <int N>
static hipError_t layouts_n(const xrt_plan* p, const float* coeffs, hipStream_t s)
{
    const int nx = p->g.nx, ny = p->g.ny;
    dim3 gv((unsigned)((p->pitch_v + kBlock - 1) / kBlock), (unsigned)ny);
    hipLaunchKernelGGL(k_layout_v<N>, gv, dim3(kBlock), 0, s, coeffs, nx, ny, p->pitch_v, p->cv,
                       p->dv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 gh((unsigned)((p->pitch_h + kTr - 1) / kTr), (unsigned)((nx + kTr - 1) / kTr));
    hipLaunchKernelGGL(k_layout_h<N>, gh, dim3(kBlock), 0, s, coeffs, nx, ny, p->pitch_h, p->ch,
                       p->dh);
    return hipGetLastError();
}

static FwdArgs make_fwd_args(const xrt_plan* p, float* sino)
{
    FwdArgs a;
    a.m = p->m;
    a.hdr = p->hdr;
    a.xc = p->xc;
    a.kap = p->kap;
    a.idx = p->idx;
    a.cv = p->cv;
    a.dv = p->dv;
    a.ch = p->ch;
    a.dh = p->dh;
    a.pitch_v = p->pitch_v;
    a.pitch_h = p->pitch_h;
    a.nx = p->g.nx;
    a.ny = p->g.ny;
    a.h = p->g.h;
    a.sino = sino;
    a.part = p->part;
    a.spart = p->spart;
    a.counter = p->fctr;
    a.persist = p->fwd_persist;
    a.lines_per_item = p->fwd_lpi;
    a.sub = p->fwd_sub;
    a.strips_v = p->strips_v;
    a.strips_h = p->strips_h;
    a.strip = 0;
    a.q = 0;
    a.nblk = (int)((p->m + kBlock - 1) / kBlock);
    a.nblk_pad = (a.nblk + 7) / 8 * 8;
    return a;
}

static AdjArgs make_adj_args(const xrt_plan* p, float* out, int mode)
{
    const int ti = mode == kAdjHoriz ? kTileJ : kTileI, tj = mode == kAdjHoriz ? kTileI : kTileJ;
    AdjArgs a;
    a.xc = p->xc;
    a.kap = p->kap;
    a.sw = p->sw;
    a.off = p->off;
    a.nx = p->g.nx;
    a.ny = p->g.ny;
    a.nbk_v = p->nbk_v;
    a.nbk_h = p->nbk_h;
    a.boff_v = p->boff_v;
    a.boff_h = p->boff_h;
    a.tiles_i = (p->g.nx + ti - 1) / ti;
    a.tiles_j = (p->g.ny + tj - 1) / tj;
    a.ntiles = a.tiles_i * a.tiles_j;
    a.ntiles_pad = (a.ntiles + 7) / 8 * 8;
    a.out = out;
    a.split = 1;
    a.part = nullptr;
    a.accumulate = 0;
    return a;
}

template <int N>
static hipError_t forward_n(const xrt_plan* p, float* sino, hipStream_t s)
{
    FwdArgs a = make_fwd_args(p, sino);
    if (p->fwd_persist) {
        hipError_t e = launch_reset_counters(p->fctr, 1, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_forward_persist<N>, dim3((unsigned)p->fwd_grid), dim3(kBlock), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_fwd_reduce<N>, dim3((unsigned)a.nblk), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    // the split between vertical and horizontal lines is known on the device
    // only: the grid of each launch covers all m lines and blocks past the
    // launch's range return at once
    const int ns = p->strips_v > p->strips_h ? p->strips_v : p->strips_h;
    for (int sq = 0; sq < ns * p->fwd_sub; ++sq) {
        const int st = sq / p->fwd_sub;
        a.strip = st;
        a.q = sq - st * p->fwd_sub;
        if (st < p->strips_v) {
            hipLaunchKernelGGL((k_forward<N, true>), dim3((unsigned)a.nblk_pad), dim3(kBlock), 0, s, a);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (st < p->strips_h) {
            hipLaunchKernelGGL((k_forward<N, false>), dim3((unsigned)a.nblk_pad), dim3(kBlock), 0, s,
                               a);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_fwd_reduce<N>, dim3((unsigned)a.nblk), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_forward(const xrt_plan* p, const float* coeffs, float* sino, hipStream_t s)
{
    if (p->m == 0) return hipSuccess;
    hipError_t e;
    switch (p->degree) {
    case kBox3:  // the coefficient layouts only (the difference arrays go unused)
        e = layouts_n<0>(p, coeffs, s);
        if (e == hipSuccess) e = forward_n<kBox3>(p, sino, s);
        break;
    case 0: e = layouts_n<0>(p, coeffs, s); if (e == hipSuccess) e = forward_n<0>(p, sino, s); break;
    case 1: e = layouts_n<1>(p, coeffs, s); if (e == hipSuccess) e = forward_n<1>(p, sino, s); break;
    case 2: e = layouts_n<2>(p, coeffs, s); if (e == hipSuccess) e = forward_n<2>(p, sino, s); break;
    default: e = layouts_n<3>(p, coeffs, s); if (e == hipSuccess) e = forward_n<3>(p, sino, s); break;
    }
    return e;
}

// The vertical lines on kTileI x kTileJ tiles write the image; the
// horizontal lines on the transposed tiles then add to it (same stream, so
// the second launch sees the first's writes).
template <int N, int MODE>
static hipError_t adjoint_pass(const xrt_plan* p, float* out, hipStream_t s)
{
    AdjArgs a = make_adj_args(p, out, MODE);
    a.split = p->adj_split;
    a.part = p->adj_part;
    a.accumulate = MODE == kAdjHoriz ? 1 : 0;
    hipLaunchKernelGGL((k_adjoint<N, MODE>), dim3((unsigned)a.ntiles_pad, (unsigned)a.split), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.split == 1) return e;
    const int64_t npix = (int64_t)p->g.nx * p->g.ny;
    hipLaunchKernelGGL(k_adj_reduce, dim3((unsigned)((npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a.part,
                       a.split, npix, a.accumulate, out);
    return hipGetLastError();
}

static NonFiniteArgs make_nonfinite_args(const xrt_plan* p, const float* sw, float* out)
{
    NonFiniteArgs a;
    a.m = p->m;
    a.hdr = p->hdr;
    a.xc = p->xc;
    a.kap = p->kap;
    a.sw = sw;
    a.nx = p->g.nx;
    a.ny = p->g.ny;
    a.degree = geom_degree(p->degree);
    a.box = p->degree == kBox3 ? 1 : 0;
    a.out = out;
    return a;
}

hipError_t launch_adj_nonfinite(const xrt_plan* p, const float* sw, float* out, hipStream_t s)
{
    if (p->m == 0) return hipSuccess;
    const NonFiniteArgs a = make_nonfinite_args(p, sw, out);
    hipLaunchKernelGGL(k_adj_nonfinite, dim3((unsigned)((p->m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int N>
static hipError_t adjoint_n(const xrt_plan* p, float* out, hipStream_t s)
{
    if (p->adj_merge) {
        const int64_t npix = (int64_t)p->g.nx * p->g.ny;
        AdjArgs v = make_adj_args(p, out, kAdjVert), h = make_adj_args(p, out, kAdjHoriz);
        v.split = h.split = p->adj_split;
        v.part = p->adj_part;
        h.part = p->adj_part + (size_t)p->adj_split * (size_t)npix;
        const int gx = v.ntiles_pad > h.ntiles_pad ? v.ntiles_pad : h.ntiles_pad;
        hipLaunchKernelGGL(k_adjoint_both<N>, dim3((unsigned)gx, (unsigned)(2 * p->adj_split)), dim3(kBlock), 0, s,
                           v, h);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_adj_reduce, dim3((unsigned)((npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           p->adj_part, 2 * p->adj_split, npix, 0, out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_adj_nonfinite(p, p->sw, out, s);
    }
    hipError_t e = adjoint_pass<N, kAdjVert>(p, out, s);
    if (e != hipSuccess) return e;
    e = adjoint_pass<N, kAdjHoriz>(p, out, s);
    if (e != hipSuccess) return e;
    return launch_adj_nonfinite(p, p->sw, out, s);
}

static hipError_t sort_sino(const xrt_plan* p, const float* sino, hipStream_t s)
{
    if (p->m > 0) {
        SortSinoArgs a;
        a.m = p->m;
        a.hdr = p->hdr;
        a.kap = p->kap;
        a.idx = p->idx;
        a.sino = sino;
        a.h = p->g.h;
        a.sw = p->sw;
        hipLaunchKernelGGL(k_sort_sino, dim3((unsigned)((p->m + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, s, a);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_adjoint(const xrt_plan* p, const float* sino, float* out, hipStream_t s)
{
    hipError_t e = sort_sino(p, sino, s);
    if (e != hipSuccess) return e;
    switch (p->degree) {
    case kBox3: return adjoint_n<kBox3>(p, out, s);
    case 0: return adjoint_n<0>(p, out, s);
    case 1: return adjoint_n<1>(p, out, s);
    case 2: return adjoint_n<2>(p, out, s);
    default: return adjoint_n<3>(p, out, s);
    }
}

hipError_t launch_nnz(const xrt_plan* p, unsigned long long* out, hipStream_t s)
{
    if (p->m == 0) return hipSuccess;
    NnzArgs a;
    a.m = p->m;
    a.hdr = p->hdr;
    a.xc = p->xc;
    a.kap = p->kap;
    a.nx = p->g.nx;
    a.ny = p->g.ny;
    a.degree = p->degree;
    a.out = out;
    hipLaunchKernelGGL(k_nnz, dim3((unsigned)((p->m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batch (host side)
size_t batch_prob_size() { return sizeof(BatchProb); }

int batch_strips(const xrt_plan* p) { return p->strips_v > p->strips_h ? p->strips_v : p->strips_h; }

void batch_fill(const xrt_plan* p, float* sino, float* back, float* spart, void* dst)
{
    BatchProb b;
    b.f = make_fwd_args(p, sino);
    b.a = make_adj_args(p, back, kAdjVert);
    b.ah = make_adj_args(p, back, kAdjHoriz);
    b.ah.accumulate = 1;
    b.degree = p->degree;
    b.nstrip = batch_strips(p);
    b.m_vert = p->m_vert;
    b.m_valid = p->m_valid;
    b.spart = spart;
    b.nf = make_nonfinite_args(p, p->sw, back);
    memcpy(dst, &b, sizeof(b));
}

hipError_t launch_batch_fwd_reduce(const void* probs, int p, int64_t m, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_fwd_reduce, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       static_cast<const BatchProb*>(probs), p);
    return hipGetLastError();
}

hipError_t launch_layouts(const xrt_plan* p, const float* coeffs, hipStream_t s)
{
    if (p->m == 0) return hipSuccess;
    switch (p->degree) {
    case 0: return layouts_n<0>(p, coeffs, s);
    case 1: return layouts_n<1>(p, coeffs, s);
    case 2: return layouts_n<2>(p, coeffs, s);
    case 3: return layouts_n<3>(p, coeffs, s);
    default: return layouts_n<0>(p, coeffs, s);  // box spline: the coefficient layouts only
    }
}

hipError_t launch_sort_sino(const xrt_plan* p, const float* sino, hipStream_t s) { return sort_sino(p, sino, s); }

// k_adj_nonfinite over every problem of a batch (blockIdx.y = problem)
__global__ void __launch_bounds__(kBlock) k_batch_nonfinite(const BatchProb* probs)
{
    adj_nonfinite_line(probs[blockIdx.y].nf, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

hipError_t launch_batch_nonfinite(const void* probs, int count, int64_t max_m, hipStream_t s)
{
    if (max_m == 0 || count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_nonfinite, dim3((unsigned)((max_m + kBlock - 1) / kBlock), (unsigned)count),
                       dim3(kBlock), 0, s, static_cast<const BatchProb*>(probs));
    return hipGetLastError();
}

hipError_t launch_reset_counters(unsigned int* c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3((unsigned)n), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_batch_forward(const void* probs, const int2* items, int nitems, unsigned int* counter,
                                int lines_per_item, int grid, hipStream_t s)
{
    BatchArgs b;
    b.probs = static_cast<const BatchProb*>(probs);
    b.items = items;
    b.nitems = nitems;
    b.counter = counter;
    b.lines_per_item = lines_per_item;
    hipLaunchKernelGGL(k_batch_forward, dim3((unsigned)grid), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_adjoint(const void* probs, const int2* items, int nitems, unsigned int* counter, int grid,
                                int horizontal, hipStream_t s)
{
    BatchArgs b;
    b.probs = static_cast<const BatchProb*>(probs);
    b.items = items;
    b.nitems = nitems;
    b.counter = counter;
    b.lines_per_item = kBlock;
    if (horizontal) hipLaunchKernelGGL(k_batch_adjoint<kAdjHoriz>, dim3((unsigned)grid), dim3(kBlock), 0, s, b);
    else hipLaunchKernelGGL(k_batch_adjoint<kAdjVert>, dim3((unsigned)grid), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

}  // namespace xrt
