// Kernels of composed programs: one data-parallel kernel per construct in the
// forward pass (its output view is the tape entry the reverse pass reads), and
// the generated adjoint of each construct in the reverse pass.  Shadows are
// FP64 and accumulate with +=, as in the generated code of section 4.
#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

namespace {

constexpr int kBS = 256;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

__device__ __forceinline__ double map_f(int fn, double s) {
    return fn == 0 ? s * s : psi_from_sq(s * s);
}
__device__ __forceinline__ double map_df(int fn, double s) {
    return fn == 0 ? 2.0 * s : dpsi_from(s, s * s);
}

__global__ void __launch_bounds__(kBS)
k_scale(int64_t n, const double* __restrict__ a, double alpha, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) y[i] = alpha * a[i];
}

__global__ void __launch_bounds__(kBS)
k_stencil(int64_t n, const double* __restrict__ a, ProgTaps taps, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < taps.n; ++t) {
        const int64_t j = i + taps.off[t];
        if (j >= 0 && j < n) s += taps.coef[t] * a[j];
    }
    y[i] = s;
}

__global__ void __launch_bounds__(kBS)
k_gather(int64_t E, int32_t k, const int32_t* __restrict__ conn, const double* __restrict__ B,
         const double* __restrict__ a, double* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += B[e * k + j] * a[conn[e * k + j]];
    y[e] = s;
}

__global__ void __launch_bounds__(kBS)
k_add(int64_t n, const double* __restrict__ a, double alpha, const double* __restrict__ b,
      double beta, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) y[i] = alpha * a[i] + beta * b[i];
}

__global__ void __launch_bounds__(kBS)
k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
      double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) y[i] = a[i] * b[i];
}

__global__ void __launch_bounds__(kBS)
k_map(int64_t n, const double* __restrict__ a, int fn, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) y[i] = map_f(fn, a[i]);
}

__global__ void __launch_bounds__(kBS)
k_sum(int64_t n, const double* __restrict__ a, double* __restrict__ partials) {
    __shared__ double lds[kBS / kWave];
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    const double s = block_sum<kBS>(i < n ? a[i] : 0.0, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ---------------------------------------------------------- reverse pass

// abar += alpha * ybar
__global__ void __launch_bounds__(kBS)
k_r_scale(int64_t n, const double* __restrict__ yb, double alpha, double* __restrict__ ab) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) ab[i] += alpha * yb[i];
}

// The reverse of a stencil reads ybar through several index expressions; it
// is rescheduled by the written index: abar_j += sum_t c_t ybar_{j - o_t}.
__global__ void __launch_bounds__(kBS)
k_r_stencil(int64_t n, const double* __restrict__ yb, ProgTaps taps, double* __restrict__ ab) {
    const int64_t j = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int t = 0; t < taps.n; ++t) {
        const int64_t i = j - taps.off[t];
        if (i >= 0 && i < n) s += taps.coef[t] * yb[i];
    }
    ab[j] += s;
}

// The reverse of a gather writes through an index that is a view entry: atomic.
__global__ void __launch_bounds__(kBS)
k_r_gather(int64_t E, int32_t k, const int32_t* __restrict__ conn, const double* __restrict__ B,
           const double* __restrict__ yb, double* __restrict__ ab) {
    const int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (e >= E) return;
    const double v = yb[e];
    for (int j = 0; j < k; ++j) atomic_add_f64(ab + conn[e * k + j], B[e * k + j] * v);
}

// abar += alpha ybar, bbar += beta ybar (either may be absent; a == b allowed:
// the same thread does both updates in order).
__global__ void __launch_bounds__(kBS)
k_r_add(int64_t n, const double* __restrict__ yb, double alpha, double* ab, double beta,
        double* bb) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const double v = yb[i];
    if (ab) ab[i] += alpha * v;
    if (bb) bb[i] += beta * v;
}

// abar += b ybar, bbar += a ybar (a and b are the stored forward values).
__global__ void __launch_bounds__(kBS)
k_r_mul(int64_t n, const double* __restrict__ yb, const double* a, const double* b, double* ab,
        double* bb) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const double v = yb[i], av = a[i], bv = b[i];
    if (ab) ab[i] += bv * v;
    if (bb) bb[i] += av * v;
}

// abar += fn'(a) ybar (a is the stored forward value).
__global__ void __launch_bounds__(kBS)
k_r_map(int64_t n, const double* __restrict__ yb, const double* __restrict__ a, int fn,
        double* __restrict__ ab) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) ab[i] += map_df(fn, a[i]) * yb[i];
}

// The reverse of the sum: broadcast the seed, abar += fbar.
__global__ void __launch_bounds__(kBS)
k_r_sum(int64_t n, double fbar, double* __restrict__ ab) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) ab[i] += fbar;
}

// ------------------------------------------------------------ prefix scan
//
// Inclusive scan in three launches over chunks of kScanItems entries: chunk
// totals, an exclusive scan of the totals by one workgroup, then each chunk's
// local scan offset by its prefix.  With rev set, entry i is read and written
// at n-1-i, which turns the prefix scan into the suffix scan of the reverse
// pass: abar_j += sum_{i >= j} ybar_i.  Summation order is fixed.

constexpr int kScanPer = 8;
constexpr int kScanItems = kBS * kScanPer;

__device__ __forceinline__ int64_t scan_at(int64_t n, int64_t i, int rev) { return rev ? n - 1 - i : i; }

// Exclusive scan of one value per thread over the workgroup; *total gets the sum.
__device__ __forceinline__ double block_excl_scan(double v, double* lds, double* total) {
    constexpr int NW = kBS / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double t = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += t;
    }
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const double t = lds[i];
        if (i < w) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + (inc - v);
}

__global__ void __launch_bounds__(kBS)
k_scan_totals(int64_t n, const double* __restrict__ a, int rev, double* __restrict__ totals) {
    __shared__ double lds[kBS / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (base + q < n) s += a[scan_at(n, base + q, rev)];
    const double t = block_sum<kBS>(s, lds);
    if (threadIdx.x == 0) totals[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBS)
k_scan_top(int64_t nchunks, double* __restrict__ totals) {
    __shared__ double lds[kBS / kWave];
    double carry = 0.0;
    for (int64_t b = 0; b < nchunks; b += kBS) {
        const int64_t i = b + threadIdx.x;
        const double v = i < nchunks ? totals[i] : 0.0;
        double tot;
        const double ex = block_excl_scan(v, lds, &tot);
        if (i < nchunks) totals[i] = carry + ex;
        carry += tot;
    }
}

// accumulate 0: y = scan; 1: y += scan.
__global__ void __launch_bounds__(kBS)
k_scan_apply(int64_t n, const double* __restrict__ a, int rev, const double* __restrict__ prefix,
             double* __restrict__ y, int accumulate) {
    __shared__ double lds[kBS / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
    double v[kScanPer];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = base + q < n ? a[scan_at(n, base + q, rev)] : 0.0;
        s += v[q];
    }
    double tot;
    double run = prefix[blockIdx.x] + block_excl_scan(s, lds, &tot);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        run += v[q];
        if (base + q < n) {
            const int64_t j = scan_at(n, base + q, rev);
            if (accumulate)
                y[j] += run;
            else
                y[j] = run;
        }
    }
}

hipError_t launch_scan(int64_t n, const double* a, int rev, double* scratch, double* y,
                       int accumulate, hipStream_t s) {
    const int64_t nchunks = (n + kScanItems - 1) / kScanItems;
    hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nchunks), dim3(kBS), 0, s, n, a, rev, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBS), 0, s, nchunks, scratch);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(kBS), 0, s, n, a, rev, scratch,
                       y, accumulate);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_prog_fwd(const ProgOpDev& o, hipStream_t s) {
    if (o.n == 0) return hipSuccess;
    switch (o.kind) {
        case P_SCALE: hipLaunchKernelGGL(k_scale, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.alpha, o.y); break;
        case P_STENCIL: hipLaunchKernelGGL(k_stencil, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.taps, o.y); break;
        case P_GATHER: hipLaunchKernelGGL(k_gather, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.k, o.conn, o.B, o.a, o.y); break;
        case P_ADD: hipLaunchKernelGGL(k_add, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.alpha, o.b, o.beta, o.y); break;
        case P_MUL: hipLaunchKernelGGL(k_mul, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.b, o.y); break;
        case P_MAP: hipLaunchKernelGGL(k_map, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.fn, o.y); break;
        case P_SUM: hipLaunchKernelGGL(k_sum, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.y); break;
        case P_SCAN: return launch_scan(o.n, o.a, 0, o.scratch, o.y, 0, s);
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prog_rev(const ProgOpDev& o, hipStream_t s) {
    if (o.n == 0) return hipSuccess;
    switch (o.kind) {
        case P_SCALE: hipLaunchKernelGGL(k_r_scale, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.yb, o.alpha, o.ab); break;
        case P_STENCIL: hipLaunchKernelGGL(k_r_stencil, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.yb, o.taps, o.ab); break;
        case P_GATHER: hipLaunchKernelGGL(k_r_gather, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.k, o.conn, o.B, o.yb, o.ab); break;
        case P_ADD: hipLaunchKernelGGL(k_r_add, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.yb, o.alpha, o.ab, o.beta, o.bb); break;
        case P_MUL: hipLaunchKernelGGL(k_r_mul, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.yb, o.a, o.b, o.ab, o.bb); break;
        case P_MAP: hipLaunchKernelGGL(k_r_map, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.yb, o.a, o.fn, o.ab); break;
        case P_SUM: hipLaunchKernelGGL(k_r_sum, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.alpha, o.ab); break;
        case P_SCAN: return launch_scan(o.n, o.yb, 1, o.scratch, o.ab, 1, s);
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t prog_sum_blocks(int64_t n) { return (n + kBS - 1) / kBS; }

int64_t prog_scan_chunks(int64_t n) { return (n + kScanItems - 1) / kScanItems; }

}  // namespace pg
