// Small kernels shared by the plans: the fixed-order final sums of per-
// workgroup partials, fills and conversions, and the plan-time kernels
// (connectivity validation, the exclusive scan and the transposed
// connectivity of the gather adjoint).
#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

namespace {

// Thread t adds partials t, t + B, t + 2B, ... in that order (B threads),
// then the workgroup reduces in a fixed butterfly.  The loads of up to kSumU
// consecutive terms of a thread are issued together before they are added,
// so a thread waits for memory once per kSumU terms, not once per term.
constexpr int kSumU = 8;

__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int64_t b, int64_t e) {
    double s = 0.0;
    const int64_t B = blockDim.x;
    for (int64_t q = b + threadIdx.x; q < e; q += kSumU * B) {
        double v[kSumU];
#pragma unroll
        for (int u = 0; u < kSumU; ++u) v[u] = q + u * B < e ? p[q + u * B] : 0.0;
#pragma unroll
        for (int u = 0; u < kSumU; ++u)
            if (q + u * B < e) s += v[u];
    }
    return s;
}

__global__ void __launch_bounds__(1024)
k_final_sum(const double* __restrict__ partials, int64_t n, double* __restrict__ out) {
    __shared__ double lds[16];
    const double s = block_sum_dyn(strided_sum(partials, 0, n), lds);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void __launch_bounds__(256)
k_segmented_sum(const double* __restrict__ partials, const int64_t* __restrict__ seg,
                int64_t nseg, double* __restrict__ out) {
    __shared__ double lds[16];
    const int64_t i = blockIdx.x;
    if (i >= nseg) return;
    const double s = block_sum_dyn(strided_sum(partials, seg[i], seg[i + 1]), lds);
    if (threadIdx.x == 0) out[i] = s;
}

// Zeroes bytes [0, head + 16 n16 + tail) of p, where p + head is 16-byte
// aligned and head, tail < 16: 16-byte stores over the aligned middle, single
// bytes at the two ends (workgroup 0).
__global__ void __launch_bounds__(256)
k_zero16(uint8_t* __restrict__ p, int64_t head, int64_t n16, int64_t tail) {
    uint4* __restrict__ mid = reinterpret_cast<uint4*>(p + head);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        mid[i] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0) {
        const int t = (int)threadIdx.x;
        if (t < head) p[t] = 0;
        if (t < tail) p[head + 16 * n16 + t] = 0;
    }
}

__global__ void __launch_bounds__(256) k_zero1(uint8_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// dst (FP32) (=|+=) src (FP64); with clear, src is left zero for the next call.
__global__ void __launch_bounds__(256)
k_f64_to_f32(double* __restrict__ src, float* __restrict__ dst, int64_t n, int accumulate, int clear,
             const double* __restrict__ partials, int64_t np, double* __restrict__ f_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = src[i];
        if (clear) src[i] = 0.0;
        dst[i] = accumulate ? static_cast<float>((double)dst[i] + v) : static_cast<float>(v);
    }
    // Workgroup 0 also sums the objective's partials in the fixed order of
    // k_final_sum, saving the reduction its own launch.
    if (f_out && blockIdx.x == 0) {
        __shared__ double lds[16];
        const double s = block_sum_dyn(strided_sum(partials, 0, np), lds);
        if (threadIdx.x == 0) f_out[0] = s;
    }
}

// y = alpha[0] * x in FP64, rounded once to T (y may alias x).
template <typename T>
__global__ void __launch_bounds__(256)
k_scale(int64_t n, const double* __restrict__ alpha, const T* x, T* y) {
    const double a = alpha[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = static_cast<T>(a * static_cast<double>(x[i]));
}

__global__ void __launch_bounds__(256)
k_add_f64(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] += src[i];
}

// ------------------------------------------------------- plan-time kernels

__global__ void __launch_bounds__(256)
k_validate_count(const int32_t* __restrict__ conn, int64_t n_items, int64_t n_nodes,
                 int32_t* __restrict__ cnt, int32_t* __restrict__ flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += stride) {
        const int32_t n = conn[i];
        if (n < 0 || (int64_t)n >= n_nodes)
            bad = 1;
        else if (cnt)
            atomicAdd(cnt + n, 1);
    }
    if (bad) atomicOr(flag, 1);
}

// One workgroup per element-pass workgroup: its node numbers are put in
// their home slots of an S-slot table; an insert that finds another node
// there is counted (any two distinct nodes of a workgroup that share a home
// slot give at least one such insert, whatever the order).
template <int S>
__global__ void __launch_bounds__(256)
k_table_check(const int32_t* __restrict__ conn, int64_t n_elems, int32_t k, int64_t span,
              uint32_t shift, int32_t* __restrict__ miss) {
    __shared__ int32_t key[S];
    for (int q = threadIdx.x; q < S; q += blockDim.x) key[q] = -1;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * span;
    const int64_t e1 = e0 + span < n_elems ? e0 + span : n_elems;
    int m = 0;
    for (int64_t q = e0 * k + threadIdx.x; q < e1 * k; q += blockDim.x) {
        const int32_t nd = conn[q];
        const int32_t old = atomicCAS(&key[agg_slot((uint32_t)nd, shift, (uint32_t)S)], -1, nd);
        m += (old != -1 && old != nd) ? 1 : 0;
    }
    if (m) atomicAdd(miss, m);
}

// Exclusive scan in three launches: per-chunk totals, a scan of the totals
// by one workgroup, then per-chunk local scans offset by the chunk prefix.
constexpr int kScanBS = 256;
constexpr int kScanIPT = 16;
constexpr int64_t kScanChunk = (int64_t)kScanBS * kScanIPT;

__device__ __forceinline__ int64_t block_exclusive_scan_i64(int64_t v, int64_t* lds,
                                                            int64_t* total) {
    // Hillis-Steele inside each wave, then across waves through LDS.
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    const int nw = blockDim.x >> 6;
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < nw; ++i) {
            int64_t t = lds[i];
            lds[i] = run;
            run += t;
        }
        lds[nw] = run;
    }
    __syncthreads();
    const int64_t r = x - v + lds[wid];
    *total = lds[nw];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanBS)
k_scan_chunk_totals(const int32_t* __restrict__ in, int64_t n, int64_t* __restrict__ totals) {
    __shared__ double lds[16];
    const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
    double s = 0.0;  // exact: totals are < 2^31
    for (int i = 0; i < kScanIPT; ++i) {
        const int64_t idx = c0 + (int64_t)i * kScanBS + threadIdx.x;
        if (idx < n) s += (double)in[idx];
    }
    s = block_sum<kScanBS>(s, lds);
    if (threadIdx.x == 0) totals[blockIdx.x] = (int64_t)s;
}

__global__ void __launch_bounds__(kScanBS)
k_scan_totals(int64_t* __restrict__ totals, int64_t nchunks) {
    __shared__ int64_t lds[kScanBS / 64 + 1];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nchunks; c0 += kScanBS) {
        const int64_t idx = c0 + threadIdx.x;
        const int64_t v = idx < nchunks ? totals[idx] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan_i64(v, lds, &tot);
        if (idx < nchunks) totals[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[nchunks] = carry;
}

__global__ void __launch_bounds__(kScanBS)
k_scan_chunk_apply(const int32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ prefix,
                   int32_t* __restrict__ out, int64_t nchunks) {
    __shared__ int64_t lds[kScanBS / 64 + 1];
    const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
    // Each thread scans kScanIPT consecutive items.
    int32_t vals[kScanIPT];
    int64_t local = 0;
    for (int i = 0; i < kScanIPT; ++i) {
        const int64_t idx = c0 + (int64_t)threadIdx.x * kScanIPT + i;
        vals[i] = idx < n ? in[idx] : 0;
        local += vals[i];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan_i64(local, lds, &tot) + prefix[blockIdx.x];
    for (int i = 0; i < kScanIPT; ++i) {
        const int64_t idx = c0 + (int64_t)threadIdx.x * kScanIPT + i;
        if (idx < n) out[idx] = (int32_t)run;
        run += vals[i];
    }
    if (blockIdx.x == nchunks - 1 && threadIdx.x == 0) out[n] = (int32_t)prefix[nchunks];
}

__global__ void __launch_bounds__(256)
k_csr_fill(const int32_t* __restrict__ conn, int64_t n_items, int32_t* __restrict__ cursor,
           int32_t* __restrict__ inc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += stride) {
        const int32_t pos = atomicAdd(cursor + conn[i], 1);
        inc[pos] = (int32_t)i;
    }
}

// Rows of the transposed connectivity are short (8 for a hex mesh); an
// insertion sort per node makes their order ascending, hence deterministic.
__global__ void __launch_bounds__(256)
k_csr_sort_rows(const int32_t* __restrict__ offs, int64_t n_nodes, int32_t* __restrict__ inc) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const int32_t p0 = offs[n], p1 = offs[n + 1];
    for (int32_t a = p0 + 1; a < p1; ++a) {
        const int32_t key = inc[a];
        int32_t b = a - 1;
        while (b >= p0 && inc[b] > key) {
            inc[b + 1] = inc[b];
            --b;
        }
        inc[b + 1] = key;
    }
}
inline unsigned stream_grid(int64_t n, int per_block, int cap = 4096) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_final_sum(const double* partials, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(1024), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_segmented_sum(const double* partials, const int64_t* seg, int64_t nseg,
                                double* out, hipStream_t s) {
    if (nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_segmented_sum, dim3((unsigned)nseg), dim3(256), 0, s, partials, seg,
                       nseg, out);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const int64_t head = std::min<int64_t>((int64_t)((16 - a % 16) % 16), (int64_t)bytes);
    const int64_t n16 = ((int64_t)bytes - head) / 16, tail = (int64_t)bytes - head - 16 * n16;
    hipLaunchKernelGGL(k_zero16, dim3(stream_grid(n16, 256, 1 << 20)), dim3(256), 0, s,
                       (uint8_t*)p, head, n16, tail);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(double* src, float* dst, int64_t n, int accumulate, int clear,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_f64_to_f32, dim3(stream_grid(n, 256 * 4, 8192)), dim3(256), 0, s, src,
                       dst, n, accumulate, clear, nullptr, (int64_t)0, nullptr);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32_sum(double* src, float* dst, int64_t n, int accumulate, int clear,
                                 const double* partials, int64_t np, double* f_out, hipStream_t s) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(stream_grid(n, 256 * 4, 8192)), dim3(256), 0, s, src,
                       dst, n, accumulate, clear, partials, np, f_out);
    return hipGetLastError();
}

hipError_t launch_scale(Dtype dt, int64_t n, const double* alpha, const void* x, void* y,
                        hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 g(stream_grid(n, 256 * 4, 8192));
    if (dt == F64)
        hipLaunchKernelGGL(k_scale<double>, g, dim3(256), 0, s, n, alpha,
                           static_cast<const double*>(x), static_cast<double*>(y));
    else
        hipLaunchKernelGGL(k_scale<float>, g, dim3(256), 0, s, n, alpha,
                           static_cast<const float*>(x), static_cast<float*>(y));
    return hipGetLastError();
}

hipError_t launch_add_f64(const double* src, double* dst, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_f64, dim3(stream_grid(n, 256 * 4, 8192)), dim3(256), 0, s, src, dst,
                       n);
    return hipGetLastError();
}

hipError_t launch_validate_count(const int32_t* conn, int64_t n_items, int64_t n_nodes,
                                 int32_t* cnt, int32_t* flag, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_count, dim3(stream_grid(n_items, 256 * 8, 8192)), dim3(256), 0,
                       s, conn, n_items, n_nodes, cnt, flag);
    return hipGetLastError();
}

hipError_t launch_table_check(const int32_t* conn, int64_t n_elems, int32_t k, int64_t span,
                              uint32_t shift, int slots, int32_t* miss, hipStream_t s) {
    if (n_elems == 0 || span <= 0) return hipSuccess;
    const int64_t nw = (n_elems + span - 1) / span;
    if (nw > 0x7fffffffLL) return hipErrorInvalidValue;
    if (slots == 2048)
        hipLaunchKernelGGL(k_table_check<2048>, dim3((unsigned)nw), dim3(256), 0, s, conn, n_elems,
                           k, span, shift, miss);
    else if (slots == 4096)
        hipLaunchKernelGGL(k_table_check<4096>, dim3((unsigned)nw), dim3(256), 0, s, conn, n_elems,
                           k, span, shift, miss);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int64_t scan_scratch_items(int64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int64_t* scratch,
                                 hipStream_t s) {
    const int64_t nchunks = (n + kScanChunk - 1) / kScanChunk;
    if (nchunks == 0) {
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(256), 0, s, (uint8_t*)out, (int64_t)4);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_chunk_totals, dim3((unsigned)nchunks), dim3(kScanBS), 0, s, in, n,
                       scratch);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBS), 0, s, scratch, nchunks);
    hipLaunchKernelGGL(k_scan_chunk_apply, dim3((unsigned)nchunks), dim3(kScanBS), 0, s, in, n,
                       scratch, out, nchunks);
    return hipGetLastError();
}

hipError_t launch_csr_fill_sort(const int32_t* conn, int64_t n_items, int64_t n_nodes,
                                const int32_t* offs, int32_t* cursor, int32_t* inc,
                                hipStream_t s) {
    if (n_nodes > 0) {
        hipError_t e = hipMemcpyAsync(cursor, offs, sizeof(int32_t) * (size_t)n_nodes,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    if (n_items > 0)
        hipLaunchKernelGGL(k_csr_fill, dim3(stream_grid(n_items, 256 * 8, 8192)), dim3(256), 0, s,
                           conn, n_items, cursor, inc);
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_csr_sort_rows, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0,
                           s, offs, n_nodes, inc);
    return hipGetLastError();
}

// Rows of conn, B and w copied into the order of a list of elements (the
// colour classes, class by class): out row r is element list[r].  One thread
// per (row, entry).
template <typename T>
__global__ void k_permute_rows(const int32_t* __restrict__ list, int64_t n, int32_t k,
                               const int32_t* __restrict__ conn, const T* __restrict__ B,
                               const T* __restrict__ w, int32_t* __restrict__ pconn,
                               T* __restrict__ pB, T* __restrict__ pw) {
    const int64_t items = n * k;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < items;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / k, j = q - r * k;
        const int64_t e = list[r];
        pconn[q] = conn[e * k + j];
        pB[q] = B[e * k + j];
        if (j == 0) pw[r] = w[e];
    }
}

hipError_t launch_permute_rows(const int32_t* list, int64_t n, int32_t k, const int32_t* conn,
                               const void* B, const void* w, bool f64, int32_t* pconn, void* pB,
                               void* pw, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned grid = stream_grid(n * k, 256, 1 << 16);
    if (f64)
        hipLaunchKernelGGL(k_permute_rows<double>, dim3(grid), dim3(256), 0, s, list, n, k, conn,
                           static_cast<const double*>(B), static_cast<const double*>(w), pconn,
                           static_cast<double*>(pB), static_cast<double*>(pw));
    else
        hipLaunchKernelGGL(k_permute_rows<float>, dim3(grid), dim3(256), 0, s, list, n, k, conn,
                           static_cast<const float*>(B), static_cast<const float*>(w), pconn,
                           static_cast<float*>(pB), static_cast<float*>(pw));
    return hipGetLastError();
}

// out[q] = B[idx[q]]: the coefficients of B in the order of a list of
// incidences (the transposed connectivity, node by node).
template <typename T>
__global__ void k_gather_entries(const int32_t* __restrict__ idx, int64_t n, const T* __restrict__ B,
                                 T* __restrict__ out) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        out[q] = B[idx[q]];
}

hipError_t launch_gather_entries(const int32_t* idx, int64_t n, const void* B, bool f64, void* out,
                                 hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned grid = stream_grid(n, 256, 1 << 16);
    if (f64)
        hipLaunchKernelGGL(k_gather_entries<double>, dim3(grid), dim3(256), 0, s, idx, n,
                           static_cast<const double*>(B), static_cast<double*>(out));
    else
        hipLaunchKernelGGL(k_gather_entries<float>, dim3(grid), dim3(256), 0, s, idx, n,
                           static_cast<const float*>(B), static_cast<float*>(out));
    return hipGetLastError();
}

}  // namespace pg
