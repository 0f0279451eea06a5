// Element-connectivity objective and its reverse pass on gfx950.
//
//   forward (section 4's gather + nonlinearity + parallel_sum, generalised):
//     u_e = sum_j B[e,j] x[conn[e,j]],  t_e = w_e psi(u_e),  f = sum_e t_e
//   reverse (seed fbar, broadcast to every t_e, local derivative, transposed
//   read of x):
//     v_e = fbar w_e psi'(u_e),  xbar[conn[e,j]] += v_e B[e,j]
//
// One thread owns EPT elements.  Loads are issued for all of them before any
// arithmetic (conn and B rows as 16-byte vectors, then the x gathers) so each
// wave keeps several kilobytes in flight; f is reduced per workgroup in a
// fixed butterfly order and the per-workgroup partials are summed by one
// workgroup afterwards, so f is bitwise repeatable.  The reverse scatter is
// either a hardware FP64 atomic add (the race case of section 3.3: the write
// index is itself a view entry), a plain read-add-write inside one colour
// class, or deferred to the node-parallel gather below.
#include <type_traits>

#include "elem_tile.hpp"

namespace pg {

namespace {

// Compile-time K: every row lives in registers.
template <typename T, int K, int MODE, int EPT, int AGG>
__global__ void __launch_bounds__(1024)
k_mesh_elem(MeshView m, MeshPass p) {
    __shared__ double lds[16];
    __shared__ AggOf<AGG> agg;
    const int64_t n_items = p.elist ? p.elist_n : m.n_elems;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    double fb = 1.0;
    if constexpr (has_rev(MODE)) fb = p.fbar ? p.fbar[0] : 1.0;
    TileArgs a{m.conn, m.B, m.w, p.x, p.xd, p.u_in, p.u_store, p.v_out, p.gacc, p.elist,
               p.hash_shift};
    AggOf<AGG>* tab = nullptr;
    if constexpr (AGG > 0) tab = &agg;
    const double tsum = elem_tile<T, K, MODE, EPT, AGG>(a, (int64_t)lb * blockDim.x * EPT, n_items,
                                                        0, fb, tab);
    if constexpr (has_sum(MODE)) {
        const double s = block_sum_dyn(tsum, lds);
        if (threadIdx.x == 0) p.partials[p.partial_base + lb] = s;
    }
}

// Runtime k (any 1 <= k <= 32): rows are streamed twice (forward, reverse)
// through the cache instead of held in registers.
template <typename T, int MODE>
__global__ void __launch_bounds__(1024)
k_mesh_elem_dyn(MeshView m, MeshPass p) {
    __shared__ double lds[16];
    const T* __restrict__ B = static_cast<const T*>(m.B);
    const T* __restrict__ W = static_cast<const T*>(m.w);
    const T* __restrict__ X = static_cast<const T*>(p.x);
    const T* __restrict__ XD = static_cast<const T*>(p.xd);
    const int32_t* __restrict__ conn = m.conn;
    const int k = m.k;
    const int64_t n_items = p.elist ? p.elist_n : m.n_elems;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t idx = (int64_t)lb * blockDim.x + threadIdx.x;
    double fb = 1.0;
    if constexpr (has_rev(MODE)) fb = p.fbar ? p.fbar[0] : 1.0;
    double tsum = 0.0;
    if (idx < n_items) {
        const int64_t e = p.elist ? (int64_t)p.elist[idx] : idx;
        double u = 0.0;
        if (p.u_in) {
            u = p.u_in[e];
        } else {
            for (int j = 0; j < k; ++j) u += to_f64(B[e * k + j]) * to_f64(X[conn[e * k + j]]);
            if (p.u_store) p.u_store[e] = u;
        }
        const double s2 = u * u, wd = to_f64(W[e]);
        if constexpr (has_obj(MODE)) tsum = wd * psi_from_sq(s2);
        double v = 0.0;
        if constexpr (has_rev(MODE)) v = fb * wd * dpsi_from(u, s2);
        if constexpr (MODE == M_HVP || MODE == M_JVP) {
            double q = 0.0;
            for (int j = 0; j < k; ++j) q += to_f64(B[e * k + j]) * to_f64(XD[conn[e * k + j]]);
            if constexpr (MODE == M_HVP) v = wd * ddpsi_from_sq(s2) * q;
            if constexpr (MODE == M_JVP) tsum = wd * dpsi_from(u, s2) * q;
        }
        if constexpr (writes_v(MODE)) p.v_out[e] = v;
        if constexpr (is_atomic(MODE)) {
            for (int j = 0; j < k; ++j)
                atomic_add_f64(p.gacc + conn[e * k + j], v * to_f64(B[e * k + j]));
        }
        if constexpr (is_colour(MODE)) {
            for (int j = 0; j < k; ++j) {
                double* g = p.gacc + conn[e * k + j];
                *g = *g + v * to_f64(B[e * k + j]);
            }
        }
    }
    if constexpr (has_sum(MODE)) {
        const double s = block_sum_dyn(tsum, lds);
        if (threadIdx.x == 0) p.partials[p.partial_base + lb] = s;
    }
}

template <typename T, int K>
__global__ void __launch_bounds__(1024)
k_mesh_node_gather(int64_t n_nodes, int32_t k, const int32_t* __restrict__ offs,
                   const int32_t* __restrict__ inc, const double* __restrict__ v,
                   const T* __restrict__ B, T* __restrict__ grad, int accumulate) {
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t n = (int64_t)lb * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const int32_t p0 = offs[n], p1 = offs[n + 1];
    double acc = 0.0;
    for (int32_t q = p0; q < p1; ++q) {
        const int32_t idx = inc[q];
        const int32_t e = K > 0 ? idx / K : idx / k;
        acc += v[e] * to_f64(B[idx]);
    }
    if (accumulate)
        grad[n] = static_cast<T>(to_f64(grad[n]) + acc);
    else
        grad[n] = static_cast<T>(acc);
}

__global__ void __launch_bounds__(1024)
k_final_sum(const double* __restrict__ partials, int64_t n, double* __restrict__ out) {
    __shared__ double lds[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
    s = block_sum_dyn(s, lds);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void __launch_bounds__(256)
k_segmented_sum(const double* __restrict__ partials, const int64_t* __restrict__ seg,
                int64_t nseg, double* __restrict__ out) {
    __shared__ double lds[16];
    const int64_t i = blockIdx.x;
    if (i >= nseg) return;
    double s = 0.0;
    for (int64_t q = seg[i] + threadIdx.x; q < seg[i + 1]; q += blockDim.x) s += partials[q];
    s = block_sum_dyn(s, lds);
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

__global__ void __launch_bounds__(256)
k_f64_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n, int accumulate) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = accumulate ? static_cast<float>((double)dst[i] + src[i]) : static_cast<float>(src[i]);
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

template <typename T, int K, int MODE, int EPT>
hipError_t launch_elem_t(const MeshView& m, const MeshPass& p, hipStream_t s) {
    const int64_t n_items = p.elist ? p.elist_n : m.n_elems;
    const int64_t nb = mesh_blocks(n_items, p.block, EPT);
    if (nb == 0) return hipSuccess;
    // Combine in LDS when the workgroup's contributions fit the table twice over
    // at worst (all distinct); meshes with locality fill it far less.  The
    // plan picks the table size (p.agg_slots) from simulated workgroups.
    const bool agg = is_atomic(MODE) && p.combine && (int64_t)p.block * EPT * K <= 2 * kAggSlots;
    if (agg && p.agg_slots == kAggSlotsSmall && EPT == 1)
        PG_LAUNCH((k_mesh_elem<T, K, MODE, EPT, kAggSlotsSmall>), dim3((unsigned)nb), dim3(p.block),
                  0, s, m, p);
    else if (agg)
        PG_LAUNCH((k_mesh_elem<T, K, MODE, EPT, kAggSlots>), dim3((unsigned)nb), dim3(p.block), 0,
                  s, m, p);
    else
        PG_LAUNCH((k_mesh_elem<T, K, MODE, EPT, 0>), dim3((unsigned)nb), dim3(p.block), 0, s, m, p);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_elem_dyn_t(const MeshView& m, const MeshPass& p, hipStream_t s) {
    const int64_t n_items = p.elist ? p.elist_n : m.n_elems;
    const int64_t nb = mesh_blocks(n_items, p.block, 1);
    if (nb == 0) return hipSuccess;
    PG_LAUNCH((k_mesh_elem_dyn<T, MODE>), dim3((unsigned)nb), dim3(p.block), 0, s, m, p);
    return hipGetLastError();
}

template <typename T, int K, int MODE>
hipError_t launch_elem_ept(const MeshView& m, const MeshPass& p, hipStream_t s) {
    switch (p.ept) {
        case 1: return launch_elem_t<T, K, MODE, 1>(m, p, s);
        case 2: return launch_elem_t<T, K, MODE, 2>(m, p, s);
        case 4: return launch_elem_t<T, K, MODE, 4>(m, p, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODE>
hipError_t launch_elem_k(const MeshView& m, const MeshPass& p, hipStream_t s) {
    switch (m.k) {
        case 8: return launch_elem_ept<T, 8, MODE>(m, p, s);
        case 2: return launch_elem_ept<T, 2, MODE>(m, p, s);
        case 4: return launch_elem_ept<T, 4, MODE>(m, p, s);
        default: {
            MeshPass q = p;
            q.ept = 1;
            return launch_elem_dyn_t<T, MODE>(m, q, s);
        }
    }
}

template <typename T>
hipError_t launch_elem_mode(const MeshView& m, MeshMode mode, const MeshPass& p, hipStream_t s) {
    switch (mode) {
        case M_PRIMAL: return launch_elem_k<T, M_PRIMAL>(m, p, s);
        case M_GRAD_ATOMIC: return launch_elem_k<T, M_GRAD_ATOMIC>(m, p, s);
        case M_GRAD_V: return launch_elem_k<T, M_GRAD_V>(m, p, s);
        case M_ADJ_ATOMIC: return launch_elem_k<T, M_ADJ_ATOMIC>(m, p, s);
        case M_ADJ_V: return launch_elem_k<T, M_ADJ_V>(m, p, s);
        case M_HVP: return launch_elem_k<T, M_HVP>(m, p, s);
        case M_GRAD_COLOUR: return launch_elem_k<T, M_GRAD_COLOUR>(m, p, s);
        case M_ADJ_COLOUR: return launch_elem_k<T, M_ADJ_COLOUR>(m, p, s);
        case M_JVP: return launch_elem_k<T, M_JVP>(m, p, s);
    }
    return hipErrorInvalidValue;
}

inline unsigned stream_grid(int64_t n, int per_block, int cap = 4096) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

LaunchEvents& armed_launch_events() {
    thread_local LaunchEvents ev;
    return ev;
}

int64_t mesh_blocks(int64_t n_items, int block, int ept) {
    const int64_t per = (int64_t)block * ept;
    return per > 0 ? (n_items + per - 1) / per : 0;
}

hipError_t launch_mesh_elem(const MeshView& m, MeshMode mode, const MeshPass& p, hipStream_t s) {
    if (p.block <= 0 || p.block > 1024 || p.block % 64) return hipErrorInvalidValue;
    return m.dtype == F64 ? launch_elem_mode<double>(m, mode, p, s)
                          : launch_elem_mode<float>(m, mode, p, s);
}

hipError_t launch_mesh_node_gather(const MeshView& m, const int32_t* offs, const int32_t* inc,
                                   const double* v, void* grad, int accumulate, int block,
                                   hipStream_t s) {
    if (m.n_nodes == 0) return hipSuccess;
    const unsigned nb = (unsigned)((m.n_nodes + block - 1) / block);
    if (m.dtype == F64) {
        if (m.k == 8)
            hipLaunchKernelGGL((k_mesh_node_gather<double, 8>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const double*)m.B, (double*)grad,
                               accumulate);
        else
            hipLaunchKernelGGL((k_mesh_node_gather<double, 0>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const double*)m.B, (double*)grad,
                               accumulate);
    } else {
        if (m.k == 8)
            hipLaunchKernelGGL((k_mesh_node_gather<float, 8>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const float*)m.B, (float*)grad,
                               accumulate);
        else
            hipLaunchKernelGGL((k_mesh_node_gather<float, 0>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const float*)m.B, (float*)grad,
                               accumulate);
    }
    return hipGetLastError();
}

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

hipError_t launch_f64_to_f32(const double* src, float* dst, int64_t n, int accumulate,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_f64_to_f32, dim3(stream_grid(n, 256 * 4, 8192)), dim3(256), 0, s, src,
                       dst, n, accumulate);
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

}  // namespace pg
