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
               p.hash_shift, buffer_bytes<T>(m.n_nodes)};
    AggOf<AGG>* tab = nullptr;
    if constexpr (AGG > 0) tab = &agg;
    // LDS table clear before the gather for FP64 rows, after it for FP32
    // rows (measured: 0.5 us and 0.7 us faster respectively on 128^3).
    constexpr bool clear_early = !std::is_same<T, float>::value;
    const double tsum = elem_tile<T, K, MODE, EPT, AGG, clear_early>(
        a, (int64_t)lb * blockDim.x * EPT, n_items, 0, fb, tab);
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

// Node-parallel sum over the transposed connectivity: node n adds
// v_e * B[e, j] over its incidences in ascending (e, j) order.  B's
// coefficients are read in incidence order from `binc` (copied at bind), so
// they stream; the incidences are taken four at a time so that their loads
// are in flight together, the additions staying in order.
template <typename T, int K>
__global__ void __launch_bounds__(1024)
k_mesh_node_gather(int64_t n_nodes, int32_t k, const int32_t* __restrict__ offs,
                   const int32_t* __restrict__ inc, const double* __restrict__ v,
                   const T* __restrict__ binc, T* __restrict__ grad, int accumulate) {
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t n = (int64_t)lb * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const int32_t p0 = offs[n], p1 = offs[n + 1];
    double acc = 0.0;
    for (int32_t q = p0; q < p1; q += 4) {
        int32_t e[4];
        double b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool in = q + r < p1;
            const int32_t idx = in ? inc[q + r] : 0;
            e[r] = in ? (K > 0 ? idx / K : idx / k) : -1;
            b[r] = in ? to_f64(binc[q + r]) : 0.0;
        }
        double ve[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) ve[r] = e[r] >= 0 ? v[e[r]] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (e[r] >= 0) acc += ve[r] * b[r];
    }
    if (accumulate)
        grad[n] = static_cast<T>(to_f64(grad[n]) + acc);
    else
        grad[n] = static_cast<T>(acc);
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
                                   const void* binc, const double* v, void* grad, int accumulate,
                                   int block, hipStream_t s) {
    if (m.n_nodes == 0) return hipSuccess;
    const unsigned nb = (unsigned)((m.n_nodes + block - 1) / block);
    if (m.dtype == F64) {
        if (m.k == 8)
            hipLaunchKernelGGL((k_mesh_node_gather<double, 8>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const double*)binc, (double*)grad,
                               accumulate);
        else
            hipLaunchKernelGGL((k_mesh_node_gather<double, 0>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const double*)binc, (double*)grad,
                               accumulate);
    } else {
        if (m.k == 8)
            hipLaunchKernelGGL((k_mesh_node_gather<float, 8>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const float*)binc, (float*)grad,
                               accumulate);
        else
            hipLaunchKernelGGL((k_mesh_node_gather<float, 0>), dim3(nb), dim3(block), 0, s,
                               m.n_nodes, m.k, offs, inc, v, (const float*)binc, (float*)grad,
                               accumulate);
    }
    return hipGetLastError();
}

}  // namespace pg
