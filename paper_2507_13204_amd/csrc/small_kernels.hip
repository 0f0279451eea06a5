// Small single meshes in one launch per call.
//
// A call on a mesh of a few workgroups is bound by launch latency, and the
// multi-launch form spends three launches on a gradient (fill, element pass,
// final sum).  Here one launch does it all: the element work is the same as
// the element pass (rows, gather, psi, the LDS-combined atomic scatter), but
// the contributions go to a workspace buffer W that is zero between calls.
// Each workgroup makes its scatter and its partial of f visible device-wide
// and takes a ticket; the last workgroup to take one writes grad from W (or
// adds W into it), clears W for the next call, sums the partials in their
// fixed order into f and re-arms the ticket.  The grid is at most
// kSmallMaxBlocks workgroups, so the one device-scope fence per thread is
// cheap.  No workgroup waits for another.
#include "device_common.hpp"
#include "elem_tile.hpp"
#include "launch.hpp"

namespace pg {

namespace {

constexpr int kSmallU = 8;  // W entries a thread has in flight in the last workgroup

template <typename T, int K, int MODE, int AGG>
__global__ void __launch_bounds__(1024)
k_mesh_small(MeshView m, MeshPass p, SmallPass sp) {
    __shared__ double lds[16];
    __shared__ AggOf<AGG> agg;
    __shared__ int last;
    const int64_t bs = blockDim.x;
    const uint32_t lb = blockIdx.x;
    double fb = 1.0;
    if constexpr (has_rev(MODE)) fb = p.fbar ? p.fbar[0] : 1.0;
    TileArgs a{m.conn, m.B, m.w, p.x, p.xd, p.u_in, p.u_store, p.v_out, p.gacc, p.elist,
               p.hash_shift};
    AggOf<AGG>* tab = nullptr;
    if constexpr (AGG > 0) tab = &agg;
    const double tsum = elem_tile<T, K, MODE, 1, AGG>(a, (int64_t)lb * bs, m.n_elems, 0, fb, tab);
    if constexpr (has_rev(MODE)) __threadfence();  // this thread's atomics are visible
    double s = 0.0;
    if constexpr (has_sum(MODE)) s = block_sum_dyn(tsum, lds);
    if (threadIdx.x == 0) {
        if constexpr (has_sum(MODE)) p.partials[lb] = s;
        __threadfence();  // the workgroup's partial and scatter before its ticket
        last = atomicAdd(sp.ticket, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every workgroup's scatter and partial are visible
    if constexpr (has_rev(MODE)) {
        T* __restrict__ g = static_cast<T*>(sp.grad);
        double* __restrict__ W = p.gacc;
        const int64_t n = m.n_nodes;
        for (int64_t q = threadIdx.x; q < n; q += kSmallU * bs) {
            double v[kSmallU];
#pragma unroll
            for (int u = 0; u < kSmallU; ++u) v[u] = q + u * bs < n ? W[q + u * bs] : 0.0;
#pragma unroll
            for (int u = 0; u < kSmallU; ++u) {
                const int64_t i = q + u * bs;
                if (i < n) {
                    W[i] = 0.0;
                    g[i] = sp.accumulate ? static_cast<T>(to_f64(g[i]) + v[u]) : static_cast<T>(v[u]);
                }
            }
        }
    }
    if constexpr (has_sum(MODE)) {
        double v = 0.0;
        for (int q = threadIdx.x; q < (int)gridDim.x; q += (int)bs) v += p.partials[q];
        v = block_sum_dyn(v, lds);
        if (threadIdx.x == 0 && sp.f_out) sp.f_out[0] = v;
    }
    if (threadIdx.x == 0) *sp.ticket = 0;
}

template <typename T, int K, int MODE>
hipError_t launch_small_t(const MeshView& m, const MeshPass& p, const SmallPass& sp, hipStream_t s) {
    const dim3 grid((unsigned)mesh_blocks(m.n_elems, p.block, 1)), block(p.block);
    const bool agg = is_atomic(MODE) && p.combine && (int64_t)p.block * K <= 2 * kAggSlots;
    if constexpr (is_atomic(MODE)) {
        if (agg && p.agg_slots == kAggSlotsSmall)
            PG_LAUNCH((k_mesh_small<T, K, MODE, kAggSlotsSmall>), grid, block, 0, s, m, p, sp);
        else if (agg)
            PG_LAUNCH((k_mesh_small<T, K, MODE, kAggSlots>), grid, block, 0, s, m, p, sp);
        else
            PG_LAUNCH((k_mesh_small<T, K, MODE, 0>), grid, block, 0, s, m, p, sp);
    } else {
        PG_LAUNCH((k_mesh_small<T, K, MODE, 0>), grid, block, 0, s, m, p, sp);
    }
    return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_small_mode(const MeshView& m, MeshMode mode, const MeshPass& p,
                             const SmallPass& sp, hipStream_t s) {
    switch (mode) {
        case M_PRIMAL: return launch_small_t<T, K, M_PRIMAL>(m, p, sp, s);
        case M_GRAD_ATOMIC: return launch_small_t<T, K, M_GRAD_ATOMIC>(m, p, sp, s);
        case M_ADJ_ATOMIC: return launch_small_t<T, K, M_ADJ_ATOMIC>(m, p, sp, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_small_k(const MeshView& m, MeshMode mode, const MeshPass& p, const SmallPass& sp,
                          hipStream_t s) {
    switch (m.k) {
        case 2: return launch_small_mode<T, 2>(m, mode, p, sp, s);
        case 4: return launch_small_mode<T, 4>(m, mode, p, sp, s);
        case 8: return launch_small_mode<T, 8>(m, mode, p, sp, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool mesh_small_eligible(const MeshView& m, int block) {
    return (m.k == 2 || m.k == 4 || m.k == 8) && m.n_elems > 0 &&
           mesh_blocks(m.n_elems, block, 1) <= kSmallMaxBlocks && m.n_nodes <= kSmallMaxNodes;
}

hipError_t launch_mesh_small(const MeshView& m, MeshMode mode, const MeshPass& p,
                             const SmallPass& sp, hipStream_t s) {
    if (!mesh_small_eligible(m, p.block) || !sp.ticket) return hipErrorInvalidValue;
    if (mode != M_PRIMAL && (!p.gacc || !sp.grad)) return hipErrorInvalidValue;
    return m.dtype == F64 ? launch_small_k<double>(m, mode, p, sp, s)
                          : launch_small_k<float>(m, mode, p, sp, s);
}

}  // namespace pg
