// Small single meshes in one launch per call.
//
// A call on a mesh of a few workgroups is bound by launch latency, and the
// multi-launch form spends three launches on a gradient (fill, element pass,
// final sum).  Here one launch does it all: the element work is the same as
// the element pass (rows, gather, psi, the LDS-combined atomic scatter), but
// the contributions go to a workspace buffer W that is zero between calls.
// Once a workgroup's scatter is visible device-wide it counts itself done on
// each node range it touched (the plan lists them); the last workgroup done
// on a range writes grad there from W (or adds W into it) and clears W there
// for the next call, so that work is spread over the grid instead of left to
// one workgroup.  Each workgroup's partial of f goes the same way through a
// single ticket: the last workgroup sums the partials in their fixed order.
// The grid is at most kSmallMaxBlocks workgroups, so the device-scope fences
// are cheap.  No workgroup waits for another.
#include "device_common.hpp"
#include "elem_tile.hpp"
#include "launch.hpp"

namespace pg {

namespace {

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
               p.hash_shift, buffer_bytes<T>(m.n_nodes)};
    AggOf<AGG>* tab = nullptr;
    if constexpr (AGG > 0) tab = &agg;
    const double tsum = elem_tile<T, K, MODE, 1, AGG>(a, (int64_t)lb * bs, m.n_elems, 0, fb, tab);
    // Publication costs one device-scope fence per workgroup, not one per
    // wave: every wave first waits until its own atomics are performed, then
    // wave 0 (after the barrier) writes the partial, releases at device scope
    // and takes the counts.  The L2 write-back of its release covers the
    // whole workgroup's completed atomics.
    if constexpr (is_atomic(MODE)) __builtin_amdgcn_s_waitcnt(0);
    double s = 0.0;
    if constexpr (has_sum(MODE)) s = block_sum_dyn(tsum, lds);
    __syncthreads();
    static_assert(kSmallMaxRanges < kWave - 1, "the ticket lane must not take a range");
    __shared__ int fin[kSmallMaxRanges];
    __shared__ int any_fin;
    int r0 = 0, nr = 0;
    if constexpr (is_atomic(MODE)) {
        r0 = sp.wg_off[lb];
        nr = sp.wg_off[lb + 1] - r0;
    }
    if (threadIdx.x < kWave) {
        if constexpr (has_sum(MODE))
            if (threadIdx.x == 0) p.partials[lb] = s;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // The ticket (last lane; a workgroup has at most kSmallMaxRanges < 63
        // ranges) and the range counts (lanes 0 .. nr-1) are taken in the same
        // batch of atomics, so the workgroup waits for one round trip, not two.
        int ticket = 0;
        if constexpr (has_sum(MODE))
            if (threadIdx.x == kWave - 1) ticket = atomicAdd(sp.ticket, 1);
        if constexpr (is_atomic(MODE)) {
            bool mine = false;
            if ((int)threadIdx.x < nr) {
                const int r = sp.wg_list[r0 + threadIdx.x];
                mine = atomicAdd(sp.range_done + r, 1) == sp.range_need[r] - 1;
                fin[threadIdx.x] = mine;
            }
            const bool any = __any(mine);
            if (threadIdx.x == 0) any_fin = any;
        }
        if constexpr (has_sum(MODE))
            if (threadIdx.x == kWave - 1) last = ticket == (int)gridDim.x - 1;
    }
    __syncthreads();
    if constexpr (is_atomic(MODE)) {
        if (any_fin) {
            // Last on some ranges: every scatter into them is visible after
            // wave 0's acquire (the caches it invalidates serve all waves).
            if (threadIdx.x < kWave) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            T* __restrict__ g = static_cast<T*>(sp.grad);
            double* __restrict__ W = p.gacc;
            for (int i = 0; i < nr; ++i) {
                if (!fin[i]) continue;
                const int r = sp.wg_list[r0 + i];
                const int64_t n0 = (int64_t)r * kSmallRange;
                const int64_t n1 = n0 + kSmallRange < m.n_nodes ? n0 + kSmallRange : m.n_nodes;
                for (int64_t q = n0 + threadIdx.x; q < n1; q += bs) {
                    const double v = W[q];
                    W[q] = 0.0;
                    g[q] = sp.accumulate ? static_cast<T>(to_f64(g[q]) + v) : static_cast<T>(v);
                }
                if (threadIdx.x == 0) sp.range_done[r] = 0;
            }
        }
    }
    if constexpr (has_sum(MODE)) {
        if (last) {
            if (threadIdx.x < kWave) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            double v = 0.0;
            for (int q = threadIdx.x; q < (int)gridDim.x; q += (int)bs) v += p.partials[q];
            v = block_sum_dyn(v, lds);
            if (threadIdx.x == 0) {
                if (sp.f_out) sp.f_out[0] = v;
                *sp.ticket = 0;
            }
        }
    }
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
        case M_HVP: return launch_small_t<T, K, M_HVP>(m, p, sp, s);
        case M_JVP: return launch_small_t<T, K, M_JVP>(m, p, sp, s);
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
    const bool scatter = mode == M_GRAD_ATOMIC || mode == M_ADJ_ATOMIC || mode == M_HVP;
    if (scatter && (!p.gacc || !sp.grad || !sp.range_done || !sp.range_need || !sp.wg_off ||
                    !sp.wg_list))
        return hipErrorInvalidValue;
    return m.dtype == F64 ? launch_small_k<double>(m, mode, p, sp, s)
                          : launch_small_k<float>(m, mode, p, sp, s);
}

}  // namespace pg
