// Deterministic adjoint scatter in two fixed-order levels (no atomics).
//
// Level 1, one workgroup per tile of consecutive elements: each thread
// writes its element's k contributions v_e B[e, j] into LDS; then, for every
// node the tile touches (its "local nodes", known from the plan), one thread
// adds that node's contributions from LDS in ascending (element, corner)
// order and writes the tile's partial for the node to a staging array.
// Level 2, one thread per node: the node's partials from the tiles that touch
// it are added in ascending tile order, overwriting (or adding to) grad.
// Every sum has a fixed order, so the gradient is bitwise repeatable; the
// staging writes are coalesced and no zero fill of grad is needed.  This is
// the conclusion's "reschedule the reverse threads" remedy applied at the
// workgroup level, with the workgroup-local reschedule done in LDS.
//
// Level 1 has two forms.  The general one reads, with the element rows, the
// tile's local incidence lists built at bind.  The corner-round form serves
// connectivities the plan has checked at bind: inside every tile no two
// elements put the same node at the same corner, and one hash of the node
// number gives the tile's distinct nodes distinct LDS slots.  Each node's
// partial is then built in k rounds, round j adding every element's corner-j
// contribution with a plain read-add-write (no two threads of a round touch
// one slot), a barrier between rounds: the additions to a slot come in
// ascending corner order, the same on every run, and no per-incidence data is
// read.  The partials are stored at stage[tile * slots + slot]; the plan lists
// each node's positions in ascending tile order for level 2.
#include "device_common.hpp"
#include "elem_tile.hpp"
#include "launch.hpp"

namespace pg {

namespace {

// The tile's local-node offsets, tile-relative, as 16-byte chunks: at most
// two chunks per thread for k <= 8 (nl + 1 <= tile * k + 1 entries).
struct OffChunks {
    typedef short v8 __attribute__((ext_vector_type(8)));
    v8 c[2];
};

// OBJ: also the objective partial per tile.  K > 0: row length known at
// compile time (rows in registers, vector loads); K == 0: runtime m.k.
// The tile's positions and offsets are loaded first, with the element rows,
// and land in LDS beside the contributions, so the per-node sums below touch
// LDS only.
template <typename T, int K, bool OBJ>
__global__ void __launch_bounds__(1024)
k_mesh_tiled(MeshView m, MeshPass p, TiledView tv) {
    extern __shared__ double c_lds[];
    __shared__ double lds[16];
    const T* __restrict__ B = static_cast<const T*>(m.B);
    const T* __restrict__ W = static_cast<const T*>(m.w);
    const T* __restrict__ X = static_cast<const T*>(p.x);
    const int k = K > 0 ? K : m.k;
    const int cap = tv.tile * k;
    int16_t* li_lds = reinterpret_cast<int16_t*>(c_lds + cap);
    int16_t* lo_lds = li_lds + cap;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t e0 = t * blockDim.x, e = e0 + threadIdx.x;
    const bool ok = e < m.n_elems;
    const int64_t sb = tv.tbase[t];
    const int nl = (int)(tv.tbase[t + 1] - sb);
    const int16_t* __restrict__ li = tv.lidx + e0 * k;
    const int16_t* __restrict__ lo = tv.loff + t * (int64_t)tv.lstride;
    const double fb = p.fbar ? p.fbar[0] : 1.0;
    double tsum = 0.0;
    if constexpr (K > 0) {
        typedef short vk __attribute__((ext_vector_type(K)));
        static_assert(K <= 8, "two offset chunks per thread cover tile * K + 1 entries for K <= 8");
        vk pos{};
        if (ok) pos = *reinterpret_cast<const vk*>(li + (int64_t)threadIdx.x * K);
        OffChunks oc;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int c = (int)threadIdx.x + r * (int)blockDim.x;
            if (c * 8 <= nl) oc.c[r] = *reinterpret_cast<const OffChunks::v8*>(lo + c * 8);
        }
        int32_t cr[K];
        T br[K];
        double u = 0.0, wd = 0.0;
        if (ok) {
            load_conn_row<T, K>(m.conn, e, cr);
            load_b_row<K>(B, e, br);
            wd = to_f64(W[e]);
            if (p.u_in) {
                u = p.u_in[e];
            } else {
                T xv[K];
#pragma unroll
                for (int j = 0; j < K; ++j) xv[j] = X[cr[j]];
#pragma unroll
                for (int j = 0; j < K; ++j) u += to_f64(br[j]) * to_f64(xv[j]);
            }
        }
        const double s2 = u * u;
        if constexpr (OBJ) tsum = wd * psi_from_sq(s2);
        const double v = fb * wd * dpsi_from(u, s2);
#pragma unroll
        for (int j = 0; j < K; ++j) c_lds[threadIdx.x * K + j] = ok ? v * to_f64(br[j]) : 0.0;
        if (ok) *reinterpret_cast<vk*>(li_lds + threadIdx.x * K) = pos;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int c = (int)threadIdx.x + r * (int)blockDim.x;
            if (c * 8 <= nl) *reinterpret_cast<OffChunks::v8*>(lo_lds + c * 8) = oc.c[r];
        }
    } else {
        const int cnt = (int)((m.n_elems - e0 < (int64_t)blockDim.x ? m.n_elems - e0 : blockDim.x) * k);
        for (int q = threadIdx.x; q < cnt; q += blockDim.x) li_lds[q] = li[q];
        for (int q = threadIdx.x; q <= nl; q += blockDim.x) lo_lds[q] = lo[q];
        double u = 0.0, wd = 0.0;
        if (ok) {
            wd = to_f64(W[e]);
            if (p.u_in) {
                u = p.u_in[e];
            } else {
                for (int j = 0; j < k; ++j) u += to_f64(B[e * k + j]) * to_f64(X[m.conn[e * k + j]]);
            }
        }
        const double s2 = u * u;
        if constexpr (OBJ) tsum = wd * psi_from_sq(s2);
        const double v = fb * wd * dpsi_from(u, s2);
        for (int j = 0; j < k; ++j) c_lds[threadIdx.x * k + j] = ok ? v * to_f64(B[e * k + j]) : 0.0;
    }
    __syncthreads();
    // The tile's local nodes: partial sums in ascending (element, corner) order.
    for (int l = threadIdx.x; l < nl; l += blockDim.x) {
        double s = 0.0;
        const int q1 = lo_lds[l + 1];
        for (int q = lo_lds[l]; q < q1; ++q) s += c_lds[li_lds[q]];
        tv.stage[sb + l] = s;
    }
    if constexpr (OBJ) {
        const double s = block_sum_dyn(tsum, lds);
        if (threadIdx.x == 0) p.partials[t] = s;
    }
}

// Corner-round level 1 (see the header): S direct-mapped slots per tile,
// slot(n) = (n + (n >> 12) * shift) mod S, collision-free in every tile (the
// plan checked it).
template <int S>
struct RoundTable {
    int32_t key[S];
    double val[S];
};

template <typename T, int K, bool OBJ, int S>
__global__ void __launch_bounds__(512)
k_mesh_tiled_rounds(MeshView m, MeshPass p, TiledView tv) {
    __shared__ RoundTable<S> tab;
    __shared__ double lds[16];
    const T* __restrict__ B = static_cast<const T*>(m.B);
    const T* __restrict__ W = static_cast<const T*>(m.w);
    const T* __restrict__ X = static_cast<const T*>(p.x);
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t e = t * blockDim.x + threadIdx.x;
    const bool ok = e < m.n_elems;
    const double fb = p.fbar ? p.fbar[0] : 1.0;
    const uint32_t shift = tv.round_shift;
    // Lanes past the last element read its rows (no tile starts past it) and
    // add nothing: the loads and the gather need no branch, so the gather is
    // issued once conn has arrived.  The slot table is cleared while the
    // gather is in flight.  Only the adjoint (no objective) can be handed
    // stored forward values.
    const int64_t ec = ok ? e : m.n_elems - 1;
    int32_t cr[K];
    T br[K];
    load_conn_row<T, K>(m.conn, ec, cr);
    load_b_row<K>(B, ec, br);
    const double wd = to_f64(W[ec]);
    double u = 0.0;
    bool stored = false;
    if constexpr (!OBJ) stored = p.u_in != nullptr;
    if (stored) {
        u = p.u_in[ec];
        for (int q = threadIdx.x; q < S; q += blockDim.x) {
            tab.key[q] = -1;
            tab.val[q] = 0.0;
        }
    } else {
        T xv[K];
#pragma unroll
        for (int j = 0; j < K; ++j) xv[j] = X[cr[j]];
        for (int q = threadIdx.x; q < S; q += blockDim.x) {
            tab.key[q] = -1;
            tab.val[q] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) u += to_f64(br[j]) * to_f64(xv[j]);
    }
    const double s2 = u * u;
    double tsum = 0.0;
    if constexpr (OBJ) tsum = ok ? wd * psi_from_sq(s2) : 0.0;
    const double v = ok ? fb * wd * dpsi_from(u, s2) : 0.0;
    __syncthreads();  // the table is clear
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (ok) {
            const uint32_t n = (uint32_t)cr[j];
            const uint32_t sl = (n + (n >> 12) * shift) & (uint32_t)(S - 1);
            tab.val[sl] += v * to_f64(br[j]);
            tab.key[sl] = cr[j];
        }
        __syncthreads();
    }
    double* __restrict__ st = tv.stage + t * S;
    for (int q = threadIdx.x; q < S; q += blockDim.x)
        if (tab.key[q] >= 0) st[q] = tab.val[q];
    if constexpr (OBJ) {
        const double sm = block_sum_dyn(tsum, lds);
        if (threadIdx.x == 0) p.partials[t] = sm;
    }
}

// Slots are taken four at a time so that their loads are in flight together;
// the additions stay in ascending slot order.
template <typename T>
__global__ void __launch_bounds__(256)
k_node_tiled(int64_t n_nodes, const int32_t* __restrict__ noff, const int32_t* __restrict__ npos,
             const double* __restrict__ stage, T* __restrict__ grad, int accumulate) {
    const int64_t n = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const int32_t q0 = noff[n], q1 = noff[n + 1];
    double s = 0.0;
    for (int32_t q = q0; q < q1; q += 4) {
        int32_t pp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) pp[r] = q + r < q1 ? npos[q + r] : -1;
        double v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = pp[r] >= 0 ? stage[pp[r]] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (pp[r] >= 0) s += v[r];
    }
    grad[n] = accumulate ? static_cast<T>(to_f64(grad[n]) + s) : static_cast<T>(s);
}

template <typename T, bool OBJ, int S>
hipError_t launch_rounds_k(const MeshView& m, const MeshPass& p, const TiledView& tv,
                           hipStream_t s) {
    const dim3 grid((unsigned)tv.n_tiles), block(tv.tile);
    switch (m.k) {
        case 2: PG_LAUNCH((k_mesh_tiled_rounds<T, 2, OBJ, S>), grid, block, 0, s, m, p, tv); break;
        case 4: PG_LAUNCH((k_mesh_tiled_rounds<T, 4, OBJ, S>), grid, block, 0, s, m, p, tv); break;
        case 8: PG_LAUNCH((k_mesh_tiled_rounds<T, 8, OBJ, S>), grid, block, 0, s, m, p, tv); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool OBJ>
hipError_t launch_tiled_t(const MeshView& m, const MeshPass& p, const TiledView& tv, hipStream_t s) {
    if (tv.round_slots == 2048) return launch_rounds_k<T, OBJ, 2048>(m, p, tv, s);
    if (tv.round_slots == 4096) return launch_rounds_k<T, OBJ, 4096>(m, p, tv, s);
    if (tv.round_slots != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)tv.n_tiles), block(tv.tile);
    const size_t shmem = tiled_lds_bytes(tv.tile, m.k);
    switch (m.k) {
        case 2: PG_LAUNCH((k_mesh_tiled<T, 2, OBJ>), grid, block, shmem, s, m, p, tv); break;
        case 4: PG_LAUNCH((k_mesh_tiled<T, 4, OBJ>), grid, block, shmem, s, m, p, tv); break;
        case 8: PG_LAUNCH((k_mesh_tiled<T, 8, OBJ>), grid, block, shmem, s, m, p, tv); break;
        default: PG_LAUNCH((k_mesh_tiled<T, 0, OBJ>), grid, block, shmem, s, m, p, tv); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t tiled_lds_bytes(int tile, int32_t k) {
    const size_t cap = (size_t)tile * (size_t)k;
    return sizeof(double) * cap + sizeof(int16_t) * cap + sizeof(int16_t) * (cap + 8);
}

int tiled_tile_elems(int block, int32_t k) {
    // The LDS holds tile * k doubles (at most 32 KiB) with their int16
    // positions and offsets (tile * k <= 4096 for k <= 32).
    int t = (4096 / k) / 64 * 64;
    if (t < 64) t = 64;
    return block < t ? block : t;
}

hipError_t launch_mesh_tiled(const MeshView& m, const MeshPass& p, const TiledView& tv, bool obj,
                             hipStream_t s) {
    if (tv.n_tiles == 0) return hipSuccess;
    if (m.dtype == F64)
        return obj ? launch_tiled_t<double, true>(m, p, tv, s) : launch_tiled_t<double, false>(m, p, tv, s);
    return obj ? launch_tiled_t<float, true>(m, p, tv, s) : launch_tiled_t<float, false>(m, p, tv, s);
}

hipError_t launch_node_tiled(const MeshView& m, const TiledView& tv, void* grad, int accumulate,
                             hipStream_t s) {
    if (m.n_nodes == 0) return hipSuccess;
    const dim3 grid((unsigned)((m.n_nodes + 255) / 256)), block(256);
    if (m.dtype == F64)
        hipLaunchKernelGGL(k_node_tiled<double>, grid, block, 0, s, m.n_nodes, tv.noff, tv.npos, tv.stage,
                           (double*)grad, accumulate);
    else
        hipLaunchKernelGGL(k_node_tiled<float>, grid, block, 0, s, m.n_nodes, tv.noff, tv.npos, tv.stage,
                           (float*)grad, accumulate);
    return hipGetLastError();
}

}  // namespace pg
