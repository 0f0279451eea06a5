// Many uneven meshes in one persistent launch.
//
// The plan cuts every instance into tiles of block*EPT elements and orders the
// tiles largest instance first; a grid sized to the resident capacity of the
// device walks that list round-robin (tile g, g + grid, g + 2 grid, ...), so
// the assignment is static and the objective deterministic.  Each tile
// reduces its objective terms into its own slot, laid out instance by
// instance, and one segmented reduction per instance follows.  This is the
// fusion the paper's conclusion asks for: one launch instead of one (or two)
// per instance, and no host round trip.  Inside a tile the work is exactly
// the single-mesh element pass (elem_tile.hpp) with the instance's node
// offset and seed.
#include <type_traits>

#include "elem_tile.hpp"
#include "persist.hpp"

namespace pg {

namespace {

struct TileRec {
    int64_t first, end, shift_noff, slot_inst;
};

__device__ __forceinline__ TileRec load_tile(const int64_t* tiles, int64_t t) {
    const longlong2* p = reinterpret_cast<const longlong2*>(tiles + 4 * t);
    const longlong2 a = p[0], b = p[1];
    return TileRec{a.x, a.y, b.x, b.y};
}

constexpr int64_t kSlotMask = (1LL << 40) - 1;
constexpr int64_t kNoffMask = (1LL << 40) - 1;

// Logical workgroup l (XCD-remapped, so l .. l + grid/8 - 1 share an XCD)
// takes tiles l, l + grid, ...; consecutive tiles of an instance therefore run
// at the same time on one XCD and share its L2.  The next tile's record is
// loaded while the current tile is processed.
template <typename T, int K, int MODE, int EPT, bool AGG>
__global__ void __launch_bounds__(1024)
k_batch_persistent(BatchView bv, BatchPass p) {
    __shared__ double lds[16];
    __shared__ typename std::conditional<AGG, AggTable, int>::type agg;
    AggTable* tab = nullptr;
    if constexpr (AGG) tab = &agg;
    TileArgs a{bv.conn, bv.B, bv.w, p.x, nullptr, p.u_in, p.u_store, nullptr,
               static_cast<double*>(p.grad), nullptr, 0u};
    const int64_t G = gridDim.x;
    int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    TileRec cur{};
    if (tile < bv.n_tiles) cur = load_tile(bv.tiles, tile);
    for (; tile < bv.n_tiles; tile += G) {
        TileRec nxt{};
        if (tile + G < bv.n_tiles) nxt = load_tile(bv.tiles, tile + G);
        const int64_t inst = cur.slot_inst >> 40;
        double fb = 1.0;
        if constexpr (has_rev(MODE)) fb = p.fbar ? p.fbar[inst] : 1.0;
        a.hash_shift = (uint32_t)(cur.shift_noff >> 40);
        const double tsum = elem_tile<T, K, MODE, EPT, AGG>(a, cur.first, cur.end,
                                                            cur.shift_noff & kNoffMask, fb, tab);
        if constexpr (has_obj(MODE)) {
            const double s = block_sum_dyn(tsum, lds);
            if (threadIdx.x == 0) p.partials[cur.slot_inst & kSlotMask] = s;
        }
        cur = nxt;
    }
}

// Runtime k: one element per thread, rows streamed through the cache.
template <typename T, int MODE>
__global__ void __launch_bounds__(1024)
k_batch_persistent_dyn(BatchView bv, BatchPass p) {
    __shared__ double lds[16];
    const T* __restrict__ B = static_cast<const T*>(bv.B);
    const T* __restrict__ W = static_cast<const T*>(bv.w);
    const T* __restrict__ X = static_cast<const T*>(p.x);
    double* __restrict__ G = static_cast<double*>(p.grad);
    const int32_t* __restrict__ conn = bv.conn;
    const int k = bv.k;
    for (int64_t tile = xcd_remap(blockIdx.x, gridDim.x); tile < bv.n_tiles; tile += gridDim.x) {
        const TileRec r = load_tile(bv.tiles, tile);
        const int64_t inst = r.slot_inst >> 40;
        const int64_t e = r.first + threadIdx.x;
        double tsum = 0.0;
        if (e < r.end) {
            double u = 0.0;
            if (p.u_in) {
                u = p.u_in[e];
            } else {
                for (int j = 0; j < k; ++j)
                    u += to_f64(B[e * k + j]) * to_f64(X[(r.shift_noff & kNoffMask) + conn[e * k + j]]);
                if (p.u_store) p.u_store[e] = u;
            }
            const double s2 = u * u, wd = to_f64(W[e]);
            if constexpr (has_obj(MODE)) tsum = wd * psi_from_sq(s2);
            if constexpr (has_rev(MODE)) {
                const double v = (p.fbar ? p.fbar[inst] : 1.0) * wd * dpsi_from(u, s2);
                for (int j = 0; j < k; ++j)
                    atomic_add_f64(G + (r.shift_noff & kNoffMask) + conn[e * k + j],
                                   v * to_f64(B[e * k + j]));
            }
        }
        if constexpr (has_obj(MODE)) {
            const double s = block_sum_dyn(tsum, lds);
            if (threadIdx.x == 0) p.partials[r.slot_inst & kSlotMask] = s;
        }
    }
}

template <typename T, int K, int MODE, int EPT>
hipError_t launch_agg(const BatchView& b, const BatchPass& p, hipStream_t s) {
    const bool agg = is_atomic(MODE) && p.combine && (int64_t)p.block * EPT * K <= 2 * kAggSlots;
    if constexpr (is_atomic(MODE) && EPT == 1) {
        if (agg) {
            BatchTiles tiles{b.tiles, b.n_tiles};
            TileArgs a{b.conn, b.B, b.w, p.x, nullptr, p.u_in, nullptr, nullptr,
                       static_cast<double*>(p.grad), nullptr, 0u};
            auto kern = k_atomic_persistent<T, K, MODE, BatchTiles>;
            PG_LAUNCH(kern, dim3(resident_grid(kern, p.block, b.n_tiles, p.grid)),
                               dim3(p.block), 0, s, tiles, a, p.fbar, 1, p.partials);
            return hipGetLastError();
        }
    }
    if (agg) {
        auto kern = k_batch_persistent<T, K, MODE, EPT, true>;
        PG_LAUNCH(kern, dim3(resident_grid(kern, p.block, b.n_tiles, p.grid)),
                           dim3(p.block), 0, s, b, p);
    } else {
        auto kern = k_batch_persistent<T, K, MODE, EPT, false>;
        PG_LAUNCH(kern, dim3(resident_grid(kern, p.block, b.n_tiles, p.grid)),
                           dim3(p.block), 0, s, b, p);
    }
    return hipGetLastError();
}

template <typename T, int K, int MODE>
hipError_t launch_ept(const BatchView& b, const BatchPass& p, hipStream_t s) {
    switch (b.tile_elems / p.block) {
        case 1: return launch_agg<T, K, MODE, 1>(b, p, s);
        case 2: return launch_agg<T, K, MODE, 2>(b, p, s);
        case 4: return launch_agg<T, K, MODE, 4>(b, p, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODE>
hipError_t launch_k(const BatchView& b, const BatchPass& p, hipStream_t s) {
    switch (b.k) {
        case 8: return launch_ept<T, 8, MODE>(b, p, s);
        case 4: return launch_ept<T, 4, MODE>(b, p, s);
        case 2: return launch_ept<T, 2, MODE>(b, p, s);
        default:
            if (b.tile_elems != p.block) return hipErrorInvalidValue;
            {
                auto kern = k_batch_persistent_dyn<T, MODE>;
                PG_LAUNCH(kern, dim3(resident_grid(kern, p.block, b.n_tiles, p.grid)),
                                   dim3(p.block), 0, s, b, p);
            }
            return hipGetLastError();
    }
}

template <typename T>
hipError_t launch_mode(const BatchView& b, BatchMode mode, const BatchPass& p, hipStream_t s) {
    switch (mode) {
        case B_PRIMAL: return launch_k<T, M_PRIMAL>(b, p, s);
        case B_GRAD_ATOMIC: return launch_k<T, M_GRAD_ATOMIC>(b, p, s);
        case B_ADJ_ATOMIC: return launch_k<T, M_ADJ_ATOMIC>(b, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch_persistent(const BatchView& b, BatchMode mode, const BatchPass& p,
                                   hipStream_t s) {
    if (b.n_tiles == 0) return hipSuccess;
    if (p.block <= 0 || p.block > 1024 || p.block % 64) return hipErrorInvalidValue;
    return b.dtype == F64 ? launch_mode<double>(b, mode, p, s) : launch_mode<float>(b, mode, p, s);
}

}  // namespace pg
