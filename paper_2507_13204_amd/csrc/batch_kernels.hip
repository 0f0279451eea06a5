// Many uneven meshes in one launch.
//
// The plan cuts every instance into tiles of block*EPT elements and orders the
// tiles largest instance first; the launch has one workgroup per tile, and
// the hardware dispatcher hands tiles out in that order as workgroups retire
// (longest-processing-time-first list scheduling with no host involvement).
// Each tile reduces its objective terms into its own slot, laid out instance
// by instance, and one segmented reduction per instance follows, so the
// objective is deterministic.  This is the fusion the paper's conclusion
// asks for: one launch instead of one (or two) per instance, and no host
// round trip.  Inside a tile the work is exactly the single-mesh element
// pass (elem_tile.hpp) with the instance's node offset, hash rotation and
// seed.  (A persistent grid walking the list round-robin, with the next
// tile's rows prefetched, measured 15% slower on 256 hex meshes.)
#include <type_traits>

#include "elem_tile.hpp"

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

// One workgroup per tile.  Logical tile l = XCD-remapped block id, so
// consecutive tiles of an instance run on one XCD at the same time and share
// its L2.
template <typename T, int K, int MODE, int EPT, int AGG>
__global__ void __launch_bounds__(1024)
k_batch_tiles(BatchView bv, BatchPass p) {
    __shared__ double lds[16];
    __shared__ AggOf<AGG> agg;
    AggOf<AGG>* tab = nullptr;
    if constexpr (AGG > 0) tab = &agg;
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const TileRec cur = load_tile(bv.tiles, tile);
    const int64_t inst = cur.slot_inst >> 40;
    double fb = 1.0;
    if constexpr (has_rev(MODE)) fb = p.fbar ? p.fbar[inst] : 1.0;
    // 64-bit gather addresses: the 32-bit buffer offsets that help the
    // single mesh measured 0.8% slower here
    TileArgs a{bv.conn, bv.B, bv.w, p.x, nullptr, p.u_in, p.u_store, nullptr,
               static_cast<double*>(p.grad), nullptr, (uint32_t)(cur.shift_noff >> 40), 0u};
    const double tsum = elem_tile<T, K, MODE, EPT, AGG, false>(a, cur.first, cur.end,
                                                               cur.shift_noff & kNoffMask, fb, tab);
    if constexpr (has_obj(MODE)) {
        const double s = block_sum_dyn(tsum, lds);
        if (threadIdx.x == 0) p.partials[cur.slot_inst & kSlotMask] = s;
    }
}

// Runtime k: one element per thread, rows streamed through the cache.
template <typename T, int MODE>
__global__ void __launch_bounds__(1024)
k_batch_tiles_dyn(BatchView bv, BatchPass p) {
    __shared__ double lds[16];
    const T* __restrict__ B = static_cast<const T*>(bv.B);
    const T* __restrict__ W = static_cast<const T*>(bv.w);
    const T* __restrict__ X = static_cast<const T*>(p.x);
    double* __restrict__ G = static_cast<double*>(p.grad);
    const int32_t* __restrict__ conn = bv.conn;
    const int k = bv.k;
    const TileRec r = load_tile(bv.tiles, xcd_remap(blockIdx.x, gridDim.x));
    const int64_t inst = r.slot_inst >> 40, noff = r.shift_noff & kNoffMask;
    const int64_t e = r.first + threadIdx.x;
    double tsum = 0.0;
    if (e < r.end) {
        double u = 0.0;
        if (p.u_in) {
            u = p.u_in[e];
        } else {
            for (int j = 0; j < k; ++j) u += to_f64(B[e * k + j]) * to_f64(X[noff + conn[e * k + j]]);
            if (p.u_store) p.u_store[e] = u;
        }
        const double s2 = u * u, wd = to_f64(W[e]);
        if constexpr (has_obj(MODE)) tsum = wd * psi_from_sq(s2);
        if constexpr (has_rev(MODE)) {
            const double v = (p.fbar ? p.fbar[inst] : 1.0) * wd * dpsi_from(u, s2);
            for (int j = 0; j < k; ++j) atomic_add_f64(G + noff + conn[e * k + j], v * to_f64(B[e * k + j]));
        }
    }
    if constexpr (has_obj(MODE)) {
        const double s = block_sum_dyn(tsum, lds);
        if (threadIdx.x == 0) p.partials[r.slot_inst & kSlotMask] = s;
    }
}

template <typename T, int K, int MODE, int EPT>
hipError_t launch_agg(const BatchView& b, const BatchPass& p, hipStream_t s) {
    const bool agg = is_atomic(MODE) && p.combine && (int64_t)p.block * EPT * K <= 2 * kAggSlots;
    if (agg)
        PG_LAUNCH((k_batch_tiles<T, K, MODE, EPT, kAggSlots>), dim3((unsigned)b.n_tiles), dim3(p.block), 0,
                  s, b, p);
    else
        PG_LAUNCH((k_batch_tiles<T, K, MODE, EPT, 0>), dim3((unsigned)b.n_tiles), dim3(p.block), 0,
                  s, b, p);
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
            PG_LAUNCH((k_batch_tiles_dyn<T, MODE>), dim3((unsigned)b.n_tiles), dim3(p.block), 0, s, b, p);
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

hipError_t launch_batch(const BatchView& b, BatchMode mode, const BatchPass& p,
                                   hipStream_t s) {
    if (b.n_tiles == 0) return hipSuccess;
    if (p.block <= 0 || p.block > 1024 || p.block % 64) return hipErrorInvalidValue;
    return b.dtype == F64 ? launch_mode<double>(b, mode, p, s) : launch_mode<float>(b, mode, p, s);
}

}  // namespace pg
