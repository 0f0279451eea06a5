// Many uneven meshes in one persistent launch.
//
// The plan cuts every instance into tiles of block*EPT elements and orders the
// tiles largest instance first; a fixed grid of workgroups walks that list
// round-robin (tile g, g + grid, g + 2 grid, ...), so the assignment is static
// and the result deterministic.  Each tile reduces its objective terms into
// its own slot, laid out instance by instance, and one segmented reduction
// per instance follows.  This is the fusion the paper's conclusion asks for:
// one launch instead of one (or two) per instance, and no host round trip.
#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

namespace {

template <typename T, int K, int MODE, int EPT>
__global__ void __launch_bounds__(1024)
k_batch_persistent(BatchView bv, BatchPass p) {
    __shared__ double lds[16];
    const T* __restrict__ B = static_cast<const T*>(bv.B);
    const T* __restrict__ W = static_cast<const T*>(bv.w);
    const T* __restrict__ X = static_cast<const T*>(p.x);
    double* __restrict__ G = static_cast<double*>(p.grad);
    const int32_t* __restrict__ conn = bv.conn;
    const int kk = K > 0 ? K : bv.k;
    const int bs = blockDim.x;
    for (int64_t tile = blockIdx.x; tile < bv.n_tiles; tile += gridDim.x) {
        const int64_t inst = bv.tile_inst[tile];
        const int64_t first = bv.tile_first[tile];
        const int64_t end = bv.inst_elem_end[inst];
        const int64_t noff = bv.inst_node_off[inst];
        double fb = 1.0;
        if (MODE != B_PRIMAL && p.fbar) fb = p.fbar[inst];
        double tsum = 0.0;
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int64_t e = first + (int64_t)i * bs + threadIdx.x;
            if (e < end && e < first + (int64_t)bs * EPT) {
                double u = 0.0;
                if (p.u_in) {
                    u = p.u_in[e];
                } else if constexpr (K > 0) {
                    int32_t c[K > 0 ? K : 1];
                    double bb[K > 0 ? K : 1];
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        c[j] = conn[e * K + j];
                        bb[j] = to_f64(B[e * K + j]);
                    }
#pragma unroll
                    for (int j = 0; j < K; ++j) u += bb[j] * to_f64(X[noff + c[j]]);
                } else {
                    for (int j = 0; j < kk; ++j)
                        u += to_f64(B[e * kk + j]) * to_f64(X[noff + conn[e * kk + j]]);
                }
                if (p.u_store) p.u_store[e] = u;
                const double s2 = u * u, wd = to_f64(W[e]);
                if (MODE != B_ADJ_ATOMIC) tsum += wd * psi_from_sq(s2);
                if (MODE != B_PRIMAL) {
                    const double v = fb * wd * dpsi_from(u, s2);
                    for (int j = 0; j < kk; ++j)
                        atomic_add_f64(G + noff + conn[e * kk + j], v * to_f64(B[e * kk + j]));
                }
            }
        }
        if (MODE != B_ADJ_ATOMIC) {
            const double s = block_sum_dyn(tsum, lds);
            if (threadIdx.x == 0) p.partials[bv.tile_slot[tile]] = s;
        }
    }
}

template <typename T, int K, int MODE>
hipError_t launch_ept(const BatchView& b, const BatchPass& p, hipStream_t s) {
    const int ept = b.tile_elems / p.block;
    switch (ept) {
        case 1: hipLaunchKernelGGL((k_batch_persistent<T, K, MODE, 1>), dim3(p.grid), dim3(p.block), 0, s, b, p); break;
        case 2: hipLaunchKernelGGL((k_batch_persistent<T, K, MODE, 2>), dim3(p.grid), dim3(p.block), 0, s, b, p); break;
        case 4: hipLaunchKernelGGL((k_batch_persistent<T, K, MODE, 4>), dim3(p.grid), dim3(p.block), 0, s, b, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_k(const BatchView& b, const BatchPass& p, hipStream_t s) {
    if (b.k == 8) return launch_ept<T, 8, MODE>(b, p, s);
    return launch_ept<T, 0, MODE>(b, p, s);
}

template <typename T>
hipError_t launch_mode(const BatchView& b, BatchMode mode, const BatchPass& p, hipStream_t s) {
    switch (mode) {
        case B_PRIMAL: return launch_k<T, B_PRIMAL>(b, p, s);
        case B_GRAD_ATOMIC: return launch_k<T, B_GRAD_ATOMIC>(b, p, s);
        case B_ADJ_ATOMIC: return launch_k<T, B_ADJ_ATOMIC>(b, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch_persistent(const BatchView& b, BatchMode mode, const BatchPass& p,
                                   hipStream_t s) {
    if (b.n_tiles == 0) return hipSuccess;
    if (p.grid <= 0 || p.block <= 0 || p.block > 1024 || p.block % 64) return hipErrorInvalidValue;
    return b.dtype == F64 ? launch_mode<double>(b, mode, p, s) : launch_mode<float>(b, mode, p, s);
}

}  // namespace pg
