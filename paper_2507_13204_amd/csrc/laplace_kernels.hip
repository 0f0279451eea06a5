// The paper's section 4 example on gfx950:
//   f(x, b) = || A (3x) - b ||^2,   A = 1D Laplacian (2, -1, -1; rows
//   truncated at both ends), with gradients in x and b.
//
// The generated code of the paper runs five kernels and a host round trip
// (scale, stencil + square, sum; seed, broadcast, reverse stencil with
// atomics, reverse scale).  Here one kernel does the forward replay, the
// seed, the broadcast and the reverse pass:
//   GATHER (the reverse threads rescheduled, as the conclusion proposes):
//     thread i recomputes y_{i-1}, y_i, y_{i+1} from its neighbourhood and
//     writes xbar_i = 3 (2 ybar_i - ybar_{i-1} - ybar_{i+1}) and bbar_i =
//     -ybar_i directly: no atomics, no zero fill, deterministic;
//   ATOMIC (the paper's schedule): thread j scatters -3 ybar_j, 6 ybar_j,
//     -3 ybar_j into xbar_{j-1}, xbar_j, xbar_{j+1} with FP64 atomics.
// The objective's terms y_j^2 are reduced per workgroup (fixed order).  For
// small n (at most kLapFusedBlocks workgroups) the last workgroup to finish,
// found by a ticket counter, adds the per-workgroup partials in their fixed
// order and writes f, so a call is one launch: a device-scope fence per
// workgroup is cheap at that grid size.
#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

namespace {

constexpr int64_t kLapFusedBlocks = 64;

template <typename T>
__device__ __forceinline__ double lap_y(int64_t i, int64_t n, const T* __restrict__ x,
                                        const T* __restrict__ b) {
    double v = 2.0 * (3.0 * to_f64(x[i])) - to_f64(b[i]);
    if (i != 0) v -= 3.0 * to_f64(x[i - 1]);
    if (i != n - 1) v -= 3.0 * to_f64(x[i + 1]);
    return v;
}

// MODE 0: objective; 1: gradient, gather form; 2: gradient, atomic form.
// FUSED: the last workgroup also sums the partials into f_out (when not null)
// and re-arms the ticket for the next launch.
template <typename T, int MODE, bool FUSED>
__global__ void __launch_bounds__(256)
k_laplace1d(int64_t n, const T* __restrict__ x, const T* __restrict__ b, double* __restrict__ gx,
            T* __restrict__ gx_t, T* __restrict__ gb, const double* __restrict__ fbar,
            double* __restrict__ partials, int accumulate, int32_t* __restrict__ ticket,
            double* __restrict__ f_out) {
    __shared__ double lds[4];
    __shared__ int last;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double t = 0.0;
    if (i < n) {
        const double y = lap_y(i, n, x, b);
        t = y * y;
        if (MODE != 0) {
            const double fb = fbar ? fbar[0] : 1.0;
            const double yb = fb * 2.0 * y;
            if (gb) gb[i] = accumulate ? static_cast<T>(to_f64(gb[i]) - yb) : static_cast<T>(-yb);
            if (MODE == 1 && gx_t) {
                double v = 2.0 * yb;
                if (i != 0) v -= fb * 2.0 * lap_y(i - 1, n, x, b);
                if (i != n - 1) v -= fb * 2.0 * lap_y(i + 1, n, x, b);
                const double g = 3.0 * v;
                gx_t[i] = accumulate ? static_cast<T>(to_f64(gx_t[i]) + g) : static_cast<T>(g);
            }
            if (MODE == 2 && gx) {
                if (i != 0) atomic_add_f64(gx + i - 1, -3.0 * yb);
                atomic_add_f64(gx + i, 6.0 * yb);
                if (i != n - 1) atomic_add_f64(gx + i + 1, -3.0 * yb);
            }
        }
    }
    const double s = block_sum<256>(t, lds);
    if constexpr (!FUSED) {
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    } else {
        if (threadIdx.x == 0) {
            partials[blockIdx.x] = s;
            __threadfence();  // the partial is visible before the ticket is taken
            last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
        }
        __syncthreads();
        if (last) {
            __threadfence();  // every other workgroup's partial is visible
            double v = 0.0;
            for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) v += partials[q];
            v = block_sum<256>(v, lds);
            if (threadIdx.x == 0) {
                if (f_out) f_out[0] = v;
                *ticket = 0;
            }
        }
    }
}

template <typename T, bool FUSED>
hipError_t launch_t(int64_t n, int mode, const void* x, const void* b, double* gx64, void* gx,
                    void* gb, const double* fbar, double* partials, int accumulate,
                    int32_t* ticket, double* f_out, hipStream_t s) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    const T* xp = static_cast<const T*>(x);
    const T* bp = static_cast<const T*>(b);
    switch (mode) {
        case 0:
            PG_LAUNCH((k_laplace1d<T, 0, FUSED>), dim3(nb), dim3(256), 0, s, n, xp, bp, nullptr,
                      nullptr, nullptr, fbar, partials, accumulate, ticket, f_out);
            break;
        case 1:
            PG_LAUNCH((k_laplace1d<T, 1, FUSED>), dim3(nb), dim3(256), 0, s, n, xp, bp, nullptr,
                      static_cast<T*>(gx), static_cast<T*>(gb), fbar, partials, accumulate, ticket,
                      f_out);
            break;
        case 2:
            PG_LAUNCH((k_laplace1d<T, 2, FUSED>), dim3(nb), dim3(256), 0, s, n, xp, bp, gx64,
                      nullptr, static_cast<T*>(gb), fbar, partials, accumulate, ticket, f_out);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int64_t laplace1d_blocks(int64_t n) { return (n + 255) / 256; }

bool laplace1d_fused(int64_t n) { return n > 0 && laplace1d_blocks(n) <= kLapFusedBlocks; }

hipError_t launch_laplace1d(int64_t n, Dtype dt, int mode, const void* x, const void* b,
                            double* gx64, void* gx, void* gb, const double* fbar,
                            double* partials, int accumulate, int32_t* ticket, double* f_out,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (laplace1d_fused(n)) {
        if (!ticket) return hipErrorInvalidValue;
        return dt == F64 ? launch_t<double, true>(n, mode, x, b, gx64, gx, gb, fbar, partials,
                                                  accumulate, ticket, f_out, s)
                         : launch_t<float, true>(n, mode, x, b, gx64, gx, gb, fbar, partials,
                                                 accumulate, ticket, f_out, s);
    }
    return dt == F64 ? launch_t<double, false>(n, mode, x, b, gx64, gx, gb, fbar, partials,
                                               accumulate, nullptr, nullptr, s)
                     : launch_t<float, false>(n, mode, x, b, gx64, gx, gb, fbar, partials,
                                              accumulate, nullptr, nullptr, s);
}

}  // namespace pg
