// Dense row reduction with hierarchical (team / vector) parallelism:
//   f(x) = sum_i w_i psi((A x)_i),   grad = A^T (fbar w (.) psi'(A x)).
//
// A workgroup is the team of one row at a time: its lanes read the row with
// 16-byte coalesced loads, reduce their products with wavefront butterflies,
// and combine the waves through LDS.  In the fused kernel every thread keeps
// its slice of x and of the running column sums in registers while the
// workgroup walks a contiguous band of rows, so A is read from HBM exactly
// once for f and the gradient together; the per-band column sums are then
// added in a fixed order (deterministic, no atomics).
#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

namespace {

constexpr int kFusedBS = 512;
constexpr int kMaxQ = 16;

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};

__device__ __forceinline__ void to_arr(const double2& v, double* o) {
    o[0] = v.x;
    o[1] = v.y;
}
__device__ __forceinline__ void to_arr(const float4& v, double* o) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
}

// Broadcast sum over the workgroup: every thread receives the total.
__device__ __forceinline__ double block_allsum(double v, double* lds) {
    const int nw = blockDim.x / kWave;
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += lds[i];  // same order in every thread
    __syncthreads();
    return r;
}

template <typename T, int Q>
__global__ void __launch_bounds__(kFusedBS)
k_dense_fused(DenseView d, const T* __restrict__ x, const double* __restrict__ fbar, int want_grad,
              double* __restrict__ partials, double* __restrict__ colpart, int ngroups) {
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    __shared__ double lds[kFusedBS / kWave];
    const T* __restrict__ A = static_cast<const T*>(d.A);
    const T* __restrict__ w = static_cast<const T*>(d.w);
    const int64_t cols = d.cols;
    const int64_t nvec = cols / VN;  // cols is a multiple of VN here
    const int g = blockIdx.x;
    const int64_t r0 = d.rows * g / ngroups, r1 = d.rows * (g + 1) / ngroups;
    const double fb = fbar ? fbar[0] : 1.0;

    double xr[Q][VN], acc[Q][VN];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t vi = threadIdx.x + (int64_t)kFusedBS * q;
        if (vi < nvec) {
            V v = reinterpret_cast<const V*>(x)[vi];
            to_arr(v, xr[q]);
        } else {
#pragma unroll
            for (int c = 0; c < VN; ++c) xr[q][c] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < VN; ++c) acc[q][c] = 0.0;
    }
    V cur[Q], nxt[Q];
    auto load_row = [&](int64_t i, V (&dst)[Q]) {
        const V* row = reinterpret_cast<const V*>(A + i * cols);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t vi = threadIdx.x + (int64_t)kFusedBS * q;
            if (vi < nvec)
                dst[q] = row[vi];
            else
                dst[q] = V{};
        }
    };
    double tsum = 0.0;
    if (r0 < r1) load_row(r0, cur);
    for (int64_t i = r0; i < r1; ++i) {
        if (i + 1 < r1) load_row(i + 1, nxt);
        double dot = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double a[VN];
            to_arr(cur[q], a);
#pragma unroll
            for (int c = 0; c < VN; ++c) dot += a[c] * xr[q][c];
        }
        const double r = block_allsum(dot, lds);
        const double s2 = r * r, wi = to_f64(w[i]);
        tsum += wi * psi_from_sq(s2);
        if (want_grad) {
            const double v = fb * wi * dpsi_from(r, s2);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double a[VN];
                to_arr(cur[q], a);
#pragma unroll
                for (int c = 0; c < VN; ++c) acc[q][c] += v * a[c];
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) cur[q] = nxt[q];
    }
    if (threadIdx.x == 0) partials[g] = tsum;
    if (want_grad) {
        double* out = colpart + (int64_t)g * cols;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t vi = threadIdx.x + (int64_t)kFusedBS * q;
            if (vi < nvec) {
#pragma unroll
                for (int c = 0; c < VN; ++c) out[vi * VN + c] = acc[q][c];
            }
        }
    }
}

// grad[j] (=|+=) sum of colpart[g, j] over the bands: kColSlices slices of
// consecutive bands, each summed in ascending order by one thread, then the
// slices added in ascending order (deterministic).  32 columns per
// workgroup so the launch covers the device even for 10^4 columns.
constexpr int kColW = 32, kColSlices = 16;

template <typename T>
__global__ void __launch_bounds__(kColW * kColSlices)
k_dense_colsum(const double* __restrict__ colpart, int ngroups, int64_t cols, T* __restrict__ grad,
               int accumulate) {
    __shared__ double part[kColSlices][kColW];
    const int64_t j = (int64_t)blockIdx.x * kColW + threadIdx.x;
    const int y = threadIdx.y;
    double s = 0.0;
    if (j < cols) {
        const int g0 = ngroups * y / kColSlices, g1 = ngroups * (y + 1) / kColSlices;
        for (int g = g0; g < g1; ++g) s += colpart[(int64_t)g * cols + j];
    }
    part[y][threadIdx.x] = s;
    __syncthreads();
    if (y == 0 && j < cols) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kColSlices; ++q) t += part[q][threadIdx.x];
        grad[j] = accumulate ? static_cast<T>(to_f64(grad[j]) + t) : static_cast<T>(t);
    }
}

// One workgroup per row (any cols): r_i, then t_i into partials[i] and,
// when v != nullptr, v_i = fbar w_i psi'(r_i).
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_rows(DenseView d, const T* __restrict__ x, const double* __restrict__ fbar,
             double* __restrict__ partials, double* __restrict__ v) {
    __shared__ double lds[4];
    const T* __restrict__ A = static_cast<const T*>(d.A);
    const T* __restrict__ w = static_cast<const T*>(d.w);
    const int64_t i = blockIdx.x;
    const T* row = A + i * d.cols;
    double dot = 0.0;
    for (int64_t j = threadIdx.x; j < d.cols; j += blockDim.x) dot += to_f64(row[j]) * to_f64(x[j]);
    const double r = block_sum<256>(dot, lds);
    if (threadIdx.x == 0) {
        const double s2 = r * r, wi = to_f64(w[i]);
        partials[i] = wi * psi_from_sq(s2);
        if (v) v[i] = (fbar ? fbar[0] : 1.0) * wi * dpsi_from(r, s2);
    }
}

// grad (=|+=) A^T v, column-parallel: 64 columns per workgroup, 4 row slices.
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_cols(DenseView d, const double* __restrict__ v, T* __restrict__ grad, int accumulate) {
    __shared__ double part[4][64];
    const T* __restrict__ A = static_cast<const T*>(d.A);
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int y = threadIdx.y;
    double s = 0.0;
    if (j < d.cols) {
        const int64_t i0 = d.rows * y / 4, i1 = d.rows * (y + 1) / 4;
        for (int64_t i = i0; i < i1; ++i) s += to_f64(A[i * d.cols + j]) * v[i];
    }
    part[y][threadIdx.x] = s;
    __syncthreads();
    if (y == 0 && j < d.cols) {
        const double t = ((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) +
                         part[3][threadIdx.x];
        grad[j] = accumulate ? static_cast<T>(to_f64(grad[j]) + t) : static_cast<T>(t);
    }
}

template <typename T>
hipError_t fused_q(const DenseView& d, const void* x, const double* fbar, int want_grad,
                   double* partials, double* colpart, int ngroups, hipStream_t s) {
    constexpr int VN = Vec16<T>::n;
    const int64_t per_q = (int64_t)kFusedBS * VN;
    const int64_t q = (d.cols + per_q - 1) / per_q;
    const T* xp = static_cast<const T*>(x);
#define PG_FUSED_CASE(QV)                                                                        \
    if (q <= QV) {                                                                               \
        PG_LAUNCH((k_dense_fused<T, QV>), dim3(ngroups), dim3(kFusedBS), 0, s, d, xp,  \
                           fbar, want_grad, partials, colpart, ngroups);                        \
        return hipGetLastError();                                                                \
    }
    PG_FUSED_CASE(1)
    PG_FUSED_CASE(2)
    PG_FUSED_CASE(4)
    PG_FUSED_CASE(6)
    PG_FUSED_CASE(8)
    PG_FUSED_CASE(10)
    PG_FUSED_CASE(12)
    PG_FUSED_CASE(16)
#undef PG_FUSED_CASE
    return hipErrorInvalidValue;
}

}  // namespace

int64_t dense_fused_max_cols() { return (int64_t)kFusedBS * 2 * kMaxQ; }

hipError_t launch_dense_fused(const DenseView& d, const void* x, const double* fbar, int want_grad,
                              double* partials, double* colpart, int ngroups, hipStream_t s) {
    const int vn = d.dtype == F64 ? 2 : 4;
    if (d.cols % vn != 0 || d.cols > (int64_t)kFusedBS * vn * kMaxQ) return hipErrorInvalidValue;
    if (d.rows == 0) return hipSuccess;
    return d.dtype == F64 ? fused_q<double>(d, x, fbar, want_grad, partials, colpart, ngroups, s)
                          : fused_q<float>(d, x, fbar, want_grad, partials, colpart, ngroups, s);
}

hipError_t launch_dense_colsum(const double* colpart, int ngroups, int64_t cols, void* grad,
                               Dtype dt, int accumulate, hipStream_t s) {
    if (cols == 0) return hipSuccess;
    const dim3 grid((unsigned)((cols + kColW - 1) / kColW)), block(kColW, kColSlices);
    if (dt == F64)
        hipLaunchKernelGGL(k_dense_colsum<double>, grid, block, 0, s, colpart, ngroups, cols,
                           (double*)grad, accumulate);
    else
        hipLaunchKernelGGL(k_dense_colsum<float>, grid, block, 0, s, colpart, ngroups, cols,
                           (float*)grad, accumulate);
    return hipGetLastError();
}

hipError_t launch_dense_rows(const DenseView& d, const void* x, const double* fbar,
                             double* partials, double* v, hipStream_t s) {
    if (d.rows == 0) return hipSuccess;
    if (d.dtype == F64)
        hipLaunchKernelGGL(k_dense_rows<double>, dim3((unsigned)d.rows), dim3(256), 0, s, d,
                           (const double*)x, fbar, partials, v);
    else
        hipLaunchKernelGGL(k_dense_rows<float>, dim3((unsigned)d.rows), dim3(256), 0, s, d,
                           (const float*)x, fbar, partials, v);
    return hipGetLastError();
}

hipError_t launch_dense_cols(const DenseView& d, const double* v, void* grad, int accumulate,
                             hipStream_t s) {
    if (d.cols == 0) return hipSuccess;
    const dim3 grid((unsigned)((d.cols + 63) / 64)), block(64, 4);
    if (d.dtype == F64)
        hipLaunchKernelGGL(k_dense_cols<double>, grid, block, 0, s, d, v, (double*)grad, accumulate);
    else
        hipLaunchKernelGGL(k_dense_cols<float>, grid, block, 0, s, d, v, (float*)grad, accumulate);
    return hipGetLastError();
}

}  // namespace pg
