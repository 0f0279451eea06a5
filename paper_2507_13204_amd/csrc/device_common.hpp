// Device helpers shared by the HIP kernels of the gradient library (gfx950).
//
// Nothing here is shared with the CPU oracle: this is the GPU path only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pg {

constexpr int kWave = 64;  // CDNA wavefront width

// psi(s) = s^2/2 + log(1+s^2)/2 evaluated from q = s^2 (log1p keeps the
// small-|s| terms accurate).
__device__ __forceinline__ double psi_from_sq(double s2) { return 0.5 * s2 + 0.5 * log1p(s2); }

// psi'(s) = s + s/(1+s^2).
__device__ __forceinline__ double dpsi_from(double s, double s2) { return s + s / (1.0 + s2); }

// psi''(s) = 1 + (1-s^2)/(1+s^2)^2.
__device__ __forceinline__ double ddpsi_from_sq(double s2) {
    double q = 1.0 + s2;
    return 1.0 + (1.0 - s2) / (q * q);
}

// Sum over the 64 lanes of a wavefront; every lane receives the total.
// The butterfly order is fixed, so the result is bitwise repeatable.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over a workgroup of BS threads (BS a multiple of 64, <= 1024); the
// total is valid in thread 0.  lds must hold BS/64 doubles.  Fixed order.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* lds) {
    constexpr int NW = BS / kWave;
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    if (NW == 1) return v;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (wid == 0) {
        r = lane < NW ? lds[lane] : 0.0;
        r = wave_sum(r);
    }
    __syncthreads();
    return r;
}

// Runtime-size variant (blockDim.x a multiple of 64).
__device__ __forceinline__ double block_sum_dyn(double v, double* lds) {
    const int nw = blockDim.x / kWave;
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    if (nw == 1) return v;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (wid == 0) {
        r = lane < nw ? lds[lane] : 0.0;
        r = wave_sum(r);
    }
    __syncthreads();
    return r;
}

// Workgroups of one launch are dealt round-robin to the 8 XCDs (each with its
// own L2).  Remap the hardware block id so that XCD x works on one contiguous
// range of logical blocks: neighbouring elements then share an L2, which is
// where the node values they gather (and the gradient lines they update) live.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t NX = 8;
    const uint32_t q = nblocks / NX, r = nblocks % NX;
    const uint32_t x = b % NX, i = b / NX;
    return x * q + (x < r ? x : r) + i;
}

// FP64 atomic add without return value: a hardware global_atomic_add_f64.
__device__ __forceinline__ void atomic_add_f64(double* p, double v) {
    unsafeAtomicAdd(p, v);
}

template <typename T>
__device__ __forceinline__ double to_f64(T v) {
    return static_cast<double>(v);
}

}  // namespace pg
