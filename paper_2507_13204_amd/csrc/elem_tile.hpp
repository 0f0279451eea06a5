// The element work shared by the single-mesh and the mesh-batch kernels:
// row loads, the gather, psi / psi', and the reverse scatter (atomic combined
// in LDS, colour read-add-write, or per-element adjoints for the
// node-parallel gather).
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

constexpr bool has_obj(int mode) {
    return mode == M_PRIMAL || mode == M_GRAD_ATOMIC || mode == M_GRAD_V || mode == M_GRAD_COLOUR;
}
constexpr bool has_rev(int mode) { return mode != M_PRIMAL && mode != M_HVP && mode != M_JVP; }
// Modes that reduce a per-element quantity into per-workgroup partials.
constexpr bool has_sum(int mode) { return has_obj(mode) || mode == M_JVP; }
constexpr bool is_atomic(int mode) { return mode == M_GRAD_ATOMIC || mode == M_ADJ_ATOMIC || mode == M_HVP; }
constexpr bool is_colour(int mode) { return mode == M_GRAD_COLOUR || mode == M_ADJ_COLOUR; }
constexpr bool writes_v(int mode) { return mode == M_GRAD_V || mode == M_ADJ_V; }

template <typename T, int K>
__device__ __forceinline__ void load_conn_row(const int32_t* __restrict__ conn, int64_t e,
                                              int32_t (&c)[K]) {
    if constexpr (K % 4 == 0) {
        const int4* p = reinterpret_cast<const int4*>(conn + e * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            int4 v = p[q];
            c[4 * q] = v.x;
            c[4 * q + 1] = v.y;
            c[4 * q + 2] = v.z;
            c[4 * q + 3] = v.w;
        }
    } else if constexpr (K % 2 == 0) {
        const int2* p = reinterpret_cast<const int2*>(conn + e * K);
#pragma unroll
        for (int q = 0; q < K / 2; ++q) {
            int2 v = p[q];
            c[2 * q] = v.x;
            c[2 * q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) c[j] = conn[e * K + j];
    }
}

template <int K>
__device__ __forceinline__ void load_b_row(const double* __restrict__ B, int64_t e,
                                           double (&b)[K]) {
    if constexpr (K % 2 == 0) {
        const double2* p = reinterpret_cast<const double2*>(B + e * K);
#pragma unroll
        for (int q = 0; q < K / 2; ++q) {
            double2 v = p[q];
            b[2 * q] = v.x;
            b[2 * q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) b[j] = B[e * K + j];
    }
}

template <int K>
__device__ __forceinline__ void load_b_row(const float* __restrict__ B, int64_t e, float (&b)[K]) {
    if constexpr (K % 4 == 0) {
        const float4* p = reinterpret_cast<const float4*>(B + e * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            float4 v = p[q];
            b[4 * q] = v.x;
            b[4 * q + 1] = v.y;
            b[4 * q + 2] = v.z;
            b[4 * q + 3] = v.w;
        }
    } else if constexpr (K % 2 == 0) {
        const float2* p = reinterpret_cast<const float2*>(B + e * K);
#pragma unroll
        for (int q = 0; q < K / 2; ++q) {
            float2 v = p[q];
            b[2 * q] = v.x;
            b[2 * q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) b[j] = B[e * K + j];
    }
}

// Workgroup-local combining of the atomic scatter.  FP64 atomics cost one
// memory-side request per (instruction, cache line), whatever the number of
// active lanes, so the workgroup first adds its contributions into an LDS
// hash table keyed by node (open addressing, linear probing) and then issues
// one global atomic per distinct node.  The hash keeps runs of consecutive
// node numbers in consecutive slots, so the flush touches few cache lines
// per instruction; a contribution that finds no slot within kMaxProbe steps
// goes straight to global memory, so any connectivity is handled.
constexpr int kAggSlots = 4096;       // the default table
constexpr int kAggSlotsSmall = 2048;  // chosen by the plan when its workgroups touch few nodes
constexpr int kMaxProbe = 64;

template <int S>
struct AggTableT {
    static constexpr int kSlots = S;
    int32_t key[S];
    double val[S];
};
using AggTable = AggTableT<kAggSlots>;

// Home slot of node n (agg_slot: consecutive numbers in consecutive slots,
// runs a distance D apart about D * (1 + rot / 4096) slots apart).  The plan picks
// rot (and the table size) for its connectivity by simulating the table on
// sampled workgroups.
template <int S>
__device__ __forceinline__ uint32_t agg_hash(int32_t n, uint32_t rot) {
    return agg_slot((uint32_t)n, rot, (uint32_t)S);
}

template <int S>
__device__ __forceinline__ void agg_clear(AggTableT<S>& t) {
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        t.key[s] = -1;
        t.val[s] = 0.0;
    }
}

// Linear probing from slot h (probes already spent: `used`).
template <int S>
__device__ __forceinline__ void agg_add_from(AggTableT<S>& t, int32_t n, double c, double* g,
                                             uint32_t h, int used) {
#pragma nounroll
    for (int probe = used; probe < kMaxProbe; ++probe) {
        const int32_t old = atomicCAS(&t.key[h], -1, n);
        if (old == -1 || old == n) {
            atomicAdd(&t.val[h], c);
            return;
        }
        h = (h + 1) & (S - 1);
    }
    atomic_add_f64(g + n, c);
}

template <int S>
__device__ __forceinline__ void agg_add(AggTableT<S>& t, int32_t n, double c, double* g,
                                        uint32_t shift) {
    agg_add_from(t, n, c, g, agg_hash<S>(n, shift), 0);
}

// The K contributions of one row: the first probes of all K are issued
// before any result is examined, so their LDS round trips overlap instead of
// queueing one behind the other; a contribution whose home slot holds
// another node continues probing on its own.  (Two contributions of the row
// to the same node: the second compare-and-swap finds the first's key.)
template <int K, int S>
__device__ __forceinline__ void agg_add_row(AggTableT<S>& t, const int32_t (&n)[K],
                                            const double (&c)[K], double* g, uint32_t shift) {
    uint32_t h[K];
    int32_t old[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        h[j] = agg_hash<S>(n[j], shift);
        old[j] = atomicCAS(&t.key[h[j]], -1, n[j]);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (old[j] == -1 || old[j] == n[j])
            atomicAdd(&t.val[h[j]], c[j]);
        else
            agg_add_from(t, n[j], c[j], g, (h[j] + 1) & (S - 1), 1);
    }
}

template <int S>
__device__ __forceinline__ void agg_flush(const AggTableT<S>& t, double* g) {
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        const int32_t n = t.key[s];
        if (n >= 0) atomic_add_f64(g + n, t.val[s]);
    }
}

// LDS table type of a kernel combining with S slots (S = 0: no table).
template <int S>
using AggOf = typename std::conditional<(S > 0), AggTableT<(S > 0 ? S : 64)>, int>::type;

// Arguments of one element tile (device pointers; element-indexed arrays are
// indexed by the element number e, node arrays by noff + conn[e, j]).
struct TileArgs {
    const int32_t* conn;
    const void* B;
    const void* w;
    const void* x;
    const void* xd;        // M_HVP direction
    const double* u_in;    // stored forward values (replace the gather)
    double* u_store;       // store forward values here
    double* v_out;         // per-element adjoints (M_*_V)
    double* gacc;          // FP64 accumulation target (atomic / colour modes)
    const int32_t* elist;  // element list (item -> element); nullptr: identity
    uint32_t hash_shift;   // LDS table hash parameter (atomic modes)
    uint32_t x_bytes;      // bytes of x when below 4 GiB: the gather then takes
                           // 32-bit offsets; 0: 64-bit addresses
};

// Bytes of an array of n elements of T as a buffer-resource size, or 0 when
// they reach 4 GiB (the gather then falls back to 64-bit addresses).
template <typename T>
__host__ __device__ inline uint32_t buffer_bytes(int64_t n) {
    const uint64_t b = (uint64_t)(n > 0 ? n : 0) * sizeof(T);
    return b > 0 && b <= 0xFFFFFFFFull ? (uint32_t)b : 0u;
}

// Flags word of a raw (unformatted) buffer resource on the gfx9 family.
constexpr int kRawBufferFlags = 0x00020000;

// x[n] read through a buffer resource with a 32-bit byte offset: one VGPR
// per address instead of two, and an offset past the resource's size reads
// zero instead of faulting.
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t n) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(n * 8u), 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(n * 4u), 0, 0));
}

// The element work of one workgroup: items first + i*blockDim + tid (i < EPT)
// below `end`.  Loads for all owned elements are issued before any
// arithmetic; with AGG > 0 the atomic scatter is combined in `tab`, an
// AGG-slot LDS table (every thread
// of the workgroup must call this).  Returns this thread's sum of the
// objective terms w_e psi(u_e) (0 when the mode has no objective).
// UIN: whether the forward values come from a.u_in (set) or from the gather
// (separate instantiations, so the gather path carries no branch around an
// optional load).  Requires first < end.
template <typename T, int K, int MODE, int EPT, int AGG, bool UIN, bool CLEAR_EARLY>
__device__ __forceinline__ double elem_tile_body(const TileArgs& a, int64_t first, int64_t end,
                                                 int64_t noff, double fb, AggOf<AGG>* tab) {
    const T* __restrict__ B = static_cast<const T*>(a.B);
    const T* __restrict__ W = static_cast<const T*>(a.w);
    const T* __restrict__ X = static_cast<const T*>(a.x) + noff;
    const T* __restrict__ XD = static_cast<const T*>(a.xd);
    const int32_t* __restrict__ conn = a.conn;
    const int bs = blockDim.x;
    int64_t e[EPT];
    bool ok[EPT];
    int32_t c[EPT][K];
    T b[EPT][K];
    T wv[EPT];
    double u[EPT];
    // Lanes past `end` read the rows of element end - 1 (no workgroup is
    // launched with first >= end) and contribute nothing: the loads and the
    // gather then need no branch.
    const int64_t last = end - 1;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int64_t idx = first + (int64_t)i * bs + threadIdx.x;
        ok[i] = idx < end;
        const int64_t ic = ok[i] ? idx : last;
        e[i] = a.elist ? (int64_t)a.elist[ic] : ic;
    }
    // Phase 1: rows of conn, B and w for every owned element.
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        load_conn_row<T, K>(conn, e[i], c[i]);
        load_b_row<K>(B, e[i], b[i]);
        wv[i] = W[e[i]];
    }
    // The LDS table is cleared (the previous tile's flush ended with a
    // barrier) either here, while the row loads are in flight, or after the
    // gather (CLEAR_EARLY = false).  Early, the clear loop sits between the
    // row loads and the gather, and the compiler then issues the gather only
    // once every row load (B and w too, not just conn) has arrived; late, the
    // gather leaves as soon as conn is in, and the clear adds to the wait
    // before the first barrier.  Measured on MI355X: early is 0.5 us faster
    // on the 128^3 single mesh in FP64, late 0.7 us faster in FP32 and 2.7%
    // faster on the 256-mesh batch.
    if constexpr (CLEAR_EARLY && is_atomic(MODE) && AGG > 0) agg_clear(*tab);
    // Phase 2: the gather (or the stored forward value); the HVP and JVP
    // gather the direction's entries in the same round trip.
    constexpr bool DIR = MODE == M_HVP || MODE == M_JVP;
    [[maybe_unused]] T dv[EPT][K];
    if constexpr (UIN) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) u[i] = a.u_in[e[i]];
    } else {
        T xv[EPT][K];
        if (a.x_bytes) {
            // 32-bit offsets through a buffer resource: fewer registers per
            // gather in flight (59 instead of 75 VGPRs in the FP64 gradient
            // pass: 8 waves per SIMD instead of 6)
            const __amdgpu_buffer_rsrc_t r =
                __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)a.x_bytes, kRawBufferFlags);
#pragma unroll
            for (int i = 0; i < EPT; ++i)
#pragma unroll
                for (int j = 0; j < K; ++j) xv[i][j] = buffer_load<T>(r, (uint32_t)c[i][j]);
            if constexpr (DIR) {
                const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
                    (void*)(XD + noff), (short)0, (int)a.x_bytes, kRawBufferFlags);
#pragma unroll
                for (int i = 0; i < EPT; ++i)
#pragma unroll
                    for (int j = 0; j < K; ++j) dv[i][j] = buffer_load<T>(rd, (uint32_t)c[i][j]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < EPT; ++i)
#pragma unroll
                for (int j = 0; j < K; ++j) xv[i][j] = X[c[i][j]];
            if constexpr (DIR) {
#pragma unroll
                for (int i = 0; i < EPT; ++i)
#pragma unroll
                    for (int j = 0; j < K; ++j) dv[i][j] = XD[noff + c[i][j]];
            }
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) acc += to_f64(b[i][j]) * to_f64(xv[i][j]);
            u[i] = acc;
        }
        if (a.u_store) {
#pragma unroll
            for (int i = 0; i < EPT; ++i)
                if (ok[i]) a.u_store[e[i]] = u[i];
        }
    }
    if constexpr (!CLEAR_EARLY && is_atomic(MODE) && AGG > 0) agg_clear(*tab);
    // Phase 3: nonlinearity, objective terms and local adjoints (selects,
    // not products with zero, keep the lanes past `end` out even where their
    // values are not finite).
    double tsum = 0.0;
    double v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const double s = u[i], s2 = s * s;
        const double wd = to_f64(wv[i]);
        if constexpr (has_obj(MODE)) tsum += ok[i] ? wd * psi_from_sq(s2) : 0.0;
        if constexpr (has_rev(MODE)) v[i] = ok[i] ? fb * wd * dpsi_from(s, s2) : 0.0;
        if constexpr (MODE == M_HVP || MODE == M_JVP) {
            double q = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) q += to_f64(b[i][j]) * to_f64(dv[i][j]);
            if constexpr (MODE == M_HVP) v[i] = ok[i] ? wd * ddpsi_from_sq(s2) * q : 0.0;
            if constexpr (MODE == M_JVP) tsum += ok[i] ? wd * dpsi_from(s, s2) * q : 0.0;
        }
    }
    // Phase 4: the reverse scatter.
    double* __restrict__ G = a.gacc ? a.gacc + noff : nullptr;
    if constexpr (writes_v(MODE)) {
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if (ok[i]) a.v_out[e[i]] = v[i];
    }
    if constexpr (is_atomic(MODE) && AGG > 0) {
        __syncthreads();  // the table is clear
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if (ok[i]) {
                int32_t nn[K];
                double cc[K];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    nn[j] = (int32_t)(noff + c[i][j]);
                    cc[j] = v[i] * to_f64(b[i][j]);
                }
                agg_add_row<K, AGG>(*tab, nn, cc, a.gacc, a.hash_shift);
            }
        __syncthreads();
        agg_flush(*tab, a.gacc);
        __syncthreads();
    } else if constexpr (is_atomic(MODE)) {
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if (ok[i]) {
#pragma unroll
                for (int j = 0; j < K; ++j) atomic_add_f64(G + c[i][j], v[i] * to_f64(b[i][j]));
            }
    }
    if constexpr (is_colour(MODE)) {
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if (ok[i]) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    double* g = G + c[i][j];
                    *g = *g + v[i] * to_f64(b[i][j]);
                }
            }
    }
    return tsum;
}

template <typename T, int K, int MODE, int EPT, int AGG, bool CLEAR_EARLY = true>
__device__ __forceinline__ double elem_tile(const TileArgs& a, int64_t first, int64_t end,
                                            int64_t noff, double fb, AggOf<AGG>* tab) {
    // Only the adjoint-only modes can be handed stored forward values; the
    // others take the gather path with no branch at all (a runtime branch
    // between the two bodies in one kernel again made the compiler wait for
    // every row load before the gather).
    if constexpr (!has_obj(MODE) && MODE != M_HVP && MODE != M_JVP)
        if (a.u_in)
            return elem_tile_body<T, K, MODE, EPT, AGG, true, CLEAR_EARLY>(a, first, end, noff, fb,
                                                                           tab);
    return elem_tile_body<T, K, MODE, EPT, AGG, false, CLEAR_EARLY>(a, first, end, noff, fb, tab);
}

}  // namespace pg
