// Kernels of composed programs.  Non-pointwise constructs (stencil, gather,
// scan) run one kernel each way; chains of pointwise constructs run as fused
// groups (k_group), which recompute their forward values in registers in the
// reverse pass instead of reading them from a tape.  Shadows are FP64; a
// shadow's first contribution in the reverse pass stores, later ones add
// (the generated code of section 4 zeroes every shadow and adds).
#include <algorithm>

#include "device_common.hpp"
#include "elem_tile.hpp"
#include "launch.hpp"

namespace pg {

namespace {

constexpr int kBS = 256;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

__device__ __forceinline__ double map_f(int fn, double s) {
    return fn == 0 ? s * s : psi_from_sq(s * s);
}
__device__ __forceinline__ double map_df(int fn, double s) {
    return fn == 0 ? 2.0 * s : dpsi_from(s, s * s);
}

__global__ void __launch_bounds__(kBS)
k_stencil(int64_t n, const double* __restrict__ a, ProgTaps taps, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < taps.n; ++t) {
        const int64_t j = i + taps.off[t];
        if (j >= 0 && j < n) s += taps.coef[t] * a[j];
    }
    y[i] = s;
}

// ---------------------------------------------------------- reverse pass

// The reverse of a stencil reads ybar through several index expressions; it
// is rescheduled by the written index: abar_j += sum_t c_t ybar_{j - o_t}.
__global__ void __launch_bounds__(kBS)
k_r_stencil(int64_t n, const double* __restrict__ yb, ProgTaps taps, double* __restrict__ ab,
            int accumulate) {
    const int64_t j = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int t = 0; t < taps.n; ++t) {
        const int64_t i = j - taps.off[t];
        if (i >= 0 && i < n) s += taps.coef[t] * yb[i];
    }
    if (accumulate)
        ab[j] += s;
    else
        ab[j] = s;
}

// ------------------------------------------------------------ prefix scan
//
// Inclusive scan in three launches over chunks of kScanItems entries: chunk
// totals, an exclusive scan of the totals by one workgroup, then each chunk's
// local scan offset by its prefix.  With rev set, entry i is read and written
// at n-1-i, which turns the prefix scan into the suffix scan of the reverse
// pass: abar_j += sum_{i >= j} ybar_i.  Summation order is fixed.

constexpr int kScanPer = 8;
constexpr int kScanItems = kBS * kScanPer;

__device__ __forceinline__ int64_t scan_at(int64_t n, int64_t i, int rev) { return rev ? n - 1 - i : i; }

// Exclusive scan of one value per thread over the workgroup; *total gets the sum.
__device__ __forceinline__ double block_excl_scan(double v, double* lds, double* total) {
    constexpr int NW = kBS / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double t = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += t;
    }
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const double t = lds[i];
        if (i < w) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + (inc - v);
}

__global__ void __launch_bounds__(kBS)
k_scan_totals(int64_t n, const double* __restrict__ a, int rev, double* __restrict__ totals) {
    __shared__ double lds[kBS / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (base + q < n) s += a[scan_at(n, base + q, rev)];
    const double t = block_sum<kBS>(s, lds);
    if (threadIdx.x == 0) totals[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBS)
k_scan_top(int64_t nchunks, double* __restrict__ totals) {
    __shared__ double lds[kBS / kWave];
    double carry = 0.0;
    for (int64_t b = 0; b < nchunks; b += kBS) {
        const int64_t i = b + threadIdx.x;
        const double v = i < nchunks ? totals[i] : 0.0;
        double tot;
        const double ex = block_excl_scan(v, lds, &tot);
        if (i < nchunks) totals[i] = carry + ex;
        carry += tot;
    }
}

// accumulate 0: y = scan; 1: y += scan.
__global__ void __launch_bounds__(kBS)
k_scan_apply(int64_t n, const double* __restrict__ a, int rev, const double* __restrict__ prefix,
             double* __restrict__ y, int accumulate) {
    __shared__ double lds[kBS / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
    double v[kScanPer];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = base + q < n ? a[scan_at(n, base + q, rev)] : 0.0;
        s += v[q];
    }
    double tot;
    double run = prefix[blockIdx.x] + block_excl_scan(s, lds, &tot);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        run += v[q];
        if (base + q < n) {
            const int64_t j = scan_at(n, base + q, rev);
            if (accumulate)
                y[j] += run;
            else
                y[j] = run;
        }
    }
}

hipError_t launch_scan(int64_t n, const double* a, int rev, double* scratch, double* y,
                       int accumulate, hipStream_t s) {
    const int64_t nchunks = (n + kScanItems - 1) / kScanItems;
    hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nchunks), dim3(kBS), 0, s, n, a, rev, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBS), 0, s, nchunks, scratch);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(kBS), 0, s, n, a, rev, scratch,
                       y, accumulate);
    return hipGetLastError();
}

// ------------------------------------------- segment sum and broadcast
//
// One 64-lane wave per segment, four segments per workgroup.  The segment
// sum reduces lane-strided partial sums with a fixed butterfly
// (deterministic); its reverse, and the broadcast, write each entry of the
// segment from the segment's value; the broadcast's reverse is the segment
// sum of the output shadow.

constexpr int kSegPerBlock = kBS / kWave;

__global__ void __launch_bounds__(kBS)
k_segsum(int64_t n_seg, const int64_t* __restrict__ offs, const double* __restrict__ a,
         double* __restrict__ y, int accumulate) {
    const int64_t s = (int64_t)blockIdx.x * kSegPerBlock + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (s >= n_seg) return;  // whole waves leave together
    const int64_t b = offs[s], e = offs[s + 1];
    double t = 0.0;
    for (int64_t i = b + lane; i < e; i += kWave) t += a[i];
    t = wave_sum(t);
    if (lane == 0) {
        if (accumulate)
            y[s] += t;
        else
            y[s] = t;
    }
}

__global__ void __launch_bounds__(kBS)
k_segbcast(int64_t n_seg, const int64_t* __restrict__ offs, const double* __restrict__ a,
           double* __restrict__ y, int accumulate) {
    const int64_t s = (int64_t)blockIdx.x * kSegPerBlock + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (s >= n_seg) return;
    const int64_t b = offs[s], e = offs[s + 1];
    const double v = a[s];
    for (int64_t i = b + lane; i < e; i += kWave) {
        if (accumulate)
            y[i] += v;
        else
            y[i] = v;
    }
}

__global__ void __launch_bounds__(kBS)
k_validate_offsets(const int64_t* __restrict__ offs, int64_t n_seg, int64_t n, int32_t* flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s <= n_seg; s += stride) {
        const int64_t o = offs[s];
        if (s == 0 && o != 0) bad = 1;
        if (s == n_seg && o != n) bad = 1;
        if (s < n_seg && offs[s + 1] < o) bad = 1;
        if (o < 0 || o > n) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

inline unsigned seg_blocks(int64_t n_seg) { return (unsigned)((n_seg + kSegPerBlock - 1) / kSegPerBlock); }

// ------------------------------------------------------------ fused groups

// NS FP64 slots addressed by a wave-uniform index.  A private array indexed
// at run time would live in scratch memory; here every access is a switch on
// the uniform index whose cases use constant indices, so the slots stay in
// VGPRs and an access costs a few scalar branches.  (Chains of selects over
// the slots measured twice as slow on the 128^3 mesh program.)  Launches
// pick the smallest NS (4, 8 or 16) that holds the group's leaves and ops.
#define PG_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)
template <int NS>
struct Slots {
    double r[NS];
    __device__ __forceinline__ Slots() {
#pragma unroll
        for (int q = 0; q < NS; ++q) r[q] = 0.0;
    }
    __device__ __forceinline__ double get(int i) const {
        switch (i) {
#define PG_GET(q) \
    case q:       \
        if constexpr (q < NS) return r[q < NS ? q : 0]; else return 0.0;
            PG_CASES(PG_GET)
#undef PG_GET
        }
        return 0.0;
    }
    __device__ __forceinline__ void set(int i, double v) {
        switch (i) {
#define PG_SET(q) \
    case q:       \
        if constexpr (q < NS) r[q < NS ? q : 0] = v; break;
            PG_CASES(PG_SET)
#undef PG_SET
        }
    }
    __device__ __forceinline__ void add(int i, double v) {
        switch (i) {
#define PG_ADD(q) \
    case q:       \
        if constexpr (q < NS) r[q < NS ? q : 0] += v; break;
            PG_CASES(PG_ADD)
#undef PG_ADD
        }
    }
};
#undef PG_CASES
static_assert(kGSlots == 16, "at most sixteen slots");

// Row of the fused gather: K > 0 keeps it in registers (vector loads);
// K < 0 is the generic row length, read again in the reverse scatter.
template <int K>
struct GatherRow {
    static constexpr int N = K > 0 ? K : 1;
    int32_t c[N];
    double b[N];
};

// K: fused gather row length (0 none, -1 generic); NS: slots; BS: workgroup;
// S: slots of the LDS table of the fused gather's scatter (0 without one).
template <int K, int MODE, int BS, int NS, int S>
__global__ void __launch_bounds__(BS) k_group(GroupDev g) {
    constexpr bool REV = MODE != G_FWD;
    constexpr bool FWD = MODE != G_REV;
    constexpr bool AGG = REV && K != 0;
    static_assert(AGG == (S > 0), "a table exactly when the reverse scatters a fused gather");
    constexpr int NL = NS < kGLeaves ? NS : kGLeaves;
    __shared__ double lds[BS / kWave];
    __shared__ int last_wg;
    __shared__ typename std::conditional<AGG, AggTableT<S>, int>::type tab;
    const bool scatter = AGG && g.gsrc_shadow != nullptr;
    const int64_t i = xcd_remap(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    const bool ok = i < g.n;
    const int L = g.n_leaves;
    Slots<NS> r;
    GatherRow<K> row;
    // The reverse of a group without ops (a gather of its own) is linear: it
    // needs the gather rows but no forward values.
    const bool values = FWD || g.n_ops > 0;
    if (ok) {
        // Every load first: the gather row, the gathered entries (issued as
        // soon as the row's connectivity is in: the leaves' loads sit behind
        // branches, and issued before the gather they made the gather wait
        // for B as well), then the leaves.
        double xv[K > 0 ? K : 1];
        if constexpr (K > 0) {
            load_conn_row<double, K>(g.gconn, i, row.c);
            load_b_row<K>(g.gB, i, row.b);
            if (values) {
#pragma unroll
                for (int j = 0; j < K; ++j) xv[j] = g.gsrc[row.c[j]];
            }
        }
#pragma unroll
        for (int l = 0; l < NL; ++l)
            if (l < L && l != g.gather_slot) r.r[l] = g.leaf[l][i];
        if (!values) {
        } else if constexpr (K > 0) {
            double u = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) u += row.b[j] * xv[j];
            r.set(g.gather_slot, u);
        } else if constexpr (K < 0) {
            double u = 0.0;
            for (int j = 0; j < g.gk; ++j) u += g.gB[i * g.gk + j] * g.gsrc[g.gconn[i * g.gk + j]];
            r.set(g.gather_slot, u);
        }
        (void)values;
        for (int j = 0; j < g.n_ops; ++j) {
            const GOp o = g.ops[j];
            const double x = r.get(o.a);
            double v;
            switch (o.kind) {
                case P_SCALE: v = o.alpha * x; break;
                case P_ADD: v = o.alpha * x + o.beta * r.get(o.b); break;
                case P_MUL: v = x * r.get(o.b); break;
                default: v = map_f(o.fn, x); break;
            }
            r.set(L + j, v);
        }
        if constexpr (FWD) {
            for (int x = 0; x < g.n_exports; ++x) g.export_val[x][i] = r.get(g.export_slot[x]);
        }
    }
    if constexpr (FWD) {
        if (g.sum_slot >= 0) {
            const double t = block_sum<BS>(ok ? r.get(g.sum_slot) : 0.0, lds);
            if (threadIdx.x == 0) g.partials[blockIdx.x] = t;
        }
    }
    if constexpr (REV) {
        Slots<NS> a;
        if (ok) {
            if (g.sum_slot >= 0) a.add(g.sum_slot, g.seed ? *g.seed : 1.0);
            for (int x = 0; x < g.n_exports; ++x)
                if (g.export_shadow[x]) a.add(g.export_slot[x], g.export_shadow[x][i]);
            for (int j = g.n_ops - 1; j >= 0; --j) {
                const GOp o = g.ops[j];
                const double yb = a.get(L + j);
                switch (o.kind) {
                    case P_SCALE: a.add(o.a, o.alpha * yb); break;
                    case P_ADD:
                        a.add(o.a, o.alpha * yb);
                        a.add(o.b, o.beta * yb);
                        break;
                    case P_MUL: {
                        const double av = r.get(o.a), bv = r.get(o.b);
                        a.add(o.a, bv * yb);
                        a.add(o.b, av * yb);
                        break;
                    }
                    default: a.add(o.a, map_df(o.fn, r.get(o.a)) * yb); break;
                }
            }
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                if (l >= L || l == g.gather_slot || !g.leaf_shadow[l]) continue;
                double* p = g.leaf_shadow[l] + i;
                if (g.leaf_acc[l])
                    *p += a.r[l];
                else
                    *p = a.r[l];
            }
        }
        if constexpr (AGG) {
            if (scatter) {
                // The table is cleared only now, so the loads above were not held up.
                agg_clear(tab);
                __syncthreads();
                if (ok) {
                    const double ub = a.get(g.gather_slot);
                    if constexpr (K > 0) {
                        double cc[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) cc[j] = row.b[j] * ub;
                        agg_add_row<K>(tab, row.c, cc, g.gsrc_shadow, g.hash_shift);
                    } else {
                        for (int j = 0; j < g.gk; ++j)
                            agg_add(tab, g.gconn[i * g.gk + j], g.gB[i * g.gk + j] * ub,
                                    g.gsrc_shadow, g.hash_shift);
                    }
                }
                __syncthreads();
                agg_flush(tab, g.gsrc_shadow);
            }
        }
    }
    if constexpr (FWD) {
        if (g.sum_slot >= 0 && g.ticket) {
            if (threadIdx.x == 0) {
                __threadfence();  // this workgroup's partial before its ticket
                last_wg = atomicAdd(g.ticket, 1) == (int)gridDim.x - 1;
            }
            __syncthreads();
            if (last_wg) {
                __threadfence();  // every partial is visible
                double v = 0.0;
                for (int q = threadIdx.x; q < (int)gridDim.x; q += BS) v += g.partials[q];
                v = block_sum<BS>(v, lds);
                if (threadIdx.x == 0) {
                    *g.f_out = v;
                    *g.ticket = 0;
                }
            }
        }
    }
}

template <int K, int NS>
hipError_t launch_group_k(const GroupDev& g, int mode, hipStream_t s) {
    constexpr int BS = kGroupBlock, BSS = K != 0 ? kGroupBlockScatter : kGroupBlock;
    constexpr int SB = K != 0 ? kAggSlots : 0, SS = K != 0 ? kAggSlotsSmall : 0;
    const dim3 grid((unsigned)group_blocks(g.n, BS)), block(BS);
    const dim3 grid_s((unsigned)group_blocks(g.n, BSS)), block_s(BSS);
    const bool small = g.agg_slots == kAggSlotsSmall;
    switch (mode) {
        case G_FWD: PG_LAUNCH((k_group<K, G_FWD, BS, NS, 0>), grid, block, 0, s, g); break;
        case G_REV:
            if (small)
                PG_LAUNCH((k_group<K, G_REV, BSS, NS, SS>), grid_s, block_s, 0, s, g);
            else
                PG_LAUNCH((k_group<K, G_REV, BSS, NS, SB>), grid_s, block_s, 0, s, g);
            break;
        default:
            if (small)
                PG_LAUNCH((k_group<K, G_FWDREV, BSS, NS, SS>), grid_s, block_s, 0, s, g);
            else
                PG_LAUNCH((k_group<K, G_FWDREV, BSS, NS, SB>), grid_s, block_s, 0, s, g);
            break;
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_group_ns(const GroupDev& g, int mode, hipStream_t s) {
    const int need = g.n_leaves + g.n_ops;
    if (need <= 4) return launch_group_k<K, 4>(g, mode, s);
    if (need <= 8) return launch_group_k<K, 8>(g, mode, s);
    return launch_group_k<K, 16>(g, mode, s);
}

}  // namespace

int64_t group_blocks(int64_t n, int bs) { return (n + bs - 1) / bs; }

// A group with a fused gather scatters through the LDS table in its reverse
// pass; a larger workgroup combines more contributions per table clear and
// flush (512 threads measured best for eight-node rows, as for the mesh).
int group_block_size(const GroupDev& g, int mode) {
    return (g.gather_slot >= 0 && mode != G_FWD) ? kGroupBlockScatter : kGroupBlock;
}

hipError_t launch_group(const GroupDev& g, int mode, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    if (g.n_leaves + g.n_ops > kGSlots || g.n_leaves > kGLeaves || g.n_ops > kGOps)
        return hipErrorInvalidValue;
    if (g.gather_slot < 0) return launch_group_ns<0>(g, mode, s);
    const bool vec = (reinterpret_cast<uintptr_t>(g.gconn) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(g.gB) % 16 == 0);
    if (vec) {
        switch (g.gk) {
            case 2: return launch_group_ns<2>(g, mode, s);
            case 3: return launch_group_ns<3>(g, mode, s);
            case 4: return launch_group_ns<4>(g, mode, s);
            case 8: return launch_group_ns<8>(g, mode, s);
            default: break;
        }
    }
    return launch_group_ns<-1>(g, mode, s);
}

hipError_t launch_prog_fwd(const ProgOpDev& o, hipStream_t s) {
    if (o.n == 0) return hipSuccess;
    switch (o.kind) {
        case P_STENCIL: hipLaunchKernelGGL(k_stencil, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.a, o.taps, o.y); break;
        case P_SCAN: return launch_scan(o.n, o.a, 0, o.scratch, o.y, 0, s);
        case P_SEGSUM:
            hipLaunchKernelGGL(k_segsum, dim3(seg_blocks(o.n_seg)), dim3(kBS), 0, s, o.n_seg, o.offs, o.a, o.y, 0);
            break;
        case P_BCAST:
            hipLaunchKernelGGL(k_segbcast, dim3(seg_blocks(o.n_seg)), dim3(kBS), 0, s, o.n_seg, o.offs, o.a, o.y, 0);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prog_rev(const ProgOpDev& o, hipStream_t s) {
    // a broadcast's reverse writes every segment's adjoint, even with no outputs
    if (o.kind == P_BCAST ? o.n_seg == 0 : o.n == 0) return hipSuccess;
    switch (o.kind) {
        case P_STENCIL: hipLaunchKernelGGL(k_r_stencil, dim3(nblocks(o.n)), dim3(kBS), 0, s, o.n, o.yb, o.taps, o.ab, o.accumulate); break;
        case P_SCAN: return launch_scan(o.n, o.yb, 1, o.scratch, o.ab, o.accumulate, s);
        case P_SEGSUM:  // reverse of a segment sum: broadcast of the output shadow
            hipLaunchKernelGGL(k_segbcast, dim3(seg_blocks(o.n_seg)), dim3(kBS), 0, s, o.n_seg, o.offs, o.yb, o.ab, o.accumulate);
            break;
        case P_BCAST:  // reverse of a broadcast: segment sum of the output shadow
            hipLaunchKernelGGL(k_segsum, dim3(seg_blocks(o.n_seg)), dim3(kBS), 0, s, o.n_seg, o.offs, o.yb, o.ab, o.accumulate);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t prog_scan_chunks(int64_t n) { return (n + kScanItems - 1) / kScanItems; }

hipError_t launch_validate_offsets(const int64_t* offs, int64_t n_seg, int64_t n, int32_t* flag,
                                   hipStream_t s) {
    const int64_t g = std::min<int64_t>((n_seg + kBS) / kBS, 4096);
    hipLaunchKernelGGL(k_validate_offsets, dim3((unsigned)g), dim3(kBS), 0, s, offs, n_seg, n, flag);
    return hipGetLastError();
}

}  // namespace pg
