// Persistent, software-pipelined element pass with an LDS-combined atomic
// scatter, shared by the single-mesh and mesh-batch launchers.
//
// A grid sized to the device's resident capacity walks the tiles (logical
// workgroup l, XCD-remapped, takes tiles l, l + grid, ...).  For each tile it
//   1. issues the row loads (conn, B, w) of its NEXT tile,
//   2. gathers x and evaluates psi / psi' for the current tile,
//   3. adds the tile's contributions per node into the LDS table,
//   4. flushes the table with one global atomic per distinct node, resetting
//      each slot as it reads it (so the table is cleared once per workgroup,
//      not once per tile),
//   5. reduces the tile's objective terms into the tile's partial slot.
// The next tile's loads are in flight while steps 2-5 of the current one run.
#pragma once

#include "elem_tile.hpp"

namespace pg {

struct TileDesc {
    int64_t first, end, noff, slot, inst;
    uint32_t shift;
};

// One mesh: tile t = elements [t*span, min(E, (t+1)*span)), partial slot t.
struct MeshTiles {
    int64_t n_elems, span, n;
    uint32_t shift;
    __device__ __forceinline__ TileDesc get(int64_t t) const {
        const int64_t f = t * span;
        return TileDesc{f, f + span < n_elems ? f + span : n_elems, 0, t, 0, shift};
    }
};

// A batch: packed records {first, end, (hash shift << 40) | node offset,
// (instance << 40) | slot}.
struct BatchTiles {
    const int64_t* rec;
    int64_t n;
    __device__ __forceinline__ TileDesc get(int64_t t) const {
        const longlong2* p = reinterpret_cast<const longlong2*>(rec + 4 * t);
        const longlong2 a = p[0], b = p[1];
        constexpr int64_t lo = (1LL << 40) - 1;
        return TileDesc{a.x, a.y, b.x & lo, b.y & lo, b.y >> 40, (uint32_t)(b.x >> 40)};
    }
};

template <typename T, int K>
struct RowRegs {
    int32_t c[K];
    T b[K];
    T w;
    int64_t e;
    bool ok;
};

template <typename T, int K>
__device__ __forceinline__ void load_rows(RowRegs<T, K>& r, const TileArgs& a, const TileDesc& d) {
    r.e = d.first + threadIdx.x;
    r.ok = r.e < d.end;
    if (r.ok) {
        load_conn_row<T, K>(a.conn, r.e, r.c);
        load_b_row<K>(static_cast<const T*>(a.B), r.e, r.b);
        r.w = static_cast<const T*>(a.w)[r.e];
    }
}

// MODE: M_GRAD_ATOMIC or M_ADJ_ATOMIC.  fbar: nullptr (seed 1), one seed, or
// one seed per instance (fbar_per_inst).
template <typename T, int K, int MODE, class Tiles>
__global__ void __launch_bounds__(1024)
k_atomic_persistent(Tiles tiles, TileArgs a, const double* fbar, int fbar_per_inst,
                    double* partials) {
    __shared__ double lds[16];
    __shared__ AggTable tab;
    agg_clear(tab);
    __syncthreads();
    const int64_t G = gridDim.x;
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    RowRegs<T, K> cur, nxt;
    TileDesc dc{}, dn{};
    if (t < tiles.n) {
        dc = tiles.get(t);
        load_rows<T, K>(cur, a, dc);
    }
    for (; t < tiles.n; t += G) {
        if (t + G < tiles.n) {
            dn = tiles.get(t + G);
            load_rows<T, K>(nxt, a, dn);
        }
        const T* __restrict__ X = static_cast<const T*>(a.x) + dc.noff;
        double u = 0.0;
        if (a.u_in) {
            if (cur.ok) u = a.u_in[cur.e];
        } else if (cur.ok) {
            T xv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) xv[j] = X[cur.c[j]];
#pragma unroll
            for (int j = 0; j < K; ++j) u += to_f64(cur.b[j]) * to_f64(xv[j]);
        }
        const double s2 = u * u, wd = cur.ok ? to_f64(cur.w) : 0.0;
        double tsum = 0.0;
        if constexpr (MODE == M_GRAD_ATOMIC) tsum = wd * psi_from_sq(s2);
        const double fb = fbar ? fbar[fbar_per_inst ? dc.inst : 0] : 1.0;
        const double v = fb * wd * dpsi_from(u, s2);
        if (cur.ok) {
            int32_t nn[K];
            double cc[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                nn[j] = (int32_t)(dc.noff + cur.c[j]);
                cc[j] = v * to_f64(cur.b[j]);
            }
            agg_add_row<K>(tab, nn, cc, a.gacc, dc.shift);
        }
        __syncthreads();
        for (int s = threadIdx.x; s < kAggSlots; s += blockDim.x) {
            const int32_t n = tab.key[s];
            if (n >= 0) {
                atomic_add_f64(a.gacc + n, tab.val[s]);
                tab.key[s] = -1;
                tab.val[s] = 0.0;
            }
        }
        if constexpr (MODE == M_GRAD_ATOMIC) {
            const double s = block_sum_dyn(tsum, lds);  // its barriers also end the flush
            if (threadIdx.x == 0) partials[dc.slot] = s;
        } else {
            __syncthreads();
        }
        cur = nxt;
        dc = dn;
    }
}

// Workgroups that fit on the device at once for this kernel, capped by the tiles.
template <typename Kern>
unsigned resident_grid(Kern kern, int block, int64_t n_tiles, int cap) {
    int dev = 0, cus = 256, occ = 1;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, 0) != hipSuccess || occ < 1)
        occ = 1;
    int64_t g = (int64_t)cus * occ;
    if (cap > 0 && g > cap) g = cap;
    if (g > n_tiles) g = n_tiles;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace pg
