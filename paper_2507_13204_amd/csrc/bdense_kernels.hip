// Batched dense objective on the matrix cores:
//   forward   Y = A X,  f = sum W (.) psi(Y)  (epilogue),  V = W (.) psi'(Y)
//   backward  G = fbar * A^T V
//
// Both products are m x m by m x n contractions, tiled 128 x 128 x 16 per
// workgroup of 16 (FP64) or 8 (FP32) waves; each wave owns a 64 x 16 or
// 64 x 32 block of C as MFMA 16x16x4 accumulators (FP64: v_mfma_f64_16x16x4_f64; FP32:
// v_mfma_f32_16x16x4_f32, whose accumulation inside the instruction is FP32, so
// the FP32 path adds each 16-deep k-tile's result into FP64 accumulators and
// restarts the matrix-core accumulators from zero: FP32 sums stay 16 terms
// long, every longer accumulation is FP64).
// Tiles are staged k-major in LDS (double buffered, the next tile prefetched
// into registers while the current one feeds the matrix cores).  The
// nonlinearity and its derivative are fused into the forward epilogue, so
// neither Y nor psi(Y) round-trips through HBM; the objective is reduced per
// tile and then in a fixed order (deterministic).
#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace pg {

namespace {

constexpr int BM = 128, BN = 128, BK = 16;
// Workgroup shape per element type: the waves tile the 128 x 128 block as
// 2 x WAVES_N blocks of 64 x WN, each wave holding 4 x NY MFMA accumulators.
// One workgroup per compute unit at the benchmark's shape (256 tiles), so
// more waves per workgroup is what hides the load and LDS latency: FP64
// uses 16 waves (measured 0.70 -> 0.56 ms from 4 waves), FP32 8 (its
// 16-byte loads need at least four elements per thread and operand).
template <typename T>
struct Cfg {
    static constexpr int NTHR = sizeof(T) == 8 ? 1024 : 512;
    static constexpr int WAVES_N = NTHR / 128, WN = BN / WAVES_N, NY = WN / 16;
    static constexpr int kPerThread = BM * BK / NTHR;  // elements of each operand tile per thread
};
constexpr int PAD = 4;  // LDS row padding (elements) against bank conflicts on transposed stores

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    using acc_t = d4;
    __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static double get(const acc_t& c, int r) { return c[r]; }
    // Output row (within the 16 x 16 block) of register r in lanes 16*g .. 16*g+15.
    __device__ static int row(int g, int r) { return g + 4 * r; }
};

template <>
struct Mfma<float> {
    using acc_t = f4;
    __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static double get(const acc_t& c, int r) { return (double)c[r]; }
    __device__ static int row(int g, int r) { return 4 * g + r; }
};


enum Epi { EPI_FWD = 0, EPI_BWD = 1 };

// One k-tile of both operands staged in registers on its way to LDS.
template <typename T>
struct Stage {
    T a[Cfg<T>::kPerThread];
    T b[Cfg<T>::kPerThread];
};

// C[M x N] = op(A)[M x K] * Bm[K x N].
//   TRANS_A == false: op(A)[i][k] = A[i * lda + k]   (forward, A is m x m)
//   TRANS_A == true:  op(A)[i][k] = A[k * lda + i]   (backward, A^T)
// FULL: every tile is in bounds and rows are 16-byte aligned, so operands are
// read with 16-byte vector loads and no bounds checks.  The k loop keeps two
// tiles in flight in registers (loaded two steps ahead) on top of the LDS
// double buffer: at one workgroup per compute unit the matrix-core time of a
// k-step is shorter than the latency of its loads.
template <typename T, bool TRANS_A, int EPI, bool FULL>
__global__ void __launch_bounds__(Cfg<T>::NTHR)
k_gemm_mfma(const T* __restrict__ A, const T* __restrict__ Bm, int64_t M, int64_t N, int64_t K,
            const T* __restrict__ W, double* __restrict__ partials, T* __restrict__ Vout,
            const double* __restrict__ fbar, T* __restrict__ Gout, int accumulate) {
    using MF = Mfma<T>;
    using acc_t = typename MF::acc_t;
    constexpr int NTHR = Cfg<T>::NTHR, WAVES_N = Cfg<T>::WAVES_N, WN = Cfg<T>::WN, NY = Cfg<T>::NY;
    constexpr int kPerThread = Cfg<T>::kPerThread;
    // Vector width of the operand loads: 16 bytes, or fewer elements when a
    // thread moves fewer per tile.
    constexpr int VN = (int)(16 / sizeof(T)) < kPerThread ? (int)(16 / sizeof(T)) : kPerThread;
    constexpr int NV = kPerThread / VN;  // vectors per operand per thread
    static_assert(NV >= 1 && kPerThread % VN == 0, "16-byte loads need whole vectors per thread");
    static_assert(NY >= 1 && WN % 16 == 0, "each wave needs whole 16-column MFMA blocks");
    __shared__ T As[2][BK][BM + PAD];
    __shared__ T Bs[2][BK][BN + PAD];
    __shared__ double red[NTHR / kWave];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;  // wave's 64 x WN block within the tile
    const int64_t i0 = (int64_t)blockIdx.y * BM, j0 = (int64_t)blockIdx.x * BN;

    // Element q of this thread's share of a tile, as (i, k) of op(A) and (k, j) of B.
    auto a_coord = [&](int q, int& ii, int& kk) {
        if constexpr (FULL) {
            const int v = tid + NTHR * (q / VN), c = q % VN;
            if (TRANS_A) {
                kk = v / (BM / VN);
                ii = (v % (BM / VN)) * VN + c;
            } else {
                ii = v / (BK / VN);
                kk = (v % (BK / VN)) * VN + c;
            }
        } else {
            const int p = tid + NTHR * q;
            if (TRANS_A) {
                kk = p / BM;
                ii = p % BM;
            } else {
                ii = p / BK;
                kk = p % BK;
            }
        }
    };
    auto b_coord = [&](int q, int& kk, int& jj) {
        if constexpr (FULL) {
            const int v = tid + NTHR * (q / VN), c = q % VN;
            kk = v / (BN / VN);
            jj = (v % (BN / VN)) * VN + c;
        } else {
            const int p = tid + NTHR * q;
            kk = p / BN;
            jj = p % BN;
        }
    };
    auto gload = [&](Stage<T>& st, int64_t k0) {
        if constexpr (FULL) {
            typedef T V __attribute__((ext_vector_type(VN)));
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                int ii, kk, bk, bj;
                a_coord(v * VN, ii, kk);
                b_coord(v * VN, bk, bj);
                const T* pa = TRANS_A ? A + (k0 + kk) * K + (i0 + ii) : A + (i0 + ii) * K + (k0 + kk);
                const V va = *reinterpret_cast<const V*>(pa);
                const V vb = *reinterpret_cast<const V*>(Bm + (k0 + bk) * N + (j0 + bj));
#pragma unroll
                for (int c = 0; c < VN; ++c) {
                    st.a[v * VN + c] = va[c];
                    st.b[v * VN + c] = vb[c];
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                int ii, kk, bk, bj;
                a_coord(q, ii, kk);
                b_coord(q, bk, bj);
                const int64_t gi = i0 + ii, gk = k0 + kk;
                T va = T(0);
                if (gi < M && gk < K) va = TRANS_A ? A[gk * K + gi] : A[gi * K + gk];
                st.a[q] = va;
                const int64_t gk2 = k0 + bk, gj = j0 + bj;
                st.b[q] = (gk2 < K && gj < N) ? Bm[gk2 * N + gj] : T(0);
            }
        }
    };
    auto lstore = [&](const Stage<T>& st, int buf) {
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            int ii, kk, bk, bj;
            a_coord(q, ii, kk);
            b_coord(q, bk, bj);
            As[buf][kk][ii] = st.a[q];
            Bs[buf][bk][bj] = st.b[q];
        }
    };

    acc_t acc[4][NY];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NY; ++b) acc[a][b] = MF::zero();
    // FP32 operands: FP64 running sums of the per-k-tile MFMA results.
    constexpr bool kWide = std::is_same<T, float>::value;
    double wide[kWide ? 4 : 1][kWide ? NY : 1][4];
    if constexpr (kWide) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NY; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) wide[a][b][r] = 0.0;
    }
    auto fold = [&]() {
        if constexpr (kWide) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < NY; ++b) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) wide[a][b][r] += MF::get(acc[a][b], r);
                    acc[a][b] = MF::zero();
                }
        }
    };

    const int li = lane & 15, lk = lane >> 4;
    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            T a[4], b[NY];
#pragma unroll
            for (int x = 0; x < 4; ++x) a[x] = As[buf][ks * 4 + lk][wm * 64 + x * 16 + li];
#pragma unroll
            for (int y = 0; y < NY; ++y) b[y] = Bs[buf][ks * 4 + lk][wn * WN + y * 16 + li];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < NY; ++y) acc[x][y] = MF::mac(a[x], b[y], acc[x][y]);
        }
    };

    // Tile j lives in stage j % 2 and LDS buffer j % 2.
    const int64_t nk = (K + BK - 1) / BK;
    Stage<T> s0, s1;
    if (nk > 0) gload(s0, 0);
    if (nk > 1) gload(s1, BK);
    if (nk > 0) lstore(s0, 0);
    __syncthreads();
    for (int64_t t = 0; t < nk; t += 2) {
        // even step: compute tile t from buffer 0; tile t+1 waits in s1
        if (t + 2 < nk) gload(s0, (t + 2) * BK);
        compute(0);
        fold();
        if (t + 1 < nk) lstore(s1, 1);
        __syncthreads();
        if (t + 1 >= nk) break;
        // odd step: compute tile t+1 from buffer 1; tile t+2 waits in s0
        if (t + 3 < nk) gload(s1, (t + 3) * BK);
        compute(1);
        fold();
        if (t + 2 < nk) lstore(s0, 0);
        __syncthreads();
    }

    // Accumulator (x, y) register r of lane l holds C[row][col] with
    // col = y*16 + l%16 and row = x*16 + MF::row(l/16, r) inside the wave
    // block: the FP64 instruction interleaves rows across registers
    // (l/16 + 4r), the FP32 one keeps them in consecutive registers
    // (4(l/16) + r).
    double tsum = 0.0;
    const double fb = (EPI == EPI_BWD && fbar) ? fbar[0] : 1.0;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = i0 + wm * 64 + x * 16 + MF::row(lk, r);
                const int64_t gj = j0 + wn * WN + y * 16 + li;
                if (gi < M && gj < N) {
                    double c;
                    if constexpr (kWide)
                        c = wide[x][y][r];
                    else
                        c = MF::get(acc[x][y], r);
                    const int64_t o = gi * N + gj;
                    if constexpr (EPI == EPI_FWD) {
                        const double s2 = c * c, wv = to_f64(W[o]);
                        tsum += wv * psi_from_sq(s2);
                        if (Vout) Vout[o] = static_cast<T>(wv * dpsi_from(c, s2));
                    } else {
                        const double g = fb * c;
                        Gout[o] = accumulate ? static_cast<T>(to_f64(Gout[o]) + g) : static_cast<T>(g);
                    }
                }
            }
    if constexpr (EPI == EPI_FWD) {
        const double s = block_sum<NTHR>(tsum, red);
        if (tid == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

}  // namespace

int64_t bdense_fwd_tiles(int64_t m, int64_t n) { return ((m + BM - 1) / BM) * ((n + BN - 1) / BN); }

namespace {

// Vector path: whole tiles only, and the per-call operand (X or V) 16-byte
// aligned (A and W are checked when the plan is made).
bool full_tiles(const BDenseView& b, const void* op) {
    return b.m % BM == 0 && b.n % BN == 0 && b.m % BK == 0 && (uintptr_t)op % 16 == 0;
}

template <typename T, bool TRANS, int EPI>
void launch_gemm(const BDenseView& b, dim3 grid, hipStream_t s, const T* A, const T* Bm, const T* W,
                 double* partials, T* V, const double* fbar, T* G, int accumulate) {
    if (full_tiles(b, Bm))
        PG_LAUNCH((k_gemm_mfma<T, TRANS, EPI, true>), grid, dim3(Cfg<T>::NTHR), 0, s, A, Bm, b.m,
                           b.n, b.m, W, partials, V, fbar, G, accumulate);
    else
        PG_LAUNCH((k_gemm_mfma<T, TRANS, EPI, false>), grid, dim3(Cfg<T>::NTHR), 0, s, A, Bm, b.m,
                           b.n, b.m, W, partials, V, fbar, G, accumulate);
}

}  // namespace

hipError_t launch_bdense_fwd(const BDenseView& b, const void* X, double* partials, void* V,
                             hipStream_t s) {
    if (b.m == 0 || b.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((b.n + BN - 1) / BN), (unsigned)((b.m + BM - 1) / BM));
    if (b.dtype == F64)
        launch_gemm<double, false, EPI_FWD>(b, grid, s, (const double*)b.A, (const double*)X,
                                            (const double*)b.W, partials, (double*)V, nullptr,
                                            nullptr, 0);
    else
        launch_gemm<float, false, EPI_FWD>(b, grid, s, (const float*)b.A, (const float*)X,
                                           (const float*)b.W, partials, (float*)V, nullptr,
                                           nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_bdense_bwd(const BDenseView& b, const void* V, const double* fbar, void* G,
                             int accumulate, hipStream_t s) {
    if (b.m == 0 || b.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((b.n + BN - 1) / BN), (unsigned)((b.m + BM - 1) / BM));
    if (b.dtype == F64)
        launch_gemm<double, true, EPI_BWD>(b, grid, s, (const double*)b.A, (const double*)V, nullptr,
                                           nullptr, nullptr, fbar, (double*)G, accumulate);
    else
        launch_gemm<float, true, EPI_BWD>(b, grid, s, (const float*)b.A, (const float*)V, nullptr,
                                          nullptr, nullptr, fbar, (float*)G, accumulate);
    return hipGetLastError();
}

}  // namespace pg
