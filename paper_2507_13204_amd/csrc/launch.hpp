// Internal host-side launchers of the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pg {

// Event pair armed by the timing hook for the next dominant-kernel launch.
// PG_LAUNCH hands it to hipExtLaunchKernelGGL, which stamps the events with
// the kernel's own start and end (no dispatch gap inside the pair), then
// disarms it; with nothing armed it is a plain launch.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& armed_launch_events();

}  // namespace pg

#define PG_LAUNCH(kernel, grid, block, shmem, stream, ...)                                       \
    do {                                                                                         \
        ::pg::LaunchEvents& ev_ = ::pg::armed_launch_events();                                   \
        if (ev_.start) {                                                                         \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0,    \
                                  __VA_ARGS__);                                                  \
            ev_ = ::pg::LaunchEvents{};                                                          \
        } else {                                                                                 \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                 \
        }                                                                                        \
    } while (0)

namespace pg {

enum Dtype { F64 = 0, F32 = 1 };

// ------------------------------------------------------------------ meshes

// What one element-parallel pass computes.
enum MeshMode {
    M_PRIMAL = 0,       // u_e, t_e = w_e psi(u_e), per-block partial sums of t
    M_GRAD_ATOMIC = 1,  // primal + v_e = fbar w_e psi'(u_e) scattered with atomics
    M_GRAD_V = 2,       // primal + v_e written out (for the node-parallel gather)
    M_ADJ_ATOMIC = 3,   // v_e scattered with atomics, no objective
    M_ADJ_V = 4,        // v_e written out, no objective
    M_HVP = 5,          // c_e = w_e psi''(u_e) (G d)_e scattered with atomics
    M_GRAD_COLOUR = 6,  // primal + v_e scattered with plain read-add-write
    M_ADJ_COLOUR = 7,   // v_e scattered with plain read-add-write, no objective
    M_JVP = 8           // forward tangent: per-block sums of w_e psi'(u_e) (G d)_e
};

struct MeshView {
    int64_t n_nodes = 0;
    int64_t n_elems = 0;
    int32_t k = 0;
    Dtype dtype = F64;
    const int32_t* conn = nullptr;
    const void* B = nullptr;
    const void* w = nullptr;
};

// Slot of node number u in an S-slot LDS combining table (S a power of two,
// 64 to 4096).  Node numbers are taken in blocks of 64; block b = u / 64 goes
// to slot block b + floor(b * rot / 4096) (wrapped), the node to the same
// place inside it.  So consecutive node numbers take consecutive slots (a
// whole block of 64 slots is skipped every 4096 / rot blocks, which keeps a
// wave's 64 lanes on 64 consecutive LDS banks and a flush instruction on few
// cache lines), and two runs of numbers a distance D apart land about
// D * (1 + rot / 4096) slots apart whatever their alignment: the plan picks
// rot (1 <= rot < 4096) so that the runs one workgroup touches (the node rows
// of neighbouring planes of a structured mesh, say) do not overlap.
// floor(b * rot / 4096) is taken as (b >> 12) * rot + ((b mod 4096) * rot >> 12)
// in 32-bit arithmetic.  The kernels and the plan's simulation of the table
// share this definition.
__host__ __device__ inline uint32_t agg_slot(uint32_t u, uint32_t rot, uint32_t S) {
    const uint32_t r = rot & 4095u, b = u >> 6;
    return (u + 64u * ((b >> 12) * r + (((b & 4095u) * r) >> 12))) & (S - 1);
}
constexpr uint32_t kHashRotDefault = 320;  // used where no plan has chosen one

struct MeshPass {
    const void* x = nullptr;       // node values (dtype)
    const void* xd = nullptr;      // direction for M_HVP (dtype)
    const double* u_in = nullptr;  // stored u (replaces the gather when set)
    double* u_store = nullptr;     // store u here when set
    double* v_out = nullptr;       // per-element v for M_*_V
    double* gacc = nullptr;        // FP64 accumulation target (atomic / colour modes)
    const double* fbar = nullptr;  // device seed (nullptr means 1)
    double* partials = nullptr;    // per-block partial sums of t
    const int32_t* elist = nullptr;  // element list (colour passes); nullptr = all
    int64_t elist_n = 0;
    int64_t partial_base = 0;      // first partial slot of this launch
    int block = 256;
    int ept = 1;
    int combine = 1;               // combine atomic contributions in LDS first
    uint32_t hash_shift = kHashRotDefault;  // LDS table hash parameter (see agg_slot)
    int agg_slots = 4096;          // LDS table size: 4096 or 2048 (see choose_hash_shift)
};

// Number of workgroups an element pass over n items launches.
int64_t mesh_blocks(int64_t n_items, int block, int ept);

// One launch per call for small single meshes (small_kernels.hip).  The
// scatter gathers in p.gacc (FP64, n_nodes entries, zero between calls).
// Nodes are split in ranges of kSmallRange; a workgroup that has scattered
// counts itself done on every range its elements touch (plus, for workgroup
// 0, every range no element touches), and the last workgroup done on a range
// writes grad there from p.gacc and clears p.gacc there.  The last workgroup
// to take the ticket sums the partials into f.
struct SmallPass {
    int32_t* ticket = nullptr;           // f's ticket, zero between calls
    int32_t* range_done = nullptr;       // per range, zero between calls
    const int32_t* range_need = nullptr; // per range: workgroups that count on it (>= 1)
    const int32_t* wg_off = nullptr;     // workgroup w's ranges: wg_list[wg_off[w] .. wg_off[w+1])
    const int32_t* wg_list = nullptr;
    void* grad = nullptr;       // gradient output (dtype), gradient modes
    double* f_out = nullptr;    // f, objective modes (may be null)
    int accumulate = 0;         // add into grad instead of overwriting it
};
constexpr int64_t kSmallMaxBlocks = 64;
constexpr int64_t kSmallMaxNodes = 16384;
constexpr int kSmallRange = 512;
constexpr int kSmallMaxRanges = (int)(kSmallMaxNodes / kSmallRange);
bool mesh_small_eligible(const MeshView& m, int block);
// mode: M_PRIMAL, M_GRAD_ATOMIC, M_ADJ_ATOMIC, M_HVP (scatters like the
// gradient) or M_JVP (sums like the objective).
hipError_t launch_mesh_small(const MeshView& m, MeshMode mode, const MeshPass& p,
                             const SmallPass& sp, hipStream_t s);

// Plan-time structures of the two-level deterministic adjoint (tiled_kernels.hip):
// tile t = elements [t * tile, (t + 1) * tile); its local nodes are the
// distinct nodes it touches, in ascending order, with staging slots
// tbase[t] .. tbase[t+1]-1; loff (tile t's entries at t * lstride, int16,
// tile-relative) holds, per local node, the range of its incidences in lidx
// (tile-relative positions e_local * k + j, ascending); noff / npos list, per
// node, its staging slots in ascending tile order.
struct TiledView {
    int64_t n_tiles = 0;
    int tile = 0;
    int lstride = 0;  // tile * k + 8: room for nl + 1 offsets read as 16-byte chunks
    const int64_t* tbase = nullptr;
    const int16_t* loff = nullptr;
    const int16_t* lidx = nullptr;
    double* stage = nullptr;
    const int32_t* noff = nullptr;
    const int32_t* npos = nullptr;
    // Corner-round form of level 1 (0: the general form): slots per tile
    // (2048 or 4096; the tile is then at most 512 elements) and the slot hash
    // rotation, both chosen at bind; stage then holds n_tiles * round_slots
    // entries, tile t's at t * round_slots + slot.
    int round_slots = 0;
    uint32_t round_shift = 0;
};
int tiled_tile_elems(int block, int32_t k);
// Dynamic LDS of one level-1 workgroup: contributions, positions and offsets.
size_t tiled_lds_bytes(int tile, int32_t k);
// Level 1 (obj: with the objective partial per tile into p.partials) and level 2.
hipError_t launch_mesh_tiled(const MeshView& m, const MeshPass& p, const TiledView& tv, bool obj,
                             hipStream_t s);
hipError_t launch_node_tiled(const MeshView& m, const TiledView& tv, void* grad, int accumulate,
                             hipStream_t s);

hipError_t launch_mesh_elem(const MeshView& m, MeshMode mode, const MeshPass& p, hipStream_t s);

// Node-parallel gather of the reverse pass over the transposed connectivity:
// g[n] (+)= sum_{p in offs[n]..offs[n+1]} v[inc[p]/k] * B[inc[p]].
hipError_t launch_mesh_node_gather(const MeshView& m, const int32_t* offs, const int32_t* inc,
                                   const void* binc, const double* v, void* grad, int accumulate,
                                   int block, hipStream_t s);

// out[0] (=|+=) sum of partials[0..n) in a fixed order (one workgroup).
hipError_t launch_final_sum(const double* partials, int64_t n, double* out, hipStream_t s);

// Segmented: out[i] = sum partials[seg[i]..seg[i+1]) for i < nseg.
hipError_t launch_segmented_sum(const double* partials, const int64_t* seg, int64_t nseg,
                                double* out, hipStream_t s);

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// out[q] = B[idx[q]] for q < n (B's coefficients in incidence order).
hipError_t launch_gather_entries(const int32_t* idx, int64_t n, const void* B, bool f64, void* out,
                                 hipStream_t s);
// conn, B and w rows gathered into the order of `list` (n rows of k entries).
hipError_t launch_permute_rows(const int32_t* list, int64_t n, int32_t k, const int32_t* conn,
                               const void* B, const void* w, bool f64, int32_t* pconn, void* pB,
                               void* pw, hipStream_t s);

// dst (FP32) (=|+=) src (FP64); clear: src is zeroed as it is read.
hipError_t launch_f64_to_f32(double* src, float* dst, int64_t n, int accumulate, int clear,
                             hipStream_t s);
// The same conversion, and f_out[0] = the fixed-order sum of partials[0..np)
// (k_final_sum's order) from the first workgroup: one launch instead of two.
hipError_t launch_f64_to_f32_sum(double* src, float* dst, int64_t n, int accumulate, int clear,
                                 const double* partials, int64_t np, double* f_out, hipStream_t s);
// dst (FP64) += src (FP64).
hipError_t launch_add_f64(const double* src, double* dst, int64_t n, hipStream_t s);
// y = alpha[0] * x (n entries of dt; FP64 product, rounded once; y may alias x).
hipError_t launch_scale(Dtype dt, int64_t n, const double* alpha, const void* x, void* y,
                        hipStream_t s);

// Plan-time structures.
// flag |= 1 if any conn entry is outside [0, n_nodes); cnt[node] += 1 when cnt.
hipError_t launch_validate_count(const int32_t* conn, int64_t n_items, int64_t n_nodes,
                                 int32_t* cnt, int32_t* flag, hipStream_t s);
// For an element pass whose workgroup w takes elements [w * span, (w + 1) *
// span) (k node numbers each): *miss += the number of inserts, over all
// workgroups, that find another node in their home slot of an S-slot LDS
// table with hash rotation `shift` (S = 2048 or 4096).  Zero means no
// workgroup of the pass probes.
hipError_t launch_table_check(const int32_t* conn, int64_t n_elems, int32_t k, int64_t span,
                              uint32_t shift, int slots, int32_t* miss, hipStream_t s);
// Exclusive scan: out[0..n] with out[n] = total.  scratch holds
// scan_scratch_items(n) int64 values.
int64_t scan_scratch_items(int64_t n);
hipError_t launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int64_t* scratch,
                                 hipStream_t s);
// inc[cursor[conn[i]]++] = i, then each row of inc sorted ascending.
hipError_t launch_csr_fill_sort(const int32_t* conn, int64_t n_items, int64_t n_nodes,
                                const int32_t* offs, int32_t* cursor, int32_t* inc, hipStream_t s);

// ---------------------------------------------------------------- batches

struct BatchView {
    int32_t n_inst = 0;
    int32_t k = 0;
    Dtype dtype = F64;
    const int32_t* conn = nullptr;
    const void* B = nullptr;
    const void* w = nullptr;
    // Work list, one 32-byte record per tile in processing order:
    // {first element, one past the last element,
    //  (LDS hash shift << 40) | node offset of the instance,
    //  (instance << 40) | partial slot}.  Slots are laid out instance by
    // instance, so the segmented reduction sums each instance in order.
    const int64_t* tiles = nullptr;
    int64_t n_tiles = 0;
    int tile_elems = 0;                   // elements per tile
};

enum BatchMode { B_PRIMAL = 0, B_GRAD_ATOMIC = 1, B_ADJ_ATOMIC = 2 };

struct BatchPass {
    const void* x = nullptr;
    void* grad = nullptr;          // FP64 accumulation target
    const double* fbar = nullptr;  // per instance (nullptr means 1)
    double* partials = nullptr;    // one slot per tile
    const double* u_in = nullptr;
    double* u_store = nullptr;
    int block = 256;
    int combine = 1;               // combine atomic contributions per tile in LDS
};

hipError_t launch_batch(const BatchView& b, BatchMode mode, const BatchPass& p,
                                   hipStream_t s);

// The LDS table hash parameter for a connectivity: `tiles` holds, per sampled
// workgroup tile, the node numbers its elements touch (in element order);
// returns the candidate shift with the fewest simulated probe steps.
// LDS table choices from sampled workgroup tiles (node numbers each touches):
// the best hash rotation for an S-slot table (its simulated probe count in
// *cost_out when not null), and, for single meshes, the table size too.
uint32_t choose_hash_shift(const int32_t* const* tiles, const int64_t* counts, int64_t n_tiles,
                           int slots, int64_t* cost_out);
void choose_table(const int32_t* const* tiles, const int64_t* counts, int64_t n_tiles, int* slots,
                  uint32_t* shift);

// ------------------------------------------------------------------ dense

struct DenseView {
    int64_t rows = 0, cols = 0;
    Dtype dtype = F64;
    const void* A = nullptr;
    const void* w = nullptr;
};

// Fused single pass over A: per row r_i = A_i . x (workgroup reduction),
// t_i, v_i = fbar w_i psi'(r_i); colpart[g, :] = sum over the rows of
// workgroup g of v_i A_i.  partials[g] = sum of t over its rows.
// Returns hipErrorInvalidValue if cols exceed the register-resident limit.
int64_t dense_fused_max_cols();
hipError_t launch_dense_fused(const DenseView& d, const void* x, const double* fbar, int want_grad,
                              double* partials, double* colpart, int ngroups, hipStream_t s);
// grad[j] (=|+=) sum_g colpart[g, j] in fixed order (dtype of grad).
hipError_t launch_dense_colsum(const double* colpart, int ngroups, int64_t cols, void* grad,
                               Dtype dt, int accumulate, hipStream_t s);
// Two-pass fallback: r = A x per row (one workgroup per row), v stored.
hipError_t launch_dense_rows(const DenseView& d, const void* x, const double* fbar,
                             double* partials, double* v, hipStream_t s);
// grad (=|+=) A^T v (column-parallel).
hipError_t launch_dense_cols(const DenseView& d, const double* v, void* grad, int accumulate,
                             hipStream_t s);

// --------------------------------------------------------- batched dense

struct BDenseView {
    int64_t m = 0, n = 0;
    Dtype dtype = F64;
    const void* A = nullptr;
    const void* W = nullptr;
};

// Forward: Y = A X on the matrix cores with the epilogue
// t = W psi(Y) (per-tile partial sums) and, when V != nullptr,
// V = W psi'(Y) (FP64 or dtype per vdt).
int64_t bdense_fwd_tiles(int64_t m, int64_t n);
hipError_t launch_bdense_fwd(const BDenseView& b, const void* X, double* partials, void* V,
                             hipStream_t s);
// Backward: G (=|+=) fbar * A^T V.
hipError_t launch_bdense_bwd(const BDenseView& b, const void* V, const double* fbar, void* G,
                             int accumulate, hipStream_t s);

}  // namespace pg

namespace pg {

// ------------------------------------------- the paper's section 4 example

// mode 0: objective; 1: gradient (gather form, writes gx / gb of dtype);
// 2: gradient (atomic form: FP64 atomics into gx64, which must be zeroed
// or hold the values to add to; gb of dtype).  partials: one per 256 nodes.
// When laplace1d_fused(n) the launch also writes f to f_out (if not null)
// through the zero-initialised ticket; otherwise the caller sums the partials.
int64_t laplace1d_blocks(int64_t n);
bool laplace1d_fused(int64_t n);
hipError_t launch_laplace1d(int64_t n, Dtype dt, int mode, const void* x, const void* b,
                            double* gx64, void* gx, void* gb, const double* fbar,
                            double* partials, int accumulate, int32_t* ticket, double* f_out,
                            hipStream_t s);

}  // namespace pg

namespace pg {

// ------------------------------------------------------- composed programs

enum ProgKind { P_INPUT = 0, P_CONST = 1, P_SCALE, P_STENCIL, P_GATHER, P_ADD, P_MUL, P_MAP, P_SUM, P_SCAN,
                P_SEGSUM, P_BCAST };

constexpr int kMaxTaps = 16;

struct ProgTaps {
    int32_t n = 0;
    int32_t off[kMaxTaps] = {};
    double coef[kMaxTaps] = {};
};

// One stand-alone non-pointwise construct (stencil, scan, segment sum,
// broadcast; gathers run as group kernels) as its kernels see it.
// Forward: y = op(a) over n outputs.  Reverse: ab receives the adjoint of
// the output shadow yb, stored (accumulate 0) or added (accumulate 1).
// The scan uses scratch (prog_scan_chunks(n) doubles) for
// its chunk totals.  Segment sum and broadcast take segment offsets offs
// (n_seg + 1 entries): the sum has n = n_seg outputs, the broadcast n =
// offs[n_seg].
struct ProgOpDev {
    int kind = 0;
    int64_t n = 0;
    const double* a = nullptr;
    double* y = nullptr;
    ProgTaps taps;
    const double* yb = nullptr;
    double* ab = nullptr;
    int accumulate = 1;
    double* scratch = nullptr;
    const int64_t* offs = nullptr;
    int64_t n_seg = 0;
};

hipError_t launch_prog_fwd(const ProgOpDev& o, hipStream_t s);
hipError_t launch_prog_rev(const ProgOpDev& o, hipStream_t s);
int64_t prog_scan_chunks(int64_t n);
// Sets *flag nonzero unless offs[0] == 0, offs is non-decreasing and
// offs[n_seg] == n.
hipError_t launch_validate_offsets(const int64_t* offs, int64_t n_seg, int64_t n, int32_t* flag,
                                   hipStream_t s);

// A fused group: a chain of pointwise constructs (scale, add, mul, map) over
// one index range, evaluated per entry in registers.  Slots 0..n_leaves-1
// hold the leaves (views read from outside the group, or the output of one
// fused gather); op j writes slot n_leaves + j.  Forward: exported slots are
// written to memory and the summed slot is reduced into per-workgroup
// partials.  Reverse: the forward slots are recomputed from the leaves, the
// adjoints start from the export shadows and the seed of the sum, run
// through the ops in reverse order, and leave through the leaf shadows
// (stored or added) and, for a fused gather, through an LDS-combined atomic
// scatter into the gather operand's shadow.
constexpr int kGSlots = 16, kGLeaves = 8, kGOps = 12, kGExports = 8;

struct GOp {
    int32_t kind = 0, a = 0, b = 0, fn = 0;
    double alpha = 1.0, beta = 1.0;
};

struct GroupDev {
    int64_t n = 0;
    int32_t n_leaves = 0, n_ops = 0, n_exports = 0;
    int32_t sum_slot = -1;
    int32_t gather_slot = -1;
    int32_t gk = 0;
    const int32_t* gconn = nullptr;
    const double* gB = nullptr;
    const double* gsrc = nullptr;
    double* gsrc_shadow = nullptr;
    uint32_t hash_shift = kHashRotDefault;
    int agg_slots = 4096;  // LDS table of the fused gather's scatter: 4096 or 2048
    const double* seed = nullptr;  // device seed of f (nullptr means 1)
    const double* leaf[kGLeaves] = {};
    double* leaf_shadow[kGLeaves] = {};
    int32_t leaf_acc[kGLeaves] = {};
    GOp ops[kGOps];
    int32_t export_slot[kGExports] = {};
    double* export_val[kGExports] = {};
    const double* export_shadow[kGExports] = {};
    double* partials = nullptr;
    // Sum group of a small grid: the last workgroup to take the ticket (zero
    // between launches; re-armed by that workgroup) sums the partials into f.
    int32_t* ticket = nullptr;
    double* f_out = nullptr;
};

enum GroupMode { G_FWD = 0, G_REV = 1, G_FWDREV = 2 };

// Workgroup size of a group launch (the number of sum partials it writes is
// group_blocks(n, group_block_size(g, mode))).
constexpr int kGroupBlock = 256, kGroupBlockScatter = 512;
hipError_t launch_group(const GroupDev& g, int mode, hipStream_t s);
int64_t group_blocks(int64_t n, int bs);
int group_block_size(const GroupDev& g, int mode);

}  // namespace pg
