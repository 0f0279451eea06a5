// C ABI of the gradient library: plan construction, argument validation,
// workspace layout and dispatch to the HIP kernels.  Host code only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "pgrad.h"
#include "launch.hpp"

using namespace pg;

namespace {

thread_local char g_err[512] = "";

pg_status fail(pg_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

}  // namespace

namespace pg {
// Shared with the other ABI translation units (composed programs).
pg_status set_error(pg_status s, const char* msg) {
    snprintf(g_err, sizeof g_err, "%s", msg);
    return s;
}
void clear_error() { g_err[0] = 0; }
}  // namespace pg

namespace {

#define PG_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) return fail(PG_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

enum Kind { K_MESH = 1, K_DENSE = 2, K_BDENSE = 3, K_BATCH = 4, K_LAPLACE = 5 };

constexpr size_t kAlign = PG_WORKSPACE_ALIGN;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t total = 0;
    size_t take(size_t bytes) {
        const size_t off = total;
        total += align_up(bytes);
        return off;
    }
};

size_t esize(pg_dtype d) { return d == PG_F64 ? 8 : 4; }

bool overlap(const void* a, size_t an, const void* b, size_t bn) {
    if (!a || !b || an == 0 || bn == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bn && b0 < a0 + an;
}

constexpr size_t NONE = ~size_t(0);

}  // namespace

namespace pg {

// Candidate parameters of the LDS table hash (agg_slot), tried in this order;
// the first that gives the sampled workgroups no probes is taken.
static const uint32_t kShiftCandidates[] = {256, 640, 384, 896, 160, 1152, 96, 1664,
                                            512, 2304, 200, 3000, 320, 1400, 768, 2600,
                                            48, 1800, 1024, 3500, 136, 450, 1300, 2048};
// Workgroups sampled per mesh (or per instance of a batch) to choose it.
constexpr int kHashSamples = 64;

// Probe count of an S-slot table with rotation `shift` on the sampled tiles
// (an insert that finds no slot within kProbe steps counts 4 * kProbe: it
// goes to a global atomic); stops early past `stop_at`.
int64_t table_cost(const int32_t* const* tiles, const int64_t* counts, int64_t n_tiles, int slots,
                   uint32_t shift, int64_t stop_at) {
    constexpr int kProbe = 64;
    std::vector<int32_t> key((size_t)slots);
    const uint32_t mask = (uint32_t)slots - 1;
    int64_t cost = 0;
    for (int64_t t = 0; t < n_tiles && cost < stop_at; ++t) {
        std::fill(key.begin(), key.end(), -1);
        for (int64_t q = 0; q < counts[t]; ++q) {
            const int32_t n = tiles[t][q];
            const uint32_t u = (uint32_t)n;
            uint32_t h = agg_slot(u, shift, (uint32_t)slots);
            int probe = 0;
            while (probe < kProbe && key[h] != -1 && key[h] != n) {
                h = (h + 1) & mask;
                ++probe;
            }
            if (probe == kProbe) {
                cost += 4 * kProbe;
            } else {
                key[h] = n;
                cost += probe;
            }
        }
    }
    return cost;
}

uint32_t choose_hash_shift(const int32_t* const* tiles, const int64_t* counts, int64_t n_tiles,
                           int slots, int64_t* cost_out) {
    uint32_t best = kShiftCandidates[0];
    int64_t best_cost = INT64_MAX;
    for (uint32_t cand : kShiftCandidates) {
        const int64_t cost = table_cost(tiles, counts, n_tiles, slots, cand, best_cost);
        if (cost < best_cost) {
            best_cost = cost;
            best = cand;
        }
        if (best_cost == 0) break;
    }
    if (cost_out) *cost_out = best_cost;
    return best;
}

void choose_table(const int32_t* const* tiles, const int64_t* counts, int64_t n_tiles, int* slots,
                  uint32_t* shift) {
    int64_t c_big = 0, c_small = 0;
    const uint32_t s_big = choose_hash_shift(tiles, counts, n_tiles, 4096, &c_big);
    const uint32_t s_small = choose_hash_shift(tiles, counts, n_tiles, 2048, &c_small);
    // A workgroup clears and flushes every slot of its table: the smaller
    // table saves 2048 slot visits per workgroup, worth it while its extra
    // probes stay below a quarter of that.
    const int64_t saved = n_tiles * 2048 / 4;
    if (n_tiles > 0 && c_small - c_big < saved) {
        *slots = 2048;
        *shift = s_small;
    } else {
        *slots = 4096;
        *shift = s_big;
    }
}

}  // namespace pg

struct pg_plan_s {
    Kind kind;
    pg_dtype dtype;
    pg_options opt;
    // mesh / batch
    MeshView mesh;
    int64_t mesh_blocks_n = 0;
    uint32_t hash_shift = kHashRotDefault;  // LDS table hash parameter chosen at bind time
    int agg_slots = 4096;        // LDS table size chosen at bind time
    // colour classes: elements of colour c are elist[colour_off[c] .. colour_off[c+1])
    std::vector<int64_t> colour_off;
    size_t o_elist = NONE;
    // colour-major copies of conn, B and w (rows class by class)
    size_t o_pconn = NONE, o_pB = NONE, o_pw = NONE;
    // batch
    BatchView batch;
    std::vector<pg_instance> inst;
    int64_t n_nodes_total = 0, n_elems_total = 0;
    std::vector<int64_t> h_tiles, h_seg;
    // dense
    DenseView dense;
    int dense_groups = 0;
    bool dense_fused = false;
    // the section 4 example
    int64_t lap_n = 0;
    bool lap_atomic = false;
    // batched dense
    BDenseView bd;
    int64_t bd_tiles = 0;
    // workspace
    size_t ws_bytes = 0;
    size_t o_partials = NONE, o_flag = NONE, o_u = NONE, o_v = NONE, o_offs = NONE,
           o_cursor = NONE, o_inc = NONE, o_binc = NONE, o_scan = NONE, o_gacc = NONE, o_colpart = NONE,
           o_tiles = NONE, o_vmat = NONE, o_tbase = NONE, o_loff = NONE, o_lidx = NONE,
           o_stage = NONE, o_noff = NONE, o_npos = NONE, o_small = NONE, o_ticket = NONE,
           o_small_meta = NONE;
    bool small = false;       // each call one launch (small_kernels.hip)
    int tiled_tile = 0;       // elements per tile of the two-level deterministic adjoint
    int64_t tiled_nt = 0;
    int tiled_round_slots = 0;      // corner-round level 1: slots per tile (0: general form)
    uint32_t tiled_round_shift = 0; // its slot hash rotation
    size_t n_partials = 0;
    char* ws = nullptr;
    bool bound = false;
    bool tape_valid = false;
    const void* tape_x = nullptr;
    size_t tape_bytes = 0;      // one call's tape (pg_tape_bytes)
    int64_t tape_budget = 0;    // what PG_CKPT_AUTO compared it against
    // measurement hook
    int32_t timing_mode = 0;
    std::vector<hipEvent_t> ev;  // pairs: ev[2i] start, ev[2i+1] stop
    int64_t ev_n = 0;

    template <typename P>
    P* at(size_t off) const {
        return off == NONE ? nullptr : reinterpret_cast<P*>(ws + off);
    }
};

namespace {

// 512 threads: with LDS combining of the atomic scatter this is the fastest
// element pass on a 128^3 hex mesh (four element rows per workgroup share
// their node rows in the LDS table); it is also the default elsewhere.
constexpr int kDefaultBlock = 512;

// Layout of the one-launch path's range tables (int32): range_done and
// range_need (kSmallMaxRanges each), wg_off (kSmallMaxBlocks + 1), wg_list
// (at most kSmallMaxRanges per workgroup).
constexpr int64_t small_meta_ints() {
    return 2 * kSmallMaxRanges + (kSmallMaxBlocks + 1) + kSmallMaxBlocks * kSmallMaxRanges;
}

// Entries per tile of the int16 local-node offsets: at most tile * k + 1 are
// used; the rest pads every tile to whole 16-byte chunks.
int tiled_stride(const pg_plan_s* p) { return p->tiled_tile * p->mesh.k + 8; }

pg_status check_opts(const pg_options* o, pg_options* out) {
    *out = pg_default_options();
    if (o) *out = *o;
    if (out->adjoint < PG_ADJ_AUTO || out->adjoint > PG_ADJ_TILED)
        return fail(PG_EINVAL, "options.adjoint %d is not a pg_adjoint_kind", out->adjoint);
    if (out->adjoint == PG_ADJ_AUTO) out->adjoint = PG_ADJ_ATOMIC;
    if (out->ckpt != PG_RECOMPUTE && out->ckpt != PG_STORE && out->ckpt != PG_CKPT_AUTO)
        return fail(PG_EINVAL, "options.ckpt %d is not a pg_ckpt", out->ckpt);
    if (out->reserved != 0) return fail(PG_EINVAL, "options.reserved must be 0");
    if (out->tape_budget < 0) return fail(PG_EINVAL, "options.tape_budget must be >= 0");
    if (out->block == 0) out->block = kDefaultBlock;
    if (out->block < 64 || out->block > 1024 || out->block % 64)
        return fail(PG_EINVAL, "options.block %d must be a multiple of 64 in [64, 1024]",
                    out->block);
    if (out->tile == 0) out->tile = 1;
    if (out->tile != 1 && out->tile != 2 && out->tile != 4)
        return fail(PG_EINVAL, "options.tile %d must be 1, 2 or 4", out->tile);
    if (out->accumulate != 0 && out->accumulate != 1)
        return fail(PG_EINVAL, "options.accumulate must be 0 or 1");
    if (out->scatter < 0 || out->scatter > 3)
        return fail(PG_EINVAL, "options.scatter must be 0, 1, 2 or 3");
    if (out->onepass != 0 && out->onepass != 1)
        return fail(PG_EINVAL, "options.onepass must be 0 or 1");
    return PG_OK;
}

pg_status check_dtype(pg_dtype d) {
    if (d != PG_F64 && d != PG_F32) return fail(PG_EDTYPE, "dtype %d is not PG_F64 or PG_F32", (int)d);
    return PG_OK;
}

bool k_in_registers(int32_t k) { return k == 2 || k == 4 || k == 8; }

pg_plan_s* new_plan(Kind kind, pg_dtype dt, const pg_options& o) {
    pg_plan_s* p = new (std::nothrow) pg_plan_s();
    if (!p) return nullptr;
    p->kind = kind;
    p->dtype = dt;
    p->opt = o;
    return p;
}

// PG_CKPT_AUTO: store the tape when one call's tape fits the budget (the
// caller's, or a quarter of the free device memory now), else recompute.
pg_status resolve_ckpt(pg_plan_s* p, size_t tape_bytes) {
    p->tape_bytes = tape_bytes;
    if (p->opt.ckpt != PG_CKPT_AUTO) return PG_OK;
    int64_t budget = p->opt.tape_budget;
    if (budget == 0) {
        size_t free_b = 0, total_b = 0;
        hipError_t e = hipMemGetInfo(&free_b, &total_b);
        if (e != hipSuccess) return fail(PG_EHIP, "hipMemGetInfo: %s", hipGetErrorString(e));
        budget = (int64_t)(free_b / 4);
    }
    p->tape_budget = budget;
    p->opt.ckpt = (tape_bytes > 0 && (int64_t)tape_bytes <= budget) ? PG_STORE : PG_RECOMPUTE;
    return PG_OK;
}

// Frees a plan that failed before it was handed to the caller.
pg_status drop_plan(pg_plan_s* p, pg_status st) {
    delete p;
    return st;
}

constexpr int kMaxColours = 64;

// ------------------------------------------------------------- mesh layout

void layout_mesh(pg_plan_s* p) {
    Layout L;
    const MeshView& m = p->mesh;
    const int ept = k_in_registers(m.k) ? p->opt.tile : 1;
    p->opt.tile = ept;
    p->mesh_blocks_n = mesh_blocks(m.n_elems, p->opt.block, ept);
    p->n_partials = (size_t)std::max<int64_t>(p->mesh_blocks_n, 1);
    p->small = p->opt.onepass == 0 && p->opt.adjoint == PG_ADJ_ATOMIC &&
               mesh_small_eligible(m, p->opt.block);
    if (p->small) {
        // one element per thread: the grid can exceed the tiled pass's
        p->n_partials = std::max<size_t>(p->n_partials, (size_t)mesh_blocks(m.n_elems, p->opt.block, 1));
        p->o_small = L.take(sizeof(double) * (size_t)m.n_nodes);
        p->o_ticket = L.take(sizeof(int32_t) * 4);
        // range_done, range_need, wg_off, wg_list
        p->o_small_meta = L.take(sizeof(int32_t) * (size_t)small_meta_ints());
    }
    p->o_partials = L.take(sizeof(double) * p->n_partials);
    p->o_flag = L.take(sizeof(int32_t) * 4);
    if (p->opt.ckpt == PG_STORE) p->o_u = L.take(sizeof(double) * (size_t)m.n_elems);
    if (p->opt.adjoint == PG_ADJ_GATHER) {
        p->o_v = L.take(sizeof(double) * (size_t)m.n_elems);
        p->o_offs = L.take(sizeof(int32_t) * (size_t)(m.n_nodes + 1));
        p->o_cursor = L.take(sizeof(int32_t) * (size_t)m.n_nodes);
        p->o_inc = L.take(sizeof(int32_t) * (size_t)(m.n_elems * m.k));
        // B's coefficients in incidence order (read as a stream by the node pass)
        p->o_binc = L.take(esize(p->dtype) * (size_t)(m.n_elems * m.k));
        p->o_scan = L.take(sizeof(int64_t) * (size_t)scan_scratch_items(m.n_nodes));
    }
    if (p->opt.adjoint == PG_ADJ_TILED) {
        // Sized for the worst case (every incidence its own local node); the
        // actual counts are known only at bind, from the connectivity.
        const int64_t inc = m.n_elems * m.k;
        p->tiled_tile = tiled_tile_elems(p->opt.block, m.k);
        p->tiled_nt = (m.n_elems + p->tiled_tile - 1) / p->tiled_tile;
        p->n_partials = (size_t)std::max<int64_t>(std::max<int64_t>(p->mesh_blocks_n, p->tiled_nt), 1);
        p->o_partials = L.take(sizeof(double) * p->n_partials);
        p->o_tbase = L.take(sizeof(int64_t) * (size_t)(p->tiled_nt + 1));
        p->o_loff = L.take(sizeof(int16_t) * (size_t)p->tiled_nt * (size_t)tiled_stride(p));
        p->o_lidx = L.take(sizeof(int16_t) * (size_t)std::max<int64_t>(inc, 1));
        // staging: the general form's partials (at most one per incidence) or
        // the corner-round form's tile * 4096 slots, whichever is larger
        p->o_stage = L.take(sizeof(double) *
                            (size_t)std::max<int64_t>(std::max<int64_t>(inc, p->tiled_nt * 4096), 1));
        p->o_noff = L.take(sizeof(int32_t) * (size_t)(m.n_nodes + 1));
        p->o_npos = L.take(sizeof(int32_t) * (size_t)std::max<int64_t>(inc, 1));
    }
    if (p->opt.adjoint == PG_ADJ_COLOUR) {
        // One extra partial slot per colour class (a class ends a workgroup early).
        p->n_partials = (size_t)std::max<int64_t>(p->mesh_blocks_n, 1) + kMaxColours;
        p->o_partials = L.take(sizeof(double) * p->n_partials);
        p->o_elist = L.take(sizeof(int32_t) * (size_t)m.n_elems);
        // Colour-major copies of the rows: a class's elements lie every other
        // element in the numbering, so reading them in place fetches lines
        // shared with the other classes; the copies are read contiguously.
        p->o_pconn = L.take(sizeof(int32_t) * (size_t)(m.n_elems * m.k));
        p->o_pB = L.take(esize(p->dtype) * (size_t)(m.n_elems * m.k));
        p->o_pw = L.take(esize(p->dtype) * (size_t)m.n_elems);
    }
    // FP32 gradients accumulate in an FP64 buffer before rounding once.
    if (p->dtype == PG_F32) p->o_gacc = L.take(sizeof(double) * (size_t)m.n_nodes);
    p->ws_bytes = L.total;
}

// ------------------------------------------------------------ batch layout

void layout_batch(pg_plan_s* p) {
    Layout L;
    const int te = p->opt.block * p->opt.tile;
    p->batch.tile_elems = te;
    // Work list: tiles of every instance, largest instance first (LPT), then
    // by instance index and tile index; one workgroup per tile, dispatched in
    // list order.
    const int32_t ni = (int32_t)p->inst.size();
    std::vector<int32_t> order(ni);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return p->inst[a].n_elems > p->inst[b].n_elems;
    });
    p->h_seg.assign(ni + 1, 0);
    for (int32_t i = 0; i < ni; ++i)
        p->h_seg[i + 1] = p->h_seg[i] + (p->inst[i].n_elems + te - 1) / te;
    const int64_t nt = p->h_seg[ni];
    p->h_tiles.clear();
    p->h_tiles.reserve((size_t)(4 * nt));
    for (int32_t oi : order) {
        const pg_instance& in = p->inst[oi];
        const int64_t tiles = (in.n_elems + te - 1) / te;
        for (int64_t t = 0; t < tiles; ++t) {
            const int64_t first = in.elem_off + t * te;
            p->h_tiles.push_back(first);
            p->h_tiles.push_back(std::min(first + te, in.elem_off + in.n_elems));
            p->h_tiles.push_back(in.node_off | ((int64_t)kHashRotDefault << 40));
            p->h_tiles.push_back(((int64_t)oi << 40) | (p->h_seg[oi] + t));
        }
    }
    p->batch.n_tiles = nt;
    p->n_partials = (size_t)std::max<int64_t>(nt, 1);
    p->o_partials = L.take(sizeof(double) * p->n_partials);
    p->o_flag = L.take(sizeof(int32_t) * 4);
    // tables: tile records (4 x int64 each), then the instance segments (ni + 1)
    p->o_tiles = L.take(sizeof(int64_t) * (size_t)(4 * nt + ni + 1));
    if (p->opt.ckpt == PG_STORE) p->o_u = L.take(sizeof(double) * (size_t)p->n_elems_total);
    if (p->dtype == PG_F32) p->o_gacc = L.take(sizeof(double) * (size_t)p->n_nodes_total);
    p->ws_bytes = L.total;
}

// ------------------------------------------------------------ dense layout

void layout_dense(pg_plan_s* p) {
    Layout L;
    const DenseView& d = p->dense;
    const int64_t vn = p->dtype == PG_F64 ? 2 : 4;
    p->dense_fused = d.cols <= dense_fused_max_cols() * (p->dtype == PG_F64 ? 1 : 2) && d.cols % vn == 0;
    p->dense_groups = (int)std::max<int64_t>(1, std::min<int64_t>(d.rows, 256));
    p->n_partials = (size_t)std::max<int64_t>(std::max<int64_t>(d.rows, p->dense_groups), 1);
    p->o_partials = L.take(sizeof(double) * p->n_partials);
    p->o_flag = L.take(sizeof(int32_t) * 4);
    p->o_v = L.take(sizeof(double) * (size_t)std::max<int64_t>(d.rows, 1));
    if (p->dense_fused)
        p->o_colpart = L.take(sizeof(double) * (size_t)p->dense_groups * (size_t)d.cols);
    p->ws_bytes = L.total;
}

void layout_bdense(pg_plan_s* p) {
    Layout L;
    p->bd_tiles = bdense_fwd_tiles(p->bd.m, p->bd.n);
    p->n_partials = (size_t)std::max<int64_t>(p->bd_tiles, 1);
    p->o_partials = L.take(sizeof(double) * p->n_partials);
    p->o_flag = L.take(sizeof(int32_t) * 4);
    // V = W (.) psi'(A X) in the plan dtype: the stored tape (PG_STORE) or the
    // recomputed operand of the backward product.
    p->o_vmat = L.take(esize(p->dtype) * (size_t)p->bd.m * (size_t)p->bd.n);
    p->ws_bytes = L.total;
}

pg_status need_bound(pg_plan p) {
    if (!p) return fail(PG_EINVAL, "plan is NULL");
    if (!p->bound) return fail(PG_ESTATE, "plan has no workspace bound (call pg_bind_workspace)");
    return PG_OK;
}

constexpr int64_t kMaxTimed = 4096;

// Record the start (or stop) event of a timed launch at this level.
// Timing of one dominant kernel: arms the plan's next event pair for the
// next PG_LAUNCH, which stamps it with the kernel's own start and end; the
// pair counts only if a launch took it (an empty input launches nothing).
hipError_t tkern(pg_plan p, bool start) {
    if (p->timing_mode != 1 || p->ev_n >= kMaxTimed) return hipSuccess;
    LaunchEvents& a = armed_launch_events();
    if (start) {
        a.start = p->ev[2 * p->ev_n];
        a.stop = p->ev[2 * p->ev_n + 1];
    } else if (a.start == nullptr) {
        ++p->ev_n;
    } else {
        a = LaunchEvents{};
    }
    return hipSuccess;
}

// Timing of a range of launches (several kernels, or a whole call): events
// recorded on the stream around it.
hipError_t tmark(pg_plan p, int level, bool start, hipStream_t s) {
    if (p->timing_mode != level || p->ev_n >= kMaxTimed) return hipSuccess;
    hipError_t e = hipEventRecord(p->ev[2 * p->ev_n + (start ? 0 : 1)], s);
    if (!start && e == hipSuccess) ++p->ev_n;
    return e;
}

size_t x_bytes(pg_plan p) {
    switch (p->kind) {
        case K_MESH: return esize(p->dtype) * (size_t)p->mesh.n_nodes;
        case K_BATCH: return esize(p->dtype) * (size_t)p->n_nodes_total;
        case K_DENSE: return esize(p->dtype) * (size_t)p->dense.cols;
        case K_BDENSE: return esize(p->dtype) * (size_t)(p->bd.m * p->bd.n);
        case K_LAPLACE: return esize(p->dtype) * (size_t)p->lap_n;
    }
    return 0;
}

size_t f_count(pg_plan p) { return p->kind == K_BATCH ? p->inst.size() : 1; }

// Operands a result must not overlap.
pg_status check_out_alias(pg_plan p, const void* out, size_t out_bytes, const void* x,
                          const char* what) {
    if (overlap(out, out_bytes, x, x_bytes(p))) return fail(PG_EALIAS, "%s overlaps x", what);
    if (overlap(out, out_bytes, p->ws, p->ws_bytes))
        return fail(PG_EALIAS, "%s overlaps the workspace", what);
    const size_t es = esize(p->dtype);
    switch (p->kind) {
        case K_MESH:
        case K_BATCH: {
            const int64_t E = p->kind == K_MESH ? p->mesh.n_elems : p->n_elems_total;
            const int32_t k = p->kind == K_MESH ? p->mesh.k : p->batch.k;
            const void* conn = p->kind == K_MESH ? (const void*)p->mesh.conn : (const void*)p->batch.conn;
            const void* B = p->kind == K_MESH ? p->mesh.B : p->batch.B;
            const void* w = p->kind == K_MESH ? p->mesh.w : p->batch.w;
            if (overlap(out, out_bytes, conn, 4 * (size_t)(E * k)) ||
                overlap(out, out_bytes, B, es * (size_t)(E * k)) ||
                overlap(out, out_bytes, w, es * (size_t)E))
                return fail(PG_EALIAS, "%s overlaps conn, B or w", what);
            break;
        }
        case K_DENSE:
            if (overlap(out, out_bytes, p->dense.A, es * (size_t)(p->dense.rows * p->dense.cols)) ||
                overlap(out, out_bytes, p->dense.w, es * (size_t)p->dense.rows))
                return fail(PG_EALIAS, "%s overlaps A or w", what);
            break;
        case K_BDENSE:
            if (overlap(out, out_bytes, p->bd.A, es * (size_t)(p->bd.m * p->bd.m)) ||
                overlap(out, out_bytes, p->bd.W, es * (size_t)(p->bd.m * p->bd.n)))
                return fail(PG_EALIAS, "%s overlaps A or W", what);
            break;
        case K_LAPLACE: break;  // its entry points check their own operands
    }
    return PG_OK;
}

pg_status check_tape(pg_plan p, const void* tape, const void* x) {
    if (p->kind != K_MESH && p->kind != K_BATCH && p->kind != K_BDENSE)
        return fail(PG_EUNSUPPORTED, "this plan kind records no tape");
    if (!tape && p->tape_bytes > 0) return fail(PG_EINVAL, "tape is NULL");
    if ((uintptr_t)tape % 16) return fail(PG_EINVAL, "tape must be 16-byte aligned");
    return check_out_alias(p, tape, p->tape_bytes, x, "tape");
}

MeshPass base_pass(pg_plan p, const void* x) {
    MeshPass q;
    q.x = x;
    q.partials = p->at<double>(p->o_partials);
    q.block = p->opt.block;
    q.ept = p->opt.tile;
    q.combine = p->opt.scatter != 1;
    q.hash_shift = p->hash_shift;
    q.agg_slots = p->agg_slots;
    return q;
}

// ------------------------------------------------------------ mesh driver

enum Want { W_OBJ = 1, W_GRAD = 2 };

// A caller-owned tape of one call (pg_objective_tape / pg_adjoint_tape);
// both null for the plan-level calls, which use the workspace's tape.
struct CallTape {
    void* out = nullptr;       // forward values written here
    const void* in = nullptr;  // forward values read from here
};

// The workspace's tape may be read for x only if the last pg_objective
// stored it from the same x and nothing has overwritten it since.
pg_status stored_tape_ok(pg_plan p, const void* x) {
    if (!p->tape_valid)
        return fail(PG_ESTATE, "no stored forward values: call pg_objective first (a batched-dense "
                               "gradient or recomputing adjoint overwrites them)");
    if (p->tape_x != x)
        return fail(PG_ESTATE, "the stored forward values were computed from another x "
                               "(pg_objective was last called with a different pointer)");
    return PG_OK;
}

TiledView tiled_view(pg_plan p) {
    TiledView v;
    v.n_tiles = p->tiled_nt;
    v.tile = p->tiled_tile;
    v.tbase = p->at<int64_t>(p->o_tbase);
    v.lstride = tiled_stride(p);
    v.loff = p->at<int16_t>(p->o_loff);
    v.lidx = p->at<int16_t>(p->o_lidx);
    v.stage = p->at<double>(p->o_stage);
    v.noff = p->at<int32_t>(p->o_noff);
    v.npos = p->at<int32_t>(p->o_npos);
    v.round_slots = p->tiled_round_slots;
    v.round_shift = p->tiled_round_shift;
    return v;
}

// The one-launch path's counters and tables in the workspace.
SmallPass small_pass(pg_plan p) {
    SmallPass sp;
    int32_t* meta = p->at<int32_t>(p->o_small_meta);
    sp.ticket = p->at<int32_t>(p->o_ticket);
    sp.range_done = meta;
    sp.range_need = meta + kSmallMaxRanges;
    sp.wg_off = meta + 2 * kSmallMaxRanges;
    sp.wg_list = sp.wg_off + (kSmallMaxBlocks + 1);
    return sp;
}

pg_status mesh_run(pg_plan p, const void* x, const double* fbar, void* grad, double* f_out,
                   int want, const CallTape& t, hipStream_t s) {
    const MeshView& m = p->mesh;
    MeshPass q = base_pass(p, x);
    const bool f32 = p->dtype == PG_F32;
    const bool acc = p->opt.accumulate != 0;
    const bool obj = (want & W_OBJ) != 0;
    const bool grd = (want & W_GRAD) != 0;
    if (p->small) {
        // One launch: the element work, the scatter into the zeroed buffer,
        // and (last workgroup) grad from the buffer, the buffer cleared, f.
        SmallPass sp = small_pass(p);
        sp.accumulate = acc;
        sp.f_out = obj ? f_out : nullptr;
        MeshMode mode = M_PRIMAL;
        if (!grd) {
            q.u_store = t.out ? static_cast<double*>(t.out) : p->at<double>(p->o_u);
        } else {
            q.fbar = fbar;
            if (!obj && t.in) {
                q.u_in = static_cast<const double*>(t.in);
            } else if (!obj && p->opt.ckpt == PG_STORE) {
                pg_status ts = stored_tape_ok(p, x);
                if (ts) return ts;
                q.u_in = p->at<double>(p->o_u);
            }
            q.gacc = p->at<double>(p->o_small);
            sp.grad = grad;
            mode = obj ? M_GRAD_ATOMIC : M_ADJ_ATOMIC;
        }
        PG_HIP(tkern(p, true));
        PG_HIP(launch_mesh_small(m, mode, q, sp, s));
        PG_HIP(tkern(p, false));
        if (!grd && !t.out && q.u_store) {
            p->tape_valid = true;
            p->tape_x = x;
        }
        return PG_OK;
    }
    if (!grd) {
        q.u_store = t.out ? static_cast<double*>(t.out) : p->at<double>(p->o_u);
        PG_HIP(tkern(p, true));
        PG_HIP(launch_mesh_elem(m, M_PRIMAL, q, s));
        PG_HIP(tkern(p, false));
        if (f_out) PG_HIP(launch_final_sum(q.partials, p->mesh_blocks_n, f_out, s));
        if (!t.out && q.u_store) {
            p->tape_valid = true;
            p->tape_x = x;
        }
        return PG_OK;
    }
    q.fbar = fbar;
    if (!obj && t.in) {
        q.u_in = static_cast<const double*>(t.in);
    } else if (!obj && p->opt.ckpt == PG_STORE) {
        pg_status ts = stored_tape_ok(p, x);
        if (ts) return ts;
        q.u_in = p->at<double>(p->o_u);
    }
    if (p->opt.adjoint == PG_ADJ_COLOUR) {
        // Elements of one colour share no node: plain read-add-write, one
        // pass per colour in a fixed order (deterministic).
        // FP32: the FP64 buffer is zero between calls (cleared by the conversion)
        q.gacc = f32 ? p->at<double>(p->o_gacc) : static_cast<double*>(grad);
        if (!f32 && !acc) PG_HIP(launch_zero(q.gacc, sizeof(double) * (size_t)m.n_nodes, s));
        const int32_t* elist = p->at<int32_t>(p->o_elist);
        // The passes read the colour-major row copies, except when stored
        // forward values (indexed by element) are read or written.
        const bool copies = !q.u_in && !q.u_store;
        const size_t esz = esize(p->dtype);
        int64_t slot = 0;
        PG_HIP(tmark(p, 1, true, s));
        for (size_t c = 0; c + 1 < p->colour_off.size(); ++c) {
            const int64_t off = p->colour_off[c], cnt = p->colour_off[c + 1] - off;
            q.partial_base = slot;
            if (cnt == 0) continue;
            if (copies) {
                MeshView mc = m;
                mc.n_elems = cnt;
                mc.conn = p->at<int32_t>(p->o_pconn) + off * m.k;
                mc.B = p->at<char>(p->o_pB) + (size_t)(off * m.k) * esz;
                mc.w = p->at<char>(p->o_pw) + (size_t)off * esz;
                q.elist = nullptr;
                q.elist_n = 0;
                PG_HIP(launch_mesh_elem(mc, obj ? M_GRAD_COLOUR : M_ADJ_COLOUR, q, s));
            } else {
                q.elist = elist + off;
                q.elist_n = cnt;
                PG_HIP(launch_mesh_elem(m, obj ? M_GRAD_COLOUR : M_ADJ_COLOUR, q, s));
            }
            slot += mesh_blocks(cnt, q.block, k_in_registers(m.k) ? q.ept : 1);
        }
        PG_HIP(tmark(p, 1, false, s));
        if (f32 && obj && f_out)  // the conversion's first workgroup also sums f
            PG_HIP(launch_f64_to_f32_sum(q.gacc, static_cast<float*>(grad), m.n_nodes, acc, 1,
                                         q.partials, slot, f_out, s));
        else if (f32)
            PG_HIP(launch_f64_to_f32(q.gacc, static_cast<float*>(grad), m.n_nodes, acc, 1, s));
        if (!f32 && obj && f_out) PG_HIP(launch_final_sum(q.partials, slot, f_out, s));
        return PG_OK;
    }
    if (p->opt.adjoint == PG_ADJ_TILED) {
        // Level 1 writes every tile's partials (and f's partials); level 2
        // overwrites or adds to grad, so no fill is needed.
        const TiledView tv = tiled_view(p);
        PG_HIP(tmark(p, 1, true, s));
        PG_HIP(launch_mesh_tiled(m, q, tv, obj, s));
        PG_HIP(launch_node_tiled(m, tv, grad, acc, s));
        PG_HIP(tmark(p, 1, false, s));
        if (obj && f_out) PG_HIP(launch_final_sum(q.partials, p->tiled_nt, f_out, s));
        return PG_OK;
    }
    if (p->opt.adjoint == PG_ADJ_GATHER) {
        q.v_out = p->at<double>(p->o_v);
        PG_HIP(tmark(p, 1, true, s));
        PG_HIP(launch_mesh_elem(m, obj ? M_GRAD_V : M_ADJ_V, q, s));
        PG_HIP(launch_mesh_node_gather(m, p->at<int32_t>(p->o_offs), p->at<int32_t>(p->o_inc),
                                       p->at<char>(p->o_binc), q.v_out, grad, acc, 256, s));
        PG_HIP(tmark(p, 1, false, s));
    } else {  // atomic
        if (f32) {
            q.gacc = p->at<double>(p->o_gacc);  // zero between calls (cleared by the conversion)
        } else {
            q.gacc = static_cast<double*>(grad);
            if (!acc) PG_HIP(launch_zero(grad, sizeof(double) * (size_t)m.n_nodes, s));
        }
        PG_HIP(tkern(p, true));
        PG_HIP(launch_mesh_elem(m, obj ? M_GRAD_ATOMIC : M_ADJ_ATOMIC, q, s));
        PG_HIP(tkern(p, false));
        if (f32 && obj && f_out)  // the conversion's first workgroup also sums f
            PG_HIP(launch_f64_to_f32_sum(q.gacc, static_cast<float*>(grad), m.n_nodes, acc, 1,
                                         q.partials, p->mesh_blocks_n, f_out, s));
        else if (f32)
            PG_HIP(launch_f64_to_f32(q.gacc, static_cast<float*>(grad), m.n_nodes, acc, 1, s));
        if (!f32 && obj && f_out) PG_HIP(launch_final_sum(q.partials, p->mesh_blocks_n, f_out, s));
        return PG_OK;
    }
    if (obj && f_out) PG_HIP(launch_final_sum(q.partials, p->mesh_blocks_n, f_out, s));
    return PG_OK;
}

// ------------------------------------------------- LDS table hash choice

// Sampled tiles of one mesh: every tile when there are at most `want`,
// else `want` tiles spread evenly.  One copy per sampled tile, all issued
// before a single wait.  (With a single strided 2D copy of the same rows,
// plans bound inside a rocprofv3 run chose hash parameters that left long
// probe chains: the 256-mesh batch took 6 ms instead of 1.1.)
pg_status sample_mesh_tiles(const int32_t* conn, int64_t n_elems, int32_t k, int64_t noff,
                            int64_t span, int want, std::vector<std::vector<int32_t>>& tiles,
                            hipStream_t s) {
    const int64_t nt = (n_elems + span - 1) / span;
    const int64_t ns = std::min<int64_t>(nt, want);
    const size_t first = tiles.size();
    for (int64_t i = 0; i < ns; ++i) {
        const int64_t t = nt > 1 ? i * (nt - 1) / std::max<int64_t>(ns - 1, 1) : 0;
        const int64_t e0 = t * span, e1 = std::min(n_elems, (t + 1) * span);
        tiles.emplace_back((size_t)((e1 - e0) * k));
        PG_HIP(hipMemcpyAsync(tiles.back().data(), conn + e0 * k,
                              sizeof(int32_t) * tiles.back().size(), hipMemcpyDeviceToHost, s));
    }
    PG_HIP(hipStreamSynchronize(s));
    if (noff)
        for (size_t i = first; i < tiles.size(); ++i)
            for (auto& v : tiles[i]) v = (int32_t)(v + noff);
    return PG_OK;
}

uint32_t shift_of(const std::vector<std::vector<int32_t>>& tiles) {
    std::vector<const int32_t*> ptr;
    std::vector<int64_t> cnt;
    for (const auto& t : tiles) {
        ptr.push_back(t.data());
        cnt.push_back((int64_t)t.size());
    }
    return choose_hash_shift(ptr.data(), cnt.data(), (int64_t)tiles.size(), 4096, nullptr);
}

void table_of(const std::vector<std::vector<int32_t>>& tiles, int* slots, uint32_t* shift) {
    std::vector<const int32_t*> ptr;
    std::vector<int64_t> cnt;
    for (const auto& t : tiles) {
        ptr.push_back(t.data());
        cnt.push_back((int64_t)t.size());
    }
    choose_table(ptr.data(), cnt.data(), (int64_t)tiles.size(), slots, shift);
}

// Structures of the two-level deterministic adjoint (on the host, at bind):
// per tile its sorted distinct nodes and, per local node, the tile-relative
// positions of its incidences in ascending order; per node, its staging
// slots in ascending tile order.
// Corner-round form of the tiled adjoint's first level (tiled_kernels.hip):
// usable when k is 2, 4 or 8, tiles have at most 512 elements, inside every
// tile no two elements put the same node at the same corner, and some slot
// count S (2048 or 4096) and hash rotation give every tile's distinct nodes
// distinct slots.  On success *slots, *shift are set and tile_nodes[t] holds
// tile t's distinct nodes.
bool rounds_eligible(const std::vector<int32_t>& conn, int64_t E, int k, int T, int64_t N,
                     std::vector<std::vector<int32_t>>& tile_nodes, int* slots, uint32_t* shift) {
    (void)N;
    if ((k != 2 && k != 4 && k != 8) || T > 512 || E == 0) return false;
    const int64_t nt = (E + T - 1) / T;
    if (nt * 4096 >= ((int64_t)1 << 31)) return false;
    // Per tile, by sorting (memory of one tile, whatever the node count):
    // each corner's nodes distinct, then the tile's distinct nodes.
    tile_nodes.assign((size_t)nt, {});
    std::vector<int32_t> col;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t e0 = t * T, e1 = std::min(E, e0 + T);
        for (int j = 0; j < k; ++j) {
            col.clear();
            for (int64_t e = e0; e < e1; ++e) col.push_back(conn[(size_t)(e * k + j)]);
            std::sort(col.begin(), col.end());
            if (std::adjacent_find(col.begin(), col.end()) != col.end()) {
                tile_nodes.clear();
                return false;
            }
        }
        auto& v = tile_nodes[(size_t)t];
        v.assign(conn.begin() + e0 * k, conn.begin() + e1 * k);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    for (int S : {2048, 4096}) {
        std::vector<int64_t> owner((size_t)S, -1);
        int64_t stamp = 0;
        for (uint32_t sh = 1; sh < (uint32_t)S; sh += 2) {
            bool good = true;
            for (int64_t t = 0; t < nt && good; ++t, ++stamp) {
                for (const int32_t n : tile_nodes[(size_t)t]) {
                    const uint32_t u = (uint32_t)n;
                    const uint32_t sl = (u + (u >> 12) * sh) & (uint32_t)(S - 1);
                    if (owner[sl] == stamp) {
                        good = false;
                        break;
                    }
                    owner[sl] = stamp;
                }
            }
            if (good) {
                *slots = S;
                *shift = sh;
                return true;
            }
        }
    }
    return false;
}

pg_status mesh_tiled_build(pg_plan p, hipStream_t s) {
    const MeshView& m = p->mesh;
    const int k = m.k, T = p->tiled_tile;
    const int64_t E = m.n_elems, N = m.n_nodes, nt = p->tiled_nt, inc = E * k;
    std::vector<int32_t> conn((size_t)inc);
    if (inc > 0) {
        PG_HIP(hipMemcpyAsync(conn.data(), m.conn, sizeof(int32_t) * (size_t)inc, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    }
    p->tiled_round_slots = 0;
    p->tiled_round_shift = 0;
    {
        std::vector<std::vector<int32_t>> tile_nodes;
        int S = 0;
        uint32_t sh = 0;
        if (rounds_eligible(conn, E, k, T, N, tile_nodes, &S, &sh)) {
            // node -> its tiles' staging positions t * S + slot, ascending t
            std::vector<int32_t> noff((size_t)N + 1, 0);
            int64_t total = 0;
            for (const auto& v : tile_nodes) {
                for (const int32_t n : v) noff[(size_t)n + 1]++;
                total += (int64_t)v.size();
            }
            for (int64_t n = 0; n < N; ++n) noff[(size_t)n + 1] += noff[(size_t)n];
            std::vector<int32_t> npos((size_t)std::max<int64_t>(total, 1));
            std::vector<int32_t> fill(noff.begin(), noff.end() - 1);
            for (int64_t t = 0; t < nt; ++t)
                for (const int32_t n : tile_nodes[(size_t)t]) {
                    const uint32_t u = (uint32_t)n;
                    const uint32_t sl = (u + (u >> 12) * sh) & (uint32_t)(S - 1);
                    npos[(size_t)fill[(size_t)n]++] = (int32_t)(t * S + sl);
                }
            PG_HIP(hipMemcpyAsync(p->at<int32_t>(p->o_noff), noff.data(), sizeof(int32_t) * noff.size(),
                                  hipMemcpyHostToDevice, s));
            if (total > 0)
                PG_HIP(hipMemcpyAsync(p->at<int32_t>(p->o_npos), npos.data(),
                                      sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, s));
            PG_HIP(hipStreamSynchronize(s));
            p->tiled_round_slots = S;
            p->tiled_round_shift = sh;
            return PG_OK;
        }
    }
    std::vector<int64_t> tbase((size_t)nt + 1, 0);
    const int ls = tiled_stride(p);
    std::vector<int16_t> loff((size_t)std::max<int64_t>(nt * ls, 1), 0);
    std::vector<int16_t> lidx((size_t)std::max<int64_t>(inc, 1));
    std::vector<int32_t> stage_node;  // node of each staging slot
    stage_node.reserve((size_t)inc);
    std::vector<std::pair<int32_t, int32_t>> items;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t e0 = t * T, e1 = std::min(E, e0 + T);
        const int32_t cnt = (int32_t)((e1 - e0) * k);
        int16_t* lo = loff.data() + (size_t)(t * ls);
        int32_t nl = 0;
        items.resize((size_t)cnt);
        for (int32_t q = 0; q < cnt; ++q) items[(size_t)q] = {conn[(size_t)(e0 * k + q)], q};
        std::sort(items.begin(), items.end());  // by node, then by position
        for (int32_t q = 0; q < cnt; ++q) {
            if (q == 0 || items[(size_t)q].first != items[(size_t)q - 1].first) {
                lo[nl++] = (int16_t)q;
                stage_node.push_back(items[(size_t)q].first);
            }
            lidx[(size_t)(e0 * k + q)] = (int16_t)items[(size_t)q].second;
        }
        lo[nl] = (int16_t)cnt;
        tbase[(size_t)t + 1] = (int64_t)stage_node.size();
    }
    const int64_t S = (int64_t)stage_node.size();
    // node -> staging slots, in ascending slot (hence tile) order
    std::vector<int32_t> noff((size_t)N + 1, 0), npos((size_t)std::max<int64_t>(S, 1));
    for (int64_t q = 0; q < S; ++q) noff[(size_t)stage_node[(size_t)q] + 1]++;
    for (int64_t n = 0; n < N; ++n) noff[(size_t)n + 1] += noff[(size_t)n];
    std::vector<int32_t> fill(noff.begin(), noff.end() - 1);
    for (int64_t q = 0; q < S; ++q) npos[(size_t)fill[(size_t)stage_node[(size_t)q]]++] = (int32_t)q;
    PG_HIP(hipMemcpyAsync(p->at<int64_t>(p->o_tbase), tbase.data(), sizeof(int64_t) * tbase.size(),
                          hipMemcpyHostToDevice, s));
    if (nt > 0)
        PG_HIP(hipMemcpyAsync(p->at<int16_t>(p->o_loff), loff.data(), sizeof(int16_t) * (size_t)(nt * ls),
                              hipMemcpyHostToDevice, s));
    if (inc > 0)
        PG_HIP(hipMemcpyAsync(p->at<int16_t>(p->o_lidx), lidx.data(), sizeof(int16_t) * (size_t)inc,
                              hipMemcpyHostToDevice, s));
    PG_HIP(hipMemcpyAsync(p->at<int32_t>(p->o_noff), noff.data(), sizeof(int32_t) * noff.size(),
                          hipMemcpyHostToDevice, s));
    if (S > 0)
        PG_HIP(hipMemcpyAsync(p->at<int32_t>(p->o_npos), npos.data(), sizeof(int32_t) * (size_t)S,
                              hipMemcpyHostToDevice, s));
    PG_HIP(hipStreamSynchronize(s));
    return PG_OK;
}


// Greedy colouring in element order (plan time, on the host): element e
// takes the smallest colour that no earlier element sharing one of its nodes
// has.  Node masks record the colours already present at each node, so one
// pass over conn suffices.  Then elements are listed colour by colour, in
// ascending order inside a colour.
pg_status mesh_colour(pg_plan p, hipStream_t s) {
    const MeshView& m = p->mesh;
    const int64_t items = m.n_elems * m.k;
    std::vector<int32_t> conn((size_t)items);
    if (items > 0) {
        PG_HIP(hipMemcpyAsync(conn.data(), m.conn, sizeof(int32_t) * (size_t)items,
                              hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    }
    std::vector<uint64_t> node_mask((size_t)m.n_nodes, 0);
    std::vector<int32_t> colour((size_t)m.n_elems);
    int ncol = 0;
    for (int64_t e = 0; e < m.n_elems; ++e) {
        uint64_t used = 0;
        for (int32_t j = 0; j < m.k; ++j) used |= node_mask[(size_t)conn[(size_t)(e * m.k + j)]];
        if (~used == 0)
            return fail(PG_EUNSUPPORTED, "element %lld needs more than %d colours", (long long)e,
                        kMaxColours);
        const int c = __builtin_ctzll(~used);
        colour[(size_t)e] = c;
        ncol = std::max(ncol, c + 1);
        for (int32_t j = 0; j < m.k; ++j) node_mask[(size_t)conn[(size_t)(e * m.k + j)]] |= 1ull << c;
    }
    p->colour_off.assign((size_t)ncol + 1, 0);
    for (int64_t e = 0; e < m.n_elems; ++e) p->colour_off[(size_t)colour[(size_t)e] + 1]++;
    for (int c = 0; c < ncol; ++c) p->colour_off[(size_t)c + 1] += p->colour_off[(size_t)c];
    std::vector<int32_t> elist((size_t)m.n_elems);
    std::vector<int64_t> fill(p->colour_off.begin(), p->colour_off.end() - 1);
    for (int64_t e = 0; e < m.n_elems; ++e) elist[(size_t)fill[(size_t)colour[(size_t)e]]++] = (int32_t)e;
    if (m.n_elems > 0) {
        PG_HIP(hipMemcpyAsync(p->at<int32_t>(p->o_elist), elist.data(),
                              sizeof(int32_t) * (size_t)m.n_elems, hipMemcpyHostToDevice, s));
        PG_HIP(hipStreamSynchronize(s));
    }
    return PG_OK;
}

// Range tables of the one-launch path (host, at bind): the node ranges each
// workgroup's elements touch, how many workgroups count on each range, and
// every untouched range given to workgroup 0 so that it is written too.  The
// node buffer, the counts and the ticket start at zero.
pg_status mesh_small_build(pg_plan p, hipStream_t s) {
    const MeshView& m = p->mesh;
    const int64_t G = mesh_blocks(m.n_elems, p->opt.block, 1);
    const int R = (int)((m.n_nodes + kSmallRange - 1) / kSmallRange);
    std::vector<int32_t> conn((size_t)(m.n_elems * m.k));
    PG_HIP(hipMemcpyAsync(conn.data(), m.conn, sizeof(int32_t) * conn.size(), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> meta((size_t)small_meta_ints(), 0);
    int32_t* need = meta.data() + kSmallMaxRanges;
    int32_t* wg_off = need + kSmallMaxRanges;
    int32_t* wg_list = wg_off + (kSmallMaxBlocks + 1);
    std::vector<char> touched((size_t)R);
    int32_t pos = 0;
    for (int64_t w = 0; w < G; ++w) {
        std::fill(touched.begin(), touched.end(), 0);
        const int64_t e0 = w * p->opt.block, e1 = std::min(m.n_elems, e0 + p->opt.block);
        for (int64_t q = e0 * m.k; q < e1 * m.k; ++q) touched[(size_t)(conn[(size_t)q] / kSmallRange)] = 1;
        if (w == 0) {
            // ranges no workgroup touches are counted on by workgroup 0
            std::vector<char> any((size_t)R, 0);
            for (int32_t c : conn) any[(size_t)(c / kSmallRange)] = 1;
            for (int r = 0; r < R; ++r)
                if (!any[(size_t)r]) touched[(size_t)r] = 1;
        }
        wg_off[w] = pos;
        for (int r = 0; r < R; ++r)
            if (touched[(size_t)r]) {
                wg_list[pos++] = r;
                need[r]++;
            }
    }
    wg_off[G] = pos;
    PG_HIP(hipMemcpyAsync(p->at<int32_t>(p->o_small_meta), meta.data(), sizeof(int32_t) * meta.size(),
                          hipMemcpyHostToDevice, s));
    PG_HIP(launch_zero(p->at<double>(p->o_small), sizeof(double) * (size_t)m.n_nodes, s));
    PG_HIP(launch_zero(p->at<int32_t>(p->o_ticket), sizeof(int32_t) * 4, s));
    PG_HIP(hipStreamSynchronize(s));
    return PG_OK;
}

pg_status mesh_bind(pg_plan p, hipStream_t s) {
    const MeshView& m = p->mesh;
    int32_t* flag = p->at<int32_t>(p->o_flag);
    PG_HIP(launch_zero(flag, sizeof(int32_t) * 4, s));
    // FP32 plans: the FP64 accumulation buffer is zero between calls.
    if (p->o_gacc != NONE) PG_HIP(launch_zero(p->at<double>(p->o_gacc), sizeof(double) * (size_t)m.n_nodes, s));
    const int64_t items = m.n_elems * m.k;
    if (p->opt.adjoint == PG_ADJ_GATHER) {
        int32_t* cnt = p->at<int32_t>(p->o_cursor);
        PG_HIP(launch_zero(cnt, sizeof(int32_t) * (size_t)m.n_nodes, s));
        PG_HIP(launch_validate_count(m.conn, items, m.n_nodes, cnt, flag, s));
    } else {
        PG_HIP(launch_validate_count(m.conn, items, m.n_nodes, nullptr, flag, s));
    }
    int32_t hflag = 0;
    PG_HIP(hipMemcpyAsync(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (hflag) return fail(PG_ERANGE, "connectivity has an entry outside [0, %lld)", (long long)m.n_nodes);
    if (p->small) {
        pg_status sst = mesh_small_build(p, s);
        if (sst != PG_OK) return sst;
    }
    if (p->opt.scatter != 1 && m.n_elems > 0) {
        std::vector<std::vector<int32_t>> tiles;
        pg_status hst = sample_mesh_tiles(m.conn, m.n_elems, m.k, 0,
                                          (int64_t)p->opt.block * p->opt.tile, kHashSamples, tiles, s);
        if (hst != PG_OK) return hst;
        table_of(tiles, &p->agg_slots, &p->hash_shift);
        // The 2048-slot table is kept only if no workgroup of the pass finds
        // two of its nodes on one home slot: the sample can miss the few
        // workgroups where the hash puts two node runs in one window, and
        // their probe chains cost far more than the smaller table saves.
        if (p->opt.scatter == 0 && p->agg_slots == 2048) {
            PG_HIP(launch_table_check(m.conn, m.n_elems, m.k, (int64_t)p->opt.block * p->opt.tile,
                                      p->hash_shift, 2048, flag + 1, s));
            int32_t miss = 0;
            PG_HIP(hipMemcpyAsync(&miss, flag + 1, sizeof miss, hipMemcpyDeviceToHost, s));
            PG_HIP(hipStreamSynchronize(s));
            if (miss) {
                p->agg_slots = 4096;
                p->hash_shift = shift_of(tiles);
            }
        }
        if (p->opt.scatter >= 2) {  // the caller fixed the table size
            p->agg_slots = p->opt.scatter == 2 ? 4096 : 2048;
            std::vector<const int32_t*> ptr;
            std::vector<int64_t> cnt;
            for (const auto& t : tiles) {
                ptr.push_back(t.data());
                cnt.push_back((int64_t)t.size());
            }
            p->hash_shift = choose_hash_shift(ptr.data(), cnt.data(), (int64_t)tiles.size(),
                                              p->agg_slots, nullptr);
        }
    }
    if (p->opt.adjoint == PG_ADJ_COLOUR) {
        pg_status cst = mesh_colour(p, s);
        if (cst != PG_OK) return cst;
        PG_HIP(launch_permute_rows(p->at<int32_t>(p->o_elist), m.n_elems, m.k, m.conn, m.B, m.w,
                                   m.dtype == F64, p->at<int32_t>(p->o_pconn),
                                   p->at<char>(p->o_pB), p->at<char>(p->o_pw), s));
    }
    if (p->opt.adjoint == PG_ADJ_TILED) {
        pg_status tst = mesh_tiled_build(p, s);
        if (tst != PG_OK) return tst;
    }
    if (p->opt.adjoint == PG_ADJ_GATHER) {
        int32_t* offs = p->at<int32_t>(p->o_offs);
        PG_HIP(launch_exclusive_scan(p->at<int32_t>(p->o_cursor), m.n_nodes, offs,
                                     p->at<int64_t>(p->o_scan), s));
        PG_HIP(launch_csr_fill_sort(m.conn, items, m.n_nodes, offs, p->at<int32_t>(p->o_cursor),
                                    p->at<int32_t>(p->o_inc), s));
        PG_HIP(launch_gather_entries(p->at<int32_t>(p->o_inc), items, m.B, m.dtype == F64,
                                     p->at<char>(p->o_binc), s));
        PG_HIP(hipStreamSynchronize(s));
    }
    return PG_OK;
}

// ----------------------------------------------------------- batch driver

pg_status batch_bind(pg_plan p, hipStream_t s) {
    int32_t* flag = p->at<int32_t>(p->o_flag);
    PG_HIP(launch_zero(flag, sizeof(int32_t) * 4, s));
    // FP32 plans: the FP64 accumulation buffer is zero between calls.
    if (p->o_gacc != NONE)
        PG_HIP(launch_zero(p->at<double>(p->o_gacc), sizeof(double) * (size_t)p->n_nodes_total, s));
    // Validate each instance's connectivity against its own node count.
    for (const pg_instance& in : p->inst) {
        if (in.n_elems == 0) continue;
        PG_HIP(launch_validate_count(p->batch.conn + in.elem_off * p->batch.k,
                                     in.n_elems * p->batch.k, in.n_nodes, nullptr, flag, s));
    }
    // LDS table hash parameter per instance, written into its tile records.
    const int64_t nt = p->batch.n_tiles, ni = (int64_t)p->inst.size();
    if (p->opt.scatter != 1) {
        std::vector<uint32_t> shift((size_t)ni, kHashRotDefault);
        for (int64_t i = 0; i < ni; ++i) {
            const pg_instance& in = p->inst[(size_t)i];
            if (in.n_elems == 0) continue;
            std::vector<std::vector<int32_t>> tiles;
            pg_status hst = sample_mesh_tiles(p->batch.conn + in.elem_off * p->batch.k, in.n_elems,
                                              p->batch.k, in.node_off, p->batch.tile_elems, kHashSamples,
                                              tiles, s);
            if (hst != PG_OK) return hst;
            shift[(size_t)i] = shift_of(tiles);
        }
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t inst = p->h_tiles[(size_t)(4 * t + 3)] >> 40;
            p->h_tiles[(size_t)(4 * t + 2)] =
                (p->h_tiles[(size_t)(4 * t + 2)] & ((1LL << 40) - 1)) |
                ((int64_t)shift[(size_t)inst] << 40);
        }
    }
    // Upload the work list and instance tables.
    std::vector<int64_t> tab;
    tab.reserve((size_t)(4 * nt + ni + 1));
    tab.insert(tab.end(), p->h_tiles.begin(), p->h_tiles.end());
    tab.insert(tab.end(), p->h_seg.begin(), p->h_seg.end());
    int64_t* dtab = p->at<int64_t>(p->o_tiles);
    if (!tab.empty())
        PG_HIP(hipMemcpyAsync(dtab, tab.data(), sizeof(int64_t) * tab.size(),
                              hipMemcpyHostToDevice, s));
    int32_t hflag = 0;
    PG_HIP(hipMemcpyAsync(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (hflag) return fail(PG_ERANGE, "an instance's connectivity has an entry outside its node range");
    p->batch.tiles = dtab;
    return PG_OK;
}

pg_status batch_run(pg_plan p, const void* x, const double* fbar, void* grad, double* f_out,
                    int want, const CallTape& t, hipStream_t s) {
    const bool f32 = p->dtype == PG_F32;
    const bool acc = p->opt.accumulate != 0;
    const bool obj = (want & W_OBJ) != 0;
    const bool grd = (want & W_GRAD) != 0;
    const int64_t ni = (int64_t)p->inst.size();
    const int64_t* seg = p->at<int64_t>(p->o_tiles) + 4 * p->batch.n_tiles;
    BatchPass q;
    q.x = x;
    q.partials = p->at<double>(p->o_partials);
    q.block = p->opt.block;
    q.combine = p->opt.scatter != 1;
    q.fbar = fbar;
    if (!grd) {
        q.u_store = t.out ? static_cast<double*>(t.out) : p->at<double>(p->o_u);
        PG_HIP(tkern(p, true));
        PG_HIP(launch_batch(p->batch, B_PRIMAL, q, s));
        PG_HIP(tkern(p, false));
        if (f_out) PG_HIP(launch_segmented_sum(q.partials, seg, ni, f_out, s));
        if (!t.out && q.u_store) {
            p->tape_valid = true;
            p->tape_x = x;
        }
        return PG_OK;
    }
    if (!obj && t.in) {
        q.u_in = static_cast<const double*>(t.in);
    } else if (!obj && p->opt.ckpt == PG_STORE) {
        pg_status ts = stored_tape_ok(p, x);
        if (ts) return ts;
        q.u_in = p->at<double>(p->o_u);
    }
    if (f32) {
        q.grad = p->at<double>(p->o_gacc);  // zero between calls (cleared by the conversion)
    } else {
        q.grad = grad;
        if (!acc) PG_HIP(launch_zero(grad, sizeof(double) * (size_t)p->n_nodes_total, s));
    }
    PG_HIP(tkern(p, true));
    PG_HIP(launch_batch(p->batch, obj ? B_GRAD_ATOMIC : B_ADJ_ATOMIC, q, s));
    PG_HIP(tkern(p, false));
    if (f32)
        PG_HIP(launch_f64_to_f32(static_cast<double*>(q.grad), static_cast<float*>(grad), p->n_nodes_total,
                                 acc, 1, s));
    if (obj && f_out) PG_HIP(launch_segmented_sum(q.partials, seg, ni, f_out, s));
    return PG_OK;
}

// ----------------------------------------------------------- dense driver

pg_status dense_run(pg_plan p, const void* x, const double* fbar, void* grad, double* f_out,
                    int want, hipStream_t s) {
    const DenseView& d = p->dense;
    double* partials = p->at<double>(p->o_partials);
    const bool grd = (want & W_GRAD) != 0;
    const bool obj = (want & W_OBJ) != 0;
    const Dtype dt = p->dtype == PG_F64 ? F64 : F32;
    if (d.rows == 0 || d.cols == 0) {
        // f = sum over no rows (or psi(0) = 0 on every row) and a zero gradient.
        if (grd && !p->opt.accumulate) PG_HIP(launch_zero(grad, esize(p->dtype) * (size_t)d.cols, s));
        if (f_out && obj) PG_HIP(launch_final_sum(partials, 0, f_out, s));
        return PG_OK;
    }
    // The fused kernel reads x with 16-byte vector loads.
    if (p->dense_fused && ((uintptr_t)x % 16) == 0) {
        PG_HIP(tkern(p, true));
        PG_HIP(launch_dense_fused(d, x, fbar, grd ? 1 : 0, partials, p->at<double>(p->o_colpart),
                                  p->dense_groups, s));
        PG_HIP(tkern(p, false));
        if (grd)
            PG_HIP(launch_dense_colsum(p->at<double>(p->o_colpart), p->dense_groups, d.cols, grad,
                                       dt, p->opt.accumulate, s));
        if (f_out && obj) PG_HIP(launch_final_sum(partials, p->dense_groups, f_out, s));
    } else {
        double* v = grd ? p->at<double>(p->o_v) : nullptr;
        PG_HIP(tmark(p, 1, true, s));
        PG_HIP(launch_dense_rows(d, x, fbar, partials, v, s));
        PG_HIP(tmark(p, 1, false, s));
        if (grd) PG_HIP(launch_dense_cols(d, v, grad, p->opt.accumulate, s));
        if (f_out && obj) PG_HIP(launch_final_sum(partials, d.rows, f_out, s));
    }
    return PG_OK;
}

// --------------------------------------------------- batched dense driver

pg_status bdense_run(pg_plan p, const void* X, const double* fbar, void* G, double* f_out,
                     int want, const CallTape& t, hipStream_t s) {
    double* partials = p->at<double>(p->o_partials);
    void* V = p->ws + p->o_vmat;
    const bool grd = (want & W_GRAD) != 0;
    const bool obj = (want & W_OBJ) != 0;
    if (!grd) {
        const bool store = p->opt.ckpt == PG_STORE && !t.out;
        PG_HIP(tkern(p, true));
        PG_HIP(launch_bdense_fwd(p->bd, X, partials, t.out ? t.out : store ? V : nullptr, s));
        PG_HIP(tkern(p, false));
        if (f_out) PG_HIP(launch_final_sum(partials, p->bd_tiles, f_out, s));
        if (store) {
            p->tape_valid = true;
            p->tape_x = X;
        }
        return PG_OK;
    }
    const void* Vin = V;
    if (!obj && t.in) {
        Vin = t.in;
    } else if (obj || p->opt.ckpt == PG_RECOMPUTE) {
        // V(X) goes to the workspace buffer, which is also the stored tape:
        // a tape recorded from another X is gone.
        PG_HIP(launch_bdense_fwd(p->bd, X, partials, V, s));
        p->tape_valid = false;
        if (obj && f_out) PG_HIP(launch_final_sum(partials, p->bd_tiles, f_out, s));
    } else {
        pg_status ts = stored_tape_ok(p, X);
        if (ts) return ts;
    }
    PG_HIP(tkern(p, true));
    PG_HIP(launch_bdense_bwd(p->bd, Vin, fbar, G, p->opt.accumulate, s));
    PG_HIP(tkern(p, false));
    return PG_OK;
}

pg_status run_kind(pg_plan p, const void* x, const double* fbar, void* grad, double* f_out,
                   int want, const CallTape& t, hipStream_t s) {
    switch (p->kind) {
        case K_MESH: return mesh_run(p, x, fbar, grad, f_out, want, t, s);
        case K_BATCH: return batch_run(p, x, fbar, grad, f_out, want, t, s);
        case K_DENSE: return dense_run(p, x, fbar, grad, f_out, want, s);
        case K_BDENSE: return bdense_run(p, x, fbar, grad, f_out, want, t, s);
        case K_LAPLACE:
            return fail(PG_EUNSUPPORTED, "use pg_laplace1d_objective / pg_laplace1d_gradient");
    }
    return fail(PG_EINVAL, "unknown plan kind");
}

pg_status run(pg_plan p, const void* x, const double* fbar, void* grad, double* f_out, int want,
              pg_stream stream, const CallTape& t = CallTape{}) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_HIP(tmark(p, 2, true, s));
    pg_status st = run_kind(p, x, fbar, grad, f_out, want, t, s);
    if (st != PG_OK) return st;
    PG_HIP(tmark(p, 2, false, s));
    return PG_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

pg_options pg_default_options(void) {
    pg_options o;
    o.adjoint = PG_ADJ_AUTO;
    o.ckpt = PG_RECOMPUTE;
    o.block = 0;
    o.tile = 0;
    o.accumulate = 0;
    o.scatter = 0;
    o.onepass = 0;
    o.reserved = 0;
    o.tape_budget = 0;
    return o;
}

const char* pg_last_error(void) { return g_err; }

int pg_version(void) { return PGRAD_VERSION; }

pg_status pg_mesh_plan(pg_plan* plan, int64_t n_nodes, int64_t n_elems, int32_t k,
                       const int32_t* conn, const void* B, const void* w, pg_dtype dtype,
                       const pg_options* opts, size_t* workspace_bytes) {
    g_err[0] = 0;
    if (!plan || !workspace_bytes) return fail(PG_EINVAL, "plan and workspace_bytes must not be NULL");
    pg_status st = check_dtype(dtype);
    if (st) return st;
    pg_options o;
    if ((st = check_opts(opts, &o))) return st;
    if (n_nodes < 0 || n_elems < 0) return fail(PG_EINVAL, "n_nodes and n_elems must be >= 0");
    if (k < 1 || k > PG_MAX_K) return fail(PG_EINVAL, "k = %d outside [1, %d]", k, PG_MAX_K);
    if (n_nodes >= (1LL << 31) || n_elems * (int64_t)k >= (1LL << 31))
        return fail(PG_EINVAL, "sizes exceed the int32 index range");
    if (n_elems > 0 && (!conn || !B || !w)) return fail(PG_EINVAL, "conn, B and w must not be NULL");
    if (n_elems > 0 && n_nodes == 0) return fail(PG_ERANGE, "elements reference nodes but n_nodes is 0");
    if (((uintptr_t)conn % 16) || ((uintptr_t)B % 16) || ((uintptr_t)w % 8))
        return fail(PG_EINVAL, "conn and B must be 16-byte aligned, w 8-byte aligned");
    pg_plan_s* p = new_plan(K_MESH, dtype, o);
    if (!p) return fail(PG_EINVAL, "out of host memory");
    p->mesh.n_nodes = n_nodes;
    p->mesh.n_elems = n_elems;
    p->mesh.k = k;
    p->mesh.dtype = dtype == PG_F64 ? F64 : F32;
    p->mesh.conn = conn;
    p->mesh.B = B;
    p->mesh.w = w;
    if ((st = resolve_ckpt(p, sizeof(double) * (size_t)n_elems))) return drop_plan(p, st);
    layout_mesh(p);
    *workspace_bytes = p->ws_bytes;
    *plan = p;
    return PG_OK;
}

pg_status pg_mesh_batch_plan(pg_plan* plan, int32_t n_inst, const pg_instance* inst, int32_t k,
                             const int32_t* conn, const void* B, const void* w, pg_dtype dtype,
                             const pg_options* opts, size_t* workspace_bytes) {
    g_err[0] = 0;
    if (!plan || !workspace_bytes) return fail(PG_EINVAL, "plan and workspace_bytes must not be NULL");
    pg_status st = check_dtype(dtype);
    if (st) return st;
    pg_options o;
    if ((st = check_opts(opts, &o))) return st;
    if (o.adjoint != PG_ADJ_ATOMIC) return fail(PG_EUNSUPPORTED, "mesh batches use the atomic adjoint");
    if (n_inst < 0 || (n_inst > 0 && !inst)) return fail(PG_EINVAL, "bad instance table");
    if (n_inst >= (1 << 23)) return fail(PG_EINVAL, "at most 2^23 - 1 instances per batch");
    if (k < 1 || k > PG_MAX_K) return fail(PG_EINVAL, "k = %d outside [1, %d]", k, PG_MAX_K);
    int64_t nn = 0, ne = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        const pg_instance& in = inst[i];
        if (in.n_nodes < 0 || in.n_elems < 0 || in.node_off < 0 || in.elem_off < 0)
            return fail(PG_EINVAL, "instance %d has a negative size or offset", i);
        if (in.n_nodes >= (1LL << 31)) return fail(PG_EINVAL, "instance %d too large", i);
        if (in.n_elems > 0 && in.n_nodes == 0)
            return fail(PG_ERANGE, "instance %d has elements but no nodes", i);
        nn = std::max(nn, in.node_off + in.n_nodes);
        ne = std::max(ne, in.elem_off + in.n_elems);
    }
    if (ne * (int64_t)k >= (1LL << 31) || nn >= (1LL << 31))
        return fail(PG_EINVAL, "sizes exceed the int32 index range");
    if (ne > 0 && (!conn || !B || !w)) return fail(PG_EINVAL, "conn, B and w must not be NULL");
    if (((uintptr_t)conn % 16) || ((uintptr_t)B % 16) || ((uintptr_t)w % 8))
        return fail(PG_EINVAL, "conn and B must be 16-byte aligned, w 8-byte aligned");
    pg_plan_s* p = new_plan(K_BATCH, dtype, o);
    if (!p) return fail(PG_EINVAL, "out of host memory");
    p->inst.assign(inst, inst + n_inst);
    p->n_nodes_total = nn;
    p->n_elems_total = ne;
    p->batch.n_inst = n_inst;
    p->batch.k = k;
    p->batch.dtype = dtype == PG_F64 ? F64 : F32;
    p->batch.conn = conn;
    p->batch.B = B;
    p->batch.w = w;
    if (!k_in_registers(k)) p->opt.tile = 1;
    if ((st = resolve_ckpt(p, sizeof(double) * (size_t)ne))) return drop_plan(p, st);
    layout_batch(p);
    *workspace_bytes = p->ws_bytes;
    *plan = p;
    return PG_OK;
}

pg_status pg_dense_plan(pg_plan* plan, int64_t rows, int64_t cols, const void* A, const void* w,
                        pg_dtype dtype, const pg_options* opts, size_t* workspace_bytes) {
    g_err[0] = 0;
    if (!plan || !workspace_bytes) return fail(PG_EINVAL, "plan and workspace_bytes must not be NULL");
    pg_status st = check_dtype(dtype);
    if (st) return st;
    pg_options o;
    if ((st = check_opts(opts, &o))) return st;
    if (rows < 0 || cols < 0) return fail(PG_EINVAL, "rows and cols must be >= 0");
    if (rows >= (1LL << 31) || cols >= (1LL << 31)) return fail(PG_EINVAL, "sizes exceed the int32 range");
    if (rows > 0 && cols > 0 && (!A || !w)) return fail(PG_EINVAL, "A and w must not be NULL");
    if ((uintptr_t)A % 16) return fail(PG_EINVAL, "A must be 16-byte aligned");
    pg_plan_s* p = new_plan(K_DENSE, dtype, o);
    if (!p) return fail(PG_EINVAL, "out of host memory");
    p->dense.rows = rows;
    p->dense.cols = cols;
    p->dense.dtype = dtype == PG_F64 ? F64 : F32;
    p->dense.A = A;
    p->dense.w = w;
    if ((st = resolve_ckpt(p, 0))) return drop_plan(p, st);
    layout_dense(p);
    *workspace_bytes = p->ws_bytes;
    *plan = p;
    return PG_OK;
}

pg_status pg_bdense_plan(pg_plan* plan, int64_t m, int64_t n, const void* A, const void* W,
                         pg_dtype dtype, const pg_options* opts, size_t* workspace_bytes) {
    g_err[0] = 0;
    if (!plan || !workspace_bytes) return fail(PG_EINVAL, "plan and workspace_bytes must not be NULL");
    pg_status st = check_dtype(dtype);
    if (st) return st;
    pg_options o;
    if ((st = check_opts(opts, &o))) return st;
    if (m < 0 || n < 0) return fail(PG_EINVAL, "m and n must be >= 0");
    if (m >= (1LL << 31) || n >= (1LL << 31) || m * n >= (1LL << 40))
        return fail(PG_EINVAL, "sizes exceed the supported range");
    if (m > 0 && (!A || (n > 0 && !W))) return fail(PG_EINVAL, "A and W must not be NULL");
    if (((uintptr_t)A % 16) || ((uintptr_t)W % 16)) return fail(PG_EINVAL, "A and W must be 16-byte aligned");
    pg_plan_s* p = new_plan(K_BDENSE, dtype, o);
    if (!p) return fail(PG_EINVAL, "out of host memory");
    p->bd.m = m;
    p->bd.n = n;
    p->bd.dtype = dtype == PG_F64 ? F64 : F32;
    p->bd.A = A;
    p->bd.W = W;
    if ((st = resolve_ckpt(p, esize(dtype) * (size_t)(m * n)))) return drop_plan(p, st);
    layout_bdense(p);
    *workspace_bytes = p->ws_bytes;
    *plan = p;
    return PG_OK;
}

pg_status pg_workspace_size(pg_plan plan, size_t* workspace_bytes) {
    if (!plan || !workspace_bytes) return fail(PG_EINVAL, "plan and workspace_bytes must not be NULL");
    *workspace_bytes = plan->ws_bytes;
    return PG_OK;
}

pg_status pg_bind_workspace(pg_plan p, void* workspace, size_t bytes, pg_stream stream) {
    g_err[0] = 0;
    if (!p) return fail(PG_EINVAL, "plan is NULL");
    if (p->ws_bytes > 0 && !workspace) return fail(PG_EWORKSPACE, "workspace is NULL");
    if (bytes < p->ws_bytes)
        return fail(PG_EWORKSPACE, "workspace has %zu bytes, the plan needs %zu", bytes, p->ws_bytes);
    if ((uintptr_t)workspace % kAlign)
        return fail(PG_EWORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    p->ws = static_cast<char*>(workspace);
    p->bound = false;
    p->tape_valid = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    pg_status st = PG_OK;
    switch (p->kind) {
        case K_MESH: st = mesh_bind(p, s); break;
        case K_BATCH: st = batch_bind(p, s); break;
        case K_LAPLACE:
            PG_HIP(launch_zero(p->at<int32_t>(p->o_flag), sizeof(int32_t) * 4, s));
            PG_HIP(hipStreamSynchronize(s));
            break;
        case K_DENSE:
        case K_BDENSE: break;
    }
    if (st == PG_OK) p->bound = true;
    return st;
}

pg_status pg_objective(pg_plan p, const void* x, double* f_out, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if (!x && x_bytes(p) > 0) return fail(PG_EINVAL, "x is NULL");
    if (!f_out) return fail(PG_EINVAL, "f_out is NULL");
    if ((st = check_out_alias(p, f_out, sizeof(double) * f_count(p), x, "f_out"))) return st;
    return run(p, x, nullptr, nullptr, f_out, W_OBJ, stream);
}

pg_status pg_gradient(pg_plan p, const void* x, void* grad, double* f_out, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if ((!x || !grad) && x_bytes(p) > 0) return fail(PG_EINVAL, "x and grad must not be NULL");
    if ((st = check_out_alias(p, grad, x_bytes(p), x, "grad"))) return st;
    if (f_out && (st = check_out_alias(p, f_out, sizeof(double) * f_count(p), x, "f_out"))) return st;
    if (overlap(f_out, sizeof(double) * f_count(p), grad, x_bytes(p)))
        return fail(PG_EALIAS, "f_out overlaps grad");
    return run(p, x, nullptr, grad, f_out, W_OBJ | W_GRAD, stream);
}

pg_status pg_adjoint(pg_plan p, const void* x, const double* fbar, void* grad, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if ((!x || !grad) && x_bytes(p) > 0) return fail(PG_EINVAL, "x and grad must not be NULL");
    if (!fbar) return fail(PG_EINVAL, "fbar is NULL");
    if ((st = check_out_alias(p, grad, x_bytes(p), x, "grad"))) return st;
    if (overlap(fbar, sizeof(double) * f_count(p), grad, x_bytes(p)))
        return fail(PG_EALIAS, "fbar overlaps grad");
    if (p->opt.ckpt == PG_STORE && (p->kind == K_MESH || p->kind == K_BATCH || p->kind == K_BDENSE) &&
        (st = stored_tape_ok(p, x)))
        return st;
    return run(p, x, fbar, grad, nullptr, W_GRAD, stream);
}

pg_status pg_tape_bytes(pg_plan p, size_t* bytes) {
    g_err[0] = 0;
    if (!p || !bytes) return fail(PG_EINVAL, "plan and bytes must not be NULL");
    if (p->kind != K_MESH && p->kind != K_BATCH && p->kind != K_BDENSE)
        return fail(PG_EUNSUPPORTED, "this plan kind records no tape");
    *bytes = p->tape_bytes;
    return PG_OK;
}

pg_status pg_objective_tape(pg_plan p, const void* x, double* f_out, void* tape, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if (!x && x_bytes(p) > 0) return fail(PG_EINVAL, "x is NULL");
    if (!f_out) return fail(PG_EINVAL, "f_out is NULL");
    if ((st = check_out_alias(p, f_out, sizeof(double) * f_count(p), x, "f_out"))) return st;
    if ((st = check_tape(p, tape, x))) return st;
    if (overlap(f_out, sizeof(double) * f_count(p), tape, p->tape_bytes))
        return fail(PG_EALIAS, "f_out overlaps the tape");
    CallTape t;
    t.out = tape;
    return run(p, x, nullptr, nullptr, f_out, W_OBJ, stream, t);
}

pg_status pg_adjoint_tape(pg_plan p, const double* fbar, const void* tape, void* grad,
                          pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if (!grad && x_bytes(p) > 0) return fail(PG_EINVAL, "grad is NULL");
    if (!fbar) return fail(PG_EINVAL, "fbar is NULL");
    if ((st = check_out_alias(p, grad, x_bytes(p), nullptr, "grad"))) return st;
    if ((st = check_tape(p, tape, nullptr))) return st;
    if (overlap(grad, x_bytes(p), tape, p->tape_bytes)) return fail(PG_EALIAS, "grad overlaps the tape");
    if (overlap(fbar, sizeof(double) * f_count(p), grad, x_bytes(p)))
        return fail(PG_EALIAS, "fbar overlaps grad");
    CallTape t;
    t.in = tape;
    // x is not read when the forward values come from the tape.
    return run(p, nullptr, fbar, grad, nullptr, W_GRAD, stream, t);
}

pg_status pg_hvp(pg_plan p, const void* x, const void* v, void* hv, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if (p->kind != K_MESH) return fail(PG_EUNSUPPORTED, "pg_hvp supports mesh plans only");
    if ((!x || !v || !hv) && x_bytes(p) > 0) return fail(PG_EINVAL, "x, v and hv must not be NULL");
    if ((st = check_out_alias(p, hv, x_bytes(p), x, "hv"))) return st;
    if (overlap(hv, x_bytes(p), v, x_bytes(p))) return fail(PG_EALIAS, "hv overlaps v");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MeshView& m = p->mesh;
    MeshPass q = base_pass(p, x);
    q.xd = v;
    if (p->small) {  // one launch: the scatter into the zeroed buffer, hv written range by range
        SmallPass sp = small_pass(p);
        sp.grad = hv;
        sp.accumulate = p->opt.accumulate;
        q.gacc = p->at<double>(p->o_small);
        PG_HIP(launch_mesh_small(m, M_HVP, q, sp, s));
        return PG_OK;
    }
    const bool f32 = p->dtype == PG_F32;
    q.gacc = f32 ? p->at<double>(p->o_gacc) : static_cast<double*>(hv);  // FP32: zero between calls
    if (!f32 && !p->opt.accumulate) PG_HIP(launch_zero(q.gacc, sizeof(double) * (size_t)m.n_nodes, s));
    PG_HIP(launch_mesh_elem(m, M_HVP, q, s));
    if (f32)
        PG_HIP(launch_f64_to_f32(q.gacc, static_cast<float*>(hv), m.n_nodes, p->opt.accumulate, 1, s));
    return PG_OK;
}

pg_status pg_timing(pg_plan p, int32_t mode) {
    if (!p) return fail(PG_EINVAL, "plan is NULL");
    if (mode < 0 || mode > 2) return fail(PG_EINVAL, "timing mode %d not in {0, 1, 2}", mode);
    if (mode != 0 && p->ev.empty()) {
        p->ev.resize(2 * kMaxTimed);
        // Timing-only events: no system-scope fence (cache writeback) at record,
        // which would otherwise be counted in the kernel's time.
        for (auto& e : p->ev) PG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    p->timing_mode = mode;
    p->ev_n = 0;
    armed_launch_events() = LaunchEvents{};
    return PG_OK;
}

pg_status pg_timing_read(pg_plan p, double* total_ms, int64_t* count) {
    if (!p || !total_ms || !count) return fail(PG_EINVAL, "NULL argument");
    double tot = 0.0;
    if (p->ev_n > 0) {
        PG_HIP(hipEventSynchronize(p->ev[2 * (p->ev_n - 1) + 1]));
        for (int64_t i = 0; i < p->ev_n; ++i) {
            float ms = 0.f;
            PG_HIP(hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]));
            tot += ms;
        }
    }
    *total_ms = tot;
    *count = p->ev_n;
    p->ev_n = 0;
    return PG_OK;
}

pg_status pg_laplace1d_plan(pg_plan* plan, int64_t n, pg_dtype dtype, const pg_options* opts,
                            size_t* workspace_bytes) {
    g_err[0] = 0;
    if (!plan || !workspace_bytes) return fail(PG_EINVAL, "plan and workspace_bytes must not be NULL");
    pg_status st = check_dtype(dtype);
    if (st) return st;
    const int32_t want = opts ? opts->adjoint : PG_ADJ_AUTO;
    pg_options o;
    if ((st = check_opts(opts, &o))) return st;
    if (want == PG_ADJ_COLOUR || want == PG_ADJ_TILED)
        return fail(PG_EUNSUPPORTED, "no colour or tiled schedule for this example");
    if (n < 0 || n >= (1LL << 40)) return fail(PG_EINVAL, "n out of range");
    pg_plan_s* p = new_plan(K_LAPLACE, dtype, o);
    if (!p) return fail(PG_EINVAL, "out of host memory");
    p->lap_n = n;
    p->lap_atomic = want == PG_ADJ_ATOMIC;
    if ((st = resolve_ckpt(p, 0))) return drop_plan(p, st);
    Layout L;
    p->n_partials = (size_t)std::max<int64_t>(laplace1d_blocks(n), 1);
    p->o_partials = L.take(sizeof(double) * p->n_partials);
    p->o_flag = L.take(sizeof(int32_t) * 4);  // the fused final sum's ticket
    if (p->lap_atomic && dtype == PG_F32) p->o_gacc = L.take(sizeof(double) * (size_t)n);
    p->ws_bytes = L.total;
    *workspace_bytes = p->ws_bytes;
    *plan = p;
    return PG_OK;
}

namespace {
pg_status laplace_args(pg_plan p, const void* x, const void* b) {
    pg_status st = need_bound(p);
    if (st) return st;
    if (p->kind != K_LAPLACE) return fail(PG_EUNSUPPORTED, "not a pg_laplace1d_plan");
    if (p->lap_n > 0 && (!x || !b)) return fail(PG_EINVAL, "x and b must not be NULL");
    return PG_OK;
}
}  // namespace

pg_status pg_laplace1d_objective(pg_plan p, const void* x, const void* b, double* f_out,
                                 pg_stream stream) {
    g_err[0] = 0;
    pg_status st = laplace_args(p, x, b);
    if (st) return st;
    if (!f_out) return fail(PG_EINVAL, "f_out is NULL");
    const size_t xb = x_bytes(p);
    if (overlap(f_out, 8, x, xb) || overlap(f_out, 8, b, xb) || overlap(f_out, 8, p->ws, p->ws_bytes))
        return fail(PG_EALIAS, "f_out overlaps an input or the workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* partials = p->at<double>(p->o_partials);
    const Dtype dt = p->dtype == PG_F64 ? F64 : F32;
    PG_HIP(tmark(p, 2, true, s));
    int32_t* ticket = p->at<int32_t>(p->o_flag);
    const bool fused = laplace1d_fused(p->lap_n);
    PG_HIP(tkern(p, true));
    PG_HIP(launch_laplace1d(p->lap_n, dt, 0, x, b, nullptr, nullptr, nullptr, nullptr, partials, 0,
                            ticket, f_out, s));
    PG_HIP(tkern(p, false));
    if (!fused) PG_HIP(launch_final_sum(partials, laplace1d_blocks(p->lap_n), f_out, s));
    PG_HIP(tmark(p, 2, false, s));
    return PG_OK;
}

pg_status pg_laplace1d_gradient(pg_plan p, const void* x, const void* b, void* gx, void* gb,
                                double* f_out, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = laplace_args(p, x, b);
    if (st) return st;
    const size_t xb = x_bytes(p);
    const void* outs[3] = {gx, gb, f_out};
    const size_t ob[3] = {xb, xb, 8};
    for (int i = 0; i < 3; ++i) {
        if (overlap(outs[i], ob[i], x, xb) || overlap(outs[i], ob[i], b, xb) ||
            overlap(outs[i], ob[i], p->ws, p->ws_bytes))
            return fail(PG_EALIAS, "an output overlaps an input or the workspace");
        for (int j = 0; j < i; ++j)
            if (overlap(outs[i], ob[i], outs[j], ob[j])) return fail(PG_EALIAS, "outputs overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* partials = p->at<double>(p->o_partials);
    const Dtype dt = p->dtype == PG_F64 ? F64 : F32;
    const int acc = p->opt.accumulate;
    int32_t* ticket = p->at<int32_t>(p->o_flag);
    const bool fused = laplace1d_fused(p->lap_n);
    PG_HIP(tmark(p, 2, true, s));
    if (p->lap_atomic) {
        double* g64 = nullptr;
        if (gx) {
            g64 = dt == F64 ? static_cast<double*>(gx) : p->at<double>(p->o_gacc);
            if (dt == F32 || !acc) PG_HIP(launch_zero(g64, sizeof(double) * (size_t)p->lap_n, s));
        }
        PG_HIP(tkern(p, true));
        PG_HIP(launch_laplace1d(p->lap_n, dt, 2, x, b, g64, nullptr, gb, nullptr, partials, acc,
                                ticket, f_out, s));
        PG_HIP(tkern(p, false));
        if (gx && dt == F32) PG_HIP(launch_f64_to_f32(g64, static_cast<float*>(gx), p->lap_n, acc, 0, s));
    } else {
        PG_HIP(tkern(p, true));
        PG_HIP(launch_laplace1d(p->lap_n, dt, 1, x, b, nullptr, gx, gb, nullptr, partials, acc,
                                ticket, f_out, s));
        PG_HIP(tkern(p, false));
    }
    if (f_out && !fused) PG_HIP(launch_final_sum(partials, laplace1d_blocks(p->lap_n), f_out, s));
    PG_HIP(tmark(p, 2, false, s));
    return PG_OK;
}

pg_status pg_jvp(pg_plan p, const void* x, const void* d, double* jvp_out, pg_stream stream) {
    g_err[0] = 0;
    pg_status st = need_bound(p);
    if (st) return st;
    if (p->kind != K_MESH) return fail(PG_EUNSUPPORTED, "pg_jvp supports mesh plans only");
    if ((!x || !d) && x_bytes(p) > 0) return fail(PG_EINVAL, "x and d must not be NULL");
    if (!jvp_out) return fail(PG_EINVAL, "jvp_out is NULL");
    if ((st = check_out_alias(p, jvp_out, sizeof(double), x, "jvp_out"))) return st;
    if (overlap(jvp_out, sizeof(double), d, x_bytes(p))) return fail(PG_EALIAS, "jvp_out overlaps d");
    hipStream_t s = static_cast<hipStream_t>(stream);
    MeshPass q = base_pass(p, x);
    q.xd = d;
    if (p->small) {  // one launch: the last workgroup sums the partials
        SmallPass sp = small_pass(p);
        sp.f_out = jvp_out;
        PG_HIP(launch_mesh_small(p->mesh, M_JVP, q, sp, s));
        return PG_OK;
    }
    PG_HIP(launch_mesh_elem(p->mesh, M_JVP, q, s));
    PG_HIP(launch_final_sum(q.partials, p->mesh_blocks_n, jvp_out, s));
    return PG_OK;
}

pg_status pg_scale(pg_dtype dtype, int64_t n, const double* alpha, const void* x, void* y,
                   pg_stream stream) {
    g_err[0] = 0;
    pg_status st = check_dtype(dtype);
    if (st) return st;
    if (n < 0) return fail(PG_EINVAL, "n must be >= 0");
    if (!alpha) return fail(PG_EINVAL, "alpha is NULL");
    if (n > 0 && (!x || !y)) return fail(PG_EINVAL, "x and y must not be NULL");
    const size_t nb = esize(dtype) * (size_t)n;
    if (x != y && overlap(x, nb, y, nb)) return fail(PG_EALIAS, "x and y overlap without being equal");
    if (overlap(alpha, sizeof(double), y, nb)) return fail(PG_EALIAS, "alpha overlaps y");
    PG_HIP(launch_scale(dtype == PG_F64 ? F64 : F32, n, alpha, x, y, static_cast<hipStream_t>(stream)));
    return PG_OK;
}

pg_status pg_plan_info(pg_plan p, pg_plan_info_t* info) {
    g_err[0] = 0;
    if (!p || !info) return fail(PG_EINVAL, "plan and info must not be NULL");
    pg_plan_info_t r;
    std::memset(&r, 0, sizeof r);
    r.kind = (int32_t)p->kind;
    r.dtype = (int32_t)p->dtype;
    r.adjoint = p->kind == K_LAPLACE ? (p->lap_atomic ? PG_ADJ_ATOMIC : PG_ADJ_GATHER) : p->opt.adjoint;
    r.ckpt = p->opt.ckpt;
    r.block = p->opt.block;
    r.tile = p->opt.tile;
    const bool table = (p->kind == K_MESH || p->kind == K_BATCH) && p->opt.adjoint == PG_ADJ_ATOMIC &&
                       p->opt.scatter != 1;
    r.lds_slots = table && p->bound ? (p->kind == K_BATCH ? 4096 : p->agg_slots) : 0;
    if (p->kind == K_MESH && p->opt.adjoint == PG_ADJ_TILED && p->bound)
        r.lds_slots = p->tiled_round_slots;
    r.one_launch = p->small ? 1 : 0;
    r.n_colours = p->colour_off.empty() ? 0 : (int32_t)(p->colour_off.size() - 1);
    r.bound = p->bound ? 1 : 0;
    r.workspace_bytes = (int64_t)p->ws_bytes;
    r.tape_bytes = (int64_t)p->tape_bytes;
    r.tape_budget = p->tape_budget;
    *info = r;
    return PG_OK;
}

pg_status pg_plan_export(pg_plan p, int32_t what, void* host_dst, size_t capacity, size_t* bytes) {
    g_err[0] = 0;
    if (!p || !bytes) return fail(PG_EINVAL, "plan and bytes must not be NULL");
    if (!p->bound) return fail(PG_ESTATE, "plan has no workspace bound (call pg_bind_workspace)");
    if (p->kind != K_MESH) return fail(PG_EUNSUPPORTED, "only mesh plans export structures");
    const MeshView& m = p->mesh;
    const void* dev = nullptr;
    const void* host = nullptr;
    size_t nb = 0;
    switch (what) {
        case PG_EXPORT_CSR_OFFS:
        case PG_EXPORT_CSR_INC:
            if (p->opt.adjoint != PG_ADJ_GATHER)
                return fail(PG_EUNSUPPORTED, "the transposed connectivity belongs to the gather adjoint");
            if (what == PG_EXPORT_CSR_OFFS) {
                dev = p->at<int32_t>(p->o_offs);
                nb = sizeof(int32_t) * (size_t)(m.n_nodes + 1);
            } else {
                dev = p->at<int32_t>(p->o_inc);
                nb = sizeof(int32_t) * (size_t)(m.n_elems * m.k);
            }
            break;
        case PG_EXPORT_COLOUR_OFFS:
        case PG_EXPORT_COLOUR_ELEMS:
            if (p->opt.adjoint != PG_ADJ_COLOUR)
                return fail(PG_EUNSUPPORTED, "colour classes belong to the colour adjoint");
            if (what == PG_EXPORT_COLOUR_OFFS) {
                host = p->colour_off.data();
                nb = sizeof(int64_t) * p->colour_off.size();
            } else {
                dev = p->at<int32_t>(p->o_elist);
                nb = sizeof(int32_t) * (size_t)m.n_elems;
            }
            break;
        default: return fail(PG_EINVAL, "unknown export %d", what);
    }
    *bytes = nb;
    if (!host_dst) return PG_OK;
    if (capacity < nb) return fail(PG_EINVAL, "capacity %zu < %zu bytes", capacity, nb);
    if (nb == 0) return PG_OK;
    if (host)
        std::memcpy(host_dst, host, nb);
    else
        PG_HIP(hipMemcpy(host_dst, dev, nb, hipMemcpyDeviceToHost));
    return PG_OK;
}

pg_status pg_plan_destroy(pg_plan p) {
    if (p) {
        // A launch that failed after arming leaves the pair armed: drop it.
        LaunchEvents& a = armed_launch_events();
        for (auto& e : p->ev)
            if (a.start == e || a.stop == e) a = LaunchEvents{};
        for (auto& e : p->ev) (void)hipEventDestroy(e);
    }
    delete p;
    return PG_OK;
}

}  // extern "C"
