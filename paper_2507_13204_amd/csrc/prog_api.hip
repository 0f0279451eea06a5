// C ABI of composed programs: building, activity analysis, tape layout, and
// the generated forward and reverse passes.  Host code only.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <new>
#include <vector>

#include "launch.hpp"
#include "pgrad.h"

namespace pg {
pg_status set_error(pg_status s, const char* msg);
void clear_error();
}  // namespace pg

using namespace pg;

namespace {

pg_status perr(pg_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(s, buf);
}

#define PG_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return perr(PG_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = PG_WORKSPACE_ALIGN;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr size_t NONE = ~size_t(0);

struct Op {
    int kind = P_INPUT;
    int64_t n = 0;          // length of the output view
    int32_t a = -1, b = -1; // operand views
    double alpha = 1.0, beta = 1.0;
    int fn = 0;
    ProgTaps taps;
    int32_t a0 = -1;        // operand and taps as built (the plan may fold a scale into a stencil)
    ProgTaps taps0;
    int32_t k = 0;
    const int32_t* conn = nullptr;
    const double* B = nullptr;
    const double* data = nullptr;  // P_CONST
    const int64_t* offs = nullptr; // P_SEGSUM, P_BCAST: segment offsets (n_seg + 1)
    int64_t n_seg = 0;
    int32_t input_index = -1;      // P_INPUT
    // plan
    bool live = false;       // feeds the summed view
    bool active = false;     // depends on an input
    int32_t group = -1;      // fused group holding this pointwise construct
    bool fused = false;      // a gather evaluated inside its consuming group
    bool stored = false;     // forward value materialised
    bool exported = false;   // group member read from outside its group
    bool folded = false;     // a scale folded into the stencil reading it
    size_t val_off = NONE;   // forward value in the workspace (intermediates)
    size_t shd_off = NONE;   // shadow in the workspace (active intermediates)
};

bool pointwise(int kind) { return kind == P_SCALE || kind == P_ADD || kind == P_MUL || kind == P_MAP; }

struct Group {
    std::vector<int32_t> members, leaves;
    int32_t gather = -1;  // fused gather view (one of the leaves)
    bool export_gather = false;  // a gather of its own: no ops, its value written out
    bool sealed = false, has_sum = false;
    int32_t pos = 0;      // schedule position: its last member (the end for a sum-only group)
    uint32_t hash_shift = kHashRotDefault;
    int agg_slots = 4096;
};

// One step of the forward schedule: a non-pointwise construct or a group.
struct Item {
    bool group;
    int32_t id;
    int32_t pos;
};

// How a reverse step delivers into an operand's shadow.
enum Deliver { D_STORE = 0, D_ADD = 1, D_ATOMIC = 2 };

}  // namespace

struct pg_prog_s {
    std::vector<Op> ops;  // one per view, in creation order (view id = index)
    int32_t sum_view = -1;
    int32_t n_inputs = 0;
    int32_t fusion = 1;
    bool planned = false;
    std::vector<Group> groups;
    std::vector<Item> sched;                       // forward order
    int32_t sum_group = -1;
    bool sum_ticket = false;  // the sum group's last workgroup writes f (no reduction launch)
    std::vector<int32_t> zero_views;               // shadows cleared before the reverse pass
    std::vector<int32_t> op_acc;                   // per view: delivery of a construct's reverse
    std::vector<std::vector<int32_t>> leaf_acc;    // per group, per leaf
    size_t ws_bytes = 0, partials_off = NONE, fscratch_off = NONE, flag_off = NONE, scan_off = NONE;
    int64_t tape_bytes = 0;
    std::vector<size_t> input_shadow_off;  // internal shadows for inputs without a grad buffer
    char* ws = nullptr;
    pg_prog_stats stats{};
};

namespace {

pg_status add_view(pg_prog p, const Op& op, int32_t* view) {
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (p->sum_view >= 0) return perr(PG_ESTATE, "the program already ended with pg_prog_sum");
    if (!view) return perr(PG_EINVAL, "view is NULL");
    p->ops.push_back(op);
    p->ops.back().a0 = op.a;
    p->ops.back().taps0 = op.taps;
    p->planned = false;
    *view = (int32_t)p->ops.size() - 1;
    return PG_OK;
}

pg_status check_view(pg_prog p, int32_t v) {
    if (v < 0 || v >= (int32_t)p->ops.size()) return perr(PG_EINVAL, "view %d does not exist", v);
    return PG_OK;
}

double* at(pg_prog p, size_t off) { return off == NONE ? nullptr : reinterpret_cast<double*>(p->ws + off); }

}  // namespace

extern "C" {

pg_status pg_prog_create(pg_prog* prog) {
    clear_error();
    if (!prog) return perr(PG_EINVAL, "prog is NULL");
    pg_prog_s* p = new (std::nothrow) pg_prog_s();
    if (!p) return perr(PG_EINVAL, "out of host memory");
    *prog = p;
    return PG_OK;
}

pg_status pg_prog_input(pg_prog p, int64_t n, int32_t* view) {
    clear_error();
    if (n < 0 || n >= (1LL << 31)) return perr(PG_EINVAL, "input length out of range");
    Op op;
    op.kind = P_INPUT;
    op.n = n;
    op.input_index = p ? p->n_inputs : -1;
    pg_status st = add_view(p, op, view);
    if (st == PG_OK) ++p->n_inputs;
    return st;
}

pg_status pg_prog_const(pg_prog p, int64_t n, const double* data, int32_t* view) {
    clear_error();
    if (n < 0 || n >= (1LL << 31)) return perr(PG_EINVAL, "length out of range");
    if (n > 0 && !data) return perr(PG_EINVAL, "data is NULL");
    Op op;
    op.kind = P_CONST;
    op.n = n;
    op.data = data;
    return add_view(p, op, view);
}

pg_status pg_prog_scale(pg_prog p, int32_t a, double alpha, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    Op op;
    op.kind = P_SCALE;
    op.n = p->ops[a].n;
    op.a = a;
    op.alpha = alpha;
    return add_view(p, op, view);
}

pg_status pg_prog_stencil(pg_prog p, int32_t a, int32_t n_taps, const int32_t* offsets,
                          const double* coeffs, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    if (n_taps < 1 || n_taps > kMaxTaps || !offsets || !coeffs)
        return perr(PG_EINVAL, "n_taps must be in [1, %d] with host offsets and coeffs", kMaxTaps);
    Op op;
    op.kind = P_STENCIL;
    op.n = p->ops[a].n;
    op.a = a;
    op.taps.n = n_taps;
    for (int t = 0; t < n_taps; ++t) {
        op.taps.off[t] = offsets[t];
        op.taps.coef[t] = coeffs[t];
    }
    return add_view(p, op, view);
}

pg_status pg_prog_gather(pg_prog p, int32_t a, int64_t n_elems, int32_t k, const int32_t* conn,
                         const double* B, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    if (n_elems < 0 || n_elems >= (1LL << 31) || k < 1 || k > PG_MAX_K || n_elems * k >= (1LL << 31))
        return perr(PG_EINVAL, "gather sizes out of range");
    if (n_elems > 0 && (!conn || !B)) return perr(PG_EINVAL, "conn and B must not be NULL");
    Op op;
    op.kind = P_GATHER;
    op.n = n_elems;
    op.a = a;
    op.k = k;
    op.conn = conn;
    op.B = B;
    return add_view(p, op, view);
}

pg_status pg_prog_add(pg_prog p, int32_t a, double alpha, int32_t b, double beta, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st || (st = check_view(p, b))) return st;
    if (p->ops[a].n != p->ops[b].n) return perr(PG_EINVAL, "add: operand lengths differ");
    Op op;
    op.kind = P_ADD;
    op.n = p->ops[a].n;
    op.a = a;
    op.b = b;
    op.alpha = alpha;
    op.beta = beta;
    return add_view(p, op, view);
}

pg_status pg_prog_mul(pg_prog p, int32_t a, int32_t b, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st || (st = check_view(p, b))) return st;
    if (p->ops[a].n != p->ops[b].n) return perr(PG_EINVAL, "mul: operand lengths differ");
    Op op;
    op.kind = P_MUL;
    op.n = p->ops[a].n;
    op.a = a;
    op.b = b;
    return add_view(p, op, view);
}

pg_status pg_prog_map(pg_prog p, int32_t a, pg_map_fn fn, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    if (fn != PG_MAP_SQUARE && fn != PG_MAP_PSI) return perr(PG_EINVAL, "unknown map function");
    Op op;
    op.kind = P_MAP;
    op.n = p->ops[a].n;
    op.a = a;
    op.fn = (int)fn;
    return add_view(p, op, view);
}

pg_status pg_prog_scan(pg_prog p, int32_t a, int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    Op op;
    op.kind = P_SCAN;
    op.n = p->ops[a].n;
    op.a = a;
    return add_view(p, op, view);
}

pg_status pg_prog_segment_sum(pg_prog p, int32_t a, int64_t n_seg, const int64_t* offsets,
                              int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    if (n_seg < 0 || n_seg >= (1LL << 31) || !offsets)
        return perr(PG_EINVAL, "n_seg out of range or offsets NULL");
    Op op;
    op.kind = P_SEGSUM;
    op.n = n_seg;
    op.a = a;
    op.offs = offsets;
    op.n_seg = n_seg;
    return add_view(p, op, view);
}

pg_status pg_prog_broadcast(pg_prog p, int32_t a, const int64_t* offsets, int64_t n_out,
                            int32_t* view) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    if (n_out < 0 || n_out >= (1LL << 31) || !offsets)
        return perr(PG_EINVAL, "n_out out of range or offsets NULL");
    Op op;
    op.kind = P_BCAST;
    op.n = n_out;
    op.a = a;
    op.offs = offsets;
    op.n_seg = p->ops[(size_t)a].n;
    return add_view(p, op, view);
}

pg_status pg_prog_sum(pg_prog p, int32_t a) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    pg_status st = check_view(p, a);
    if (st) return st;
    if (p->sum_view >= 0) return perr(PG_ESTATE, "the program already ended with pg_prog_sum");
    p->sum_view = a;
    p->planned = false;
    return PG_OK;
}

pg_status pg_prog_fusion(pg_prog p, int32_t level) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (level != 0 && level != 1) return perr(PG_EINVAL, "fusion level must be 0 or 1");
    p->fusion = level;
    p->planned = false;
    return PG_OK;
}

pg_status pg_prog_plan(pg_prog p, size_t* workspace_bytes) {
    clear_error();
    if (!p || !workspace_bytes) return perr(PG_EINVAL, "NULL argument");
    if (p->sum_view < 0) return perr(PG_ESTATE, "the program has no pg_prog_sum");
    std::vector<Op>& ops = p->ops;
    const int32_t nv = (int32_t)ops.size(), S = p->sum_view;
    for (Op& op : ops) {
        op.a = op.a0;
        op.taps = op.taps0;
        op.folded = false;
    }
    // A scale whose only reader is a stencil folds into the stencil's
    // coefficients: c (alpha a) = (c alpha) a, forward and reverse alike.
    if (p->fusion) {
        std::vector<int32_t> readers((size_t)nv, 0);
        for (const Op& op : ops) {
            if (op.a >= 0) readers[(size_t)op.a]++;
            if (op.b >= 0) readers[(size_t)op.b]++;
        }
        readers[(size_t)S]++;
        for (int32_t v = 0; v < nv; ++v) {
            Op& st = ops[(size_t)v];
            if (st.kind != P_STENCIL) continue;
            while (ops[(size_t)st.a].kind == P_SCALE && readers[(size_t)st.a] == 1) {
                Op& sc = ops[(size_t)st.a];
                for (int t = 0; t < st.taps.n; ++t) st.taps.coef[t] *= sc.alpha;
                sc.folded = true;
                st.a = sc.a;  // the scale's own read of its operand moves to the stencil
            }
        }
    }
    // Liveness: only what feeds the summed view runs.
    for (Op& op : ops) {
        op.live = false;
        op.group = -1;
        op.fused = op.stored = op.exported = false;
        op.val_off = op.shd_off = NONE;
    }
    ops[(size_t)S].live = true;
    for (int32_t v = S; v >= 0; --v) {
        if (!ops[(size_t)v].live) continue;
        if (ops[(size_t)v].a >= 0) ops[(size_t)ops[(size_t)v].a].live = true;
        if (ops[(size_t)v].b >= 0) ops[(size_t)ops[(size_t)v].b].live = true;
    }
    // Activity: a view is active if it is an input or reads an active view.
    for (Op& op : ops)
        op.active = op.kind == P_INPUT || (op.a >= 0 && ops[(size_t)op.a].active) ||
                    (op.b >= 0 && ops[(size_t)op.b].active);

    // Fused groups of pointwise constructs.  A group runs where its last
    // member is; once a construct outside it reads a member, it is sealed
    // (it must run before that reader) and takes no further members.
    std::vector<Group>& G = p->groups;
    G.clear();
    auto add_leaf = [&](Group& g, int32_t u) {
        if (std::find(g.leaves.begin(), g.leaves.end(), u) == g.leaves.end()) g.leaves.push_back(u);
    };
    auto read_member = [&](int32_t u, int32_t reader_group) {
        const int32_t gu = ops[(size_t)u].group;
        if (gu >= 0 && gu != reader_group) {
            G[(size_t)gu].sealed = true;
            ops[(size_t)u].exported = true;
        }
    };
    auto leaves_after = [&](const std::vector<int32_t>& gs, int32_t v) {
        // leaves of the union of groups gs plus construct v
        std::vector<int32_t> mem, lv;
        for (int32_t gi : gs) mem.insert(mem.end(), G[(size_t)gi].members.begin(), G[(size_t)gi].members.end());
        mem.push_back(v);
        auto add = [&](int32_t u) {
            if (u < 0 || std::find(mem.begin(), mem.end(), u) != mem.end()) return;
            if (std::find(lv.begin(), lv.end(), u) == lv.end()) lv.push_back(u);
        };
        for (int32_t gi : gs)
            for (int32_t u : G[(size_t)gi].leaves) add(u);
        add(ops[(size_t)v].a);
        add(ops[(size_t)v].b);
        return std::make_pair(mem.size(), lv.size());
    };
    for (int32_t v = 0; v < nv; ++v) {
        Op& op = ops[(size_t)v];
        if (!op.live || op.kind == P_INPUT || op.kind == P_CONST) continue;
        if (!pointwise(op.kind)) {
            read_member(op.a, -1);
            continue;
        }
        std::vector<int32_t> cand;
        if (p->fusion) {
            for (int32_t u : {op.a, op.b}) {
                if (u < 0) continue;
                const int32_t gu = ops[(size_t)u].group;
                if (gu >= 0 && !G[(size_t)gu].sealed &&
                    std::find(cand.begin(), cand.end(), gu) == cand.end())
                    cand.push_back(gu);
            }
            auto fits = [&](const std::vector<int32_t>& gs) {
                const auto ml = leaves_after(gs, v);
                return (int)ml.first <= kGOps && (int)ml.second <= kGLeaves &&
                       (int)(ml.first + ml.second) <= kGSlots;
            };
            if (!cand.empty() && !fits(cand)) {
                std::vector<int32_t> one;
                for (int32_t gi : cand)
                    if (fits({gi})) {
                        one.push_back(gi);
                        break;
                    }
                cand = one;
            }
        }
        int32_t gi;
        if (cand.empty()) {
            gi = (int32_t)G.size();
            G.emplace_back();
        } else {
            gi = cand[0];
            for (size_t c = 1; c < cand.size(); ++c) {  // merge into the first
                Group& src = G[(size_t)cand[c]];
                for (int32_t m : src.members) ops[(size_t)m].group = gi;
                G[(size_t)gi].members.insert(G[(size_t)gi].members.end(), src.members.begin(), src.members.end());
                for (int32_t u : src.leaves) add_leaf(G[(size_t)gi], u);
                src.members.clear();
                src.leaves.clear();
            }
        }
        Group& g = G[(size_t)gi];
        g.members.push_back(v);
        op.group = gi;
        std::sort(g.members.begin(), g.members.end());
        // leaves: operands outside the group (drop any that became members)
        std::vector<int32_t> lv;
        for (int32_t u : g.leaves)
            if (ops[(size_t)u].group != gi) lv.push_back(u);
        g.leaves = lv;
        for (int32_t u : {op.a, op.b}) {
            if (u < 0) continue;
            read_member(u, gi);
            if (ops[(size_t)u].group != gi) add_leaf(g, u);
        }
    }
    // The sum joins the group holding the summed view, else a group of its own.
    if (ops[(size_t)S].group >= 0) {
        p->sum_group = ops[(size_t)S].group;
    } else {
        p->sum_group = (int32_t)G.size();
        G.emplace_back();
        G.back().leaves.push_back(S);
        G.back().pos = nv;
    }
    G[(size_t)p->sum_group].has_sum = true;
    // Gathers read only by one group (as a leaf) run inside it, unless that
    // group also reads the gather's operand (its shadow would then take a
    // plain store and atomics in one kernel).
    if (p->fusion) {
        std::vector<int32_t> readers((size_t)nv, 0), reader_group((size_t)nv, -1);
        for (int32_t v = 0; v < nv; ++v) {
            const Op& op = ops[(size_t)v];
            if (!op.live || op.kind == P_INPUT || op.kind == P_CONST || pointwise(op.kind)) continue;
            readers[(size_t)op.a]++;
        }
        for (size_t gi = 0; gi < G.size(); ++gi)
            for (int32_t u : G[gi].leaves) {
                readers[(size_t)u]++;
                reader_group[(size_t)u] = (int32_t)gi;
            }
        for (int32_t v = 0; v < nv; ++v) {
            Op& op = ops[(size_t)v];
            if (!op.live || op.kind != P_GATHER || readers[(size_t)v] != 1 || reader_group[(size_t)v] < 0)
                continue;
            Group& g = G[(size_t)reader_group[(size_t)v]];
            if (g.gather >= 0 || std::find(g.leaves.begin(), g.leaves.end(), op.a) != g.leaves.end())
                continue;
            g.gather = v;
            op.fused = true;
        }
    }
    // Every other gather runs in a group of its own that writes its value out,
    // so it gets the same row loads and LDS-combined reverse scatter.
    for (int32_t v = 0; v < nv; ++v) {
        const Op& op = ops[(size_t)v];
        if (!op.live || op.kind != P_GATHER || op.fused) continue;
        G.emplace_back();
        G.back().leaves.push_back(v);
        G.back().gather = v;
        G.back().export_gather = true;
        G.back().pos = v;
    }
    // Forward schedule.
    p->sched.clear();
    for (size_t gi = 0; gi < G.size(); ++gi) {
        Group& g = G[gi];
        if (g.members.empty() && !g.has_sum && g.gather < 0) continue;  // merged away
        if (!g.members.empty()) g.pos = g.members.back();
        p->sched.push_back(Item{true, (int32_t)gi, g.pos});
    }
    for (int32_t v = 0; v < nv; ++v) {
        const Op& op = ops[(size_t)v];
        if (op.live && op.kind != P_GATHER && !pointwise(op.kind) && op.kind != P_INPUT &&
            op.kind != P_CONST)
            p->sched.push_back(Item{false, v, v});
    }
    std::sort(p->sched.begin(), p->sched.end(),
              [](const Item& x, const Item& y) { return x.pos < y.pos; });
    // Materialised views: outputs of stand-alone constructs and group exports.
    for (Op& op : ops) {
        if (!op.live || op.kind == P_INPUT || op.kind == P_CONST || op.fused) continue;
        op.stored = !pointwise(op.kind) || op.exported;
    }
    // Reverse deliveries: walk the reverse schedule; a shadow's first
    // delivery stores, later ones add; an atomic delivery needs a cleared
    // shadow.  The sum group runs first (fused with its forward when asked).
    p->op_acc.assign((size_t)nv, D_ADD);
    p->leaf_acc.assign(G.size(), {});
    p->zero_views.clear();
    std::vector<char> touched((size_t)nv, 0);
    auto deliver = [&](int32_t v, bool atomic) -> int32_t {
        if (!ops[(size_t)v].active) return D_ADD;
        if (atomic) {
            if (!touched[(size_t)v]) p->zero_views.push_back(v);
            touched[(size_t)v] = 1;
            return D_ATOMIC;
        }
        const int32_t d = touched[(size_t)v] ? D_ADD : D_STORE;
        touched[(size_t)v] = 1;
        return d;
    };
    for (size_t r = p->sched.size(); r-- > 0;) {
        const Item& it = p->sched[r];
        if (it.group) {
            Group& g = G[(size_t)it.id];
            std::vector<int32_t>& la = p->leaf_acc[(size_t)it.id];
            la.assign(g.leaves.size(), D_ADD);
            for (size_t l = 0; l < g.leaves.size(); ++l) {
                if (g.leaves[l] == g.gather) continue;
                la[l] = deliver(g.leaves[l], false);
            }
            if (g.gather >= 0) deliver(ops[(size_t)g.gather].a, true);
        } else {
            const Op& op = ops[(size_t)it.id];
            if (!op.active) continue;
            p->op_acc[(size_t)it.id] = deliver(op.a, false);
        }
    }
    for (int32_t v = 0; v < nv; ++v)
        if (ops[(size_t)v].kind == P_INPUT && !touched[(size_t)v]) p->zero_views.push_back(v);

    // Workspace layout.
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    p->tape_bytes = 0;
    for (Op& op : ops) {
        if (!op.stored) continue;
        op.val_off = take(sizeof(double) * (size_t)op.n);
        p->tape_bytes += (int64_t)(sizeof(double) * (size_t)op.n);
        if (op.active) op.shd_off = take(sizeof(double) * (size_t)op.n);
    }
    p->input_shadow_off.assign((size_t)p->n_inputs, NONE);
    for (const Op& op : ops)
        if (op.kind == P_INPUT)
            p->input_shadow_off[(size_t)op.input_index] = take(sizeof(double) * (size_t)op.n);
    p->partials_off =
        take(sizeof(double) * (size_t)std::max<int64_t>(group_blocks(ops[(size_t)S].n, kGroupBlock), 1));
    p->fscratch_off = take(sizeof(double));
    p->flag_off = take(sizeof(int32_t) * 4);
    int64_t scan_chunks = 0;  // one totals buffer, reused by every scan in turn
    for (const Op& op : ops)
        if (op.live && op.kind == P_SCAN) scan_chunks = std::max(scan_chunks, prog_scan_chunks(op.n));
    p->scan_off = scan_chunks ? take(sizeof(double) * (size_t)scan_chunks) : NONE;
    p->ws_bytes = off;

    // What the transformation produced.
    pg_prog_stats& st = p->stats;
    st = pg_prog_stats{};
    for (const Item& it : p->sched) {
        if (it.group) {
            const Group& g = G[(size_t)it.id];
            ++st.groups;
            ++st.fwd_kernels;
            bool rev = g.gather >= 0 && ops[(size_t)ops[(size_t)g.gather].a].active;
            for (int32_t u : g.leaves) rev = rev || (u != g.gather && ops[(size_t)u].active);
            if (rev && !(p->fusion && g.has_sum)) ++st.rev_kernels;
            if (g.gather >= 0) {
                if (!g.export_gather) ++st.fused_gathers;
                if (ops[(size_t)ops[(size_t)g.gather].a].active) ++st.atomic_ops;
            }
        } else {
            const Op& op = ops[(size_t)it.id];
            const int32_t nk = op.kind == P_SCAN ? 3 : 1;  // a scan is three launches each way
            st.fwd_kernels += nk;
            if (!op.active) continue;
            st.rev_kernels += nk;
            if (op.kind == P_STENCIL && op.taps.n > 1) ++st.rescheduled_ops;
        }
    }
    // The fixed-order reduction of the sum's partials: a launch of its own,
    // or (fused, at most 64 workgroups) the sum group's last workgroup.
    p->sum_ticket = p->fusion && ops[(size_t)S].n > 0 && ops[(size_t)S].n <= 64 * (int64_t)kGroupBlock;
    if (!p->sum_ticket) st.fwd_kernels += 1;
    for (const Op& op : ops) {
        if (op.folded) ++st.folded_ops;
        else if (!op.live && op.kind != P_INPUT && op.kind != P_CONST) ++st.dead_ops;
    }
    st.tape_bytes = p->tape_bytes;
    st.workspace_bytes = (int64_t)p->ws_bytes;
    p->planned = true;
    p->ws = nullptr;
    *workspace_bytes = p->ws_bytes;
    return PG_OK;
}

pg_status pg_prog_bind_workspace(pg_prog p, void* ws, size_t bytes) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (!p->planned) return perr(PG_ESTATE, "call pg_prog_plan first");
    if (!ws || bytes < p->ws_bytes || (uintptr_t)ws % kAlign)
        return perr(PG_EWORKSPACE, "workspace must hold %zu bytes, %zu-byte aligned", p->ws_bytes, kAlign);
    // Every gather's connectivity must address its operand: checked once here.
    int32_t* flag = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + p->flag_off);
    PG_HIP(launch_zero(flag, sizeof(int32_t) * 4, nullptr));
    for (const Op& op : p->ops)
        if (op.kind == P_GATHER)
            PG_HIP(launch_validate_count(op.conn, op.n * op.k, p->ops[(size_t)op.a].n, nullptr, flag,
                                         nullptr));
    int32_t hflag = 0;
    PG_HIP(hipMemcpy(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost));
    if (hflag) return perr(PG_ERANGE, "a gather's connectivity has an entry outside its operand");
    // Segment offsets must start at 0, not decrease and end at the summed length.
    for (const Op& op : p->ops) {
        if (op.kind != P_SEGSUM && op.kind != P_BCAST) continue;
        const int64_t total = op.kind == P_SEGSUM ? p->ops[(size_t)op.a].n : op.n;
        PG_HIP(launch_validate_offsets(op.offs, op.n_seg, total, flag, nullptr));
    }
    PG_HIP(hipMemcpy(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost));
    if (hflag) return perr(PG_ERANGE, "segment offsets are not 0 = o_0 <= ... <= o_n_seg = length");
    // LDS table size and hash rotation of each fused gather's scatter, chosen
    // on sampled workgroups.
    for (Group& g : p->groups) {
        if (g.gather < 0) continue;
        const Op& op = p->ops[(size_t)g.gather];
        const int64_t span = kGroupBlockScatter, nt = (op.n + span - 1) / span;
        const int64_t ns = std::min<int64_t>(nt, 64);
        std::vector<std::vector<int32_t>> tiles;
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t t = nt > 1 ? q * (nt - 1) / std::max<int64_t>(ns - 1, 1) : 0;
            const int64_t e0 = t * span, e1 = std::min(op.n, e0 + span);
            tiles.emplace_back((size_t)((e1 - e0) * op.k));
            if (tiles.back().empty()) continue;
            PG_HIP(hipMemcpy(tiles.back().data(), op.conn + e0 * op.k,
                             sizeof(int32_t) * tiles.back().size(), hipMemcpyDeviceToHost));
        }
        std::vector<const int32_t*> ptr;
        std::vector<int64_t> cnt;
        for (const auto& t : tiles) {
            ptr.push_back(t.data());
            cnt.push_back((int64_t)t.size());
        }
        if (tiles.empty()) continue;
        choose_table(ptr.data(), cnt.data(), (int64_t)tiles.size(), &g.agg_slots, &g.hash_shift);
        // The smaller table only if no workgroup of the gather would probe in it.
        if (g.agg_slots == 2048) {
            PG_HIP(launch_zero(flag + 2, sizeof(int32_t), nullptr));
            PG_HIP(launch_table_check(op.conn, op.n, op.k, span, g.hash_shift, 2048, flag + 2, nullptr));
            int32_t miss = 0;
            PG_HIP(hipMemcpy(&miss, flag + 2, sizeof miss, hipMemcpyDeviceToHost));
            if (miss) {
                g.agg_slots = 4096;
                g.hash_shift = choose_hash_shift(ptr.data(), cnt.data(), (int64_t)tiles.size(), 4096,
                                                 nullptr);
            }
        }
    }
    p->ws = static_cast<char*>(ws);
    return PG_OK;
}

pg_status pg_prog_run(pg_prog p, const double* const* inputs, double* f_out, double* const* grads,
                      const double* fbar, pg_stream stream) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (!p->planned || !p->ws) return perr(PG_ESTATE, "plan the program and bind a workspace first");
    if (p->n_inputs > 0 && !inputs) return perr(PG_EINVAL, "inputs is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::vector<Op>& ops = p->ops;
    const size_t nv = ops.size();
    // Device pointers of every view's forward value and shadow.
    std::vector<const double*> val(nv, nullptr);
    std::vector<double*> shd(nv, nullptr);
    for (size_t v = 0; v < nv; ++v) {
        const Op& op = ops[v];
        if (op.kind == P_INPUT) {
            val[v] = inputs[op.input_index];
            if (op.n > 0 && !val[v]) return perr(PG_EINVAL, "input %d is NULL", op.input_index);
            double* g = grads ? grads[op.input_index] : nullptr;
            shd[v] = g ? g : at(p, p->input_shadow_off[(size_t)op.input_index]);
        } else if (op.kind == P_CONST) {
            val[v] = op.data;
        } else {
            val[v] = at(p, op.val_off);
            shd[v] = at(p, op.shd_off);
        }
    }
    const bool rev = grads != nullptr;
    double* partials = at(p, p->partials_off);
    double* scratch = at(p, p->scan_off);
    const int64_t n_sum = ops[(size_t)p->sum_view].n;

    auto group_dev = [&](int32_t gi) {
        const Group& g = p->groups[(size_t)gi];
        GroupDev d;
        d.n = g.members.empty() ? ops[(size_t)g.leaves[0]].n : ops[(size_t)g.members[0]].n;
        d.n_leaves = (int32_t)g.leaves.size();
        d.n_ops = (int32_t)g.members.size();
        auto slot = [&](int32_t u) -> int32_t {
            for (size_t l = 0; l < g.leaves.size(); ++l)
                if (g.leaves[l] == u) return (int32_t)l;
            for (size_t m = 0; m < g.members.size(); ++m)
                if (g.members[m] == u) return (int32_t)(g.leaves.size() + m);
            return -1;
        };
        for (size_t l = 0; l < g.leaves.size(); ++l) {
            const int32_t u = g.leaves[l];
            if (u == g.gather) continue;
            d.leaf[l] = val[(size_t)u];
            d.leaf_shadow[l] = ops[(size_t)u].active ? shd[(size_t)u] : nullptr;
            d.leaf_acc[l] = p->leaf_acc[(size_t)gi][l] == D_ADD;
        }
        for (size_t m = 0; m < g.members.size(); ++m) {
            const Op& op = ops[(size_t)g.members[m]];
            GOp& o = d.ops[m];
            o.kind = op.kind;
            o.a = slot(op.a);
            o.b = op.b >= 0 ? slot(op.b) : 0;
            o.fn = op.fn;
            o.alpha = op.alpha;
            o.beta = op.kind == P_ADD ? op.beta : 0.0;  // the kernel reads scale as alpha a + 0 b
            if (op.exported) {
                d.export_slot[d.n_exports] = (int32_t)(g.leaves.size() + m);
                d.export_val[d.n_exports] = at(p, op.val_off);
                d.export_shadow[d.n_exports] = op.active ? shd[(size_t)g.members[m]] : nullptr;
                ++d.n_exports;
            }
        }
        if (g.has_sum) {
            d.sum_slot = slot(p->sum_view);
            d.partials = partials;
            d.seed = fbar;
            if (p->sum_ticket) {
                d.ticket = reinterpret_cast<int32_t*>(p->ws + p->flag_off) + 1;  // zeroed at bind
                d.f_out = f_out ? f_out : at(p, p->fscratch_off);
            }
        }
        if (g.gather >= 0) {
            const Op& go = ops[(size_t)g.gather];
            d.gather_slot = slot(g.gather);
            d.gk = go.k;
            d.gconn = go.conn;
            d.gB = go.B;
            d.gsrc = val[(size_t)go.a];
            d.gsrc_shadow = ops[(size_t)go.a].active ? shd[(size_t)go.a] : nullptr;
            d.hash_shift = g.hash_shift;
            d.agg_slots = g.agg_slots;
            if (g.export_gather) {
                d.export_slot[d.n_exports] = d.gather_slot;
                d.export_val[d.n_exports] = at(p, go.val_off);
                d.export_shadow[d.n_exports] = go.active ? shd[(size_t)g.gather] : nullptr;
                ++d.n_exports;
            }
        }
        return d;
    };
    auto op_dev = [&](int32_t v) {
        const Op& op = ops[(size_t)v];
        ProgOpDev d;
        d.kind = op.kind;
        d.n = op.n;
        d.a = val[(size_t)op.a];
        d.y = at(p, op.val_off);
        d.taps = op.taps;
        d.yb = shd[(size_t)v];
        d.ab = ops[(size_t)op.a].active ? shd[(size_t)op.a] : nullptr;
        d.accumulate = p->op_acc[(size_t)v] != D_STORE;
        d.scratch = scratch;
        d.offs = op.offs;
        d.n_seg = op.n_seg;
        return d;
    };

    // Shadows that take atomic additions (and gradients nothing reaches) start at zero.
    if (rev)
        for (int32_t v : p->zero_views)
            PG_HIP(launch_zero(shd[(size_t)v], sizeof(double) * (size_t)ops[(size_t)v].n, s));
    // Forward pass; with fusion the sum group runs its reverse in the same pass.
    const bool fused_last = rev && p->fusion;
    int64_t n_partials = 0;
    for (const Item& it : p->sched) {
        if (it.group) {
            const int mode = (it.id == p->sum_group && fused_last) ? G_FWDREV : G_FWD;
            const GroupDev d = group_dev(it.id);
            if (it.id == p->sum_group) n_partials = group_blocks(n_sum, group_block_size(d, mode));
            PG_HIP(launch_group(d, mode, s));
        } else {
            PG_HIP(launch_prog_fwd(op_dev(it.id), s));
        }
    }
    if (!p->sum_ticket)
        PG_HIP(launch_final_sum(partials, n_partials, f_out ? f_out : at(p, p->fscratch_off), s));
    if (!rev) return PG_OK;
    // Reverse pass: the schedule backwards, reads turned into deliveries.
    for (size_t r = p->sched.size(); r-- > 0;) {
        const Item& it = p->sched[r];
        if (it.group) {
            if (it.id == p->sum_group && fused_last) continue;
            const GroupDev d = group_dev(it.id);
            bool any = d.gsrc_shadow != nullptr;
            for (int l = 0; l < d.n_leaves; ++l) any = any || d.leaf_shadow[l] != nullptr;
            if (any) PG_HIP(launch_group(d, G_REV, s));
        } else {
            const Op& op = ops[(size_t)it.id];
            if (!op.active) continue;
            PG_HIP(launch_prog_rev(op_dev(it.id), s));
        }
    }
    return PG_OK;
}

pg_status pg_prog_info(pg_prog p, pg_prog_stats* stats) {
    clear_error();
    if (!p || !stats) return perr(PG_EINVAL, "NULL argument");
    if (!p->planned) return perr(PG_ESTATE, "call pg_prog_plan first");
    *stats = p->stats;
    return PG_OK;
}

pg_status pg_prog_destroy(pg_prog p) {
    delete p;
    return PG_OK;
}

}  // extern "C"
