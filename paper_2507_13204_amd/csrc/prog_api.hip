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
    int32_t k = 0;
    const int32_t* conn = nullptr;
    const double* B = nullptr;
    const double* data = nullptr;  // P_CONST
    int32_t input_index = -1;      // P_INPUT
    // plan
    bool active = false;
    size_t val_off = NONE;   // forward value in the workspace (intermediates)
    size_t shd_off = NONE;   // shadow in the workspace (active intermediates)
};

}  // namespace

struct pg_prog_s {
    std::vector<Op> ops;  // one per view, in creation order (view id = index)
    int32_t sum_view = -1;
    int32_t n_inputs = 0;
    bool planned = false;
    size_t ws_bytes = 0, partials_off = NONE, fscratch_off = NONE, flag_off = NONE, scan_off = NONE;
    int64_t tape_bytes = 0;
    std::vector<size_t> input_shadow_off;  // internal shadows for inputs without a grad buffer
    char* ws = nullptr;
    // info
    int32_t fwd_kernels = 0, rev_kernels = 0, atomic_ops = 0, rescheduled_ops = 0;
};

namespace {

pg_status add_view(pg_prog p, const Op& op, int32_t* view) {
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (p->sum_view >= 0) return perr(PG_ESTATE, "the program already ended with pg_prog_sum");
    if (!view) return perr(PG_EINVAL, "view is NULL");
    p->ops.push_back(op);
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

pg_status pg_prog_plan(pg_prog p, size_t* workspace_bytes) {
    clear_error();
    if (!p || !workspace_bytes) return perr(PG_EINVAL, "NULL argument");
    if (p->sum_view < 0) return perr(PG_ESTATE, "the program has no pg_prog_sum");
    // Activity: a view is active if it is an input or reads an active view.
    for (Op& op : p->ops) {
        op.active = op.kind == P_INPUT ||
                    (op.a >= 0 && p->ops[op.a].active) || (op.b >= 0 && p->ops[op.b].active);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    p->tape_bytes = 0;
    for (Op& op : p->ops) {
        op.val_off = op.shd_off = NONE;
        if (op.kind == P_INPUT || op.kind == P_CONST) continue;
        op.val_off = take(sizeof(double) * (size_t)op.n);  // recorded between kernels
        p->tape_bytes += (int64_t)(sizeof(double) * (size_t)op.n);
        if (op.active) op.shd_off = take(sizeof(double) * (size_t)op.n);
    }
    p->input_shadow_off.assign((size_t)p->n_inputs, NONE);
    for (const Op& op : p->ops)
        if (op.kind == P_INPUT)
            p->input_shadow_off[(size_t)op.input_index] = take(sizeof(double) * (size_t)op.n);
    const int64_t ns = p->ops[(size_t)p->sum_view].n;
    p->partials_off = take(sizeof(double) * (size_t)std::max<int64_t>(prog_sum_blocks(ns), 1));
    p->fscratch_off = take(sizeof(double));
    p->flag_off = take(sizeof(int32_t) * 4);
    int64_t scan_chunks = 0;  // one totals buffer, reused by every scan in turn
    for (const Op& op : p->ops)
        if (op.kind == P_SCAN) scan_chunks = std::max(scan_chunks, prog_scan_chunks(op.n));
    p->scan_off = scan_chunks ? take(sizeof(double) * (size_t)scan_chunks) : NONE;
    p->ws_bytes = off;
    // What the transformation generates.
    p->fwd_kernels = 0;
    p->rev_kernels = 0;
    p->atomic_ops = 0;
    p->rescheduled_ops = 0;
    for (const Op& op : p->ops) {
        if (op.kind == P_INPUT || op.kind == P_CONST) continue;
        const int32_t nk = op.kind == P_SCAN ? 3 : 1;  // a scan is three launches each way
        p->fwd_kernels += nk;
        if (!op.active) continue;
        p->rev_kernels += nk;
        if (op.kind == P_GATHER && p->ops[op.a].active) ++p->atomic_ops;
        if (op.kind == P_STENCIL && op.taps.n > 1 && p->ops[op.a].active) ++p->rescheduled_ops;
    }
    p->fwd_kernels += 2;  // the sum's partials and its final fixed-order reduction
    if (p->ops[(size_t)p->sum_view].active) ++p->rev_kernels;  // broadcast of the seed
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
    p->ws = static_cast<char*>(ws);
    return PG_OK;
}

pg_status pg_prog_run(pg_prog p, const double* const* inputs, double* f_out, double* const* grads,
                      pg_stream stream) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (!p->planned || !p->ws) return perr(PG_ESTATE, "plan the program and bind a workspace first");
    if (p->n_inputs > 0 && !inputs) return perr(PG_EINVAL, "inputs is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Device pointers of every view's forward value and shadow.
    const size_t nv = p->ops.size();
    std::vector<const double*> val(nv, nullptr);
    std::vector<double*> shd(nv, nullptr);
    for (size_t v = 0; v < nv; ++v) {
        const Op& op = p->ops[v];
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
    // Forward pass: one kernel per construct, outputs recorded on the tape.
    for (size_t v = 0; v < nv; ++v) {
        const Op& op = p->ops[v];
        if (op.kind == P_INPUT || op.kind == P_CONST) continue;
        ProgOpDev d;
        d.kind = op.kind;
        d.n = op.n;
        d.a = val[(size_t)op.a];
        d.b = op.b >= 0 ? val[(size_t)op.b] : nullptr;
        d.y = at(p, op.val_off);
        d.alpha = op.alpha;
        d.beta = op.beta;
        d.fn = op.fn;
        d.taps = op.taps;
        d.k = op.k;
        d.conn = op.conn;
        d.B = op.B;
        d.scratch = at(p, p->scan_off);
        PG_HIP(launch_prog_fwd(d, s));
    }
    const Op& so = p->ops[(size_t)p->sum_view];
    double* partials = at(p, p->partials_off);
    double* fdst = f_out ? f_out : at(p, p->fscratch_off);
    {
        ProgOpDev d;
        d.kind = P_SUM;
        d.n = so.n;
        d.a = val[(size_t)p->sum_view];
        d.y = partials;
        PG_HIP(launch_prog_fwd(d, s));
        PG_HIP(launch_final_sum(partials, prog_sum_blocks(so.n), fdst, s));
    }
    if (!grads) return PG_OK;
    // Shadows start at zero; requested input gradients are the input shadows.
    for (size_t v = 0; v < nv; ++v)
        if (shd[v] && p->ops[v].active) PG_HIP(launch_zero(shd[v], sizeof(double) * (size_t)p->ops[v].n, s));
    // Reverse of the sum: broadcast the seed 1 into the summed view's shadow.
    if (so.active) {
        ProgOpDev d;
        d.kind = P_SUM;
        d.n = so.n;
        d.alpha = 1.0;
        d.ab = shd[(size_t)p->sum_view];
        PG_HIP(launch_prog_rev(d, s));
    }
    // Reverse pass: constructs in reverse order, reads turned into accumulations.
    for (size_t r = nv; r-- > 0;) {
        const Op& op = p->ops[r];
        if (op.kind == P_INPUT || op.kind == P_CONST || !op.active) continue;
        ProgOpDev d;
        d.kind = op.kind;
        d.n = op.n;
        d.a = val[(size_t)op.a];
        d.b = op.b >= 0 ? val[(size_t)op.b] : nullptr;
        d.alpha = op.alpha;
        d.beta = op.beta;
        d.fn = op.fn;
        d.taps = op.taps;
        d.k = op.k;
        d.conn = op.conn;
        d.B = op.B;
        d.yb = shd[r];
        d.ab = p->ops[(size_t)op.a].active ? shd[(size_t)op.a] : nullptr;
        d.bb = (op.b >= 0 && p->ops[(size_t)op.b].active) ? shd[(size_t)op.b] : nullptr;
        d.scratch = at(p, p->scan_off);
        if (!d.ab && !d.bb) continue;
        PG_HIP(launch_prog_rev(d, s));
    }
    return PG_OK;
}

pg_status pg_prog_info(pg_prog p, int32_t* fwd_kernels, int32_t* rev_kernels, int32_t* atomic_ops,
                       int32_t* rescheduled_ops, int64_t* tape_bytes) {
    clear_error();
    if (!p) return perr(PG_EINVAL, "program is NULL");
    if (!p->planned) return perr(PG_ESTATE, "call pg_prog_plan first");
    if (fwd_kernels) *fwd_kernels = p->fwd_kernels;
    if (rev_kernels) *rev_kernels = p->rev_kernels;
    if (atomic_ops) *atomic_ops = p->atomic_ops;
    if (rescheduled_ops) *rescheduled_ops = p->rescheduled_ops;
    if (tape_bytes) *tape_bytes = p->tape_bytes;
    return PG_OK;
}

pg_status pg_prog_destroy(pg_prog p) {
    delete p;
    return PG_OK;
}

}  // extern "C"
