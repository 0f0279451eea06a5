// The one entry point that allocates nothing: the FP64 mesh gradient with its
// per-workgroup partial sums of f kept in a fixed device array instead of a
// bound workspace.  Host code plus the array itself.
//
// The array `scratch` is a file-scope __device__ symbol.  Its name in host
// code is only a host-side stand-in, so it is never handed to a kernel or a
// copy: the device address of each GPU's copy is looked up once per device
// with hipGetSymbolAddress (with that device current) and kept in
// g_scratch_ptr, and only that address is used.  Every call on a device
// shares that device's copy; calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"
#include "pgrad.h"

namespace pg {
pg_status set_error(pg_status s, const char* msg);
void clear_error();
}  // namespace pg

namespace {

using namespace pg;

constexpr int kNoallocBlock = 512;
constexpr int64_t kNoallocPartials = PG_NOALLOC_MAX_WORKGROUPS;
constexpr int kMaxDevices = 64;

// One FP64 partial of f per workgroup of the element pass (512 KiB per GPU).
static __device__ __align__(256) double scratch[kNoallocPartials];

double* g_scratch_ptr[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices] = {};

// The device address of the current device's copy of `scratch`, looked up on
// the first call made on that device.
pg_status scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char msg[256];
        snprintf(msg, sizeof msg, "hipGetDevice: %s", hipGetErrorString(e));
        return set_error(PG_EHIP, msg);
    }
    if (dev < 0 || dev >= kMaxDevices) return set_error(PG_EUNSUPPORTED, "device index out of range");
    std::call_once(g_scratch_once[dev], [dev] {
        void* ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (g_scratch_err[dev] == hipSuccess) g_scratch_ptr[dev] = static_cast<double*>(ptr);
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev]) {
        char msg[256];
        snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch): %s",
                 hipGetErrorString(g_scratch_err[dev]));
        return set_error(PG_EHIP, msg);
    }
    *out = g_scratch_ptr[dev];
    return PG_OK;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
    if (!a || !b || an == 0 || bn == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bn && b0 < a0 + an;
}

pg_status hip_fail(const char* what, hipError_t e) {
    char msg[256];
    snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    return set_error(PG_EHIP, msg);
}

}  // namespace

extern "C" pg_status pg_mesh_gradient_noalloc(int64_t n_nodes, int64_t n_elems, int32_t k,
                                              const int32_t* conn, const double* B,
                                              const double* w, const double* x, double* grad,
                                              double* f_out, pg_stream stream) {
    clear_error();
    if (n_nodes < 0 || n_elems < 0) return set_error(PG_EINVAL, "n_nodes and n_elems must be >= 0");
    if (k < 1 || k > PG_MAX_K) return set_error(PG_EINVAL, "k must be in [1, PG_MAX_K]");
    if (n_nodes >= ((int64_t)1 << 31)) return set_error(PG_EINVAL, "n_nodes must be < 2^31");
    if (n_elems * (int64_t)k >= ((int64_t)1 << 31))
        return set_error(PG_EINVAL, "n_elems * k must be < 2^31");
    const int64_t blocks = mesh_blocks(n_elems, kNoallocBlock, 1);
    if (blocks > kNoallocPartials)
        return set_error(PG_EINVAL,
                         "n_elems exceeds what the fixed scratch array holds "
                         "(at most PG_NOALLOC_MAX_WORKGROUPS * 512 elements)");
    if (n_elems > 0 && (!conn || !B || !w)) return set_error(PG_EINVAL, "conn, B and w must not be NULL");
    if (n_nodes > 0 && (!x || !grad)) return set_error(PG_EINVAL, "x and grad must not be NULL");
    if (!f_out) return set_error(PG_EINVAL, "f_out is NULL");
    const size_t xb = sizeof(double) * (size_t)n_nodes;
    if (overlaps(grad, xb, x, xb)) return set_error(PG_EALIAS, "grad overlaps x");
    if (overlaps(f_out, sizeof(double), grad, xb)) return set_error(PG_EALIAS, "f_out overlaps grad");
    if (overlaps(grad, xb, conn, sizeof(int32_t) * (size_t)(n_elems * k)) ||
        overlaps(grad, xb, B, sizeof(double) * (size_t)(n_elems * k)) ||
        overlaps(grad, xb, w, sizeof(double) * (size_t)n_elems))
        return set_error(PG_EALIAS, "grad overlaps an operand");
    double* partials = nullptr;
    pg_status st = scratch_address(&partials);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);

    MeshView m;
    m.n_nodes = n_nodes;
    m.n_elems = n_elems;
    m.k = k;
    m.dtype = F64;
    m.conn = conn;
    m.B = B;
    m.w = w;
    MeshPass q;
    q.x = x;
    q.gacc = grad;
    q.partials = partials;
    q.block = kNoallocBlock;
    q.ept = 1;
    q.combine = 1;
    hipError_t e = launch_zero(grad, xb, s);
    if (e != hipSuccess) return hip_fail("fill of grad", e);
    e = launch_mesh_elem(m, M_GRAD_ATOMIC, q, s);
    if (e != hipSuccess) return hip_fail("element pass", e);
    e = launch_final_sum(partials, blocks, f_out, s);
    if (e != hipSuccess) return hip_fail("final sum", e);
    return PG_OK;
}
