/*
 * pgrad.h -- reverse-mode gradients of data-parallel scalar objectives on
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates objectives of the shape studied in Liegeois, Kelley,
 * Phipps, Rajamanickam and Vassilev, "Performance Portable Gradient
 * Computations Using Source Transformation": a data-parallel gather
 * (parallel_for), an element-wise nonlinearity, and a parallel sum
 * (parallel_reduce / the parallel_sum builtin of section 3.2), together with
 * their reverse-mode gradients: seed the result adjoint, broadcast it to every
 * summand (reverse of a sum), multiply by the local derivative at the stored
 * or recomputed forward value (section 4: the tape lives between kernels),
 * and transpose every read of x into an accumulation into the shadow of x
 * (section 3.1, view-access rule), which becomes an atomic update when the
 * read index is itself a view entry (section 3.3, race detection).
 *
 *   psi(s)  = s^2/2 + log(1 + s^2)/2,   psi'(s) = s + s/(1 + s^2)
 *
 * CONVENTIONS
 *   - Every pointer is DEVICE memory unless its comment says "host".
 *   - Every call that takes a stream enqueues its work on that stream
 *     (a hipStream_t passed as pg_stream; NULL is the legacy default stream)
 *     and returns without waiting, except pg_bind_workspace, which waits.
 *   - The caller owns every device buffer (inputs, outputs, workspace).  A
 *     plan keeps NON-OWNING pointers to its constant operands (conn, B, w,
 *     A, W); they must stay alive and unchanged while the plan is used.  The
 *     library allocates no device memory; a plan owns only host memory.
 *   - All arrays are dense row-major.  Index arrays are int32.
 *   - Floating-point arrays are FP64 (PG_F64) or FP32 (PG_F32) as the plan's
 *     dtype says; objective values f and the seeds fbar are always FP64, and
 *     every reduction and accumulation is carried out in FP64.
 *   - Gradients are taken with respect to x (or X) only; conn, B, w, A and W
 *     are inactive (section 3.1: index metadata is never differentiated).
 *   - Errors are reported as pg_status codes; argument errors are detected
 *     before anything is enqueued and leave every output untouched.
 *     pg_last_error() returns a thread-local message for the last non-OK
 *     status.  No C++ exception crosses this interface.
 *   - A plan must not be used concurrently from two streams: its workspace
 *     holds per-call scratch (partial sums, counters, the stored tape).
 */
#ifndef PGRAD_H
#define PGRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PGRAD_VERSION 2
#define PG_MAX_K 32           /* maximum nodes per element */
#define PG_WORKSPACE_ALIGN 256 /* required alignment of the workspace */

typedef struct pg_plan_s* pg_plan;
typedef void* pg_stream; /* a hipStream_t */

typedef enum {
    PG_OK = 0,
    PG_EINVAL = 1,       /* bad size, null pointer, bad option */
    PG_ERANGE = 2,       /* connectivity entry outside [0, n_nodes) */
    PG_EDTYPE = 3,       /* unknown dtype */
    PG_EALIAS = 4,       /* an output overlaps an input or the workspace */
    PG_EWORKSPACE = 5,   /* workspace missing, too small or misaligned */
    PG_EHIP = 6,         /* a HIP runtime call or launch failed */
    PG_EUNSUPPORTED = 7, /* valid request this plan kind does not offer */
    PG_ESTATE = 8        /* plan used before pg_bind_workspace, or no stored
                            forward values for this x (see pg_adjoint) */
} pg_status;

typedef enum { PG_F64 = 0, PG_F32 = 1 } pg_dtype;

/* How the reverse pass accumulates x-bar (section 3.3 race rule; the
 * conclusion's "reschedule the reverse threads" remedy). */
typedef enum {
    PG_ADJ_AUTO = 0,   /* library choice (currently PG_ADJ_ATOMIC) */
    PG_ADJ_ATOMIC = 1, /* element-parallel scatter with FP64 atomic adds */
    PG_ADJ_GATHER = 2, /* deterministic: node-parallel gather over the
                          transposed (node -> element) connectivity, built
                          at bind with B's coefficients copied into its
                          order (per incidence 4 + element-size bytes of
                          workspace, besides the offsets) */
    PG_ADJ_COLOUR = 3, /* deterministic: element colour classes, one
                          non-atomic pass per colour; the bind copies conn,
                          B and w into colour-major order in the workspace
                          (per element k * 4 + (k + 1) * element-size bytes
                          more), which the passes read unless a stored tape
                          is in use */
    PG_ADJ_TILED = 4   /* deterministic: each workgroup sums its tile's
                          contributions per node in LDS in a fixed order
                          (local incidence lists built at bind), then a
                          node-parallel pass adds the tiles' partials in
                          tile order; no atomics, no fill of grad.  When
                          the bind finds that no tile puts one node at one
                          corner twice and that one slot hash separates
                          every tile's nodes (structured meshes do), the
                          per-node sums are built instead in one round per
                          corner, in ascending corner order, reading no
                          incidence lists; pg_plan_info reports that form's
                          slot count in lds_slots (0: the general form).
                          Mesh plans only; the workspace is sized for the
                          worst case (12 + 2 + 4 bytes per incidence more
                          than the atomic plan, or 32 KiB per 512-element
                          tile if larger). */
} pg_adjoint_kind;

/* What the forward pass keeps for the reverse pass (section 4: intermediates
 * are recorded in views between kernels; the conclusion: a tape whose size is
 * deduced once, outside the kernels). */
typedef enum {
    PG_RECOMPUTE = 0, /* the reverse pass recomputes the gathered values */
    PG_STORE = 1,     /* pg_objective stores them in the workspace */
    PG_CKPT_AUTO = 2  /* chosen by memory when the plan is made: PG_STORE if
                         one call's tape (pg_tape_bytes) fits
                         options.tape_budget bytes, else PG_RECOMPUTE.  A
                         budget of 0 means a quarter of the device memory
                         that hipMemGetInfo reports free at that moment.
                         pg_plan_info reports the choice. */
} pg_ckpt;

typedef struct {
    int32_t adjoint;    /* pg_adjoint_kind */
    int32_t ckpt;       /* pg_ckpt */
    int32_t block;      /* threads per workgroup, 0 = default (multiple of 64, <= 1024) */
    int32_t tile;       /* work items per thread, 0 = default (1, 2 or 4) */
    int32_t accumulate; /* 0: gradients overwrite grad; 1: add into grad
                           (the shadow-argument convention of the generated
                           gradient in section 4) */
    int32_t scatter;    /* atomic adjoint only: 0 = default (combine each
                           workgroup's contributions per node in an LDS hash
                           table, then one global atomic per node; a single
                           mesh's plan picks a 2048- or 4096-slot table by
                           simulating it on sampled workgroups, and keeps
                           2048 only if a check of every workgroup at bind
                           finds no two nodes on one home slot), 1 = one
                           global atomic per contribution, 2 = combine in a
                           4096-slot table, 3 = combine in a 2048-slot table
                           (2 and 3: single meshes; batches treat them as 0) */
    int32_t onepass;    /* single meshes, atomic adjoint, k = 2, 4 or 8: 0 =
                           default (a mesh of at most 64 workgroups and 16,384
                           nodes runs each objective, gradient, adjoint, HVP
                           or JVP call as one launch: the contributions gather in a
                           workspace buffer and the last workgroup to finish
                           writes grad from it, clears it and sums f), 1 = the
                           multi-launch path at every size */
    int32_t reserved;   /* must be 0 */
    int64_t tape_budget; /* PG_CKPT_AUTO: bytes the stored tape may take
                            (0: a quarter of the free device memory) */
} pg_options;

/* One instance of a mesh batch: its nodes are x[node_off .. node_off+n_nodes)
 * and its elements are rows elem_off .. elem_off+n_elems of conn, B and w.
 * conn holds instance-local node numbers in [0, n_nodes). */
typedef struct {
    int64_t n_nodes;
    int64_t n_elems;
    int64_t node_off;
    int64_t elem_off;
} pg_instance;

/* pg_options with every field at its default. */
pg_options pg_default_options(void);

/* ------------------------------------------------------------------ plans */

/* Element-connectivity objective (the stencil example of section 4 written
 * for a general connectivity table):
 *   f(x) = sum_e w[e] * psi( u_e ),  u_e = sum_{j<k} B[e*k+j] * x[conn[e*k+j]]
 *   grad = G^T ( fbar * w (.) psi'(G x) ),  G[e, conn[e,j]] += B[e,j]
 * conn: n_elems*k int32, B: n_elems*k, w: n_elems (dtype), all device.
 * 1 <= k <= PG_MAX_K; n_nodes < 2^31; n_elems*k < 2^31.
 * *workspace_bytes (host, out) receives the workspace size this plan needs.
 * *plan (host, out) is written only on PG_OK. */
pg_status pg_mesh_plan(pg_plan* plan, int64_t n_nodes, int64_t n_elems, int32_t k,
                       const int32_t* conn, const void* B, const void* w, pg_dtype dtype,
                       const pg_options* opts, size_t* workspace_bytes);

/* Dense row reduction (hierarchical team/vector parallelism, named as future
 * work in the conclusion):  f(x) = sum_i w[i] psi((A x)_i),
 * grad = A^T (fbar * w (.) psi'(A x)).  A: rows x cols, w: rows (dtype). */
pg_status pg_dense_plan(pg_plan* plan, int64_t rows, int64_t cols, const void* A, const void* w,
                        pg_dtype dtype, const pg_options* opts, size_t* workspace_bytes);

/* Batched dense objective over the columns of X (m x n):
 *   f(X) = sum_{i,j} W[i,j] psi((A X)_{ij}),  grad = A^T (fbar * W (.) psi'(A X)).
 * A: m x m, W: m x n (dtype).  The contractions run on the matrix cores. */
pg_status pg_bdense_plan(pg_plan* plan, int64_t m, int64_t n, const void* A, const void* W,
                         pg_dtype dtype, const pg_options* opts, size_t* workspace_bytes);

/* Many independent meshes in one launch.  inst (host) has n_inst entries;
 * conn, B, w are the concatenations described by pg_instance.  Objectives
 * are per instance: f_out and fbar have n_inst entries. */
pg_status pg_mesh_batch_plan(pg_plan* plan, int32_t n_inst, const pg_instance* inst, int32_t k,
                             const int32_t* conn, const void* B, const void* w, pg_dtype dtype,
                             const pg_options* opts, size_t* workspace_bytes);

/* The paper's section 4 example, with both of its inputs active:
 *   f(x, b) = || A (3 x) - b ||^2,  A the n x n 1D Laplacian (2 on the
 *   diagonal, -1 on the first off-diagonals, rows truncated at both ends),
 *   df/dx = 6 A (3 A x - b),  df/db = -2 (3 A x - b).
 * options.adjoint: PG_ADJ_GATHER or PG_ADJ_AUTO (each thread recomputes its
 * neighbours' residuals and writes its own gradient entry: the reverse
 * threads rescheduled), or PG_ADJ_ATOMIC (the paper's schedule: every
 * residual scatters into three entries of df/dx with atomic adds).
 * x, b, gx, gb: n entries of the plan dtype.  For n <= 16,384 the last
 * workgroup to finish reduces f (a ticket in the workspace, zero between
 * calls), so the objective and the gather-form gradient are one launch each. */
pg_status pg_laplace1d_plan(pg_plan* plan, int64_t n, pg_dtype dtype, const pg_options* opts,
                            size_t* workspace_bytes);
pg_status pg_laplace1d_objective(pg_plan plan, const void* x, const void* b, double* f_out,
                                 pg_stream stream);
/* gx (df/dx) and gb (df/db) may each be NULL; f_out may be NULL. */
pg_status pg_laplace1d_gradient(pg_plan plan, const void* x, const void* b, void* gx, void* gb,
                                double* f_out, pg_stream stream);

/* Workspace size of a plan (host out). */
pg_status pg_workspace_size(pg_plan plan, size_t* workspace_bytes);

/* Bind a caller-owned device workspace of at least the queried size,
 * aligned to PG_WORKSPACE_ALIGN, to the plan; validate the connectivity
 * (PG_ERANGE if an entry is outside [0, n_nodes)) and build the plan's
 * device structures (transposed connectivity, colour classes, work lists).
 * Enqueued on stream and WAITS for it.  Rebinding is allowed.  Some parts of
 * the workspace are set to zero here and every call leaves them zero again
 * (the FP64 accumulation buffer of FP32 plans, the buffers and counters of
 * one-launch calls): the caller must not write to a bound workspace, and
 * after a call that failed with PG_EHIP the plan should be bound again. */
pg_status pg_bind_workspace(pg_plan plan, void* workspace, size_t bytes, pg_stream stream);

/* ------------------------------------------------------------- evaluation */

/* f_out (device, FP64, 1 entry or n_inst for a batch) = f(x).
 * With ckpt == PG_STORE the forward values are kept for pg_adjoint. */
pg_status pg_objective(pg_plan plan, const void* x, double* f_out, pg_stream stream);

/* One call, both passes (section 4's generated gradient: forward replay,
 * seed 1, reverse pass): f_out = f(x) (may be NULL), grad = df/dx.
 * grad has the shape of x and must not overlap x, the operands or the
 * workspace. */
pg_status pg_gradient(pg_plan plan, const void* x, void* grad, double* f_out, pg_stream stream);

/* Reverse pass only, seeded with fbar (device FP64, 1 entry or n_inst):
 * grad = fbar * df/dx.  With ckpt == PG_STORE it reads the values the last
 * pg_objective stored in the workspace, and returns PG_ESTATE (nothing
 * enqueued) unless that call was made with the same x pointer and no later
 * call has overwritten them (a batched-dense pg_gradient or recomputing
 * adjoint reuses that buffer).  The caller must not have changed the
 * contents of x in between: the library compares pointers, not values.
 * With PG_RECOMPUTE it recomputes them from x. */
pg_status pg_adjoint(pg_plan plan, const void* x, const double* fbar, void* grad,
                     pg_stream stream);

/* ----------------------------------------------- per-call tape (section 4)
 *
 * The paper's generated gradient records the forward values its reverse pass
 * reads in views made for that call.  These calls do the same with a tape
 * the caller owns, so any number of forward passes can be outstanding on one
 * plan (the backward of an autograd function keeps its own tape), whatever
 * the plan's ckpt option.  What a tape holds:
 *   mesh and mesh batch: u_e = sum_j B[e,j] x[conn[e,j]] for every element,
 *     FP64 (n_elems entries; a batch's concatenated elements);
 *   batched dense: V = W (.) psi'(A X), m x n in the plan dtype.
 * Dense plans and the section 4 example have no tape (PG_EUNSUPPORTED).
 * tape: device memory of pg_tape_bytes bytes, 16-byte aligned, not
 * overlapping any operand, output or the workspace. */
pg_status pg_tape_bytes(pg_plan plan, size_t* bytes);
/* f_out = f(x) as pg_objective, and the forward values written to tape. */
pg_status pg_objective_tape(pg_plan plan, const void* x, double* f_out, void* tape,
                            pg_stream stream);
/* grad = fbar * df/dx from the forward values in tape (written by
 * pg_objective_tape of this plan); x is not read. */
pg_status pg_adjoint_tape(pg_plan plan, const double* fbar, const void* tape, void* grad,
                          pg_stream stream);

/* y[i] = alpha[0] * x[i] for i < n, evaluated in FP64 and rounded once to
 * dtype; y may equal x.  alpha: device FP64.  The seed of a scalar objective
 * (section 3.2: the adjoint of the sum broadcasts the seed) applied to a
 * gradient formed with seed 1, as when f and its gradient are computed in
 * one forward call and the backward of an autograd function receives
 * grad_output afterwards. */
pg_status pg_scale(pg_dtype dtype, int64_t n, const double* alpha, const void* x, void* y,
                   pg_stream stream);

/* ------------------------------------------------- allocation-free call
 *
 * For callers that cannot allocate device memory or bind a workspace: code
 * recorded under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  The same FP64 gradient as pg_gradient on a mesh plan
 * with the default options (atomic adjoint combined per workgroup in a
 * 4096-slot LDS table, 512-thread workgroups, grad overwritten), but with no
 * plan: grad is cleared by a fill kernel, the element pass scatters into it,
 * and the per-workgroup partial sums of f go to a fixed device array of
 * PG_NOALLOC_MAX_WORKGROUPS doubles (512 KiB, one copy per GPU, held until
 * the process ends) that one more workgroup reduces into f_out in a fixed
 * order.  Nothing is allocated and nothing waits on the host.
 *   n_nodes, n_elems >= 0; 1 <= k <= PG_MAX_K; n_nodes < 2^31;
 *   n_elems * k < 2^31; n_elems <= 512 * PG_NOALLOC_MAX_WORKGROUPS
 *   (PG_EINVAL otherwise, nothing enqueued).
 *   conn (int32, n_elems * k), B (n_elems * k), w (n_elems), x (n_nodes):
 *   device FP64 inputs; grad (n_nodes, device, overwritten) must not overlap
 *   x or the operands (PG_EALIAS); f_out: device, 1 FP64.
 * conn is NOT validated (no plan, so no bind-time check): every entry must
 * lie in [0, n_nodes), as pg_bind_workspace of a mesh plan on the same
 * connectivity verifies.  Calls on one GPU share its array: calls that
 * overlap in time on that GPU (two streams) race; calls ordered on one
 * stream do not.  PG_EHIP if a launch fails. */
#define PG_NOALLOC_MAX_WORKGROUPS 65536
pg_status pg_mesh_gradient_noalloc(int64_t n_nodes, int64_t n_elems, int32_t k,
                                   const int32_t* conn, const double* B, const double* w,
                                   const double* x, double* grad, double* f_out,
                                   pg_stream stream);

/* ------------------------------------------------------------ plan queries */

typedef struct {
    int32_t kind;          /* 1 mesh, 2 dense, 3 batched dense, 4 mesh batch, 5 section 4 example */
    int32_t dtype;         /* pg_dtype */
    int32_t adjoint;       /* resolved pg_adjoint_kind (never PG_ADJ_AUTO) */
    int32_t ckpt;          /* resolved pg_ckpt (never PG_CKPT_AUTO) */
    int32_t block;         /* threads per workgroup of the element pass */
    int32_t tile;          /* elements per thread */
    int32_t lds_slots;     /* LDS table of the combined atomic scatter, or of the
                              tiled adjoint's corner-round form (0: none; set at bind) */
    int32_t one_launch;    /* 1 if every call is one launch */
    int32_t n_colours;     /* colour classes (colour adjoint, after bind), else 0 */
    int32_t bound;         /* 1 after a successful pg_bind_workspace */
    int64_t workspace_bytes;
    int64_t tape_bytes;    /* pg_tape_bytes */
    int64_t tape_budget;   /* the budget PG_CKPT_AUTO compared against (0 if not AUTO) */
} pg_plan_info_t;
pg_status pg_plan_info(pg_plan plan, pg_plan_info_t* info);

/* Copy one integer structure of a bound mesh plan to host memory, so that it
 * can be compared with an independent construction (the conclusion's
 * rescheduled reverse threads need them exact):
 *   PG_EXPORT_CSR_OFFS    int32[n_nodes + 1]: row offsets of the transposed
 *                         connectivity (gather adjoint);
 *   PG_EXPORT_CSR_INC     int32[n_elems * k]: per node, its incidences
 *                         e * k + j with conn[e,j] == node, ascending;
 *   PG_EXPORT_COLOUR_OFFS int64[n_colours + 1]: class c is entries
 *                         [offs[c], offs[c+1]) of the element list;
 *   PG_EXPORT_COLOUR_ELEMS int32[n_elems]: elements, class by class,
 *                         ascending inside a class (colour adjoint).
 * host_dst NULL: only *bytes (host, out) is set.  Otherwise capacity must be
 * at least that size.  Waits for the plan's last bind (a device-to-host copy
 * on the null stream).  PG_EUNSUPPORTED if the plan has no such structure. */
typedef enum {
    PG_EXPORT_CSR_OFFS = 0,
    PG_EXPORT_CSR_INC = 1,
    PG_EXPORT_COLOUR_OFFS = 2,
    PG_EXPORT_COLOUR_ELEMS = 3
} pg_export_what;
pg_status pg_plan_export(pg_plan plan, int32_t what, void* host_dst, size_t capacity,
                         size_t* bytes);

/* Hessian-vector product of the mesh objective (tangent over reverse,
 * named as future work in the conclusion):
 *   hv = G^T ( w (.) psi''(G x) (.) (G v) ).  Mesh plans only. */
pg_status pg_hvp(pg_plan plan, const void* x, const void* v, void* hv, pg_stream stream);

/* Forward tangent (directional derivative) of the mesh objective, the other
 * derivative mode the conclusion names:
 *   jvp_out[0] (device FP64) = f'(x) . d = sum_e w_e psi'(u_e) (G d)_e.
 * Mesh plans only; reduced in a fixed order. */
pg_status pg_jvp(pg_plan plan, const void* x, const void* d, double* jvp_out, pg_stream stream);

/* ----------------------------------------------------- composed programs */

/* A program is a chain of data-parallel operations on 1D FP64 views ending in
 * a parallel sum, differentiated by the library with the rules of section 3,
 * one construct at a time:
 *   - every view that depends on an input gets a shadow view of the same
 *     size (section 3.1); views that depend on no input are inactive and get
 *     none;
 *   - reads become accumulations into the shadow and writes become reads of
 *     it (section 3.1, view accesses), so the reverse pass runs the ops in
 *     reverse order;
 *   - the reverse of the final sum is a broadcast of the seed (section 3.2,
 *     parallel_sum);
 *   - only what feeds the sum runs; a shadow's first delivery in the
 *     reverse pass stores and later ones add, so shadows need no clearing
 *     except where atomics deliver;
 *   - forward values the reverse pass reads are recorded on a tape between
 *     kernels (section 4) or recomputed inside a fused group (see
 *     pg_prog_fusion); the tape is sized when the program is planned and
 *     bound once (conclusion: size-deduced tape allocated outside the
 *     kernels);
 *   - an accumulation whose index is itself a view entry (gather through a
 *     connectivity table) races and uses atomic adds; one that reads through
 *     several index expressions (a stencil) is rescheduled into a gather by
 *     the written index, so it needs none (section 3.3; conclusion).
 * Build a program with the pg_prog_* builders (view ids are returned in
 * *view, in creation order), then plan, bind a workspace and run. */
typedef struct pg_prog_s* pg_prog;
typedef enum { PG_MAP_SQUARE = 0, PG_MAP_PSI = 1 } pg_map_fn;

pg_status pg_prog_create(pg_prog* prog);
/* Active input of n entries; its device pointer is given to pg_prog_run. */
pg_status pg_prog_input(pg_prog prog, int64_t n, int32_t* view);
/* Inactive operand of n entries (device pointer kept, not owned). */
pg_status pg_prog_const(pg_prog prog, int64_t n, const double* data, int32_t* view);
/* y = alpha * a */
pg_status pg_prog_scale(pg_prog prog, int32_t a, double alpha, int32_t* view);
/* y_i = sum_t coeffs[t] * a_{i + offsets[t]}, taps outside [0, n) dropped
 * (offsets, coeffs: host arrays of n_taps entries, copied; n_taps <= 16). */
pg_status pg_prog_stencil(pg_prog prog, int32_t a, int32_t n_taps, const int32_t* offsets,
                          const double* coeffs, int32_t* view);
/* y_e = sum_j B[e*k + j] * a[conn[e*k + j]] for e < n_elems (device conn and
 * B kept, not owned; conn entries must lie in [0, length of a)). */
pg_status pg_prog_gather(pg_prog prog, int32_t a, int64_t n_elems, int32_t k, const int32_t* conn,
                         const double* B, int32_t* view);
/* y = alpha * a + beta * b (equal lengths) */
pg_status pg_prog_add(pg_prog prog, int32_t a, double alpha, int32_t b, double beta,
                      int32_t* view);
/* y = a (.) b (equal lengths) */
pg_status pg_prog_mul(pg_prog prog, int32_t a, int32_t b, int32_t* view);
/* y = fn(a) elementwise: PG_MAP_SQUARE (s^2) or PG_MAP_PSI (psi above) */
pg_status pg_prog_map(pg_prog prog, int32_t a, pg_map_fn fn, int32_t* view);
/* y_i = sum_{j <= i} a_j (inclusive prefix sum).  The reverse of a scan is
 * the scan of the output shadow taken from the other end, abar_j +=
 * sum_{i >= j} ybar_i: the rule the paper's conclusion lists as missing for
 * parallel_scan.  Fixed summation order (deterministic). */
pg_status pg_prog_scan(pg_prog prog, int32_t a, int32_t* view);
/* y_s = sum of a over [offsets[s], offsets[s+1]) for s < n_seg (a partial
 * parallel_reduce); its reverse broadcasts the output shadow over each
 * segment (section 3.2: a reduction's adjoint is a broadcast).  offsets:
 * device int64, n_seg + 1 entries, kept, not owned; checked in
 * pg_prog_bind_workspace (PG_ERANGE unless 0 = offsets[0] <= ... <=
 * offsets[n_seg] = length of a).  One wave per segment, fixed order. */
pg_status pg_prog_segment_sum(pg_prog prog, int32_t a, int64_t n_seg, const int64_t* offsets,
                              int32_t* view);
/* y_i = a_s for offsets[s] <= i < offsets[s+1] (n_out = offsets[len(a)]
 * outputs); the reverse is the segment sum of the output shadow.  offsets:
 * as above with n_seg = length of a, last entry n_out. */
pg_status pg_prog_broadcast(pg_prog prog, int32_t a, const int64_t* offsets, int64_t n_out,
                            int32_t* view);
/* f = sum of view a.  Ends the program. */
pg_status pg_prog_sum(pg_prog prog, int32_t a);
/* Checks the program, runs the activity analysis, lays out the tape and the
 * shadows; *workspace_bytes (host out) is what pg_prog_bind_workspace needs. */
pg_status pg_prog_plan(pg_prog prog, size_t* workspace_bytes);
/* workspace: device memory of at least the planned bytes, 256-byte aligned,
 * owned by the caller and used by every later run (tape, shadows, partials).
 * Checks every gather's connectivity against its operand on the device, on the
 * null stream, and waits for it (PG_ERANGE if an entry is out of range). */
pg_status pg_prog_bind_workspace(pg_prog prog, void* workspace, size_t bytes);
/* inputs: host array of device pointers, one per input in creation order.
 * f_out: device FP64 (may be NULL).  grads: NULL (objective only) or a host
 * array with one device pointer per input (NULL entries skipped); each is
 * overwritten with fbar * df/d(input).  fbar: device FP64 seed of f (NULL
 * means 1; the backward of an autograd function passes grad_output).
 * Enqueued on stream; no host synchronisation, so a run can be captured in
 * a HIP graph. */
pg_status pg_prog_run(pg_prog prog, const double* const* inputs, double* f_out,
                      double* const* grads, const double* fbar, pg_stream stream);
/* What the transformation produced (filled by pg_prog_info, host out). */
typedef struct {
    int32_t fwd_kernels;      /* launches of the forward pass (shadow clearing not counted) */
    int32_t rev_kernels;      /* launches of the reverse pass */
    int32_t atomic_ops;       /* reverse deliveries made atomic by the race rule (gathers) */
    int32_t rescheduled_ops;  /* reverse stencils rescheduled into gathers (no atomics) */
    int32_t groups;           /* fused groups of pointwise constructs (the sum's included) */
    int32_t fused_gathers;    /* gathers evaluated inside their consuming group */
    int32_t dead_ops;         /* constructs that do not feed the sum (never run) */
    int32_t folded_ops;       /* scales folded into the coefficients of the one
                                 stencil that reads them (fusion 1) */
    int64_t tape_bytes;       /* forward values recorded between kernels */
    int64_t workspace_bytes;
} pg_prog_stats;

/* Fusion level, before pg_prog_plan.  1 (default): a scale read only by a
 * stencil is folded into the stencil's coefficients (the two are linear);
 * chains of pointwise constructs (scale, add, mul, map) run as one kernel
 * per group, keep their
 * intermediates in registers and recompute them in the reverse pass (no
 * tape); a gather read only by one group runs inside it, its reverse being
 * an LDS-combined atomic scatter; the group holding the sum runs its
 * forward and reverse in one pass (the seed of f is the constant 1), and
 * when the summed view has at most 16,384 entries its last workgroup, found
 * by a ticket in the workspace, reduces f (no separate reduction launch).  The
 * conclusion of the paper names kernel fusion and recomputation as ways to
 * cut the cost of the generated gradient.  0: one kernel per construct each
 * way (the sum's partials are taken by the kernel producing the summed
 * view), every value another construct reads recorded. */
pg_status pg_prog_fusion(pg_prog prog, int32_t level);
pg_status pg_prog_info(pg_prog prog, pg_prog_stats* stats);
pg_status pg_prog_destroy(pg_prog prog);

/* Measurement hook.  mode 0: off; 1: time the dominant kernel of every
 * subsequent evaluation (the element pass of a mesh or batch, the fused row
 * pass of a dense plan, the forward or backward product of a batched dense
 * plan, the pass of the section 4 example); 2: time each whole evaluation
 * call.  In mode 1 a single dominant kernel is launched with
 * hipExtLaunchKernelGGL, which stamps a pair of HIP events with the
 * kernel's own start and end; phases of several kernels (the colour
 * passes, the gather variant, the dense row/column fallback) and mode 2 are
 * bracketed by events recorded on the call's stream.  Events are owned by
 * the plan (up to 4096 pairs).  pg_timing_read waits for the last recorded
 * event, returns the sum of the elapsed times (milliseconds, host out) and
 * the number of timed launches (host out), and clears the record.
 * Enabling resets the record. */
pg_status pg_timing(pg_plan plan, int32_t mode);
pg_status pg_timing_read(pg_plan plan, double* total_ms, int64_t* count);

pg_status pg_plan_destroy(pg_plan plan);

/* Thread-local description of the last non-OK status ("" if none). */
const char* pg_last_error(void);

int pg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PGRAD_H */
