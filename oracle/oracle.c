/*
 * FP64 reference oracle for the reverse-mode gradient library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP kernels.
 *
 * It computes, plainly and slowly, in FP64:
 *
 *   mesh     f(x)  = sum_e w_e psi(u_e),  u_e = sum_j B[e,j] x[conn[e,j]]
 *            grad  = G^T (fbar * w (.) psi'(G x))
 *   dense    f(x)  = sum_i w_i psi((A x)_i),    grad = A^T (fbar * w (.) psi'(A x))
 *   batched  f(X)  = sum_ij W_ij psi((A X)_ij), column by column (dense form)
 *
 * with psi(s) = s^2/2 + log(1+s^2)/2 and psi'(s) = s + s/(1+s^2).
 *
 * Paper correspondence (Liegeois et al., "Performance Portable Gradient
 * Computations Using Source Transformation"):
 *   - the gather u = G x is the stencil parallel_for of the section 4 example
 *     generalised to an element connectivity table; an index that is itself a
 *     view access is the race case of section 3.3;
 *   - the element nonlinearity plays the role of the squaring kernel;
 *   - f is the parallel_sum reduction (section 3.2, builtin parallel_sum);
 *   - the reverse pass seeds the result adjoint with fbar (1 for a gradient),
 *     broadcasts it to every term (reverse of a sum), multiplies by the local
 *     derivative at the forward value, and transposes every read of x into an
 *     accumulation into the shadow of x (section 3.1, view-access rule; the
 *     generated gradient of section 4).
 * Reverse mode computes the exact derivative of the program up to rounding, so
 * the oracle is the analytic chain rule written out.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -o liboracle.so -lm
 * (no contraction, so every multiply and add rounds as written).
 *
 * Status codes: 0 ok, 1 invalid sizes / null pointer, 2 connectivity entry
 * outside [0, n_nodes).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ERANGE 2

/* ---------------------------------------------------------------- scalars */

/* psi(s) = s^2/2 + log(1 + s^2)/2 */
static double psi(double s) { return 0.5 * s * s + 0.5 * log1p(s * s); }

/* psi'(s) = s + s / (1 + s^2) */
static double dpsi(double s) { return s + s / (1.0 + s * s); }

/* psi''(s) = 1 + (1 - s^2) / (1 + s^2)^2 */
static double ddpsi(double s) {
    double q = 1.0 + s * s;
    return 1.0 + (1.0 - s * s) / (q * q);
}

int orc_psi(int64_t n, const double* s, double* out) {
    if (n < 0 || (n > 0 && (!s || !out))) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) out[i] = psi(s[i]);
    return ORC_OK;
}

int orc_dpsi(int64_t n, const double* s, double* out) {
    if (n < 0 || (n > 0 && (!s || !out))) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) out[i] = dpsi(s[i]);
    return ORC_OK;
}

int orc_ddpsi(int64_t n, const double* s, double* out) {
    if (n < 0 || (n > 0 && (!s || !out))) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) out[i] = ddpsi(s[i]);
    return ORC_OK;
}

/* ------------------------------------------------- compensated summation */

/* Neumaier's improved Kahan-Babuska sum (Neumaier 1974). */
typedef struct {
    double s, c;
} nsum_t;

static void nsum_add(nsum_t* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum_t* a) { return a->s + a->c; }

/* Error-free transformations (Knuth TwoSum; TwoProduct via fused multiply-add),
 * as used by Dot2 of Ogita, Rump and Oishi, "Accurate sum and dot product",
 * SIAM J. Sci. Comput. 26(6), 2005. */
static void two_sum(double a, double b, double* s, double* e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double* p, double* e) {
    double h = a * b;
    *e = fma(a, b, -h);
    *p = h;
}

/* Dot2 accumulator: p + s carries a result as if computed in twice the
 * working precision and rounded once. */
typedef struct {
    double p, s;
} dot2_t;

static void dot2_add(dot2_t* d, double a, double b) {
    double h, r, q;
    two_prod(a, b, &h, &r);
    two_sum(d->p, h, &d->p, &q);
    d->s = d->s + (q + r);
}

static double dot2_get(const dot2_t* d) { return d->p + d->s; }

/* ----------------------------------------------------------------- meshes */

static int mesh_args_ok(int64_t N, int64_t E, int32_t k, const int32_t* conn) {
    if (N < 0 || E < 0 || k <= 0) return 0;
    if (E > 0 && !conn) return 0;
    return 1;
}

/* Connectivity is index metadata and is never differentiated; every entry
 * must address a node (section 3.1: extents and indices are inactive). */
int orc_mesh_check(int64_t N, int64_t E, int32_t k, const int32_t* conn) {
    if (!mesh_args_ok(N, E, k, conn)) return ORC_EINVAL;
    for (int64_t i = 0; i < E * (int64_t)k; ++i)
        if (conn[i] < 0 || (int64_t)conn[i] >= N) return ORC_ERANGE;
    return ORC_OK;
}

/* u = G x:  u[e] = sum over j ascending of B[e,j] * x[conn[e,j]]. */
int orc_mesh_gather(int64_t N, int64_t E, int32_t k, const int32_t* conn, const double* B,
                    const double* x, double* u) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    for (int64_t e = 0; e < E; ++e) {
        double acc = 0.0;
        for (int32_t j = 0; j < k; ++j) {
            double prod = B[e * k + j] * x[conn[e * k + j]];
            acc = acc + prod;
        }
        u[e] = acc;
    }
    return ORC_OK;
}

/* g = G^T v:  g zeroed, then for e ascending, j ascending,
 * g[conn[e,j]] += v[e] * B[e,j]  (the transposed read of x). */
int orc_mesh_scatter(int64_t N, int64_t E, int32_t k, const int32_t* conn, const double* B,
                     const double* v, double* g) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    for (int64_t i = 0; i < N; ++i) g[i] = 0.0;
    for (int64_t e = 0; e < E; ++e)
        for (int32_t j = 0; j < k; ++j) {
            double c = v[e] * B[e * k + j];
            g[conn[e * k + j]] += c;
        }
    return ORC_OK;
}

/* Per-element terms t[e] = w[e] * psi(u[e]) and, optionally, u itself. */
int orc_mesh_terms(int64_t N, int64_t E, int32_t k, const int32_t* conn, const double* B,
                   const double* w, const double* x, double* t, double* u_out) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    double* u = u_out ? u_out : (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    if (!u) return ORC_EINVAL;
    orc_mesh_gather(N, E, k, conn, B, x, u);
    for (int64_t e = 0; e < E; ++e) t[e] = w[e] * psi(u[e]);
    if (!u_out) free(u);
    return ORC_OK;
}

/* f = sum_e w[e] psi(u[e]), Neumaier-compensated over ascending e. */
int orc_mesh_objective(int64_t N, int64_t E, int32_t k, const int32_t* conn, const double* B,
                       const double* w, const double* x, double* f_out) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    if (!f_out) return ORC_EINVAL;
    nsum_t acc = {0.0, 0.0};
    for (int64_t e = 0; e < E; ++e) {
        double u = 0.0;
        for (int32_t j = 0; j < k; ++j) {
            double prod = B[e * k + j] * x[conn[e * k + j]];
            u = u + prod;
        }
        nsum_add(&acc, w[e] * psi(u));
    }
    *f_out = nsum_get(&acc);
    return ORC_OK;
}

/* Reverse mode: forward replay (gather, terms, sum), then seed fbar,
 * broadcast to every term, local derivative v[e] = fbar * w[e] * psi'(u[e]),
 * and the transposed gather g = G^T v.  g is overwritten. */
int orc_mesh_gradient(int64_t N, int64_t E, int32_t k, const int32_t* conn, const double* B,
                      const double* w, const double* x, double fbar, double* f_out, double* g) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    double* u = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double* v = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    if (!u || !v) {
        free(u);
        free(v);
        return ORC_EINVAL;
    }
    orc_mesh_gather(N, E, k, conn, B, x, u);
    nsum_t acc = {0.0, 0.0};
    for (int64_t e = 0; e < E; ++e) nsum_add(&acc, w[e] * psi(u[e]));
    if (f_out) *f_out = nsum_get(&acc);
    for (int64_t e = 0; e < E; ++e) v[e] = fbar * w[e] * dpsi(u[e]);
    orc_mesh_scatter(N, E, k, conn, B, v, g);
    free(u);
    free(v);
    return ORC_OK;
}

#ifdef ORC_OMP
#include <omp.h>

/* The same gradient with its loops spread over the host's threads (built
 * only as liboracle_omp.so, with -fopenmp -DORC_OMP; the CPU-baseline
 * timing uses it, the parity tests use the plain build).  Thread t takes a
 * contiguous block of elements in every loop; f is a Neumaier sum per
 * thread, and the partial sums are added in thread order; each thread
 * scatters into a private zeroed copy of g, and the copies are added node
 * by node in thread order.  Returns the number of threads used, or a
 * negative status. */
int orc_mesh_gradient_threads(int64_t N, int64_t E, int32_t k, const int32_t* conn,
                              const double* B, const double* w, const double* x, double fbar,
                              double* f_out, double* g) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return -st;
    const int T = omp_get_max_threads();
    double* u = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double* gt = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * (size_t)T);
    nsum_t* part = (nsum_t*)malloc(sizeof(nsum_t) * (size_t)T);
    if (!u || !gt || !part) {
        free(u);
        free(gt);
        free(part);
        return -ORC_EINVAL;
    }
#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num();
        const int64_t e0 = E * t / T, e1 = E * (t + 1) / T;
        nsum_t acc = {0.0, 0.0};
        for (int64_t e = e0; e < e1; ++e) {
            double a = 0.0;
            for (int32_t j = 0; j < k; ++j) {
                double prod = B[e * k + j] * x[conn[e * k + j]];
                a = a + prod;
            }
            u[e] = a;
            nsum_add(&acc, w[e] * psi(a));
        }
        part[t] = acc;
        double* gl = gt + (size_t)N * (size_t)t;
        for (int64_t i = 0; i < N; ++i) gl[i] = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            double v = fbar * w[e] * dpsi(u[e]);
            for (int32_t j = 0; j < k; ++j) gl[conn[e * k + j]] += v * B[e * k + j];
        }
#pragma omp barrier
        const int64_t n0 = N * t / T, n1 = N * (t + 1) / T;
        for (int64_t i = n0; i < n1; ++i) {
            double s = 0.0;
            for (int q = 0; q < T; ++q) s += gt[(size_t)N * (size_t)q + (size_t)i];
            g[i] = s;
        }
    }
    if (f_out) {
        nsum_t acc = {0.0, 0.0};
        for (int t = 0; t < T; ++t) {
            nsum_add(&acc, part[t].s);
            nsum_add(&acc, part[t].c);
        }
        *f_out = nsum_get(&acc);
    }
    free(u);
    free(gt);
    free(part);
    return T;
}
#endif

/* Hessian-vector product of the mesh objective:
 * H d = G^T ( w (.) psi''(G x) (.) (G d) ). */
int orc_mesh_hvp(int64_t N, int64_t E, int32_t k, const int32_t* conn, const double* B,
                 const double* w, const double* x, const double* d, double* hd) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    double* u = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    if (!u || !q) {
        free(u);
        free(q);
        return ORC_EINVAL;
    }
    orc_mesh_gather(N, E, k, conn, B, x, u);
    orc_mesh_gather(N, E, k, conn, B, d, q);
    for (int64_t e = 0; e < E; ++e) q[e] = w[e] * ddpsi(u[e]) * q[e];
    orc_mesh_scatter(N, E, k, conn, B, q, hd);
    free(u);
    free(q);
    return ORC_OK;
}

/* Transposed connectivity: for node n, the incidences (e*k + j) with
 * conn[e,j] == n, in ascending order; offs[n] .. offs[n+1] delimit them.
 * A counting sort taken in ascending (e, j) order yields the rows sorted. */
int orc_mesh_csr(int64_t N, int64_t E, int32_t k, const int32_t* conn, int32_t* offs,
                 int32_t* inc) {
    int st = orc_mesh_check(N, E, k, conn);
    if (st) return st;
    for (int64_t i = 0; i <= N; ++i) offs[i] = 0;
    for (int64_t i = 0; i < E * (int64_t)k; ++i) offs[conn[i] + 1] += 1;
    for (int64_t n = 0; n < N; ++n) offs[n + 1] += offs[n];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    if (!fill) return ORC_EINVAL;
    for (int64_t n = 0; n < N; ++n) fill[n] = offs[n];
    for (int64_t i = 0; i < E * (int64_t)k; ++i) inc[fill[conn[i]]++] = (int32_t)i;
    free(fill);
    return ORC_OK;
}

/* Number of node conflicts of a colouring: pairs of distinct elements of one
 * colour that share a node, counted once per (node, colour) excess.  A valid
 * colouring for a race-free non-atomic scatter returns 0. */
int64_t orc_colour_conflicts(int64_t N, int64_t E, int32_t k, const int32_t* conn,
                             const int32_t* colour, int32_t n_colours) {
    if (orc_mesh_check(N, E, k, conn) != ORC_OK || n_colours <= 0) return -1;
    int64_t conflicts = 0;
    int64_t* last = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!last) return -1;
    for (int32_t c = 0; c < n_colours; ++c) {
        for (int64_t n = 0; n < N; ++n) last[n] = -1;
        for (int64_t e = 0; e < E; ++e) {
            if (colour[e] != c) continue;
            for (int32_t j = 0; j < k; ++j) {
                int32_t n = conn[e * k + j];
                if (last[n] >= 0 && last[n] != e) ++conflicts;
                last[n] = e;
            }
        }
    }
    free(last);
    return conflicts;
}

/* Greedy colouring in element order, from its definition: element e takes
 * the smallest colour that no earlier element sharing a node with it has
 * (e' < e with conn[e', i] == conn[e, j] for some i, j).  The elements that
 * share a node with e are found through the transposed connectivity
 * (orc_mesh_csr).  colour[E] is written; returns the number of colours, or
 * -1 on bad arguments or if more than max_colours are needed.  Used to
 * check, exactly, the colour classes the library builds for its non-atomic
 * reverse scatter (the conclusion's rescheduled reverse threads). */
int32_t orc_greedy_colour(int64_t N, int64_t E, int32_t k, const int32_t* conn, int32_t max_colours,
                          int32_t* colour) {
    if (orc_mesh_check(N, E, k, conn) != ORC_OK || max_colours <= 0) return -1;
    int32_t* offs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 1));
    int32_t* inc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(E * k > 0 ? E * k : 1));
    char* taken = (char*)malloc((size_t)max_colours);
    if (!offs || !inc || !taken) {
        free(offs);
        free(inc);
        free(taken);
        return -1;
    }
    orc_mesh_csr(N, E, k, conn, offs, inc);
    int32_t n_colours = 0;
    for (int64_t e = 0; e < E; ++e) {
        memset(taken, 0, (size_t)max_colours);
        for (int32_t j = 0; j < k; ++j) {
            int32_t n = conn[e * k + j];
            for (int32_t q = offs[n]; q < offs[n + 1]; ++q) {
                int64_t other = inc[q] / k; /* incidence e' * k + i */
                if (other < e) taken[colour[other]] = 1;
            }
        }
        int32_t c = 0;
        while (c < max_colours && taken[c]) ++c;
        if (c == max_colours) {
            n_colours = -1;
            break;
        }
        colour[e] = c;
        if (c + 1 > n_colours) n_colours = c + 1;
    }
    free(offs);
    free(inc);
    free(taken);
    return n_colours;
}

/* ------------------------------------------------------------------ dense */

/* r = A x with Dot2 per row (ascending column index). */
static void dense_rows(int64_t rows, int64_t cols, const double* A, int64_t lda,
                       const double* x, int64_t incx, double* r) {
    for (int64_t i = 0; i < rows; ++i) {
        dot2_t d = {0.0, 0.0};
        for (int64_t j = 0; j < cols; ++j) dot2_add(&d, A[i * lda + j], x[j * incx]);
        r[i] = dot2_get(&d);
    }
}

/* g = A^T v with Dot2 per column (ascending row index). g has stride incg. */
static void dense_cols(int64_t rows, int64_t cols, const double* A, int64_t lda,
                       const double* v, double* g, int64_t incg, dot2_t* acc) {
    for (int64_t j = 0; j < cols; ++j) acc[j].p = acc[j].s = 0.0;
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t j = 0; j < cols; ++j) dot2_add(&acc[j], A[i * lda + j], v[i]);
    for (int64_t j = 0; j < cols; ++j) g[j * incg] = dot2_get(&acc[j]);
}

/* Dense objective: f = sum_i w_i psi((A x)_i).  r_out (optional) gets A x. */
int orc_dense_objective(int64_t rows, int64_t cols, const double* A, const double* x,
                        const double* w, double* f_out, double* r_out) {
    if (rows < 0 || cols < 0 || !f_out) return ORC_EINVAL;
    double* r = r_out ? r_out : (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
    if (!r) return ORC_EINVAL;
    dense_rows(rows, cols, A, cols, x, 1, r);
    nsum_t acc = {0.0, 0.0};
    for (int64_t i = 0; i < rows; ++i) nsum_add(&acc, w[i] * psi(r[i]));
    *f_out = nsum_get(&acc);
    if (!r_out) free(r);
    return ORC_OK;
}

/* Dense gradient: grad = A^T (fbar * w (.) psi'(A x)); f returned too. */
int orc_dense_gradient(int64_t rows, int64_t cols, const double* A, const double* x,
                       const double* w, double fbar, double* f_out, double* g) {
    if (rows < 0 || cols < 0) return ORC_EINVAL;
    double* r = (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
    dot2_t* acc = (dot2_t*)malloc(sizeof(dot2_t) * (size_t)(cols > 0 ? cols : 1));
    if (!r || !acc) {
        free(r);
        free(acc);
        return ORC_EINVAL;
    }
    dense_rows(rows, cols, A, cols, x, 1, r);
    nsum_t fs = {0.0, 0.0};
    for (int64_t i = 0; i < rows; ++i) nsum_add(&fs, w[i] * psi(r[i]));
    if (f_out) *f_out = nsum_get(&fs);
    for (int64_t i = 0; i < rows; ++i) r[i] = fbar * w[i] * dpsi(r[i]);
    dense_cols(rows, cols, A, cols, r, g, 1, acc);
    free(r);
    free(acc);
    return ORC_OK;
}

/* Batched dense, selected columns: for each listed column c of X (m x n,
 * row-major) the dense objective and gradient with x = X[:,c], w = W[:,c]:
 * f_cols[t] = sum_i W[i,c] psi((A X)_{i,c}),
 * G_cols[:, t] (m x ncols row-major) = A^T (W[:,c] (.) psi'((A X)[:,c])).
 * The total objective is the sum over all n columns. */
int orc_bdense_columns(int64_t m, int64_t n, const double* A, const double* X, const double* W,
                       int64_t ncols, const int64_t* cols, double* f_cols, double* G_cols) {
    if (m < 0 || n < 0 || ncols < 0) return ORC_EINVAL;
    double* xc = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* r = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    dot2_t* acc = (dot2_t*)malloc(sizeof(dot2_t) * (size_t)(m > 0 ? m : 1));
    if (!xc || !r || !acc) {
        free(xc);
        free(r);
        free(acc);
        return ORC_EINVAL;
    }
    int st = ORC_OK;
    for (int64_t t = 0; t < ncols; ++t) {
        int64_t c = cols[t];
        if (c < 0 || c >= n) {
            st = ORC_ERANGE;
            break;
        }
        for (int64_t i = 0; i < m; ++i) xc[i] = X[i * n + c];
        dense_rows(m, m, A, m, xc, 1, r);
        nsum_t fs = {0.0, 0.0};
        for (int64_t i = 0; i < m; ++i) nsum_add(&fs, W[i * n + c] * psi(r[i]));
        f_cols[t] = nsum_get(&fs);
        for (int64_t i = 0; i < m; ++i) r[i] = W[i * n + c] * dpsi(r[i]);
        dense_cols(m, m, A, m, r, G_cols + t, ncols, acc);
    }
    free(xc);
    free(r);
    free(acc);
    return st;
}

/* Compensated sum of an array (Neumaier), for reductions of per-instance
 * or per-column partial results. */
double orc_sum(int64_t n, const double* a) {
    nsum_t acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nsum_add(&acc, a[i]);
    return nsum_get(&acc);
}

/* ------------------------------------------- the paper's section 4 example */

/* f(x, b) = || A (3x) - b ||^2 with A the n x n 1D Laplacian (2 on the
 * diagonal, -1 on the first off-diagonals, rows truncated at both ends, as the
 * `j != 0` / `j != n-1` guards of the example do).  Its reverse pass:
 * ybar = 2 y (reverse of the square and of the sum, seed fbar), then the
 * transposed stencil for xbar (A is symmetric) times 3, and bbar = -ybar.
 * gx and gb are overwritten; either may be NULL. */
int orc_laplace1d_gradient(int64_t n, const double* x, const double* b, double fbar,
                           double* f_out, double* gx, double* gb) {
    if (n < 0 || (n > 0 && (!x || !b))) return ORC_EINVAL;
    double* y = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!y) return ORC_EINVAL;
    nsum_t acc = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        double v = 2.0 * (3.0 * x[j]) - b[j];
        if (j != 0) v = v - 3.0 * x[j - 1];
        if (j != n - 1) v = v - 3.0 * x[j + 1];
        y[j] = v;
        nsum_add(&acc, v * v);
    }
    if (f_out) *f_out = nsum_get(&acc);
    for (int64_t j = 0; j < n; ++j) y[j] = fbar * 2.0 * y[j];  /* ybar */
    if (gx) {
        for (int64_t i = 0; i < n; ++i) {
            double v = 2.0 * y[i];
            if (i != 0) v = v - y[i - 1];
            if (i != n - 1) v = v - y[i + 1];
            gx[i] = 3.0 * v;
        }
    }
    if (gb)
        for (int64_t j = 0; j < n; ++j) gb[j] = -y[j];
    free(y);
    return ORC_OK;
}
