/*
 * asp.h -- C ABI of the additive sweeping preconditioner for the PML-truncated
 * Helmholtz equation (F. Liu and L. Ying, "Additive Sweeping Preconditioner for
 * the Helmholtz Equation"), running inside restarted GMRES on one AMD MI355X.
 *
 * The problem (Section 1, eq. (helm); Section 2 PML; eq. (2D) of Section 3.1,
 * eq. (3D) of Section 4.1): on the unit square / cube with n interior grid points
 * per side, h = 1/(n+1), find u with
 *
 *     sum_k s_k d_k (s_k d_k u) + omega^2 / c(x)^2 u = f,   u = 0 on the boundary,
 *
 * discretized by the centered scheme, with a PML of width eta = pml_eta*h and
 * strength C on every side (the setting of the experiments, Sections 3.2 and
 * 4.2).  The library works on the symmetric form of that system (each row
 * divided by prod_k s_k(i_k), Section 3.1 remark 4), A u = f / prod_k s_k, which
 * has the same solution u.
 *
 * Conventions shared by every entry point:
 *   - Grid vectors are column-major (x1 fastest, Section 3.1), length N = n^dim.
 *   - Complex vectors are interleaved (re, im) IEEE double, i.e. complex128.
 *     A batch of nrhs vectors is stored vector after vector (nrhs * N entries).
 *   - Vector arguments marked "device" are device pointers on the current HIP
 *     device; the caller owns them and keeps them alive until the work that the
 *     call enqueued on the plan's stream has finished.
 *   - All device work is enqueued on the plan's stream (asp_opts.stream or
 *     asp_set_stream).  Calls that return results to host memory (asp_gmres,
 *     asp_layers, asp_tables, asp_info) synchronize that stream.
 *   - No call aborts or throws: every failure is reported by the return code;
 *     asp_last_error() gives a text description.  After ASP_ERR_DEVICE the plan
 *     must only be destroyed.
 *   - A plan is not thread safe; use one plan per host thread or lock it.
 */
#ifndef ASP_H
#define ASP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct asp_plan asp_plan;

typedef enum {
    ASP_OK = 0,
    ASP_ERR_ARG = 1,       /* invalid argument (sizes, NaN/non-positive c, bad pointers) */
    ASP_ERR_OOM = 2,       /* device or host allocation failed */
    ASP_ERR_STATE = 3,     /* call out of order (apply/gmres before factor) */
    ASP_ERR_BREAKDOWN = 4, /* zero or non-finite pivot in a layer factorization */
    ASP_ERR_NOCONV = 5,    /* GMRES reached maxit; iters/relres/u still filled in */
    ASP_ERR_DEVICE = 6     /* a HIP runtime call failed */
} asp_status;

typedef enum {
    ASP_PREC_FP64 = 0,     /* layer factors and layer solves in complex double */
    ASP_PREC_FP32 = 1,     /* layer factors and layer solves in complex float;
                              GMRES, stencil and all grid vectors stay complex double */
    ASP_PREC_BF16X3 = 2    /* FP32 factors as ASP_PREC_FP32, with matrix products as real-split
                              products on bf16 matrix cores: each FP32 operand x = hi + lo with
                              hi = bf16(x), lo = bf16(x - hi), and x*y ~ hi*hi + hi*lo + lo*hi
                              accumulated in FP32 (about 16 significant bits per product).
                              3D: the Schur-complement (trailing) updates of the block
                              inversions; 2D: the layer solves (each block step S_k^-1 times
                              the step vectors), the boundary maps they produce and the
                              sweep-map products */
} asp_prec;

typedef enum { ASP_SUB_M = 0, ASP_SUB_R = 1, ASP_SUB_L = 2 } asp_sub_kind;

typedef enum {
    ASP_FACT3D_ND = 0,      /* nested dissection (Section 4.1): the unknowns grouped into
                               columns along the sweep axis, the n x n columns ordered by
                               nested dissection, multifrontal elimination;
                               O(n^2 L^2 log n) factor entries per problem */
    ASP_FACT3D_BLOCKS = 1,  /* a dense block recurrence along x1: n blocks of n L
                               unknowns, O(n^3 L^2) factor entries per problem */
    ASP_FACT3D_RECURSIVE = 2 /* the recursive sweep (Section 5): each quasi-2D auxiliary
                               problem is not factored exactly but solved by one
                               application of the additive sweeping preconditioner
                               along x2 (inner layers and auxiliary PML as the outer
                               ones: layer_b lines, pml_eta / pml_aux), whose quasi-1D
                               problems are factored by the block recurrence along x1
                               (blocks of L_x3 x L_x2 unknowns).  G~ is then approximate
                               (the outer GMRES is flexible); equal layer widths only */
} asp_fact3d;

typedef enum {
    ASP_SWEEP2D_MAPS = 0,      /* the factorization also computes, for every R_p and L_p with
                                  1 < p < m, the dense n x n map from the boundary data it
                                  receives to the boundary line it hands on; a sweep step is
                                  then one map product, and all R/L solves run at once after
                                  the sweeps.  O(n^3 / b) map entries and setup O(n^3 L^2 / b) */
    ASP_SWEEP2D_SEQUENTIAL = 1 /* Algorithm 2 as stated: the sweeps solve R_2 .. R_m and
                                  L_{m-1} .. L_1 one after another (each R/L pair in one launch),
                                  each handing its boundary line to the next; no maps */
} asp_sweep2d;

typedef struct {
    double C;       /* PML strength (Section 2, "an appropriate positive constant"); default 25 */
    int prec;       /* asp_prec; default ASP_PREC_FP64 */
    void* stream;   /* hipStream_t for all device work; default 0 (the null stream) */
    int host_only;  /* nonzero: build the partition and tables on the host only, touch no
                       device; the plan then supports asp_layers, asp_tables, asp_info,
                       asp_last_error and asp_destroy (other calls return ASP_ERR_STATE) */
    int pml_aux;    /* width (grid lines) of the auxiliary PML on the pads that face a
                       neighbouring layer: the thinner auxiliary PML of the Section 3.1
                       remarks, eta_aux = pml_aux * h.  Pads at the domain boundary keep
                       the boundary PML.  0 (default): pml_eta; otherwise 2..pml_eta,
                       else ASP_ERR_ARG */
    int n_layers;   /* 0 (default): layers of layer_b physical lines each, the last one
                       holding the remainder.  > 0: arbitrary layer widths (Section 3.1
                       remarks: the layers need not have equal widths); layer_widths
                       then holds n_layers widths and layer_b is ignored */
    const int* layer_widths;  /* HOST pointer, n_layers entries: physical grid lines of
                       layer p = 1..m along the sweep axis, each >= 1, summing to
                       n - 2(pml_eta - 1); read during asp_setup only, not kept.
                       Layer 1 also takes the pml_eta - 1 PML lines below it, layer m
                       those above it.  Violations: ASP_ERR_ARG */
    int fact3d;     /* asp_fact3d: how the quasi-2D auxiliary problems of a 3D plan are
                       factored; default ASP_FACT3D_ND.  ND and BLOCKS give the same
                       operator G~, RECURSIVE an approximation of it.  Ignored by 2D
                       plans; other values ASP_ERR_ARG */
    int sweep2d;    /* asp_sweep2d: how a 2D apply moves boundary values between layers;
                       default ASP_SWEEP2D_MAPS.  Both give the same operator.  Ignored by
                       3D plans; other values ASP_ERR_ARG */
} asp_opts;

typedef struct {
    int dim, n, m;            /* dimension, points per side, number of layers (Section 2) */
    int n_sub;                /* 3m - 2 auxiliary problems (Algorithms 1 and 3) */
    int max_lines;            /* largest number of sweep lines of one auxiliary problem */
    size_t factor_bytes;      /* device bytes the factors (and sweep maps) occupy once
                                 asp_factor has run; known right after asp_setup */
    size_t workspace_bytes;   /* device bytes of the apply/GMRES workspaces now allocated,
                                 and of the 3D nested-dissection factorization's work
                                 buffers, which stay between factorizations */
    int factored;             /* nonzero once asp_factor has succeeded */
    size_t factor_work_bytes; /* device bytes of the work buffers asp_factor allocates besides
                                 the factors: the 3D level, panel and pivot buffers (2D
                                 plans need none: the boundary maps are built without
                                 scratch).  They stay allocated (and are counted in
                                 workspace_bytes) until asp_release_workspace; known right
                                 after asp_setup */
} asp_plan_info;

/* Fill *opts with the defaults (C = 25, FP64, null stream, device plan). */
void asp_default_opts(asp_opts* opts);

/* asp_setup -- build a plan for one discretized problem (Section 1 eq. (helm),
 * Section 2 PML and partition, Sections 3.1 / 4.1 auxiliary domains).
 *   plan     out: new plan; owned by the caller, release with asp_destroy.  On
 *            failure *plan is either NULL or a plan that only supports
 *            asp_last_error and asp_destroy.
 *   dim      2 or 3; the sweep axis is x2 (2D) or x3 (3D), the slowest index.
 *   c        HOST pointer, n^dim velocities (column-major), finite and > 0;
 *            copied, the caller may free it on return.
 *   omega    angular frequency, > 0.
 *   n        interior points per side; n - 2(pml_eta - 1) >= 1.
 *   layer_b  grid lines per interior layer (Section 2, b), >= 1; ignored when
 *            opts->n_layers > 0 (arbitrary widths).
 *   pml_eta  PML width in grid units (eta = pml_eta * h, Section 2), >= 2.
 *   opts     NULL for defaults.
 * Only host work and uploads of small tables; no factorization.
 * Errors: ASP_ERR_ARG, ASP_ERR_OOM, ASP_ERR_DEVICE. */
asp_status asp_setup(asp_plan** plan, int dim, const double* c, double omega, int n,
                     int layer_b, int pml_eta, const asp_opts* opts);

/* asp_factor -- Algorithm 1 (2D) / 3 (3D): factor every auxiliary problem
 * H^M_q (q = 1..m), H^R_p (p = 2..m), H^L_p (p = 1..m-1).  The factors stay
 * resident in device memory until asp_destroy.  Every call recomputes them
 * (deterministically: the result is the same each time).
 * Errors: ASP_ERR_OOM, ASP_ERR_BREAKDOWN (singular or non-finite pivot),
 * ASP_ERR_DEVICE, ASP_ERR_ARG (dimension not supported by this build). */
asp_status asp_factor(asp_plan* plan);

/* asp_apply -- z = M^-1 r, Algorithm 2 (2D) / 4 (3D): the m M-solves, the
 * right-going and left-going sweeps over the boundary values, and the sum.
 *   nrhs >= 1 right-hand sides.
 *   r  device, nrhs * N complex128, symmetric-form residuals; read only.
 *   z  device, nrhs * N complex128, written; must not alias r.
 * Errors: ASP_ERR_STATE (not factored), ASP_ERR_ARG, ASP_ERR_OOM, ASP_ERR_DEVICE. */
asp_status asp_apply(asp_plan* plan, const void* r, void* z, int nrhs);

/* Size of the fixed device array asp_apply_noalloc works in.  Each device the
 * library runs on holds one such array from the library's load until the
 * process ends. */
#define ASP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* asp_apply_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): z = M^-1 r exactly as asp_apply computes it (the same kernels,
 * bitwise the same result), but the apply's work buffers are carved from the
 * fixed array of ASP_NOALLOC_SCRATCH_BYTES bytes instead of the plan's
 * workspaces, and the call allocates and frees nothing (nor does it record
 * timing events: asp_timing_read does not see it).
 *   r, z, nrhs as for asp_apply.  The plan must be factored (asp_factor
 *   allocates the factors; this call only reads them).  2D plans and 3D plans
 *   factored by nested dissection.  The work buffers grow with n, the layer
 *   count and nrhs: 2D n = 127 fits with up to 16 right-hand sides in either
 *   precision, 3D n = 31 with 16.
 * Every call on one device uses that device's array and leaves the last
 * call's contents in it (nothing in it has to start at zero): calls that
 * overlap on one device (other streams, other plans, other host threads) race
 * and give wrong results.
 * Errors: ASP_ERR_ARG (bad arguments; a 3D plan factored by the block
 * recurrence; work buffers for nrhs right-hand sides larger than
 * ASP_NOALLOC_SCRATCH_BYTES, the message giving both sizes), ASP_ERR_STATE
 * (not factored), ASP_ERR_DEVICE. */
asp_status asp_apply_noalloc(asp_plan* plan, const void* r, void* z, int nrhs);

/* asp_matvec -- y = A x with the symmetric-form 5-point (2D) / 7-point (3D)
 * PML operator of eq. (2D) / (3D), complex double, for nrhs >= 1 vectors.
 *   x  device, nrhs * N complex128;  y  device, nrhs * N complex128, no alias.
 * Errors: ASP_ERR_ARG, ASP_ERR_DEVICE. */
asp_status asp_matvec(asp_plan* plan, const void* x, void* y, int nrhs);

/* asp_gmres -- solve A u = f / prod s for nrhs independent right-hand sides
 * with restarted GMRES (Sections 3.2, 4.2) right-preconditioned by asp_apply
 * (flexible form, so a reduced-precision preconditioner is allowed).  x0 = 0;
 * a right-hand side stops when its true relative residual
 * ||f/prod s - A u|| / ||f/prod s|| is <= tol.
 *   f       device, nrhs * N complex128, the PHYSICAL right-hand side f.
 *   u       device, nrhs * N complex128, written with the solution.
 *   nrhs    >= 1.
 *   tol     > 0;  1 <= restart <= 64;  maxit >= 1 (total Arnoldi steps per RHS).
 *   iters   HOST, [nrhs]: Arnoldi steps (= preconditioner applies) per RHS.
 *   relres  HOST, [nrhs]: final true relative residual per RHS.
 * Factors the plan first if needed.  Workspaces ((2 restart + 3) * nrhs * N
 * complex128) are allocated on first use and kept by the plan.
 * Errors: ASP_ERR_NOCONV (some RHS not converged; outputs filled), ASP_ERR_ARG,
 * ASP_ERR_OOM, ASP_ERR_BREAKDOWN, ASP_ERR_DEVICE. */
asp_status asp_gmres(asp_plan* plan, const void* f, void* u, int nrhs, double tol,
                     int restart, int maxit, int* iters, double* relres);

/* asp_subsolve -- one auxiliary Green's operator on its own (Section 3.1,
 * "Auxiliary Green's operators"): G~^M_p (kind ASP_SUB_M, p = 1..m),
 * G~^R_p (ASP_SUB_R, p = 2..m) or G~^L_p (ASP_SUB_L, p = 1..m-1).
 *   in   device; M: nrhs * (N_p) values y on X_p (column-major restriction);
 *        R/L: nrhs * n^(dim-1) boundary values w.  complex128.
 *   out  device; nrhs * N_p complex128: the solution restricted to X_p.
 * N_p = n^(dim-1) * |X_p|; nrhs >= 1.  Requires a factored plan.
 * Errors: ASP_ERR_ARG, ASP_ERR_STATE, ASP_ERR_OOM, ASP_ERR_DEVICE. */
asp_status asp_subsolve(asp_plan* plan, int kind, int p, const void* in, void* out, int nrhs);

/* asp_layers -- the partition and auxiliary grids (Section 2; Sections 3.1 /
 * 4.1 "Auxiliary domains"), 1-based grid lines along the sweep axis.
 *   m       HOST out: number of layers.
 *   layers  HOST, NULL or [m][2]: (first, last) line of X_p.
 *   subs    HOST, NULL or [3m-2][6]: (kind, p, lo, hi, phi, psi) for M_1..M_m,
 *           R_2..R_m, L_1..L_{m-1}: the lines lo..hi of the extended grid and
 *           the zero region [phi, psi] of its sweep-axis PML profile. */
asp_status asp_layers(const asp_plan* plan, int* m, int* layers, int* subs);

/* asp_tables -- the PML tables the plan uses (Section 2; eq. (1D) evaluation
 * at integer and half-integer points), for checking.
 *   sub     -1: the boundary PML of one axis (lines 1..n);
 *           0..3m-3: the sweep-axis profile of auxiliary problem `sub`
 *           (order of asp_layers).
 *   s_int   HOST [len][2] complex: s at the lines (len = n or the problem's lines).
 *   s_half  HOST [len+1][2] complex: s at the half lines before/after them. */
asp_status asp_tables(const asp_plan* plan, int sub, double* s_int, double* s_half);

/* Kernel classes for asp_timing_read. */
typedef enum {
    ASP_K_FACTOR = 0,     /* layer factorizations (Algorithm 1) */
    ASP_K_TRANSFER = 1,   /* boundary-to-boundary maps of the auxiliary problems (setup) */
    ASP_K_SOLVE_M = 2,    /* the M-solves G~^M_q of an apply */
    ASP_K_SOLVE_RL = 3,   /* G~^R_p / G~^L_p solves of an apply */
    ASP_K_SWEEP = 4,      /* the sequential boundary-value sweeps of an apply */
    ASP_K_COMBINE = 5,    /* the final sum of an apply */
    ASP_K_STENCIL = 6,    /* y = A x */
    ASP_K_KRYLOV = 7,     /* Gram-Schmidt, norms, updates of GMRES */
    ASP_K_COUNT = 8
} asp_kernel_class;

/* asp_timing_enable -- start (enable != 0, counters reset) or stop recording a
 * HIP event pair around every kernel launch of the plan, on the plan's stream.
 * asp_timing_read -- for one class: number of launches, summed device time
 * (ms), and the algorithmic bytes moved and floating-point operations of
 * those launches (the minimum traffic and work of the operation, counted by
 * the host from the launch sizes).  Synchronizes the stream.  Any pointer may
 * be NULL. */
asp_status asp_timing_enable(asp_plan* plan, int enable);
asp_status asp_timing_read(asp_plan* plan, int cls, int* launches, double* ms, double* bytes,
                           double* flops);

/* asp_workspace_estimate -- device bytes of the workspaces asp_gmres allocates
 * for nrhs right-hand sides and the given restart length (apply scratch,
 * sweep data, Krylov basis); host only.
 * asp_release_workspace -- free those workspaces (and the factorization's
 * kept work buffers) now, keeping the factors (a factor cache keeps idle plans
 * this way); the next call allocates again.
 * Synchronizes the plan's stream. */
asp_status asp_workspace_estimate(const asp_plan* plan, int nrhs, int restart, size_t* bytes);
asp_status asp_release_workspace(asp_plan* plan);

/* asp_set_cache_limit -- device memory the library may keep for reuse, per
 * device (serving loops that create, trim and destroy plans; no section of
 * the paper).  Device blocks that plans give back (asp_release_workspace,
 * asp_destroy, the factorization's work buffers, workspaces replaced by larger
 * ones) are kept, up to `bytes` per device, and handed out again to later
 * requests of at least their size and at most an eighth (or 2 MiB) more,
 * instead of going back to the driver: a driver free of a large block takes
 * milliseconds per gigabyte and waits for the whole device.  0 (the default)
 * keeps nothing.  Lowering the limit returns the excess at once; an
 * allocation that fails returns the whole cache and tries again.  Returns the
 * previous limit.  Thread-safe.  Kept bytes are device memory that other
 * allocators in the process cannot use.
 * asp_cached_bytes -- bytes kept, over all devices. */
size_t asp_set_cache_limit(size_t bytes);
size_t asp_cached_bytes(void);

/* asp_info -- sizes and memory of the plan.  asp_set_stream -- change the stream
 * used by later calls.  asp_destroy -- free everything (NULL is ignored).
 * asp_last_error -- description of the last failure of this plan (never NULL). */
asp_status asp_info(const asp_plan* plan, asp_plan_info* info);
asp_status asp_set_stream(asp_plan* plan, void* stream);
void asp_destroy(asp_plan* plan);
const char* asp_last_error(const asp_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* ASP_H */
