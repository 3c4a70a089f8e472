/*
 * stbem: space-time Galerkin boundary elements for the 2D heat equation on
 * one AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Dohr, Merta, Of, Steinbach, Zapletal, "A parallel solver for a
 * preconditioned space-time boundary element method for the heat equation"
 * (arXiv:1811.05224).  Model problem eq.(1): alpha du/dt - Laplace u = 0 in
 * Omega x (0,T), u = g on Gamma x (0,T), u(.,0) = u0.  The Neumann datum w
 * solves the Galerkin system eq.(4)
 *     V_h w = (1/2 M_h + K_h) g - M_h^0 u0
 * with V_h (single layer, piecewise constants), K_h (double layer, trial
 * functions continuous piecewise linear in space x constant in time), M_h
 * (mass) and M_h^0 (initial potential on a triangulation of Omega).  GMRES is
 * preconditioned with C_V^{-1} = Mt^{-1} D_h Mt^{-1} (Sec. 2, Theorem 1): D_h
 * is the hypersingular operator on the dual mesh (integration-by-parts form)
 * and Mt the lumped dual mass matrix (Sec. 4).
 *
 * Conventions
 *   - Gamma_h: closed counter-clockwise polygon, segment i = [x_i, x_{i+1}],
 *     outward normal (e_y, -e_x).  P1 node n is vertex x_n.  Dual node i is the
 *     midpoint of segment i.
 *   - Time elements tau_m = (t_m, t_{m+1}], m = 0..n_t-1, t_0 = 0.
 *   - DOF order is time-major: l = m * n_bnd + i.  All vectors have
 *     N = n_bnd * n_t entries (u0 has n_vtx entries) and are float64.
 *   - V_h, K_h, D_h (and their alpha-derivatives) are causal: block (k, m) of
 *     size n_bnd x n_bnd vanishes for m > k (Sec. 3, block lower triangular).
 *     They are stored packed: block (k, m), k >= m, at element offset
 *     (k (k+1)/2 + m) * n_bnd^2, row-major (row = test index i).
 *   - M_h^0 is stored dense, row-major N x n_vtx.
 *   - Pointers named *_dev are device pointers owned by the caller; host
 *     inputs of stbem_create are copied.  `stream` is a hipStream_t (NULL =
 *     the null stream); every call is stream-ordered unless stated.
 *
 * Errors: 0 on success, negative STBEM_E* on failure (nothing is changed),
 * positive STBEM_WARN_* when a result was produced with a caveat.
 * stbem_last_error() describes the last failure of a context.  No call
 * throws or aborts.  A context is not thread-safe; use one per stream.
 */
#ifndef STBEM_H
#define STBEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stbem_ctx stbem_ctx;

/* error codes */
#define STBEM_OK 0
#define STBEM_EINVAL (-1)         /* bad argument (null pointer, size, flag) */
#define STBEM_EMESH (-2)          /* polygon not closed/CCW, zero-length segment, bad triangle */
#define STBEM_EALPHA (-3)         /* alpha <= 0 or not finite */
#define STBEM_ETIME (-4)          /* time nodes not strictly increasing from 0 */
#define STBEM_ENOMEM (-5)         /* device allocation failed */
#define STBEM_ENOTASSEMBLED (-6)  /* operator used before stbem_assemble */
#define STBEM_EHIP (-7)           /* HIP runtime error (message in stbem_last_error) */
#define STBEM_WARN_NOT_CONVERGED 1
#define STBEM_WARN_IR_STAGNATION 2

/* operators (bit mask for stbem_assemble, single value elsewhere) */
#define STBEM_V 1u      /* single layer V_h                    (eq. 4) */
#define STBEM_K 2u      /* double layer K_h                    (eq. 4) */
#define STBEM_D 4u      /* hypersingular D_h on the dual mesh  (Sec. 2) */
#define STBEM_M0 8u     /* initial potential M_h^0             (eq. 4) */
#define STBEM_DV 16u    /* dV_h / d alpha */
#define STBEM_DK 32u    /* dK_h / d alpha */
#define STBEM_DM0 64u   /* dM_h^0 / d alpha */

/* storage precision of V_h and D_h for the refinement solve */
#define STBEM_FP64 0
#define STBEM_FP32_IR 1

typedef struct {
    double alpha;              /* heat capacity constant, > 0              (eq. 1) */
    int n_t;                   /* number of time elements                          */
    const double* t_nodes;     /* host, n_t + 1 nodes, t_0 = 0 < t_1 < ... = T     */
    int n_bnd;                 /* number of boundary segments (>= 3)               */
    const double* bnd_xy;      /* host, 2 * n_bnd: CCW polygon vertices (x, y)      */
    int n_vtx;                 /* vertices of Omega_h (0: no M_h^0)                */
    const double* vtx_xy;      /* host, 2 * n_vtx                                  */
    int n_tri;                 /* triangles of Omega_h                             */
    const int* tri;            /* host, 3 * n_tri vertex indices, CCW              */
} stbem_problem;

/* Validate the problem, copy it to the device and build quadrature tables. */
int stbem_create(const stbem_problem* prob, stbem_ctx** out);
/* Free everything the context owns. Null is accepted. */
int stbem_destroy(stbem_ctx* ctx);
const char* stbem_last_error(const stbem_ctx* ctx);

/* Device memory for the matrices: if set, the context obtains and returns
 * its matrix storage through these callbacks (e.g. a framework's caching
 * allocator); otherwise it uses hipMalloc/hipFree. */
typedef void* (*stbem_alloc_fn)(size_t bytes, void* user);
typedef void (*stbem_free_fn)(void* ptr, void* user);
int stbem_set_allocator(stbem_ctx* ctx, stbem_alloc_fn alloc, stbem_free_fn release, void* user);

/* Sizes: N, n_bnd, n_t, n_vtx, entries of one packed causal matrix. */
int stbem_sizes(const stbem_ctx* ctx, long long* n, int* n_bnd, int* n_t, int* n_vtx, long long* packed_entries);

/* Assemble the operators in `mask` (STBEM_V | ...) of eq.(4) and, for
 * STBEM_D, of Theorem 1 (Sec. 2) into context storage.  Every entry is an
 * exact-in-time (E1 closed form / Laguerre series) and fixed-rule-in-space
 * Galerkin integral computed in FP64; blocks with tau_m after tau_k are never
 * computed (Sec. 3, block lower triangular).
 * precision = STBEM_FP64: FP64 storage (8 bytes per entry).
 * precision = STBEM_FP32_IR: only STBEM_V and STBEM_D may be in `mask` (else
 *   STBEM_EINVAL; also refused in block-Toeplitz mode).  V_h is stored as the
 *   float pair hi = fl32(V), lo = fl32(V - hi) (about 48 bits together), D_h
 *   as float (D_h only shapes the preconditioner; its separated time blocks
 *   are computed in FP32 arithmetic with one Gauss point fewer per direction
 *   than in FP64, within about 3e-7 of the block maximum); 12 bytes per entry
 *   pair instead of 16.  The FP64 storage of these operators is freed, and
 *   operators that need FP64 V_h or D_h (FP64 solves) are unavailable until
 *   they are assembled again in FP64.
 * Re-assembling an operator replaces its storage; assembling V_h or D_h in
 * FP64 drops FP32 copies made from the previous FP64 storage.  Allocation
 * failure returns STBEM_ENOMEM (the storage of the failed operator is not
 * kept). */
int stbem_assemble(stbem_ctx* ctx, unsigned mask, int precision, void* stream);

/* Free the storage of the operators in `mask` (for STBEM_V / STBEM_D also
 * their FP32 storage), e.g. K_h and M_h^0 once the right-hand side is formed.
 * Synchronisation is the caller's: no kernel may still use that storage. */
int stbem_release(stbem_ctx* ctx, unsigned mask);

/* Device pointer and size in bytes of an assembled operator's FP64 storage
 * (op is one of STBEM_V ... STBEM_DM0); owned by the context.
 * STBEM_ENOTASSEMBLED if the operator has no FP64 storage. */
int stbem_matrix(stbem_ctx* ctx, unsigned op, const double** dev_ptr, size_t* bytes);

/* FP32 storage of V_h (hi and lo; lo is NULL when the FP32 copy was made from
 * a resident FP64 V_h by stbem_prepare_ir) or D_h (hi only, lo = NULL),
 * same packed layout as the FP64 storage; bytes = size of one float array.
 * Owned by the context.  STBEM_ENOTASSEMBLED if there is none. */
int stbem_matrix_f32(stbem_ctx* ctx, unsigned op, const float** hi_dev, const float** lo_dev, size_t* bytes);

/* y = A x (trans = 0) or y = A^T x (trans = 1) for an assembled operator
 * (STBEM_V, STBEM_K, STBEM_D, STBEM_DV, STBEM_DK: N-vectors;
 *  STBEM_M0, STBEM_DM0: x has n_vtx entries for trans = 0, N for trans = 1).
 * FP64 storage is used when present; V_h held only in FP32 storage is applied
 * as hi + lo with FP64 accumulation, D_h held only in FP32 as float.
 * x and y must not overlap.  The matrix-vector product streams every stored
 * entry once and adds partial sums in a fixed order (bitwise reproducible). */
int stbem_apply(stbem_ctx* ctx, unsigned op, int trans, const double* x_dev, double* y_dev, void* stream);

/* For callers that cannot allocate device memory (work under HIP stream or
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * y = A x (trans = 0) or A^T x (trans = 1) like stbem_apply, for the causal
 * operators STBEM_V, STBEM_K, STBEM_D, STBEM_DV, STBEM_DK in packed storage
 * (FP64, or the FP32 storage of V_h / D_h), with no device allocation or
 * free and no host synchronisation.  The partial sums go to a fixed device
 * buffer of STBEM_NOALLOC_SCRATCH_BYTES owned by the library: one per GPU,
 * held from the first stbem_create on that GPU until the process ends.
 * The block rows are processed in ranges whose partials fit that buffer;
 * one block row must fit, so n_t * n_bnd <= STBEM_NOALLOC_SCRATCH_BYTES / 8
 * (4194304), else STBEM_EINVAL.  trans = 0 gives bitwise the y of
 * stbem_apply; trans = 1 too when all partials fit one range
 * (n_t (n_t + 1) / 2 * n_bnd <= 4194304), otherwise the same sums added in
 * another order.  STBEM_EINVAL for STBEM_M0 / STBEM_DM0 and in block-Toeplitz
 * mode.  Every call on a GPU uses that GPU's one buffer, which keeps the last
 * call's contents: calls that overlap in time on one GPU (other streams,
 * other host threads, other contexts) race and give wrong results; calls
 * ordered on one stream are safe.  x and y must not overlap. */
#define STBEM_NOALLOC_SCRATCH_BYTES (32LL << 20)
int stbem_apply_noalloc(stbem_ctx* ctx, unsigned op, int trans, const double* x_dev, double* y_dev, void* stream);

/* M_h g for g in X_h^{1,0} (trans = 0) or M_h^T x (trans = 1). */
int stbem_mass(stbem_ctx* ctx, int trans, const double* x_dev, double* y_dev, void* stream);

/* Preconditioner of Theorem 1 (Sec. 2) with the lumped mass of Sec. 4:
 * z = Mt^{-1} D_h Mt^{-1} r (trans = 1: D_h^T), Mt[(m,i)] = h_m (L_{i-1} +
 * 2 L_i + L_{i+1})/4 the row sums of the dual-primal mass matrix.  Needs
 * STBEM_D (FP64 storage, else FP32 storage).  r and z are N-vectors that must
 * not overlap.  Stream-ordered; uses work vectors kept by the context. */
int stbem_precondition(stbem_ctx* ctx, int trans, const double* r_dev, double* z_dev, void* stream);

/* Right-hand side of eq.(4): f = (1/2 M_h + K_h) g - M_h^0 u0.
 * Needs STBEM_K; u0_dev may be NULL (u0 = 0).  If STBEM_M0 is not assembled,
 * M_h^0 u0 is computed in row chunks without storing M_h^0 (for meshes where
 * the N x n_vtx matrix does not fit); the result is the same product. */
int stbem_rhs(stbem_ctx* ctx, const double* g_dev, const double* u0_dev, double* f_dev, void* stream);

/* Adjoint of the right-hand side operator of eq.(4) in g:
 * out = (1/2 M_h + K_h)^T lam, the gradient of a functional J(w) in the
 * Dirichlet data g when lam solves V_h^T lam = dJ/dw.  Needs STBEM_K.
 * lam and out are N-vectors (device) that must not overlap. */
int stbem_rhs_adjoint(stbem_ctx* ctx, const double* lam_dev, double* out_dev, void* stream);

/* FP32 copies for the refinement solve from resident FP64 storage: V_h as
 * float hi = fl32(V) (the outer residual then reads the FP64 V_h) and D_h as
 * float.  Nothing is done for an operator that already has FP32 storage.
 * stbem_solve calls it on first use of STBEM_FP32_IR.  Needs STBEM_V. */
int stbem_prepare_ir(stbem_ctx* ctx, void* stream);

typedef struct {
    double tol;        /* stop when ||C (f - A w)|| <= tol ||C f|| (C: preconditioner) */
    int max_it;        /* GMRES iterations (no restart); inner iterations for IR    */
    int mode;          /* STBEM_FP64 or STBEM_FP32_IR                             */
    int trans;         /* 1: solve V_h^T w = f (adjoint), preconditioned with D_h^T */
    int precondition;  /* 0: plain GMRES                                          */
    double inner_tol;  /* IR: relative tolerance of each inner FP32 solve         */
    int max_outer;     /* IR: outer refinement steps                              */
    double ir_tol;     /* IR: stop when ||f - V w|| <= ir_tol ||f|| (FP64 residual) */
} stbem_solve_opts;

typedef struct {
    int iters;             /* GMRES iterations (IR: summed over inner solves)      */
    int outer;             /* IR outer steps                                      */
    double relres;         /* final preconditioned relative residual estimate     */
    double true_relres;    /* ||f - V w|| / ||f|| at the end, FP64 accumulation
                              with the FP64 V_h (or hi + lo if V_h is FP32 only) */
} stbem_solve_info;

/* Solve the Galerkin system eq.(4), V_h w = f (or V_h^T w = f for an
 * adjoint), with GMRES left-preconditioned by C_V^{-1} = Mt^{-1} D_h Mt^{-1}
 * (Sec. 2, Theorem 1 and the lumped mass of Sec. 4): x0 = 0, no restart,
 * classical Gram-Schmidt twice, Givens rotations; stops when
 * ||C (f - V w)|| <= tol ||C f|| (Sec. 4 solves to a relative precision).
 * STBEM_FP64 needs FP64 V_h (and D_h when preconditioned).
 * STBEM_FP32_IR (iterative refinement): r = f - V w in FP64 accumulation
 * with the FP64 V_h if resident, else with the pair hi + lo; inner
 * preconditioned GMRES to inner_tol on float V_h (hi) and float D_h with the
 * Krylov basis and its orthogonalisation in float64; w += correction; stops
 * when ||r|| <= ir_tol ||f||.  Missing FP32 copies are made from FP64
 * storage (stbem_prepare_ir).
 * f and w are N-vectors that must not overlap.  Synchronises the stream.
 * Returns STBEM_WARN_NOT_CONVERGED if tol was not reached (w holds the last
 * iterate), STBEM_WARN_IR_STAGNATION if an outer step did not halve the
 * residual. */
int stbem_solve(stbem_ctx* ctx, const double* f_dev, double* w_dev, const stbem_solve_opts* opts,
                stbem_solve_info* info, void* stream);

/* d J / d alpha contribution lambda^T (dK_h g - dM_h^0 u0 - dV_h w) for an
 * adjoint state lambda (from a trans = 1 solve): the alpha-derivative of
 * eq.(4), V_h w = (1/2 M_h + K_h) g - M_h^0 u0, with M_h independent of
 * alpha.  Each of dV_h w, dK_h g and dM_h^0 u0 (u0_dev may be NULL: no
 * initial term) uses the stored matrix when STBEM_DV / STBEM_DK / STBEM_DM0
 * is assembled; otherwise it is recomputed without storing the matrix:
 * ranges of block rows are assembled into a buffer of at most 1 GiB (at
 * least one block row) by the same kernels and contracted at once, M_h^0's
 * derivative in row chunks.  Results agree with the stored path to
 * rounding.  Not available in block-Toeplitz mode without the stored
 * matrices (STBEM_ENOTASSEMBLED).  Synchronises the stream on the recomputed
 * path.  The scalar is written to out_dev[0] (device).  */
int stbem_grad_alpha(stbem_ctx* ctx, const double* lambda_dev, const double* w_dev, const double* g_dev,
                     const double* u0_dev, double* out_dev, void* stream);

/* Sampled entries A[(k,i),(m,j)] of V/K/D/dV/dK (eq.(4); Theorem 1)
 * computed directly by the assembly kernels' device code (idx_dev: n
 * quadruples (k, m, i, j) as int32; out_dev: n).  An entry above the block
 * diagonal (k < m) is 0; a quadruple outside the matrix (an index < 0,
 * k or m >= n_t, i or j >= n_bnd) gives NaN. */
int stbem_entries(stbem_ctx* ctx, unsigned op, long long n, const int* idx_dev, double* out_dev, void* stream);

/* The representation formula (Sec. 1, eq. (2)) at n points of Q:
 *   u(x, t) = (M~0 u0)(x, t) + (V~ w)(x, t) - (W g)(x, t)
 * for the discrete data w (X_h^{0,0} coefficients, e.g. a solution of
 * stbem_solve), g (nodal x time element) and u0 (nodal, may be NULL: u0 = 0).
 * pts_dev: n triples (x, y, t), x strictly inside the polygon, 0 < t <= T
 * (checked on the host: the points are copied back, the stream is
 * synchronised; STBEM_EINVAL otherwise).  out_dev: n triples (M~0 u0,
 * V~ w, W g), so u = out0 + out1 - out2.  The time integrals are closed
 * forms in E1 and exp; space integrals use Gauss rules on pieces graded
 * towards the foot of the point (boundary) and on regularly refined
 * triangles (initial potential). */
int stbem_potential(stbem_ctx* ctx, long long n, const double* pts_dev, const double* w_dev, const double* g_dev,
                    const double* u0_dev, double* out_dev, void* stream);

/* Block-Toeplitz storage for uniform time steps (on = 1).  With equal steps
 * the block (k, m) of V_h, K_h, D_h and their alpha-derivatives depends on
 * k - m only (the time integrals depend on the lags), so only the N_I blocks
 * (d, 0), d = 0..N_I-1, are assembled and stored: block d at element offset
 * d * n_bnd^2, row-major; products are sum over lags of one GEMM each
 * (rocBLAS).  Returns STBEM_EINVAL if the steps differ by more than 1e-12
 * relative.  Switching frees the assembled causal operators (and the FP32
 * copies) after a device synchronisation; they must be assembled again.
 * The FP32 refinement needs packed storage and is refused in this mode.
 * stbem_sizes still reports the packed size; stbem_matrix reports the
 * stored bytes. */
int stbem_set_toeplitz(stbem_ctx* ctx, int on);

/* Launch timing, for measuring kernels in place.  With on = 1 every launch
 * of the assembly kernels and of the matrix-vector kernels is bracketed by
 * HIP events recorded on the stream it runs on (a few microseconds of host
 * work per launch); on = 0 stops.  Either call first waits for and drops the
 * records taken so far.  stbem_kernel_times sums the records per kernel name
 * (the names of the kernels in the library): launches, event time in ms, the
 * work units the launches processed (matrix entries for the V_h, K_h, D_h
 * kernels and the matrix-vector kernels, (row, triangle) pairs for the M_h^0
 * moment kernels, matrix entries for the M_h^0 gather) and, for the far-field
 * (series) assembly kernels, their algorithmic operation count: per node
 * pair of the Gauss rule a fixed setup and evaluation cost (with an
 * exponential counted as 29 operations) plus a fixed cost per series term,
 * times the terms of each block, plus the combination per entry.  It writes
 * at most `cap` records to `out` (host) and returns the number of names, or
 * a negative error; it waits for the recorded events. */
typedef struct {
    char name[48];
    long long launches;
    double ms;
    double units;
    double flops;      /* algorithmic floating-point operations of the launches
                          (FMA = 2) from the library's operation count of the
                          series-based far-field kernels; 0 for other kernels */
} stbem_kernel_time;
int stbem_set_timing(stbem_ctx* ctx, int on);
int stbem_kernel_times(stbem_ctx* ctx, stbem_kernel_time* out, int cap);

#ifdef __cplusplus
}
#endif
#endif /* STBEM_H */
