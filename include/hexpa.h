/*
 * hexpa — partial-assembly (PA) action of high-order H1 mass and diffusion operators
 * on hexahedral meshes, and the CG solves that run on it, for AMD Instinct MI355X (gfx950).
 *
 * The operator is the decomposition A = P^T G^T B^T D B G P of the paper's eq. (1)
 * (Sec. II-B): G maps the global (L-)vector to element (E-)vectors through a DOF map,
 * B evaluates the tensor-product basis at quadrature points by sum factorization
 * (eq. (2)), and D is the block-diagonal quadrature-point data that partial assembly
 * precomputes and stores.  On one device P = I.
 *
 * Conventions shared by every call
 *  - reference element [0,1]^3; local node I = i + d*j + d*d*k with d = p+1 (i fastest);
 *    nodes are Gauss-Lobatto-Legendre points; quadrature is q1d-point Gauss-Legendre per axis;
 *  - hex corner c = a + 2b + 4c' sits at reference vertex (a, b, c') (lexicographic);
 *  - quadrature point r = a + q1d*(b + q1d*c) (a fastest);
 *  - all vector arguments of pa_apply/pa_diag/pa_load/cg_solve are DEVICE pointers owned
 *    by the caller (e.g. torch tensors), FP64, length ndof unless stated;
 *    mesh/coefficient descriptors point to HOST memory, copied during pa_setup
 *    (the caller may free them afterwards);
 *  - `stream` is a hipStream_t (NULL = legacy default stream); calls marked
 *    "asynchronous" only enqueue work on it;
 *  - every int-returning call returns PA_OK (0) or a negative status; the message of the
 *    last failure on the calling thread is available from pa_last_error().  No C++
 *    exception crosses this interface.  Null pointers, sizes that do not match the
 *    operator, and unsupported (p, q1d) pairs are rejected before any launch.
 */
#ifndef HEXPA_H
#define HEXPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define PA_OK 0
#define PA_ERR_ARG (-1)           /* bad pointer, size or option */
#define PA_ERR_HIP (-2)           /* a HIP runtime call failed */
#define PA_ERR_UNSUPPORTED (-3)   /* (p, q1d, ops) combination not compiled in */
#define PA_ERR_MESH (-4)          /* an element has det J <= 0 at a quadrature point */
#define PA_ERR_NOT_CONVERGED (-5) /* solver hit max_it before the tolerance */
#define PA_ERR_BREAKDOWN (-6)     /* solver breakdown: p^T A p <= 0 or a non-finite scalar */
#define PA_ERR_IO (-7)            /* file read/write/format error */

/* ------------------------------------------------------------------ operator bits */
#define PA_MASS 1u      /* (kappa u, v)               D = w kappa det J            (1 value / qp) */
#define PA_DIFFUSION 2u /* (kappa grad u, grad v)     D = w kappa adj(J) adj(J)^T / det J
                           (symmetric 3x3, 6 values / qp, order 00,01,02,11,12,22) */

/* ------------------------------------------------------------------ descriptors */
typedef struct {
    int32_t nvert;
    const double *vert_xyz; /* host [nvert][3] vertex coordinates */
    int32_t nelem;
    const int32_t *hex;     /* host [nelem][8] vertex indices, corner c = a + 2b + 4c' */
    /* Structured box: nx = ny = nz = n > 0 means elements are ordered e = ex + n*(ey + n*ez)
       and the library numbers DOFs on the (n p + 1)^3 lattice: node (ex p + i, ey p + j, ez p + k)
       gets index I + M*(J + M*K), M = n p + 1.  Otherwise (0,0,0) and elem_dofs is required. */
    int32_t nx, ny, nz;
    const int32_t *elem_dofs; /* optional host [nelem][(p+1)^3] DOF map (used when nx == 0) */
    int32_t ndof;             /* number of DOFs when elem_dofs is given; ignored for boxes */
    /* Essential (Dirichlet) DOFs: ess_mode 0 = none, 1 = all DOFs on the box boundary
       (structured boxes only), 2 = ess_marker[ndof] (host, nonzero = essential). */
    int32_t ess_mode;
    const uint8_t *ess_marker;
} pa_mesh_desc;

#define PA_COEFF_CONST 0 /* kappa = value */
#define PA_COEFF_SINE 1  /* kappa = value + amp sin(freq pi x) sin(freq pi y) sin(freq pi z) */
#define PA_COEFF_GRID 2  /* kappa = trilinear interpolation of grid[gz][gy][gx] (x fastest)
                            on [0,1]^3, clamped to the cube */
typedef struct {
    int32_t kind;
    double value, amp, freq;
    const double *grid; /* host */
    int32_t gx, gy, gz;
} pa_coeff_desc;

/* Apply-kernel variants (pa_set_variant).  pa_setup selects the faster contraction unit
   measured on MI355X for the order and operator: VALU for p <= 4 and for the mass operator
   alone up to p = 6, MFMA otherwise. */
#define PA_VARIANT_MFMA 0    /* fused kernel, FP64 MFMA contractions, atomic scatter */
#define PA_VARIANT_VALU 1    /* fused kernel, FP64 vector-ALU contractions, atomic scatter */
#define PA_VARIANT_MFMA_COLORED 2 /* MFMA contractions, 8 colour launches, plain read-modify-write
                                     scatter: bitwise reproducible */
#define PA_VARIANT_MFMA_UNFUSED 3 /* unfused: forward contractions, D and transposed contractions
                                     as three kernels through an HBM buffer of the quadrature-point
                                     tensor (handle-owned, allocated on first use: nelem x
                                     (3 | 1 | 4) x Q^3 doubles); FP64 MFMA contractions */
#define PA_VARIANT_VALU_UNFUSED 4 /* the same with FP64 vector-ALU contractions */
#define PA_VARIANT_MFMA_MF 5      /* fused matrix-free: no stored D; the kernel recomputes D at each
                                     quadrature point from the element's vertices and the coefficient
                                     (the setup kernel's arithmetic); FP64 MFMA contractions */
#define PA_VARIANT_VALU_MF 6      /* the same with FP64 vector-ALU contractions */

typedef struct pa_op pa_op;

typedef struct {
    int32_t p, q1d, ops, nelem, ndof, ness, ncomp, variant;
    int32_t elems_per_block;   /* elements per element group of the selected variant's kernel */
    int32_t threads_per_block; /* its workgroup size */
    int64_t qdata_bytes; /* bytes of stored quadrature-point data D */
    int64_t map_bytes;   /* bytes of the DOF map G */
} pa_info_t;

/* ------------------------------------------------------------------ operator calls */

/* Build the PA operator (paper Sec. II-B: "precompute and store ... D at quadrature
   points").  Copies the mesh to the device, builds the DOF map G, the 1-D basis tables
   (values B and derivatives at the q1d Gauss points) and computes D in FP64 on the
   device.  order p in [1,8], q1d in {p+1, p+2}; ops = PA_MASS, PA_DIFFUSION or both
   (A = M + K).  Synchronous.  On success *out owns all device memory it allocated. */
int pa_setup(const pa_mesh_desc *mesh, int order, int q1d, const pa_coeff_desc *coeff,
             uint32_t ops, void *stream, pa_op **out);

/* y = A x (eq. (1) with P = I: gather G, contractions B, D at quadrature points,
   transposed contractions B^T, scatter-add G^T), one fused kernel.  y is overwritten.
   x and y must not alias.  Asynchronous. */
int pa_apply(pa_op *op, const double *x, double *y, void *stream);

/* y += A x: the same fused kernel without zeroing y first (one kernel launch; used to
   accumulate several operators into one vector and to time the kernel alone).
   x and y must not alias.  Asynchronous. */
int pa_apply_add(pa_op *op, const double *x, double *y, void *stream);

/* Mixed-precision apply, y = A x (unconstrained), for the inner solver of iterative
   refinement: x and y are device FP32 vectors [ndof]; the quadrature data is an FP32 copy
   of D (rounded once from FP64, made on first use); the element tiles and every
   intermediate of the sum-factorised contractions are rounded to FP16 (fmt = PA_LP_FP16)
   or BF16 (PA_LP_BF16) as they enter v_mfma_f32_16x16x16{f16,bf16}, which accumulates in
   FP32.  For the diffusion operator alone in BF16, each element tile is first centred on
   its mean (diffusion annihilates constants, so y is unchanged in exact arithmetic and the
   rounding acts on the deviation from the mean).  FP16 needs |x| well inside its range:
   callers scale x by a power of two.  y is overwritten.  Asynchronous. */
#define PA_LP_FP16 0
#define PA_LP_BF16 1
int pa_apply_lp(pa_op *op, const float *x, float *y, int fmt, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
   loops, harnesses that forbid hipMalloc): y = A x with the unfused apply (variant
   PA_VARIANT_MFMA_UNFUSED or PA_VARIANT_VALU_UNFUSED; forward contractions, D-step and
   transposed contractions as three kernels), whose quadrature-point tensor is staged in
   a fixed 128 MiB device array of the library (one per GPU, held until the process ends)
   instead of handle memory that pa_apply allocates on first use.  Allocates nothing.
   The tensor needs nelem x (1 | 3 | 4 for mass | diffusion | both) x q1d^3 doubles; a
   larger operator gets PA_ERR_ARG before any launch (at most 16 Mi doubles, e.g. 25,890
   elements of p = 4 diffusion with q1d = 6).  The operator's device must be current.
   Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
   streams or threads, any operator) race and must be serialised by the caller.  Each
   call writes every entry it reads before reading it, so nothing needs clearing
   between calls.  y is overwritten; x and y must not alias.  Asynchronous. */
int pa_apply_unfused_noalloc(pa_op *op, int variant, const double *x, double *y, void *stream);

/* y = A_c x with A_c = (I - E) A (I - E) + E, E = indicator of the essential DOFs.
   Uses handle-owned scratch; calls on one handle must not overlap.  Asynchronous. */
int pa_apply_constrained(pa_op *op, const double *x, double *y, void *stream);

/* d = diag(A) (constrained = 0) or diag(A_c) (constrained != 0: 1 on essential rows),
   computed by sum factorization over the stored D (three one-index contractions with the
   per-axis tables B^2, B G and G^2; 256-thread workgroups of one element at high order
   and up to sixteen at low order).  Asynchronous. */
int pa_diag(pa_op *op, double *d, int constrained, void *stream);

/* Load vector b = G^T B^T (w det J f): f given at quadrature points, device
   [nelem][q1d^3] in the quadrature-point order above; b overwritten.  Asynchronous. */
int pa_load(pa_op *op, const double *f_qp, double *b, void *stream);

/* Physical coordinates of the quadrature points, device out [nelem][q1d^3][3]. Asynchronous. */
int pa_qpoints(pa_op *op, double *xyz, void *stream);

/* Physical coordinates of the DOF nodes, device out [ndof][3].  Asynchronous. */
int pa_nodes(pa_op *op, double *xyz, void *stream);

/* Copy the DOF map G to host memory [nelem][(p+1)^3].  Synchronous. */
int pa_get_elem_dofs(pa_op *op, int32_t *host_out);

/* Copy the essential-DOF list to host memory [ness] (ascending).  Synchronous. */
int pa_get_ess(pa_op *op, int32_t *host_out);

/* Select the apply kernel (PA_VARIANT_*).  Takes effect for later calls. */
int pa_set_variant(pa_op *op, int variant);

/* Limit every apply launch on this handle to at most max_workgroups workgroups (0, the
   default, restores the persistent grid: the number of workgroups the device keeps
   resident, or fewer when the mesh has fewer element groups).  The apply kernels are
   persistent: each workgroup walks a strided list of element groups and prefetches the
   DOF map, x and D of its next group while it contracts the current one.  Large meshes
   always take that path; a cap lets a small mesh take it too (several groups per
   workgroup), which is what tests of that path use.  Results do not depend on the cap
   beyond the order of the atomic additions.  Takes effect for later calls. */
int pa_set_grid_cap(pa_op *op, int max_workgroups);

int pa_info(const pa_op *op, pa_info_t *info);
void pa_destroy(pa_op *op);
const char *pa_last_error(void);

/* ------------------------------------------------------------------ solver */
#define PA_CG_PLAIN 0      /* CG, no preconditioner */
#define PA_CG_JACOBI 1     /* Jacobi-preconditioned CG, M = diag(A_c) */
#define PA_CG_MIXED_IR 2   /* FP64 iterative refinement around an inner Jacobi-PCG that runs
                              in FP32 vectors with the 16-bit-MFMA apply (pa_apply_lp) */
#define PA_CG_FCG 3        /* flexible CG, FCG(1), preconditioned by a pa_lp handle (learned
                              network and/or p = 1 coarse correction); on breakdown it falls
                              back to Jacobi-PCG from the current iterate */
#define PA_CG_MIXED_FCG 4  /* FP64 flexible CG, FCG(1), whose preconditioner is the inner
                              mixed-precision solve of MIXED_IR (Jacobi-PCG on FP32 vectors
                              with the 16-bit-MFMA apply, inner_rtol / inner_max): the outer
                              recurrence keeps its direction instead of restarting */
#define PA_CG_MIXED_RU 5   /* one Jacobi-PCG recurrence on FP32 vectors with the 16-bit-MFMA
                              apply, never restarted; at most every inner_max iterations its
                              residual is replaced by the FP64 residual b - A x and the FP32
                              correction is added to x in FP64 (reliable updates); max_it
                              bounds the total iterations; iters reports the replacements */

typedef struct pa_lp pa_lp;

typedef struct {
    double rtol;         /* stop when ||r_k||_2 <= rtol ||b||_2 (recursive residual; for
                            MIXED_IR the FP64 residual recomputed every outer step) */
    int32_t max_it;      /* iterations (MIXED_IR: outer refinement steps) */
    int32_t mode;        /* PA_CG_* */
    int32_t check_every; /* read the residual norm back to the host every k iterations (>=1) */
    int32_t constrained; /* 1: solve with A_c; the essential entries of x are set to b's */
    int32_t lp_fmt;      /* MIXED_IR: PA_LP_FP16 or PA_LP_BF16 */
    int32_t inner_max;   /* MIXED_IR: inner iterations per refinement step */
    double inner_rtol;   /* MIXED_IR: inner relative tolerance per refinement step */
    pa_lp *lp;           /* FCG: the preconditioner, bound to this operator */
    int32_t n_capture;   /* JACOBI, FCG: number of iterates to record (0: none) */
    int32_t pad_;
    const int32_t *capture_at; /* host [n_capture] ascending iteration numbers k >= 0 */
    double *capture_x;         /* device [n_capture][ndof]; receives x_k when iteration k ends
                                  (k = 0: the initial guess); rows of iterations not reached
                                  are left untouched */
} pa_cg_opts;

typedef struct {
    int32_t iters, status;
    double rel_res_recursive; /* ||r_k|| / ||b|| at exit (recursion; MIXED_IR: FP64 residual) */
    double rel_res_true;      /* ||b - A x|| / ||b|| recomputed in FP64 at exit */
    double seconds;           /* wall time of the iteration (excludes diag and setup) */
    int32_t inner_iters_total; /* MIXED_IR: inner PCG iterations over all refinement steps */
    int32_t fallback;          /* FCG: 1 if it broke down and finished as Jacobi-PCG */
} pa_cg_result;

/* Solve A x = b (or A_c x = b) by (preconditioned) CG (Saad, Alg. 9.1), all vector work
   and reductions in FP64 on the device; or, with PA_CG_MIXED_IR, by iterative refinement:
   r = b - A x in FP64, an inner Jacobi-PCG on the scaled residual in FP32 vectors with
   pa_apply_lp and FP64 dot products, x += correction in FP64.  x is the initial guess on entry and the
   solution on exit.  Synchronous on `stream`.  Returns PA_OK, PA_ERR_NOT_CONVERGED
   (x holds the last iterate) or PA_ERR_BREAKDOWN. */
int cg_solve(pa_op *op, const double *b, double *x, const pa_cg_opts *opts,
             pa_cg_result *res, void *stream);

/* ------------------------------------------------------------------ learned preconditioner
   Two-level preconditioner for FCG on a structured box with diffusion (p + 1 in {3, 4, 5}):
       z = J r + W G^T NN(G r) + P1 A1^{-1} P1^T r,   then z = 0 on the essential DOFs,
   with J = diag(A_c)^{-1} (Jacobi): the network learns a correction to Jacobi, so an
   untrained network (zero output layer, the default initialisation) gives Jacobi plus
   the coarse correction.
   NN: per element, a 3-layer convolutional network on the (p+1)^3 nodal tile
   (3x3x3 cross-correlation, zero padding, bias; 2 -> 16 -> 16 -> 1 channels, ReLU between
   layers) whose input channels are G_e r / s_e (s_e = RMS of G_e r over the tile) and
   log kappa at the nodes, and whose output is multiplied by s_e, so the map is positively
   1-homogeneous in r (exactly so in FP32 for power-of-two scalings).  W = 1 / (number of
   elements sharing a DOF): element outputs are averaged.  P1 = nodal interpolation from the p = 1 space on the same mesh, A1 = the p = 1
   operator (same coefficient and operator bits, 3-point Gauss), constrained on the box
   boundary; A1^{-1} is a fixed number of Jacobi-PCG iterations from 0 on A1's 27-point
   stencil.  Parameters are FP32; training runs the network in FP32; inference runs it in
   FP32 or in FP16 with FP32 accumulation (infer_fp16); vectors are FP64.
   Parameters: flat FP32 array W1 [16][2][27], b1 [16], W2 [16][16][27], b2 [16],
   W3 [1][16][27], b3 [1] with tap = tx + 3 ty + 9 tz for the neighbour
   (i + tx - 1, j + ty - 1, k + tz - 1) of local node (i, j, k). */
#define PA_LP_LOSS_ENERGY 0 /* L = (z - t)^T A_c (z - t) / t^T A_c t */
#define PA_LP_LOSS_L2 1     /* L = ||z - t||^2 / ||t||^2 (free DOFs) */
typedef struct {
    int32_t use_net;      /* 1: add the network's correction to Jacobi; 0: Jacobi only */
    int32_t use_coarse;   /* 1: add the p = 1 coarse correction */
    int32_t coarse_iters; /* Jacobi-PCG iterations of the coarse solve, >= 1 */
    int32_t loss;         /* PA_LP_LOSS_* */
    int32_t seed;         /* seed of the default (He-normal) parameter initialisation */
    int32_t infer_fp16;   /* 1: apply the network with FP16 MFMA (FP32 accumulation) in one
                             fused kernel; 0: FP32 vector-ALU kernels (training always uses FP32) */
    double lr;            /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
    double net_scale;     /* factor on the network's correction when the preconditioner is
                             applied (a damping, like omega of damped Jacobi); training
                             always uses 1.  Values <= 0 mean 1. */
} pa_lp_opts;

/* Create a preconditioner bound to op (which must outlive the binding): builds the coarse
   operator and its stencil, the log-kappa tiles and the DOF multiplicities.  Synchronous. */
int pa_lp_create(pa_op *op, const pa_lp_opts *opts, pa_lp **out);
/* Re-bind to another operator with the same box, order and essential DOFs (a new
   coefficient draw): rebuilds every operator-dependent array, keeps the parameters and
   the Adam state.  Synchronous. */
int pa_lp_bind(pa_lp *lp, pa_op *op);
/* Change use_net, use_coarse, coarse_iters, loss and lr (seed is ignored). */
int pa_lp_configure(pa_lp *lp, const pa_lp_opts *opts);
int pa_lp_num_params(void);
/* Copy the n = pa_lp_num_params() parameters to/from host memory; set also resets the
   Adam moments and step counter.  Synchronous. */
int pa_lp_get_params(pa_lp *lp, float *host, int n);
int pa_lp_set_params(pa_lp *lp, const float *host, int n);
/* The network's log-kappa input, device [nelem][(p+1)^3] FP32.  Asynchronous. */
int pa_lp_logk(pa_lp *lp, float *dev_out);
/* z = M(r) (the full preconditioner above), device FP64 [ndof]; r must vanish on the
   essential DOFs.  Uses handle-owned work arrays: calls on one handle must not overlap.
   Asynchronous. */
int pa_lp_apply(pa_lp *lp, const double *r, double *z, void *stream);
/* z = P1 A1^{-1} P1^T r only (zero on the essential DOFs).  Asynchronous. */
int pa_lp_coarse(pa_lp *lp, const double *r, double *z, void *stream);
/* z = W G^T NN(G r) only, the network's correction (zero on the essential DOFs).
   Asynchronous. */
int pa_lp_net(pa_lp *lp, const double *r, double *z, void *stream);
/* Loss of the network part z_NN(r) against target t (device, zero on essential DOFs)
   and its gradient w.r.t. the parameters, written to grad_host [n] if not NULL (the
   handle's gradient buffer is overwritten).  Synchronous; *loss receives L. */
int pa_lp_loss_grad(pa_lp *lp, const double *r, const double *t, double *loss, float *grad_host, void *stream);
/* One training step on the pair from iterate xk of A_c x = b with known solution xstar:
   r = b - A_c xk, e = xstar - xk, target t = e - J r - (coarse part of M)(r) (the last
   term when the coarse correction is on); then loss, gradient and one Adam update.  If loss is not
   NULL the call synchronises and stores L.  Asynchronous otherwise. */
int pa_lp_train_step(pa_lp *lp, const double *b, const double *xstar, const double *xk, double *loss,
                     void *stream);
/* Training over a set of systems (the epoch and draw loop of the training phase).  For
   each epoch and each draw d: bind the handle to ops[d] (same box, order and essential
   DOFs as the handle's operator: coefficient draws), form b = A_c x*_d, solve A_c x = b
   from x = 0 to 1e-10 (or capture_at[n_capture-1] + 1 iterations) by FCG preconditioned
   by the handle as it currently is (PA_LP_CAPTURE_FCG) or by FP64 Jacobi-PCG
   (PA_LP_CAPTURE_JACOBI), recording the iterates x_k at k in capture_at, then run one
   pa_lp_train_step per recorded iterate, in an order shuffled by a counter-based generator
   seeded from (seed, epoch, draw).  Device buffers of size (n_capture + 2) ndof doubles are
   allocated for the call.  The handle stays bound to the last operator.  Synchronous on
   `stream`. */
#define PA_LP_CAPTURE_FCG 0
#define PA_LP_CAPTURE_JACOBI 1
typedef struct {
    int32_t ndraws;
    int32_t capture;            /* PA_LP_CAPTURE_* */
    pa_op *const *ops;          /* host [ndraws] operators (not owned) */
    const double *const *xstar; /* host [ndraws] DEVICE pointers [ndof]: the known solutions */
    const int32_t *capture_at;  /* host [n_capture] ascending iteration numbers >= 0 (0: x = 0) */
    int32_t n_capture;
    int32_t epochs;             /* passes over the draws, >= 1 */
    uint32_t seed;
    int32_t pad_;
} pa_train_set;
typedef struct {
    int32_t steps;          /* training steps taken */
    int32_t max_steps;      /* capacity of loss (0: losses not recorded) */
    double *loss;           /* host [max_steps]: the loss of each step, in order */
    double seconds_capture; /* wall time of binding, right-hand sides and capture solves */
    double seconds_train;   /* wall time of the training steps */
} pa_train_log;
int pa_lp_train(pa_lp *lp, const pa_train_set *set, pa_train_log *log, void *stream);
/* Parameters to/from a file: magic "HEXPALP1", int32 version 1, int32 count, the FP32
   values, and a 64-bit FNV-1a checksum of them.  PA_ERR_IO on any mismatch. */
int pa_lp_save(pa_lp *lp, const char *path);
int pa_lp_load(pa_lp *lp, const char *path);
void pa_lp_destroy(pa_lp *lp);

/* ------------------------------------------------------------------ the paper's operator
   The off-diagonal blocks of the acoustic-gravity block operator (Sec. II-C, eq. (4)):
   pressure p in the continuous order-p space (GLL nodes; DOF map and numbering as for
   pa_setup on a structured box), velocity u in the discontinuous order-pu space (Lagrange
   basis on the pu+1 Gauss-Legendre points per axis, three scalar components, stored
   element by element: u[e][c][J], J = j1 + du (j2 + du j3), du = pu + 1), q1d-point Gauss
   rule.  With the quadrature-point data E_cm = w adj(J)_mc (9 values per point, stored
   FP64 [nelem][9][q1d^3]):
       G p   = (grad p, tau)  (velocity space),
       G^T u = (u, grad v)    (pressure space).
   Supported (p, pu, q1d): (4, 3, 5), the paper's discretisation, and (2, 1, 3). */
typedef struct pa_mixed pa_mixed;
typedef struct {
    int32_t p, pu, q1d;
    int32_t pad_;
    double rho;  /* density: velocity mass (rho u, tau) */
    double bulk; /* bulk modulus K: pressure mass (K^{-1} p, v) */
} pa_mixed_desc;
typedef struct {
    int32_t p, pu, q1d, nelem;
    int32_t ndof_p;          /* pressure DOFs ((n p + 1)^3 on an n^3 box) */
    int32_t ndof_u;          /* velocity DOFs, nelem * 3 * (pu+1)^3 */
    int32_t elems_per_block; /* elements per workgroup of the fused kernel */
    int32_t pad_;
    int64_t qdata_bytes;
} pa_mixed_info_t;
/* Build the operator on a structured box (mesh->nx = ny = nz > 0; elem_dofs and ess_mode
   are ignored): DOF map, 1-D tables of both spaces and E_cm on the device.  PA_ERR_MESH if
   det J <= 0 at a quadrature point.  Synchronous. */
int pa_mixed_setup(const pa_mesh_desc *mesh, const pa_mixed_desc *desc, void *stream, pa_mixed **out);
/* yu = G p and yp = -G^T u in one fused kernel (Sec. III-G: D and D^T applied in the same
   kernel; the pressure scatter by atomics): device vectors u, yu [ndof_u], p, yp [ndof_p];
   outputs overwritten and not aliasing inputs.  Asynchronous. */
int pa_mixed_apply(pa_mixed *m, const double *u, const double *p, double *yu, double *yp, void *stream);
/* Row-sum lumped masses: mu [nelem][(pu+1)^3] = rho sum_q w detJ psi_J (the same for each
   velocity component), mp [ndof_p] = sum_e sum_q w detJ phi_I / bulk.  Asynchronous. */
int pa_mixed_lumped(pa_mixed *m, double *mu, double *mp, void *stream);
/* nsteps classical RK4 steps of the semi-discrete system with lumped masses (Sec. II-C,
   no boundary terms: u . n = 0 on the box): u' = -Mu^{-1} G p, p' = Mp^{-1} G^T u.  u and p
   (device) are advanced in place; four fused applies per step; handle-owned work vectors
   (allocated on first use).  Asynchronous. */
int pa_mixed_rk4(pa_mixed *m, double *u, double *p, double dt, int nsteps, void *stream);
/* As pa_set_grid_cap, for the fused mixed kernel (tests of the multi-group walk). */
int pa_mixed_set_grid_cap(pa_mixed *m, int max_workgroups);
int pa_mixed_info(const pa_mixed *m, pa_mixed_info_t *info);
void pa_mixed_destroy(pa_mixed *m);

/* ------------------------------------------------------------------ diagnostics */

/* One FP64 MFMA on the device, writing the raw accumulator so a test can pin which entry
   of the product each lane holds (the layout the apply kernels assume).  Device pointers.
   shape 16: v_mfma_f64_16x16x4f64 with A[16][4], B[4][16] row-major; lane l supplies
             A[l%16][l/16] and B[l/16][l%16]; writes Draw[4*l + v] (256 doubles).
   shape 4:  v_mfma_f64_4x4x4f64 (four 4x4x4 blocks) with A[4][4][4], B[4][4][4] (block,
             row, col); lane l supplies A[b][l&3][l>>4] and B[b][l>>4][l&3] with
             b = (l>>2)&3; writes Draw[l] (64 doubles).
   Returns PA_ERR_ARG for another shape. */
int pa_debug_mfma_f64(int shape, const double *A, const double *B, double *D, void *stream);

/* One v_mfma_f32_16x16x16f16 (bf16 = 0) or v_mfma_f32_16x16x16bf16_1k (bf16 != 0) on the
   device, with A[16][16], B[16][16] FP32 row-major device arrays rounded to the 16-bit
   format as they are loaded (round to nearest even); lane l supplies A[l%16][4(l/16)+t] and
   B[4(l/16)+t][l%16], t = 0..3.  Writes the raw FP32 accumulator Draw[4*l + v] (256 floats):
   the layout the mixed-precision apply assumes is Draw[4l+v] = (A B)[4(l/16)+v][l%16]. */
int pa_debug_mfma16(int bf16, const float *A, const float *B, float *D, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HEXPA_H */
