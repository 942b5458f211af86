/*
 * nps.h -- C ABI of the MI355X neural-preconditioned Poisson solver.
 *
 * The library solves the reduced pressure Poisson system A~ x~ = b~ of a
 * voxel grid whose cells are labelled fluid / air (Dirichlet, p = 0) / solid
 * (Neumann), with the NPSDO iteration (Alg. 1 of arXiv 2310.00177: steepest
 * descent on the network-preconditioned residual, A-orthogonalised against
 * the last n_ortho directions, exact line search) and the spatially-varying-
 * kernel network of Alg. 2 (CConv and Aff blocks of Sec. "Architecture",
 * extended to 3D) as the preconditioner.  The matrix is never formed: it is
 * implied by the labels (Sec. "Spatial Discretization").
 *
 * Conventions shared by every entry point
 *   - Grids are (nz, ny, nx) arrays, x fastest, row-major, no padding.
 *   - Labels are uint8: 0 FLUID, 1 AIR, 2 SOLID.  Cells outside the grid are
 *     solid.  Vectors are full-grid; entries outside fluid are ignored on
 *     input and written as zero on output (pad/unpad rule of Sec. "Neural
 *     Preconditioner").
 *   - Pointers ending in _d are device pointers (HBM of the current HIP
 *     device); pointers ending in _h are host pointers.  The caller owns every
 *     buffer; the library keeps no pointer after a call returns, except the
 *     device buffer handed to nps_net_create, which must outlive the net.
 *   - `stream` is a hipStream_t (0 = the null stream).  Calls enqueue work on
 *     it; nps_solve synchronises with it before returning, the parity hooks
 *     do not.
 *   - No solve-path call allocates device memory: scratch comes from the
 *     caller's workspace, sized by nps_workspace_bytes.  Its contents on
 *     entry do not matter (each call writes what it later reads), so one
 *     workspace may serve any sequence of calls on one stream.
 *   - Return value: NPS_OK (0), a soft status (> 0: outputs valid), or a
 *     hard error (< 0: outputs untouched).  nps_last_error() returns a
 *     thread-local message for the last failure.
 */
#ifndef NPS_H
#define NPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum nps_status {
    NPS_OK = 0,
    NPS_NOT_CONVERGED = 1,   /* max_iter reached: x holds the last iterate   */
    NPS_EINVAL = -1,         /* bad argument (null pointer, tol <= 0, ...)    */
    NPS_ESHAPE = -2,         /* a dimension not divisible by 2^(levels-1)     */
    NPS_ELABEL = -3,         /* a label outside {0, 1, 2}                     */
    NPS_ENOFLUID = -4,       /* no fluid cell                                 */
    NPS_ENONFINITE = -5,     /* NaN or Inf in b on a fluid cell               */
    NPS_EBREAKDOWN = -6,     /* d.Ad <= 0 or not finite: no descent direction */
    NPS_ENOMEM = -7,         /* workspace or device buffer too small          */
    NPS_EDEVICE = -8         /* a HIP runtime call failed                     */
};

enum nps_label { NPS_FLUID = 0, NPS_AIR = 1, NPS_SOLID = 2 };

/* Arithmetic of the network and the Krylov vectors.
 *   NPS_FP64        everything in double.
 *   NPS_FP32        network and Krylov vectors in float; dot products
 *                   accumulate in double; the exit test uses the true
 *                   residual b - A x evaluated in double.
 *   NPS_MIXED_BF16  network kernels generated on bf16 matrix cores with fp32
 *   NPS_MIXED_FP16  accumulation (fp16 for the _FP16 variant), Krylov vectors
 *                   in float, the solution accumulated in double and the
 *                   residual b - A x formed in double from it every
 *                   iteration.                                               */
enum nps_precision { NPS_FP64 = 0, NPS_FP32 = 1, NPS_MIXED_BF16 = 2, NPS_MIXED_FP16 = 3 };

/* Krylov method around the network preconditioner P (Sec. "Algorithm" and
 * the appendix comparing PCG variants).  All three take the literal residual
 * b - A x every iteration and apply P to r / ||r|| (P is linear in r).
 *   NPS_NPSDO  Alg. 1: d = P(r), A-orthogonalised against the last n_ortho
 *              directions, alpha = r.d / d.Ad (n_ortho = 0: steepest descent).
 *   NPS_PCG    preconditioned CG: d_k = s_k + beta d_(k-1), s = P(r),
 *              beta = r_k.s_k / r_(k-1).s_(k-1), alpha = r.s / d.Ad.
 *   NPS_FPCG   flexible PCG: beta = s_k.(r_k - r_(k-1)) / r_(k-1).s_(k-1),
 *              otherwise as NPS_PCG.
 * The two PCG forms keep one previous direction: they require n_ortho = 1. */
enum nps_method { NPS_NPSDO = 0, NPS_PCG = 1, NPS_FPCG = 2 };

typedef struct { int nz, ny, nx; } nps_dims;

typedef struct {
    double tol;          /* stop when ||b - A x||_2 < tol * ||b||_2 (> 0)             */
    int max_iter;        /* iteration cap (>= 0)                                      */
    int n_ortho;         /* directions to A-orthogonalise against, 0..4 (paper: 2);  *
                          * 1 for NPS_PCG and NPS_FPCG                                */
    int precision;       /* enum nps_precision                                        */
    int fixed_iters;     /* 1: run exactly max_iter iterations, no convergence test    */
    int method;          /* enum nps_method (0 = NPSDO)                               */
    int symmetric;       /* 1: precondition with P^T o P, the symmetric variant of    *
                          * the appendix on symmetry (kernels of every level are     *
                          * kept in the workspace; size it with                      *
                          * nps_solve_workspace_bytes)                               */
} nps_opts;

typedef struct {
    int iterations;              /* NPSDO iterations performed                        */
    int status;                  /* same code nps_solve returned                      */
    double rel_residual;         /* true ||b - A x|| / ||b|| at exit, in double       */
    double rel_residual_rec;     /* the iteration's own (recursive) residual estimate */
    int refinements;             /* true-residual recomputations performed (one per   *
                                  * iteration and one for x0: every precision forms   *
                                  * b - A x in double from the double iterate each    *
                                  * iteration, so the Krylov vectors never drift from *
                                  * the true residual and no restart is needed)       */
    int n_fluid;                 /* number of fluid cells                              */
    double t_setup_ms;           /* nps_solve: validation + setup on the stream (HIP  *
                                  * events), ms; 0 from the request server            */
    double t_iter_ms;            /* nps_solve: mean time per iteration after setup,   *
                                  * result copy-out included, ms                      */
} nps_info;

typedef struct nps_net nps_net;

/* Number of parameters of an L-level network: (2L-1) CConv blocks of
 * 27*81 weights + 27 biases and 2(L-1) Aff blocks of 81 weights + 1 bias
 * (25,174 at L = 6, the "~25k" of Sec. "Architecture"). */
size_t nps_param_count(int levels);

/* Device bytes nps_net_create needs for an L-level network. */
size_t nps_net_bytes(int levels);

/* Build a network from a float64 host blob of nps_param_count(levels)
 * entries, laid out (Alg. 2 block order):
 *   for l = 1..L   CConv_1^l: W[27][3][3][3][3], B[27]
 *   for l = 1..L-1 CConv_2^l: W, B
 *   for l = 1..L-1 Aff_1^l: Wbar[3][3][3][3], Bbar;  Aff_2^l: Wbar, Bbar
 * W[t][c][oz+1][oy+1][ox+1]: t = 9(az+1) + 3(ay+1) + (ax+1) is the kernel tap
 * applied to r(p + a), c the image channel, o the image-window offset.
 * levels must be 2..6.  The preprocessed weights are copied into dev_buf
 * (nps_net_bytes(levels) bytes, 256-byte aligned) on `stream`; the blob may
 * be freed on return.  *out is a host handle released by nps_net_destroy. */
int nps_net_create(const double* params_h, size_t n_params, int levels,
                   void* dev_buf_d, size_t dev_bytes, void* stream, nps_net** out);
void nps_net_destroy(nps_net* net);
int nps_net_levels(const nps_net* net);

/* Workspace bytes for nps_solve / nps_apply_precond at these dims (not the
 * symmetric variant).  0 on invalid arguments. */
size_t nps_workspace_bytes(nps_dims dims, int levels, int precision, int n_ortho);

/* Workspace bytes for nps_solve with exactly these options (any method,
 * symmetric or not).  0 on invalid arguments. */
size_t nps_solve_workspace_bytes(nps_dims dims, int levels, const nps_opts* opts);

/* Solve A~ x~ = b~ (Alg. 1 with the network of Alg. 2 as preconditioner).
 *   labels_d  uint8[nz*ny*nx]   cell labels.
 *   b_d       double[nz*ny*nx]  right-hand side (read on fluid cells only).
 *   x_d       double[nz*ny*nx]  solution, written on every cell (0 off fluid).
 *   x0 = 0.  Precondition: every fluid component touches an air cell
 *   (otherwise A~ is singular and the iteration reports NPS_EBREAKDOWN or
 *   NPS_NOT_CONVERGED).  b = 0 gives x = 0 after 0 iterations.
 *   On NPS_OK / NPS_NOT_CONVERGED, x_d and *info are valid.  On
 *   NPS_EBREAKDOWN x_d holds the last iterate.  The stream is synchronised. */
int nps_solve(const nps_net* net, const uint8_t* labels_d, nps_dims dims,
              const double* b_d, double* x_d, const nps_opts* opts, nps_info* info,
              void* ws_d, size_t ws_bytes, void* stream);

/* Parity hook: y = A x, the mixed-BC 7-point matrix of Sec. "Spatial
 * Discretization" (diagonal = number of fluid or air face neighbours,
 * -1 per fluid face neighbour, zero rows off fluid).  precision NPS_FP64:
 * x_d, y_d are double; NPS_FP32: float.  Not synchronised. */
int nps_apply_laplacian(const uint8_t* labels_d, nps_dims dims, const void* x_d, void* y_d,
                        int precision, void* stream);

/* Parity hook: d = P(I, r), one evaluation of the network (Alg. 2) with the
 * same kernels nps_solve uses.  precision NPS_FP64: r_d, d_d double; all
 * other precisions: float.  The workspace is sized by nps_workspace_bytes
 * with the same dims/levels/precision.  Not synchronised. */
int nps_apply_precond(const nps_net* net, const uint8_t* labels_d, nps_dims dims,
                      const void* r_d, void* d_d, int precision,
                      void* ws_d, size_t ws_bytes, void* stream);

/* nps_apply_precond without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same kernels and results as
 * nps_apply_precond; its scratch is a static device array of 128 MiB
 * (134,217,728 bytes) that each GPU the library runs on holds until the
 * process ends, so the call allocates nothing.  Grids whose network
 * evaluation needs more scratch than that (about 10 bytes per cell in FP32
 * and the mixed modes, 20 in FP64, plus the stored kernels of the coarse
 * levels: 224^3 fits in FP32, 160^3 in FP64, 256^3 does not) are rejected
 * with NPS_ENOMEM before any work is enqueued.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race; serialise them.  Not synchronised. */
int nps_apply_precond_noalloc(const nps_net* net, const uint8_t* labels_d, nps_dims dims,
                              const void* r_d, void* d_d, int precision, void* stream);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of solves of different grids.
 *
 * The server owns one device arena (hbm_budget bytes, allocated once by
 * nps_server_create) and up to max_slots streams.  nps_server_submit queues
 * a request (first in, first out) without copying it: labels_h and b_h are
 * borrowed and must stay valid and unchanged until nps_server_poll has
 * returned the request's result or the server is destroyed.  nps_server_step
 * never blocks: it admits queued requests while the arena has room for their
 * footprint (nps_server_request_bytes) and a slot is free (admission copies
 * the request's inputs into a pinned staging buffer, reused across requests
 * of one size, and sends them on the slot's stream), and advances every admitted
 * request by at most one NPSDO iteration on its own stream, so iterations of
 * different requests overlap on the device.  A finished request leaves its
 * slot and its arena space at once; nps_server_poll returns NPS_PENDING (2)
 * until its result is ready, then copies x (double, full grid) to x_h,
 * fills *info, *latency_ms (submission to completion) and releases the
 * request; a request that failed validation (a hard error) leaves x_h
 * untouched.  Every request is solved exactly as nps_solve would solve it
 * alone (same kernels, same per-request reductions): results do not depend
 * on what else is in flight.  Not thread-safe: one host thread per server.
 * ------------------------------------------------------------------------ */
enum { NPS_PENDING = 2 };
typedef struct nps_server nps_server;

int nps_server_create(const nps_net* net, size_t hbm_budget, int max_slots, nps_server** out);
void nps_server_destroy(nps_server* srv);
size_t nps_server_request_bytes(const nps_server* srv, nps_dims dims, const nps_opts* opts);
int nps_server_submit(nps_server* srv, const uint8_t* labels_h, nps_dims dims, const double* b_h,
                      const nps_opts* opts, uint64_t* req_id);
/* *n_active: requests on the device after the step; *n_queued: waiting. */
int nps_server_step(nps_server* srv, int* n_active, int* n_queued);
int nps_server_poll(nps_server* srv, uint64_t req_id, double* x_h, nps_info* info, double* latency_ms);

/* ------------------------------------------------------------------------
 * Training (loss of Sec. "Training": || b - A P(I, b) ||_2 per system).
 * precision NPS_FP64 (double vectors; parameter sums on the vector ALU),
 * NPS_FP32 (float vectors; the weight-gradient contraction over cells on
 * fp32 matrix cores) or NPS_MIXED_BF16 (float vectors; per-cell kernels
 * formed from the count-form weights rounded to bf16, as on the mixed solve's
 * matrix cores, and the weight-gradient contraction on bf16 matrix cores with
 * fp32 accumulation); every level keeps its per-cell kernels in the
 * workspace.
 *   nps_net_forward   y = P(I, r); keeps the per-level activations (the
 *                     down inputs, x1, the up outputs, the CConv_2 outputs)
 *                     in ws for the backward pass of the same system.
 *   nps_train_loss    res = b - A y on fluid, *loss_h = ||res||_2 (host),
 *                     gy = dL/dy = -A res / ||res|| (A is symmetric).
 *   nps_net_backward  adds dL/dparams (double, nps_param_count(levels),
 *                     blob layout of nps_net_create) into grad_d, given r
 *                     (the forward input) and gy; uses the activations the
 *                     last nps_net_forward left in ws.  Not synchronised.
 * ------------------------------------------------------------------------ */
size_t nps_train_workspace_bytes(nps_dims dims, int levels, int precision);

/* y = P(I, .)^T g: the adjoint of the network in its input vector (the
 * network is linear in it), i.e. Alg. 2 run backwards with each linear step
 * replaced by its adjoint -- the second half of the symmetric variant
 * P^T o P of the appendix on symmetry.  g_d, y_d: vectors of the precision's
 * type (NPS_FP64 double, NPS_FP32 float), device, caller-owned; y is 0 off
 * fluid.  Workspace: nps_train_workspace_bytes.  Not synchronised. */
int nps_apply_precond_transpose(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* g_d,
                                void* y_d, int precision, void* ws_d, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Right-hand sides from Ritz vectors (the training data of Sec. "Training":
 * Lanczos on the system matrix, Ritz vectors, normalised random linear
 * combinations).  FP64 throughout; n = nz*ny*nx.
 *
 * nps_lanczos: m Lanczos steps on A~ (the matrix of nps_solve, matrix-free)
 *   from v0_d restricted to fluid cells; reorth = 1: full
 *   reorthogonalisation (classical Gram-Schmidt, twice, on rocBLAS; it
 *   re-reads the whole basis every step, O(m^2 n) traffic), reorth = 0: the
 *   plain three-term recurrence (same Krylov space, the basis loses
 *   orthogonality as Ritz values converge).  Outputs, device,
 *   caller-owned: V_d double[m*n] (column j = v_(j+1), contiguous n values,
 *   zero off fluid), alpha_d double[m] (diagonal of T_m), beta_d double[m]
 *   (beta_d[j] couples v_(j+1) and v_(j+2); the last is the norm of the final
 *   residual).  *steps_h = the steps before an invariant subspace was
 *   reached (m if none; later columns and coefficients are zero).
 *   Workspace: nps_lanczos_workspace_bytes.  Synchronises the stream.
 * nps_ritz_rhs: the Ritz pairs of T_m (rocSOLVER's tridiagonal divide and conquer;
 *   theta_d double[m] ascending) and k right-hand sides
 *   rhs_d[:, i] = V Y c_i / ||V Y c_i|| for the columns c_i of coef_d
 *   (double[m*k], column-major: the caller draws the random coefficients).
 *   rhs_d double[n*k], column-major.  Workspace: nps_ritz_workspace_bytes.
 *   Synchronises the stream; NPS_EBREAKDOWN if the eigensolver fails.
 * Both create a rocBLAS handle on first use per device and thread.
 * ------------------------------------------------------------------------ */
size_t nps_lanczos_workspace_bytes(nps_dims dims, int m);
int nps_lanczos(const uint8_t* labels_d, nps_dims dims, int m, int reorth, const double* v0_d, double* V_d,
                double* alpha_d, double* beta_d, int* steps_h, void* ws_d, size_t ws_bytes, void* stream);
size_t nps_ritz_workspace_bytes(int m, int k);
int nps_ritz_rhs(const double* V_d, nps_dims dims, int m, const double* alpha_d, const double* beta_d,
                 const double* coef_d, int k, double* rhs_d, double* theta_d, void* ws_d, size_t ws_bytes,
                 void* stream);

/* Asymmetry of the network on x, y (appendix on symmetry):
 *   *s_h = |x.P(y) - y.P(x)| / sqrt(|x.P(x)| |y.P(y)|)   (0 if the root is 0).
 * Also leaves P(x) in px_d and P(y) in py_d.  Vectors of the precision's
 * vector type (double for NPS_FP64, else float), device, caller-owned; dots
 * accumulate in double.  Workspace: nps_workspace_bytes(dims, levels,
 * precision, 0).  Synchronises the stream (the result is a host value). */
int nps_asymmetry(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* x_d, const void* y_d,
                  void* px_d, void* py_d, int precision, void* ws_d, size_t ws_bytes, double* s_h, void* stream);
int nps_net_forward(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* r_d, void* y_d,
                    int precision, void* ws_d, size_t ws_bytes, void* stream);
int nps_train_loss(const uint8_t* labels_d, nps_dims dims, int levels, const void* b_d, const void* y_d,
                   void* gy_d, double* loss_h, int precision, void* ws_d, size_t ws_bytes, void* stream);
int nps_net_backward(const nps_net* net, const uint8_t* labels_d, nps_dims dims, const void* r_d,
                     const void* gy_d, double* grad_d, int precision, void* ws_d, size_t ws_bytes, void* stream);

/* One training step over a batch (Sec. "Training": the loss averaged over a
 * batch of systems): for each system i < batch, y_i = P(I_i, b_i) and
 * loss_i = || b_i - A_i y_i ||_2; adds d(mean_i loss_i)/dparams into grad_d
 * (double, nps_param_count(levels), blob layout of nps_net_create; not
 * zeroed) and writes the mean loss to *loss_h.
 *   labels_d  uint8[batch][nz*ny*nx]  the systems' labels, back to back.
 *   b_d       [batch][nz*ny*nx]       right-hand sides (double for NPS_FP64,
 *                                     float otherwise), zero off fluid.
 * The systems run one after another in one workspace of
 * nps_train_workspace_bytes(dims, levels, precision) bytes: each forward
 * keeps its per-level activations for its own backward pass.  Synchronises
 * the stream (the loss is a host value). */
int nps_train_step(const nps_net* net, const uint8_t* labels_d, nps_dims dims, int batch, const void* b_d,
                   double* grad_d, double* loss_h, int precision, void* ws_d, size_t ws_bytes, void* stream);

/* Per-kernel timing.  While enabled (on != 0, per calling thread), every
 * kernel the library launches is bracketed by a pair of HIP events recorded
 * on the launch stream.  nps_profile_read synchronises those events, writes
 * one record per kernel name (at most max_records, in first-launch order)
 * to out_h, stores the number of names in *n_records, and clears the
 * accumulated records.  Returns NPS_ENOMEM if more than 1,000,000 launches
 * were recorded since the last read (later ones are dropped). */
typedef struct {
    char name[40];        /* kernel name, e.g. "net_down_l1"               */
    int launches;         /* launches recorded                             */
    double total_ms;      /* sum of event-to-event durations               */
    double cells;         /* sum over launches of the cells of the level   */
} nps_kernel_stat;

int nps_profile_enable(int on);
int nps_profile_read(nps_kernel_stat* out_h, int max_records, int* n_records);

/* Thread-local description of the last error ("" if none). */
const char* nps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NPS_H */
