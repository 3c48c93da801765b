/*
 * helm.h -- C ABI of the MI355X (gfx950) frequency-domain 3D Helmholtz
 * library: matrix-free operator apply, ML-GMRES-preconditioned solves and the
 * adjoint-state least-squares misfit gradient.
 *
 * Problem (Da Silva & Herrmann, arXiv:1703.09268, Preamble, eqs. helmholtz
 * and mainprob; Appendix A, the linear system L u + omega^2 A diag(m) u = q):
 *
 *   H(m) u = q,   H = L + omega^2 A diag(m),   m = 1/v^2  [s^2/m^2]
 *
 * on a rectangular grid that already includes the absorbing layer (the
 * paper's extended domain Omega'), zero Dirichlet data outside the grid.
 * L is the layer-stretched 7-point Laplacian (A = I), or the compact
 * 27-point Laplacian on rows away from the layer with the 7-point stretched
 * row inside it (A = 27-point mass distribution, real symmetric).
 *
 * Layer (the paper leaves the damping function open; this is the library's
 * definition): per axis, with node coordinate t and
 *   d(t) = max(0, npml - t, t - (n - 1 - npml)),
 *   sigma(t) = sigma_max (d / npml)^2,
 *   sigma_max = 3 v_ref ln(1/pml_R) / (2 npml h),
 *   s(t) = 1 + i sigma(t) / omega,
 * the derivative d/dx becomes (1/s) d/dx; the 7-point row is
 *   sum_a cp_a (u[p+e_a] - u[p]) - cm_a (u[p] - u[p-e_a]),
 *   cp = 1/(h^2 s(p) s(p+1/2)),  cm = 1/(h^2 s(p) s(p-1/2)).
 *
 * Data layout (all entry points)
 *   * Grids are C-ordered [nx][ny][nz], z fastest, index (i*ny + j)*nz + k.
 *   * Complex numbers are interleaved {re, im}; HELM_C64 = 2 x float,
 *     HELM_C128 = 2 x double.  The model m is float for HELM_C64 and double
 *     for HELM_C128.
 *   * Several right-hand sides (nrhs) are stored one after the other:
 *     element p of right-hand side r is at offset r*N + p, N = nx*ny*nz.
 *   * Arrays marked "dev" are device pointers (hipMalloc or a torch tensor's
 *     data_ptr on the current device); "host" marks host memory.
 *
 * Ownership: the caller owns every buffer it passes and keeps it alive until
 * the work on `stream` has completed; the library never frees caller memory.
 * The context owns a workspace pool (grown on demand, freed by
 * helm_destroy).  `stream` is a hipStream_t (NULL = the null stream); all
 * device work is enqueued on it.  A context is not thread-safe: use one per
 * host thread.
 *
 * Errors: every entry point returns a helm_status; nothing throws or aborts
 * across the ABI.  On an error return helm_last_error(ctx) describes it.
 * Invalid arguments (null pointers, sizes < 3, npml >= n/2, omega <= 0,
 * nrhs < 1, out-of-grid source or receiver nodes, unknown enums, more than
 * 65535 (frequency, source) pairs, or more than 65535 2D problems
 * nfreq*nsrc*nky in the 2.5D entry point) return HELM_E_INVAL before any
 * device work is enqueued.  The pair limit is that of a launch's second grid
 * dimension, which the per-pair kernels index by pair.
 * Non-finite inputs: with the environment variable HELM_CHECK=1 every call
 * but helm_apply_noalloc first scans its device inputs -- the model, the
 * operator input or right-hand sides, initial guesses (warm_start), the
 * derivative input, and the data rows of the selected (frequency, source)
 * pairs -- and returns HELM_E_INVAL naming the array that holds a NaN or
 * Inf; the scan runs on `stream` and synchronises it.  Without it such
 * values propagate (a solve then returns HELM_BREAKDOWN).
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HELM_OK = 0,
  HELM_NOT_CONVERGED = 1, /* tolerance not reached in max_cycles */
  HELM_BREAKDOWN = 2,     /* non-finite residual (NaN / Inf input) */
  HELM_E_INVAL = -1,
  HELM_E_NOMEM = -2,
  HELM_E_HIP = -3,
  HELM_E_UNSUPPORTED = -4
} helm_status;

typedef enum { HELM_C64 = 0, HELM_C128 = 1 } helm_dtype;
typedef enum { HELM_7PT = 0, HELM_27PT = 1 } helm_stencil;
typedef enum { HELM_GMRES = 0, HELM_FGMRES_ML = 1 } helm_method;

/* Grid, layer and discretisation of one Helmholtz operator. */
typedef struct {
  int32_t n[3];    /* nodes per axis, layer included (each >= 3; n[0] = 1:
                      the 2D operator of the (n[1], n[2]) plane, 7-point) */
  double h;        /* grid spacing [m]                                     */
  int32_t npml;    /* layer width in nodes on each face (0 = no layer)     */
  double pml_R;    /* nominal reflection coefficient of the layer, (0, 1)  */
  double v_ref;    /* reference velocity of the layer profile [m/s]        */
  int32_t stencil; /* helm_stencil                                         */
  int32_t dtype;   /* helm_dtype                                           */
  double w27[7];   /* 27-point weights w1,w2,w3 (Laplacian) and wm1..wm4
                      (mass: centre, 6 faces, 12 edges, 8 corners); used
                      only with HELM_27PT; w1+w2+w3 = 1 and
                      wm1+6wm2+12wm3+8wm4 = 1 are expected, not enforced   */
} helm_grid;

/* Solver options (paper, ML-GMRES section; defaults by helm_default_opts). */
typedef struct {
  int32_t method;     /* HELM_GMRES: restarted GMRES(restart) on H;
                         HELM_FGMRES_ML: FGMRES(restart) preconditioned by
                         the recursive multilevel V-cycle                   */
  int32_t restart;    /* Krylov dimension of the outer solver (<= 32)      */
  int32_t max_cycles; /* restart cycles of the outer solver                */
  double tol;         /* target FP64 relative residual ||q - H u|| / ||q|| */
  int32_t ks_o, ks_i; /* smoother GMRES: cycles, Krylov dimension          */
  int32_t kc_o, kc_i; /* coarse (F)GMRES: cycles, Krylov dimension         */
  int32_t levels;     /* number of grids (2..4)                            */
  int32_t warm_start; /* 1: u holds the initial guess on entry             */
} helm_solver_opts;

/* Per right-hand-side result of a solve. */
typedef struct {
  int32_t status;     /* helm_status of this right-hand side              */
  int32_t cycles;     /* outer restart cycles performed                    */
  int32_t inner_its;  /* outer Arnoldi steps performed                     */
  int32_t pad_;
  int64_t matvecs;    /* fine-grid operator applications (incl. residuals) */
  double relres_fp64; /* ||q - H u|| / ||q|| of the returned iterate, FP64 */
} helm_solve_info;

typedef struct helm_ctx helm_ctx;

/* Create a context bound to HIP device `device` (hipSetDevice is called on
 * every entry).  *ctx receives the handle.  Fails with HELM_E_HIP if the
 * device does not exist. */
helm_status helm_create(helm_ctx** ctx, int device);

/* Synchronise the context's device and release the workspace. */
helm_status helm_destroy(helm_ctx* ctx);

/* Text of the last error on this context (static storage inside the
 * context; empty string when none).  ctx may be NULL (global message). */
const char* helm_last_error(const helm_ctx* ctx);

/* Library version string. */
const char* helm_version(void);

/* Fill *o with the paper's settings: FGMRES(5) preconditioned by the
 * 3-grid V-cycle with (ks_o, ks_i, kc_o, kc_i) = (3, 5, 3, 5), relative
 * residual 1e-6 (paper, ML-GMRES section, preconditioner-performance
 * experiment), max_cycles 50. */
void helm_default_opts(helm_solver_opts* o);

/* Device bytes the context's workspace needs for a solve with these
 * arguments (0 if the arguments are invalid). */
size_t helm_workspace_bytes(const helm_grid* g, const helm_solver_opts* o,
                            int nrhs);

/* y = H(m) x  (adjoint = 0)  or  y = H(m)^H x  (adjoint = 1) for nrhs
 * right-hand sides sharing m and omega (the discrete operator of the
 * Preamble; the paper's H*x and H'*x).
 *   m     dev, N reals (float for C64, double for C128)
 *   omega angular frequency 2 pi f [rad/s], > 0
 *   x, y  dev, nrhs*N complex of g->dtype; must not overlap.
 * Asynchronous on `stream`. */
helm_status helm_apply(helm_ctx* ctx, const helm_grid* g, const void* m,
                       double omega, int adjoint, int nrhs, const void* x,
                       void* y, void* stream);

/* helm_apply for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, operator and results (bitwise) as helm_apply, which
 * allocates its cached operator description on a cache miss; this variant
 * builds that description (layer tables, right-hand-side descriptors,
 * stencil workgroup maps) with one setup kernel into a fixed 8 MiB scratch
 * array of the library, one copy per GPU, kept until the process ends.  It
 * calls no allocation routine, copies nothing from the host and does not
 * synchronise: two kernel launches on `stream`.  The x chunk of the stencil
 * tiles is the library's heuristic (no tile timing).
 * Limits: the description must fit in 8 MiB (about 2^20 stencil workgroups
 * over all right-hand sides; for complex128 or odd-nz 27-point operators,
 * which use one workgroup per 256 points, nrhs * N up to about 5 * 10^8);
 * larger requests return HELM_E_INVAL before any device work.
 * Every call on one GPU overwrites that GPU's scratch array: calls that
 * overlap on one GPU (on different streams, or from different contexts or
 * host threads) race; calls ordered on one stream do not. */
helm_status helm_apply_noalloc(helm_ctx* ctx, const helm_grid* g,
                               const void* m, double omega, int adjoint,
                               int nrhs, const void* x, void* y,
                               void* stream);

/* Solve H(m) u = q (adjoint = 0) or H(m)^H u = q (adjoint = 1) for nrhs
 * right-hand sides sharing m and omega (the paper's H\Q, all sources of one
 * frequency as one block) with the solver in *o (NULL = defaults).
 *   q     dev, nrhs*N complex of g->dtype
 *   u     dev, nrhs*N complex of g->dtype; initial guess if o->warm_start,
 *         otherwise ignored on entry; overwritten with the solution
 *   info  host, nrhs entries (may be NULL)
 * The outer iterate and its residual are kept in FP64 (mixed-precision
 * refinement) for HELM_C64; inner Krylov work is in the grid's dtype.
 * Returns HELM_OK when every right-hand side reached o->tol,
 * HELM_NOT_CONVERGED if any did not (u still holds the best iterate),
 * HELM_BREAKDOWN if a residual became non-finite.  Synchronises `stream`
 * once per outer cycle (convergence test) and before returning. */
helm_status helm_solve(helm_ctx* ctx, const helm_grid* g, const void* m,
                       double omega, int adjoint, int nrhs, const void* q,
                       void* u, const helm_solver_opts* o,
                       helm_solve_info* info, void* stream);

/* One problem of a batched solve. */
typedef struct {
  helm_grid grid;   /* every problem of a batch: same dtype and stencil      */
  const void* m;    /* dev, N reals (float for C64, double for C128)          */
  double omega;     /* angular frequency, > 0                                 */
  const void* q;    /* dev, N complex right-hand side                         */
  void* u;          /* dev, N complex solution (initial guess if warm_start)  */
} helm_problem;

/* Solve nprob independent problems of different sizes, frequencies and
 * models together (not in the paper, whose parallelism is over workers:
 * this is the same solver as helm_solve applied to all problems at once).
 * Every kernel of the solve covers all problems in one launch; one outer
 * FGMRES cycle (Arnoldi steps with their V-cycles) is captured once as a
 * hipGraph and replayed; problems that converge are masked off while the
 * others continue.  Same options, precision and status semantics as
 * helm_solve; info (host, nprob entries, may be NULL).  All problems use
 * H (adjoint = 0) or H^H (adjoint = 1). */
helm_status helm_solve_batched(helm_ctx* ctx, int nprob, const helm_problem* probs,
                               int adjoint, const helm_solver_opts* o,
                               helm_solve_info* info, void* stream);

/* misfit_gradient flags */
#define HELM_MG_FORWARD_ONLY 1 /* solve forward, return f; no gradient     */
#define HELM_MG_REUSE_U 2      /* u_store already holds H^{-1} q           */
#define HELM_MG_ACCUMULATE 4   /* g += gradient instead of g = gradient    */
#define HELM_MG_U_FP64 8       /* u_store holds complex128 fields (the FP64
                                  outer iterates) even for HELM_C64 grids;
                                  u_store must not be NULL                  */
#define HELM_MG_RENORMALISE 16 /* f and g are divided by the number of
                                  selected (frequency, source) pairs: the
                                  average of the subsampled objective       */

/* Least-squares misfit and its adjoint-state gradient summed over the
 * selected (frequency, source) pairs (paper: Preamble eq. mainprob, the sum
 * over sources and frequencies; Listing of PDEfunc, case OBJ; Table
 * derivstuff rows u, V, grad f; Appendix A, eq. dHadj; the source/frequency
 * mask and the averaged subsampled objective of the Software Design and
 * stochastic-inversion sections):
 *   q_fs = amp_fs e_{src_s} / h^3                (on-node point source)
 *   u_fs = H_f^{-1} q_fs,   r_fs = P_r u_fs - d_fs
 *   f    = c * 1/2 sum_{(f,s) selected} ||r_fs||^2
 *   v_fs = -H_f^{-H} P_r^T r_fs
 *   g    = c * sum_{(f,s) selected} Re(omega_f^2 conj(u_fs) * (A^H v_fs))
 * with H_f = H(m) at omega_f, c = 1 (c = 1/#selected with
 * HELM_MG_RENORMALISE).  All selected pairs are solved together: one
 * forward and one adjoint multi-right-hand-side solve whose right-hand
 * sides may have different frequencies (every kernel covers all of them).
 * The receiver residual is formed from the FP64 outer iterate of the
 * forward solve (or from u_store with HELM_MG_REUSE_U; store the fields with
 * HELM_MG_U_FP64 to keep that residual accurate when r is much smaller than
 * u at the receivers).
 * Arguments:
 *   m        dev, N reals (float for C64, double for C128)
 *   nfreq    number of frequencies (>= 1); omega host double [nfreq],
 *            angular frequencies, each > 0
 *   nsrc     number of sources (>= 1); src_idx host int32 [nsrc][3] node
 *            indices (i, j, k)
 *   src_amp  host double [nfreq][nsrc][2] complex amplitudes (NULL = all 1)
 *   mask     host uint8 [nfreq][nsrc]: nonzero selects the pair (NULL = all
 *            pairs); unselected pairs are neither solved nor summed
 *   nrec     number of receivers (>= 1); rec_idx host int32 [nrec][3]
 *   d        dev, [nfreq][nsrc][nrec] complex of g->dtype, observed data
 *            (rows of unselected pairs are not read)
 *   f        host, receives the misfit (FP64 accumulation)
 *   grad     dev, N reals (float for C64, double for C128); overwritten
 *            (or accumulated into with HELM_MG_ACCUMULATE); may be NULL
 *            with HELM_MG_FORWARD_ONLY
 *   u_store  dev, [nfreq][nsrc][N] complex of g->dtype (complex128 with
 *            HELM_MG_U_FP64) or NULL: receives the forward fields of the
 *            selected pairs (or supplies them with HELM_MG_REUSE_U); rows of
 *            unselected pairs are left untouched
 *   flags    HELM_MG_* bits
 *   info     host, 2*nfreq*nsrc entries or NULL: forward solve of pair
 *            (f, s) at f*nsrc + s, adjoint solve at nfreq*nsrc + f*nsrc + s;
 *            entries of unselected pairs and of solves not run are zero
 * Invalid arguments (see the top of this file; also a NULL u_store with
 * HELM_MG_REUSE_U or HELM_MG_U_FP64, unknown flag bits) return HELM_E_INVAL
 * before any device work.  With no pair selected f = 0 and g = 0 (or
 * unchanged with HELM_MG_ACCUMULATE).  Returns the worst status of the
 * solves. */
helm_status misfit_gradient(helm_ctx* ctx, const helm_grid* g, const void* m,
                            int nfreq, const double* omega, int nsrc,
                            const int32_t* src_idx, const double* src_amp,
                            const uint8_t* mask, int nrec,
                            const int32_t* rec_idx, const void* d, double* f,
                            void* grad, void* u_store, int flags,
                            const helm_solver_opts* o, helm_solve_info* info,
                            void* stream);

/* misfit_gradient with sources and receivers anywhere inside the grid (the
 * paper's Kaiser-windowed sinc interpolation operators Ps and Pr: Software
 * Design section and the PDEfunc listing).  Same arguments and results as
 * misfit_gradient, except:
 *   src_pos  host double [nsrc][3], rec_pos host double [nrec][3]: positions
 *            in node units (node (i, j, k) sits at (i, j, k)), each inside
 *            [0, n_a - 1]
 *   radius   half-width r of the windowed sinc in nodes (1..8)
 *   kaiser_b shape b of the Kaiser window (>= 0)
 * A point at x contributes, per axis, w(i) = sinc(i - x) I0(b sqrt(1 - ((i -
 * x)/r)^2)) / I0(b) to the 2r nodes floor(x) - r + 1 .. floor(x) + r that lie
 * inside the grid; the 3D weights are the product of the axes.  The source
 * is q = amp sum_n w_n e_n / h^3, the receiver value (P_r u)_k = sum_n w_{k,n}
 * u_n; an on-node position reduces to misfit_gradient's point source and
 * sampling.  Out-of-range positions, radius or b return HELM_E_INVAL. */
helm_status misfit_gradient_offgrid(helm_ctx* ctx, const helm_grid* g,
                                    const void* m, int nfreq,
                                    const double* omega, int nsrc,
                                    const double* src_pos,
                                    const double* src_amp,
                                    const uint8_t* mask, int nrec,
                                    const double* rec_pos, int radius,
                                    double kaiser_b, const void* d, double* f,
                                    void* grad, void* u_store, int flags,
                                    const helm_solver_opts* o,
                                    helm_solve_info* info, void* stream);

/* pde_derivative modes (the paper's PDEfunc cases of the same names) */
#define HELM_JACOB_FORW 1 /* output = J dm                       */
#define HELM_JACOB_ADJ 2  /* output = J^* y                      */
#define HELM_HESS_GN 3    /* output = H_GN dm = J^* J dm         */
#define HELM_HESS 4       /* output = (Hessian of the misfit) dm */

/* Linearised modelling and second-order products of the least-squares
 * misfit, summed over the selected (frequency, source) pairs (paper: Table
 * derivstuff rows Du, J, T, T^*, DT^*, H_GN and the Hessian; Table
 * derivcosts, 2 / 2 / 3 / 4 PDE solves per pair; the Listing of PDEfunc,
 * cases JACOB_FORW, JACOB_ADJ, HESS_GN, HESS; Appendix A, eqs. dU2, dH,
 * dHadj, DTadj).  Per selected pair (f, s), with H = H_f, u = H^{-1} q_fs
 * (q_fs, P_r, mask, c and the pair arguments exactly as in
 * misfit_gradient), real model perturbation dm and
 *   T dm = omega_f^2 A (u * dm),   T^* z = omega_f^2 conj(u) * (A^H z):
 *   HELM_JACOB_FORW  du = -H^{-1} T dm;          output[f][s] = P_r du
 *   HELM_JACOB_ADJ   v = -H^{-H} P_r^T y_fs;     output = c sum Re(T^* v)
 *   HELM_HESS_GN     w = -H^{-H} P_r^T P_r du;   output = c sum Re(T^* w)
 *   HELM_HESS        v = -H^{-H} P_r^T (P_r u - d_fs),
 *                    dv = H^{-H}(-omega_f^2 dm * (A v) - P_r^T P_r du);
 *                    output = c sum Re(omega_f^2 conj(du) * (A v))
 *                                   + Re(T^* dv)
 * (the derivative of H^H v = -P_r^T r: the sign and the DH[dm]^H form of
 * its first term follow from differentiating the adjoint equation).
 * Arguments (the pair arguments as in misfit_gradient):
 *   mode     HELM_JACOB_FORW / HELM_JACOB_ADJ / HELM_HESS_GN / HELM_HESS
 *   input    dev: dm, N reals (float for C64, double for C128), or, for
 *            HELM_JACOB_ADJ, y, [nfreq][nsrc][nrec] complex of g->dtype
 *   d        dev [nfreq][nsrc][nrec] complex: observed data (HELM_HESS
 *            only; may be NULL otherwise)
 *   output   dev: HELM_JACOB_FORW [nfreq][nsrc][nrec] complex (rows of
 *            unselected pairs are zeroed); otherwise N reals, overwritten
 *            (added to with HELM_MG_ACCUMULATE)
 *   u_store  dev or NULL: the forward fields, as in misfit_gradient
 *   flags    HELM_MG_REUSE_U, HELM_MG_U_FP64, HELM_MG_ACCUMULATE,
 *            HELM_MG_RENORMALISE (c = 1/#selected; applies to the
 *            model-space outputs)
 *   info     host, 4*nfreq*nsrc entries or NULL: solve k of pair (f, s) at
 *            k*nfreq*nsrc + f*nsrc + s; k = 0 the forward fields (zero with
 *            HELM_MG_REUSE_U), then in the order of the formulas above
 *            (JACOB_FORW: du; JACOB_ADJ: v; HESS_GN: du, w; HESS: v, du,
 *            dv); unused entries are zero
 * Invalid arguments return HELM_E_INVAL before any device work.  Returns
 * the worst status of the solves. */
helm_status pde_derivative(helm_ctx* ctx, int mode, const helm_grid* g,
                           const void* m, int nfreq, const double* omega,
                           int nsrc, const int32_t* src_idx,
                           const double* src_amp, const uint8_t* mask,
                           int nrec, const int32_t* rec_idx, const void* input,
                           const void* d, void* output, void* u_store,
                           int flags, const helm_solver_opts* o,
                           helm_solve_info* info, void* stream);

/* pde_derivative with off-grid sources and receivers: the arguments of
 * pde_derivative with src_idx / rec_idx replaced by src_pos / rec_pos,
 * radius and kaiser_b as in misfit_gradient_offgrid. */
helm_status pde_derivative_offgrid(helm_ctx* ctx, int mode,
                                   const helm_grid* g, const void* m,
                                   int nfreq, const double* omega, int nsrc,
                                   const double* src_pos,
                                   const double* src_amp, const uint8_t* mask,
                                   int nrec, const double* rec_pos,
                                   int radius, double kaiser_b,
                                   const void* input, const void* d,
                                   void* output, void* u_store, int flags,
                                   const helm_solver_opts* o,
                                   helm_solve_info* info, void* stream);

/* Wavefield Reconstruction Inversion (the paper's penalty method: Penalty
 * Method subsection, eqs. wri and wrifieldeq; Appendix B, derivative
 * expressions for WRI), summed over the selected (frequency, source) pairs.
 * Per pair, with q, P_r, the amplitudes, mask and c as in misfit_gradient:
 *   u_fs = argmin_u 1/2 ||P_r u - d_fs||^2 + lambda^2/2 ||H_f u - q_fs||^2,
 *          i.e. (P_r^T P_r + lambda^2 H^H H) u = P_r^T d + lambda^2 H^H q
 *   f    = c sum (1/2 ||P_r u_fs - d_fs||^2 + lambda^2/2 ||H_f u_fs - q_fs||^2)
 *   g    = c sum lambda^2 Re(omega_f^2 conj(u_fs) * (A^H (H_f u_fs - q_fs)))
 * The field is computed as u = H^{-1}(q + H^{-H} P_r^T y) with y from
 * conjugate gradients on the receiver-space system
 * (P_r H^{-1} H^{-H} P_r^T + lambda^2 I) y = d - P_r H^{-1} q, started at
 * y = 0 and stopped when its residual falls to cg_tol times the initial one
 * (or after cg_max steps); every step costs one adjoint and one forward
 * ML-GMRES solve per active pair, all pairs batched.  The field is
 * accumulated in FP64 and H u - q formed in FP64.
 * Arguments as misfit_gradient, plus:
 *   lambda   penalty weight (> 0)
 *   cg_tol   relative residual target of the receiver-space CG, [0, 1)
 *   cg_max   CG step limit (>= 0; 0 returns the reduced field H^{-1} q)
 *   u_store  dev or NULL: receives the WRI fields of the selected pairs
 *            ([nfreq][nsrc][N], complex128 with HELM_MG_U_FP64)
 *   flags    HELM_MG_FORWARD_ONLY (f only), HELM_MG_ACCUMULATE,
 *            HELM_MG_U_FP64, HELM_MG_RENORMALISE
 *   info     host, nfreq*nsrc entries or NULL: the CG of pair (f, s) at
 *            f*nsrc + s: status (0 converged, 1 step limit, 2 breakdown),
 *            cycles = CG steps, matvecs = ML-GMRES solves (1 + 2 steps),
 *            relres_fp64 = final CG relative residual
 * Invalid arguments return HELM_E_INVAL before any device work.  Returns
 * the worst of the solves' and the CGs' statuses. */
helm_status wri_misfit_gradient(helm_ctx* ctx, const helm_grid* g,
                                const void* m, int nfreq, const double* omega,
                                int nsrc, const int32_t* src_idx,
                                const double* src_amp, const uint8_t* mask,
                                int nrec, const int32_t* rec_idx,
                                const void* d, double lambda, double cg_tol,
                                int cg_max, double* f, void* grad,
                                void* u_store, int flags,
                                const helm_solver_opts* o,
                                helm_solve_info* info, void* stream);

/* 2.5D modelling, misfit and gradient (paper: the 2.5D subsection) for a 3D
 * model invariant along one axis ("y"), on a 2D grid: g->n[0] = 1, the
 * plane (n[1], n[2]) carrying the paper's (x, z), 7-point operator.  (A grid
 * with n[0] = 1 is the 2D operator in every entry point: the first axis has
 * no coupling and no layer, the layers act on the plane's two axes, the
 * point source is amp e_s / h^2, and the multigrid levels keep n[0] = 1.)
 * Per frequency f: K_f = min(p_kc omega_f / v_min, pi / h); Gauss-Legendre
 * nodes k_i and weights w_i (i < nky) of [0, K_f]; per selected (f, s) and i
 * the 2D field u~_{f,s,i} solves
 *   (L + omega_f^2 (m - k_i^2 / omega_f^2)) u~ = amp_fs e_{src_s} / h^2
 * (all of them in one batched solve), and
 *   d_pred[f][s][r] = sum_i (w_i / pi) cos(k_i (rec_y[r] - src_y[s])) u~(rec_r)
 *   f = c 1/2 sum_{(f,s) selected} ||d_pred - d||^2   (d = 0 when NULL)
 *   g = c sum Re(omega_f^2 conj(u~_{f,s,i}) * v_{f,s,i}),
 *       v = -H_i^{-H} P_r^T (c_{f,s,i} * (d_pred - d)_{f,s})
 * with c = 1 (1/#selected pairs with HELM_MG_RENORMALISE); the quadrature is
 * fixed by (nky, p_kc, v_min), so g is the exact gradient of f.
 * Arguments:
 *   m        dev, N reals of g->dtype (the model on the plane)
 *   nky      quadrature nodes (1..4096); p_kc (> 0): the cut at p_kc times
 *            the critical wavenumber omega / v_min (v_min > 0, m/s)
 *   src_idx  host int32 [nsrc][2]: plane node (j, k); src_y host double
 *            [nsrc]: coordinate along the invariant axis (m)
 *   rec_idx  host int32 [nrec][2], rec_y host double [nrec]: the same for
 *            the receivers
 *   src_amp, mask as in misfit_gradient
 *   d        dev [nfreq][nsrc][nrec] complex of g->dtype, observed data, or
 *            NULL with HELM_MG_FORWARD_ONLY
 *   f        host, the misfit;  grad  dev, N reals (NULL with FORWARD_ONLY)
 *   d_pred   dev [nfreq][nsrc][nrec] complex or NULL: receives the
 *            modelled data of the selected pairs
 *   flags    HELM_MG_FORWARD_ONLY, HELM_MG_ACCUMULATE, HELM_MG_RENORMALISE
 *   info     host, 2*nfreq*nsrc*nky entries or NULL: the forward solve of
 *            (f, s, i) at (f*nsrc + s)*nky + i, the adjoint solve after all
 *            forward entries
 * Invalid arguments (a 3D grid, nky, p_kc, v_min, nodes outside the plane,
 * non-finite coordinates, flags) return HELM_E_INVAL before any device
 * work.  Returns the worst status of the solves. */
helm_status misfit_gradient_25d(helm_ctx* ctx, const helm_grid* g,
                                const void* m, int nfreq, const double* omega,
                                int nky, double p_kc, double v_min, int nsrc,
                                const int32_t* src_idx, const double* src_y,
                                const double* src_amp, const uint8_t* mask,
                                int nrec, const int32_t* rec_idx,
                                const double* rec_y, const void* d, double* f,
                                void* grad, void* d_pred, int flags,
                                const helm_solver_opts* o,
                                helm_solve_info* info, void* stream);

/* Parameters of the inversion driver (fwi_invert). */
typedef struct {
  int32_t band_size;      /* frequencies per band (>= 1)                      */
  int32_t band_overlap;   /* frequencies shared by consecutive bands,
                             0 <= band_overlap < band_size                    */
  int32_t r_sub;          /* iterations per draw: r_sub * ceil(nsrc / p)      */
  int32_t memory;         /* stored L-BFGS pairs (0..16)                      */
  int32_t batch;          /* initial subset size p; <= 0 or >= nsrc: every
                             source (no random draw)                          */
  int32_t subproblems;    /* draws per band (T, >= 1)                         */
  int32_t batch_increase; /* growth of p after a failed line search (>= 0)    */
  int32_t max_ls;         /* line-search trials per iteration (1..60)         */
  uint64_t seed;          /* SplitMix64 seed of the source draws              */
  double c1;              /* sufficient-decrease constant, (0, 1)             */
  double gtol;            /* stop a draw when max|g_F| <= gtol * its value at
                             the draw's start (>= 0)                          */
  double step0;           /* max-norm length of a steepest-descent trial
                             step, > 0 (model units)                          */
  double lo, hi;          /* scalar bounds, used where lo / hi arrays are
                             NULL                                             */
} helm_fwi_params;

/* Summary of one draw (subproblem) of fwi_invert. */
typedef struct {
  int32_t band, draw;     /* band index, draw index within the band           */
  int32_t nsel;           /* sources in the draw                              */
  int32_t max_iters;      /* r_sub * ceil(nsrc / p)                           */
  int32_t iters;          /* iterations performed (a failed one included)     */
  int32_t failed;         /* 1: ended by a failed line search                 */
  int32_t evals;          /* objective + gradient evaluations                 */
  int32_t status;         /* worst helm_status of the draw's solves           */
  double f_start, f_end;  /* subset objective at the draw's first and last
                             iterate                                          */
} helm_fwi_draw;

/* One L-BFGS iteration of fwi_invert. */
typedef struct {
  int32_t band, draw, iter, nsel;
  int32_t trials;         /* line-search trials                               */
  int32_t accepted;       /* 1: a trial met the sufficient decrease           */
  int32_t status;         /* worst helm_status of the draw's solves so far    */
  int32_t pad_;
  double f;               /* subset objective at the iterate                  */
  double f_new;           /* at the accepted (or last) trial                  */
  double step;            /* accepted t (or half the last one tried)          */
  double pgmax;           /* max |g_F| at the iterate                         */
} helm_fwi_record;

/* Number of draws fwi_invert performs: bands * subproblems, bands =
 * 1 + ceil(max(0, nfreq - band_size) / (band_size - band_overlap)); -1 for
 * invalid arguments. */
int helm_fwi_draw_count(int nfreq, const helm_fwi_params* p);

/* Full-waveform inversion by frequency continuation, stochastic source
 * subsets and a box-constrained L-BFGS (paper: the 2D inversion example --
 * bands of band_size frequencies overlapping by band_overlap, a fixed number
 * of bound-constrained L-BFGS iterations per band, warm-started band to band,
 * the source/frequency mask selecting the band -- and the stochastic
 * inversion section -- min over m_LB <= m <= m_UB of the average of f_i over
 * a uniformly drawn subset I_k of p sources, r_sub ceil(nsrc / p)
 * iterations per draw, the result warm-starting the next draw, p grown by
 * batch_increase after a failed line search).  Per band, per draw: the
 * objective is misfit_gradient over the band's frequencies and the drawn
 * sources with HELM_MG_RENORMALISE; the projected L-BFGS is
 *   F   = points not held at a bound by the gradient (x <= lo with g > 0,
 *         x >= hi with g < 0 are held);
 *   d   = -H g on F by the two-loop recursion over the stored pairs restricted
 *         to F (initial scaling s.y / y.y of the newest), 0 off F; d =
 *         -g_F step0 / max|g_F| with no pair or when g.d >= 0;
 *   stop the draw when max|g_F| <= gtol * its value at the draw's start;
 *   x_t = clamp(x + t d, lo, hi), t = 1, 1/2, ... (max_ls trials) until
 *         f(x_t) <= f(x) + c1 g.(x_t - x); a failed search ends the draw;
 *   keep (x_t - x, g_t - g) when s.y > 1e-10 |s| |y| (memory pairs, oldest
 *         dropped); every draw starts with an empty memory.
 * Subsets: a partial Fisher-Yates shuffle of 0..nsrc-1 whose step-i swap
 * partner is i + (u mod (nsrc - i)), u the next output of SplitMix64 (Steele,
 * Lea and Flood 2014) seeded with p->seed, one counter for the whole run
 * (drawing every source consumes none); sorted ascending.  The L-BFGS
 * vectors are FP64 on the device (4 + 2 (memory + 1) vectors of N doubles
 * in the context's workspace); the solves read the trial model in the
 * grid's real type.
 * Arguments (the pair arguments as in misfit_gradient):
 *   m        dev, N reals of g->dtype: the starting model, overwritten by
 *            the result (clamped into the bounds first)
 *   lo, hi   dev, N doubles each, or NULL for p->lo / p->hi: the bounds
 *            (lo = hi clamps a point, e.g. a water layer)
 *   d        dev [nfreq][nsrc][nrec] complex of g->dtype: observed data
 *   p        host: the driver parameters
 *   draws    host, helm_fwi_draw_count() entries or NULL
 *   sources  host, [draws][nsrc] int32 or NULL: each draw's sources
 *            ascending, padded with -1
 *   recs     host, rec_cap entries or NULL: the iterations in order (the
 *            first rec_cap of them); *nrecs (host, may be NULL) receives the
 *            total number of iterations
 * Invalid arguments return HELM_E_INVAL before any device work, except bounds
 * with lo > hi (or NaN) somewhere in the arrays, which return HELM_E_INVAL
 * after one checking kernel, m unchanged.  Returns the worst status of all
 * solves. */
helm_status fwi_invert(helm_ctx* ctx, const helm_grid* g, void* m,
                       const double* lo, const double* hi, int nfreq,
                       const double* omega, int nsrc, const int32_t* src_idx,
                       const double* src_amp, int nrec,
                       const int32_t* rec_idx, const void* d,
                       const helm_fwi_params* p, const helm_solver_opts* o,
                       helm_fwi_draw* draws, int32_t* sources,
                       helm_fwi_record* recs, int rec_cap, int* nrecs,
                       void* stream);

/* fwi_invert with off-grid sources and receivers: src_idx / rec_idx replaced
 * by src_pos / rec_pos, radius and kaiser_b as in misfit_gradient_offgrid. */
helm_status fwi_invert_offgrid(helm_ctx* ctx, const helm_grid* g, void* m,
                               const double* lo, const double* hi, int nfreq,
                               const double* omega, int nsrc,
                               const double* src_pos, const double* src_amp,
                               int nrec, const double* rec_pos, int radius,
                               double kaiser_b, const void* d,
                               const helm_fwi_params* p,
                               const helm_solver_opts* o, helm_fwi_draw* draws,
                               int32_t* sources, helm_fwi_record* recs,
                               int rec_cap, int* nrecs, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
