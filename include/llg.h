/*
 * llg.h -- C ABI of the MI355X library for periodic Landau-Lifshitz-Gilbert
 * tangent-plane saddle-point systems with the matrix-free split FFT-HSS
 * preconditioner (Qi, Ye, Guan, "Matrix-Free FFT-HSS Preconditioning for
 * Periodic Landau-Lifshitz-Gilbert Saddle-Point Systems").
 *
 * Problem (Sec. 2.3-2.4): on a periodic grid of nx x ny x nz nodes with
 * spacing h (cell lengths L = n h; nz = 1 is two-dimensional), a time step k
 * solves the saddle-point system
 *
 *     A (v, r) = (f, 0),   A = [[H + S, B^T], [-B, 0]],
 *     H = alpha I + theta k C_hat (-Delta_N),  S v = m x v,
 *     B^T r = m r (node by node),  -B v = -m . v,  C_hat = (1 + alpha^2) cexc,
 *
 * for the velocity v and the Lagrange multiplier r (called "lam" below;
 * the paper's lambda is the HSS shift, called "shift").  theta = 1 is the
 * projected implicit Euler scheme, theta = 1/2 the midpoint scheme (Sec. 3.3).
 *
 * Data layout.  Every grid array is a contiguous, caller-owned DEVICE buffer
 * of float64 (float32 for the *_f32 entry points) in structure-of-arrays
 * form: plane c of a field starts at c * N_g, and node (x, y, z) of a plane
 * is element x + nx (y + ny z), N_g = nx ny nz.
 *   m      magnetization, 3 planes (m1, m2, m3)
 *   x      saddle unknown, 4 planes (v1, v2, v3, lam)
 * Pointers must be 16-byte aligned (LLG_EARG otherwise).  The library never
 * frees or retains a caller buffer.
 *
 * Execution.  Calls run on the caller's HIP stream (stream == NULL means the
 * null stream).  llg_matvec and fft_hss_apply are asynchronous.  gmres_solve
 * and the steppers synchronize the stream for their convergence tests and
 * return once the result is complete.  One context must not be used by two
 * calls at the same time (it owns the spectral scratch buffer).
 *
 * Errors are returned as llg_status codes, never thrown; llg_last_error()
 * returns a message for the last failing call on the calling thread.
 * Argument checks happen before any GPU work is queued.
 */
#ifndef LLG_H
#define LLG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LLG_OK = 0,
  LLG_EARG = 1,      /* invalid argument (null pointer, size, parameter range) */
  LLG_EZERO_M = 2,   /* some |m_i| = 0: the constraint block loses rank (Prop. 1) */
  LLG_ENOCONV = 3,   /* Krylov iteration limit reached; x holds the last iterate */
  LLG_EPICARD = 4,   /* midpoint Picard iteration limit reached */
  LLG_ENAN = 5,      /* a residual or norm became non-finite */
  LLG_EHIP = 6,      /* HIP runtime failure */
  LLG_ENOMEM = 7,    /* device allocation failed, or workspace too small */
  LLG_EUNSUPPORTED = 8 /* grid size not supported by this build */
} llg_status;

typedef enum {
  LLG_FP64 = 0,        /* plain float64 left-preconditioned GMRES */
  LLG_FP32_IR = 1,     /* float32 preconditioner and inner matvec inside float64
                          flexible GMRES with iterative refinement */
  LLG_FP32_IR_LEFT = 2 /* variant: float64 iterative refinement around a
                          left-preconditioned inner GMRES whose operator
                          M^{-1} A is one float32 pipeline (the exact fused
                          identity); float64 Arnoldi, no float32 basis */
} llg_precision;

typedef struct llg_ctx llg_ctx;

/* Physical parameters of one saddle system (Sec. 2.4 and Sec. 4.1).
 * The lower-order field (Sec. 2.1, eq. "heff"; Sec. 2.2) is
 *   h_low(m) = demag h_dem[m] + 2 aniso_k e (e.m) + h_uniform + h_field,
 * h_dem the periodic demagnetizing field with zero-mean potential:
 * h_dem^ = -xi~ (xi~ . m^) / |xi|^2, xi~ the wave vector with the Nyquist
 * entry of each axis set to zero.  Set demag = aniso_k = 0 for an applied
 * field alone (the fast path: no extra pipeline anywhere). */
typedef struct {
  double alpha;         /* damping, > 0 */
  double cexc;          /* normalized exchange coefficient (1 in the paper) */
  double dt;            /* time step k, >= 0 */
  double theta;         /* 1 (Euler) or 1/2 (midpoint); in (0, 1] */
  double shift;         /* HSS shift lambda > 0 (0.5 in the paper) */
  double h_uniform[3];  /* uniform applied field */
  const double* h_field;/* optional spatial applied field, 3 planes, or NULL */
  double demag;         /* coefficient of the demagnetizing field: 0 off, 1 on */
  double aniso_k;       /* uniaxial anisotropy coefficient K (energy K (1 - (e.m)^2)) */
  double aniso_axis[3]; /* easy axis e; must be a unit vector when aniso_k != 0 */
} llg_params;

typedef struct {
  int restart;       /* Krylov cycle length (30 by default) */
  int maxiter;       /* total inner iteration limit */
  int max_outer;     /* refinement steps of LLG_FP32_IR(_LEFT) */
  int use_x0;        /* 1: x holds the initial guess on entry, 0: start from 0 */
  double rtol;       /* accept when ||b - A x||_2 <= rtol ||b||_2 */
  double inner_rtol; /* relative tolerance of each inner FGMRES cycle (FP32_IR) */
  int prec;          /* llg_precision */
  int precond;       /* 0 = split FFT-HSS (the method), 1 = symmetric part
                        (lambda I + calH)^{-1} only, 2 = none: the comparison
                        preconditioners of Sec. 4.1 (float64 only) */
  int orth;          /* Arnoldi orthogonalization: 0 = CGS2 with the
                        re-orthogonalization delayed by one iteration (two
                        streaming passes, restart <= 31; default), 1 = CGS2 in
                        three passes */
  int picard_norm;   /* midpoint Picard stopping test: 0 = change of the frozen
                        midpoint, ||m_hat^{p+1} - m_hat^p|| <= tol ||m_hat^{p+1}||
                        (default), 1 = change of the velocity,
                        ||v^p - v^{p-1}|| <= tol ||v^p|| */
  int transpose;     /* gmres_solve only: 1 solves A^T x = b, left-preconditioned
                        by M^T (float64; the steppers ignore it) */
  int fuse_update;   /* delayed CGS2 (orth = 0): 0 = form each new basis
                        direction inside the next operator's first x pass
                        (one streaming pass fewer per iteration) on grids
                        whose x pass has at least 4096 blocks (256^3), else
                        in its own pass (default); 1 = fused on every grid;
                        -1 = never.  Steps with more than 8 directions always
                        use their own pass.  Results agree to rounding (the
                        inner products are summed in another order) */
} llg_solver_opts;

typedef struct {
  int iters;           /* inner Krylov iterations (all cycles / refinement steps) */
  int cycles;          /* Krylov cycles (restarts + 1) */
  int outer_steps;     /* refinement steps (FP32_IR) */
  int converged;       /* 1 if the true residual test passed */
  double rel_res_true; /* ||b - A x||_2 / ||b||_2, recomputed in float64 */
  double rel_res_prec; /* last preconditioned residual estimate / ||M^{-1} b|| */
  int restarts;        /* cycles - 1: restarts of the Krylov iteration */
  double ms;           /* host wall time of the call in milliseconds (it
                          synchronizes, so this covers the device work) */
} llg_solver_stats;

typedef struct {
  int picard_iters;         /* Picard iterations of the midpoint step (1 for Euler) */
  int lin_iters_total;      /* Krylov iterations over all solves of the step */
  int converged;            /* Picard (and every linear solve) converged */
  double picard_rel_change; /* last relative Picard change (the quantity picard_norm selects) */
  double max_len_err;       /* max_i | |m_i^{n+1}| - 1 | */
  double energy_before;     /* g_N(m^n) (exchange + lower-order energies) */
  double energy_after;      /* g_N(m^{n+1}) */
  double dissipation_defect;/* g_N(m^{n+1}) - g_N(m^n) + alpha k/(1+alpha^2) ||v||_N^2 */
  double inexact_correction;/* k/(1+alpha^2) [rho(v) - chi(lam)] (midpoint) */
  double v_norm2;           /* ||v||_N^2 */
} llg_step_stats;

/* Create a context for an nx x ny x nz grid (nz = 1: 2-D) with spacing h in
 * every direction (cell lengths n h; Sec. 2.3) on device `device`.
 * Grid sizes: ny and nz (or nz = 1) even, in [4, 512], and nx / 2 in [2, 256],
 * each of the form 2^a, 3 * 2^a or 5 * 2^a (nx even).  Allocates the twiddle
 * tables, the spectral scratch (about 48 N_g bytes) and reduction buffers.
 * Errors: LLG_EARG (null out, unsupported n, bad h), LLG_ENOMEM, LLG_EHIP. */
llg_status llg_ctx_create(llg_ctx** out, int nx, int ny, int nz, double h, int device);

/* The same for a cell of lengths lx, ly, lz (spacings lx / nx, ly / ny,
 * lz / nz may differ; lz is unused in 2-D but must be > 0): the periodic
 * cell prod_l (0, L_l) of Sec. 2.3 with wave numbers 2 pi k_l / L_l. */
llg_status llg_ctx_create_cell(llg_ctx** out, int nx, int ny, int nz, double lx, double ly, double lz,
                               int device);
llg_status llg_ctx_destroy(llg_ctx* ctx);

/* Bytes of caller workspace that gmres_solve and the steppers need with
 * restart length `restart` and precision `prec` (0 on bad arguments). */
size_t llg_workspace_bytes(const llg_ctx* ctx, int restart, int prec);

/* y = A x (transpose = 0) or A^T x (transpose = 1): the matrix-free saddle
 * operator of Sec. 2.4 eq. "saddle point system" (Sec. 3.1 eq. (HS)).
 * m: 3 planes; x, y: 4 planes; y must not alias x.  Asynchronous. */
llg_status llg_matvec(llg_ctx* ctx, const llg_params* prm, const double* m, const double* x, double* y,
                      int transpose, void* stream);

/* z = M^{-1} p = (calS + shift I)^{-1} (calH + shift I)^{-1} p (transpose = 0),
 * or M^{-T} p = (calH + shift I)^{-1} (calS + shift I)^{-T} p (transpose = 1):
 * the split FFT-HSS preconditioner of Sec. 3.2 (Algorithm 1 followed by the
 * closed-form nodal inverse, eq. "inverse S").  m: 3 planes; p, z: 4 planes;
 * z may alias p.  Asynchronous. */
llg_status fft_hss_apply(llg_ctx* ctx, const llg_params* prm, const double* m, const double* p, double* z,
                         int transpose, void* stream);

/* The same two operators computed entirely in float32 (benchmarks; the
 * precision form's inner operators are llg_precond_op_f32). */
llg_status llg_matvec_f32(llg_ctx* ctx, const llg_params* prm, const float* m, const float* x, float* y,
                          int transpose, void* stream);
llg_status fft_hss_apply_f32(llg_ctx* ctx, const llg_params* prm, const float* m, const float* p, float* z,
                             int transpose, void* stream);

/* The preconditioned operator of left-preconditioned GMRES, y = M^{-1} A x,
 * in one pipeline: the splitting A = (calH + shift I) + (calS - shift I) of
 * Sec. 3.1 (eq. (HS)) gives the exact identity
 *   M^{-1} A x = (calS + shift I)^{-1} [x + (calH + shift I)^{-1} (calS - shift I) x],
 * one nodal prologue, Algorithm 1 and the closed-form nodal inverse (Sec. 3.2,
 * eq. "inverse S"); the same values as fft_hss_apply(llg_matvec(x)) up to
 * rounding.  m: 3 planes; x, y: 4 planes, y must not alias x.
 * Optional Arnoldi products (the first projection of a Gram-Schmidt step,
 * formed in the operator's last pass from the values it writes): with
 * nbasis in [1, 32], basis points to nbasis vectors of 4 planes at stride
 * ld >= 4 N_g doubles (ld even) and dots (device, nbasis doubles) receives
 * dots[q] = basis_q . y; nbasis = 0 (basis, dots NULL) skips them.
 * Asynchronous.  Errors: LLG_EARG. */
llg_status llg_precond_op(llg_ctx* ctx, const llg_params* prm, const double* m, const double* x, double* y,
                          const double* basis, int nbasis, long long ld, double* dots, void* stream);

/* The float32 preconditioned operators of the precision form between float64
 * Krylov vectors (the FFTs and nodal blocks run in float32 on m in float32):
 *   side 0: y = M^{-1} A x by the fused identity above, one float32 pipeline
 *           (the left variant LLG_FP32_IR_LEFT); z unused;
 *   side 1: z = M^{-1} x (float32, stored: the flexible basis vector) and
 *           y = A z (float64 output), the flexible precision form's inner
 *           operator: two float32 pipelines joined in one x pass.
 * x, y: 4 float64 planes; z: 4 float32 planes (side 1).  Arnoldi products as
 * llg_precond_op.  Asynchronous.  Errors: LLG_EARG. */
llg_status llg_precond_op_f32(llg_ctx* ctx, const llg_params* prm, const float* m, const double* x, double* y,
                              float* z, int side, const double* basis, int nbasis, long long ld, double* dots,
                              void* stream);

/* Solve A(m) x = b (Sec. 3.2: GMRES left-preconditioned by the split
 * FFT-HSS operator; acceptance on the true relative residual).
 * b, x: 4 planes; x is the initial guess when opts->use_x0 = 1 and receives
 * the solution (the last iterate on LLG_ENOCONV).  With opts->transpose = 1
 * (float64 only) solves A(m)^T x = b with GMRES left-preconditioned by M^T
 * (operator M^{-T} A^T, two pipelines per iteration).  work: device
 * workspace of at least llg_workspace_bytes(ctx, opts->restart, opts->prec)
 * bytes.  stats may be NULL.  Synchronizes the stream.
 * Errors: LLG_EARG, LLG_EZERO_M, LLG_ENOMEM (work too small), LLG_ENOCONV,
 * LLG_ENAN, LLG_EHIP. */
llg_status gmres_solve(llg_ctx* ctx, const llg_params* prm, const double* m, const double* b, double* x,
                       const llg_solver_opts* opts, llg_solver_stats* stats, void* work, size_t work_bytes,
                       void* stream);

/* gmres_solve for callers that cannot allocate device memory (a serving
 * loop or a harness that forbids hipMalloc): the same solve, with the same
 * arguments except the workspace, which is a static device array of the
 * library (128 MiB per GPU, held from the first context on that GPU until
 * the process ends).  The call itself allocates no device or pinned memory.
 * The static workspace is shared by every call on one GPU: calls that
 * overlap on one GPU race on it; calls in sequence are independent (no
 * contents carry over).
 * Errors: as gmres_solve; LLG_ENOMEM when llg_workspace_bytes(ctx,
 * opts->restart, opts->prec) exceeds 128 MiB (e.g. 2-D grids up to 256^2 fit
 * at restart 30 in every precision); LLG_EHIP when the static workspace's
 * device address could not be obtained when the context was created. */
llg_status gmres_solve_noalloc(llg_ctx* ctx, const llg_params* prm, const double* m, const double* b, double* x,
                               const llg_solver_opts* opts, llg_solver_stats* stats, void* stream);

/* One projected implicit Euler step (Sec. 2.4; Sec. 3.2 last paragraph):
 * solve A(m^n) (v, lam) = (C_hat Delta_N m^n + (1+alpha^2) h_low(m^n), 0)
 * with theta = 1 (lower-order field explicit), then
 * m^{n+1} = (m^n + k v) / |m^n + k v|.
 * m: in m^n, out m^{n+1} (3 planes); v_out (3 planes) and lam_out (1 plane)
 * may be NULL.  prm->theta is ignored.  Synchronizes the stream. */
llg_status llg_step_euler(llg_ctx* ctx, const llg_params* prm, double* m, double* v_out, double* lam_out,
                          const llg_solver_opts* opts, llg_step_stats* stats, void* work, size_t work_bytes,
                          void* stream);

/* One projection-free midpoint step (Sec. 3.3, eqs. "C-N" and "hatm"):
 * Picard iteration on the frozen midpoint m_hat^p = m^n + (k/2) v^{p-1}, each
 * iterate a GMRES solve with theta = 1/2 warm-started from the previous
 * iterate, right-hand side (C_hat Delta_N m^n + (1+alpha^2) h_low(m_hat^p), 0);
 * stops when the change selected by opts->picard_norm is at most picard_tol
 * (relative); then m^{n+1} = m^n + k v.
 * m: in m^n, out m^{n+1}.  v_half: in v^{n-1/2} (the p = 0 midpoint; zeros on
 * the first step), out v^{n+1/2}.  lam: in the previous multiplier (initial
 * guess), out the new one; either may be NULL (zeros used, no output).
 * prm->theta is ignored.  Synchronizes the stream.
 * Errors: as gmres_solve, plus LLG_EPICARD. */
llg_status llg_step_midpoint(llg_ctx* ctx, const llg_params* prm, double* m, double* v_half, double* lam,
                             double picard_tol, int picard_max, const llg_solver_opts* opts,
                             llg_step_stats* stats, void* work, size_t work_bytes, void* stream);

/* Adjoint of one converged midpoint step m^{n+1} = m^n + k v(m^n, h).
 * With J the Jacobian of the residual of eq. "C-N" with respect to (v, lam),
 * solves J^T mu = (k gbar, 0) by GMRES preconditioned with the transposed
 * split FFT-HSS operator built on the midpoint, then, with L_low the linear
 * part of the lower-order field (demagnetization and anisotropy),
 *   gbar  <- gbar - [v x mu_v + C_hat (-Delta_N) mu_v + lam mu_v - v mu_lam
 *                    - (1 + alpha^2) L_low mu_v]
 *   hbar_field   += (1 + alpha^2) mu_v            (3 planes, may be NULL)
 *   hbar_uniform += (1 + alpha^2) sum_i mu_v,i    (3 host doubles, may be NULL)
 * m_n, v, lam: the forward step's input magnetization, velocity and
 * multiplier.  gbar: in dL/dm^{n+1}, out dL/dm^n.
 * The solve: without a lower-order field (demag = aniso_k = 0) and with
 * opts->orth = 0, GMRES right-preconditioned by M^{-T} in one pipeline per
 * iteration, using J^T = calH + N with N node-wise:
 *   J^T M^{-T} = [I + (N - shift I)(calH + shift I)^{-1}] (calS + shift I)^{-T};
 * otherwise left-preconditioned GMRES on M^{-T} J^T (two pipelines per
 * iteration).  Either is accepted on the true residual ||(k gbar, 0) - J^T mu||.
 * Synchronizes. */
llg_status llg_step_midpoint_adjoint(llg_ctx* ctx, const llg_params* prm, const double* m_n, const double* v,
                                     const double* lam, double* gbar, double* hbar_field, double* hbar_uniform,
                                     const llg_solver_opts* opts, llg_solver_stats* stats, void* work,
                                     size_t work_bytes, void* stream);

/* Right-hand side of one time step (Sec. 2.4, eq. "total system"):
 * b = (C_hat Delta_N m + (1 + alpha^2) h_low(m), 0), the Euler form with the
 * lower-order field evaluated at m (the applied field alone when demag =
 * aniso_k = 0).  m: 3 planes; b: 4 planes (last plane zeroed).
 * Asynchronous. */
llg_status llg_rhs(llg_ctx* ctx, const llg_params* prm, const double* m, double* b, void* stream);

/* Discrete energy g_N(m) = |Omega|/N_g sum_i [cexc/2 m_i.(-Delta_N m)_i
 *   - demag/2 m_i.h_dem[m]_i + aniso_k (1 - (e.m_i)^2) - m_i.h_i]
 * (exchange, demagnetization, anisotropy, Zeeman; Sec. 2.1 and Sec. 3.3,
 * Proposition on the energy law; divide by |Omega| for the normalized energy
 * of Sec. 4.6).  Result to the host double *energy.  One pipeline whose last
 * pass reduces the energy density; allocates nothing.  Synchronizes. */
llg_status llg_energy(llg_ctx* ctx, const llg_params* prm, const double* m, double* energy, void* stream);

/* Instrumentation: per-kernel timing with HIP events.
 * llg_profile_enable(ctx, 1) clears the record and from then on brackets
 * every kernel the context launches with a pair of HIP events recorded on the
 * launch stream, together with the algorithmic bytes of that launch (one
 * read of its inputs and one write of its outputs); llg_profile_enable(ctx,
 * 0) stops recording.  llg_profile_read synchronizes the recorded events and
 * fills up to max_entries per-kernel totals, returning the number of kernel
 * kinds seen (or -1 on error).  name points to a static string. */
typedef struct {
  const char* name;
  int launches;
  double total_ms;
  double bytes;
} llg_kernel_profile;

llg_status llg_profile_enable(llg_ctx* ctx, int enable);
int llg_profile_read(llg_ctx* ctx, llg_kernel_profile* out, int max_entries);

/* Restrict the recording to the kernel kinds named in `kinds`, a
 * comma-separated list of the names llg_profile_read reports (e.g.
 * "cgs_update_dots,cgs_dots"); NULL or "" selects every kind (the default).
 * Fewer bracketed launches means less event overhead in a timed region.
 * Errors: LLG_EARG (null context, unknown name; selection unchanged). */
llg_status llg_profile_select(llg_ctx* ctx, const char* kinds);

/* Message describing the last error on this thread ("" if none). */
const char* llg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LLG_H */
