/*
 * tem.h -- C ABI of the MI355X (gfx950) library for transient electromagnetic
 * forward modelling with a shared-pole rational approximant of exp(-t M^-1 K).
 *
 * The method (Borner & Guttel, "Fast parallel transient electromagnetic
 * modeling using a uniform-in-time approximation to the exponential"):
 *   eq. (ode):   K u + M u' = 0,  M u(0) = f   (curl-curl stiffness K, conductivity
 *                mass M, loop source f; Sec. 2.2)
 *   eq. (expm):  u(t) = exp(-t M^-1 K) b,  b = M^-1 f
 *   eq. (ratfam) and (rmj):  one set of poles xi_i for all channels t_k,
 *                u(t_k) ~ Re sum_j c_j(t_k) x_j,   (K - xi_j M) x_j = f,
 *   with c_j(t_k) = 2 alpha_j^[k] for a conjugate pair and alpha_j^[k] for a
 *   real pole, and all channels formed at once as the product S R (Sec. 3.2).
 *
 * Discretization: a tensor grid of nx*ny*nz hexahedral cells with one unknown
 * per edge (tangential E at the edge midpoint, lumped mass), PEC walls.
 *
 * Conventions shared by every entry point:
 *   - cells (i, j, k) with x fastest; k = 0 is the bottom layer, z points up;
 *     per-cell arrays are [nz][ny][nx];
 *   - "storage edge order": Ex[nz+1][ny+1][nx], then Ey[nz+1][ny][nx+1], then
 *     Ez[nz][ny+1][nx+1], x fastest; n_storage = sum of the three; boundary
 *     edges are present and zero;
 *   - all floating point is IEEE binary64 unless stated;
 *   - complex arrays are interleaved (re, im) pairs of doubles;
 *   - pointers are host pointers unless the argument says "device";
 *   - the caller owns every buffer it passes; the context owns its device
 *     workspace and frees it in tem_destroy;
 *   - every call is ordered on the context's HIP stream; calls that return
 *     host data synchronize that stream before returning;
 *   - one context must not be used by two threads at once.
 *
 * Errors: every int-returning call returns TEM_OK (0) or a negative status
 * below; tem_last_error gives a message.  On error the outputs are
 * unspecified, except that TEM_ENOCONV still fills the stats and the outputs
 * from the best iterate.
 */
#ifndef TEM_H
#define TEM_H

#ifdef __cplusplus
extern "C" {
#endif

#define TEM_MAX_SHIFTS 64

enum tem_status {
  TEM_OK = 0,
  TEM_EINVAL = -1,      /* invalid argument (sizes, non-finite or non-positive values, geometry) */
  TEM_ENOMEM = -2,      /* device allocation failed or request exceeds the device budget */
  TEM_ENOCONV = -3,     /* a shifted system did not reach rtol within max_iter */
  TEM_EBREAKDOWN = -4,  /* Krylov breakdown (zero or non-finite recurrence coefficient) */
  TEM_EHIP = -5,        /* a HIP runtime call failed */
  TEM_ESTATE = -6       /* call out of order (e.g. adjoint without a matching forward) */
};

/* flags for tem_set_conductivity */
#define TEM_SIGMA_LOG 1     /* input is ln(sigma) instead of sigma */
#define TEM_DEVICE_PTR 2    /* input/output pointer is a device pointer */

typedef struct tem_ctx tem_ctx;

/* Rectangular transmitter loop on node lines of the surface node plane k_s:
 * corners at nodes (i0, j0) and (i1, j1), 0 < i0 < i1 < nx, 0 < j0 < j1 < ny,
 * current `current` [A] counter-clockwise seen from +z.  Its source vector is
 * f_e = current * l_e * (+-1) on the loop edges (Sec. 2.1 step-off source,
 * f = (q, Phi) of Sec. 2.2). */
typedef struct { int i0, i1, j0, j1; double current; } tem_loop;

/* Receiver on the surface z-face of cell column (i, j) in node plane k_s,
 * 0 <= i < nx, 0 <= j < ny.  It records dB_z/dt = -(curl e)_z =
 * -(circulation of e around the face)/(face area) (Sec. 5 observation). */
typedef struct { int i, j; } tem_receiver;

typedef struct {
  int precision;     /* 0: FP64 Krylov sweeps.  1: the multi-shift sweep keeps the complex
                        per-shift search directions p_j in FP32 (the iterates x_j, the shared
                        real seed recurrence and its residuals stay FP64) and stops at a
                        recursive scaled residual of 1e-10; FP64 residuals rho_j then drive
                        refinement passes, each a batched COCG with complex FP32 vectors on
                        (K + s_j M) d_j = rho_j to a 1e-2 reduction and x_j += omega_j d_j in
                        FP64 with the step omega_j minimizing the FP64 residual, so no pass
                        raises it.  Every pass is bounded (8192 COCG iterations per shift, and
                        a shift whose correction stops improving by 10% over 1024 iterations
                        stops early); a shift whose FP64 residual falls by less than 10% in a
                        pass is not refined further.  Contraction and receivers are FP64. */
  double rtol;       /* per-shift target in the scaled system y = M^1/2 x, g = M^-1/2 f:
                        precision 0 stops shift j when |zeta_j| ||r||_2 <= rtol ||g||_2
                        (<= 0 selects 1e-12); precision 1 refines until the FP64 residual
                        ||g - (A + s_j) y_j||_2 <= rtol ||g||_2 (<= 0 selects 1e-5; with
                        1e-8 S/m air FP32 corrections stop improving near 1e-6) */
  int max_iter;      /* cap on seed iterations per solve; <= 0 selects 2000000 */
  int block;         /* iterations between deferred shift updates (8, 16, 32 or 64; other
                        values round down); <= 0 selects 64 */
  double seed_shift; /* real seed shift of the shared recurrence; <= 0 selects
                        max(min_j Re s_j, 1e-3 min_j |s_j|), s_j = -xi_j */
  int refine_max;    /* precision 1: cap on refinement passes; <= 0 selects 8; a shift
                        still above rtol after the cap gives TEM_ENOCONV */
  int keep_solutions;/* nonzero: keep X on the device for tem_adjoint / tem_solutions */
  int profile;       /* nonzero: one solver block in 16 is issued as direct launches whose
                        dispatches record HIP events (fills kernel_ms / kernel_launches of
                        tem_stats with the sampled launches); results are unchanged */
  int method;        /* 0: the shifted iterates x_j and directions p_j are kept on the device
                        (J complex vectors each) and updated every block.  1: two-pass form
                        with no per-shift vectors: pass 1 runs the shared seed recurrence
                        alone, recording its coefficients and the receiver values of its
                        residuals, and the data follow from the shifted recurrences replayed
                        on the host (one pass when no fields are requested); with fields,
                        pass 2 regenerates the residuals bitwise and accumulates every
                        channel as (entries x 64) x (64 x T) FP64 MFMA products.  Method 1 is
                        FP64 only, keeps no solutions (keep_solutions must be 0) and reports
                        no true residuals (-1). */
} tem_solve_opts;

/* kernel classes reported by tem_stats.kernel_ms */
#define TEM_K_STENCIL 0     /* seed stencil: p = r + beta p; q = (A + s0) p; (p, q).  In the one-kernel
                               form (the default) the whole seed step: r -= alpha q; p = r + beta p;
                               q = (A + s0) p; four inner products */
#define TEM_K_UPDATE 1      /* seed update: r -= alpha q; (r, r) (two-kernel form only) */
#define TEM_K_BLOCK 2       /* deferred shift update of x_j, p_j every block */
#define TEM_K_OTHER 3       /* init, true residual, contraction, receivers */

typedef struct {
  int iterations;                       /* seed iterations of the last source */
  int converged;                        /* 1 if every shift met rtol */
  int n_shifts;
  int iters_per_shift[TEM_MAX_SHIFTS];  /* iterations while shift j was active (last source) */
  double est_res[TEM_MAX_SHIFTS];       /* |zeta_j| ||r|| / ||g|| at the stop (last source) */
  double true_res[TEM_MAX_SHIFTS];      /* FP64 ||g - (A + s_j) y_j|| / ||g|| (last source) */
  int refine_passes;                    /* precision 1 */
  double seconds;                       /* wall time of the call */
  double unknown_updates;               /* sum over sources and shifts of n * active iterations */
  double kernel_ms[4];                  /* with opts->profile: summed HIP-event time per kernel class */
  long long kernel_launches[4];         /* with opts->profile: launches per kernel class */
} tem_stats;

/* Create a context for an nx*ny*nz grid with cell widths hx[nx], hy[ny], hz[nz]
 * [m] (all > 0 and finite) and the ground surface at node plane k_surface
 * (0 < k_surface < nz).  The grid plays the role of the mesh T_h of Sec. 2.2
 * (a tensor grid of hexahedra with edge unknowns instead of the paper's
 * tetrahedra), inside the PEC box of the Sec. 2.1 boundary condition.  device: HIP device ordinal.  hip_stream: a hipStream_t
 * cast to void*, or NULL for the default stream.  On success *ctx owns device
 * memory for the operator coefficients; no conductivity is set yet.  Grids
 * whose real edge field 3 (nx+1)(ny+1)(nz+1) doubles reaches 4 GiB (about
 * 560^3 cells) return TEM_EINVAL. */
int tem_setup_grid(tem_ctx **ctx, int nx, int ny, int nz,
                   const double *hx, const double *hy, const double *hz,
                   int k_surface, int device, void *hip_stream);

/* Set the per-cell conductivity sigma[nz][ny][nx] [S/m] (or ln sigma with
 * TEM_SIGMA_LOG), which defines the lumped mass M (Sec. 2.2, [M]_ij =
 * (sigma Phi_j, Phi_i)).  Values must be finite and sigma > 0.  With
 * TEM_DEVICE_PTR the array is read from device memory.  Invalidates any
 * stored forward state. */
int tem_set_conductivity(tem_ctx *ctx, const double *sigma, int flags);

/* Shared poles and residues for the channels t[T] (t > 0, finite) by RKFIT
 * (Sec. 3.2, eq. (ratfam), objective eq. (rkfit) with weights w[T], NULL ->
 * all 1).  degree: the number of poles m-hat (2..2*TEM_MAX_SHIFTS); 0 picks
 * the Table 1 degree for tol and the ratio max(t)/min(t).  Outputs, for the
 * J <= J_max poles kept (one per conjugate pair, with Im > 0, then the real
 * poles):
 *   xi[2*J]    the poles xi_j (re, im) [1/s];
 *   c[2*J*T]   c_j(t_k) at c[2*(j*T + k)] (re, im) with the factor 2 of a
 *              pair folded in, so u(t_k) = Re sum_j c_j(t_k) x_j;
 *   err[T]     eq. (error): max_{x>=0} |exp(-t_k x) - r^[k](x)| (may be NULL).
 * Host only; uses no device. */
int tem_poles(int T, const double *t, const double *w, int degree, double tol,
              int J_max, int *J, double *xi, double *c, double *err);

/* Single-time best approximation (Sec. 3.1): the type-[m/m] rational
 * function r_m(x) = alpha0 + sum_i alpha_i / (x - xi_i) with the smallest
 * uniform error to exp(-x) on x >= 0 (Halphen's 2 H^(-m-1/2) asymptotically,
 * Sec. 3.3; Table 1's first column gives m for a tolerance).  m in [1, 32];
 * beyond m = 14 the error stays at the FP64 floor (about 2e-14).  Outputs,
 * for the J <= m poles kept (one per conjugate pair, with Im > 0, then the
 * real poles: J = ceil(m/2) while the poles pair up, as they do up to
 * m = 14), in host arrays of 2*m doubles the caller owns:
 *   xi[2*J]   the poles xi_j (re, im) of r_m in the variable x = t lambda;
 *   a[2*J]    the residues with the factor 2 of a pair folded in, so
 *             r_m(x) = alpha0 + Re sum_j a_j / (x - xi_j);
 *   alpha0    the constant term (r_m at infinity);
 *   err       the uniform error (may be NULL).
 * Host only; uses no device.  Returns TEM_EINVAL for m out of range. */
int tem_poles_single(int m, int *J, double *xi, double *a, double *alpha0, double *err);

/* Forward model (Sec. 3.2): for each of the n_src loops, solve the J shifted
 * complex-symmetric systems (K - xi_j M) x_j = f on the device and form
 *   data[(s*T + k)*n_rx + r] = dB_z/dt at receiver r, channel k   [T/s]  (host)
 *   fields (optional, device, NULL to skip): u(t_k) in storage edge order at
 *          fields[(s*T + k)*n_storage + e]                          [V/m]
 * xi[2*J] and c[2*J*T] are as produced by tem_poles (host).  opts may be NULL
 * (defaults), stats may be NULL.  With opts->keep_solutions the solutions of
 * every source stay on the device for tem_adjoint and tem_solutions. */
int tem_forward(tem_ctx *ctx, const tem_loop *src, int n_src,
                const tem_receiver *rx, int n_rx, int T, int J,
                const double *xi, const double *c, const tem_solve_opts *opts,
                double *data, double *fields, tem_stats *stats);

/* Single-time forward model (Sec. 3.1, eq. (rba)): for each of the n_src
 * loops and every channel t_k, k < T (t[T] > 0, host),
 *   u(t_k) = alpha0 b + Re sum_j a_j (t_k K - xi_j M)^-1 f,   b = M^-1 f,
 * with (xi, a, alpha0, J) as produced by tem_poles_single (host arrays of
 * 2*J doubles, J in [1, 32]).  Every channel has its own J shifted systems,
 * (K + s M) x = f / t_k with s = -xi_j / t_k, J*T in all; they share one
 * multi-shift seed recurrence when J*T <= 320, else they are sorted by |s|
 * and cut into equal sweeps of at most 320 shifts (64 when the context is
 * attached to a solve engine), and they are contracted with the coefficients
 * a_j / t_k on the device.  Outputs as for tem_forward: data
 * (host, may be NULL with n_rx = 0) and fields (device, NULL to skip) at
 * fields[(s*T + k)*n_storage + e].  FP64 only: opts->precision and
 * opts->method must be 0 and opts->keep_solutions 0 (TEM_EINVAL otherwise);
 * rtol, max_iter, block and seed_shift apply to every sweep.  Device memory:
 * (J*T + 1) complex vectors per concurrent source (up to 4).  stats: n_shifts
 * = J*T; iterations = seed iterations of the last source summed over its
 * sweeps; iters_per_shift[k], est_res[k] and true_res[k] hold, per channel k,
 * the maxima over that channel's J systems of every source.  No adjoint or
 * Jacobian follows this call (they return TEM_ESTATE). */
int tem_forward_single(tem_ctx *ctx, const tem_loop *src, int n_src,
                       const tem_receiver *rx, int n_rx, int T, const double *t,
                       int J, const double *xi, const double *a, double alpha0,
                       const tem_solve_opts *opts, double *data, double *fields,
                       tem_stats *stats);

/* Adjoint (Sec. 4): given w[(s*T + k)*n_rx + r] = dphi/d data (host) for the
 * last tem_forward call, compute
 *   grad[c] = dphi/d ln sigma_c = -Re sum_s sum_j s_j lambda_j^T (dM/d ln sigma_c) x_j,
 *   (K + s_j M) lambda_j = sum_k c_j(t_k) Q^T w_k,  s_j = -xi_j,
 * for every cell c (grad[nz*ny*nx], host).  The forward solutions x_j are
 * the ones kept by a forward with keep_solutions; without it they are
 * recomputed here source by source (one more FP64 multi-shift solve per
 * source, holding one source's solutions instead of all), with the same
 * result for a precision-0 forward.  Returns TEM_ESTATE if no forward ran
 * since the last tem_set_conductivity. */
int tem_adjoint(tem_ctx *ctx, const double *w, double *grad_log_sigma, tem_stats *stats);

/* Jacobian action (Sec. 4, "Using iterative solvers": the action J x that
 * CGLS needs beside J^T y, which tem_adjoint gives): for a change dm[c] of
 * ln sigma per cell ([nz][ny][nx], host), the first-order change of the data
 * of the last tem_forward,
 *   ddata[(s*T + k)*n_rx + r] = Re sum_j c_j(t_k) q_r . dx_j   (host),
 *   (K + s_j M) dx_j = -s_j (dM/d ln sigma . dm) x_j,   s_j = -xi_j,
 * where dM/d ln sigma_c = sigma_c V_c / 4 on the 12 edges of cell c.  The J
 * sensitivity systems have different right-hand sides and are solved by one
 * batched FP64 COCG per source.  Needs the forward's solutions
 * (keep_solutions), else TEM_ESTATE. */
int tem_jacobian_apply(tem_ctx *ctx, const double *dm, double *ddata, tem_stats *stats);

/* Copy the stored solutions x_j of source s (storage edge order, complex):
 * X[2*(j*n_storage + e)] (re, im), host.  Needs keep_solutions. */
int tem_solutions(tem_ctx *ctx, int s, double *X);

/* Apply the shifted operator: y = (K + shift M) x for a complex vector x in
 * storage edge order (host, interleaved); boundary entries of x are ignored
 * and those of y are zero.  For operator checks. */
int tem_apply(tem_ctx *ctx, double shift_re, double shift_im, const double *x, double *y);

/* The operator of tem_apply, y = (K + shift M) x, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no allocating routine.
 *   x, y   DEVICE pointers to n_storage complex values each (interleaved re, im,
 *          storage edge order), owned by the caller; they must not alias.
 *          Boundary entries of x are ignored; those of y are written as zero.
 * Staging lives in one fixed device array of 64 MiB per GPU (held until the
 * process ends), which must hold 2 * 3 (nx+1)(ny+1)(nz+1) * 16 + 256 bytes:
 * larger grids (about 87^3 cells and up) return TEM_EINVAL without launching
 * anything.  The array is shared by every call on that GPU and keeps the last
 * call's contents, so calls that overlap on one GPU (other threads, streams or
 * contexts) race: serialize them.  Work is ordered after the context's stream
 * and the context's stream is made to wait for it; the call does not
 * synchronize.  Results equal tem_apply's. */
int tem_apply_noalloc(tem_ctx *ctx, double shift_re, double shift_im, const double *x, double *y);

/* Solve engine (serving, form 5): a worker thread on `device` that advances
 * the multi-shift solves of every context attached to it together, in
 * batched launches replayed as HIP graphs: per seed iteration one stencil
 * launch and one update launch cover the tiles of every job (the loop sources
 * and adjoint receiver rows of all attached contexts' calls in progress), and
 * per 64 iterations one shift-block and one block-update launch cover all
 * their poles.  Jobs join and leave at 64-iteration boundaries.  The poles of
 * all systems are independent work (Sec. 3.2, eq. (rmj); Sec. 5.3 runs them
 * in parallel processes); here several requests' poles share every launch.
 * max_jobs: jobs per batch (1..16, <= 0 selects 16); more wait for a place.
 * Each job's arithmetic (tiles, reductions and their order) does not depend
 * on the other jobs in its batch, so results are bitwise the same alone or
 * batched.  FP64 sweeps only: precision-1 calls of attached contexts run
 * their own launches.  Destroy an engine only after every call of its
 * attached contexts has returned. */
typedef struct tem_engine tem_engine;
int tem_engine_create(tem_engine **eng, int device, int max_jobs);

/* Route the FP64 multi-shift solves of ctx (forward and adjoint) through eng
 * (NULL detaches).  ctx and eng must be on the same device.  Calls on ctx stay
 * synchronous for its caller; several threads, each with its own context,
 * share the engine.  A solve through the engine always uses 64-iteration
 * blocks (tem_solve_opts.block and .profile are ignored).  Only grids with
 * fewer 64 x 8 x 2-node seed tiles than the device has compute units (on a
 * 256-CU MI355X, cubes up to 56^3 cells) use the engine; solves of larger
 * grids fill the device alone and keep their own launches, whether or not an
 * engine is attached. */
int tem_attach_engine(tem_ctx *ctx, tem_engine *eng);

/* Batching statistics: blocks launched, job-blocks (sum over blocks of the jobs
 * in each), the most jobs and the most distinct contexts in one block. */
int tem_engine_stats(tem_engine *eng, long long *blocks, long long *job_blocks, int *max_jobs,
                     int *max_contexts);

void tem_engine_destroy(tem_engine *eng);

/* Sizes: n_storage edges and n interior unknowns of the context's grid. */
int tem_sizes(const tem_ctx *ctx, long long *n_storage, long long *n_unknowns);

void tem_destroy(tem_ctx *ctx);

/* Message of the last failing call on ctx (or of the last failing
 * context-less call when ctx is NULL).  Valid until the next call. */
const char *tem_last_error(const tem_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* TEM_H */
