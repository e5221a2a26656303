/*
 * biot_mg.h -- C ABI of the MI355X (gfx950) monolithic multigrid solver for the
 * reduced-quadrature (RQ) three-field Biot system of Adler, He, Hu, MacLachlan and Ohm,
 * "Monolithic multigrid for a reduced-quadrature discretization of poroelasticity"
 * (arXiv:2107.04060).
 *
 * Problem (Sec. 2.1, eqs. discrete1-discrete3, block_form; Sec. 2.3, block_form_rq):
 * one backward-Euler step of Biot's model on the unit square, uniform n x n mesh with
 * every square cut from its top-left to its bottom-right corner (Appendix A), spaces
 * P1 + face bubbles (displacement u), RT0 (Darcy velocity w), P0 (pressure p); the
 * symmetric saddle-point matrix
 *     A = [[A_u^RQ, 0, alpha B_u^T], [0, tau M_w, tau B_w^T], [alpha B_u, tau B_w, -(1/M) M_p]]
 * with A_u^RQ = 2 mu A_eps + lambda B_u^T M_p^{-1} B_u (Appendix A), Dirichlet data u = 0
 * and w.n = 0 on the whole boundary (those DoFs are eliminated), or the mixed conditions of
 * Terzaghi's column (Sec. 5; biot_problem.bc).
 *
 * Solver (Sec. 3 and 5.1): FGMRES (right preconditioned, flexible, from x0 = 0 or a given guess) with one
 * monolithic geometric-multigrid V(nu1, nu2) cycle as preconditioner: rediscretized
 * coarse operators, block prolongation diag(P_u, P_w, P_p) with the divergence-
 * preserving P_u of Sec. 3.1, restriction P^T, additive Vanka (Sec. 3.2.1) or inexact
 * Braess-Sarazin (Sec. 3.2.2, Appendix D) relaxation, exact solve on the coarsest mesh.
 *
 * Vector layout.  Every vector crossing this ABI is a DEVICE pointer to FP64 values in
 * the canonical free-DoF order of its mesh level (n_l = n >> l cells per side):
 *     [u_x(interior vertices), u_y(interior vertices), b_H, b_V, b_D (interior edges),
 *      w_H, w_V, w_D (interior edges), p_L, p_U]
 * each block row-major in (j, i); H(i,j) is the edge (i,j)-(i+1,j) with unit normal +y,
 * V(i,j) the edge (i,j)-(i,j+1) with normal +x, D(i,j) the diagonal (i,j+1)-(i+1,j)
 * with normal (1,1)/sqrt(2); L(i,j) = {(i,j),(i+1,j),(i,j+1)}, U(i,j) = {(i+1,j),
 * (i+1,j+1),(i,j+1)}.  Length 10 n^2 - 8 n + 2 (BIOT_BC_TERZAGHI: biot_problem.bc).  Bubble DoFs are normal displacements
 * at edge midpoints (basis 4 l_p l_q n_e), RT0 DoFs normal fluxes (normal component 1).
 * Per-triangle arrays are ordered [L(j n + i) for all cells, then U(j n + i)].
 *
 * Ownership.  The caller allocates and owns every pointer it passes; the library never
 * frees caller memory and keeps no caller pointer after a call returns.  All device work
 * of a call is enqueued on `stream` (a hipStream_t, NULL = default stream); calls return
 * after enqueueing unless stated otherwise (solve synchronizes with the stream once per
 * FGMRES iteration to read the Hessenberg column).  A context is not thread safe; several
 * contexts may coexist; contexts on different streams may run concurrently from different
 * host threads.  Device memory is allocated by biot_assemble and biot_setup_hierarchy, and
 * by the first biot_solve with a given restart length m (the Krylov workspace: 2 m + 4
 * finest-level FP64 vectors and a few scalars, kept for later solves with restart <= m);
 * biot_solve_noalloc allocates nothing (it works in a fixed device array of the library);
 * biot_export_layout, a diagnostic call, allocates and frees a temporary buffer.
 *
 * Errors.  Every int-returning function returns one of the BIOT_* codes below and, on
 * failure, leaves a message for biot_last_error().  No C++ exception crosses the ABI.  An
 * invalid argument is rejected before anything changes, and after BIOT_ERR_NAN from
 * biot_solve (NaN or Inf in the right-hand side or met during the iteration) the context
 * stays valid for further solves.
 */
#ifndef BIOT_MG_H
#define BIOT_MG_H

#ifdef __cplusplus
extern "C" {
#endif

#define BIOT_OK 0
#define BIOT_NOT_CONVERGED 1      /* solve: maxit reached; x holds the last iterate      */
#define BIOT_ERR_ARG (-1)         /* invalid argument (message says which)               */
#define BIOT_ERR_HIP (-2)         /* a HIP runtime call failed                            */
#define BIOT_ERR_OOM (-3)         /* device allocation failed                             */
#define BIOT_ERR_SINGULAR (-4)    /* zero / non-positive pivot in a setup factorization   */
#define BIOT_ERR_NAN (-5)         /* NaN or Inf met in the Krylov iteration               */

#define BIOT_SMOOTHER_VANKA 0     /* additive Vanka, 20-DoF vertex patches (Sec. 3.2.1)  */
#define BIOT_SMOOTHER_BSR 1       /* inexact Braess-Sarazin (Sec. 3.2.2, Appendix D)     */

#define BIOT_BC_DIRICHLET 0      /* u = 0 and w.n = 0 on the whole boundary (Sec. 5.1)  */
#define BIOT_BC_TERZAGHI 1       /* Terzaghi's column (Sec. 5): see biot_problem.bc       */

#define BIOT_PREC_FP64 0          /* whole preconditioner in FP64                         */
#define BIOT_PREC_FP32_SMOOTHER 1 /* V-cycle vectors, residuals and transfers in FP32;
                                     patch solves and the coarsest solve in FP64 arithmetic;
                                     FGMRES and its true residual in FP64                  */
#define BIOT_PREC_FP32_PATCH 2    /* as BIOT_PREC_FP32_SMOOTHER, and the variable-K Vanka
                                     patch eliminations in FP32 arithmetic as well (faster:
                                     half the registers).  Their error is FP32 roundoff times
                                     the conditioning of the patch blocks: fine for moderate
                                     permeability contrast, not for strong contrast (1e6)
                                     with near-incompressibility, where the cycle stops
                                     being a usable preconditioner; use
                                     BIOT_PREC_FP32_SMOOTHER there.  Constant K and BSR are
                                     as in BIOT_PREC_FP32_SMOOTHER.                        */

typedef struct biot_ctx biot_ctx;

/* Physical and discretization parameters of one time step (Sec. 2, 2.1). */
typedef struct {
    int n;              /* cells per side of the finest mesh; power of two, 4 <= n <= 8192 */
    double lambda;      /* Lame lambda >= 0                                                 */
    double mu;          /* Lame mu > 0                                                      */
    double alpha;       /* Biot-Willis coefficient (any real, usually in (0, 1])           */
    double inv_M;       /* 1/M, reciprocal Biot modulus; > 0                                */
    double mu_f;        /* fluid viscosity > 0                                              */
    double tau;         /* time step > 0                                                    */
    double K_scalar;    /* permeability used when K_tri == NULL; > 0                        */
    const double* K_tri;/* device pointer to 2 n^2 per-triangle permeabilities (> 0), or NULL;
                           read during biot_assemble only, checked on the device as in
                           biot_update_K                                                     */
    int bc;             /* boundary conditions (0 = BIOT_BC_DIRICHLET, as above).
                           BIOT_BC_TERZAGHI: the column of Sec. 5 (Terzaghi's problem), loaded and
                           drained on x = 0 (natural: u, the bubbles and w.n of that face are
                           free; the traction and the zero pressure enter through the right-hand
                           side), fixed and impermeable on x = 1 (u = 0, w.n = 0), rollers on
                           y = 0 and y = 1 (u_y = 0, bubble and w.n of their edges 0).  The
                           canonical order is then [u_x (vertices with i < n), u_y (i < n,
                           0 < j < n), b_H (0 < j < n), b_V (i < n), b_D (all), w_H, w_V, w_D (as
                           b), p_L, p_U], each block row-major in (j, i): the full numbering with
                           the eliminated DoFs skipped, length 10 n^2 - 2 n.  1/M = 0 (M =
                           infinity) is allowed, n <= 256.  This path runs on compressed-row
                           operators and explicit patch inverses (natural boundaries break the
                           translation-invariant stencil of the Dirichlet path): additive Vanka in
                           FP64 only; biot_solve_noalloc, biot_grad_logK, biot_kernel_timing and
                           the patch table of biot_export_layout return BIOT_ERR_ARG.          */
} biot_problem;

/* Multigrid options (Sec. 3, 4.3, 5.1). */
typedef struct {
    int levels;         /* mesh levels incl. the finest, >= 2; coarsest n >> (levels-1) >= 2 */
    int smoother;       /* BIOT_SMOOTHER_VANKA or BIOT_SMOOTHER_BSR                          */
    int nu1, nu2;       /* pre / post smoothing steps, 0..16                                 */
    double omega;       /* outer relaxation weight (Vanka and BSR)                           */
    double omega_J;     /* BSR: weighted-Jacobi weight on the approximate Schur complement   */
    int precision;      /* BIOT_PREC_FP64, BIOT_PREC_FP32_SMOOTHER or BIOT_PREC_FP32_PATCH    */
    int schur_sweeps;   /* BSR: 0 or 1 = the single weighted-Jacobi step with omega_J on the
                           approximate Schur complement (Sec. 3.2.2); k in 2..64 = k Jacobi
                           sweeps with weight omega_S from zero instead, a short inner
                           iteration towards exact BSR (two more launches per sweep level-wide,
                           more robust for small K and nu near 1/2)                         */
    double omega_S;     /* BSR with schur_sweeps >= 2: weight of the sweeps, in (0, 1]       */
    int gamma;          /* cycle index, 0 or 1 = V-cycle, 2 = W-cycle, up to 4: the coarse
                           correction of each level is gamma cycles of the next, each further
                           one on the residual the previous ones left (the coarsest direct
                           solve is not repeated); more robust BSR for small K (Sec. 5.1)   */
    int vanka_colors;   /* Vanka: 0 = additive (Sec. 3.2.1, weights D_l); 4 = multiplicative in
                           four colours (i mod 2) + 2 (j mod 2) of the patch vertex, each colour
                           on the residual the previous one left, unweighted (a colour's patches
                           share no DoF); four launches per smoothing step; 3 = the same in
                           three colours (i + 2 j) mod 3, the fewest this triangulation allows
                           (patches share DoFs only across mesh edges): three launches     */
    int schur_cg;       /* BSR: 0 = as schur_sweeps says; k in 1..64 = the pressure correction
                           from k steps of conjugate gradients on the approximate Schur complement
                           S_hat = c_u M_p + tau B_w D_w^{-1} B_w^T (symmetric positive definite),
                           preconditioned by diag(S_hat), from zero: exact BSR (Sec. 3.2.2) in the
                           limit.  Five launches per CG step and level, dot products reduced on
                           the device in a fixed order (no host synchronization).  Excludes
                           schur_sweeps >= 2.                                                 */
    int gamma_from;     /* with gamma >= 2: only levels l >= gamma_from (0 = finest) repeat their
                           coarse correction gamma times, finer levels take one; 0 = every level
                           (the W-cycle).  A W-cycle below a V-cycle: the coarse levels, cheap in
                           bytes, are revisited, the fine ones are not.                        */
    int fcycle;         /* with gamma >= 2: 0 = every further coarse correction is a cycle of
                           the same kind (W-cycle); 1 = the further ones are V-cycles, the
                           first one of the same kind (the F-cycle: below the first repeating
                           level, level m is visited m + 1 times rather than 2^m).  Neither is
                           the paper's V-cycle: both are standard multigrid cycle shapes.      */
    int gamma_to;       /* with gamma >= 2: 0 = no upper limit; k >= 1: levels l >= k take one
                           coarse correction again, so only gamma_from <= l < gamma_to repeat
                           (below gamma_to the cycle is a V-cycle, visited as often as level
                           gamma_to)                                                          */
    double vanka_shift; /* bc = BIOT_BC_TERZAGHI: every Vanka patch matrix is shifted on its
                           diagonal, + vanka_shift on the displacement and Darcy entries and
                           - vanka_shift on the pressure entries (a small compressibility; Sec. 5,
                           Terzaghi's problem, shifts the blocks by 1e-8 because with 1/M = 0 an
                           interior patch matrix is singular, so vanka_shift > 0 is required
                           there); 0 with BIOT_BC_DIRICHLET                                   */
    int csr_below;      /* 0 = off; k > 0 (Vanka, Dirichlet): the smoothing levels below the
                           finest with n_l <= k cells per side run on compressed-row operators and
                           explicit patch inverses instead of the fused stencil kernels (the same
                           operator, patches, colours and cycle; one short launch per colour step
                           where the fused stencil launch is bound by the latency of a single
                           block).  These levels compute in FP64 in every precision form (the
                           FP32 forms convert at the first of them).  A performance option: the
                           result is the same up to rounding.                                   */
    int additive_levels;/* with vanka_colors 3 or 4: the finest additive_levels levels take the
                           additive step (Sec. 3.2.1, weights D_l) instead of the colours, the
                           coarser ones the multiplicative form; 0 = every level multiplicative */
    double omega_additive; /* the weight of those additive levels; 0 = omega                   */
} biot_mg_opts;

/* FGMRES controls (in) and results (out). */
typedef struct {
    double tol;         /* in: stop when ||b - A x||_2 <= tol ||b||_2 (true residual; side 0)
                           or ||M^{-1}(b - A x)||_2 <= tol ||M^{-1} b||_2 (side 1)           */
    int restart;        /* in: Krylov dimension m per cycle, 1..200                          */
    int maxit;          /* in: maximum total iterations                                      */
    int iters;          /* out: iterations performed                                         */
    int converged;      /* out: 1 if the tolerance was met                                   */
    double rel_res_true;/* out: ||b - A x||_2 / ||b||_2 recomputed in FP64 at the end        */
    int side;           /* in: 0 = right-preconditioned flexible GMRES (Sec. 5.1; default);
                           1 = left-preconditioned GMRES on M^{-1} A x = M^{-1} b, stopping on
                           the preconditioned residual (a reading of the paper's "relative
                           residual" under which its Vanka iteration counts are reproduced; M,
                           one V-cycle, must then be a fixed linear operator, i.e. no
                           schur_cg)                                                          */
    double rel_res_prec;/* out (side 1): ||M^{-1}(b - A x)||_2 / ||M^{-1} b||_2 at the end   */
    double reorth;      /* in: the classical Gram-Schmidt step takes a second pass when the first
                           one cancels, |w_1| < eta |w_0| (the Daniel-Gragg-Kaufman-Stewart test);
                           eta = reorth in (0, 1], or 1/sqrt(2) when 0 (the default).  A smaller
                           eta skips the pass unless more digits cancel (eta = 0.01: two)      */
    int x0;             /* in: 0 = start from x = 0 (default); 1 = x holds the initial guess on
                           entry (canonical order).  The stopping test stays relative to ||b||
                           (side 0) or ||M^{-1} b|| (side 1), so a good guess saves iterations:
                           a time-stepping caller passes the previous step's solution, the
                           reading under which the paper's Table 5 counts are reproduced.
                           Other values are rejected (BIOT_ERR_ARG)                          */
} biot_solve_info;

/* Assemble the rediscretized operator on the finest mesh (Sec. 2.3, block_form_rq):
 * validates `prob`, allocates the context, uploads the stencil of the element matrices
 * and the per-triangle 1/K.  Returns the context in *out (NULL on failure). */
int biot_assemble(const biot_problem* prob, void* stream, biot_ctx** out);

/* Build the multigrid hierarchy (Sec. 3): per-level rediscretized operators with 1/K
 * averaged over the four children of each coarse triangle, transfer tables, Vanka /
 * BSR patch data, dense inverse of the coarsest operator (Sec. 5.1).  May be called
 * again with other options. */
int biot_setup_hierarchy(biot_ctx* ctx, const biot_mg_opts* opts, void* stream);

/* z = M^{-1} r: one V(nu1, nu2) cycle from a zero initial guess on the finest level.
 * r and z: device FP64, canonical order of the finest level; may not alias. */
int biot_vcycle(biot_ctx* ctx, const double* r, double* z, void* stream);

/* Solve A x = b by FGMRES preconditioned with biot_vcycle (Sec. 5.1), from x0 = 0 or, with
 * info->x0 = 1, from the guess x holds on entry.
 * b, x: device FP64, canonical order, may not alias.  info: host pointer (in/out).
 * Returns BIOT_OK, BIOT_NOT_CONVERGED (x = last iterate) or an error code. */
int biot_solve(biot_ctx* ctx, const double* b, double* x, biot_solve_info* info, void* stream);

/* biot_solve for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same FGMRES, the same kernels and the
 * same result as biot_solve, with the Krylov workspace ((2 m + 4) padded finest-level vectors
 * and the Gram-Schmidt partial sums) carved from a fixed 64 MiB device array that the library
 * holds on every GPU it runs on until the process ends, instead of from allocations.  No
 * hipMalloc, hipFree or other allocating call is made; the host reads the Gram-Schmidt results
 * by plain copies (no pinned memory).  Limits: restart m <= 32, and the padded finest level
 * must fit: (2 m + 4) ((n + 4) ceil((n + 4) / 16) 16 10) 8 bytes plus about 272 KB within 64 MiB
 * (n <= 64 at m = 32, n = 128 up to m = 19); larger requests return BIOT_ERR_ARG and change
 * nothing.  The array is shared by every call on one GPU and keeps the last call's contents
 * (each call clears what must start at zero): calls that overlap in time on one GPU, from
 * several threads or on several streams, race and must not be issued.  Arguments, ownership
 * and return codes as biot_solve; the context must have a hierarchy. */
int biot_solve_noalloc(biot_ctx* ctx, const double* b, double* x, biot_solve_info* info, void* stream);

/* y = A_l x on mesh level l (0 = finest): the rediscretized operator (block_form_rq). */
int biot_apply_operator(biot_ctx* ctx, int level, const double* x, double* y, void* stream);

/* One relaxation step on level l: x <- x + omega M_l^{-1} (b - A_l x) with the smoother
 * chosen in setup (Vanka: Sec. 3.2.1; BSR: Sec. 3.2.2).  x is updated in place. */
int biot_smooth(biot_ctx* ctx, int level, double* x, const double* b, void* stream);

/* r_c = P_l^T r_f: restriction from level l to level l+1 (Sec. 3, eq. block_interp). */
int biot_restrict(biot_ctx* ctx, int level, const double* r_f, double* r_c, void* stream);

/* x_f += P_l x_c: prolongation from level l+1 to level l, divergence preserving for u
 * (Sec. 3.1). */
int biot_prolong_add(biot_ctx* ctx, int level, const double* x_c, double* x_f, void* stream);

/* Re-assemble for new per-triangle permeabilities (Sec. 2.1: K enters the Darcy block
 * tau M_w(K) only): K_tri is a device pointer to 2 n^2 values.  Every value is checked on the
 * device first (K > 0, finite, 1/K finite and non-zero; the call synchronizes the stream for
 * the check); on failure BIOT_ERR_ARG is returned and nothing changes.  Then 1/K is updated
 * on every level, with the patch data and the coarsest inverse.  The hierarchy options stay. */
int biot_update_K(biot_ctx* ctx, const double* K_tri, void* stream);

/* As biot_update_K for the log-permeability theta_T = ln K_T (device pointer, 2 n^2 values;
 * checked on the device: finite with |theta| < 700): 1/K_T = exp(-theta_T) is formed on the
 * device, the parametrization whose derivative biot_grad_logK returns. */
int biot_update_logK(biot_ctx* ctx, const double* theta_tri, void* stream);

/* Per-triangle gradient of lambda^T A x with respect to theta_T = ln K_T, negated:
 *   g_T = -lam^T (dA/dtheta_T) x = tau mu_f exp(-theta_T) lam_w|_T^T M_w^T(K=1) w|_T,
 * the adjoint gradient of a loss L(x) when lam solves A lam = dL/dx (A is symmetric,
 * Sec. 2.1).  x, lam: canonical finest-level vectors; g_tri: 2 n^2 outputs. */
int biot_grad_logK(biot_ctx* ctx, const double* x, const double* lam, double* g_tri, void* stream);

/* Layout export (host memory): the mesh numbering of Sec. 2.1 (squares cut as Appendix A
 * draws them) and the 20-DoF vertex patches of Sec. 3.2.1 (Fig. patches, right), for checking
 * the library's index arithmetic against another implementation.
 * counts (optional, 12 ints): [n, n_free, 10 block sizes].
 * patch_table (optional, host, ((n+1)^2 - 2) x 20 ints): the 20-slot Vanka patch of every
 * vertex except (0,0) and (n,n), vertices in row-major (j, i) order, slots
 *   [ux(v), uy(v), b on H(i-1,j), H(i,j), V(i,j-1), V(i,j), D(i-1,j), D(i,j-1),
 *    w on the same six edges, p on L(i,j), L(i-1,j), L(i,j-1), U(i-1,j-1), U(i-1,j), U(i,j-1)]
 * holding canonical indices, -1 for absent or eliminated DoFs.  Computed on the device by
 * the same index arithmetic the Vanka kernels use, into a temporary device buffer of
 * ((n+1)^2 - 2) x 20 ints that this call allocates and frees (a diagnostic call: the one
 * exception to the allocation rule above).  Synchronizes the stream. */
int biot_export_layout(biot_ctx* ctx, int* counts, int* patch_table, void* stream);

/* Kernel timing with HIP events (instrumentation, not a step of the method: no passage of
 * the paper defines it; it measures the HBM traffic rate of the finest-level kernels).  The
 * first launches timed after enable = 1 create HIP events (host-side runtime objects, kept by
 * the context and reused); no device memory is allocated.
 * enable = 1: start recording an event pair around every launch, on mesh level `level`,
 *             of the fused residual + additive-Vanka step (steps on an iterate that is not
 *             identically zero and that do not also add the prolongated coarse correction)
 *             and of the fused residual + restriction kernel; previous records are
 *             dropped.  Events are recorded on `stream` of the calls that launch them.
 * enable = 0: stop, synchronize `stream` and write out[0..3] = {total Vanka milliseconds,
 *             number of Vanka launches, total residual milliseconds, number of residual
 *             launches} (out: host pointer, may be NULL). */
int biot_kernel_timing(biot_ctx* ctx, int enable, int level, double* out, void* stream);

/* Free every device allocation of the context (NULL is ignored). */
void biot_destroy(biot_ctx* ctx);

/* Message of the last failure on the calling thread ("" if none). */
const char* biot_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BIOT_MG_H */
