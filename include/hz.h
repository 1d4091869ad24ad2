/*
 * hz.h -- C ABI of the MI355X (gfx950) complex Helmholtz solver library.
 *
 * The library solves the finite-element Helmholtz system of the acoustic
 * part of the paper (Sec. 3.2: Fourier transform of the homogeneous wave
 * equation gives  -w^2 psi - c^2 lap(psi) = 0, discretised by finite
 * elements on the compartment mesh), with the solver components of its
 * Sec. 4: a CSR-type sparse matrix in complex double precision, a
 * sparse matrix-vector product, rewritten basic linear-algebra kernels,
 * preconditioned Krylov methods (BiCGStab; restarted GMRES is added), and
 * a non-overlapping Schwarz domain decomposition with Robin (absorbing)
 * transmission conditions.
 *
 * Discrete problem.  On Q1 (trilinear hexahedral) elements, with
 * k = 2 pi freq / c:
 *
 *     A(k) p = f,   A(k) = K - k^2 M + i k^2 M_eta + i k B_beta
 *
 *     K_ab      = int grad(phi_a).grad(phi_b)          (stiffness)
 *     M_ab      = int phi_a phi_b                      (mass)
 *     M_eta     = sum_e eta_e M_e                      (absorption field)
 *     B_beta    = sum_w beta_w B0_w, B0_w,ab = int_{wall w} phi_a phi_b
 *     f         = M_patch g   (Neumann data g on the source faces)
 *
 * beta_w is the normalised outward admittance of wall w (Re beta >= 0
 * absorbs), eta_e a per-element loss factor (element wavenumber squared
 * k^2 (1 - i eta_e)).  A is complex symmetric (A^T = A).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: HZ_OK (0) on success; > 0: a result was written but is
 *    flagged (not converged, breakdown); < 0: error, nothing was written.
 *    hz_last_error() gives a message for the calling thread.
 *  - Pointers named *_dev are device pointers (HIP global memory of the
 *    context's device), owned by the caller, contiguous, 16-byte aligned
 *    for complex data.  All other pointers are host pointers, owned by the
 *    caller, only read during the call unless stated.
 *  - Complex numbers are pairs of IEEE doubles (re, im), the element layout
 *    of std::complex<double> and torch.complex128.
 *  - Node ids and ordering of every vector are the caller's node order.
 *  - Work is ordered on the HIP stream given to hz_assemble (0 = the null
 *    stream).  Entry points that return an info struct or host scalars
 *    synchronise that stream before returning.
 *  - One context must not be used by two threads at the same time.
 */
#ifndef HZ_H_
#define HZ_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hz_c128;

typedef struct hz_ctx_s* hz_ctx;

enum {
  HZ_OK = 0,
  HZ_NOT_CONVERGED = 1,   /* best iterate written; tolerance not reached  */
  HZ_BREAKDOWN = 2,       /* best iterate written; Krylov breakdown       */
  HZ_ERR_INVALID = -1,    /* null pointer, bad size, NaN/Inf input        */
  HZ_ERR_HIP = -2,        /* HIP runtime error                            */
  HZ_ERR_OOM = -3,        /* device allocation failed                     */
  HZ_ERR_STATE = -4       /* call order violated (e.g. no frequency set)  */
};

enum { HZ_GMRES = 0, HZ_BICGSTAB = 1, HZ_SCHWARZ = 2, HZ_BICGSTABL = 3, HZ_TFQMR = 4 };
enum { HZ_FP64 = 0, HZ_MIXED = 1 };
enum { HZ_JACOBI = 0, HZ_NONE = 1 };
enum { HZ_ORDER_GIVEN = 0, HZ_ORDER_RCM = 1 };
enum { HZ_HEX8 = 0, HZ_TET4 = 1 };
enum { HZ_SRC_NEUMANN = 0, HZ_SRC_DIRICHLET = 1 };
enum { HZ_GALERKIN = 0, HZ_GLS = 1 };

/* Mesh of trilinear hexahedra (Q1) or linear tetrahedra (P1).  All arrays
 * are host arrays read during hz_assemble only.
 *   xyz       [n_nodes][3]   node coordinates (m)
 *   hex       [n_elems][8]   element nodes; hexahedra in tensor order:
 *                            local node a + 2 b + 4 c sits at reference
 *                            corner (2a-1, 2b-1, 2c-1).  [n_elems][4] for
 *                            tetrahedra (any vertex order)
 *   bface     [n_bfaces][4]  boundary quads, tensor order a + 2 b;
 *                            [n_bfaces][3] triangles for tetrahedra
 *   bface_tag [n_bfaces]     wall id 0..5 (x-, x+, y-, y+, z-, z+)
 *   bface_src [n_bfaces]     1 = the face carries the source (Neumann) datum
 *   c, rho                   speed of sound (m/s); rho is stored only
 *   parts[3]                 structured partition counts along x, y, z for
 *                            the Schwarz method (0 = not used); requires the
 *                            mesh to be a structured box with node id
 *                            i + (nx+1) (j + (ny+1) k) and elems[3] set
 *   elems[3]                 element counts of a structured box (or 0)
 *   order                    internal node numbering of the operator rows:
 *                            HZ_ORDER_GIVEN keeps the mesh's numbering,
 *                            HZ_ORDER_RCM renumbers by reverse Cuthill-McKee
 *                            (a narrow band for unstructured meshes, whose
 *                            node ids need not follow space)
 *   sigma                    0, or a multiple of 64 (at most 2^20): rows are
 *                            then sorted by length, longest first, within
 *                            windows of sigma consecutive internal rows, so
 *                            that each 64-row slice of the sliced-ELL storage
 *                            holds rows of nearly equal length (SELL-C-sigma)
 *   elem_type                HZ_HEX8 (Q1, 2x2x2 Gauss) or HZ_TET4 (P1,
 *                            closed-form integrals; paper Sec. 3.2 solves on
 *                            an unstructured mesh)
 *   src_kind                 HZ_SRC_NEUMANN: the source faces carry a Neumann
 *                            datum g, f = M_patch g.  HZ_SRC_DIRICHLET: the
 *                            pressure is prescribed, p = g, on every node of
 *                            the source faces (set D; paper Sec. 3.2 imposes
 *                            the sun-roof spectrum as a Dirichlet
 *                            condition), by symmetric elimination: the
 *                            operator's D rows and columns are the
 *                            identity's and the load is f_F = -A_FD g_D,
 *                            f_D = g_D (hz_load then needs a frequency)
 *   fe_scheme                HZ_GALERKIN, or HZ_GLS: Galerkin least-squares
 *                            stabilisation (paper Sec. 3.2 uses stabilised
 *                            finite elements without naming the scheme; GLS
 *                            of Harari and Hughes, 1992, is taken): the
 *                            Laplacian of a linear or trilinear shape
 *                            function vanishes in an element, so the mass
 *                            coefficient k^2 becomes k^2 (1 - tau k^2) with
 *                            tau k^2 = 1 - 6 (1 - cos kh) / ((kh)^2
 *                            (2 + cos kh)), h the mean element edge length
 *                            of the mesh (the absorption term keeps k^2)
 *   Every device vector of the API stays in the mesh's node numbering
 *   whatever order and sigma are; the Schwarz method needs order
 *   HZ_ORDER_GIVEN and sigma 0 (its partition uses the structured ids),
 *   hexahedra, a Neumann source and the Galerkin scheme.                   */
typedef struct {
  int32_t n_nodes, n_elems, n_bfaces;
  const double* xyz;
  const int32_t* hex;
  const int32_t* bface;
  const int32_t* bface_tag;
  const uint8_t* bface_src;
  double c, rho;
  int32_t elems[3];
  int32_t parts[3];
  int32_t order;
  int32_t sigma;
  int32_t elem_type;
  int32_t src_kind;
  int32_t fe_scheme;
} hz_mesh;

/* Solver options (host struct).
 *   method      HZ_GMRES, HZ_BICGSTAB, HZ_BICGSTABL, HZ_TFQMR or HZ_SCHWARZ.
 *               HZ_TFQMR is Freund's transpose-free QMR (the paper's P-tfQMR,
 *               Sec. 4), stopped by its quasi-residual bound and confirmed
 *               with the true residual.
 *               HZ_BICGSTABL is BiCGStab(l) of Sleijpen and Fokkema (the
 *               paper's P-BiCGSTAB(8) family, Sec. 4): l bi-conjugate
 *               gradient steps and one l-dimensional minimal-residual step
 *               per cycle (2 l products); l = 1 is BiCGStab.
 *   restart     GMRES restart length m (1..128); l of BiCGStab(l) (1..8);
 *               Schwarz interface GMRES restart (1..1000)
 *   max_matvec  cap on operator applications (>= 1)
 *   precision   HZ_FP64: complex128 throughout.  HZ_MIXED: complex64 inner
 *               Krylov solves on a complex64 copy of the operator, with the
 *               residual, iterative refinement, Gram-Schmidt coefficients
 *               and the Hessenberg/Givens step in FP64.
 *   precond     HZ_JACOBI (right diagonal scaling) or HZ_NONE
 *   tol         stop when ||f - A p||_2 / ||f||_2 <= tol (true residual,
 *               recomputed in FP64 at exit)
 *   inner_tol   relative tolerance of inner (mixed / subdomain) solves
 *   inner_restart  GMRES restart of the inner complex64 solves; for the
 *               Schwarz method with dd_inner HZ_BICGSTABL, l of the local
 *               BiCGStab(l) (0: 4, at most 8)
 *   dd_alpha    Robin transmission coefficients of the Schwarz method
 *   dd_alpha2   (interface term alpha_st M_G; paper Sec. 4 uses optimised
 *               two-sided conditions).  A subdomain uses dd_alpha on its
 *               faces toward higher-index neighbours and dd_alpha2 on its
 *               faces toward lower-index neighbours; dd_alpha2 = 0 means
 *               dd_alpha on both sides (one-sided).  dd_alpha = 0 selects
 *               the optimised two-sided pair of hz_dd_alpha for the
 *               partition's smallest subdomain width and the mesh spacing;
 *               i k on both sides is the plain absorbing (Despres) choice
 *   dd_inner    Krylov method of the Schwarz subdomain solves (HZ_GMRES,
 *               HZ_BICGSTAB, HZ_BICGSTABL or HZ_TFQMR); for the Schwarz method inner_tol is the
 *               subdomain solves' relative tolerance (0: 1e-12) and
 *               precision HZ_MIXED runs them in complex64 with FP64
 *               refinement; restart is the interface GMRES restart
 *   dd_richardson  0: interface GMRES; N > 0: exactly N plain Schwarz
 *               iterations from zero multipliers (status reports whether
 *               the glued result reached tol)                              */
typedef struct {
  int32_t method;
  int32_t restart;
  int32_t max_matvec;
  int32_t precision;
  int32_t precond;
  int32_t inner_restart;
  double tol;
  double inner_tol;
  hz_c128 dd_alpha;
  int32_t dd_inner;
  int32_t dd_richardson;
  hz_c128 dd_alpha2;
} hz_solve_opts;

/* Filled by the solve entry points.
 *   status       same code as the return value
 *   iters        Krylov iterations (GMRES: Arnoldi steps; BiCGStab:
 *                iterations of two matvecs; Schwarz: interface iterations)
 *   matvecs      operator applications at the outer precision
 *   inner_matvecs  complex64 / subdomain operator applications
 *   relres_true  ||f - A p|| / ||f|| recomputed in FP64 at exit
 *   relres_est   the solver's own residual estimate at exit
 *   seconds      wall time of the call                                    */
typedef struct {
  int32_t status, iters, matvecs, inner_matvecs;
  double relres_true, relres_est, seconds;
} hz_solve_info;

/* Builds the context: assembles K, M, the per-wall boundary masses B0_w,
 * the source-face mass M_patch and (if eta != NULL) M_eta on the host from
 * Q1 elements with 2x2x2 (cells) / 2x2 (faces) Gauss points (paper Sec. 3.2,
 * finite-element discretisation of the Helmholtz equation), then uploads the
 * sparse pattern (sliced-ELL, 64-row slices, int32 column indices) and the
 * values to the device of the calling thread.
 *   beta   [6] wall admittances (host)
 *   eta    [n_elems] loss factors (host) or NULL (= zero field)
 *   hip_stream  hipStream_t to order all work on (NULL = null stream)
 *   out    receives the context; *out is NULL on error
 * Errors: HZ_ERR_INVALID (null/invalid mesh, index out of range, NaN),
 * HZ_ERR_OOM, HZ_ERR_HIP. */
int hz_assemble(const hz_mesh* mesh, const hz_c128* beta, const double* eta,
                void* hip_stream, hz_ctx* out);

/* Replaces the wall admittances and/or the absorption field (either may be
 * NULL to keep it).  Invalidates the current frequency (HZ_ERR_STATE on the
 * next solve until hz_set_frequency is called again). */
int hz_set_params(hz_ctx ctx, const hz_c128* beta, const double* eta);

/* Forms A(k) = K - k^2 M + i k^2 M_eta + i k B_beta for k = 2 pi freq_hz / c
 * on the device (one pass over the nonzeros) and its diagonal: the
 * finite-element operator of the Fourier-transformed wave equation at one
 * frequency (paper Sec. 3.2, the Helmholtz equation and its discretisation;
 * the wall and absorption terms are the Robin admittances and loss factors
 * described at the top of this header).  Later solves and hz_apply use it.
 * freq_hz must be finite and >= 0.  Errors: HZ_ERR_INVALID, HZ_ERR_HIP. */
int hz_set_frequency(hz_ctx ctx, double freq_hz);

/* y_dev = A(k) x_dev, complex128, n_nodes entries each (the sparse
 * matrix-vector product of paper Sec. 4).  x and y must not overlap.
 * Errors: HZ_ERR_STATE (no frequency set), HZ_ERR_INVALID (null). */
int hz_apply(hz_ctx ctx, const hz_c128* x_dev, hz_c128* y_dev);

/* Copies diag(A(k)) (n_nodes complex128) to d_dev. */
int hz_get_diag(hz_ctx ctx, hz_c128* d_dev);

/* f_dev = M_patch g_dev: the load of a Neumann datum g (nodal values,
 * n_nodes complex128) on the source faces. */
int hz_load(hz_ctx ctx, const hz_c128* g_dev, hz_c128* f_dev);

/* *out = a^H b over n complex128 entries, accumulated in FP64 with a fixed
 * reduction order (bitwise reproducible run to run).  Host result. */
int hz_dotc(hz_ctx ctx, int64_t n, const hz_c128* a_dev, const hz_c128* b_dev,
            hz_c128* out);

/* Allocation-free form of hz_dotc, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid
 * hipMalloc): out_dev[0] = a^H b over n complex128 entries, written to
 * device memory (16 bytes, caller-owned), stream-ordered on the context's
 * stream, no synchronisation.  Same kernels, grid and summation order as
 * hz_dotc, so the two results are bitwise equal.  The reduction's partial
 * sums live in a static device array of the library (16 KiB per GPU, held
 * until the process ends: at most 1024 blocks of partial sums, which covers
 * every n >= 0; a larger need is rejected with HZ_ERR_INVALID).  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (two streams, or two threads) race and
 * give wrong results; calls ordered on one stream are safe.  Each call
 * writes every partial sum it reads, so no state carries over between
 * calls.  Errors: HZ_ERR_INVALID (null pointer, n < 0), HZ_ERR_HIP. */
int hz_dotc_noalloc(hz_ctx ctx, int64_t n, const hz_c128* a_dev, const hz_c128* b_dev, hz_c128* out_dev);

/* Solves A(k) p = f at the current frequency (paper Sec. 4: preconditioned
 * Krylov methods and the optimised Schwarz method, complex double).
 *   f_dev  [n_nodes] right-hand side (not modified)
 *   p_dev  [n_nodes] in: initial guess x0, out: solution (may be all zero)
 *   info   may be NULL
 * Returns HZ_OK, HZ_NOT_CONVERGED (max_matvec reached; best iterate in
 * p_dev), HZ_BREAKDOWN, or an error (HZ_ERR_INVALID for bad options,
 * null pointers or a non-finite f; HZ_ERR_STATE if no frequency is set). */
int hz_solve(hz_ctx ctx, const hz_solve_opts* opts, const hz_c128* f_dev,
             hz_c128* p_dev, hz_solve_info* info);

/* Frequency sweep (an addition to the paper's method, which solves one
 * frequency at a time: no passage defines it; each column is the system of
 * hz_set_frequency at its own frequency): solves A(k_j) P[:, j] = F[:, j]
 * for j < nfreq (1..64)
 * with all columns advanced together: one multi-vector sparse product per
 * Krylov step shares the real K, M (and M_eta) values across columns, and
 * each chunk of inner iterations is replayed from a captured HIP graph.
 * The tile shape of the multi-vector product (columns per lane, block size,
 * row-to-XCD mapping) is chosen by a built-in autotuner at first use for
 * (n, nfreq, precision).
 *   freqs_host [nfreq] Hz
 *   F_dev, P_dev  [n_nodes][nfreq] row-major complex128 (column j of row i
 *          at i * nfreq + j); P is in: x0 (zero allowed), out: solutions
 *   infos  [nfreq] per-column results (may be NULL)
 * opts->method is HZ_GMRES (restarted GMRES(restart) advanced in lock-step,
 * every restart cycle one refinement step against the FP64 residual), or
 * HZ_BICGSTAB, HZ_BICGSTABL (l = restart) or HZ_TFQMR with independent
 * per-column scalars: BiCGStab replaces a column's recursive residual by
 * its FP64 true residual (a reliable update) when the former has dropped by
 * the factor inner_tol (complex64, default 0.1) or reached the target
 * (FP64); BiCGStab(l) and TFQMR end a column's inner solve at inner_tol
 * (complex64, default 1e-3) or at the target (FP64) and run a refinement
 * step X += correction, R = F - A X in FP64, restarting if needed.
 * Converged columns leave the batch, which is compacted to the next
 * power-of-two width.  opts->precision HZ_MIXED: complex64 Krylov
 * vectors and operator copy, FP64 residual / refinement / Gram-Schmidt
 * coefficients / Givens; HZ_FP64: complex128 throughout.  Columns converge
 * independently; the call returns when all have reached tol or one has used
 * max_matvec products.  Leaves the
 * context's current frequency unset (call hz_set_frequency before the next
 * hz_solve).  Environment: HZ_AUTOTUNE_CACHE names a text file in which
 * tuned product variants are remembered across processes. */
int hz_solve_sweep(hz_ctx ctx, int32_t nfreq, const double* freqs_host,
                   const hz_c128* F_dev, hz_c128* P_dev,
                   const hz_solve_opts* opts, hz_solve_info* infos);

/* Adjoint solve and gradient at the current frequency (an addition to the
 * paper's method: no passage defines it; it differentiates the solution of
 * the Sec. 3.2 system with respect to the wall admittances and the
 * absorption field).  With the forward
 * solution p (A p = f) and the objective's derivative g = dJ/dconj(p)
 * (for J = sum_r |p_r|^2: g = p on the receivers, 0 elsewhere), solves
 * A^H lambda = g (as A mu = conj(g), lambda = conj(mu), A being complex
 * symmetric) and accumulates
 *     dJ_dbeta[w][0] += 2 k Im(lambda^H B0_w p)      (d/d Re beta_w)
 *     dJ_dbeta[w][1] += 2 k Re(lambda^H B0_w p)      (d/d Im beta_w)
 *     dJ_deta_dev[e] += 2 k^2 Im(lambda_e^H M_e p_e)
 * where J's derivative in a real parameter t is -2 Re(lambda^H dA/dt p).
 *   p_dev, g_dev    [n_nodes] device inputs
 *   lambda_dev      [n_nodes] device output (adjoint state)
 *   dJ_dbeta        [6][2] host, accumulated (may be NULL)
 *   dJ_deta_dev     [n_elems] device FP64, accumulated (may be NULL)
 * With a Dirichlet source the parameters act on the free rows only (the
 * lifting -A_FD g_D included): lambda is the adjoint state of the
 * eliminated system with its D entries set to zero, and the formulas
 * above hold with the full p (p = g on D).                              */
int hz_solve_adjoint(hz_ctx ctx, const hz_solve_opts* opts, const hz_c128* p_dev,
                     const hz_c128* g_dev, hz_c128* lambda_dev, double* dJ_dbeta,
                     double* dJ_deta_dev, hz_solve_info* info);

/* Receiver objective of the adjoint gradient (an addition to the paper's
 * method, no defining passage): with p_dev the solution at one frequency,
 *     *J += sum_r |p[receivers[r]]|^2                    (host, accumulated)
 *     g_dev = dJ/dconj(p): p on the receiver nodes, 0 elsewhere
 * g_dev is the right-hand side hz_solve_adjoint takes.
 *   n_rec      number of receivers (>= 0)
 *   receivers  [n_rec] host array of distinct node ids (caller's numbering)
 *   p_dev, g_dev  [n_nodes] device vectors (must not overlap)
 * J is summed in a fixed order (bitwise reproducible).  Synchronises.
 * Errors: HZ_ERR_INVALID (null pointer, id out of range or repeated). */
int hz_receiver_energy(hz_ctx ctx, int32_t n_rec, const int32_t* receivers, const hz_c128* p_dev, double* J,
                       hz_c128* g_dev);

/* Optimised Robin coefficients for a Schwarz interface (host computation,
 * no context, no GPU): the interface modes xi in [pi/H, pi/h] (H subdomain
 * width, h mesh spacing, both > 0, H > h) have the transparent-condition
 * symbol l(xi) = sqrt(xi^2 - k^2) or i sqrt(k^2 - xi^2); the modes within
 * pi/(2H) of k are left out.  sides = 1: alpha[0] = alpha[1] = the p + i q
 * (p, q > 0, log grid of 80 x 80) minimising max |(l - a)/(l + a)|.
 * sides = 2: the pair p0 + i q, p1 + i q (q of the one-sided optimum)
 * minimising max |(l - a0)(l - a1)/((l + a0)(l + a1))| (pattern search in
 * log p0, log p1 from the one-sided optimum).  k > 0. */
int hz_dd_alpha(double k, double H, double h, int32_t sides, hz_c128* alpha);

/* Storage forms of the operator for the two calls below.  The complex form
 * stores one complex value and one int32 column per entry.  The split form
 * (used by the solvers whenever there is no absorption field) stores the
 * real part of every entry, int16 column offsets from the row when they all
 * fit (else int32 columns), and the imaginary parts of the few entries that
 * can have one: those carrying a wall admittance term or lying in a wall
 * node's column (the Jacobi scaling by a complex wall diagonal).  Both give
 * the same product up to rounding order.  On a structured box in its own
 * numbering (elems set, order HZ_ORDER_GIVEN, sigma 0) the split values are
 * also stored in stencil form (HZ_SPMV_STENCIL, the solvers' choice there):
 * 27 slots per row at the fixed neighbour offsets of the box, a missing
 * neighbour's slot 0, no column indices.  Environment variables HZ_SPLIT=0
 * and HZ_STENCIL=0 (read when the context is created) disable the split
 * and the stencil forms. */
enum { HZ_SPMV_SOLVER = 0, HZ_SPMV_COMPLEX = 1, HZ_SPMV_SPLIT = 2, HZ_SPMV_STENCIL = 3 };

/* Measurement of the sparse product (paper Sec. 4: the product dominates
 * the solve time).  Runs y = A x of the current operator `reps` times
 * (1..100000) on the context's stream, bracketed by two HIP events recorded
 * on that stream, and returns the average duration of one product in
 * milliseconds.  precision HZ_FP64 times the complex128 product of the FP64
 * solvers; HZ_MIXED the complex64 product of the mixed-precision inner
 * solves.  format: HZ_SPMV_SOLVER (the form the solvers use),
 * HZ_SPMV_COMPLEX, HZ_SPMV_SPLIT or HZ_SPMV_STENCIL (HZ_ERR_STATE if that
 * form is not formed).  x and y are internal buffers.  Host result; synchronises the
 * stream. */
int hz_time_spmv(hz_ctx ctx, int32_t reps, int32_t precision, int32_t format, double* avg_ms);

/* Measurement of the frequency sweep's multi-vector product (the sparse
 * product dominates, paper Sec. 4; the sweep is an addition to the paper's
 * method).  For nfreq (1..64) frequencies freqs_host (Hz), with s = nfreq
 * rounded up to a power of two, runs the product Y = A(k_c) X on every
 * column c of an internal [n][s] block in the variant the sweep's
 * autotuner picks (tuning first if needed), `reps` times (1..100000)
 * between two HIP events on the context's stream, and returns the average
 * duration of one product (ms).  bytes (may be NULL) receives its
 * algorithmic bytes in the picked variant's storage, with w = 8 (HZ_FP64)
 * or 4 (HZ_MIXED, complex64) bytes per real value and nb boundary entries:
 * values 2 w nnz (3 w nnz with an absorption field), and 4 w n s for one
 * read of X and one write of Y; the row-wise variants add column indices
 * and row pointers 4 nnz + 4 (n + 1) and boundary lists 4 (n + 1) +
 * (4 + 2 w) nb, the stencil form of a box in its own numbering (no
 * indices; its zero slots for missing neighbours not counted) a per-row
 * boundary index and the boundary values, 4 n + 2 w nb.
 * variant (may be NULL) receives the tuned variant's code.  Leaves the
 * current frequency unset, like hz_solve_sweep.  Synchronises. */
int hz_time_spmm(hz_ctx ctx, int32_t nfreq, const double* freqs_host, int32_t precision, int32_t reps,
                 double* avg_ms, int64_t* bytes, int32_t* variant);

/* One multi-vector product of the frequency sweep (the sparse product of
 * paper Sec. 4 applied to nfreq right-hand sides; an addition to the
 * paper's method, like the sweep itself): for nfreq (1..64) frequencies
 * freqs_host (Hz), y_dev[i * nfreq + c] = (A(k_c) x)[i] for every node i
 * and column c, where x is column c of x_dev ([n_nodes][nfreq] row-major
 * complex128, caller-owned device memory; y_dev the same shape, not
 * overlapping x_dev) and A(k) the unpreconditioned operator K - m(k) M +
 * i k B (+ i k^2 M_eta) of the current parameters (m(k) = k^2, or
 * k^2 (1 - tau k^2) with HZ_GLS).  precision HZ_FP64 runs
 * the sweep's complex128 product; HZ_MIXED rounds x and the operator to
 * complex64 and runs the mixed sweep's inner product (stiffness in
 * difference form), returning its result widened to complex128.  The
 * variant is the one the sweep's autotuner picks for this width (the
 * environment variable HZ_SPMM_VARIANT forces one); variant (may be NULL)
 * receives its code.  Leaves the current frequency unset.  Synchronises.
 * Errors: HZ_ERR_INVALID (null pointer, nfreq out of range, bad frequency
 * or precision, a Dirichlet source, GLS with an absorption field),
 * HZ_ERR_OOM, HZ_ERR_HIP. */
int hz_apply_sweep(hz_ctx ctx, int32_t nfreq, const double* freqs_host, int32_t precision,
                   const hz_c128* x_dev, hz_c128* y_dev, int32_t* variant);

/* Algorithmic bytes of one product of the given precision and form: every
 * stored value, index and row pointer read once, x read once and y written
 * once (n = n_nodes, nnz = CSR nonzeros, r = 8 for FP64 or 4 for FP32):
 *   complex form  (2r + 4) nnz + 4 (n + 1) + 4 r n
 *   split form    (r + idx) nnz + (r + 4) n_imag + 4 (n + 1) + 4 r n,
 *                 idx = 2 (int16 offsets) or 4, n_imag = listed imaginary
 *                 entries.
 *   stencil form  r nnz + (r + 4) n_imag + 4 (n + 1) + 4 r n (missing
 *                 neighbours' zero slots, 27 n - nnz of them, are storage,
 *                 not algorithmic bytes).
 * Requires a frequency (HZ_ERR_STATE otherwise). */
int hz_spmv_bytes(hz_ctx ctx, int32_t precision, int32_t format, int64_t* bytes);

/* Sizes of the context: n_nodes, n_elems, stored nonzeros (CSR count),
 * and the device bytes the context holds. */
int hz_sizes(hz_ctx ctx, int64_t* n_nodes, int64_t* n_elems, int64_t* nnz,
             int64_t* device_bytes);

/* Host-only (no GPU call): the internal numbering hz_assemble uses for this
 * mesh's order and sigma fields.  Reads n_nodes, n_elems, hex, elem_type,
 * order and sigma; writes perm[n_nodes] (host), perm[p] = the mesh node of internal
 * row p.  HZ_ERR_INVALID for bad fields or node ids. */
int hz_node_order(const hz_mesh* mesh, int32_t* perm);

/* Storage layout of the operator (host results; any pointer may be NULL):
 *   perm       [n_nodes] host array: perm[p] = the mesh node stored as
 *              internal row p (the identity for HZ_ORDER_GIVEN, sigma 0)
 *   slots      stored entries of the sliced-ELL arrays, padding included
 *              (each 64-row slice is as wide as its longest row)
 *   bandwidth  max |p - q| over the stored entries (p, q) in the internal
 *              numbering; int16 column offsets need it below 32768
 *   n_imag     entries listed with an imaginary part in the split form   */
int hz_layout(hz_ctx ctx, int32_t* perm, int64_t* slots, int64_t* bandwidth, int64_t* n_imag);

/* Frees the context and its device memory (NULL is ignored). */
void hz_destroy(hz_ctx ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* hz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HZ_H_ */
