/*
 * tmhip -- T-matrix multiple-scattering solve on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the shared library libtmhip.so.  Every compute step runs in HIP
 * kernels on the device selected at tm_create; PyTorch (or any caller) only
 * provides device memory and a HIP stream.
 *
 * The problem follows the statement of App. I.C ("Simulating collective
 * scattering"): N scatterers at positions x_i with T-matrices T_i in a host
 * medium of wavenumber k; incident-field coefficients a0 (expansion of the
 * incident field in regular waves about every x_i); unknown scattered
 * coefficients s with s_j = T_j (a0_j + sum_{i!=j} xi(k(x_j - x_i))^T s_i),
 * solved in the block-diagonally preconditioned form
 *      (I - T A) s = T a0,           A_ji = xi(k(x_j - x_i))^T,
 * by restarted GMRES with a matrix-free block matvec (App. I.D).
 *
 * Conventions shared by every entry point
 *   - Coefficient order per scatterer (App. I.B truncation at lmax, L =
 *     2 lmax(lmax+2) coefficients): n = p*lmax(lmax+2) + l(l+1) - 1 + m,
 *     l = 1..lmax, m = -l..l, p = 0 (M-type, grad(phi) x x) or 1 (N-type).
 *     Basis: App. I.A, normalised Legendre functions without the
 *     Condon-Shortley phase, outgoing waves h_l^(1), time factor e^{-i w t}.
 *   - Coefficient vectors are complex, interleaved (re, im), laid out
 *     [rhs][scatterer][n]; tm_c128 has the memory layout of torch.complex128.
 *   - Pointers marked "device" must be device memory of the context's GPU;
 *     "host" pointers are ordinary host memory.  The caller owns every array
 *     passed in; the context owns its tables and workspaces and frees them
 *     in tm_destroy.
 *   - Calls enqueue work on the context's stream and return without waiting,
 *     except those that fill host outputs (solve info, host result arrays),
 *     which synchronise the stream before returning, and those that allocate
 *     or re-cut the block matvec's work split (a new number of right-hand
 *     sides or matvec configuration), which first drain the stream.
 *   - One context per host thread.  Calls never throw and never abort; they
 *     return a tm_status.  tm_last_error gives a message for the last failing
 *     call on a context.
 *
 * Scope: scatterers in the z = 0 plane (the metasurface setting of the
 * paper).  On a rectangular lattice the library tabulates one translation
 * block per lattice displacement; elsewhere in the plane it forms the blocks
 * on the fly per pair (the lattice-only calls -- batched subregions, position
 * gradients, the allocation-free operator, the autotuner -- then return
 * TM_ERR_NOT_LATTICE).  lmax 1..6 (App. I.B's
 * truncation; the paper's cylinders use lmax 6).
 */
#ifndef TMHIP_H
#define TMHIP_H

#ifdef __cplusplus
extern "C" {
#endif

#define TMHIP_ABI_VERSION 1

typedef struct tm_ctx tm_ctx;

typedef struct { double re, im; } tm_c128;

typedef enum {
  TM_OK = 0,
  TM_NOT_CONVERGED = 1,     /* result written, residual above tolerance */
  TM_ERR_INVALID_ARG = -1,  /* null pointer, size or range out of bounds   */
  TM_ERR_OVERLAP = -2,      /* enclosing spheres intersect (App. I.C)      */
  TM_ERR_NOT_LATTICE = -3,  /* off the z = 0 plane, or a lattice-only call  */
  TM_ERR_OOM = -4,          /* device allocation failed                    */
  TM_ERR_HIP = -5,          /* a HIP runtime call failed                   */
  TM_ERR_NAN = -6,          /* non-finite input                            */
  TM_ERR_STATE = -7         /* call out of order (e.g. solve before T set) */
} tm_status;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The block matvec also
 * runs one of its launches on a second stream of default priority that the
 * context creates on first use and releases in tm_destroy; that launch is
 * ordered after earlier work on `hip_stream`, and later work on `hip_stream`
 * waits for it, so ordering on `hip_stream` is as if everything ran there. */
int tm_create(tm_ctx** ctx, int device, void* hip_stream);
void tm_destroy(tm_ctx* ctx);
const char* tm_status_string(int status);
const char* tm_last_error(const tm_ctx* ctx);
/* Number of coefficients per scatterer, 2 lmax(lmax+2); 0 if lmax invalid. */
int tm_coeff_count(int lmax);
int tm_abi_version(void);

/* ---- problem set-up ------------------------------------------------------ */

/* Scatterer centres and host wavenumber.  pos: host, [n][3] (x, y, z), every
 * z = 0 (TM_ERR_NOT_LATTICE otherwise), no two centres equal (TM_ERR_OVERLAP).
 * When the centres form an nx-by-ny grid of equal pitch in x and y ordered
 * index = iy*nx + ix, builds the translation tables (one block per lattice
 * displacement, App. I.C, eq. "tran_coeff") on the device in FP64 and
 * complex64; otherwise keeps the centres and the per-entry constants of
 * eq. "tran_coeff" for the on-the-fly block matvec.  Invalidates T. */
int tm_set_geometry(tm_ctx* ctx, int n, const double* pos, double k, int lmax);

/* Lattice dimensions of the current geometry (host outputs); an off-lattice
 * geometry reports nx = n, ny = 1, pitch = 0. */
int tm_get_lattice(const tm_ctx* ctx, int* nx, int* ny, double* pitch);

/* General per-scatterer T-matrices (App. I.B, eq. "def_tmatrix": s_i =
 * T_i a_exc,i with T_i mixing every (p, l, m)): T device [N][L][L]
 * complex128, row-major per scatterer in the coefficient order above.  The
 * data are copied (the caller keeps its buffer).  The solves, the operator
 * and the readout then use T_i in place of the diagonal; the per-scatterer
 * product runs in FP64 in both precisions.  There is no dT/dr for a dense T
 * (tm_grad_radius returns TM_ERR_STATE), tm_get_tmatrix_diag returns
 * TM_ERR_STATE and tm_solve_batched (diagonal T only) returns TM_ERR_STATE
 * until spheres or a diagonal T are set again.  Entries are not checked for
 * NaN.  A T whose entries between different azimuthal orders m are all
 * exactly zero (a scatterer symmetric about the z axis) is also packed into
 * its m-blocks, which the product then reads alone (same terms, same order);
 * the test runs on the device and the call waits for its one-word result. */
int tm_set_tmatrix_dense(tm_ctx* ctx, const tm_c128* T);

/* Mie T-matrix of one homogeneous sphere (the sphere case of App. I.B),
 * computed on the current HIP device, no context needed: t_out host
 * [2][lmax] with t_out[p*lmax + l-1] = -b_l (p = 0, M-type) or -a_l (p = 1,
 * N-type); dtdr_out host [2][lmax] or NULL: d t / d radius.  Requires
 * 1 <= lmax <= 6, k > 0, radius > 0, n_im >= 0 and k radius |n| <= 12.
 * Synchronous; allocates and frees a small device buffer. */
int tm_mie(int lmax, double k, double radius, double n_re, double n_im, tm_c128* t_out,
           tm_c128* dtdr_out);

/* Homogeneous spheres (Mie T-matrices, the sphere case of App. I.B):
 * radii: device, [N] (> 0, finite; no two spheres may intersect, i.e.
 * r_i + r_j < |x_i - x_j| for every pair, diagonal and farther neighbours
 * included, else TM_ERR_OVERLAP);
 * relative refractive index n_re + i n_im (n_im >= 0).  Computes the
 * diagonal T and dT/dr on the device. */
int tm_set_spheres(tm_ctx* ctx, const double* radii, double n_re, double n_im);

/* Null-field (EBCM) T-matrices of dielectric cylinders, the paper's
 * meta-atoms (App. I.B, eq. "def_tmatrix" with the surface-integral matrices
 * P, Q): scatterer i is a cylinder of radius radii[i] (device, [N]) and the
 * given height, axis along z, centred on its site, relative index
 * n_re + i n_im (n_im >= 0).  For each azimuthal order m the surface
 * integrals over the caps and the side (n_quad Gauss-Legendre nodes per face,
 * 0 = 96) give the outgoing- and regular-test matrices O_m, R_m and
 * T_m = -R_m O_m^{-1}; the T of every scatterer is computed on the device and
 * set as a dense T (as tm_set_tmatrix_dense).  The enclosing spheres
 * (radius sqrt(r^2 + h^2/4)) must not intersect (TM_ERR_OVERLAP), and
 * k r_enclosing |n| <= 12.  The null-field method converges slowly in lmax
 * for bodies with edges; lmax 6 is the paper's choice. */
int tm_set_cylinders(tm_ctx* ctx, const double* radii, double height, double n_re, double n_im,
                     int n_quad);

/* The T-matrix of one cylinder as tm_set_cylinders computes it, no context
 * needed: T_out host [L][L] in the coefficient order above.  Synchronous;
 * allocates and frees small device buffers on the current device. */
int tm_ebcm_cylinder(int lmax, double k, double radius, double height, double n_re, double n_im,
                     int n_quad, tm_c128* T_out);

/* Arbitrary diagonal T-matrices: t: device, [N][L] (entry n of T_i's
 * diagonal).  Clears dT/dr (tm_grad_radius then returns TM_ERR_STATE). */
int tm_set_tmatrix_diag(tm_ctx* ctx, const tm_c128* t);

/* Copy the current T diagonal and dT/dr (spheres only; dtdr may be NULL)
 * to device arrays [N][L]. */
int tm_get_tmatrix_diag(tm_ctx* ctx, tm_c128* t, tm_c128* dtdr);

/* ---- incident field ------------------------------------------------------ */

/* Plane waves pol_r e^{i k khat_r . x} (App. II, expansion in regular waves,
 * eqs. "integrand_p_0"/"integrand_p_1"), expanded about every scatterer:
 * khat: host [R][3] unit vectors; pol: host [R][3] complex, pol . khat = 0;
 * a0: device [R][N][L] output. */
int tm_plane_wave_rhs(tm_ctx* ctx, int n_rhs, const double* khat, const tm_c128* pol,
                      tm_c128* a0);

/* ---- solve ---------------------------------------------------------------- */

enum { TM_PREC_FP64 = 0, TM_PREC_MIXED = 1 };

typedef struct {
  double tol;        /* relative true residual ||T a0 - B s|| / ||T a0||   */
  int restart;       /* Krylov dimension per cycle: 1..1000 for tm_solve and
                        tm_adjoint_solve ((restart+1) basis vectors of 32 N
                        complex128 each), 1..200 for tm_solve_batched       */
  int max_iter;      /* total Arnoldi steps over all cycles                 */
  int precision;     /* TM_PREC_FP64: FP64 matvec throughout;
                        TM_PREC_MIXED: complex64 matvec with FP32
                        accumulation inside each cycle, FP64 Arnoldi and an
                        FP64 true residual between cycles (iterative
                        refinement)                                         */
  double inner_tol;  /* mixed only: relative residual reduction per cycle   */
  int use_x0;        /* 1: s holds the initial guess on entry               */
} tm_solve_opts;

typedef struct {
  int status;          /* TM_OK or TM_NOT_CONVERGED                          */
  int iters;           /* Arnoldi steps                                      */
  int cycles;          /* restart / refinement cycles                        */
  int matvecs_fp64;
  int matvecs_lowp;
  double rel_residual; /* final FP64 true relative residual                  */
} tm_solve_info;

/* Fill opts with defaults (tol 1e-8, restart 50, max_iter 2000, FP64,
 * inner_tol 1e-4, use_x0 0). */
void tm_default_opts(tm_solve_opts* opts);

/* Solve (I - T A) s = T a0 for each right-hand side.
 * a0: device [R][N][L]; s: device [R][N][L] (initial guess if use_x0);
 * info: host [R].  Returns TM_OK if every RHS converged, TM_NOT_CONVERGED if
 * any did not (its best iterate is still written). */
int tm_solve(tm_ctx* ctx, int n_rhs, const tm_c128* a0, tm_c128* s,
             const tm_solve_opts* opts, tm_solve_info* info);

/* Adjoint system (I - A^T T) mu = v (the transpose of App. IV's
 * Omega^T a = v in preconditioned form; the paper's adjoint unknown is
 * T mu).  v, mu: device [R][N][L]. */
int tm_adjoint_solve(tm_ctx* ctx, int n_rhs, const tm_c128* v, tm_c128* mu,
                     const tm_solve_opts* opts, tm_solve_info* info);

enum {
  TM_OP_FORWARD = 0,   /* y = (I - T A) x   */
  TM_OP_COUPLING = 1,  /* y = A x           */
  TM_OP_ADJOINT = 2,   /* y = (I - A^T T) x */
  TM_OP_COUPLING_T = 3 /* y = A^T x         */
};

/* One application of the operator (the matvec GMRES uses).  x, y: device
 * [R][N][L], must not alias.  precision: TM_PREC_FP64 or TM_PREC_MIXED
 * (complex64 blocks and inputs, FP32 accumulation, FP64 output). */
int tm_apply_operator(tm_ctx* ctx, int n_rhs, const tm_c128* x, tm_c128* y, int precision,
                      int op);

/* Allocation-free variant of tm_apply_operator, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and rounding
 * class as tm_apply_operator (the block-matvec work split differs, so
 * complex64 results differ from it by FP32 summation order).  It calls no
 * hipMalloc/hipFree and never synchronises: it enqueues kernels only.  Its
 * packed vectors, low-precision input copy, work split and partial sums live
 * in one static device array of TM_NOALLOC_SCRATCH_BYTES per GPU, held until
 * the process ends; a problem whose buffers do not fit returns
 * TM_ERR_INVALID_ARG (about 2 N n_rhs <= 1.5e6 sites x right-hand sides; the
 * work split is thinned to fit).  Calls on one GPU share that array: calls
 * that overlap in time on the same GPU (other streams, other threads, other
 * contexts) race and must be serialised by the caller.  Requires a diagonal
 * T for TM_OP_FORWARD / TM_OP_ADJOINT (TM_ERR_STATE for a dense T) and, for
 * the transposed ops, tables already built by an earlier tm_apply_operator
 * with a transposed op or tm_adjoint_solve (TM_ERR_STATE otherwise). */
#define TM_NOALLOC_SCRATCH_BYTES (128ull * 1024ull * 1024ull)
int tm_apply_operator_noalloc(tm_ctx* ctx, int n_rhs, const tm_c128* x, tm_c128* y,
                              int precision, int op);

/* ---- batched subregions --------------------------------------------------- */

/* A rectangular subregion of the current lattice: sites (ix, iy) with
 * origin_x <= ix < origin_x + side_x, origin_y <= iy < origin_y + side_y. */
typedef struct {
  int origin_x, origin_y, side_x, side_y;
} tm_subregion;

/* Solve every subregion alone (scatterers outside it are ignored: the
 * subregion-plus-padding decomposition of the paper's distribution strategy)
 * for n_rhs plane waves (khat/pol: host [R][3], as tm_plane_wave_rhs), all
 * (subregion, rhs) systems advancing together: one block-matvec launch per
 * Arnoldi step covers every system, each restart cycle is replayed from a
 * captured hipGraph when use_graph != 0, converged systems leave the batch.
 * Geometry (the full lattice) and T must be set.  subs: host [S];
 * s_out: device, the subregions' [R][N_k][L] coefficient blocks concatenated
 * in subregion order (site index within a subregion ly*side_x + lx);
 * info: host [S][R].  opts->use_x0 must be 0.  1 <= n_rhs <= 8.
 * A system whose right-hand side or residual is not finite leaves the batch
 * with info status TM_ERR_NAN (its coefficients unspecified) while the
 * others go on; the call then returns TM_NOT_CONVERGED, as when any system
 * stops at max_iter. */
int tm_solve_batched(tm_ctx* ctx, int n_sub, const tm_subregion* subs, int n_rhs,
                     const double* khat, const tm_c128* pol, tm_c128* s_out,
                     const tm_solve_opts* opts, tm_solve_info* info, int use_graph);

/* tm_solve_batched with the incident coefficients given per subregion (any
 * source, e.g. the jinc groups of tm_jinc_rhs_batched): a0 device, the
 * subregions' [R][N_k][L] blocks concatenated in subregion order (the layout
 * of s_out); everything else as tm_solve_batched. */
int tm_solve_batched_a0(tm_ctx* ctx, int n_sub, const tm_subregion* subs, int n_rhs,
                        const tm_c128* a0, tm_c128* s_out, const tm_solve_opts* opts,
                        tm_solve_info* info, int use_graph);

/* Jinc source (App. II, "Computation of Jinc Sources"): one Nyquist sample
 * of a band-limited incident field propagating along +z, centred at (x0, y0)
 * in the plane z = z0 with transverse polarisation (ax, ay).  Its field is the
 * disk of propagating plane waves
 *   E(x) = (1/2pi) int_0^{pi/2} int_0^{2pi} A(b, a) e^{i k(b, a).(x - x0)} sin b cos b da db,
 * A(b, a) = (ax, ay, -tan b (ax cos a + ay sin a)), whose transverse part in
 * the plane z = z0 is (ax, ay) J_1(k rho)/(k rho) (cylindrical J_1).  A field
 * band-limited to the light cone equals the sum of the jinc sources of its
 * lambda/2-grid samples weighted by pi/2 times the sampled field. */
typedef struct {
  double x0, y0, z0;
  tm_c128 ax, ay;
} tm_jinc;

/* Incident coefficients of jinc sources about every scatterer (App. II, the
 * expansion in regular waves with the azimuthal integral in closed form,
 * Gamma_m with Bessel J_{m-1}, J_{m+1}, and Gauss-Legendre quadrature in the
 * polar angle): src host [R]; a0 device [R][N][L].  n_beta: polar nodes, 0 =
 * 40 + k r_max (r_max the largest source-to-scatterer distance).  Each
 * source must lie outside every scatterer's enclosing sphere. */
int tm_jinc_rhs(tm_ctx* ctx, int n_src, const tm_jinc* src, int n_beta, tm_c128* a0);

/* The same for subregions (the padded source groups of Sec. 2's
 * distribution): system (k, r) is excited by the sum of the sources
 * src[groups[k R + r]] .. src[groups[k R + r + 1] - 1] (host; groups [S R + 1],
 * non-decreasing from 0 to n_src); a0 device, the subregions' [R][N_k][L]
 * blocks concatenated in subregion order (the layout of tm_solve_batched's
 * output; site index ly side_x + lx).  n_beta as above (0 = automatic over
 * every group and its subregion). */
int tm_jinc_rhs_batched(tm_ctx* ctx, int n_sub, const tm_subregion* subs, int n_rhs, int n_src,
                        const tm_jinc* src, const int* groups, int n_beta, tm_c128* a0);

/* 1 if the last tm_solve_batched replayed its restart cycles from a
 * captured hipGraph, 0 if it ran them eagerly. */
int tm_batch_graph_used(const tm_ctx* ctx);

/* Batched autotuner (the work items of the batched path, App. I.D's
 * subregion jobs sharing one launch).  on = 1: every later tm_solve_batched
 * first times one batched matvec, all systems active, for each table
 * prefetch depth (1..3 complex64, 1..2 FP64) and work split (16k, 32k, 64k
 * workgroups), in the precision of its Arnoldi steps, and keeps the fastest
 * (18 or 12 extra matvecs, synchronous).  on = 0 (default): about 32k
 * workgroups and the prefetch depth of the context's matvec variant
 * (tm_set_matvec_config; depth 1 for variants 0..7).  Every configuration
 * computes the same product up to rounding. */
int tm_set_batch_autotune(tm_ctx* ctx, int on);

/* Launch configuration the last tm_solve_batched used for `precision`
 * (TM_PREC_FP64 or TM_PREC_MIXED): table prefetch depth and work items per
 * (rhs, class) pair; both 0 before the first batched solve. */
int tm_get_batch_config(const tm_ctx* ctx, int precision, int* prefetch, int* items);

/* ---- readout ------------------------------------------------------------- */

/* Scattered field E_sca(x) = sum_i s_i^T Phi(k(x - x_i)) (App. I.C, eq.
 * "sca_fld_concise") at points: pts device [P][3] (each outside every
 * scatterer's enclosing sphere); E device [R][P][3] complex128.
 * precision: TM_PREC_FP64, or TM_PREC_MIXED (basis functions and sums in
 * FP32 with k|x - x_i| reduced modulo 2 pi in FP64). */
int tm_near_field(tm_ctx* ctx, int n_rhs, const tm_c128* s, int n_pts, const double* pts,
                  tm_c128* E, int precision);

/* Transpose (not conjugate transpose) of the near-field map s -> E_sca:
 * v[r][i][n] = sum_p sum_c w[r][p][c] Phi_n(k(x_p - x_i))_c, so that
 * sum_{p,c} w[r][p][c] E_sca[r][p][c] = sum_{i,n} v[r][i][n] s[r][i][n].
 * It turns a field-space weight into the adjoint source of App. IV (the
 * multi-point form of tm_detector_vector).  pts: device [P][3] (outside every
 * enclosing sphere); w: device [R][P][3]; v: device [R][N][L]; FP64.
 * P = 0 writes zeros.  1 <= n_rhs <= 65535. */
int tm_near_field_adjoint(tm_ctx* ctx, int n_rhs, int n_pts, const double* pts, const tm_c128* w,
                          tm_c128* v);

/* Far-field amplitude F(d) = lim_r r e^{-ikr} E_sca(r d): dirs device [D][3]
 * unit vectors; F device [R][D][3]. */
int tm_far_field(tm_ctx* ctx, int n_rhs, const tm_c128* s, int n_dir, const double* dirs,
                 tm_c128* F);

/* ---- sensitivities (App. IV) -------------------------------------------- */

/* Detector vector of a point detector: v[i][n] = sum_c w_c Phi_n(k(xd - x_i))_c
 * so that sum_c w_c E_sca,c(xd) = v^T s.  xd: host [3]; w: host [3];
 * v: device [N][L]. */
int tm_detector_vector(tm_ctx* ctx, const double* xd, const tm_c128* w, tm_c128* v);

/* Radius gradient contraction for spheres:
 * grad[r][i] = 2 Re sum_n mu[r][i][n] * dT_i,n/dr * a_exc[r][i][n],
 * a_exc = a0 + A s (exciting field).  mu, s, a0: device [R][N][L];
 * grad: device [R][N] doubles.  With mu from tm_adjoint_solve of the
 * objective's weighted detector vector this is dO/dr_i (App. IV,
 * eq. "grad_geometry_overlap").  Factor convention: for a real function f
 * of s, the 2 Re above assumes the adjoint right-hand side w = df/ds (the
 * holomorphic derivative, as the detector vector gives for O = |E|^2 with
 * conj(E) folded into w).  A caller holding instead G = 2 df/ds*, the
 * gradient convention of PyTorch, solves with w = conj(G) and halves the
 * result: df/dr_i = grad[i] / 2. */
int tm_grad_radius(tm_ctx* ctx, int n_rhs, const tm_c128* mu, const tm_c128* s,
                   const tm_c128* a0, double* grad);

/* Position gradient (App. IV, eq. "grad_pos_overlap"): the in-plane
 * derivatives of an objective O with respect to every scatterer's position,
 *   grad[r][i][a] = 2 Re[ lam^T (dA/dq_ia s + da0/dq_ia)
 *                         + sum_c w_c (d v_c / dq_ia)^T s ],   a = x, y,
 * with lam = T^T mu the adjoint unknown (mu from tm_adjoint_solve of the
 * objective's weighted detector vector), v_c the detector vectors of
 * tm_detector_vector.  The coupling term uses derivative blocks
 * d xi(k d)^T / d d_a per lattice displacement (FP64 tables built on first use,
 * four of the size of the FP64 translation table); the gradient is taken at
 * the current lattice positions.
 * mu, s, a0: device [R][N][L]; grad: device [R][N][2] doubles (written).
 * khat: host [R][3], the plane-wave directions a0 was made with (the incident
 * term i k khat_a lam_i . a0_i), or NULL when the incident field does not
 * move with the scatterers (a0 may then be NULL).  xd: host [3] detector
 * point and w: host [R][3] weights (w_c = f'(z_c), e.g. conj(E_c) for
 * O = sum_c |E_c|^2) of the detector term, both NULL to omit it; xd must lie
 * outside every enclosing sphere.  The out-of-plane derivative is not
 * computed (it couples the two z-mirror classes of the lattice blocks). */
int tm_grad_position(tm_ctx* ctx, int n_rhs, const tm_c128* mu, const tm_c128* s,
                     const tm_c128* a0, const double* khat, const double* xd,
                     const tm_c128* w, double* grad);

/* ---- matvec launch configuration (autotuner) ----------------------------- */

/* Kernel variant and work split of the block matvec for one precision.
 * variant 0..7 (operands read from global memory): bit 0 = complex products
 * from three real matrix-core products (else four), bit 1 = operands of the
 * next displacement loaded during the current one's products, bit 2 =
 * register budget for 4 (else 2) waves per SIMD; variants 8, 9, 10: source
 * windows staged in LDS per block of displacements, translation blocks
 * fetched 1, 2, 3 displacements ahead (FP64 runs variant 10 as 9: depth 3
 * does not fit its register budget), with 4-row "wide" tiles for rows past
 * the last multiple of 16.  items: target work items per (rhs, class) pair,
 * 0 = default.  All variants compute the same product.  Variants 0..7 are
 * written for lmax <= 3 (one 16-slot group per z-mirror class); at lmax 4..6
 * a request for them runs the LDS-staged kernel (variant 9 FP64, 10
 * complex64) instead. */
int tm_set_matvec_config(tm_ctx* ctx, int precision, int variant, int items);
int tm_get_matvec_config(tm_ctx* ctx, int precision, int* variant, int* items);

/* Time the LDS-staged variants (8..10; FP64: 8, 9) with a few work-item
 * counts (4k..64k workgroups) on the current geometry for n_rhs right-hand
 * sides and keep the fastest for `precision`.  Synchronises; best_ms (host,
 * nullable) receives the best block-matvec time.  Without a call, FP64 uses
 * variant 9 and complex64 variant 8 with the default work split. */
int tm_autotune(tm_ctx* ctx, int n_rhs, int precision, double* best_ms);

/* ---- progress ------------------------------------------------------------- */

/* Called on the calling thread after every restart cycle of tm_solve,
 * tm_adjoint_solve (per right-hand side) and tm_solve_batched:
 * cycles = restart cycles so far, iters = Arnoldi steps so far (the largest
 * over the batch's systems), n_live = systems still iterating (1 for a single
 * solve), max_rel_residual = largest true relative residual among them at
 * the start of the cycle.  Inside a cycle of tm_solve / tm_adjoint_solve it
 * is also called every 50 Arnoldi steps (except after the cycle's last step)
 * with cycles = completed cycles and max_rel_residual = the Givens estimate
 * of the current relative residual.  The callback must not call back into
 * the same context.  fn = NULL removes it. */
typedef void (*tm_progress_fn)(void* user, int cycles, int iters, int n_live, double max_rel_residual);
int tm_set_progress(tm_ctx* ctx, tm_progress_fn fn, void* user);

/* ---- profiling ------------------------------------------------------------ */

/* When enabled, the block-matvec launches are bracketed by HIP events on the
 * context stream and their durations accumulated per precision. */
int tm_profile_enable(tm_ctx* ctx, int enable);
/* which: 0 = FP64 block matvec, 1 = complex64 block matvec.  Synchronises. */
int tm_profile_query(tm_ctx* ctx, int which, double* total_ms, long long* launches,
                     double* flops_per_launch);
int tm_profile_reset(tm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TMHIP_H */
