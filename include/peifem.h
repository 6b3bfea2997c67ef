/*
 * peifem.h -- C ABI of the MI355X (gfx950) library for the Parareal
 * exponential-integrator Q1 finite element method (PEIFE-linear) for
 *
 *     u_t = D * Laplace(u) + f(t, x)  on a box in R^d (d = 1..3),
 *     u = 0 on the boundary, u(t0) = u0                    (paper, eq. (2.1))
 *
 * Everything runs in spectral space: the state of a time slice is the
 * coefficient vector W of u_h in the M-orthonormal eigenbasis of the Q1 mass
 * and stiffness matrices (the basis that diagonalises both at once, paper
 * Section 2.3, closing paragraph).  In that basis L_h acts as D*lambda_k on
 * coefficient k and the Euclidean norm of W is the L2 norm of u_h.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Status: PE_OK (0) on success, a negative pe_status otherwise; the
 *    message of the last failure of the calling thread is pe_last_error().
 *    No C++ exception crosses this ABI.
 *  - Memory: every pointer named d_* is DEVICE memory owned by the caller
 *    (the library never frees it); pointers named h_* or without prefix
 *    (small parameter arrays) are HOST memory, read during the call only.
 *    A pe_grid owns only its own small device tables; pe_free_grid releases
 *    them.
 *  - Layout: a state (one slice) is n_1*...*n_d coefficients in C order
 *    (last axis fastest), mode k_a = 1..n_a stored at index k_a - 1.  Arrays
 *    of slices are [slice][n_1]...[n_d], contiguous.
 *  - Precision: PE_FP64 grids hold double states; PE_SPLIT_BF16 grids hold
 *    float states and run the transforms as split-bf16 products with fp32
 *    accumulation.  Phase tables (E, B) are always double, and so are norms.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls
 *    enqueue work and return without synchronising, except where stated.
 *    A pe_grid must not be used by two host threads at once.
 */
#ifndef PEIFEM_H
#define PEIFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pe_status;
#define PE_OK 0
#define PE_E_ARG (-1)         /* invalid argument (sizes, null pointers, nodes) */
#define PE_E_HIP (-2)         /* a HIP runtime call failed */
#define PE_E_WORKSPACE (-3)   /* workspace smaller than required */
#define PE_E_NUMERIC (-4)     /* a non-finite norm was produced */
#define PE_E_UNSUPPORTED (-5) /* feature not available for this grid */

#define PE_MAX_DIM 3
#define PE_MAX_STAGES 8
#define PE_MAX_TERMS 64
#define PE_MAX_ITERS 64

typedef enum { PE_FP64 = 0, PE_SPLIT_BF16 = 1 } pe_precision;

typedef struct pe_grid_s *pe_grid;

/* Separable descriptors.  One term is
 *     amp * tau(t) * prod_a X_a(x_a),
 *     tau(t) = exp(alpha t) cos(omega t + phase) (p0 + p1 t + p2 t^2 + p3 t^3),
 *     X_a(x) = (q0 + q1 x + q2 x^2) sin(kappa x + phase).
 * A pure polynomial space factor uses kappa = 0, phase = pi/2. */
typedef struct {
  double kappa;
  double phase;
  double poly[3];
} pe_space_factor;

typedef struct {
  double alpha;
  double omega;
  double phase;
  double poly[4];
} pe_time_factor;

typedef struct {
  double amp;
  pe_time_factor time;
  pe_space_factor space[PE_MAX_DIM];
} pe_term;

/* A moving hat source (the oscillating source of the paper's Example 5.4,
 * not separable in t and x):
 *     amp tau(t) max(1 - |x_axis - c(t)| / width, 0) prod_{b != axis} X_b(x_b),
 *     c(t) = c0 + c1 sin(omega t + phase),
 * tau and X_b as in pe_term (space[axis] is ignored). */
typedef struct {
  double amp;
  int32_t axis;
  double width;
  double c0, c1, omega, phase;
  pe_time_factor time;
  pe_space_factor space[PE_MAX_DIM];
} pe_moving_hat;

#define PE_MAX_MOVING 16

/* --------------------------------------------------------------------- */

/* Build a grid: n[a] interior Q1 nodes on [lo[a], hi[a]] (n[a] + 1 elements
 * of width h_a = (hi - lo)/(n + 1), paper Section 2.1, eq. (2.2)), diffusion
 * coefficient D > 0.  Computes on the device, per axis, the closed-form
 * eigenvalues lambda_a(k) = (6/h^2)(1 - cos t_k)/(2 + cos t_k), the mass
 * eigenvalues mu_a(k) = (h/3)(2 + cos t_k), t_k = k pi/(n + 1), and the
 * orthonormal DST-I matrix S_a[k][j] = sqrt(2/(n+1)) sin(jk pi/(n+1)) (plus
 * its bf16 hi/lo split for PE_SPLIT_BF16).  quad_q (1..8) is the number of
 * Gauss-Legendre points per element and axis used for load vectors.
 * Errors: PE_E_ARG for dim outside 1..3, n < 1, n > 8191, hi <= lo, D <= 0,
 * bad precision or quad_q; PE_E_HIP on allocation failure.  On success *out
 * receives the handle.  Synchronises `stream`. */
pe_status pe_init_grid(pe_grid *out, int32_t dim, const int32_t *n, const double *lo,
                       const double *hi, double D, int32_t precision, int32_t quad_q,
                       void *stream);

/* As pe_init_grid, with periodic[a] != 0 making axis a periodic (Section 1
 * and the closing remark of Section 2 carry the method over to periodic
 * boundary conditions): n[a] nodes per period, node j at lo + j h, h =
 * (hi - lo)/n; the circulant Q1 pair has lambda_a(k) = (6/h^2)(1 - cos t_k)/
 * (2 + cos t_k) with t_k = 2 pi k / n (a zero mode included, which the phi
 * tables take at z = 0) and the orthonormal cos/sin basis; a periodic axis of
 * a state holds its modes in the order: position 0 the constant, 2k - 1 cos k,
 * 2k sin k (k = 1..n/2 - 1), n - 1 the alternating mode (k = n/2).  Loads
 * use the grid's Gauss rule on the n elements of the period, node 0 taking
 * the last one.  Grids with a periodic axis use the FFT transform (FP64; a
 * periodic n in {64, 128, 256, 512, 1024}, the other axes n + 1 in
 * {64, .., 512}) with the separate update; Dirichlet data, moving sources on
 * a periodic axis and the learned calls are not available on them.
 * Errors: as pe_init_grid, plus PE_E_ARG for these limits. */
pe_status pe_init_grid_periodic(pe_grid *out, int32_t dim, const int32_t *n, const double *lo,
                                const double *hi, double D, int32_t precision, int32_t quad_q,
                                const int32_t *periodic, void *stream);

/* Release a grid and its device tables (NULL is ignored). */
void pe_free_grid(pe_grid g);

/* How the per-axis sine transforms of pe_fine_propagate, pe_coarse_sweep's
 * forcing, pe_project and the learned calls are computed (Section 2.3: the
 * sine matrix diagonalises M and A on every axis and is applied as a fast
 * transform).
 *   PE_TRANSFORM_DENSE (default): even/odd folds plus dense products on the
 *     matrix cores.
 *   PE_TRANSFORM_FFT: each line as the imaginary part of a complex FFT of
 *     length 2(n_a + 1) of its odd extension (two lines per FFT), in LDS.
 *     FP64 grids only, every axis with n_a + 1 in {64, 128, 256, 512}.
 * Both give the same coefficients up to rounding.  The FFT's twiddle tables
 * (2(n_a + 1) complex doubles per axis) are allocated here and owned by the
 * grid.  Errors: PE_E_ARG for an unknown kind or a grid the FFT does not
 * support (the grid keeps its transform), PE_E_HIP on allocation failure.
 * Synchronises the device. */
typedef enum { PE_TRANSFORM_DENSE = 0, PE_TRANSFORM_FFT = 1 } pe_transform;
pe_status pe_set_transform(pe_grid g, int32_t kind);

/* Whether the stage-load transform of pe_fine_propagate (Section 2.3, the
 * tensor-product sine transform of the load vectors of eq. (2.6)) runs its
 * generating last-axis pass and its middle-axis pass as one kernel (enable
 * != 0, the default) or as two passes with the intermediate in device memory
 * (enable = 0).  It applies to 3D split-bf16 grids whose axis-0 pass is
 * fused with the update and whose axes 1 and 2 have Kh = 64 or 128 (n from
 * 65 to 255), with at most 32 separable forcing terms and no moving
 * sources; elsewhere the setting has no effect.  Both forms compute the same
 * products; the fused one orders each 32-wide k-step of the axis-2 product
 * differently, so results agree to fp32 rounding, not bitwise.  Errors:
 * PE_E_ARG for a null grid.  No device work. */
pe_status pe_set_fusion(pe_grid g, int32_t enable);

/* Set the forcing f (paper eq. (2.1)) as n_terms (0..PE_MAX_TERMS) separable
 * terms (host array).  Builds on the device the 1D load tables
 * C_{m,a}[j] = int X_{m,a}(x) phi_j(x) dx by the grid's Gauss rule (the load
 * vector of P_h f, paper eq. (2.6)).  Errors: PE_E_ARG.  Synchronises. */
pe_status pe_set_forcing(pe_grid g, int32_t n_terms, const pe_term *terms, void *stream);

/* Dirichlet data u = g on the boundary of the box, as n_terms (0..) separable
 * terms with time factors (host array; n_terms = 0: homogeneous data, the
 * default).  The paper states the method for homogeneous data (Section 2)
 * and notes the extension to non-homogeneous data at the start of Sections
 * 3 and 4; the reading used here: u_h(t) = sum over interior nodes of
 * U_j(t) phi_j + g_h(t), g_h the Q1 interpolant of g on the boundary nodes,
 * so the interior system keeps its matrices and its load vector gains
 *     -(M_IB g_B'(t) + D A_IB g_B(t)),
 * g_B the data at the boundary nodes.  For separable data that load is
 * 2 + 2d separable terms per data term (1D tables from the data's nodal
 * values on each axis); they join the forcing's terms, so every call that
 * evaluates the forcing (pe_fine_propagate, pe_coarse_sweep's r_n,
 * pe_parareal_solve, the learned calls) includes them.  States stay the
 * interior coefficients; the full solution adds g_h(t).  The initial state
 * comes from pe_project_state.  Errors: PE_E_ARG when the forcing's terms
 * plus (2 + 2d) n_terms exceed PE_MAX_TERMS or for null terms (the grid keeps
 * its previous data).  Synchronises `stream`. */
pe_status pe_set_boundary(pe_grid g, int32_t n_terms, const pe_term *terms, void *stream);

/* Moving hat sources (0..PE_MAX_MOVING; host array) added to the forcing of
 * every call that evaluates it (pe_fine_propagate, pe_coarse_sweep's r_n,
 * pe_parareal_solve).  Their load is the grid's q-point Gauss rule on every
 * element, like every other load (the hat's kinks fall inside elements and
 * are not treated apart); the load field is written by a quadrature kernel
 * and transformed by the non-generating passes.  The learned calls reject a
 * grid with moving sources (their inputs are the separable forcing's).
 * Errors: PE_E_ARG (count, axis outside the grid, width <= 0, non-finite
 * parameters; the grid keeps its previous sources), PE_E_HIP.  Synchronises
 * `stream`. */
pe_status pe_set_moving_sources(pe_grid g, int32_t n, const pe_moving_hat *src, void *stream);

/* Exponential Runge-Kutta tables for step h > 0 and s (1..PE_MAX_STAGES)
 * distinct nodes c[0..s-1] in [0, 1] (host):
 *     d_E[k]       = exp(-h D lambda_k)
 *     d_B[i*DOF+k] = h * b_i(h D lambda_k),
 *     b_i(z) = int_0^1 exp(-z (1 - theta)) l_i(theta) dtheta       (eq. (2.7))
 * in FP64, with l_i the Lagrange basis of the nodes; DOF = prod n_a and
 * lambda_k = sum_a lambda_a(k_a).  d_E holds DOF doubles, d_B s*DOF.
 * Errors: PE_E_ARG (h <= 0, s out of range, nodes not distinct or outside
 * [0,1], null pointers). */
pe_status pe_phi_tables(pe_grid g, double h, int32_t s, const double *c, double *d_E, double *d_B,
                        void *stream);

/* Spectral coefficients of P_h v for a time-independent separable function v
 * (n_terms terms; the time factors are ignored): d_W (one state) receives
 * (kron_a Q_a)^T F_v, F_v the load vector of v by the grid's Gauss rule.
 * This is how u0 enters (u_h(t0) = P_h u0, eq. (2.2)).  n_terms = 0 writes
 * zeros.  Needs pe_project_workspace_bytes() of d_work. */
size_t pe_project_workspace_bytes(pe_grid g);
pe_status pe_project(pe_grid g, int32_t n_terms, const pe_term *terms, void *d_W, void *d_work,
                     size_t work_bytes, void *stream);

/* The interior state of the FE function whose boundary values are the grid's
 * Dirichlet data at time t (pe_set_boundary) and which is otherwise the L2
 * projection of v (n_terms separable terms, time factors ignored): d_W
 * receives (kron_a Q_a)^T (F_v - M_IB g_B(t)).  This is the initial state
 * U(t0) with non-homogeneous data; without data it equals pe_project.  Same
 * workspace as pe_project.  Errors: PE_E_ARG (null pointers, non-finite t,
 * more than PE_MAX_TERMS terms with the data's two per data term),
 * PE_E_WORKSPACE. */
pe_status pe_project_state(pe_grid g, int32_t n_terms, const pe_term *terms, double t, void *d_W,
                           void *d_work, size_t work_bytes, void *stream);

/* Fine propagator F on all slices at once (paper, Section 2.3: F is J steps
 * of eq. (2.6) with step dt = dT/J and q nodes):
 *     d_Uout[n] = F^J(d_Uin[n]; t0 + n*dT),   n = 0..n_slices-1.
 * d_Uin and d_Uout are [n_slices][DOF] states (they must not overlap);
 * cF[0..q-1] (host) are the stage nodes, d_EF / d_BF the tables of
 * pe_phi_tables(g, dT/J, q, cF).  Each step evaluates the load vector of f at
 * the q stage times on the full grid (Gauss quadrature), transforms it to
 * spectral space by d dense per-axis DST products on the matrix cores, and
 * applies the diagonal update  V <- E V + sum_i B_i g_i.  Needs at least
 * pe_fine_workspace_bytes(g, q) bytes of d_work (unless f has no terms); more workspace lets more
 * (slice, step, stage) fields be transformed per launch (the value for
 * `fields` fields is pe_fine_workspace_bytes(g, fields)).
 * Errors: PE_E_ARG, PE_E_WORKSPACE, PE_E_HIP. */
size_t pe_fine_workspace_bytes(pe_grid g, int64_t fields);
pe_status pe_fine_propagate(pe_grid g, int32_t n_slices, double t0, double dT, int32_t J,
                            int32_t q, const double *cF, const double *d_EF, const double *d_BF,
                            const void *d_Uin, void *d_Uout, void *d_work, size_t work_bytes,
                            void *stream);

/* Coarse propagator G and the Parareal correction (paper Algorithm 1 and
 * eq. (2.8)), G(v; T_n) = E_G v + r_n (+ d_corr[n]) with
 *     r_n = dT sum_i b_i(dT D lambda) P_h f(T_n + c_i dT),   T_n = t0 + n dT.
 *  - compute_r != 0: first fill d_r[n] (n = 0..N-1) with r_n (all slices in
 *    parallel); compute_r == 0 reuses d_r as given.
 *  - d_Uprev == NULL (plain coarse sweep: the sequential coarse start of Algorithm 1):
 *        d_U[n+1] = G(d_U[n]; T_n),                 n = 0..N-1
 *  - d_Uprev != NULL and d_Fout != NULL (correction sweep, eq. (2.8)):
 *        d_U[n+1] = G(d_U[n]) + d_Fout[n] - G(d_Uprev[n])
 *    d_U[0] is read, never written.  d_U, d_Uprev are [N+1][DOF] states,
 *    d_Fout, d_r and d_corr (nullable: no learned correction) [N][DOF];
 *    d_U must not overlap any of the arrays it is computed from (PE_E_ARG
 *    when it starts at the same address as one of them).
 *  - d_norms (nullable, 3 doubles, device): d_norms[0] = sum over n = 1..N of
 *    ||d_U[n] - d_Uprev[n]||^2 (the jump; 0 without d_Uprev), d_norms[1] =
 *    sum over n = 1..N of ||d_U[n]||^2, d_norms[2] = sum over n = 0..N-1 of
 *    ||d_Uprev[n+1] - d_Fout[n]||^2 (the residual of the previous iterate
 *    when d_Fout[n] = F^J(d_Uprev[n]); 0 without d_Uprev), accumulated in
 *    FP64 in a fixed order (bitwise repeatable).
 * Needs pe_coarse_workspace_bytes(g, N, p) bytes of d_work (a smaller
 * workspace still works when it holds the norm partials and p stage fields;
 * r_n is then computed a few slices at a time). */
size_t pe_coarse_workspace_bytes(pe_grid g, int32_t n_slices, int32_t p);
pe_status pe_coarse_sweep(pe_grid g, int32_t n_slices, double t0, double dT, int32_t p,
                          const double *cG, const double *d_EG, const double *d_BG,
                          int32_t compute_r, void *d_r, const void *d_corr, const void *d_Uprev,
                          const void *d_Fout, void *d_U, double *d_norms, void *d_work,
                          size_t work_bytes, void *stream);

/* For callers that cannot allocate or pass workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the sweep
 * of pe_coarse_sweep with r given (compute_r = 0), the same kernels and the
 * same results bit for bit, whose norm partials live in a static device
 * array of the library (3 MiB per GPU, held until the process ends) instead
 * of d_work.  The call allocates nothing and takes no workspace.  Arguments
 * as in pe_coarse_sweep.  Grids are limited to PE_NOALLOC_MAX_DOF
 * coefficients.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two host threads) race and may return
 * wrong norms; calls ordered on one stream are safe (each call writes the
 * partials it reads).  Errors: PE_E_ARG (null pointers, n_slices < 1,
 * overlapping d_U, a grid beyond the limit), PE_E_HIP. */
#define PE_NOALLOC_MAX_DOF (1 << 25)
pe_status pe_coarse_sweep_noalloc(pe_grid g, int32_t n_slices, const double *d_EG,
                                  const void *d_r, const void *d_corr, const void *d_Uprev,
                                  const void *d_Fout, void *d_U, double *d_norms, void *stream);

/* ------------------------------------------------------------------------
 * Learned coarse correction (an addition to the paper's method).
 *
 * G~(v; T_n) = E_G v + r_n + delta_n with, for every mode k,
 *     delta_{n,k} = s * dT * NN(x),
 *     g_j = ghat_k(T_n + j dT / 7), j = 0..7   (spectral forcing samples),
 *     c = Q^T g,  Q[j][i] = q_i(t_j), t_j = (j - 3.5)/3.5, q_0..q_7 the
 *         orthonormal polynomials of those points (Gram-Schmidt of the
 *         monomials 1, t, .., t^7; q_i has degree i, positive leading term),
 *     s = |(c_4, .., c_7)|   (the part of the samples of degree >= 4),
 *     x = [ln(z)/8, e^{-z}, phi_1(-z), 2 phi_2(-z), c_0/|g| .. c_3/|g|,
 *          c_4/s .. c_7/s],
 *     z = D lambda_k dT,  phi_1(-z) = (1 - e^{-z})/z,  phi_2(-z) = (z - 1 + e^{-z})/z^2,
 * (delta = 0 where s = 0; zero parts give zero features).  An s-stage
 * exponential Runge-Kutta step integrates forcing that is a polynomial of
 * degree < s in time exactly (its weights, eq. (2.7), come from the Lagrange
 * interpolant), so for s >= 4 the fine-coarse difference depends only on the
 * part of degree >= 4, which sets the scale s.  NN: 12 -> 64 -> 64 -> 64
 * (GELU x Phi(x)) -> 1, bf16 weights, fp32 accumulation, on the matrix cores;
 * the inputs enter the first layer as a bf16 hi + lo pair (no input rounding).
 * Because delta does not depend on the state, the Parareal iterates k >= 1
 * are unchanged by it (Algorithm 1 with eq. (2.8) still converges to the fine
 * solution): the correction only moves U^(0) and hence the iteration count.
 * Parameters: PE_MLP_PARAMS floats, W1[12][64], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], w4[64], b4[1] (W[in][out]).  A pe_mlp holds fp32
 * master weights, their bf16 copies and Adam moments on the device.
 * Training rows: target (R_n - r_n)_k / (s dT), R_n = F^J(0), r_n = G(0)
 * on slice n (the state-independent fine/coarse forcing responses). */
#define PE_MLP_INPUTS 12
#define PE_MLP_WIDTH 64
#define PE_MLP_PARAMS 9217
#define PE_MLP_SAMPLES 8

typedef struct pe_mlp_s *pe_mlp;

/* Create a network from PE_MLP_PARAMS host floats (its initial weights;
 * Adam moments start at zero).  Synchronises.  Errors: PE_E_ARG, PE_E_HIP. */
pe_status pe_mlp_create(pe_mlp *out, const float *h_params, void *stream);
void pe_mlp_free(pe_mlp m);
/* Copy the fp32 master weights to / from host memory (synchronises). */
pe_status pe_mlp_get_params(pe_mlp m, float *h_params, void *stream);
pe_status pe_mlp_set_params(pe_mlp m, const float *h_params, void *stream);

/* y[r] = NN(x[r]) for rows of ready-made inputs d_x[rows][12] (fp32). */
pe_status pe_mlp_forward(pe_mlp m, int64_t rows, const float *d_x, float *d_y, void *stream);

/* One training step on a batch: mean squared error of NN(x) against d_t.
 * Gradients are accumulated in a fixed order (bitwise repeatable).
 * d_loss (nullable, 1 float) receives the batch loss, d_grad (nullable,
 * PE_MLP_PARAMS floats) the batch gradient; apply != 0 then takes one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step count kept in
 * the handle) with learning rate lr.  rows: 1 .. 2^24. */
pe_status pe_mlp_train_step(pe_mlp m, int64_t rows, const float *d_x, const float *d_t, float lr,
                            int32_t apply, float *d_loss, float *d_grad, void *stream);

/* Spectral forcing samples for every slice: d_samples[8n + s][k] =
 * ghat_k(t0 + n dT + s dT/7) (grid state dtype), n = 0..N-1, computed like
 * the fine stages (quadrature + transform).  Needs
 * pe_learned_samples_workspace_bytes(g, N) of d_work (smaller workspaces
 * are used a few slices at a time). */
size_t pe_learned_samples_workspace_bytes(pe_grid g, int32_t n_slices);
pe_status pe_learned_samples(pe_grid g, int32_t n_slices, double t0, double dT, void *d_samples,
                             void *d_work, size_t work_bytes, void *stream);

/* Training rows of slices n = 0..N-1 starting at t0: for every (n, k) with
 * s > rel_thresh * max s, write x (12 floats) and the target
 * (R - r)_{n,k} / (s dT) to d_x / d_t and s to d_s (nullable), in (n, k)
 * order, at most max_rows; *h_count (host) receives the number of
 * qualifying rows (it can exceed max_rows: only the first max_rows are
 * written).  d_R, d_r: [N][DOF] (state dtype).  The inputs are formed from
 * the forcing set on the grid (term spectra and time factors; no samples
 * buffer).  Needs pe_learned_rows_workspace_bytes(g, N) of d_work.
 * Synchronises. */
size_t pe_learned_rows_workspace_bytes(pe_grid g, int32_t n_slices);
pe_status pe_learned_rows(pe_grid g, int32_t n_slices, double t0, double dT, const void *d_R,
                          const void *d_r, double rel_thresh, float *d_x, float *d_t, float *d_s,
                          int64_t max_rows, int64_t *h_count, void *d_work, size_t work_bytes,
                          void *stream);

/* delta_n for slices n = 0..N-1 starting at t0 and every mode into
 * d_corr[N][DOF] (state dtype), from the forcing set on the grid.  If the
 * network produces a non-finite value anywhere, d_corr is zeroed (plain
 * coarse step) and *h_fallback (host, nullable) is set to 1.  Needs
 * pe_learned_correction_workspace_bytes(g, N) of d_work (N * 8 * n_terms
 * doubles).  Synchronises.  Errors: PE_E_ARG, PE_E_WORKSPACE, PE_E_HIP. */
size_t pe_learned_correction_workspace_bytes(pe_grid g, int32_t n_slices);
pe_status pe_learned_correction(pe_grid g, pe_mlp m, int32_t n_slices, double t0, double dT,
                                void *d_corr, int32_t *h_fallback, void *d_work,
                                size_t work_bytes, void *stream);

/* Parareal driver (paper Algorithm 1).  Stopping rule (the paper leaves it
 * open): after iteration k the relative jump
 *     ||U^(k) - U^(k-1)|| / ||U^(k)||    (all slice ends n = 1..N, FP64)
 * is compared with tol; the loop stops when jump <= tol (converged = 1) or
 * after K_max fine passes (converged = 0, still PE_OK).  Beside it the
 * relative residual of each iterate, how far it is from a fine trajectory,
 *     ||U^{n+1,(k)} - F^J(U^{n,(k)})|| / ||U^(k)||   (n = 0..N-1, FP64),
 * is reported: F^J(U^(k)) is the fine pass of iteration k + 1, so after K
 * passes the residuals of iterates 0..K-1 are known. */
typedef struct {
  double t0;
  double T;
  int32_t N;                   /* coarse slices */
  int32_t J;                   /* fine steps per slice */
  int32_t p;                   /* coarse stages */
  int32_t q;                   /* fine stages */
  double cG[PE_MAX_STAGES];
  double cF[PE_MAX_STAGES];
  int32_t K_max;               /* 1..PE_MAX_ITERS fine passes at most */
  double tol;
  const void *d_corr;          /* nullable [N][DOF] additive coarse correction */
  pe_mlp mlp;                  /* nullable: learned correction computed inside the
                                  solve (ignored when d_corr is given) */
} pe_solve_params;

typedef struct {
  int32_t iterations;          /* fine passes performed */
  int32_t converged;
  double jumps[PE_MAX_ITERS];  /* jumps[k-1]: relative jump of iterate k */
  double ms_tables;            /* phi tables (both step sizes) */
  double ms_coarse;            /* r_n and the initial coarse sweep */
  double ms_fine;              /* all fine passes */
  double ms_sweep;             /* correction sweeps + norms */
  double ms_total;
  double ms_learned;           /* forcing samples + network (inside ms_coarse) */
  int32_t fallback;            /* 1: the network output was non-finite, plain G used */
  double residuals[PE_MAX_ITERS]; /* residuals[k-1]: relative residual of iterate k-1,
                                     measured during fine pass k */
} pe_solve_report;

/* d_U0: initial state (one state, nullable = zero); d_U receives the last
 * iterate [N+1][DOF].  Needs pe_solve_workspace_bytes(g, P) of d_work (with
 * P->mlp set this includes the forcing samples and the correction).
 * Synchronises `stream` after the coarse start and once per iteration (one
 * 24-byte read-back of the jump and residual norms).  Errors: PE_E_ARG,
 * PE_E_WORKSPACE, PE_E_HIP, PE_E_NUMERIC
 * (non-finite jump). */
size_t pe_solve_workspace_bytes(pe_grid g, const pe_solve_params *P);
pe_status pe_parareal_solve(pe_grid g, const pe_solve_params *P, const void *d_U0, void *d_U,
                            void *d_work, size_t work_bytes, pe_solve_report *rep, void *stream);

/* Kernel timing, for benchmarks.  While enabled, the library brackets every
 * launch of its main kernels with HIP events recorded on the launch stream
 * and accumulates, per kernel class, the launch count, the summed event time
 * and the algorithmic work of those launches: matrix-core flops of the
 * folded transform (per field and axis pass, 2 (DOF/n_a) Kh_a^2 with two
 * fold levels, 2 (DOF/n_a) (ceil(n_a/2)^2 + floor(n_a/2)^2) with one; split
 * passes count their three bf16 products) and HBM bytes (each array read or
 * written once, unpadded).  pe_set_timing(g, 1) enables
 * and resets the counters, pe_set_timing(g, 0) disables.  pe_get_timing
 * waits for the recorded events and fills out[0..PE_K_COUNT-1].  Errors:
 * PE_E_ARG, PE_E_HIP. */
typedef enum {
  PE_K_DST_LAST = 0,  /* last-axis DST pass (with fused load quadrature) */
  PE_K_DST_MID = 1,   /* DST pass along any other axis */
  PE_K_LOAD = 2,      /* separate stage load-vector quadrature */
  PE_K_UPDATE = 3,    /* fused diagonal update */
  PE_K_SWEEP = 4,     /* coarse / correction sweep with norms */
  PE_K_MID_UPDATE = 5,  /* axis-0 DST pass fused with the diagonal update */
  PE_K_COARSE_FORCING = 6, /* every launch computing the coarse forcing r_n (its
                              quadrature, transform and update kernels) */
  PE_K_COUNT = 7
} pe_kernel_class;

typedef struct {
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} pe_kernel_stat;

pe_status pe_set_timing(pe_grid g, int32_t enable);
pe_status pe_get_timing(pe_grid g, pe_kernel_stat *out);

/* Grid queries. */
int64_t pe_grid_dof(pe_grid g);
int32_t pe_grid_precision(pe_grid g);

/* Message of the last failed call on this thread ("" if none). */
const char *pe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PEIFEM_H */
