/*
 * rfm.h -- C ABI of librfmnewton.so: randomized inexact preconditioned Newton
 * solvers (IPN and AMIPN) for random-feature-method (RFM) discretisations of
 * nonlinear PDEs, on one AMD Instinct MI355X (gfx950).
 *
 * Paper: "Robust and efficient solvers for nonlinear PDEs based on the random
 * feature method" (arXiv 2510.04170).
 *
 * Conventions for every call:
 *  - The return value is an rfm_status: 0 success, < 0 error (nothing useful
 *    was written), > 0 warning (outputs are written and usable).
 *  - rfm_last_error() gives a thread-local message for the last failing call.
 *  - Array arguments may be host or device pointers (checked with
 *    hipPointerGetAttributes); the library copies inputs during the call and
 *    never keeps a caller pointer.  Outputs go to caller buffers of the stated
 *    size.  All device work is ordered on the stream given to rfm_create, and
 *    every call that returns data to a host pointer synchronises that stream.
 *  - One problem object must not be used from two threads at once.
 *  - No C++ exception crosses this boundary.
 */
#ifndef RFM_H
#define RFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RFM_OK = 0,
  RFM_EINVAL = -1,     /* bad argument, shape or call order; nothing done */
  RFM_ENOMEM = -2,     /* device allocation failed */
  RFM_EDEVICE = -3,    /* a HIP call failed */
  RFM_ESINGULAR = -4,  /* R has a zero or non-finite diagonal entry: no preconditioner */
  RFM_ENUMERIC = -5,   /* non-finite input data or a non-finite residual */
  RFM_ENOCONV = 1,     /* warning: the outer iteration limit was reached */
  RFM_ESTALL = 2       /* warning: the line search found no decrease; u is the last iterate */
} rfm_status;

/* Message of the last failing call on this thread (never NULL). */
const char* rfm_last_error(void);

/* ------------------------------------------------------------------------
 * Problem description (Alg. 3 inputs: partition, collocation sets, basis,
 * operators, data, continuity order).
 * ---------------------------------------------------------------------- */

typedef struct rfm_problem rfm_problem;

/* Point kinds. */
enum { RFM_PDE = 0, RFM_DIRICHLET = 1, RFM_NEUMANN = 2, RFM_CONTINUITY = 3 };

/* Derivative selectors of a linear operator term. */
enum {
  RFM_D_ID = 0,                 /* the value                                   */
  RFM_D_X0 = 1, RFM_D_X1 = 2,   /* first derivative along axis k is 1 + k      */
  RFM_D_X2 = 3, RFM_D_X3 = 4,
  RFM_D_LAPLACE = 8,            /* sum of second derivatives over every axis   */
  RFM_D_LAPLACE_SPACE = 9       /* same, leaving out the last (time) axis      */
};

/* One term coeff * D u_comp of equation eq: the linear part lambda*L u (Sec. 2.1). */
typedef struct { int32_t eq, comp; double coeff; int32_t deriv; } rfm_lin_term;

/* One term coeff * prod_c u_c^pow[c] of equation eq: the nonlinear part mu*N(u)
 * restricted to polynomials of the field values.  At most 4 components. */
typedef struct { int32_t eq; double coeff; int32_t pow[4]; } rfm_poly_term;

/* One term coeff * f(u_comp) of equation eq with f one of the functions below:
 * the nonlinear part mu*N(u) for pointwise transcendental nonlinearities (the
 * cosh term of the 3-D Helmholtz problem of Sec. 6.2, e^u of the diffusion-reaction
 * problems).  Its Jacobian contribution is coeff * f'(u_comp) phi. */
typedef struct { int32_t eq, comp; double coeff; int32_t fn; } rfm_fn_term;
enum { RFM_FN_COSH = 0, RFM_FN_SINH = 1, RFM_FN_EXP = 2 };

/* Product term coeff * prod_k (D_k u_{comp_k})^{pow_k} of equation eq, with D_k
 * a derivative selector RFM_D_* of the field: the quasi-linear operators of the
 * paper's benchmarks written out, e.g. -div((1 + u^2) grad u) = -Lap u
 * - u^2 Lap u - 2 u |grad u|^2 (Sec. 3.2, Sec. 6.2).  Its Jacobian contribution
 * is, by the product rule, sum_k coeff pow_k (D_k u)^{pow_k - 1} (the other
 * factors) D_k phi. */
typedef struct { int32_t comp, deriv, pow; } rfm_factor;
typedef struct { int32_t eq; double coeff; int32_t nfac; rfm_factor fac[4]; } rfm_prod_term;

/* Create an empty problem on HIP device `device`.  dim: 1..4 coordinates
 * (time, if any, is the last one, Sec. 2.1); ncomp: 1..4 solution components,
 * with one equation per component.  hip_stream: a hipStream_t, or NULL for the
 * null stream. */
rfm_status rfm_create(rfm_problem** out, int32_t dim, int32_t ncomp, int32_t device, void* hip_stream);

/* Free everything the problem owns.  NULL is allowed. */
void rfm_destroy(rfm_problem* p);

/* Box Omega_c = prod [lo_a, hi_a] split into nsub[a] equal boxes per axis
 * (Sec. 2.2); box index e = i_0 + nsub_0 (i_1 + nsub_1 i_2 ...). */
rfm_status rfm_set_partition(rfm_problem* p, const double* lo, const double* hi, const int32_t* nsub);

/* Partition of unity (Sec. 2.2), before rfm_finalize.  RFM_POU_INDICATOR
 * (default): each box's features act on the box alone, and continuity rows join
 * neighbours.  RFM_POU_SMOOTH: u(x) = sum_e psi_e(x) sum_j phi_ej(x) u_ej with
 * psi_e = prod_a b(l_a(x)), b(y) = 1 for |y| <= 3/4, (1 - sin(2 pi |y|)) / 2 for
 * 3/4 <= |y| <= 5/4, 0 beyond, except that on an axis where the box touches
 * the boundary of Omega_c, b = 1 on the side facing it (so the psi_e sum to 1
 * on Omega_c); a row at x touches every box whose support holds x (at most
 * 2^dim), and no continuity groups are allowed (the blend is C1). */
enum { RFM_POU_INDICATOR = 0, RFM_POU_SMOOTH = 1 };
rfm_status rfm_set_partition_of_unity(rfm_problem* p, int32_t kind);

/* J tanh features per box and component (Sec. 2.2):
 *   phi_{e,c,j}(x) = tanh(sum_a W[e][c][j][a] (x_a - mu_{e,a}) / sigma_{e,a} + b[e][c][j]),
 * with mu, sigma the centre and half-width of box e.  W: [nbox][ncomp][J][dim],
 * b: [nbox][ncomp][J].  Unknowns are ordered [box][component][feature]:
 * n = nbox * ncomp * J.  J may be at most 8192 (the widest Jacobian row is
 * ncomp*J for PDE rows and 2*J for continuity rows; both must be <= 16384).
 * Rows of up to 1024 values are assembled from registers, wider rows by
 * recomputing the features over three sweeps of the row. */
rfm_status rfm_set_features(rfm_problem* p, int32_t J, const double* W, const double* b);

/* Append one point group.  Every point of the group belongs to box `owner`
 * (indicator partition of unity, Sec. 5); continuity groups also name the
 * box `neighbor` across the interface.  Rows are appended in the order
 * (equation or component, continuity order, point):
 *  RFM_PDE:        one row per equation (comp = -1) or for equation comp;
 *                  residual  sum lin + sum poly + sum fn - data[p][q]  (Alg. 3 step 1);
 *                  data: [npts][neq_sel]
 *  RFM_DIRICHLET:  u_c(x) - data[p][k]            (Alg. 3 step 3), data [npts][ncomp_sel]
 *  RFM_NEUMANN:    normal . grad u_c(x) - data[p][k],               data [npts][ncomp_sel]
 *  RFM_CONTINUITY: D^s u_c^{owner}(x) - D^s u_c^{neighbor}(x) for s < cont_order,
 *                  D^0 the value and D^1 the derivative along normal[p]
 *                  (eqs. con:1-3, Alg. 3 step 2); data must be NULL.
 * x: [npts][dim]; normal: [npts][dim] for NEUMANN and CONTINUITY, else NULL;
 * comp: -1 for all components/equations or one index; cont_order: 1 or 2.
 * npts may be 0 (nothing is added). */
rfm_status rfm_add_points(rfm_problem* p, int32_t kind, int64_t npts, const double* x, int32_t owner,
                          int32_t neighbor, const double* normal, int32_t comp, int32_t cont_order,
                          const double* data);

/* Operator P(u) = sum of linear terms + sum of polynomial terms (Sec. 2.1)
 * (+ the pointwise terms of rfm_set_fn_terms and the product terms of
 * rfm_set_prod_terms, which this call leaves in place).
 * At most 16 linear and 8 polynomial terms. */
rfm_status rfm_set_operator(rfm_problem* p, const rfm_lin_term* lin, int32_t nlin,
                            const rfm_poly_term* nl, int32_t nnl);

/* Pointwise terms coeff * f(u_comp) added to the operator (Sec. 2.1, Sec. 6.2):
 * replaces any earlier ones; at most 8 (n = 0 removes them).  eq and comp in
 * [0, ncomp), fn one of RFM_FN_*, finite coeff, else RFM_EINVAL / RFM_ENUMERIC.
 * Like rfm_set_operator it may be called again after rfm_finalize. */
rfm_status rfm_set_fn_terms(rfm_problem* p, const rfm_fn_term* terms, int32_t n);

/* Product terms (rfm_prod_term) added to the operator: replaces any earlier ones;
 * at most 8 terms (n = 0 removes them) of 1..4 factors each, with powers 1..8, eq
 * and comp in [0, ncomp), deriv a selector valid for the problem's dimension,
 * finite coeff, and at most 8 distinct (comp, deriv) pairs over all terms; else
 * RFM_EINVAL / RFM_ENUMERIC.  May be called again after rfm_finalize. */
rfm_status rfm_set_prod_terms(rfm_problem* p, const rfm_prod_term* terms, int32_t n);

/* Replaces the data of point group `group` (numbered in rfm_add_points order;
 * not a continuity group): data [npts][ncomp] for comp = -1, else [npts].
 * rfm_set_operator and rfm_set_group_data may be called again after
 * rfm_finalize -- the layout does not depend on coefficients or data -- so one
 * problem object (and the projection factor it keeps) can serve a family of
 * solves that differ only in parameters. */
rfm_status rfm_set_group_data(rfm_problem* p, int32_t group, const double* data);

/* Finish the description: builds the row and tile layout and uploads it.  Called
 * implicitly by the first compute call; no points may be added afterwards. */
rfm_status rfm_finalize(rfm_problem* p);

int64_t rfm_num_unknowns(const rfm_problem* p);  /* n, or -1 before features are set */
int64_t rfm_num_rows(const rfm_problem* p);      /* m (after rfm_finalize), else -1 */
/* nnz(J): the values the block-sparse Jacobian stores, each row over the columns of the
 * box (or boxes) its point touches (after rfm_finalize), else -1.  The algorithmic work
 * of the sketch is 2 s nnz(J) flops and of one product J x or J^T y nnz(J) values read. */
int64_t rfm_num_jacobian_values(const rfm_problem* p);

/* ------------------------------------------------------------------------
 * Solver (Alg. 1 IPN, Alg. 2 AMIPN)
 * ---------------------------------------------------------------------- */

enum { RFM_IPN = 0, RFM_AMIPN = 1 };
enum { RFM_PREC_F64 = 0, RFM_PREC_F32 = 1, RFM_PREC_BF16 = 2, RFM_PREC_FP8 = 3 };
enum { RFM_SKETCH_GAUSSIAN = 0, RFM_SKETCH_COUNT = 1 };

typedef struct {
  int32_t method;          /* RFM_IPN or RFM_AMIPN                                  */
  double sketch_factor;    /* gamma: sketch rows s = ceil(gamma * n), gamma > 1      */
  uint64_t sketch_seed;    /* key word 0 of the Philox4x64-10 sketch generator       */
  double lsqr_tol;         /* eta: LSQR atol = btol                                  */
  int32_t lsqr_max_iter;
  double outer_tol;        /* epsilon of the stop test | ||F_{k+1}|| - ||F_k|| |      */
  int32_t max_outer;       /* K                                                      */
  int32_t m_max;           /* AMIPN: inner steps per Jacobian                        */
  double tau_rel;          /* AMIPN: early-stop threshold                            */
  double row_scale_c;      /* c of the row scale c / max_j |J_ij| (Sec. 5)            */
  int32_t gs_iters;        /* golden-section iterations after a rejected full step   */
  int32_t sketch_prec;     /* RFM_PREC_F64 | RFM_PREC_BF16 | RFM_PREC_FP8 (see rfm_stage_sketch) */
  int32_t lsqr_prec;       /* RFM_PREC_F64 | RFM_PREC_F32: copy of D J in the LSQR products;
                              F32 falls back to F64 for the rest of the solve at the first
                              step whose LSQR hits lsqr_max_iter or whose line search finds
                              no decrease */
  int32_t sketch_pieces;   /* pieces of D J in a BF16/FP8 sketch, 1..16; 0: 6 (BF16), 12 (FP8) */
  int32_t sketch_kind;     /* RFM_SKETCH_GAUSSIAN (default) or RFM_SKETCH_COUNT (FP64 only) */
  int32_t verbose;         /* 1: one line per outer step on stderr                   */
  int32_t sketch_rows_per_pass; /* 0: the whole sketch B (s x n) is formed and factored at once
                              unless B, R and the QR workspace would take more than 60% of the
                              device memory; then, or with a value > 0 (rounded down to a multiple
                              of 128, at most 98,304), B is produced that many rows at a time and
                              each block folded into R (rfm_stage_sketch_qr_streamed,
                              rfm_stage_count_sketch_qr_streamed): either sketch kind. */
  int32_t jac_index0;      /* index of the solve's first Jacobian evaluation (key word 1 of the
                              sketch generator; later evaluations count up from it), so that a
                              solve can be resumed from an iterate of another one; default 0 */
} rfm_solve_opts;

#define RFM_MAX_STEPS 64
typedef struct {
  int32_t outer_iters;               /* IT */
  int32_t jac_evals;                 /* NJ: Jacobian + preconditioner evaluations */
  int32_t lsqr_iters_total;
  int32_t nsteps;                    /* Newton directions computed (<= RFM_MAX_STEPS logged) */
  int32_t lsqr_iters[RFM_MAX_STEPS];
  double alphas[RFM_MAX_STEPS];
  double resnorms[RFM_MAX_STEPS];    /* ||D F|| after each step */
  double final_resnorm;
  /* wall time per stage in seconds: host clock around the stage, which ends by waiting for
     the problem's stream (so each figure includes the launch overhead of its kernels) */
  double t_assemble, t_sketch, t_qr, t_lsqr, t_linesearch, t_total;
  int32_t status_detail;
  int32_t lsqr_fp64_fallback;        /* 1: lsqr_prec F32 was abandoned for FP64 during the solve */
  int32_t inner_steps[RFM_MAX_STEPS]; /* Newton directions computed in each outer step (IPN: 1) */
  int32_t flags[RFM_MAX_STEPS];      /* Alg. 2's Flag after each outer step: 1 = a fresh Jacobian and
                                        preconditioner for the next one (IPN: always 1) */
} rfm_solve_stats;

/* Paper values: gamma 3, eta 1e-6, epsilon 1e-10, tau 1e-3, m_max 3, c 100 (Sec. 6). */
void rfm_solve_opts_default(rfm_solve_opts* o);

/* Solve min ||F(u)|| from the initial coefficients u_inout[n]; the result is
 * written back to u_inout.  stats may be NULL. */
rfm_status rfm_solve(rfm_problem* p, const rfm_solve_opts* opts, double* u_inout, rfm_solve_stats* stats);

/* Unscaled residual F(u) (F may be NULL) and ||F||_2. */
rfm_status rfm_residual(rfm_problem* p, const double* u, double* F, double* norm);

/* The random-feature field of coefficients u (Sec. 2.2) at npts points x [npts][dim]
 * with their owner boxes owner [npts] (indicator partition: the box whose features
 * represent the field there; smooth partition: any box whose support holds the
 * point, the call sums over the boxes whose bump is non-zero at it).
 *   what RFM_EVAL_VALUE: out [npts][ncomp] = u_n(x);
 *   what RFM_EVAL_GRAD:  out [npts][ncomp][dim] = grad u_n(x), from
 *                        d_a phi = (1 - t^2) w_a / sigma_a (and the product rule with
 *                        the bump under the smooth partition); with the manufactured
 *                        gradient this gives the H1 errors the experiments report.
 * RFM_EINVAL for an owner outside [0, nbox) or another `what`, before device work. */
enum { RFM_EVAL_VALUE = 0, RFM_EVAL_GRAD = 1 };
rfm_status rfm_eval(rfm_problem* p, const double* u, int64_t npts, const double* x, const int32_t* owner,
                    int32_t what, double* out);

/* ------------------------------------------------------------------------
 * Stage calls.  Each runs one step of the per-Newton-step pipeline on the
 * problem's internal state so that it can be checked on its own.
 * ---------------------------------------------------------------------- */

/* Residual and Jacobian at u, row-scaled: D = c / max_j |J_ij| (1 for a zero
 * row), kept as the current Jacobian (Alg. 3 and Sec. 5 scaling). */
rfm_status rfm_stage_assemble(rfm_problem* p, const double* u, double row_scale_c);

/* Copies of the current scaled residual D F [m], the scale D [m], and rows
 * [r0, r0 + nrows) of the scaled Jacobian D J as a dense row-major block
 * [nrows][n]. */
rfm_status rfm_get_scaled_residual(rfm_problem* p, double* DF);
rfm_status rfm_get_row_scale(rfm_problem* p, double* D);
rfm_status rfm_get_jacobian_rows(rfm_problem* p, int64_t r0, int64_t nrows, double* out);

/* y = (D J) x  [m]   and   x = (D J)^T y  [n] with the current Jacobian. */
rfm_status rfm_jmul(rfm_problem* p, const double* x, double* y);
rfm_status rfm_jtmul(rfm_problem* p, const double* y, double* x);

/* x = (D J)^T y as rfm_jtmul, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * this call allocates nothing.  y [m] and x [n] must be device pointers; the work is
 * queued on the problem's stream and the call returns without waiting for it.  The
 * problem must be finalized with a Jacobian assembled (rfm_stage_assemble or a solve),
 * else RFM_EINVAL.  The per-tile partial sums go to a fixed device array of
 * 8,388,608 doubles (64 MiB) that the library holds on every GPU it runs on until the
 * process ends: a Jacobian needing more partials (one per stored value of a tile's
 * row, about nnz(J)/60) is refused with RFM_EINVAL.  Every call on one GPU shares
 * that array and nothing carries over between calls (each call writes every partial
 * it reads), so calls whose work overlaps on one GPU -- two streams, two threads --
 * race and must be serialised by the caller. */
rfm_status rfm_jtmul_noalloc(rfm_problem* p, const double* y, double* x);

/* Sketch B = S (D J) / sqrt(s) with s = ceil(gamma n) rows (Sec. 4.1, with a
 * Gaussian-like S in place of the count sketch), kept as the current B in FP64.
 *   prec RFM_PREC_F64: S[i][r] ~ N(0,1) from Philox4x64-10 (Salmon et al.,
 *     SC'11) with counter (i/8, r, 0, 0) and key (seed, jac_index); 64-bit
 *     output word w gives rows 8(i/8) + 2w, + 2w + 1 by Box-Muller on
 *     u1 = (hi32 + 1) 2^-32, u2 = lo32 2^-32.  Product in FP64.
 *   prec RFM_PREC_BF16 / RFM_PREC_FP8: S[i][r] = K[b] / k_s with b byte
 *     (i mod 32) of the Philox block for counter (i/32, r, 1, 0) (byte j = bits
 *     8(j%8).. of word j/8) and K the code table of rfm_sketch_table (k_s = 32
 *     for BF16, 4 for FP8).  D J is cut into `pieces` integer parts (0: 6 for
 *     BF16, 12 for FP8) on a fixed-point grid per (column, chunk): the chunks
 *     of a column block are four consecutive entries of its list of 32-row
 *     groups (rows 32g .. 32g+31 holding a row that touches the block,
 *     ascending, padded to a multiple of four); with E = floor(log2 max|D J|)+1
 *     over the chunk, part p is q_p 2^(E - b(p+1)), q_p the integer nearest the
 *     remaining value / 2^(E - b(p+1)), b = 8 (BF16) or 4 (FP8).  The matrix
 *     cores form S times each part exactly (integer sums below 2^24 in FP32);
 *     the chunk sums are combined in FP64.
 * Runs on the problem's stream and synchronizes it. */
rfm_status rfm_stage_sketch(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index, int32_t prec,
                            int32_t pieces);

/* Count sketch B = S (D J) (Sec. 4.1 as the paper states it), s = ceil(gamma n)
 * rows, kept as the current B: S[h(r)][r] = sigma(r), the only non-zero of
 * column r, with h(r) = w0 mod s and sigma(r) = +1 if bit 0 of w1 is clear, else
 * -1, where (w0, w1, ..) = Philox4x64-10 at counter (r, 0, 2, 0), key (seed,
 * jac_index).  One pass over D J; sums within a bucket in row order (no
 * atomics).  Runs on the problem's stream and synchronizes it. */
rfm_status rfm_stage_count_sketch(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index);

/* The 256 integer codes of the low-precision sketch: K[b] = the integer nearest
 * (ties to even) to k_s Phi^{-1}((b + 1/2) / 256), k_s = 32 for RFM_PREC_BF16
 * and 4 for RFM_PREC_FP8; out[256] on the host.  Needs no problem and no device. */
rfm_status rfm_sketch_table(int32_t prec, double* out);

/* Low-precision sketch operand of column block `block` (box e, component c ->
 * e * ncomp + c), as formed by the last BF16/FP8 rfm_stage_sketch: number of
 * 32-row slots (-1 on a bad argument), and for slots [slot0, slot0 + nslots)
 * the values of part `piece`, q_p 2^(E - b(p+1)), out[nslots][J][32] (row
 * 32 g + k, column j of the block at [slot][j][k]), the group g of each slot
 * (groups[nslots], -1 for padding; may be NULL) and the exponent E of the
 * slot's chunk per column (scale_exp[nslots][J]; may be NULL). */
int64_t rfm_sketch_operand_slots(rfm_problem* p, int32_t block);
rfm_status rfm_get_sketch_operand(rfm_problem* p, int32_t piece, int32_t block, int64_t slot0, int64_t nslots,
                                  double* out, int32_t* groups, int32_t* scale_exp);

/* Columns [c0, c0 + ncols) of the current sketch B, column-major [ncols][s]. */
rfm_status rfm_get_sketch_cols(rfm_problem* p, int64_t c0, int64_t ncols, double* out);
int64_t rfm_sketch_rows(const rfm_problem* p);

/* Thin QR of the current sketch (Alg. 1 step 2): keeps R [n][n] upper
 * triangular with a positive diagonal, in 64 x 64 tiles of its upper triangle
 * (n (n + 64) / 2 doubles, rounded up to whole tiles), and beside it the tiles
 * on and next to the diagonal in the triangular solves' own layout (385 n
 * doubles, n rounded up to a multiple of 64).  RFM_ESINGULAR if a diagonal
 * entry is zero or not finite. */
rfm_status rfm_stage_qr(rfm_problem* p);

/* Sketch and QR without holding B (for sketches larger than the device memory
 * allows): the s = ceil(gamma n) rows of B = S (D J) (Gaussian, prec as in
 * rfm_stage_sketch) are produced rows_per_pass at a time (a multiple of 128, at
 * most 98,304; 0 picks about an eighth of the device memory) and each block B_k
 * folded into R by the QR of [R; B_k] (R starts at 0).  R is the factor of the
 * whole B (up to rounding), with a positive diagonal; B is not kept.  Memory:
 * (512 + rows_per_pass) x n doubles for the block and R's 512 rows in work, and
 * R's storage as rfm_stage_qr.  RFM_ESINGULAR as rfm_stage_qr. */
rfm_status rfm_stage_sketch_qr_streamed(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index,
                                        int32_t prec, int32_t pieces, int64_t rows_per_pass);

/* The same for the count sketch of rfm_stage_count_sketch (Sec. 4.1): each pass
 * clears its block of B's rows and sums into it the signed rows of D J whose
 * bucket falls in the block, in ascending row order as the whole sketch does.
 * Arguments, memory and errors as rfm_stage_sketch_qr_streamed. */
rfm_status rfm_stage_count_sketch_qr_streamed(rfm_problem* p, double gamma, uint64_t seed, uint64_t jac_index,
                                              int64_t rows_per_pass);

/* Columns [c0, c0 + ncols) of R, column-major [ncols][n] (zeros below the diagonal). */
rfm_status rfm_get_r_cols(rfm_problem* p, int64_t c0, int64_t ncols, double* out);

/* x = R^{-1} y and x = R^{-T} y with the current R ([n] vectors). */
rfm_status rfm_r_solve(rfm_problem* p, const double* y, double* x);
rfm_status rfm_rt_solve(rfm_problem* p, const double* y, double* x);

/* LSQR on min || (D J) R^{-1} y - rhs || with tolerance tol (Paige-Saunders rules 1
 * and 2, atol = btol = tol), y0 = 0; returns y [n], the iteration count and the
 * stop rule (1, 2, or 0 for the iteration limit).  prec RFM_PREC_F32 multiplies
 * by D J rounded once to FP32 (products and sums in FP64); RFM_PREC_F64 by D J. */
rfm_status rfm_stage_lsqr(rfm_problem* p, const double* rhs, double tol, int32_t max_iter, int32_t prec, double* y,
                          int32_t* iters, int32_t* istop);

/* Golden-section line search on phi(a) = ||D F(u + a du)|| with the current row
 * scale D: the full step when phi(1) <= (1 - 1e-4) phi(0), else gs_iters golden
 * iterations on [0, 1]; returns the step (0 when nothing decreases phi) and phi. */
rfm_status rfm_stage_linesearch(rfm_problem* p, const double* u, const double* du, int32_t gs_iters,
                                double* alpha, double* phi);

/* ------------------------------------------------------------------------
 * Learned initial guess.  A coordinate network maps (PDE parameters, x) to
 * the solution values; its output at the PDE collocation points is projected
 * onto the random-feature basis by one sketched least-squares fit, giving the
 * first Newton iterate.  The plain zero guess stays the fallback and the
 * FP64 solver decides the final error.  (Not part of the paper's method.)
 * ---------------------------------------------------------------------- */

typedef struct rfm_mlp rfm_mlp;

/* Network in_dim -> width (tanh) x depth -> out_dim (linear last layer),
 * Glorot-uniform weights from `seed`, zero biases; device memory on `device`,
 * work on `stream` (NULL: the null stream).  Parameters are FP32; layer l
 * holds W_l [dout][din] row-major, then b_l [dout], layers in order. */
rfm_status rfm_mlp_create(rfm_mlp** out, int32_t in_dim, int32_t width, int32_t depth, int32_t out_dim,
                          uint64_t seed, int32_t device, void* stream);
void rfm_mlp_destroy(rfm_mlp* net);
int64_t rfm_mlp_num_params(const rfm_mlp* net);                 /* -1 for NULL */
rfm_status rfm_mlp_get_params(rfm_mlp* net, float* out);        /* [num_params], host or device */
rfm_status rfm_mlp_set_params(rfm_mlp* net, const float* in);   /* also clears the Adam state */

/* RFM_PREC_BF16 (default): layer products on the BF16 matrix cores with FP32
 * accumulation; RFM_PREC_F32: the same products in FP32 (for checking). */
rfm_status rfm_mlp_set_precision(rfm_mlp* net, int32_t prec);

/* Y [n][out_dim] = net(X [n][in_dim]) (host or device arrays). */
rfm_status rfm_mlp_predict(rfm_mlp* net, const float* X, int64_t n, float* Y);

/* Mean-squared error mean((net(X) - Y)^2) over all n * out_dim entries and
 * its gradient with respect to the parameters (grad [num_params] or NULL). */
rfm_status rfm_mlp_loss_grad(rfm_mlp* net, const float* X, const float* Y, int64_t n, double* loss, float* grad);

typedef struct {
  int32_t steps;           /* Adam steps                                          */
  int32_t batch;           /* samples per step (the whole set, in order, if >= n) */
  float lr, beta1, beta2, eps;
  float lr_final;          /* > 0: step size decays geometrically from lr to lr_final over the steps */
  uint64_t seed;           /* batch draw: row Philox4x64-10((step, i, 2, 0), (seed, 0))[0] mod n */
} rfm_train_opts;

/* steps 2000, batch 8192, lr 1e-3 (constant: lr_final 0), betas 0.9 / 0.999, eps 1e-8, seed 1 */
void rfm_train_opts_default(rfm_train_opts* o);

/* Minimises the mean-squared error on (X [n][in_dim], Y [n][out_dim]) with
 * Adam (Kingma & Ba 2015); loss_log [steps] (or NULL) gets each step's batch
 * loss before the update. */
rfm_status rfm_mlp_train(rfm_mlp* net, const float* X, const float* Y, int64_t n, const rfm_train_opts* opts,
                         double* loss_log);

/* The PDE collocation points of a problem, in row order: their number, and
 * x [npde][dim] with owner boxes [npde] (either may be NULL). */
int64_t rfm_num_pde_points(rfm_problem* p);
rfm_status rfm_get_pde_points(rfm_problem* p, double* x, int32_t* owner);

/* Sketched least-squares fit of field values at the PDE points onto the
 * feature basis: u_out [n] = argmin || D (Phi u - values) ||, Phi the feature
 * values at the PDE points (values [npde][ncomp]), D the row scale
 * c / max |Phi_row| (c = opts->row_scale_c); solved by LSQR (opts->lsqr_tol,
 * lsqr_max_iter) preconditioned with the R of a Gaussian sketch of D Phi
 * (opts->sketch_factor, sketch_seed), which is formed on the first call and
 * kept.  resnorm (or NULL) gets the weighted residual norm. */
rfm_status rfm_project(rfm_problem* p, const rfm_solve_opts* opts, const double* values, double* u_out,
                       double* resnorm);

/* The network inputs of one parameter draw at the problem's PDE points, in row
 * order: X [npde][nparam + dim] (host or device) with row k = (encoded params, x_k).
 * With param_lo and param_hi (each [nparam]) parameter j is encoded as
 * 2 (params[j] - lo_j) / (hi_j - lo_j) - 1, so that a family's ranges map onto
 * [-1, 1]; with both NULL the parameters are used as given.  RFM_EINVAL for only
 * one of them, or a range with lo_j >= hi_j; RFM_ENUMERIC for a non-finite
 * parameter.  Training sets and rfm_warm_start use the same encoding. */
rfm_status rfm_warm_inputs(rfm_problem* p, const double* params, const double* param_lo, const double* param_hi,
                           int32_t nparam, float* X);

/* Initial coefficients from a network with in_dim = nparam + dim: its inputs
 * at PDE point x are those of rfm_warm_inputs (encoded params, x), its outputs
 * the ncomp field values; they are projected by rfm_project.  u_out [n] gets
 * the projected coefficients if the solver's merit ||D0 F(u)|| is smaller there
 * than at the zero vector, else zeros (D0: the row scale of the Jacobian at
 * u = 0, the same for both).  info (or NULL) gets {||D0 F(projected)||,
 * ||D0 F(0)||, 1 if the projection was kept}.  Leaves the Jacobian at u = 0 as
 * the problem's current one. */
rfm_status rfm_warm_start(rfm_problem* p, rfm_mlp* net, const rfm_solve_opts* opts, const double* params,
                          const double* param_lo, const double* param_hi, int32_t nparam, double* u_out,
                          double* info);

/* ------------------------------------------------------------------------
 * Kernel timing.  While enabled, the main kernels are bracketed by HIP events
 * on the problem's stream; each record accumulates launches, seconds, and the
 * algorithmic floating-point operations and HBM bytes of those launches
 * (flops: 2 s nnz(J) for every sketch, whatever the matrix cores issue for it,
 * 2 M N K for the QR products; bytes: the stored Jacobian plus the vectors for
 * J x and J^T y, the packed triangle of R for a triangular solve).
 * ---------------------------------------------------------------------- */
typedef struct {
  char name[32];
  int64_t launches;
  double seconds;
  double flops;
  double bytes;
} rfm_kernel_stat;

/* on != 0 starts recording (clearing previous records); on == 0 stops. */
rfm_status rfm_profile_enable(rfm_problem* p, int32_t on);

/* Copies up to max records to out (synchronising the stream first) and returns
 * the number of records, or a negative status. */
int32_t rfm_profile_read(rfm_problem* p, rfm_kernel_stat* out, int32_t max);

#ifdef __cplusplus
}
#endif

#endif /* RFM_H */
