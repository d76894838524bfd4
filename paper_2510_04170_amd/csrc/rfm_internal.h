// Internal declarations of librfmnewton: device layouts, the problem object and
// the host-side launchers of every kernel.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rfm.h"

namespace rfm {

// ---------------------------------------------------------------------------
// errors: internal code throws rfm::Error, the C-ABI layer turns it into a status
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  rfm_status code;
  Error(rfm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define RFM_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      throw ::rfm::Error(e_ == hipErrorOutOfMemory ? RFM_ENOMEM : RFM_EDEVICE,                 \
                         std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

#define RFM_CHECK(cond, code, msg)                 \
  do {                                                \
    if (!(cond)) throw ::rfm::Error((code), (msg));   \
  } while (0)

// error text of the last failed call on this thread (rfm_last_error)
void set_last_error(const std::string& m);

// runs f, mapping exceptions to status codes for the C ABI
template <class F>
rfm_status guarded(F&& f) {
  try {
    f();
    return RFM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return (rfm_status)e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return RFM_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return RFM_EDEVICE;
  }
}

// ---------------------------------------------------------------------------
// device buffer (owned by the problem object)
// ---------------------------------------------------------------------------
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void resize(size_t count) {  // contents are not kept
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    RFM_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
};

// ---------------------------------------------------------------------------
// limits and layouts shared by host and device
// ---------------------------------------------------------------------------
constexpr int kMaxDim = 4;
constexpr int kMaxComp = 4;
constexpr int kMaxLin = 16;
constexpr int kMaxPoly = 8;
constexpr int kMaxFn = 8;
constexpr int kMaxProd = 8;  // product terms
constexpr int kMaxFac = 4;   // factors per product term
constexpr int kMaxQ = 8;     // distinct field quantities (component, derivative) of the product terms
constexpr int kMaxRowWidth = 16384;  // widest Jacobian row
constexpr int kTileRows = 64;       // rows per Jacobian tile
constexpr int kMaxPieces = 16;      // pieces of D J in a low-precision sketch

struct OpDesc {
  int nlin;
  int lin_eq[kMaxLin], lin_comp[kMaxLin], lin_deriv[kMaxLin];
  double lin_coeff[kMaxLin];
  int npoly;
  int poly_eq[kMaxPoly];
  int poly_pow[kMaxPoly][kMaxComp];
  double poly_coeff[kMaxPoly];
  int nfn;
  int fn_eq[kMaxFn], fn_comp[kMaxFn], fn_kind[kMaxFn];  // kind: RFM_FN_*
  double fn_coeff[kMaxFn];
  // product terms coeff prod_k v_{q_k}^{p_k} over the field quantities v_q = D_{q_deriv} u_{q_comp}
  int nq;
  int q_comp[kMaxQ], q_deriv[kMaxQ];
  int nprod;
  int prod_eq[kMaxProd], prod_nfac[kMaxProd];
  int prod_q[kMaxProd][kMaxFac], prod_pow[kMaxProd][kMaxFac];
  double prod_coeff[kMaxProd];
};

// f(v) and f'(v) of a pointwise term
__host__ __device__ inline void fn_eval(int kind, double v, double* f, double* df) {
  if (kind == RFM_FN_EXP) {
    const double e = exp(v);
    *f = e;
    *df = e;
  } else {
    const double c = cosh(v), s = sinh(v);
    *f = kind == RFM_FN_COSH ? c : s;
    *df = kind == RFM_FN_COSH ? s : c;
  }
}

struct GeomDesc {
  int dim, ncomp, J, nbox;
  int nsub[kMaxDim];
  double lo[kMaxDim], hi[kMaxDim];
  int pou;  // RFM_POU_INDICATOR or RFM_POU_SMOOTH
};

// one Jacobian row: which point, which box(es), which equation/component, which order
struct RowDesc {
  int32_t pt;
  int32_t owner;
  int32_t neighbor;
  uint8_t kind, sel, order, pad;
};

// consecutive rows with one column support: segment A (and B for continuity rows);
// values are stored row-major, nrows x (wA + wB), starting at val_off
constexpr int kMaxSeg = 8;  // column segments of a tile row (boxes touched by a smooth-partition row)

struct TileDesc {
  int32_t row0, nrows;
  int32_t colA, wA;  // indicator partition: one or two segments; smooth partition: wA = row width
  int32_t colB, wB;
  int64_t val_off;
  int64_t part_off;  // start of this tile's slot in the J^T y partial buffer
  int32_t nseg, wseg;         // segments of equal width: row value p is column seg_col[p / wseg] + p % wseg
  int32_t seg_col[kMaxSeg];
};

// feature table, structure of arrays indexed by (e * ncomp + c) * J + j
struct FeatDev {
  const double* W[kMaxDim];   // raw weights
  const double* WS[kMaxDim];  // weight / box half-width
  const double* b;
  const double* S2;           // sum_a WS_a^2
  const double* S2s;          // same over the space axes only
};

// device scalars of one LSQR run (Paige-Saunders recurrences kept on the GPU)
struct LsqrState {
  double alpha, beta;         // current normalisation of v and u
  double rhobar, phibar;
  double rho, phi, theta;     // step coefficients of the latest iteration
  double bnorm, anorm2, xnorm2;
  double rnorm, arnorm;
  double tol;
  int32_t itn, maxit;
  int32_t istop;              // 0 running / iteration limit, 1 rule 1, 2 rule 2, 3 b = 0
  int32_t done;               // 1 once a stop rule fired
  double inv_alpha, inv_beta; // 1/alpha and 1/beta (0 when the norm is 0)
  double cx, cw;              // x += cx w;  w = v - cw w
};

// ---------------------------------------------------------------------------
// the problem object
// ---------------------------------------------------------------------------
struct GroupH {
  int kind, owner, neighbor, comp, cont_order;
  int64_t pt0, npts;   // into the point arrays
  int64_t row0, nrows;
};

// event-timed kernel records (rfm_profile_*)
struct KStat {
  int64_t launches = 0;
  double seconds = 0, flops = 0, bytes = 0;
};
struct PendingEv {
  hipEvent_t a, b;
  int slot;
  double flops, bytes;
};
struct Profiler {
  bool on = false;
  std::vector<std::string> names;
  std::vector<KStat> stats;
  std::vector<PendingEv> pending;
  std::vector<hipEvent_t> pool;
  int slot_of(const char* name);
  void begin(hipStream_t s, hipEvent_t* a);
  void end(hipStream_t s, hipEvent_t a, const char* name, double flops, double bytes);
  void resolve();
  ~Profiler();
};

// RAII bracket around one kernel launch (no-op when profiling is off)
struct ProfScope {
  Profiler& pr;
  hipStream_t s;
  const char* name;
  double flops, bytes;
  hipEvent_t a = nullptr;
  ProfScope(Profiler& p, hipStream_t st, const char* n, double f, double b) : pr(p), s(st), name(n), flops(f), bytes(b) {
    if (pr.on) pr.begin(s, &a);
  }
  ~ProfScope() {
    if (pr.on && a) pr.end(s, a, name, flops, bytes);
  }
};

struct Problem {
  int dim = 0, ncomp = 0, device = 0;
  hipStream_t stream = nullptr;
  bool have_partition = false, have_features = false, have_operator = false, finalized = false;
  GeomDesc geom{};
  OpDesc op{};
  DBuf<OpDesc> d_op;      // device copy of op read by the row kernels
  OpDesc op_on_device{};  // what d_op holds
  bool have_d_op = false;
  std::vector<double> W, b;           // host copies as given
  std::vector<double> px, pnormal;    // points [npts][dim], normals [npts][dim]
  std::vector<double> rowdata;        // data per row (0 for continuity rows)
  std::vector<GroupH> groups;
  int64_t npts = 0, m = 0, n = 0;
  int J = 0;

  // layout
  std::vector<TileDesc> tiles_h;
  int64_t nvals = 0, npart = 0;
  int ntiles = 0, max_tile_w = 0;  // tile count, widest tile row
  std::vector<int32_t> cb_ptr_h, cb_tile_h, cb_off_h;  // column block -> contributing tiles
  std::vector<int64_t> sk_ptr_h, sk_off_h;  // column block -> its rows: d_J offset of each row's segment
  std::vector<int32_t> sk_row_h;            // ... and the row index
  // low-precision sketch operand: per column block, the 32-row groups of rows touching it
  std::vector<int32_t> cbs_ptr_h, slot_group_h;
  std::vector<int64_t> slot_rowoff_h;     // [slot][32]: offset of the row's segment in d_J, or -1
  int64_t nslots = 0;

  // device: geometry, features, rows, tiles
  DBuf<double> d_px, d_pnormal, d_rowdata;
  DBuf<double> d_feat;  // packed SoA feature table
  FeatDev feat{};
  DBuf<RowDesc> d_rows;
  DBuf<TileDesc> d_tiles;
  DBuf<int32_t> d_cb_ptr, d_cb_tile, d_cb_off;
  DBuf<int64_t> d_sk_ptr, d_sk_off;
  DBuf<int32_t> d_sk_row;
  DBuf<int32_t> d_rowtile;  // tile index of each row

  // device: current Jacobian (scaled), residual, scale
  DBuf<double> d_J, d_DF, d_D, d_part;
  bool have_J = false;
  DBuf<float> d_J32;                      // D J rounded to FP32 for the LSQR products
  bool have_J32 = false;
  DBuf<int32_t> d_cbs_ptr, d_slot_group;  // slots of each column block; global group of each slot (-1: padding)
  DBuf<int64_t> d_slot_rowoff;            // [slot][32]: offset of the row's segment in d_J, or -1
  DBuf<uint16_t> d_pan16, d_tab16;        // BF16 pieces [piece][slot][J][32]; code table
  DBuf<uint8_t> d_pan8, d_tab8;          // FP8 pieces [piece][slot][J][32]; code table
  DBuf<int64_t> d_cs_eoff;                // count sketch: d_J offsets of the grouped rows
  DBuf<double> d_cs_sign;                 //               their signs
  DBuf<char> d_cs_runs;                   //               runs of equal bucket
  std::vector<int32_t> cs_run_bucket;     //               bucket of each run (ascending)
  DBuf<int32_t> d_pexp;                   // exponent E of each (chunk of 4 slots, column)
  int pan_prec = -1, pan_pieces = 0;
  bool have_tables = false;

  // projection onto the feature basis at the PDE points (identity operator), R kept between calls
  rfm_problem* proj = nullptr;
  double proj_gamma = 0.0, proj_c = 0.0;
  uint64_t proj_seed = 0;
  double cur_c = 100.0;

  // device: sketch and preconditioner
  int64_t s = 0;
  DBuf<double> d_B;       // s x n column-major (becomes Q's reflectors and R)
  DBuf<double> d_tau;     // Householder scalars
  DBuf<double> d_R;       // R in tiled upper storage for the triangular solves
  DBuf<double> d_trsv;    // triangular solves: published blocks of x, then the helpers' partial sums
  DBuf<double> d_trsv_tiles;  // triangular solves: the tiles next to the diagonal in the solver's layout (from R)
  DBuf<double> d_ws;      // QR workspace
  DBuf<int32_t> d_sync;   // grid-barrier / ticket / flag words
  int64_t ws_elems = 0;
  bool have_B = false, have_R = false;
  int verbose = 0;  // progress lines on stderr from long stages (set by rfm_solve from its options)
  uint32_t barrier_epoch = 0;

  // device: work vectors
  DBuf<double> d_u, d_du, d_vec;  // coefficient vectors and scratch
  DBuf<double> d_red;             // reduction partials
  DBuf<double> d_scal;            // reduction results
  DBuf<double> d_lsab;            // line search: a_r, b_r, vu[K], vd[K], qu[nq], qd[nq] per row
  DBuf<LsqrState> d_lsqr;
  DBuf<double> d_ws_lsqr;         // LSQR vectors and partials
  DBuf<double> d_F0, d_F1;        // residual vectors of the drivers
  Profiler prof;

  ~Problem();
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ---------------------------------------------------------------------------

// k_rows.hip
void launch_assemble(Problem& P, const double* u, double c);
void launch_row_eval(Problem& P, const double* u, const double* du, double* out_ab);
void launch_phi(Problem& P, const double* ab, double alpha, const double* D, double* out_sumsq);
// field values out [npts][ncomp], or with grad its gradient out [npts][ncomp][dim]
void launch_eval_points(Problem& P, const double* u, int64_t npts, const double* x, const int32_t* owner,
                        double* out, bool grad = false);
void launch_jmul(Problem& P, const double* J, const double* x, double* y, const double* u_prev,
                 const LsqrState* st, double* red_partials);
void launch_jtmul(Problem& P, const double* J, const double* y, double* x, const LsqrState* st);
// the same products on the FP32 copy of D J (FP64 vectors and accumulation)
void launch_jmul(Problem& P, const float* J, const double* x, double* y, const double* u_prev, const LsqrState* st,
                 double* red_partials);
void launch_jtmul(Problem& P, const float* J, const double* y, double* x, const LsqrState* st);
void launch_jacobian_rows(Problem& P, int64_t r0, int64_t nrows, double* out);
// rfm_jtmul_noalloc: the fixed device scratch (looked up once per device, with the device current), its
// size in doubles, and J^T y with the tile partials in `part`
double* noalloc_scratch(int device);
size_t noalloc_scratch_doubles();
void launch_jtmul_noalloc(Problem& P, const double* y, double* x, double* part);
void launch_reduce_sum(Problem& P, const double* partials, int nparts, double* out);
void launch_residual_from_ab(Problem& P, const double* ab, double* F, double* out_sumsq);
int reduce_blocks_rows(const Problem& P);

// k_sketch.hip
void launch_sketch(Problem& P, uint64_t seed, uint64_t jac_index, int prec);
// sketch rows r0 .. r0 + nr - 1 (r0 a multiple of 128): row r0 + i of column c to out[c ldo + i]
void launch_sketch_rows(Problem& P, uint64_t seed, uint64_t jac_index, int64_t r0, int64_t nr, double* out,
                        int64_t ldo);

// network shape check (mlp.hip): throws RFM_EINVAL unless in_dim / out_dim match
void mlp_check_shape(rfm_mlp* net, int in_dim, int out_dim);

// count sketch (k_count.hip)
void count_sketch_hash(int64_t r, int64_t s, uint64_t seed, uint64_t jac, int64_t* h, double* sigma);
void launch_count_sketch(Problem& P, uint64_t seed, uint64_t jac_index);  // all of B into d_B
// hash the rows and upload the runs for (seed, jac_index); then rows r0 .. r0 + nr - 1 of B, cleared and
// summed, to out[c ldo + i] (as launch_sketch_rows)
void prepare_count_sketch(Problem& P, uint64_t seed, uint64_t jac_index);
void launch_count_sketch_rows(Problem& P, int64_t r0, int64_t nr, double* out, int64_t ldo);
// the count sketch streamed into qr_factor_streamed; returns the sketch seconds (hashing included)
double streamed_count_sketch_qr(Problem& P, uint64_t seed, uint64_t jac_index, int64_t rows_per_pass);

// low-precision forms (k_lowp.hip)
void sketch_table(int prec, double* out);
void launch_cast_panels(Problem& P, int prec, int pieces);
void launch_cast_f32(Problem& P);
void launch_sketch_lowp(Problem& P, uint64_t seed, uint64_t jac_index, int prec, int pieces);
// rows r0 .. r0 + nr - 1 (r0 a multiple of 128) after launch_cast_panels, as launch_sketch_rows
void launch_sketch_lowp_rows(Problem& P, uint64_t seed, uint64_t jac_index, int prec, int64_t r0, int64_t nr,
                             double* out, int64_t ldo);
void get_sketch_operand(Problem& P, int piece, int blk, int64_t slot0, int64_t nslots, double* out, int32_t* groups,
                        int32_t* scale_exp);

// device copy of P.op, uploaded when it changed (waits for the stream first)
const OpDesc* device_op(Problem& P);

// k_qr.hip
void qr_factor(Problem& P);   // in place on d_B, leaves R in d_R (tiled), throws RFM_ESINGULAR
// Streamed form for sketches too large to hold: the s sketch rows are produced rows_per_pass at a time
// by sketch_rows(r0, nr, out, ldo) (sketch row r0 + i of column c to out[c ldo + i]) and folded into
// R; leaves R in d_R as qr_factor does and returns the seconds spent in sketch_rows.
double qr_factor_streamed(Problem& P, const std::function<void(int64_t, int64_t, double*, int64_t)>& sketch_rows,
                          int64_t rows_per_pass);
bool qr_should_stream(const Problem& P);                   // B, R and workspace above 60% of the device memory
int64_t qr_stream_rows(const Problem& P, int64_t want);  // rows per pass: want (> 0) or about 1/8 of the memory
// Gaussian sketch (FP64, BF16 or FP8) of the current D J streamed into qr_factor_streamed; returns the
// sketch seconds (operand casts included)
double streamed_sketch_qr(Problem& P, uint64_t seed, uint64_t jac_index, int prec, int pieces, int64_t rows_per_pass);
void launch_get_r_cols(Problem& P, int64_t c0, int64_t ncols, double* out);

// k_trsv.hip
// yscale_sel: 0 -> 1, 1 -> 1/alpha (LSQR state); sub_sel: 0 -> none, 1 -> out = x - (beta/alpha) sub
void launch_trsv(Problem& P, const double* y, double* x, bool transpose, const double* sub_vec,
                 const LsqrState* st, int yscale_sel, int sub_sel, double* red_partials);
int trsv_block();
void check_trsv_error(Problem& P);
// the solver's copies of the tiles on and next to R's diagonal; after every change of d_R
void prepare_trsv(Problem& P);

// k_lsqr.hip
// prec: RFM_PREC_F64 multiplies by d_J, RFM_PREC_F32 by d_J32
void lsqr_run(Problem& P, const double* rhs, double tol, int maxit, double* y, int* iters, int* istop,
              int prec = RFM_PREC_F64);

// vector helpers (k_lsqr.hip)
void launch_axpy(Problem& P, int64_t n, double a, const double* x, double* y);
void launch_scale_copy(Problem& P, int64_t n, double a, const double* x, double* y);
void launch_neg_mul(Problem& P, int64_t n, const double* D, const double* F, double* out);  // out = -D*F (D may be null)
void launch_diff_norm2(Problem& P, int64_t n, const double* a, const double* b, const double* D, double* out);

// C-ABI bodies (solver.cpp)
rfm_status api_solve(Problem& P, const rfm_solve_opts* opts, double* u_inout, rfm_solve_stats* stats);
rfm_status api_residual(Problem& P, const double* u, double* F, double* norm);
rfm_status api_eval(Problem& P, const double* u, int64_t npts, const double* x, const int32_t* owner, int what,
                    double* out);
rfm_status api_linesearch(Problem& P, const double* u, const double* du, int gs_iters, double* alpha, double* phi);

// utilities
bool is_device_ptr(const void* p);
void copy_in(Problem& P, double* dst, const double* src, size_t count);
double read_scalar(Problem& P, const double* d);  // one device double, after the stream drains    // src host or device
void copy_out(Problem& P, double* dst, const double* src, size_t count);   // dst host or device

}  // namespace rfm
