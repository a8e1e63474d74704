// Internal declarations shared by the host plan code and the HIP kernels of the
// block-tridiagonal solver.  Not part of the public C ABI (include/tridiag.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace td {

// ---------------------------------------------------------------------------
// Block GEMM: every product in this library has the shape
//   C (Mp x ncols) = alpha * (A (Mp x kd) * B (kd x ncols) [+ sum of partials]) [+ Cin]
// with A and B column-major.  One launch runs a list of such problems (all with the
// same buffers and leading dimensions, different offsets); one work-group computes
// the full Mp rows of one 4*CT-column tile of one problem.  B may consist of
// several segments of `segrows` inner rows each, at a stride of `bseg` elements,
// so that non-adjacent blocks can form one inner dimension.
// ---------------------------------------------------------------------------
struct BDesc {
  int64_t a_off;    // A = args.A + a_off (lda = args.lda)
  int64_t b_off;    // B segment q = args.B + b_off + q * bseg (ldb = args.ldb)
  int64_t bseg;
  int64_t bs_off;   // per-inner-row scale of B: args.bscale + bs_off (if args.bscale)
  int64_t c_off;    // C = args.C + c_off (if args.C)
  int64_t cin_off;  // addend = args.Cin + cin_off (if args.Cin)
  int64_t sp_off;   // partial sums: args.Sp + sp_off + q * args.spstride, q < nsp
  int64_t x2_off;   // second output (first x2rows rows only): args.X2 + x2_off
  int32_t kd;       // inner dimension (multiple of 16)
  int32_t segrows;  // inner rows per B segment (multiple of 16, divides kd)
  int32_t nsp;      // number of partial sums to add
  int32_t pad_;
};

struct BArgs {
  const BDesc* descs;
  int32_t nprob;
  int32_t ncols;      // columns of B and C
  int32_t Mp;         // rows of A and C
  int32_t ncoltiles;
  int32_t total;      // nprob * ncoltiles
  int32_t x2rows;
  int32_t x2accum;    // nonzero: X2 += result instead of X2 = result
  int32_t brows;      // > 0: rows of each B segment at or beyond brows read as zero
  int32_t kalign;     // every descriptor's kd and segrows are multiples of kalign (0 = 16)
  double alpha;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  const double* bscale;
  double* C; int64_t ldc;
  const double* Cin; int64_t ldcin;
  const double* Sp; int64_t ldsp; int64_t spstride;
  double* X2; int64_t ldx2;
};

// Subdomain forward + backward sweeps (eq. sub3, float64).
struct SweepArgs {
  const int64_t* ks;     // p + 1 interface rows (0-based; ks[p] = N)
  const double* Dinv;    // [N][Mp][Mp]: D_i^{-1} of interior row i
  const double* alpha;   // [N][Mp][Mp]: alpha_i = D_i^{-1} B_i
  const double* adiag;   // [N][Mp]: diagonal of A_i (zero padded)
  // dense A: E_i = D_i^{-1} A_i ([N][Mp][Mp]); the forward sweep is then the recurrence
  // beta_i = E_i beta_{i-1} + G_i with G_i = D_i^{-1} F_i already in W (adiag unused)
  const double* E;
  const double* F; int64_t ldf;
  double* W; int64_t ldw;
  int32_t N, M, Mp, p, K, ncoltiles, total;
  int32_t kt_hint, rt_hint;   // columns per work-group, row tiles per wave (0 = the launcher's rule)
};

// Superposition, eq. (superposition): X_i = W_i + U_i X_{k_s} + V_i X_{k_{s+1}} for the interior rows.
struct SupArgs {
  const int64_t* ks;     // p + 1 interface rows
  const double* UV;      // U_i = UV + 2*i*Mp*Mp (Mp x 2Mp col-major, V_i in the second half)
  const double* Xi;      // interface values, ((p+2)*Mp) x K: block s+1 holds X_{k_s}, blocks 0 and p+1 are 0
  int64_t ldxi;
  const double* W; int64_t ldw;
  double* X; int64_t ldx;
  int32_t N, M, Mp, p, K, ncoltiles, total, accumulate;  // accumulate: X += result
  int32_t kt_hint, rt_hint;   // columns per work-group, row tiles per wave (0 = the launcher's rule)
};

// Float32 workspace of the low-precision solve (beta, then W): panels of W32_PANEL right-hand
// sides; within a panel, block row i holds the panel's columns of Mp rows back to back
// (column-major), so one step of a column tile touches one contiguous range instead of
// columns N Mp apart (fewer address translations: at block size 256 the bfloat16 sweep and
// superposition take 7-9% less time than with a leading dimension of N Mp).
constexpr int W32_PANEL = 64;
__host__ __device__ inline int64_t w32_off(int64_t N, int Mp, int64_t i, int row, int64_t col) {
  return ((col / W32_PANEL) * N + i) * (int64_t)W32_PANEL * Mp + (col % W32_PANEL) * Mp + row;
}
inline int64_t w32_floats(int64_t N, int64_t Mp, int64_t K) {
  return N * Mp * ((K + W32_PANEL - 1) / W32_PANEL) * W32_PANEL;
}

// Low-precision sweeps (PREC 1 = float32, 2 = bfloat16): matrices row-major in that type,
// beta / W in float32 (the workspace, panel layout of w32_off), right-hand side in float64.
struct LpSweepArgs {
  const int64_t* ks;
  const void* Dinv;      // [N][Mp][Mp] row-major
  const void* alpha;     // [N][Mp][Mp] row-major
  const double* adiag;
  const double* F; int64_t ldf;
  float* W;              // panel layout (w32_off)
  int32_t N, M, Mp, p, K, ncoltiles, total;
  int32_t kt_hint, rt_hint;   // columns per work-group, row tiles per wave (0 = the launcher's rule)
};

struct LpSupArgs {
  const int64_t* ks;
  const void* UV;        // U_0 base, [U_i V_i] row-major Mp x 2Mp at UV + i * 2 Mp^2
  const double* Xi; int64_t ldxi;
  const float* W;        // panel layout (w32_off)
  double* X; int64_t ldx;
  int32_t N, M, Mp, p, K, ncoltiles, total, accumulate;
  int32_t kt_hint, rt_hint;   // columns per work-group, row tiles per wave (0 = the launcher's rule)
};

// Batched Gauss-Jordan inversion with partial pivoting.
struct GJArgs {
  double* work;          // matrix q (Mp x Mp col-major, destroyed) at work + work_off[q],
  const int64_t* work_off;  // or at work + q * wstride when work_off is null
  int64_t wstride;
  double* out;           // inverse of matrix q at out + out_off[q]
  const int64_t* out_off;
  double* alpha;         // optional: alpha = inverse * diag(bdiag + bd_off[q]) at alpha + out_off[q]
  const double* bdiag;
  const int64_t* bd_off;
  const int32_t* tag;    // block label reported on a singular pivot
  int32_t* bad;          // atomic min of the labels of singular matrices
  // scratch of the one-launch-per-panel path (block sizes that are multiples of 64 from 128):
  int32_t* piv;          // nmat x Mp pivot rows
  double* pmin;          // nmat smallest pivot magnitudes so far (NaN once a pivot is NaN)
  double* part;          // nmat x (Mp / 32) x Mp partial row sums of the matrices' magnitudes
  int32_t nmat, Mp;
};

// Algorithm 1 on a scalar tridiagonal system (kernels_scalar.hip): subtrees of at most SC_SUB rows,
// SC_CPW right-hand sides per work-group.
constexpr int SC_SUB = 1024;
constexpr int SC_CPW = 4;
struct ScalarArgs {
  int N, K, L0, ndeep, nsub, ntop, maxsub, accumulate;
  int64_t ldf, ldx;
  const double* G;         // [depth][N]: row m of the inverse of each node's submatrix, by level
  const double* hl;        // [N] (by split row m): g_m[l] a_l
  const double* hr;        // [N]: g_m[r] b_r
  const int* lo;           // [N]: node range of split row m
  const int* hi;
  const double* F;
  double* X;
  double* Pt;              // [L0][nsub][K]: subtree parts of the top nodes' sums
  double* Xt;              // [ntop][K]: x at the top rows (top list order)
  // subtrees (nodes of level L0, by row)
  const int* sub_lo;
  const int* sub_hi;
  const int* sub_left;     // top-list position of row sub_lo - 1, or -1
  const int* sub_right;    // top-list position of row sub_hi + 1, or -1
  const int4* sub_rec;     // the subtrees' nodes, each subtree's in level order: {m, l, r, 0}
  const double2* sub_h;    // their {hl, hr}, same order
  const int* sub_off;      // [nsub]: start of subtree s in sub_rec
  const int* sub_lvoff;    // [nsub][ndeep + 1]: level starts within the subtree's records
  // top nodes (levels < L0), in level order
  const int* top_m;
  const int* top_lvl;
  const int* top_s0;       // subtrees inside the node: [top_s0, top_s1)
  const int* top_s1;
  const int* top_t0;       // top rows inside the node: toprow_sorted[top_t0 .. top_t1)
  const int* top_t1;
  const int* top_left;     // top-list position of row l - 1, or -1
  const int* top_right;    // top-list position of row r + 1, or -1
  const int* toprow_sorted;
};
hipError_t launch_scalar_gather_h(double* sub_h, const int4* rec, int nrec, const double* hl, const double* hr,
                                  hipStream_t st);
hipError_t launch_scalar_factor(const double* a, const double* b, const double* cdiag, int cs, int N, const int* lo,
                                const int* hi, const int* lvl, double* G, double* hl, double* hr, int32_t* bad,
                                hipStream_t st);
// the top levels (subtree parts of the top nodes' sums, then the top nodes) and the subtrees
hipError_t launch_scalar_top(const ScalarArgs& A, hipStream_t st);
hipError_t launch_scalar_sub(const ScalarArgs& A, hipStream_t st);

// Launch wrappers (kernels_f64.hip)
hipError_t launch_bgemm(const BArgs& a, hipStream_t st);

// Levels of Algorithm 1 with few nodes split the inner dimension [X_{l-1}; X_{r+1}] of
// X_m = S_m + H^L X_{l-1} + H^R X_{r+1} into slabs, each a separate block-GEMM problem writing
// a partial product; the combine step adds the slab partials and the partial sums of S_m,
// then writes X_m to the interface array and to the solution.
struct CombDesc {
  int64_t p_off;    // slab q of this node: P + p_off + q * Mp (ld = ldp)
  int64_t sp_off;   // partial sums of S_m: Sp + sp_off + q * spstride (ld = ldsp), q < nsp
  int64_t c_off;    // X_m in the interface array: C + c_off (ld = ldc)
  int64_t x2_off;   // X_m in the solution: X2 + x2_off (first x2rows rows; ld = ldx2)
  int32_t nslab, nsp;
};
struct CombArgs {
  const CombDesc* descs;
  int32_t nnode, Mp, ncols, x2rows, x2accum, pad_;
  const double* P; int64_t ldp;
  const double* Sp; int64_t ldsp; int64_t spstride;
  double* C; int64_t ldc;
  double* X2; int64_t ldx2;
};
hipError_t launch_level_combine(const CombArgs& a, hipStream_t st);
hipError_t launch_sweep(const SweepArgs& a, hipStream_t st);
hipError_t launch_superpose(const SupArgs& a, hipStream_t st);
hipError_t launch_gj(const GJArgs& a, hipStream_t st);
// compact inputs of P^T from those of P (formats: A' has B's, B' has A's, C' has C's)
hipError_t launch_transpose_inputs(double* At, double* Bt, double* Ct, const double* A, int fmtA, const double* B,
                                   int fmtB, const double* C, int fmtC, int N, int M, hipStream_t st);
// Dinv_t[row] = Dinv[row]^T, alpha_t[row] = Dinv_t[row] diag(bdiag_t[row])
hipError_t launch_transpose_scale(double* Dinv_t, double* alpha_t, const double* Dinv, const double* bdiag_t,
                                  const int64_t* rows, int nrows, int Mp, hipStream_t st);
// dst[b] = src[b]^T for nblk consecutive Mp x Mp blocks
hipError_t launch_transpose_blocks(double* dst, const double* src, int64_t nblk, int Mp, hipStream_t st);
int bgemm_coltile(int ncols);    // columns per work-group chosen for ncols
int sweep_coltile(int Mp, int K);

// Factor helpers
hipError_t launch_build_D(double* Dwork, int64_t wstride, int nmat, const int64_t* rows, const int32_t* first,
                          const void* C, int fmtC, const double* adiag, const double* alpha, int M, int Mp,
                          hipStream_t st);
hipError_t launch_expand_C(double* out, const void* C, int fmtC, int64_t row, int M, int Mp, hipStream_t st);
hipError_t launch_reduced(double* At, double* Ct, double* Bt, const int64_t* ks, const double* UV,
                          const void* C, int fmtC, const double* adiag, const double* bdiag, int p, int N,
                          int M, int Mp, hipStream_t st);
hipError_t launch_pad_diag(double* dst, const double* src, int N, int M, int Mp, int zero_first,
                           int zero_last, hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_band_to_blocks(int64_t n, int kl, int ku, const double* ab, int64_t ldab, int M, int64_t N,
                                 double* A, double* B, double* C, hipStream_t st);
// [A_j | B_j] as one zero-padded Mp x 2Mp column-major matrix per block row (DIAG blocks on the
// diagonal); A_0 and B_{N-1} are stored as zero
hipError_t launch_expand_AB(double* ABd, const double* A, int fmtA, const double* B, int fmtB, int N, int M, int Mp,
                            hipStream_t st);
hipError_t launch_identity(double* p, int Mp, hipStream_t st);
hipError_t launch_negate_fill_check(int32_t* flag, int32_t v, hipStream_t st);

// Solve helpers
hipError_t launch_ftilde(double* Ft, int64_t ldft, const double* F, int64_t ldf, const double* W, int64_t ldw,
                         const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp,
                         int K, hipStream_t st);
hipError_t launch_residual(double* R, int64_t ldr, const double* F, int64_t ldf, const double* X,
                           int64_t ldx, const void* A, int fmtA, const void* B, int fmtB, const void* C,
                           int fmtC, int N, int M, int K, double* colpart, int nblk, hipStream_t st);
hipError_t launch_colnorm_finish(double* out, const double* colpart, int nblk, int K, hipStream_t st);
hipError_t launch_scale_cols(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* s,
                             int invert, int64_t n, int K, hipStream_t st);
hipError_t launch_axpy_cols(double* X, int64_t ldx, const double* D, int64_t ldd, const double* s,
                            int64_t n, int K, hipStream_t st);
hipError_t launch_diag_grad(double* out, const double* Lam, int64_t ldl, const double* X, int64_t ldx,
                            int64_t n, int K, hipStream_t st);
hipError_t launch_nonfinite(int32_t* flag, const double* X, int64_t ldx, int64_t n, int K, hipStream_t st);
hipError_t launch_probe_inputs(double* A, double* B, double* C, double* F, int N, int M, int64_t K, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched solve of many independent systems in one persistent launch
// (kernels_batched.hip).  Work items are dequeued in a topological order from one
// global counter; an item waits (bounded spin) until the counter of the stage it
// depends on reaches the expected value, runs, and then increments its own counter.
// ---------------------------------------------------------------------------
constexpr int BATCH_MAXDEPTH = 16;
enum { BI_SWEEP = 0, BI_FTILDE = 1, BI_PART = 2, BI_LEVEL = 3, BI_SUP = 4, BI_RES = 5, BI_RFIN = 6 };

struct BatchItem {
  int32_t type, sys, pass, lvl;
  int32_t i0, i1;          // sweep/sup: subdomain, column tile; part/level: problem, column tile;
                           // ftilde: element chunk; res: row chunk, first column
  int32_t dep;             // counter index this item waits for (-1: none)
  int32_t need;            // value that counter must reach
  int32_t mine;            // counter index this item increments
  int32_t pad_;
};

struct BatchSys {
  LpSweepArgs sweep;       // float32 plans: input F; the correction passes read R instead
  LpSupArgs sup;
  SweepArgs sweep64;       // float64 plans
  SupArgs sup64;
  BArgs part;
  BArgs lev[BATCH_MAXDEPTH];
  double* Ft; int64_t ldft;
  const double* adiag; const double* bdiag;
  const double* F; int64_t ldf;
  double* X; int64_t ldx;
  double* R; int64_t ldr;
  const double* cA; const double* cB; const double* cC;
  double* colpart;         // [K][nchunk][2]
  double* resid;           // [passes]: max column relative residual after each pass
  int32_t N, M, Mp, p, K, rt, nchunk, rescols;
  int32_t prec;            // TD_PREC_F64 (0) or TD_PREC_F32 (1)
  int32_t pad_;
  double tol;
};

struct BatchCtl {
  int32_t head;            // next item to dequeue
  int32_t error;           // nonzero: a dependency wait timed out
  int32_t pad_[2];
};

hipError_t launch_batched(const BatchItem* items, int nitems, const BatchSys* sys, int32_t* counters, int ncounters,
                          int32_t* conv, int nsys, BatchCtl* ctl, int grid, int64_t spin_limit, hipStream_t st);
hipError_t launch_batched_stages(const BatchItem* items, const int* stage_begin, int nstages, const BatchSys* sys,
                                 int32_t* heads, int32_t* conv, int nsys, BatchCtl* ctl, int max_grid, hipStream_t st);
int batched_lds_bytes();
int batched_blocks_per_cu();

// Low-precision path (kernels_lp.hip)
hipError_t launch_cast_rowmajor(int prec, void* dst, int64_t dstride, const double* src, int64_t sstride,
                                const int64_t* list, int nmat, int rows, int cols, hipStream_t st);
hipError_t launch_sweep_lp(int prec, const LpSweepArgs& a, hipStream_t st);
hipError_t launch_superpose_lp(int prec, const LpSupArgs& a, hipStream_t st);
hipError_t launch_ftilde_f32(double* Ft, int64_t ldft, const double* F, int64_t ldf, const float* W, int64_t N,
                             const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K,
                             hipStream_t st);
// rows x right-hand sides of one work-group (or batched work item) of the stencil residual
constexpr int RES_ROWS = 1024;
constexpr int RES_COLS = 16;
constexpr int RES_ROWS_WIDE = 2048;
int residual_row_chunks(int64_t n);        // row chunks of the batched kernels' residual items
int residual_row_chunks_wide(int64_t n);   // row chunks of launch_residual_stencil
hipError_t launch_zero_absent(double* A, double* B, double* C, int N, int M, hipStream_t st);
hipError_t launch_residual_stencil(double* R, int64_t ldr, const double* F, int64_t ldf, const double* X, int64_t ldx,
                                   const double* A, const double* B, const double* C, int N, int M, int K,
                                   double* colpart, hipStream_t st);

}  // namespace td
