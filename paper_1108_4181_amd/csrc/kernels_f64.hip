// Float64 HIP kernels of the block-tridiagonal solver for gfx950 (MI355X).
//
// Dense block products run on v_mfma_f64_4x4x4f64 (four 4x4x4 blocks per
// instruction).  Used as one 16 x 4 output tile: the A operand supplies 16 rows
// (lane L holds A[L%16][L/16]), the B operand is the same 4 x 4 block in all four
// blocks (lane L holds B[L/16][L%4]), and lane L receives D[4*((L/4)%4) + L/16][L%4].
// On gfx950 this instruction sustains the full float64 matrix rate, while the
// 16x16x4 float64 form issues at well under half of it.
#include "internal.h"
#include "tile_bodies.h"

#include <cfloat>
#include <climits>

namespace td {

// ---------------------------------------------------------------------------
// Block GEMM (see BArgs): one work-group = Mp rows x 4*CT columns of one problem.
// ---------------------------------------------------------------------------
template <int RT, int CT, int KC>
__global__ void __launch_bounds__(512) k_bgemm(BArgs args) {
  __shared__ double Bs[2 * KC * (4 * CT + 2)];
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= args.total) return;
  const int prob = lg / args.ncoltiles;
  bgemm_tile<RT, CT, KC>(args, prob, lg - prob * args.ncoltiles, Bs);
}

// ---------------------------------------------------------------------------
// Combine step of a split dichotomy level (see CombDesc): one thread per element of X_m.
// ---------------------------------------------------------------------------
__global__ void k_level_combine(CombArgs a) {
  const CombDesc d = a.descs[blockIdx.y];
  const int64_t n = (int64_t)a.Mp * a.ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % a.Mp);
    const int64_t col = e / a.Mp;
    double v = 0.0;
    for (int q = 0; q < d.nslab; ++q) v += a.P[d.p_off + (int64_t)q * a.Mp + row + col * a.ldp];
    for (int q = 0; q < d.nsp; ++q) v += a.Sp[d.sp_off + q * a.spstride + row + col * a.ldsp];
    a.C[d.c_off + row + col * a.ldc] = v;
    if (row < a.x2rows) {
      double* xp = a.X2 + d.x2_off + row + col * a.ldx2;
      *xp = a.x2accum ? *xp + v : v;
    }
  }
}

hipError_t launch_level_combine(const CombArgs& a, hipStream_t st) {
  if (a.nnode <= 0 || a.ncols <= 0) return hipSuccess;
  const int64_t n = (int64_t)a.Mp * a.ncols;
  int bx = (int)((n + 255) / 256);
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_level_combine, dim3(bx, a.nnode), dim3(256), 0, st, a);
  return hipGetLastError();
}

int bgemm_coltile(int ncols) {
  if (ncols <= 8) return 8;
  if (ncols <= 16) return 16;
  return 32;
}

template <int RT>
static hipError_t launch_bgemm_rt(const BArgs& a0, hipStream_t st) {
  BArgs a = a0;
  const int nthr = a.Mp / (16 * RT) * 64;
  if (nthr < 64 * RT) return hipErrorInvalidValue;   // the tile stages B with at least 64 RT threads
  // 16-column tiles where 32-column ones would leave fewer than two work-groups per compute unit
  // (small dichotomy levels and partial sums: the device fills at the cost of half the B reuse)
  int kt = bgemm_coltile(a.ncols);
  if (kt == 32 && (int64_t)a.nprob * ((a.ncols + 31) / 32) < 512) kt = 16;
  a.ncoltiles = (a.ncols + kt - 1) / kt;
  a.total = a.nprob * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  dim3 grid(grid_pad8(a.total)), block(nthr);
  // 64-row B chunks (a quarter of the barriers) where every descriptor's inner dimension allows,
  // for block sizes from 256 (four row tiles per wave: the staging registers stay few)
  if constexpr (RT == 4) {
    if (a.kalign > 0 && a.kalign % 64 == 0) {
      switch (kt) {
        case 8: hipLaunchKernelGGL((k_bgemm<RT, 2, 64>), grid, block, 0, st, a); break;
        case 16: hipLaunchKernelGGL((k_bgemm<RT, 4, 64>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((k_bgemm<RT, 8, 64>), grid, block, 0, st, a); break;
      }
      return hipGetLastError();
    }
  }
  switch (kt) {
    case 8: hipLaunchKernelGGL((k_bgemm<RT, 2, 16>), grid, block, 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_bgemm<RT, 4, 16>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((k_bgemm<RT, 8, 16>), grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_bgemm(const BArgs& a, hipStream_t st) {
  switch (choose_rt(a.Mp)) {
    case 4: return launch_bgemm_rt<4>(a, st);
    case 2: return launch_bgemm_rt<2>(a, st);
    default: return launch_bgemm_rt<1>(a, st);
  }
}

// ---------------------------------------------------------------------------
// Subdomain sweeps, float64.  One work-group owns (subdomain s, 4*CT columns) and
// walks its interior rows: forward beta_i = D_i^{-1} (F_i + a_i o beta_{i-1})
// with beta_{k_s} = 0, then backward W_i = alpha_i W_{i+1} + beta_i with
// W_{k_{s+1}} = 0 (eq. sub3).  The operand of each step (Mp x 4*CT) stays in
// LDS; the Mp x Mp matrix of the step streams from global memory (L2-shared by
// the column tiles of the subdomain, which run on one XCD).
// ---------------------------------------------------------------------------
template <int RT, int CT>
__global__ void __launch_bounds__(512) k_sweep_f64(SweepArgs a) {
  extern __shared__ double In[];  // [Mp][4 CT + 2]
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  sweep_f64_tile<RT, CT>(a, s, lg - s * a.ncoltiles, In);
}

int sweep_coltile(int Mp, int K) {
  (void)Mp;
  if (K <= 8) return 8;
  if (K <= 16) return 16;
  return 32;
}

// a row-tile count from a hint when the block size divides into it and the waves stay at most 8
static int hinted_rt(int rule, int hint, int Mp) {
  if ((hint == 1 || hint == 2 || hint == 4) && Mp % (16 * hint) == 0 && Mp / (16 * hint) <= 8) return hint;
  return rule;
}

template <int RT>
static hipError_t launch_sweep_rt(const SweepArgs& a0, hipStream_t st) {
  SweepArgs a = a0;
  const int kt = (a.kt_hint == 8 || a.kt_hint == 16 || a.kt_hint == 32) ? a.kt_hint : sweep_coltile(a.Mp, a.K);
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t lds = (size_t)a.Mp * (kt + 2) * sizeof(double);
  dim3 grid(grid_pad8(a.total)), block(nthr);
  hipError_t e = hipSuccess;
  switch (kt) {
    case 8:
      e = hipFuncSetAttribute((const void*)k_sweep_f64<RT, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e == hipSuccess) hipLaunchKernelGGL((k_sweep_f64<RT, 2>), grid, block, lds, st, a);
      break;
    case 16:
      e = hipFuncSetAttribute((const void*)k_sweep_f64<RT, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e == hipSuccess) hipLaunchKernelGGL((k_sweep_f64<RT, 4>), grid, block, lds, st, a);
      break;
    default:
      e = hipFuncSetAttribute((const void*)k_sweep_f64<RT, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e == hipSuccess) hipLaunchKernelGGL((k_sweep_f64<RT, 8>), grid, block, lds, st, a);
      break;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& a, hipStream_t st) {
  switch (hinted_rt(choose_rt(a.Mp), a.rt_hint, a.Mp)) {
    case 4: return launch_sweep_rt<4>(a, st);
    case 2: return launch_sweep_rt<2>(a, st);
    default: return launch_sweep_rt<1>(a, st);
  }
}

// ---------------------------------------------------------------------------
// Superposition, eq. (superposition): X_i = W_i + [U_i V_i] [X_{k_s}; X_{k_{s+1}}].
// One work-group owns (subdomain s, 4*CT columns): the 2Mp x 4*CT interface panel
// stays in LDS for all interior rows of s, and the Mp x 2Mp matrices [U_i V_i]
// stream through registers one chunk ahead of the MFMAs, across row boundaries,
// so the work-group runs its rows back to back without barriers.
// ---------------------------------------------------------------------------
template <int RT, int CT>
__global__ void __launch_bounds__(512) k_superpose_f64(SupArgs a) {
  extern __shared__ double Xs[];  // [2 Mp][4 CT + 2]
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  superpose_f64_tile<RT, CT, 4>(a, s, lg - s * a.ncoltiles, Xs);
}

template <int RT, int CT>
static hipError_t launch_superpose_cfg(const SupArgs& a0, hipStream_t st) {
  SupArgs a = a0;
  constexpr int kt = 4 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t lds = (size_t)2 * a.Mp * (kt + 2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_superpose_f64<RT, CT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_superpose_f64<RT, CT>), dim3(grid_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

// Block sizes above 256: 32-column tiles with half of the interface panel in LDS at a time
// (Mp x 34 doubles: 139 KB at Mp = 512), see superpose_f64_half_tile.
template <int RT, int CT>
__global__ void __launch_bounds__(512) k_superpose_f64_half(SupArgs a) {
  extern __shared__ double Xs[];  // [Mp][4 CT + 2]
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  superpose_f64_half_tile<RT, CT, 2>(a, s, lg - s * a.ncoltiles, Xs);
}

template <int RT, int CT>
static hipError_t launch_superpose_half_cfg(const SupArgs& a0, hipStream_t st) {
  SupArgs a = a0;
  constexpr int kt = 4 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t lds = (size_t)a.Mp * (kt + 2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_superpose_f64_half<RT, CT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_superpose_f64_half<RT, CT>), dim3(grid_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

template <int RT>
static hipError_t launch_superpose_rt(const SupArgs& a, hipStream_t st) {
  // the LDS panel is 2 Mp x (4 CT + 2) doubles and must fit in 160 KB
  const int64_t bytes8 = (int64_t)2 * a.Mp * 34 * 8;
  if (a.kt_hint == 8) return launch_superpose_cfg<RT, 2>(a, st);
  if (a.kt_hint == 16 && (int64_t)2 * a.Mp * 18 * 8 <= 160 * 1024) return launch_superpose_cfg<RT, 4>(a, st);
  if (a.K <= 8) return launch_superpose_cfg<RT, 2>(a, st);
  if (RT == 4 && !a.accumulate && a.K > 16 && a.Mp % 64 == 0 && bytes8 > 160 * 1024 &&
      (int64_t)a.Mp * 34 * 8 <= 160 * 1024)
    return launch_superpose_half_cfg<4, 8>(a, st);
  if (a.K <= 16 || bytes8 > 160 * 1024 || RT == 4) return launch_superpose_cfg<RT, 4>(a, st);
  return launch_superpose_cfg<RT, (RT == 4 ? 4 : 8)>(a, st);
}

hipError_t launch_superpose(const SupArgs& a, hipStream_t st) {
  // twice the waves of the other kernels where that keeps at most 8 waves per work-group
  int rt = choose_rt(a.Mp);
  const int nw = a.Mp / (16 * rt);
  if (rt >= 2 && 2 * nw <= 8) rt /= 2;
  rt = hinted_rt(rt, a.rt_hint, a.Mp);
  switch (rt) {
    case 4: return launch_superpose_rt<4>(a, st);
    case 2: return launch_superpose_rt<2>(a, st);
    default: return launch_superpose_rt<1>(a, st);
  }
}

// ---------------------------------------------------------------------------
// Element-wise helpers of the factor
// ---------------------------------------------------------------------------

// entry (r, c) of block `row` of C in its storage format, padded to Mp with the identity
__device__ __forceinline__ double c_entry(const void* C, int fmt, int64_t row, int r, int c, int M) {
  if (r >= M || c >= M) return (r == c) ? 1.0 : 0.0;
  if (fmt == 2) {  // TRIDIAG [N][3][M]
    const double* t = (const double*)C + row * 3 * M;
    if (c == r) return t[M + r];
    if (c == r - 1) return t[r];
    if (c == r + 1) return t[2 * M + r];
    return 0.0;
  }
  return ((const double*)C)[row * (int64_t)M * M + r + (int64_t)c * M];  // DENSE
}

// D_q = C_row - a_row o alpha_{row-1} (the second term only where first[q] == 0)
__global__ void k_build_D(double* Dwork, int64_t wstride, int nmat, const int64_t* rows, const int32_t* first,
                          const void* C, int fmtC, const double* adiag, const double* alpha, int M, int Mp) {
  const int q = blockIdx.y;
  if (q >= nmat) return;
  const int64_t MM = (int64_t)Mp * Mp;
  const int64_t row = rows[q];
  const bool f = first[q] != 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MM; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % Mp), c = (int)(e / Mp);
    double v = c_entry(C, fmtC, row, r, c, M);
    if (!f) v -= adiag[row * Mp + r] * alpha[(row - 1) * MM + e];
    Dwork[q * wstride + e] = v;
  }
}

hipError_t launch_build_D(double* Dwork, int64_t wstride, int nmat, const int64_t* rows, const int32_t* first,
                          const void* C, int fmtC, const double* adiag, const double* alpha, int M, int Mp,
                          hipStream_t st) {
  if (nmat == 0) return hipSuccess;
  const int64_t MM = (int64_t)Mp * Mp;
  int bx = (int)((MM + 255) / 256);
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_build_D, dim3(bx, nmat), dim3(256), 0, st, Dwork, wstride, nmat, rows, first, C, fmtC, adiag,
                     alpha, M, Mp);
  return hipGetLastError();
}

__global__ void k_expand_C(double* out, const void* C, int fmt, int64_t row, int M, int Mp) {
  const int64_t MM = (int64_t)Mp * Mp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MM; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = c_entry(C, fmt, row, (int)(e % Mp), (int)(e / Mp), M);
}

hipError_t launch_expand_C(double* out, const void* C, int fmtC, int64_t row, int M, int Mp, hipStream_t st) {
  const int64_t MM = (int64_t)Mp * Mp;
  int bx = (int)((MM + 255) / 256);
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_expand_C, dim3(bx), dim3(256), 0, st, out, C, fmtC, row, M, Mp);
  return hipGetLastError();
}

// Blocks of the reduced system, eq. (red1), for diagonal A and B:
//   At_s = diag(a_k) U_{k-1},  Ct_s = C_k - diag(a_k) V_{k-1} - diag(b_k) U_{k+1},  Bt_s = diag(b_k) V_{k+1}
// with k = k_s.  U_{k-1}, V_{k-1} are the coefficients of X_{k_{s-1}}, X_{k_s} in row k-1 (the last
// interior row of subdomain s-1); if that subdomain has no interior row, row k-1 is itself the
// interface row k_{s-1} (U = I, V = 0).  Likewise U_{k+1}, V_{k+1} come from the first interior row of
// subdomain s, or are (U = 0, V = I) when row k+1 is the next interface row.
// UV points at U_0: U_i = UV + 2*i*Mp*Mp, V_i = U_i + Mp*Mp.
__global__ void k_reduced(double* At, double* Ct, double* Bt, const int64_t* ks, const double* UV, const void* C,
                          int fmtC, const double* adiag, const double* bdiag, int p, int N, int M, int Mp) {
  const int s = blockIdx.y;
  const int64_t MM = (int64_t)Mp * Mp;
  const int64_t k = ks[s];
  const bool left_int = (s > 0) && (k - 1 > ks[s - 1]);       // row k-1 is an interior row of s-1
  const bool right_int = (k + 1 < ks[s + 1]);                 // row k+1 is an interior row of s
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MM; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % Mp), c = (int)(e / Mp);
    const double ak = adiag[k * Mp + r], bk = bdiag[k * Mp + r];
    double at = 0.0, ct = c_entry(C, fmtC, k, r, c, M), bt = 0.0;
    if (s > 0) {
      if (left_int) {
        const double* U = UV + (k - 1) * 2 * MM;
        at = ak * U[e];
        ct -= ak * U[MM + e];
      } else {
        at = (r == c) ? ak : 0.0;
      }
    }
    if (k + 1 < N) {
      if (right_int) {
        const double* U = UV + (k + 1) * 2 * MM;
        ct -= bk * U[e];
        bt = bk * U[MM + e];
      } else {
        bt = (r == c) ? bk : 0.0;
      }
    }
    At[s * MM + e] = at;
    Ct[s * MM + e] = ct;
    Bt[s * MM + e] = bt;
  }
}

hipError_t launch_reduced(double* At, double* Ct, double* Bt, const int64_t* ks, const double* UV, const void* C,
                          int fmtC, const double* adiag, const double* bdiag, int p, int N, int M, int Mp,
                          hipStream_t st) {
  const int64_t MM = (int64_t)Mp * Mp;
  int bx = (int)((MM + 255) / 256);
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_reduced, dim3(bx, p), dim3(256), 0, st, At, Ct, Bt, ks, UV, C, fmtC, adiag, bdiag, p, N, M, Mp);
  return hipGetLastError();
}

// dst[N][Mp] = src[N][M] zero padded; optionally zero the first / last block row
__global__ void k_pad_diag(double* dst, const double* src, int N, int M, int Mp, int zero_first, int zero_last) {
  const int64_t n = (int64_t)N * Mp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / Mp;
    const int r = (int)(e % Mp);
    double v = (r < M) ? src[j * M + r] : 0.0;
    if ((zero_first && j == 0) || (zero_last && j == N - 1)) v = 0.0;
    dst[e] = v;
  }
}

hipError_t launch_pad_diag(double* dst, const double* src, int N, int M, int Mp, int zero_first, int zero_last,
                           hipStream_t st) {
  const int64_t n = (int64_t)N * Mp;
  int bx = (int)((n + 255) / 256);
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_pad_diag, dim3(bx), dim3(256), 0, st, dst, src, N, M, Mp, zero_first, zero_last);
  return hipGetLastError();
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_fill, dim3(bx), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// Band matrix (general band storage, column-major: a(i, j) at ab[ku + i - j + j * ldab]) as
// block-tridiagonal blocks of size M >= max(kl, ku): with block rows I = i / M the entries of
// block column I - 1 form -A_I (upper triangular), of block column I form C_I and of block
// column I + 1 form -B_I (lower triangular).  Rows and columns at or beyond n get a unit
// diagonal in C and no couplings.
__global__ void k_band_to_blocks(int64_t n, int kl, int ku, const double* ab, int64_t ldab, int M, int64_t N,
                                 double* A, double* B, double* C) {
  const int64_t MM = (int64_t)M * M;
  const int64_t total = 3 * N * MM;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int which = (int)(e / (N * MM));          // 0: A, 1: C, 2: B
    const int64_t f = e - which * N * MM;
    const int64_t I = f / MM;
    const int r = (int)(f % M), c = (int)((f / M) % M);
    const int64_t i = I * M + r, j = (I + which - 1) * M + c;
    double v = 0.0;
    if (j >= 0 && i < n && j < n && i - j <= kl && j - i <= ku) {
      const double a = ab[ku + i - j + j * ldab];
      v = (which == 1) ? a : -a;
    } else if (which == 1 && r == c && i >= n) {
      v = 1.0;
    }
    double* out = (which == 0) ? A : (which == 1 ? C : B);
    out[f] = v;
  }
}

hipError_t launch_band_to_blocks(int64_t n, int kl, int ku, const double* ab, int64_t ldab, int M, int64_t N,
                                 double* A, double* B, double* C, hipStream_t st) {
  const int64_t total = 3 * N * (int64_t)M * M;
  int64_t bx = (total + 255) / 256;
  if (bx > 16384) bx = 16384;
  hipLaunchKernelGGL(k_band_to_blocks, dim3((unsigned)bx), dim3(256), 0, st, n, kl, ku, ab, ldab, M, N, A, B, C);
  return hipGetLastError();
}

__global__ void k_expand_AB(double* ABd, const double* A, int fmtA, const double* B, int fmtB, int N, int M, int Mp) {
  const int64_t MM = (int64_t)Mp * Mp;
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y)
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 2 * MM; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % Mp), cc = (int)(e / Mp);
    const bool isA = cc < Mp;
    const int c = isA ? cc : cc - Mp;
    double v = 0.0;
    if (r < M && c < M && (isA ? j > 0 : j + 1 < N)) {
      const double* X = isA ? A : B;
      const int fmt = isA ? fmtA : fmtB;
      if (fmt == 1)
        v = (r == c) ? X[j * M + r] : 0.0;                      // DIAG [N][M]
      else
        v = X[j * (int64_t)M * M + r + (int64_t)c * M];         // DENSE, column-major block
    }
    ABd[j * 2 * MM + e] = v;
  }
}

hipError_t launch_expand_AB(double* ABd, const double* A, int fmtA, const double* B, int fmtB, int N, int M, int Mp,
                            hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int64_t MM = (int64_t)Mp * Mp;
  int bx = (int)((2 * MM + 255) / 256);
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_expand_AB, dim3(bx, N < 65535 ? N : 65535), dim3(256), 0, st, ABd, A, fmtA, B, fmtB, N, M, Mp);
  return hipGetLastError();
}

__global__ void k_identity(double* p, int Mp) {
  const int64_t MM = (int64_t)Mp * Mp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MM; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = ((e % Mp) == (e / Mp)) ? 1.0 : 0.0;
}

hipError_t launch_identity(double* p, int Mp, hipStream_t st) {
  const int64_t MM = (int64_t)Mp * Mp;
  int bx = (int)((MM + 255) / 256);
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_identity, dim3(bx), dim3(256), 0, st, p, Mp);
  return hipGetLastError();
}

__global__ void k_set_flag(int32_t* flag, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = v;
}

hipError_t launch_negate_fill_check(int32_t* flag, int32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, st, flag, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Solve helpers
// ---------------------------------------------------------------------------

// Right-hand side of the reduced system, eq. (red1), diagonal A and B:
//   Ft_s = F_k + diag(a_k) W_{k-1} + diag(b_k) W_{k+1},  k = k_s,
// where W of a row that is itself an interface row is zero.
__global__ void k_ftilde(double* Ft, int64_t ldft, const double* F, int64_t ldf, const double* W, int64_t ldw,
                         const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K) {
  const int64_t n = (int64_t)p * Mp * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % Mp);
    const int64_t sc = e / Mp;
    const int s = (int)(sc % p);
    const int64_t col = sc / p;
    const int64_t k = ks[s];
    double v = (r < M) ? F[k * M + r + col * ldf] : 0.0;
    if (s > 0 && k - 1 > ks[s - 1]) v += adiag[k * Mp + r] * W[(k - 1) * Mp + r + col * ldw];
    if (k + 1 < ks[s + 1]) v += bdiag[k * Mp + r] * W[(k + 1) * Mp + r + col * ldw];
    Ft[(int64_t)s * Mp + r + col * ldft] = v;
  }
}

hipError_t launch_ftilde(double* Ft, int64_t ldft, const double* F, int64_t ldf, const double* W, int64_t ldw,
                         const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K,
                         hipStream_t st) {
  const int64_t n = (int64_t)p * Mp * K;
  if (n == 0) return hipSuccess;
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_ftilde, dim3(bx), dim3(256), 0, st, Ft, ldft, F, ldf, W, ldw, ks, adiag, bdiag, p, M, Mp, K);
  return hipGetLastError();
}

// R = F - P X for compact formats (A, B diagonal or dense; C tridiagonal or dense), plus per-block
// partial sums of squares of R and of F per column: colpart[(col * nblk + blk) * 2 + {0,1}].
// One work-group per (block row j, column); entries r < M.
__global__ void k_residual(double* R, int64_t ldr, const double* F, int64_t ldf, const double* X, int64_t ldx,
                           const double* A, int fmtA, const double* B, int fmtB, const double* C, int fmtC, int N,
                           int M, int K, double* colpart, int nblk) {
  __shared__ double red[2][16];
  const int j = blockIdx.x;
  const int col = blockIdx.y;
  const int tid = threadIdx.x;
  const double* x = X + (int64_t)col * ldx;
  const double* f = F + (int64_t)col * ldf;
  const int64_t MM = (int64_t)M * M;
  double sr = 0.0, sf = 0.0;
  for (int r = tid; r < M; r += blockDim.x) {
    const int64_t g = (int64_t)j * M + r;
    double y;
    if (fmtC == 2) {
      const double* t = C + (int64_t)j * 3 * M;
      y = t[M + r] * x[g];
      if (r > 0) y += t[r] * x[g - 1];
      if (r < M - 1) y += t[2 * M + r] * x[g + 1];
    } else {
      const double* Cj = C + j * MM;
      y = 0.0;
      for (int c = 0; c < M; ++c) y += Cj[r + (int64_t)c * M] * x[(int64_t)j * M + c];
    }
    if (j > 0) {
      if (fmtA == 1) y -= A[(int64_t)j * M + r] * x[g - M];
      else {
        const double* Aj = A + j * MM;
        for (int c = 0; c < M; ++c) y -= Aj[r + (int64_t)c * M] * x[(int64_t)(j - 1) * M + c];
      }
    }
    if (j < N - 1) {
      if (fmtB == 1) y -= B[(int64_t)j * M + r] * x[g + M];
      else {
        const double* Bj = B + j * MM;
        for (int c = 0; c < M; ++c) y -= Bj[r + (int64_t)c * M] * x[(int64_t)(j + 1) * M + c];
      }
    }
    const double rv = f[g] - y;
    if (R) R[g + (int64_t)col * ldr] = rv;
    sr += rv * rv;
    sf += f[g] * f[g];
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off);
    sf += __shfl_xor(sf, off);
  }
  if ((tid & 63) == 0) { red[0][tid >> 6] = sr; red[1][tid >> 6] = sf; }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int v = 0; v < (int)(blockDim.x >> 6); ++v) { a += red[0][v]; b += red[1][v]; }
    colpart[((int64_t)col * nblk + j) * 2 + 0] = a;
    colpart[((int64_t)col * nblk + j) * 2 + 1] = b;
  }
}

hipError_t launch_residual(double* R, int64_t ldr, const double* F, int64_t ldf, const double* X, int64_t ldx,
                           const void* A, int fmtA, const void* B, int fmtB, const void* C, int fmtC, int N, int M,
                           int K, double* colpart, int nblk, hipStream_t st) {
  if (K == 0) return hipSuccess;
  int nthr = M >= 256 ? 256 : ((M + 63) / 64) * 64;
  hipLaunchKernelGGL(k_residual, dim3(N, K), dim3(nthr), 0, st, R, ldr, F, ldf, X, ldx, (const double*)A, fmtA,
                     (const double*)B, fmtB, (const double*)C, fmtC, N, M, K, colpart, nblk);
  return hipGetLastError();
}

// out[2*col] = ||R_col||, out[2*col+1] = ||F_col|| from the partial sums of squares
// colpart[col][blk][2]: one wave per column, lanes striding over the blocks, then a fixed
// shuffle tree (deterministic order)
__global__ void __launch_bounds__(256) k_colnorm_finish(double* out, const double* colpart, int nblk, int K) {
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  if (col >= K) return;
  const double2* cp = reinterpret_cast<const double2*>(colpart) + (int64_t)col * nblk;
  double a = 0.0, b = 0.0;
  for (int j = L; j < nblk; j += 64) {
    const double2 v = cp[j];
    a += v.x;
    b += v.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  if (L == 0) {
    out[2 * col] = sqrt(a);
    out[2 * col + 1] = sqrt(b);
  }
}

hipError_t launch_colnorm_finish(double* out, const double* colpart, int nblk, int K, hipStream_t st) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_colnorm_finish, dim3((K + 3) / 4), dim3(256), 0, st, out, colpart, nblk, K);
  return hipGetLastError();
}

// Y[:, col] = X[:, col] * (invert ? 1/s[2col] : s[2col])   (s holds (norm, other) pairs; norm 0 -> 0)
__global__ void k_scale_cols(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* s, int invert,
                             int64_t n, int K) {
  const int64_t tot = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / n, r = e % n;
    const double nv = s[2 * col];
    const double f = invert ? (nv > 0.0 ? 1.0 / nv : 0.0) : nv;
    Y[r + col * ldy] = X[r + col * ldx] * f;
  }
}

hipError_t launch_scale_cols(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* s, int invert,
                             int64_t n, int K, hipStream_t st) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  int bx = (int)((tot + 255) / 256);
  if (bx > 16384) bx = 16384;
  hipLaunchKernelGGL(k_scale_cols, dim3(bx), dim3(256), 0, st, Y, ldy, X, ldx, s, invert, n, K);
  return hipGetLastError();
}

// X[:, col] += s[2col] * D[:, col]
__global__ void k_axpy_cols(double* X, int64_t ldx, const double* D, int64_t ldd, const double* s, int64_t n, int K) {
  const int64_t tot = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / n, r = e % n;
    X[r + col * ldx] += s[2 * col] * D[r + col * ldd];
  }
}

hipError_t launch_axpy_cols(double* X, int64_t ldx, const double* D, int64_t ldd, const double* s, int64_t n, int K,
                            hipStream_t st) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  int bx = (int)((tot + 255) / 256);
  if (bx > 16384) bx = 16384;
  hipLaunchKernelGGL(k_axpy_cols, dim3(bx), dim3(256), 0, st, X, ldx, D, ldd, s, n, K);
  return hipGetLastError();
}

// out[r] = -sum_k Lam[r,k] X[r,k], summed in column order
__global__ void k_diag_grad(double* out, const double* Lam, int64_t ldl, const double* X, int64_t ldx, int64_t n,
                            int K) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += Lam[r + (int64_t)k * ldl] * X[r + (int64_t)k * ldx];
    out[r] = -s;
  }
}

hipError_t launch_diag_grad(double* out, const double* Lam, int64_t ldl, const double* X, int64_t ldx, int64_t n,
                            int K, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_diag_grad, dim3(bx), dim3(256), 0, st, out, Lam, ldl, X, ldx, n, K);
  return hipGetLastError();
}

__global__ void k_nonfinite(int32_t* flag, const double* X, int64_t ldx, int64_t n, int K) {
  const int64_t tot = n * K;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = X[(e % n) + (e / n) * ldx];
    if (!(v - v == 0.0)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_nonfinite(int32_t* flag, const double* X, int64_t ldx, int64_t n, int K, hipStream_t st) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  int bx = (int)((tot + 255) / 256);
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_nonfinite, dim3(bx), dim3(256), 0, st, flag, X, ldx, n, K);
  return hipGetLastError();
}

// Probe inputs of the autotuner: tridiag(-1, d, -1) blocks and hashed uniform[-1,1) right-hand sides.
__global__ void k_fill_tridiag(double* C, int N, int M, double d) {
  const int64_t n = (int64_t)N * 3 * M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int part = (int)((e / M) % 3);
    const int r = (int)(e % M);
    double v = (part == 1) ? d : -1.0;
    if ((part == 0 && r == 0) || (part == 2 && r == M - 1)) v = 0.0;
    C[e] = v;
  }
}

__global__ void k_fill_hash(double* F, int64_t n, uint64_t seed) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    F[e] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

hipError_t launch_probe_inputs(double* A, double* B, double* C, double* F, int N, int M, int64_t K, hipStream_t st) {
  hipError_t e = launch_fill(A, (int64_t)N * M, 1.0, st);
  if (e == hipSuccess) e = launch_fill(B, (int64_t)N * M, 1.0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_tridiag, dim3(256), dim3(256), 0, st, C, N, M, 4.5);
  hipLaunchKernelGGL(k_fill_hash, dim3(1024), dim3(256), 0, st, F, (int64_t)N * M * K, (uint64_t)12345);
  return hipGetLastError();
}

}  // namespace td
