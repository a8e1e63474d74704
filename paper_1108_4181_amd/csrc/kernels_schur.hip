// Kernels of the Schur-complement solver (Sec. 3, eqs. (linear_decomp), (schur_decomp),
// (domains_equation)): the block rows listed as interface columns form the set Gamma, all other
// block rows the interior set I.  The interior rows of all strips are stacked into one
// block-tridiagonal system A_II (couplings across a strip boundary are zero), solved by the
// library's own plan; these kernels move data between the full layout, the stacked interior
// layout and interface vectors, and carry the conjugate-gradient vector algebra (one
// independent iteration per right-hand side).
//
// Layouts: full vectors (N M) x K and stacked interior vectors (Nint M) x K are column-major
// with their leading dimensions; interface vectors are column-major nGp x K (nGp >= nif M,
// rows beyond nif M are padding and stay zero).  The coupling of block row c to c-1 is -A_c,
// to c+1 is -B_c (DIAG [N][M]); C is TRIDIAG [N][3][M].
#include "schur_kernels.h"

namespace td {

namespace {
constexpr int SCHUR_THREADS = 256;
constexpr int DOT_ROWS = 4096;    // rows per partial sum of a column dot product

inline int grid_for(int64_t n, int cap) {
  int64_t b = (n + SCHUR_THREADS - 1) / SCHUR_THREADS;
  if (b > cap) b = cap;
  return b < 1 ? 1 : (int)b;
}
}  // namespace

// Stacked interior coefficients: row j of the stack is full block row intcol[j]; its coupling to
// the previous stacked row is kept only if that row is block row intcol[j] - 1 (same strip).
__global__ void k_schur_interior_coeffs(double* Ai, double* Bi, double* Ci, const double* A, const double* B,
                                        const double* C, const int64_t* intcol, int64_t Nint, int M) {
  const int64_t n = Nint * M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / M;
    const int r = (int)(e - j * M);
    const int64_t c = intcol[j];
    const bool left = j > 0 && intcol[j - 1] == c - 1;
    const bool right = j + 1 < Nint && intcol[j + 1] == c + 1;
    Ai[e] = left ? A[c * M + r] : 0.0;
    Bi[e] = right ? B[c * M + r] : 0.0;
    Ci[j * 3 * M + r] = C[c * 3 * M + r];
    Ci[j * 3 * M + M + r] = C[c * 3 * M + M + r];
    Ci[j * 3 * M + 2 * M + r] = C[c * 3 * M + 2 * M + r];
  }
}

hipError_t launch_schur_interior_coeffs(double* Ai, double* Bi, double* Ci, const double* A, const double* B,
                                        const double* C, const int64_t* intcol, int64_t Nint, int M,
                                        hipStream_t st) {
  hipLaunchKernelGGL(k_schur_interior_coeffs, dim3(grid_for(Nint * M, 4096)), dim3(SCHUR_THREADS), 0, st, Ai, Bi, Ci,
                     A, B, C, intcol, Nint, M);
  return hipGetLastError();
}

// T (stacked interior) = base restricted to I  +  sgn * (A_c v_{c-1} + B_c v_{c+1}) for the
// interface neighbours of each interior row (lif / rif: interface index of block row c-1 / c+1,
// or -1).  base may be null (zero); V null drops the interface terms.  sgn = -1 gives A_IG v; sgn = +1 gives f_I - A_IG x_G.
__global__ void k_schur_scatter(double* T, int64_t ldt, const double* base, int64_t ldb, const double* V,
                                int64_t ldv, const double* A, const double* B, const int64_t* intcol,
                                const int32_t* lif, const int32_t* rif, int64_t Nint, int M, int K, double sgn) {
  const int64_t rows = Nint * M;
  const int64_t n = rows * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / rows;
    const int64_t row = e - col * rows;
    const int64_t j = row / M;
    const int r = (int)(row - j * M);
    const int64_t c = intcol[j];
    double v = base ? base[c * M + r + col * ldb] : 0.0;
    if (V) {
      const int li = lif[j], ri = rif[j];
      if (li >= 0) v += sgn * A[c * M + r] * V[(int64_t)li * M + r + col * ldv];
      if (ri >= 0) v += sgn * B[c * M + r] * V[(int64_t)ri * M + r + col * ldv];
    }
    T[row + col * ldt] = v;
  }
}

hipError_t launch_schur_scatter(double* T, int64_t ldt, const double* base, int64_t ldb, const double* V, int64_t ldv,
                                const double* A, const double* B, const int64_t* intcol, const int32_t* lif,
                                const int32_t* rif, int64_t Nint, int M, int K, double sgn, hipStream_t st) {
  hipLaunchKernelGGL(k_schur_scatter, dim3(grid_for(Nint * M * K, 16384)), dim3(SCHUR_THREADS), 0, st, T, ldt, base,
                     ldb, V, ldv, A, B, intcol, lif, rif, Nint, M, K, sgn);
  return hipGetLastError();
}

// Interface vector out (nGp x K) for interface k at block row g = icol[k]:
//   out = base_g (if base) + (withC ? C_g v_k : 0) + A_g Y(g-1) + B_g Y(g+1)
// with Y the stacked interior vectors (ileft / iright: stacked index of block rows g-1 / g+1).
// This is S v = A_GG v - A_GI (A_II^{-1} A_IG v) for base = null, withC = 1 and Y = A_II^{-1}(A_IG v),
// and the right-hand side f_G - A_GI A_II^{-1} f_I for base = f, withC = 0, Y = A_II^{-1} f_I.
// Padding rows are written as zero.
__global__ void k_schur_gather(double* out, int64_t ldo, const double* base, int64_t ldb, const double* V,
                               int64_t ldv, const double* Y, int64_t ldy, const double* A, const double* B,
                               const double* C, const int64_t* icol, const int64_t* ileft, const int64_t* iright,
                               int64_t nif, int M, int64_t nGp, int K, int withC) {
  const int64_t n = nGp * K;
  const int64_t ng = nif * M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / nGp;
    const int64_t row = e - col * nGp;
    double v = 0.0;
    if (row < ng) {
      const int64_t k = row / M;
      const int r = (int)(row - k * M);
      const int64_t g = icol[k];
      if (base) v = base[g * M + r + col * ldb];
      if (withC) {
        const double* t = C + g * 3 * M;
        const double* vk = V + k * M + col * ldv;
        v += t[M + r] * vk[r];
        if (r > 0) v += t[r] * vk[r - 1];
        if (r < M - 1) v += t[2 * M + r] * vk[r + 1];
      }
      v += A[g * M + r] * Y[ileft[k] * M + r + col * ldy];
      v += B[g * M + r] * Y[iright[k] * M + r + col * ldy];
    }
    out[row + col * ldo] = v;
  }
}

hipError_t launch_schur_gather(double* out, int64_t ldo, const double* base, int64_t ldb, const double* V, int64_t ldv,
                               const double* Y, int64_t ldy, const double* A, const double* B, const double* C,
                               const int64_t* icol, const int64_t* ileft, const int64_t* iright, int64_t nif, int M,
                               int64_t nGp, int K, int withC, hipStream_t st) {
  hipLaunchKernelGGL(k_schur_gather, dim3(grid_for(nGp * K, 16384)), dim3(SCHUR_THREADS), 0, st, out, ldo, base, ldb,
                     V, ldv, Y, ldy, A, B, C, icol, ileft, iright, nif, M, nGp, K, withC);
  return hipGetLastError();
}

// Full solution: interior rows from the stacked Y, interface rows from xG.
__global__ void k_schur_assemble(double* X, int64_t ldx, const double* Y, int64_t ldy, const double* xG, int64_t ldg,
                                 const int64_t* intcol, const int64_t* icol, int64_t Nint, int64_t nif, int M, int K) {
  const int64_t rows = (Nint + nif) * M;
  const int64_t n = rows * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / rows;
    const int64_t row = e - col * rows;
    const int64_t j = row / M;
    const int r = (int)(row - j * M);
    if (j < Nint) X[intcol[j] * M + r + col * ldx] = Y[row + col * ldy];
    else X[icol[j - Nint] * M + r + col * ldx] = xG[(j - Nint) * M + r + col * ldg];
  }
}

hipError_t launch_schur_assemble(double* X, int64_t ldx, const double* Y, int64_t ldy, const double* xG, int64_t ldg,
                                 const int64_t* intcol, const int64_t* icol, int64_t Nint, int64_t nif, int M, int K,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_schur_assemble, dim3(grid_for((Nint + nif) * M * K, 16384)), dim3(SCHUR_THREADS), 0, st, X,
                     ldx, Y, ldy, xG, ldg, intcol, icol, Nint, nif, M, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column dot products d[k] = sum_i x[i,k] y[i,k] (i < n): partial sums over DOT_ROWS rows per
// work-group, then one wave per column adds them in a fixed order (deterministic).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(SCHUR_THREADS) k_coldot_part(double* part, const double* x, const double* y,
                                                               int64_t ld, int64_t n, int nparts) {
  __shared__ double red[SCHUR_THREADS / 64];
  const int q = blockIdx.x, col = blockIdx.y;
  const int64_t r0 = (int64_t)q * DOT_ROWS;
  const int64_t r1 = r0 + DOT_ROWS < n ? r0 + DOT_ROWS : n;
  const double* xc = x + (int64_t)col * ld;
  const double* yc = y + (int64_t)col * ld;
  double s = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += SCHUR_THREADS) s += xc[r] * yc[r];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int v = 0; v < SCHUR_THREADS / 64; ++v) t += red[v];
    part[(int64_t)col * nparts + q] = t;
  }
}

__global__ void __launch_bounds__(SCHUR_THREADS) k_coldot_finish(double* d, const double* part, int nparts, int K) {
  const int col = blockIdx.x * (SCHUR_THREADS / 64) + (threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  if (col >= K) return;
  double s = 0.0;
  for (int q = L; q < nparts; q += 64) s += part[(int64_t)col * nparts + q];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (L == 0) d[col] = s;
}

int schur_dot_parts(int64_t n) { return (int)((n + DOT_ROWS - 1) / DOT_ROWS); }

hipError_t launch_coldot(double* d, double* part, const double* x, const double* y, int64_t ld, int64_t n, int K,
                         hipStream_t st) {
  const int nparts = schur_dot_parts(n);
  hipLaunchKernelGGL(k_coldot_part, dim3(nparts, K), dim3(SCHUR_THREADS), 0, st, part, x, y, ld, n, nparts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coldot_finish, dim3((K + 3) / 4), dim3(SCHUR_THREADS), 0, st, d, part, nparts, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conjugate-gradient steps, one independent iteration per column k (Sec. 3 uses CG on eq.
// (schur_decomp); a preconditioned form with z = B^{-1} r):
//   alpha_k = rz_k / (p_k . q_k)    x_k += alpha_k p_k    r_k -= alpha_k q_k
//   beta_k  = rz'_k / rz_k          p_k  = z_k + beta_k p_k
// Columns that have converged (active[k] == 0) keep alpha = beta = 0.
// ---------------------------------------------------------------------------
__global__ void k_cg_alpha(double* alpha, const double* rz, const double* pq, const int32_t* active, int K) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) alpha[k] = (active[k] && pq[k] != 0.0) ? rz[k] / pq[k] : 0.0;
}

__global__ void k_cg_update(double* x, double* r, const double* p, const double* q, const double* alpha, int64_t ld,
                            int64_t n, int K) {
  const int64_t tot = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / n;
    const int64_t i = e - col * n + col * ld;
    const double a = alpha[col];
    x[i] += a * p[i];
    r[i] -= a * q[i];
  }
}

__global__ void k_cg_direction(double* p, const double* z, const double* rz_new, const double* rz_old,
                               const int32_t* active, int64_t ld, int64_t n, int K) {
  const int64_t tot = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / n;
    const int64_t i = e - col * n + col * ld;
    const double b = (active[col] && rz_old[col] != 0.0) ? rz_new[col] / rz_old[col] : 0.0;
    p[i] = z[i] + b * p[i];
  }
}

// active[k] = ||r_k||^2 > tol^2 ||g_k||^2; stat[0] = number of active columns, stat[1] = max_k
// ||r_k|| / ||g_k|| (one work-group, fixed order)
__global__ void __launch_bounds__(SCHUR_THREADS) k_cg_status(int32_t* active, double* stat, const double* rr,
                                                             const double* gg, double tol, int K) {
  __shared__ double smax[SCHUR_THREADS / 64];
  __shared__ int scnt[SCHUR_THREADS / 64];
  double worst = 0.0;
  int cnt = 0;
  for (int k = threadIdx.x; k < K; k += SCHUR_THREADS) {
    const double g = gg[k];
    const double rel = g > 0.0 ? sqrt(rr[k] / g) : (rr[k] > 0.0 ? INFINITY : 0.0);
    const int a = !(rel <= tol);   // NaN stays active (and is reported)
    active[k] = a;
    cnt += a;
    if (!(rel <= worst)) worst = rel;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(worst, off);
    if (!(o <= worst)) worst = o;
    cnt += __shfl_xor(cnt, off);
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = worst;
    scnt[threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double w = smax[0];
    int c = scnt[0];
    for (int v = 1; v < SCHUR_THREADS / 64; ++v) {
      if (!(smax[v] <= w)) w = smax[v];
      c += scnt[v];
    }
    stat[0] = (double)c;
    stat[1] = w;
  }
}

hipError_t launch_cg_alpha(double* alpha, const double* rz, const double* pq, const int32_t* active, int K,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3((K + 255) / 256), dim3(256), 0, st, alpha, rz, pq, active, K);
  return hipGetLastError();
}
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, const double* alpha, int64_t ld,
                            int64_t n, int K, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_update, dim3(grid_for(n * K, 8192)), dim3(SCHUR_THREADS), 0, st, x, r, p, q, alpha, ld, n, K);
  return hipGetLastError();
}
hipError_t launch_cg_direction(double* p, const double* z, const double* rz_new, const double* rz_old,
                               const int32_t* active, int64_t ld, int64_t n, int K, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_direction, dim3(grid_for(n * K, 8192)), dim3(SCHUR_THREADS), 0, st, p, z, rz_new, rz_old,
                     active, ld, n, K);
  return hipGetLastError();
}
hipError_t launch_cg_status(int32_t* active, double* stat, const double* rr, const double* gg, double tol, int K,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_cg_status, dim3(1), dim3(SCHUR_THREADS), 0, st, active, stat, rr, gg, tol, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probing (Sec. 3, preconditioning): 2 (2d+1) probe vectors over the interface unknowns,
// probe (l, par) holding ones at the unknowns i with i mod (2d+1) == l on the interfaces of
// parity par (interfaces of one parity are never neighbours, so a probe of one interface
// does not pick up the coupling of the next one through their common strip).  From Y = S V the
// band matrix of half-width d: b(i, j) = (S v_{l(j), par(j)})_i for |i - j| <= d with i, j on
// the same interface, symmetrised, in general band storage (entry (i, j) at
// ab[d + i - j + j * ldab]); couplings between different interfaces are dropped.
// ---------------------------------------------------------------------------
__global__ void k_probe_vectors(double* V, int64_t ldv, int64_t nGp, int64_t ng, int M, int d) {
  const int w = 2 * d + 1;
  const int64_t tot = nGp * 2 * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / nGp;
    const int64_t i = e - col * nGp;
    const int l = (int)(col % w), par = (int)(col / w);
    double v = 0.0;
    if (i < ng && (int)(i % w) == l && (int)((i / M) & 1) == par) v = 1.0;
    V[i + col * ldv] = v;
  }
}

__global__ void k_probe_band(double* ab, int64_t ldab, const double* Y, int64_t ldy, int64_t ng, int M, int d) {
  const int w = 2 * d + 1;
  const int64_t tot = ng * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / w;
    const int o = (int)(e - j * w) - d;   // i - j
    const int64_t i = j + o;
    double v = 0.0;
    if (i >= 0 && i < ng && i / M == j / M) {
      const int64_t cj = (j % w) + (int64_t)w * ((j / M) & 1);   // probe holding unknown j
      const int64_t ci = (i % w) + (int64_t)w * ((i / M) & 1);
      v = 0.5 * (Y[i + cj * ldy] + Y[j + ci * ldy]);
    }
    ab[d + o + j * ldab] = v;
  }
}

hipError_t launch_probe_vectors(double* V, int64_t ldv, int64_t nGp, int64_t ng, int M, int d, hipStream_t st) {
  hipLaunchKernelGGL(k_probe_vectors, dim3(grid_for(nGp * 2 * (2 * d + 1), 8192)), dim3(SCHUR_THREADS), 0, st, V, ldv,
                     nGp, ng, M, d);
  return hipGetLastError();
}
hipError_t launch_probe_band(double* ab, int64_t ldab, const double* Y, int64_t ldy, int64_t ng, int M, int d,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_probe_band, dim3(grid_for(ng * (2 * d + 1), 8192)), dim3(SCHUR_THREADS), 0, st, ab, ldab, Y,
                     ldy, ng, M, d);
  return hipGetLastError();
}

}  // namespace td
