// Algorithm 1 (Sec. 2.1) on a scalar tridiagonal system (block size 1, every row an interface row):
// the dichotomy tree over rows 0..N-1 splits node [l, r] at m = floor((l + r) / 2); the factor stores,
// for every node, row m of the inverse of the node's submatrix (g_m[j], j in [l, r], kept per tree
// level in G[level * N + j]) and the two boundary coefficients hl_m = g_m[l] a_l, hr_m = g_m[r] b_r;
// the solve computes x_m = sum_j g_m[j] f_j + hl_m x_{l-1} + hr_m x_{r+1}, level by level from the root.
//
// Row j of the system reads -a_j x_{j-1} + c_j x_j - b_j x_{j+1} = f_j (a_0 and b_{N-1} ignored).
// Row m of T^{-1} for T = T[l..r]: with the eliminations from both ends,
//   DL_l = c_l, DL_j = c_j - a_j b_{j-1} / DL_{j-1}  (j = l+1 .. m-1)
//   DR_r = c_r, DR_j = c_j - b_j a_{j+1} / DR_{j+1}  (j = r-1 .. m+1)
//   g_m = 1 / (c_m - a_m b_{m-1} / DL_{m-1} - b_m a_{m+1} / DR_{m+1})   (terms absent at m = l or r)
//   g_j = g_{j+1} a_{j+1} / DL_j (j < m),  g_j = g_{j-1} b_{j-1} / DR_j (j > m).
//
// Solve layout: the nodes of level L0 (at most SC_SUB rows each) are the subtrees; the nodes above are
// the top nodes.  Kernel 1 gives, per subtree and column, the subtree's part of the sums of the top
// nodes that contain it (one per top level); kernel 2 completes the top nodes' sums and solves the top
// levels (one thread per column); kernel 3 solves each subtree's levels with f, x and one level of g in
// LDS, taking the subtree's two boundary values from kernel 2.
#include "device_common.h"
#include "internal.h"

#include <cfloat>

namespace td {

// ---------------------------------------------------------------------------------------------
// Factor: one thread per node (nodes indexed by their split row m)
// ---------------------------------------------------------------------------------------------
__global__ void k_scalar_factor(const double* __restrict__ a, const double* __restrict__ b,
                                const double* __restrict__ cdiag, int cs, int N, const int* __restrict__ lo,
                                const int* __restrict__ hi, const int* __restrict__ lvl, double* G, double* hl,
                                double* hr, int32_t* bad) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int l = lo[m], r = hi[m];
  double* g = G + (int64_t)lvl[m] * N;
  auto c = [&](int j) { return cdiag[(int64_t)j * cs]; };
  auto av = [&](int j) { return j > 0 ? a[j] : 0.0; };
  auto bv = [&](int j) { return j + 1 < N ? b[j] : 0.0; };
  bool sing = false;
  auto check = [&](double d, int j) {   // a pivot not above 1e-14 times its row's magnitude (or NaN)
    const double s = fabs(c(j)) + fabs(av(j)) + fabs(bv(j));
    if (!(fabs(d) > 1e-14 * s)) sing = true;
  };
  // left elimination: g[j] holds 1 / DL_j for j in [l, m-1]
  double inv = 0.0;
  for (int j = l; j < m; ++j) {
    const double d = (j == l) ? c(j) : c(j) - av(j) * bv(j - 1) * inv;
    check(d, j);
    inv = 1.0 / d;
    g[j] = inv;
  }
  const double invL = inv;
  // right elimination: g[j] holds 1 / DR_j for j in [m+1, r]
  inv = 0.0;
  for (int j = r; j > m; --j) {
    const double d = (j == r) ? c(j) : c(j) - bv(j) * av(j + 1) * inv;
    check(d, j);
    inv = 1.0 / d;
    g[j] = inv;
  }
  const double invR = inv;
  double s = c(m);
  if (m > l) s -= av(m) * bv(m - 1) * invL;
  if (m < r) s -= bv(m) * av(m + 1) * invR;
  check(s, m);
  const double gm = 1.0 / s;
  g[m] = gm;
  double gv = gm;
  for (int j = m - 1; j >= l; --j) {   // g_j = g_{j+1} a_{j+1} / DL_j
    gv = gv * av(j + 1) * g[j];
    g[j] = gv;
  }
  gv = gm;
  for (int j = m + 1; j <= r; ++j) {   // g_j = g_{j-1} b_{j-1} / DR_j
    gv = gv * bv(j - 1) * g[j];
    g[j] = gv;
  }
  hl[m] = g[l] * av(l);
  hr[m] = g[r] * bv(r);
  if (sing) atomicMin(bad, N + m);
}

hipError_t launch_scalar_factor(const double* a, const double* b, const double* cdiag, int cs, int N, const int* lo,
                                const int* hi, const int* lvl, double* G, double* hl, double* hr, int32_t* bad,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_factor, dim3((N + 63) / 64), dim3(64), 0, st, a, b, cdiag, cs, N, lo, hi, lvl, G, hl,
                     hr, bad);
  return hipGetLastError();
}

// the boundary coefficients of the subtrees' nodes in the order of their records (level order)
__global__ void k_scalar_gather_h(double* sub_h, const int4* rec, int nrec, const double* hl, const double* hr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrec) return;
  const int m = rec[i].x;
  sub_h[2 * i] = hl[m];
  sub_h[2 * i + 1] = hr[m];
}

hipError_t launch_scalar_gather_h(double* sub_h, const int4* rec, int nrec, const double* hl, const double* hr,
                                  hipStream_t st) {
  if (nrec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scalar_gather_h, dim3((nrec + 255) / 256), dim3(256), 0, st, sub_h, rec, nrec, hl, hr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------------------------
// Kernel 1: Pt[(lv * nsub + s) * K + k] = sum over the rows of subtree s of G[lv][j] F[j, k], lv < L0.
// Grid (nsub, ceil(K / SC_CPW)), 256 threads; each thread keeps its SC_SUB / 256 rows of the
// SC_CPW columns in registers (F read once) and walks the top levels' rows of G.
__global__ void __launch_bounds__(256) k_scalar_top_partials(const ScalarArgs A) {
  constexpr int RPT = SC_SUB / 256;
  const int s = blockIdx.x;
  const int k0 = blockIdx.y * SC_CPW;
  const int l = A.sub_lo[s], r = A.sub_hi[s];
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6;
  __shared__ double red[4][SC_CPW];
  double fv[RPT][SC_CPW];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int j = min(l + tid + 256 * i, r);   // clamped row: its product is dropped below
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) {
      const int k = min(k0 + c, A.K - 1);      // clamped column: its sum is not stored
      fv[i][c] = A.F[j + (int64_t)k * A.ldf];
    }
  }
  for (int lv = 0; lv < A.L0; ++lv) {
    const double* g = A.G + (int64_t)lv * A.N;
    double acc[SC_CPW];
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) acc[c] = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int j = l + tid + 256 * i;
      const double gj = (j <= r) ? g[min(j, r)] : 0.0;
#pragma unroll
      for (int c = 0; c < SC_CPW; ++c) acc[c] += gj * fv[i][c];
    }
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) {
      double v = acc[c];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (L == 0) red[w][c] = v;
    }
    __syncthreads();
    if (tid < SC_CPW && k0 + tid < A.K)
      A.Pt[((int64_t)lv * A.nsub + s) * A.K + k0 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
}

// Kernel 2: one wave per column.  First every top node's sum (lanes over the nodes: the subtree
// parts from kernel 1 and the top rows' own terms), then the top levels in order (the top levels
// are complete binary levels: level lv is positions [2^lv - 1, 2^(lv+1) - 1) of the top list), x in
// LDS; x of the top rows -> Xt[t * K + k] and X (written, or added when accumulating).
__global__ void __launch_bounds__(64) k_scalar_top(const ScalarArgs A) {
  extern __shared__ double sx[];           // [ntop]: the node's sum, then its x
  const int k = blockIdx.x;
  const int L = threadIdx.x;
  for (int t = L; t < A.ntop; t += 64) {
    const int lv = A.top_lvl[t];
    const double* g = A.G + (int64_t)lv * A.N;
    double S = 0.0;
    for (int q = A.top_s0[t]; q < A.top_s1[t]; ++q) S += A.Pt[((int64_t)lv * A.nsub + q) * A.K + k];
    for (int q = A.top_t0[t]; q < A.top_t1[t]; ++q) {
      const int j = A.toprow_sorted[q];
      S += g[j] * A.F[j + (int64_t)k * A.ldf];
    }
    sx[t] = S;
  }
  __syncthreads();
  for (int lv = 0; lv < A.L0; ++lv) {
    const int t1 = min((2 << lv) - 1, A.ntop);
    for (int t = (1 << lv) - 1 + L; t < t1; t += 64) {
      const int m = A.top_m[t];
      const int tl = A.top_left[t], tr = A.top_right[t];   // ancestors: their x is already in sx
      double x = sx[t];
      if (tl >= 0) x += A.hl[m] * sx[tl];
      if (tr >= 0) x += A.hr[m] * sx[tr];
      sx[t] = x;
      double* xo = A.X + m + (int64_t)k * A.ldx;
      *xo = A.accumulate ? *xo + x : x;
    }
    __syncthreads();
  }
  for (int t = L; t < A.ntop; t += 64) A.Xt[(int64_t)t * A.K + k] = sx[t];
}

// Kernel 3: grid (nsub, ceil(K / SC_CPW)), 256 threads; LDS: f and x of SC_CPW columns (with one
// boundary entry on each side) and one level of g for the subtree's rows.
__global__ void __launch_bounds__(256) k_scalar_sub(const ScalarArgs A) {
  extern __shared__ double sm[];
  const int s = blockIdx.x;
  const int k0 = blockIdx.y * SC_CPW;
  const int l = A.sub_lo[s], r = A.sub_hi[s];
  const int n = r - l + 1;                 // <= SC_SUB
  const int W = n + 2;
  double* fs = sm;                         // [SC_CPW][W]: f at rows l-1 .. r+1 (ends unused)
  double* xs = fs + SC_CPW * W;            // [SC_CPW][W]: x at rows l-1 .. r+1
  double* gs = xs + SC_CPW * W;            // [W]: g of the current level at rows l .. r (index j - l + 1)
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6;
  constexpr int RPT = SC_SUB / 256;
  {   // f of the SC_CPW columns: all loads issued before the LDS stores
    double t[SC_CPW][RPT];
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) {
      const int k = min(k0 + c, A.K - 1);
#pragma unroll
      for (int i = 0; i < RPT; ++i) t[c][i] = A.F[l + min(tid + 256 * i, n - 1) + (int64_t)k * A.ldf];
    }
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c)
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (tid + 256 * i < n) fs[c * W + 1 + tid + 256 * i] = t[c][i];
  }
  if (tid < SC_CPW) {
    const int k = min(k0 + tid, A.K - 1);
    const int tl = A.sub_left[s], tr = A.sub_right[s];
    xs[tid * W] = tl >= 0 ? A.Xt[(int64_t)tl * A.K + k] : 0.0;
    xs[tid * W + n + 1] = tr >= 0 ? A.Xt[(int64_t)tr * A.K + k] : 0.0;
  }
  // this subtree's nodes in level order: records {m, l, r, -} and coefficients {hl, hr}
  const int4* rec = A.sub_rec + A.sub_off[s];
  const double2* hh = A.sub_h + A.sub_off[s];
  const int* loff = A.sub_lvoff + s * (A.ndeep + 1);    // level boundaries within the records
  // g of the first deep level in registers; each level stores its g to LDS and loads the next one's
  double gn[RPT];
  {
    const double* g = A.G + (int64_t)A.L0 * A.N;
#pragma unroll
    for (int i = 0; i < RPT; ++i) gn[i] = g[l + min(tid + 256 * i, n - 1)];
  }
  for (int d = 0; d < A.ndeep; ++d) {
    const int b0 = loff[d], b1 = loff[d + 1];
    if (b0 == b1) break;
    __syncthreads();                                    // previous level's x and g reads are done
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (tid + 256 * i < n) gs[1 + tid + 256 * i] = gn[i];
    if (d + 1 < A.ndeep) {                              // next level's g, in flight during this level
      const double* g = A.G + (int64_t)(A.L0 + d + 1) * A.N;
#pragma unroll
      for (int i = 0; i < RPT; ++i) gn[i] = g[l + min(tid + 256 * i, n - 1)];
    }
    const int nn = b1 - b0;
    const int4 r0 = rec[b0];
    const int len0 = r0.z - r0.y + 1;                   // node sizes within a level differ by at most 1
    __syncthreads();
    if (len0 >= 32) {
      // one wave per (node, column): strided partial sums, then a wave reduction
      for (int p = w; p < nn * SC_CPW; p += 4) {
        const int q = __builtin_amdgcn_readfirstlane(b0 + p / SC_CPW), c = p % SC_CPW;
        const int4 rc = rec[q];
        const double2 h = hh[q];
        double S = 0.0;
        for (int j = rc.y + L; j <= rc.z; j += 64) S += gs[j - l + 1] * fs[c * W + j - l + 1];
        for (int off = 32; off > 0; off >>= 1) S += __shfl_xor(S, off);
        if (L == 0)
          xs[c * W + rc.x - l + 1] = S + h.x * xs[c * W + rc.y - l] + h.y * xs[c * W + rc.z - l + 2];
      }
    } else {
      // one thread per (node, column); a thread's records of the level are loaded together, QM at a
      // time (a level has at most SC_SUB / 2 nodes, so one round for SC_CPW = 4)
      constexpr int QM = (SC_SUB / 2 * SC_CPW + 255) / 256;
      const int np = nn * SC_CPW;
      for (int p0 = 0; p0 < np; p0 += 256 * QM) {
        int4 rq[QM];
        double2 hq[QM];
#pragma unroll
        for (int u = 0; u < QM; ++u) {
          const int p = min(p0 + tid + 256 * u, np - 1);
          rq[u] = rec[b0 + p / SC_CPW];
          hq[u] = hh[b0 + p / SC_CPW];
        }
#pragma unroll
        for (int u = 0; u < QM; ++u) {
          const int p = p0 + tid + 256 * u;
          if (p >= np) break;
          const int c = p % SC_CPW;
          const int4 rc = rq[u];
          double S0 = 0.0, S1 = 0.0;   // two chains of dependent additions
          int j = rc.y;
          for (; j + 1 <= rc.z; j += 2) {
            S0 += gs[j - l + 1] * fs[c * W + j - l + 1];
            S1 += gs[j - l + 2] * fs[c * W + j - l + 2];
          }
          if (j <= rc.z) S0 += gs[j - l + 1] * fs[c * W + j - l + 1];
          xs[c * W + rc.x - l + 1] =
              (S0 + S1) + hq[u].x * xs[c * W + rc.y - l] + hq[u].y * xs[c * W + rc.z - l + 2];
        }
      }
    }
  }
  __syncthreads();
  for (int c = 0; c < SC_CPW; ++c) {
    const int k = k0 + c;
    if (k >= A.K) break;
    double* xo = A.X + l + (int64_t)k * A.ldx;
    for (int i = tid; i < n; i += 256) {
      const double v = xs[c * W + 1 + i];
      xo[i] = A.accumulate ? xo[i] + v : v;
    }
  }
}

hipError_t launch_scalar_top(const ScalarArgs& A, hipStream_t st) {
  if (A.K == 0 || A.L0 == 0) return hipSuccess;
  const int cg = (A.K + SC_CPW - 1) / SC_CPW;
  hipLaunchKernelGGL(k_scalar_top_partials, dim3(A.nsub, cg), dim3(256), 0, st, A);
  hipLaunchKernelGGL(k_scalar_top, dim3(A.K), dim3(64), (size_t)A.ntop * sizeof(double), st, A);
  return hipGetLastError();
}

hipError_t launch_scalar_sub(const ScalarArgs& A, hipStream_t st) {
  if (A.K == 0) return hipSuccess;
  const int cg = (A.K + SC_CPW - 1) / SC_CPW;
  const size_t lds = (size_t)(2 * SC_CPW + 1) * (A.maxsub + 2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_scalar_sub, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scalar_sub, dim3(A.nsub, cg), dim3(256), lds, st, A);
  return hipGetLastError();
}

}  // namespace td
