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
// levels (one wave per column); kernel 3 solves each subtree's levels with f, x and one level of g in
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
// Sum over aligned groups of G lanes (G a power of two, the same in every lane) with DPP moves:
// swaps within quads, half-row and row mirrors, then row broadcasts.  The group's total ends in its
// last lane (in every lane of the group for G <= 16).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_take(double v) {   // the selected lane's v; 0 in rows outside ROWMASK
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double group_sum(double v, int G) {
  if (G >= 2) v += dpp_take<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  if (G >= 4) v += dpp_take<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  if (G >= 8) v += dpp_take<0x141, 0xF>(v);   // row_half_mirror
  if (G >= 16) v += dpp_take<0x140, 0xF>(v);  // row_mirror
  if (G >= 32) v += dpp_take<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  if (G >= 64) v += dpp_take<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Kernel 1: Pt[(lv * nsub + s) * K + k] = sum over the rows of subtree s of G[lv][j] F[j, k], lv < L0.
// Grid (nsub, ceil(K / SC_CPW)), 256 threads; each thread keeps its SC_SUB / 256 rows of the
// SC_CPW columns in registers (F read once) and walks the top levels' rows of G; each wave's sums
// (DPP, no barrier) go to LDS and one barrier at the end precedes the sum over the four waves.
constexpr int SC_MAXTOP = 24;   // top levels (L0 <= log2(N / SC_SUB) + 1 for N below 2^31)
__global__ void __launch_bounds__(256) k_scalar_top_partials(const ScalarArgs A) {
  constexpr int RPT = SC_SUB / 256;
  const int s = blockIdx.x;
  const int k0 = blockIdx.y * SC_CPW;
  const int l = A.sub_lo[s], r = A.sub_hi[s];
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6;
  __shared__ double red[SC_MAXTOP][4][SC_CPW];
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
  double gq[RPT];   // the next level's rows of G, loaded one level ahead
  auto load_g = [&](int lv) {
    const double* g = A.G + (int64_t)lv * A.N;
#pragma unroll
    for (int i = 0; i < RPT; ++i) gq[i] = g[min(l + tid + 256 * i, r)];
  };
  load_g(0);
  for (int lv = 0; lv < A.L0; ++lv) {
    double gv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) gv[i] = (l + tid + 256 * i <= r) ? gq[i] : 0.0;
    if (lv + 1 < A.L0) load_g(lv + 1);
    double acc[SC_CPW];
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) acc[c] = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int c = 0; c < SC_CPW; ++c) acc[c] += gv[i] * fv[i][c];
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) {
      const double v = group_sum(acc[c], 64);
      if (L == 63) red[lv][w][c] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < A.L0 * SC_CPW; e += 256) {
    const int lv = e / SC_CPW, c = e % SC_CPW;
    if (k0 + c < A.K)
      A.Pt[((int64_t)lv * A.nsub + s) * A.K + k0 + c] = red[lv][0][c] + red[lv][1][c] + red[lv][2][c] + red[lv][3][c];
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

// Kernel 3: grid (nsub, ceil(K / SC_CPW)), SC_SUB_THREADS threads; LDS: f of SC_CPW columns (with one
// boundary entry on each side), overwritten in place by x (row m's f is read only by the sum of the
// node split at m, which writes x_m; later levels read x only at their nodes' boundaries), and two
// levels of g for the subtree's rows (the next level's g is stored while the current one is read,
// so a level needs one barrier).  A level with at
// most SC_SUB_THREADS (node, column) pairs gives each pair a group of G lanes (the largest power of
// two with pairs x G <= SC_SUB_THREADS): the lanes sum strided rows of the node, four at a time, and
// the group's sum is formed with DPP moves, so a level costs about SC_SUB * SC_CPW / SC_SUB_THREADS
// products per thread whatever its node count; a level with more pairs takes them one per thread, in
// rounds, with the rounds' node records loaded together.
constexpr int SC_SUB_THREADS = 512;
__global__ void __launch_bounds__(SC_SUB_THREADS, 6) k_scalar_sub(const ScalarArgs A) {
  constexpr int NT = SC_SUB_THREADS;
  extern __shared__ double sm[];
  const int s = blockIdx.x;
  const int k0 = blockIdx.y * SC_CPW;
  const int l = A.sub_lo[s], r = A.sub_hi[s];
  const int n = r - l + 1;                 // <= SC_SUB
  const int W = n + 2;
  double* fs = sm;                         // [SC_CPW][W]: f, then x, at rows l-1 .. r+1 (x only at the ends)
  double* xs = fs;
  double* gsb = fs + SC_CPW * W;           // [2][W]: g of levels d (buffer d % 2) at rows l .. r (index j - l + 1)
  const int tid = threadIdx.x;
  constexpr int RPT = SC_SUB / NT;
  {   // f of the SC_CPW columns: all loads issued before the LDS stores
    double t[SC_CPW][RPT];
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c) {
      const int k = min(k0 + c, A.K - 1);
#pragma unroll
      for (int i = 0; i < RPT; ++i) t[c][i] = A.F[l + min(tid + NT * i, n - 1) + (int64_t)k * A.ldf];
    }
#pragma unroll
    for (int c = 0; c < SC_CPW; ++c)
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (tid + NT * i < n) fs[c * W + 1 + tid + NT * i] = t[c][i];
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
  // g of the first deep level to LDS buffer 0, the second one's in registers; level d stores level
  // d + 1's g (buffer (d + 1) % 2, last read by level d - 1) and loads level d + 2's
  double gn[RPT];
  {
    const double* g = A.G + (int64_t)A.L0 * A.N;
#pragma unroll
    for (int i = 0; i < RPT; ++i) gn[i] = g[l + min(tid + NT * i, n - 1)];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (tid + NT * i < n) gsb[1 + tid + NT * i] = gn[i];
    if (A.ndeep > 1) {
      const double* g1 = A.G + (int64_t)(A.L0 + 1) * A.N;
#pragma unroll
      for (int i = 0; i < RPT; ++i) gn[i] = g1[l + min(tid + NT * i, n - 1)];
    }
  }
  // a level has at most SC_SUB / 2 nodes: QM rounds of one (node, column) pair per thread
  constexpr int QM = (SC_SUB / 2 * SC_CPW + NT - 1) / NT;
  for (int d = 0; d < A.ndeep; ++d) {
    const int b0 = loff[d], b1 = loff[d + 1];
    if (b0 == b1) break;
    const int np = (b1 - b0) * SC_CPW;                  // (node, column) pairs of the level
    int G = 64;
    while (G > 1 && np * G > NT) G >>= 1;
    // this thread's node records, loaded before the barrier so that their latency overlaps it
    int4 rq[QM];
    double2 hq[QM];
    const int sub = tid & (G - 1);
    if (np <= NT) {
      const int p = min(tid / G, np - 1);
      rq[0] = rec[b0 + p / SC_CPW];
      hq[0] = hh[b0 + p / SC_CPW];
    } else {
#pragma unroll
      for (int u = 0; u < QM; ++u) {
        const int p = min(tid + NT * u, np - 1);
        rq[u] = rec[b0 + p / SC_CPW];
        hq[u] = hh[b0 + p / SC_CPW];
      }
    }
    __syncthreads();   // level d - 1's x writes and its reads of buffer (d + 1) % 2 are done
    const double* gs = gsb + (d & 1) * W;
    if (d + 1 < A.ndeep) {
      double* gw = gsb + ((d + 1) & 1) * W;
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (tid + NT * i < n) gw[1 + tid + NT * i] = gn[i];
      if (d + 2 < A.ndeep) {
        const double* g = A.G + (int64_t)(A.L0 + d + 2) * A.N;
#pragma unroll
        for (int i = 0; i < RPT; ++i) gn[i] = g[l + min(tid + NT * i, n - 1)];
      }
    }
    if (np <= NT) {
      // one round: G lanes per pair; lanes beyond the last pair repeat it and write nothing
      const int p = tid / G;
      const int c = min(p, np - 1) % SC_CPW;
      const int4 rc = rq[0];
      const double* gp = gs - l + 1;
      const double* fp = fs + c * W - l + 1;
      double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0;   // four chains, their loads issued together
      int j = rc.y + sub;
      for (; j + 3 * G <= rc.z; j += 4 * G) {
        S0 += gp[j] * fp[j];
        S1 += gp[j + G] * fp[j + G];
        S2 += gp[j + 2 * G] * fp[j + 2 * G];
        S3 += gp[j + 3 * G] * fp[j + 3 * G];
      }
      for (; j <= rc.z; j += G) S0 += gp[j] * fp[j];
      const double S = group_sum((S0 + S1) + (S2 + S3), G);
      if (p < np && sub == G - 1)
        xs[c * W + rc.x - l + 1] = S + hq[0].x * xs[c * W + rc.y - l] + hq[0].y * xs[c * W + rc.z - l + 2];
    } else {
#pragma unroll
      for (int u = 0; u < QM; ++u) {
        const int p = tid + NT * u;
        if (p >= np) break;
        const int c = p % SC_CPW;
        const int4 rc = rq[u];
        double S0 = 0.0, S1 = 0.0;
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
  __syncthreads();
  for (int c = 0; c < SC_CPW; ++c) {
    const int k = k0 + c;
    if (k >= A.K) break;
    double* xo = A.X + l + (int64_t)k * A.ldx;
    for (int i = tid; i < n; i += NT) {
      const double v = xs[c * W + 1 + i];
      xo[i] = A.accumulate ? xo[i] + v : v;
    }
  }
}

hipError_t launch_scalar_top(const ScalarArgs& A, hipStream_t st) {
  if (A.K == 0 || A.L0 == 0) return hipSuccess;
  if (A.L0 > SC_MAXTOP) return hipErrorInvalidValue;   // not reached for N below 2^31
  const int cg = (A.K + SC_CPW - 1) / SC_CPW;
  hipLaunchKernelGGL(k_scalar_top_partials, dim3(A.nsub, cg), dim3(256), 0, st, A);
  hipLaunchKernelGGL(k_scalar_top, dim3(A.K), dim3(64), (size_t)A.ntop * sizeof(double), st, A);
  return hipGetLastError();
}

hipError_t launch_scalar_sub(const ScalarArgs& A, hipStream_t st) {
  if (A.K == 0) return hipSuccess;
  const int cg = (A.K + SC_CPW - 1) / SC_CPW;
  const size_t lds = (size_t)(SC_CPW + 2) * (A.maxsub + 2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_scalar_sub, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scalar_sub, dim3(A.nsub, cg), dim3(SC_SUB_THREADS), lds, st, A);
  return hipGetLastError();
}

}  // namespace td
