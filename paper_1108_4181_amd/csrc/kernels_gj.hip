// Batched Gauss-Jordan inversion of the factor's diagonal blocks (gfx950): the block inverses
// D_i^{-1} of the subdomain elimination and the chain inverses of the dichotomy tree, with partial
// pivoting inside each block.  Float64 products on v_mfma_f64_4x4x4f64 used as 16 x 4 output tiles
// (lane layout as in kernels_f64.hip: A[L%16][L/16], B[L/16][L%4], D[4*((L/4)%4) + L/16][L%4]).
#include "device_common.h"
#include "internal.h"

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cstdlib>

namespace td {

// ---------------------------------------------------------------------------
// Batched Gauss-Jordan inversion with partial pivoting (row interchanges chosen
// by the largest remaining entry of each column; ties go to the lowest row), for
// the block sizes below 128 or not a multiple of 64 (k_gj; the others use the
// per-panel kernel k_gj_step further down, with the same pivoting rule).
// One work-group per matrix; thread i < Mp owns row i.  Columns are processed in
// panels of NB: during a panel every thread keeps its row of the panel in
// registers and publishes it to one of two LDS copies (alternating by column),
// so that one barrier per column suffices: the pivot row read from the copy of
// the previous column is never the copy being written.  The panel's combined
// transform (identity except in the NB pivot-row columns) then updates every
// other column as one rank-NB product on MFMA, with the next column tile's
// operands loaded before the current tile's products.  Rows are never
// physically swapped; the inverse is read out through the pivot permutation.
// A pivot whose magnitude is not above 1e-14 times the infinity norm of the
// matrix (or is NaN) marks the matrix singular.
// ---------------------------------------------------------------------------
// One step of a wave-wide arg-max: (v, i) against the (v, i) of the lane that the DPP control
// CTRL selects (rows outside ROWMASK keep their own); larger v wins, ties go to the smaller i.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void argmax_dpp_step(double& v, int& i) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, ROWMASK, 0xF, false);
  const double ov = __hiloint2double(ohi, olo);
  const bool take = (ov > v) | ((ov == v) & (oi < i));
  v = take ? ov : v;
  i = take ? oi : i;
}

// Wave-wide arg-max with DPP lane moves instead of LDS permutes (the pivot search sits on the
// column-to-column critical path of the elimination): swaps within quads, half-row and row
// mirrors, then row broadcasts leave the result in lane 63, which every lane reads.
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  argmax_dpp_step<0xB1, 0xF>(v, i);    // quad_perm [1,0,3,2]
  argmax_dpp_step<0x4E, 0xF>(v, i);    // quad_perm [2,3,0,1]
  argmax_dpp_step<0x141, 0xF>(v, i);   // row_half_mirror
  argmax_dpp_step<0x140, 0xF>(v, i);   // row_mirror
  argmax_dpp_step<0x142, 0xA>(v, i);   // row_bcast:15 into rows 1 and 3
  argmax_dpp_step<0x143, 0xC>(v, i);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  v = __hiloint2double(hi, lo);
  i = __builtin_amdgcn_readlane(i, 63);
}

// Arg-max of the waves' pivot candidates: lane u < 8 holds wave u's (magnitude, row), absent waves
// (-2, INT_MAX).  Three DPP steps within groups of eight lanes (rows are below 2^16, so row and wave
// pack into one key whose order is the row's); the pivot row r and its wave wr come back uniform.
__device__ __forceinline__ void slot_argmax(double v, int row, int& r, int& wr) {
  int key = (row == INT_MAX) ? INT_MAX : (row << 3) | (threadIdx.x & 7);
  argmax_dpp_step<0xB1, 0xF>(v, key);    // quad_perm [1,0,3,2]
  argmax_dpp_step<0x4E, 0xF>(v, key);    // quad_perm [2,3,0,1]
  argmax_dpp_step<0x141, 0xF>(v, key);   // row_half_mirror: lane i of eight meets lane 7 - i
  key = __builtin_amdgcn_readfirstlane(key);
  r = key >> 3;
  wr = key & 7;
}

template <int RT, int NT, int NB>
__global__ void __launch_bounds__(NT) k_gj(GJArgs g) {
  constexpr int CT = 4;           // 16 columns per update tile
  constexpr int KT = 4 * CT;
  extern __shared__ double sm[];
  const int Mp = g.Mp;
  double* Pb = sm;                         // [2][NB][Mp]: published panel rows
  double* Ys = Pb + NB * Mp;               // [NB][Mp]: pivot rows of W, all columns (after the
                                           // panel's last column, in the copy it no longer uses)
  double* wv = Pb + 2 * NB * Mp;           // [2][16] per-wave candidate values
  int* wi = (int*)(wv + 32);               // [2][16] per-wave candidate rows
  int* pivrow = wi + 32;                   // [Mp]
  int* invpiv = pivrow + Mp;               // [Mp]

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6, nw = nthr >> 6;
  const int q = blockIdx.x;
  if (q >= g.nmat) return;
  double* W = g.work + (g.work_off ? g.work_off[q] : q * g.wstride);
  const int rb = w * 16 * RT;
  const bool owner = tid < Mp;             // nthr >= Mp for every RT choice

  // infinity norm (row sums), one row per thread
  double rs = 0.0;
  if (owner) {
    // eight loads in flight per thread (Mp is a multiple of 16)
#pragma unroll 1
    for (int c0 = 0; c0 < Mp; c0 += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = W[tid + (int64_t)(c0 + u) * Mp];
#pragma unroll
      for (int u = 0; u < 8; ++u) rs += fabs(t[u]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
  if (L == 0) wv[w] = rs;
  __syncthreads();
  double norm = 0.0;
  for (int v = 0; v < nw; ++v) norm = fmax(norm, wv[v]);
  const double tol = 1e-14 * norm;
  __syncthreads();
  bool singular = false;
  bool used = false;

  for (int p0 = 0; p0 < Mp; p0 += NB) {
    double prv[NB];
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) prv[jj] = owner ? W[tid + (int64_t)(p0 + jj) * Mp] : 0.0;
    if (owner) {
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) Pb[jj * Mp + tid] = prv[jj];
    }
    // unrolled so that the panel row stays in registers (faster even where the 512-thread
    // register budget makes it spill)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int b = j & 1;
      const double* cur = Pb + b * NB * Mp;        // rows after column j-1
      double* nxt = Pb + (b ^ 1) * NB * Mp;        // rows after column j
      // pivot search on the own row
      double bv = -1.0;
      int bi = INT_MAX;
      // prv[j] by selection, so that a rolled loop would not place the array in scratch memory
      double pj = 0.0;
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) pj = (jj == j) ? prv[jj] : pj;
      if (owner && !used) {
        const double v = fabs(pj);
        bv = (v == v) ? v : DBL_MAX;   // NaN ranks first so that it is reported
        bi = tid;
      }
      wave_argmax(bv, bi);
      if (L == 0) { wv[16 * b + w] = bv; wi[16 * b + w] = bi; }
      __syncthreads();
      double b2 = wv[16 * b];
      int r = wi[16 * b];
      for (int v = 1; v < nw; ++v) {
        const double ov = wv[16 * b + v];
        const int oi = wi[16 * b + v];
        if (ov > b2 || (ov == b2 && oi < r)) { b2 = ov; r = oi; }
      }
      if (tid == 0) pivrow[p0 + j] = r;
      const double pv = cur[j * Mp + r];
      if (!(fabs(pv) > tol)) singular = true;
      const double ipv = 1.0 / pv;
      if (owner) {
        if (tid == r) {
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) prv[jj] = (jj == j) ? ipv : prv[jj] * ipv;
          used = true;
        } else {
          const double fi = pj * ipv;   // row -= pj * (pivot row / pivot); column j <- -pj / pivot
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) prv[jj] = (jj == j) ? -fi : prv[jj] - fi * cur[jj * Mp + r];
        }
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) nxt[jj * Mp + tid] = prv[jj];
      }
    }
    // the last column (NB - 1, odd) published into copy 0
    __syncthreads();
    const double* Pn = Pb;
    // pivot rows of W: four loads in flight per thread (clamped in-range indices, guarded stores)
#pragma unroll 1
    for (int e0 = tid; e0 < NB * Mp; e0 += 4 * nthr) {
      double t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * nthr, NB * Mp - 1);
        t[u] = W[pivrow[p0 + e / Mp] + (int64_t)(e % Mp) * Mp];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * nthr;
        if (e < NB * Mp) Ys[e] = t[u];
      }
    }
    __syncthreads();
    // rank-NB update of all other columns: W[:, c] += (Pn - E_R) * W[R, c]
    double av[NB / 4][RT];
#pragma unroll
    for (int kk = 0; kk < NB / 4; ++kk) {
      const int k = 4 * kk + (L >> 4);
      const int pr = pivrow[p0 + k];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + (L & 15);
        av[kk][t] = Pn[k * Mp + row] - (row == pr ? 1.0 : 0.0);
      }
    }
    const int ntile = Mp / KT;
    auto load_tile = [&](double (&acc)[RT][CT], int tile) {
      const int c0 = tile * KT;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + out_row(L);
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = W[row + (int64_t)(c0 + out_col(L) * CT + c) * Mp];
      }
    };
    auto update_tile = [&](double (&acc)[RT][CT], int tile) {
      const int c0 = tile * KT;
#pragma unroll
      for (int kk = 0; kk < NB / 4; ++kk) {
        const int k = 4 * kk + (L >> 4);
        const double* bp = &Ys[k * Mp + c0 + (L & 3) * CT];
        double bb[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) bb[c] = bp[c];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[t][c] = mfma4(av[kk][t], bb[c], acc[t][c]);
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + out_row(L);
#pragma unroll
        for (int c = 0; c < CT; ++c) W[row + (int64_t)(c0 + out_col(L) * CT + c) * Mp] = acc[t][c];
      }
    };
    // the column tiles other than the panel's own (NB a multiple of KT), in order; four register buffers
    // rotate so that every tile's operands are requested three tiles ahead of their use
    constexpr int PT = NB / KT;               // tiles covered by the panel
    const int ptile = p0 / KT;
    const int cnt = ntile - PT;
    auto tile_of = [&](int n) { return n < ptile ? n : n + PT; };
    double tb0[RT][CT], tb1[RT][CT], tb2[RT][CT], tb3[RT][CT];
    if (cnt > 0) load_tile(tb0, tile_of(0));
    if (cnt > 1) load_tile(tb1, tile_of(1));
    if (cnt > 2) load_tile(tb2, tile_of(2));
    for (int n = 0; n < cnt; n += 4) {
      if (n + 3 < cnt) load_tile(tb3, tile_of(n + 3));
      update_tile(tb0, tile_of(n));
      if (n + 1 >= cnt) break;
      if (n + 4 < cnt) load_tile(tb0, tile_of(n + 4));
      update_tile(tb1, tile_of(n + 1));
      if (n + 2 >= cnt) break;
      if (n + 5 < cnt) load_tile(tb1, tile_of(n + 5));
      update_tile(tb2, tile_of(n + 2));
      if (n + 3 >= cnt) break;
      if (n + 6 < cnt) load_tile(tb2, tile_of(n + 6));
      update_tile(tb3, tile_of(n + 3));
    }
    for (int e = tid; e < NB * Mp; e += nthr) {
      const int i = e % Mp, jj = e / Mp;
      W[i + (int64_t)(p0 + jj) * Mp] = Pn[jj * Mp + i];
    }
    __syncthreads();
  }
  if (tid == 0 && singular) atomicMin(g.bad, g.tag[q]);
  // inverse: Dinv[c][pivrow[c']] = S[pivrow[c]][c']
  for (int c = tid; c < Mp; c += nthr) invpiv[pivrow[c]] = c;
  __syncthreads();
  double* out = g.out + g.out_off[q];
  double* al = g.alpha ? g.alpha + g.out_off[q] : nullptr;
  const double* bd = g.alpha ? g.bdiag + g.bd_off[q] : nullptr;
  // eight loads in flight per thread (clamped in-range indices, guarded stores)
  const int MM = Mp * Mp;
#pragma unroll 1
  for (int e0 = tid; e0 < MM; e0 += 8 * nthr) {
    double t[8], bb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * nthr, MM - 1);
      t[u] = W[pivrow[e % Mp] + (int64_t)invpiv[e / Mp] * Mp];
      bb[u] = al ? bd[e / Mp] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nthr;
      if (e < MM) {
        out[e] = t[u];
        if (al) al[e] = t[u] * bb[u];
      }
    }
  }
}

// Pivot candidates of the one-row-per-thread panel as one 64-bit key: the magnitude's bit pattern
// (monotone in the magnitude for non-negative doubles) with its low 9 bits replaced by 511 - row, so a
// single unsigned maximum picks the largest magnitude and, among magnitudes that agree in all but
// their last 9 bits (a relative difference below 2^-43), the smallest row.  Rows already used as
// pivots get key 0; NaN ranks as the largest finite value so that it is chosen and reported.  Rows
// are below 512.  Key 0 decodes to row 511, which it is only when every other row is used.
__device__ __forceinline__ uint64_t pivot_key(double v, bool used, int row) {
  const double a = fabs(v);
  const uint64_t bits = (uint64_t)__double_as_longlong((a == a) ? a : DBL_MAX);
  return used ? 0ull : ((bits & ~511ull) | (uint64_t)(511 - row));
}
__device__ __forceinline__ int pivot_key_row(uint64_t k) { return 511 - (int)(k & 511); }

// One step of a wave-wide key maximum against the key of the lane that the DPP control CTRL
// selects (rows outside ROWMASK keep their own).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void keymax_dpp_step(uint64_t& k) {
  const int lo = (int)(uint32_t)k, hi = (int)(uint32_t)(k >> 32);
  int olo, ohi;
  if constexpr (ROWMASK == 0xF && CTRL < 0x142) {   // quad permutes and row mirrors: every lane has a source
    olo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    ohi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  } else {                                          // row broadcasts: lanes outside ROWMASK keep their own
    olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
    ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  }
  const uint64_t o = ((uint64_t)(uint32_t)ohi << 32) | (uint32_t)olo;
  k = (o > k) ? o : k;
}

// One column of gj_panel: v holds the row rotated so that v[0] is column j; the updated row is written
// one place down (column j's new entry at the end).
template <int NB>
__device__ __forceinline__ void gj_column(double (&v)[NB], int j, bool& used, double& sr, double& pm, double* cand,
                                          double* cv, int* prow, int nw) {
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6;
  const int slot = j & 1;
  const double vj = v[0];
  double rcp = 1.0 / vj;                  // used only if this lane's row wins
  asm volatile("" : "+v"(rcp));
  uint64_t key = pivot_key(vj, used, tid);
  keymax_dpp_step<0xB1, 0xF>(key);    // quad_perm [1,0,3,2]
  keymax_dpp_step<0x4E, 0xF>(key);    // quad_perm [2,3,0,1]
  keymax_dpp_step<0x141, 0xF>(key);   // row_half_mirror
  keymax_dpp_step<0x140, 0xF>(key);   // row_mirror
  keymax_dpp_step<0x142, 0xA>(key);   // row_bcast:15 into rows 1 and 3
  keymax_dpp_step<0x143, 0xC>(key);   // row_bcast:31 into rows 2 and 3
  const uint32_t klo = __builtin_amdgcn_readlane((int)(uint32_t)key, 63);
  const uint32_t khi = __builtin_amdgcn_readlane((int)(uint32_t)(key >> 32), 63);
  const uint64_t wkey = ((uint64_t)khi << 32) | klo;
  if (tid == pivot_key_row(wkey)) {
    int co = (slot * 8 + w) * NB;
    asm volatile("" : "+v"(co));   // one base register, the entries at immediate offsets
    double* cp = cand + co;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) cp[jj] = v[jj];
    cv[32 + slot * 8 + w] = rcp;
  }
  if (L == 0) cv[slot * 8 + w] = __longlong_as_double((long long)wkey);
  __syncthreads();
  uint64_t bk = (L < nw) ? (uint64_t)__double_as_longlong(cv[slot * 8 + (L & 7)]) : 0ull;
  keymax_dpp_step<0xB1, 0xF>(bk);    // quad_perm [1,0,3,2]
  keymax_dpp_step<0x4E, 0xF>(bk);    // quad_perm [2,3,0,1]
  keymax_dpp_step<0x141, 0xF>(bk);   // row_half_mirror: lane i of eight meets lane 7 - i
  const int r = __builtin_amdgcn_readfirstlane(pivot_key_row(bk));
  const int wr = r >> 6;
  int po = (slot * 8 + wr) * NB;
  asm volatile("" : "+v"(po));     // as above
  const double* pr = cand + po;
  const double ipv = cv[32 + slot * 8 + wr];
  const bool piv = (tid == r);
  const double f = piv ? 0.0 : vj * ipv;   // v <- v - v_j * (pivot row / pivot), column j <- -v_j / pivot
  double prv[NB];
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) prv[jj] = pr[jj];
  const double apv = fabs(prv[0]);
  pm = (pm != pm) ? pm : ((apv != apv) ? apv : fmin(pm, apv));
#pragma unroll
  for (int jj = 0; jj + 1 < NB; ++jj) v[jj] = v[jj + 1] - f * prv[jj + 1];
  v[NB - 1] = piv ? 1.0 : -f;
  sr = piv ? ipv : sr;
  used = used | piv;
  if (tid == 0) prow[j] = r;
}

// Gauss-Jordan elimination of one panel of NB columns, one row per thread: v[j] is the thread's entry
// of panel column j, rows with `used` set were pivots of earlier panels.  Per column every wave finds
// its best candidate with a DPP maximum of pivot keys (pivot_key), and the winning lane of each wave
// publishes that row and its reciprocal pivot, the wave's key next to them; after one work-group
// barrier every thread takes the largest of the waves' keys (a DPP maximum over eight lanes) and
// reads the pivot row from the slot of the wave that holds that row.  Slots alternate between two
// copies, so one barrier per column suffices.
//   The loop stays rolled without indexing registers at run time: the row is kept rotated so that v[0]
// is always the current column, and the update writes each entry one place down (column j's new entry
// goes to the end), so after NB columns the order is the original one again.  The pivot row is not
// scaled when it is chosen: later eliminations are linear in each row, so its entries are multiplied
// by the reciprocal pivot once after the panel (its column-j entry is kept as 1 until then), and every
// row takes the same single fused multiply-add per entry and column.  Every lane divides by its own
// entry before the key maximum, so that the winning lane's reciprocal is ready when it publishes its
// row.  The pivot row of column j goes to prow[j] (written by thread 0).  Returns the smallest pivot
// magnitude of the panel (NaN if a pivot was NaN; the caller tests it against the tolerance).  cand
// holds [2][8][NB] rows, cv [2][8] keys and, from cv[32], [2][8] reciprocals.
template <int NB>
__device__ __forceinline__ double gj_panel(double (&v)[NB], bool& used, double* cand, double* cv, int* prow,
                                           int nw) {
  double sr = 1.0;   // deferred scale of this thread's row (the reciprocal pivot if it was chosen)
  double pm = INFINITY;   // smallest pivot magnitude of the panel; NaN once a pivot is NaN
#pragma unroll 1
  for (int j = 0; j < NB; ++j) gj_column<NB>(v, j, used, sr, pm, cand, cv, prow, nw);
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) v[jj] *= sr;
  return pm;
}

// Gauss-Jordan inversion with one launch per panel, for block sizes that are multiples of 64 from 128:
// the matrix's columns form Mp / NB tiles of one panel's width, and launch k has one work-group per
// (matrix, tile).  Eliminating a set S of columns with pivot rows R is one block pivot: every other
// column c becomes c + (Z - E_R) c_R, where Z holds the columns of S after their elimination (in place,
// so Z is what the previous launch stored in panel k's columns) and c_R the entries of c in rows R
// before it.  So in launch k every tile other than panel k applies panel k's transform to its own
// columns (a rank-NB product on MFMA), and the matrix's lead work-group updates tile k + 1 the same
// way and then eliminates that panel (gj_panel, one row per thread).  Launch -1 eliminates panel 0
// while the other tiles store their partial row sums of the matrix (for the infinity norm); every
// panel keeps the smallest pivot magnitude so far in g.pmin.  In the last launch every tile writes its
// final columns through the pivot permutation into the inverse (inverse[r][piv[j]] = S[piv[r]][j] for
// the eliminated matrix S; alpha = inverse * diag(bdiag) when requested), and the lead work-group
// writes the last panel and marks the matrix singular when a pivot was not above 1e-14 times the
// infinity norm (or NaN).  A matrix thus has Mp / NB work-groups in flight instead of one, and the
// update of a panel no longer waits behind the elimination of the next.  (An earlier form inverted
// each matrix in one work-group and one launch; at block size 512 a matrix then took 6.4 ms, most of
// it the passes of one work-group's update over the 2 MB matrix.)
template <int NB, int NT>
__global__ void __launch_bounds__(NT) k_gj_step(GJArgs g, int k) {
  constexpr int RT = 4;                    // 64 rows per wave
  constexpr int CTN = NB / 4;              // 4-column output tiles per tile
  extern __shared__ double sm[];
  const int Mp = g.Mp;                     // a multiple of 64, blockDim.x == Mp
  double* Ts = sm;                         // [NB][Mp]: a tile's columns (panel or read-out)
  double* Bs = Ts + NB * Mp;               // [NB][NB]: rows R_k of the tile's columns
  double* cand = Bs + NB * NB;             // [2][8][NB]: candidate pivot rows of the waves
  double* cv = cand + 2 * 8 * NB;          // [2][8]: their pivot keys; [16 .. 23]: row-sum maxima;
                                           // [32 .. 47]: their reciprocal pivots
  int* pl = (int*)(cv + 48);               // [NB]: pivot rows of the panel eliminated here
  int* rk = pl + NB;                       // [NB]: pivot rows of panel k
  int* ri = rk + NB;                       // [Mp]: rows used as pivots (panel), pivot rows (read-out)
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const int ntile = Mp / NB;
  const bool last = (k == ntile - 1);
  // Work-groups [0, nmat8) are the lead work-groups of matrix blockIdx.x, dispatched before any
  // update; update work-group t = blockIdx.x - nmat8 takes tile t/8 % ntile of matrix
  // t % 8 + 8 (t/8 / ntile): work-groups go to the eight XCDs in turn, so every work-group of a matrix
  // runs on the XCD of its lead work-group and reads panel k from that XCD's L2.
  const int nmat8 = (g.nmat + 7) & ~7;
  int q, c;
  const bool lead = (int)blockIdx.x < nmat8;
  if (lead) {
    q = blockIdx.x;
    c = last ? k : k + 1;
    if (q >= g.nmat) return;
  } else {
    const int t = blockIdx.x - nmat8, i = t >> 3;
    q = (t & 7) + 8 * (i / ntile);
    c = i % ntile;
    if (q >= g.nmat || c == k || c == k + 1) return;
  }
  double* W = g.work + (g.work_off ? g.work_off[q] : q * g.wstride);
  int* piv = g.piv + (int64_t)q * Mp;
  double* part = g.part + (int64_t)q * ntile * Mp;   // [ntile][Mp]: partial row sums of |matrix|
  const int c0 = c * NB;
  const int rb = w * 16 * RT;

  if (k < 0 && !lead) {   // the tile's share of the row sums of the original matrix
    double rs = 0.0;
#pragma unroll
    for (int j0 = 0; j0 < NB; j0 += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = W[tid + (int64_t)(c0 + j0 + u) * Mp];
#pragma unroll
      for (int u = 0; u < 8; ++u) rs += fabs(t[u]);
    }
    part[(int64_t)c * Mp + tid] = rs;
    return;
  }

  if (k >= 0 && !(last && lead)) {
    if (tid < NB) rk[tid] = piv[k * NB + tid];
    __syncthreads();
    for (int e = tid; e < NB * NB; e += blockDim.x) {   // a row of R_k per column: one column's rows per pass
      const int j = e / NB, kk = e - j * NB;
      Bs[kk * NB + j] = W[rk[kk] + (int64_t)(c0 + j) * Mp];
    }
    double a[NB / 4][RT];                  // (Z - E_R) rows of this wave, Z = panel k's columns
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
      const int kc = 4 * k4 + (L >> 4);
      const int prw = rk[kc];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + (L & 15);
        a[k4][t] = W[row + (int64_t)(k * NB + kc) * Mp] - (row == prw ? 1.0 : 0.0);
      }
    }
    double acc[RT][CTN];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int ct = 0; ct < CTN; ++ct)
        acc[t][ct] = W[rb + 16 * t + out_row(L) + (int64_t)(c0 + 4 * ct + out_col(L)) * Mp];
    __syncthreads();   // Bs complete; every read of rows R_k of the tile precedes the stores below
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
      const double* bp = Bs + (4 * k4 + (L >> 4)) * NB + (L & 3);
      double b[CTN];
#pragma unroll
      for (int ct = 0; ct < CTN; ++ct) b[ct] = bp[4 * ct];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int ct = 0; ct < CTN; ++ct) acc[t][ct] = mfma4(a[k4][t], b[ct], acc[t][ct]);
    }
    if (!lead && !last) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int ct = 0; ct < CTN; ++ct)
          W[rb + 16 * t + out_row(L) + (int64_t)(c0 + 4 * ct + out_col(L)) * Mp] = acc[t][ct];
      return;
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int ct = 0; ct < CTN; ++ct) Ts[(4 * ct + out_col(L)) * Mp + rb + 16 * t + out_row(L)] = acc[t][ct];
  }

  if (last) {
    if (lead) {   // the last panel (final since the previous launch), and the singularity test
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) Ts[jj * Mp + tid] = W[tid + (int64_t)(c0 + jj) * Mp];
      double rs = 0.0;
      for (int cc = 0; cc < ntile; ++cc) rs += part[(int64_t)cc * Mp + tid];
      for (int off = 32; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
      if (L == 0) cv[16 + w] = rs;
    }
    ri[tid] = piv[tid];
    __syncthreads();   // Ts, the pivot rows and the row-sum maxima complete
    if (lead && tid == 0) {
      double norm = 0.0;
      for (int u = 0; u < nw; ++u) norm = fmax(norm, cv[16 + u]);
      if (!(g.pmin[q] > 1e-14 * norm)) atomicMin(g.bad, g.tag[q]);
    }
    double* out = g.out + g.out_off[q];
    double* al = g.alpha ? g.alpha + g.out_off[q] : nullptr;
    const double* bd = g.alpha ? g.bdiag + g.bd_off[q] : nullptr;
    const int prow_t = ri[tid];
#pragma unroll 8
    for (int jj = 0; jj < NB; ++jj) {
      const int oc = ri[c0 + jj];
      const double v = Ts[jj * Mp + prow_t];
      out[tid + (int64_t)oc * Mp] = v;
      if (al) al[tid + (int64_t)oc * Mp] = v * bd[oc];
    }
    return;
  }

  // the lead work-group of launch k < ntile - 1: rows already used as pivots, then the elimination
  ri[tid] = 0;
  __syncthreads();   // also orders the Ts stores above before the reads below
  for (int i = tid; i < c0; i += blockDim.x) ri[piv[i]] = 1;
  __syncthreads();
  bool used = ri[tid] != 0;
  double v[NB];
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) v[jj] = (k < 0) ? W[tid + (int64_t)jj * Mp] : Ts[jj * Mp + tid];
  if (k < 0) {   // tile 0's share of the row sums, from the original values
    double rs = 0.0;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) rs += fabs(v[jj]);
    part[tid] = rs;
  }
  const double pm = gj_panel<NB>(v, used, cand, cv, pl, nw);
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) W[tid + (int64_t)(c0 + jj) * Mp] = v[jj];
  __syncthreads();
  if (tid < NB) piv[c0 + tid] = pl[tid];
  if (tid == 0) {
    const double o = (k < 0) ? INFINITY : g.pmin[q];
    g.pmin[q] = (o != o) ? o : ((pm != pm) ? pm : fmin(o, pm));
  }
}

template <int NB, int NT>
static hipError_t launch_gj_split(const GJArgs& g, hipStream_t st) {
  const int Mp = g.Mp, ntile = Mp / NB;
  const size_t lds = (size_t)(NB * Mp + NB * NB + 2 * 8 * NB + 48) * sizeof(double) +
                     (size_t)(2 * NB + Mp) * sizeof(int);
  hipError_t e = hipFuncSetAttribute((const void*)k_gj_step<NB, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int nmat8 = grid_pad8(g.nmat);
  for (int k = -1; k < ntile; ++k)
    hipLaunchKernelGGL((k_gj_step<NB, NT>), dim3(nmat8 * (1 + ntile)), dim3(Mp), lds, st, g, k);
  return hipGetLastError();
}

// Block pivot of 32 columns onto 32 others, by a work-group of Mp threads (64 rows per wave): the
// columns from tc become c + (Z - E_R) c_R, with Z the 32 columns from zc after their elimination with
// pivot rows R (R[0 .. 32), in LDS) and c_R the rows R of c before it; a rank-32 product on MFMA with
// c_R staged in Hs ([32][32]).  Every thread's stores of Z and R must be complete before the call; at
// its return the new columns are visible to the work-group and Hs is free.
__device__ __forceinline__ void gj_half_apply(double* W, int Mp, int zc, const int* R, int tc, double* Hs) {
  constexpr int RT = 4, KW = 32, CT = 8;
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6;
  const int rb = w * 16 * RT;
  for (int e = tid; e < KW * 32; e += blockDim.x) {
    const int j = e / KW, kk = e - j * KW;
    Hs[kk * 32 + j] = W[R[kk] + (int64_t)(tc + j) * Mp];
  }
  double a[KW / 4][RT];
#pragma unroll
  for (int k4 = 0; k4 < KW / 4; ++k4) {
    const int kc = 4 * k4 + (L >> 4);
    const int prw = R[kc];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + (L & 15);
      a[k4][t] = W[row + (int64_t)(zc + kc) * Mp] - (row == prw ? 1.0 : 0.0);
    }
  }
  double acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[t][ct] = W[rb + 16 * t + out_row(L) + (int64_t)(tc + 4 * ct + out_col(L)) * Mp];
  __syncthreads();   // Hs complete; every read of rows R of the target columns precedes the stores below
#pragma unroll
  for (int k4 = 0; k4 < KW / 4; ++k4) {
    const double* bp = Hs + (4 * k4 + (L >> 4)) * 32 + (L & 3);
    double b[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) b[ct] = bp[4 * ct];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[t][ct] = mfma4(a[k4][t], b[ct], acc[t][ct]);
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) W[rb + 16 * t + out_row(L) + (int64_t)(tc + 4 * ct + out_col(L)) * Mp] = acc[t][ct];
  __syncthreads();
}

// The per-panel inversion with 64-column panels and tiles, for block sizes from 384 (multiples of 64)
// when a launch holds many matrices: there the update passes over the matrices bound the time, and
// rank-64 products halve them (Mp / 64 + 1 launches per inversion).  The lead work-group has the role
// it has in k_gj_step; in the panel launches the other tiles of a matrix are updated in turn by one
// work-group (the leads hold half of the compute units for their panels, so more work-groups would
// only queue), in the prologue and the last launch by one work-group per tile, each tile
// in four quarters of 16 columns with the rank-64 operand loaded once into registers; the lead
// work-group's updated panel goes through the matrix in global memory (a 64-column
// tile of 512 rows would take 256 KB of LDS), the last launch's other tiles write the inverse straight
// from the products' registers, and the lead eliminates its panel as two 32-column halves joined by
// gj_half_apply.
template <int NT>
__global__ void __launch_bounds__(NT) k_gj_step64(GJArgs g, int k) {
  constexpr int NB = 64, RT = 4, CTN = 4;  // CTN: 4-column output tiles of a 16-column quarter
  extern __shared__ double sm[];
  const int Mp = g.Mp;                     // a multiple of 64, blockDim.x == Mp
  double* Bs = sm;                         // [NB][NB]: rows R_k of the tile's columns
  double* cand = Bs + NB * NB;             // [2][8][NB]: candidate pivot rows of the waves
  double* cv = cand + 2 * 8 * NB;          // [2][8]: their pivot keys; [16 .. 23]: row-sum maxima;
                                           // [32 .. 47]: their reciprocal pivots
  int* pl = (int*)(cv + 48);               // [NB]: pivot rows of the panel eliminated here
  int* rk = pl + NB;                       // [NB]: pivot rows of panel k
  int* ri = rk + NB;                       // [Mp]: rows used as pivots (panel), pivot rows (read-out)
  const int tid = threadIdx.x, L = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const int ntile = Mp / NB;
  const bool last = (k == ntile - 1);
  // Work-groups [0, nmat8) are the lead work-groups of matrix blockIdx.x (dispatched first).  In the
  // panel launches work-group nmat8 + q updates every other tile of matrix q in turn, so the rank-64
  // operand is loaded once per matrix, and a launch over 128 matrices holds one work-group per compute
  // unit; in the prologue and the last launch, where the leads finish early, work-group nmat8 + t
  // takes tile t/8 % ntile of matrix t % 8 + 8 (t/8 / ntile) alone.  All work-groups of a matrix run
  // on the XCD of its lead (nmat8 is a multiple of 8).
  const int nmat8 = (g.nmat + 7) & ~7;
  const bool lead = (int)blockIdx.x < nmat8;
  const bool per_tile = (k < 0) || (k == ntile - 1);
  int q, tbeg = 0, tend = ntile;           // the update work-group's tiles [tbeg, tend)
  if (lead) {
    q = blockIdx.x;
  } else if (per_tile) {
    const int t = blockIdx.x - nmat8, i = t >> 3;
    q = (t & 7) + 8 * (i / ntile);
    tbeg = i % ntile;
    tend = tbeg + 1;
    if (tbeg == k || (k < 0 && tbeg == 0)) return;   // the lead's tile
  } else {
    q = blockIdx.x - nmat8;
  }
  if (q >= g.nmat) return;
  const int c = last ? k : k + 1;          // the lead's tile
  double* W = g.work + (g.work_off ? g.work_off[q] : q * g.wstride);
  int* piv = g.piv + (int64_t)q * Mp;
  double* part = g.part + (int64_t)q * ntile * Mp;   // [ntile][Mp]: partial row sums of |matrix|
  const int c0 = c * NB;
  const int rb = w * 16 * RT;

  if (k < 0 && !lead) {   // the other tiles' shares of the row sums of the original matrix
#pragma unroll 1
    for (int ct = max(tbeg, 1); ct < tend; ++ct) {
      double rs = 0.0;
#pragma unroll
      for (int j0 = 0; j0 < NB; j0 += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = W[tid + (int64_t)(ct * NB + j0 + u) * Mp];
#pragma unroll
        for (int u = 0; u < 8; ++u) rs += fabs(t[u]);
      }
      part[(int64_t)ct * Mp + tid] = rs;
    }
    return;
  }

  if (k >= 0 && !(last && lead)) {
    // the last launch writes the tiles' final columns into the inverse from the products' registers:
    // S[i][j] goes to inverse[invp[i]][piv[j]], invp the inverse of the pivot-row permutation
    int* invp = (int*)cand;                // [Mp] (the candidate rows are not used by these work-groups)
    if (tid < NB) rk[tid] = piv[k * NB + tid];
    if (last) {
      const int pr = piv[tid];
      ri[tid] = pr;
      invp[pr] = tid;
    }
    __syncthreads();
    double a[NB / 4][RT];                  // (Z - E_R) rows of this wave, Z = panel k's columns
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
      const int kc = 4 * k4 + (L >> 4);
      const int prw = rk[kc];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + (L & 15);
        a[k4][t] = W[row + (int64_t)(k * NB + kc) * Mp] - (row == prw ? 1.0 : 0.0);
      }
    }
    // the lead work-group updates its tile k + 1; the others their tiles but k and k + 1
#pragma unroll 1
    for (int tc = lead ? k + 1 : tbeg; tc < (lead ? k + 2 : tend); ++tc) {
      if (!lead && (tc == k || tc == k + 1)) continue;
      const int t0 = tc * NB;
      __syncthreads();   // the previous tile's reads of Bs are done
      for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int j = e / NB, kk = e - j * NB;
        Bs[kk * NB + j] = W[rk[kk] + (int64_t)(t0 + j) * Mp];
      }
      __syncthreads();   // Bs complete; every read of rows R_k of the tile precedes the stores below
#pragma unroll 1
      for (int h = 0; h < 4; ++h) {
        const int ch = t0 + 16 * h;
        double acc[RT][CTN];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int ct = 0; ct < CTN; ++ct)
            acc[t][ct] = W[rb + 16 * t + out_row(L) + (int64_t)(ch + 4 * ct + out_col(L)) * Mp];
#pragma unroll
        for (int k4 = 0; k4 < NB / 4; ++k4) {
          const double* bp = Bs + (4 * k4 + (L >> 4)) * NB + 16 * h + (L & 3);
          double b[CTN];
#pragma unroll
          for (int ct = 0; ct < CTN; ++ct) b[ct] = bp[4 * ct];
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int ct = 0; ct < CTN; ++ct) acc[t][ct] = mfma4(a[k4][t], b[ct], acc[t][ct]);
        }
        if (last) {
          double* out = g.out + g.out_off[q];
          double* al = g.alpha ? g.alpha + g.out_off[q] : nullptr;
          const double* bd = g.alpha ? g.bdiag + g.bd_off[q] : nullptr;
#pragma unroll
          for (int ct = 0; ct < CTN; ++ct) {
            const int oc = ri[ch + 4 * ct + out_col(L)];
            const double bo = al ? bd[oc] : 0.0;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
              const int64_t o = invp[rb + 16 * t + out_row(L)] + (int64_t)oc * Mp;
              out[o] = acc[t][ct];
              if (al) al[o] = acc[t][ct] * bo;
            }
          }
        } else {
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int ct = 0; ct < CTN; ++ct)
              W[rb + 16 * t + out_row(L) + (int64_t)(ch + 4 * ct + out_col(L)) * Mp] = acc[t][ct];
        }
      }
    }
    if (!lead) return;
  }

  if (last) {   // the lead work-group: the last panel (final since the previous launch), the singularity test
    {
      double rs = 0.0;
      for (int cc = 0; cc < ntile; ++cc) rs += part[(int64_t)cc * Mp + tid];
      for (int off = 32; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
      if (L == 0) cv[16 + w] = rs;
    }
    ri[tid] = piv[tid];
    __syncthreads();   // the pivot rows and the row-sum maxima complete
    if (tid == 0) {
      double norm = 0.0;
      for (int u = 0; u < nw; ++u) norm = fmax(norm, cv[16 + u]);
      if (!(g.pmin[q] > 1e-14 * norm)) atomicMin(g.bad, g.tag[q]);
    }
    double* out = g.out + g.out_off[q];
    double* al = g.alpha ? g.alpha + g.out_off[q] : nullptr;
    const double* bd = g.alpha ? g.bdiag + g.bd_off[q] : nullptr;
    const int prow_t = ri[tid];
#pragma unroll 8
    for (int jj = 0; jj < NB; ++jj) {
      const int oc = ri[c0 + jj];
      const double v = W[prow_t + (int64_t)(c0 + jj) * Mp];
      out[tid + (int64_t)oc * Mp] = v;
      if (al) al[tid + (int64_t)oc * Mp] = v * bd[oc];
    }
    return;
  }

  // the lead work-group of launch k < ntile - 1 eliminates the 64-column panel as two halves A and B
  // of 32 columns (one row per thread, gj_panel): A; B after A's transform; then A's columns take B's
  // transform, which leaves the block pivot of all 64 columns (pivot rows R_A, R_B in pl)
  ri[tid] = 0;
  __syncthreads();   // also orders the updated panel's stores above before the reads below
  for (int i = tid; i < c0; i += blockDim.x) ri[piv[i]] = 1;
  __syncthreads();
  bool used = ri[tid] != 0;
  double v[32];
  if (k < 0) {   // tile 0's share of the row sums, from the original values
    double rs = 0.0;
#pragma unroll 8
    for (int jj = 0; jj < NB; ++jj) rs += fabs(W[tid + (int64_t)(c0 + jj) * Mp]);
    part[tid] = rs;
  }
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) v[jj] = W[tid + (int64_t)(c0 + jj) * Mp];
  __builtin_amdgcn_s_waitcnt(0);   // the row is in registers before the column loop (no waits inside it)
  const double pma = gj_panel<32>(v, used, cand, cv, pl, nw);
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) W[tid + (int64_t)(c0 + jj) * Mp] = v[jj];
  __syncthreads();   // Z_A and R_A complete
  gj_half_apply(W, Mp, c0, pl, c0 + 32, Bs);
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) v[jj] = W[tid + (int64_t)(c0 + 32 + jj) * Mp];
  __builtin_amdgcn_s_waitcnt(0);
  const double pmb = gj_panel<32>(v, used, cand, cv, pl + 32, nw);
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) W[tid + (int64_t)(c0 + 32 + jj) * Mp] = v[jj];
  __syncthreads();   // Z_B and R_B complete
  gj_half_apply(W, Mp, c0 + 32, pl + 32, c0, Bs);
  if (tid < NB) piv[c0 + tid] = pl[tid];
  if (tid == 0) {
    const double o = (k < 0) ? INFINITY : g.pmin[q];
    const double pm = (pma != pma) ? pma : ((pmb != pmb) ? pmb : fmin(pma, pmb));
    g.pmin[q] = (o != o) ? o : ((pm != pm) ? pm : fmin(o, pm));
  }
}

template <int NT>
static hipError_t launch_gj_split64(const GJArgs& g, hipStream_t st) {
  constexpr int NB = 64;
  const int Mp = g.Mp, ntile = Mp / NB;
  const size_t lds = (size_t)(NB * NB + 2 * 8 * NB + 48) * sizeof(double) + (size_t)(2 * NB + Mp) * sizeof(int);
  hipError_t e = hipFuncSetAttribute((const void*)k_gj_step64<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int nmat8 = grid_pad8(g.nmat);
  for (int k = -1; k < ntile; ++k) {   // per-tile work-groups in the prologue and the last launch
    const int nwg = (k < 0 || k == ntile - 1) ? nmat8 * (1 + ntile) : 2 * nmat8;
    hipLaunchKernelGGL((k_gj_step64<NT>), dim3(nwg), dim3(Mp), lds, st, g, k);
  }
  return hipGetLastError();
}

template <int RT, int NT, int NB>
static hipError_t launch_gj_cfg(const GJArgs& g, int nthr, hipStream_t st) {
  const size_t lds = (size_t)(2 * NB * g.Mp + 32) * sizeof(double) + (size_t)(32 + 2 * g.Mp) * sizeof(int);
  hipError_t e =
      hipFuncSetAttribute((const void*)k_gj<RT, NT, NB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gj<RT, NT, NB>), dim3(g.nmat), dim3(nthr), lds, st, g);
  return hipGetLastError();
}

// work-groups of at most 256 threads get the larger register budget of that bound
template <int RT>
static hipError_t launch_gj_rt(const GJArgs& g, hipStream_t st) {
  const int nthr = g.Mp / (16 * RT) * 64;
  // panels of 32 columns halve the passes of the update over the matrix where the block size
  // divides into them and the two LDS copies fit; 16 otherwise (block sizes up to 256 here)
  if (g.Mp % 32 == 0) {
    if (nthr <= 256) return launch_gj_cfg<RT, 256, 32>(g, nthr, st);
    return launch_gj_cfg<RT, 512, 32>(g, nthr, st);
  }
  if (nthr <= 256) return launch_gj_cfg<RT, 256, 16>(g, nthr, st);
  return launch_gj_cfg<RT, 512, 16>(g, nthr, st);
}

hipError_t launch_gj(const GJArgs& g, hipStream_t st) {
  if (g.nmat == 0) return hipSuccess;
  // block sizes that are multiples of 64 from 128 (every padded size above 256 is one): one launch
  // per 32-column panel, with the caller's scratch for pivot rows, smallest pivots and row sums
  if (g.Mp % 64 == 0 && g.Mp >= 128) {
    if (!g.piv || !g.pmin || !g.part) return hipErrorInvalidValue;
    // many matrices at block sizes from 384: the update passes bound a launch, 64-column panels
    if (g.Mp >= 384 && g.nmat >= 32) return launch_gj_split64<512>(g, st);
    return g.Mp <= 256 ? launch_gj_split<32, 256>(g, st) : launch_gj_split<32, 512>(g, st);
  }
  if (g.Mp > 256) return hipErrorInvalidValue;
  switch (choose_rt(g.Mp)) {
    case 4: return launch_gj_rt<4>(g, st);
    case 2: return launch_gj_rt<2>(g, st);
    default: return launch_gj_rt<1>(g, st);
  }
}

// ---------------------------------------------------------------------------
// Transposed system P^T (blocks C'_j = C_j^T, A'_j = B_{j-1}^T, B'_j = A_{j+1}^T), built on the
// device from the plan's compact copies of P, and the block inverses of its subdomain elimination
// taken from those of P: within a subdomain the transposed elimination's pivot blocks are
// D'_i = D_i^T (induction on C'_i - A'_i D'_{i-1}^{-1} B'_{i-1} = (C_i - A_i D_{i-1}^{-1} B_{i-1})^T),
// so D'_i^{-1} = (D_i^{-1})^T and alpha'_i = D'_i^{-1} diag(b'_i).
// ---------------------------------------------------------------------------
// A' (format fmtB), B' (format fmtA), C' (format fmtC) from A, B, C; one thread per entry
__global__ void k_transpose_inputs(double* At, double* Bt, double* Ct, const double* A, int fmtA, const double* B,
                                   int fmtB, const double* C, int fmtC, int N, int M) {
  const int64_t MM = (int64_t)M * M;
  const int64_t nA = (fmtB == 1) ? (int64_t)N * M : N * MM;   // A' has B's format
  const int64_t nB = (fmtA == 1) ? (int64_t)N * M : N * MM;   // B' has A's format
  const int64_t nC = (fmtC == 2) ? (int64_t)N * 3 * M : N * MM;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nA + nB + nC;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nA) {                     // A'_j = B_{j-1}^T, A'_0 = 0
      if (fmtB == 1) {
        const int64_t j = e / M, r = e % M;
        At[e] = j > 0 ? B[(j - 1) * M + r] : 0.0;
      } else {
        const int64_t j = e / MM, q = e % MM, r = q % M, c = q / M;   // A'_j(r, c) = B_{j-1}(c, r)
        At[e] = j > 0 ? B[(j - 1) * MM + c + r * M] : 0.0;
      }
    } else if (e < nA + nB) {         // B'_j = A_{j+1}^T, B'_{N-1} = 0
      const int64_t f = e - nA;
      if (fmtA == 1) {
        const int64_t j = f / M, r = f % M;
        Bt[f] = j + 1 < N ? A[(j + 1) * M + r] : 0.0;
      } else {
        const int64_t j = f / MM, q = f % MM, r = q % M, c = q / M;
        Bt[f] = j + 1 < N ? A[(j + 1) * MM + c + r * M] : 0.0;
      }
    } else {                          // C'_j = C_j^T
      const int64_t f = e - nA - nB;
      if (fmtC == 2) {                // (sub', diag', super')(r) = (super(r-1), diag(r), sub(r+1))
        const int64_t j = f / (3 * M), q = f % (3 * M), part = q / M, r = q % M;
        const double* t = C + j * 3 * M;
        double v;
        if (part == 1) v = t[M + r];
        else if (part == 0) v = r > 0 ? t[2 * M + r - 1] : 0.0;
        else v = r + 1 < M ? t[r + 1] : 0.0;
        Ct[f] = v;
      } else {
        const int64_t j = f / MM, q = f % MM, r = q % M, c = q / M;
        Ct[f] = C[j * MM + c + r * M];
      }
    }
  }
}

hipError_t launch_transpose_inputs(double* At, double* Bt, double* Ct, const double* A, int fmtA, const double* B,
                                   int fmtB, const double* C, int fmtC, int N, int M, hipStream_t st) {
  const int64_t MM = (int64_t)M * M;
  const int64_t tot = ((fmtB == 1) ? (int64_t)N * M : N * MM) + ((fmtA == 1) ? (int64_t)N * M : N * MM) +
                      ((fmtC == 2) ? (int64_t)N * 3 * M : N * MM);
  int bx = (int)std::min<int64_t>((tot + 255) / 256, 65536);
  hipLaunchKernelGGL(k_transpose_inputs, dim3(bx), dim3(256), 0, st, At, Bt, Ct, A, fmtA, B, fmtB, C, fmtC, N, M);
  return hipGetLastError();
}

// Dinv_t[row] = Dinv[row]^T and alpha_t[row] = Dinv_t[row] diag(bdiag_t[row]) for the listed rows
// (Mp x Mp column-major blocks at row * Mp^2); 32 x 32 tiles through LDS so that both the reads and
// the writes are coalesced (edge tiles guarded when Mp is not a multiple of 32).  Grid: (tiles of
// the block, rows).
__global__ void __launch_bounds__(256) k_transpose_scale(double* Dinv_t, double* alpha_t, const double* Dinv,
                                                         const double* bdiag_t, const int64_t* rows, int Mp) {
  __shared__ double tile[32][33];
  const int64_t row = rows[blockIdx.y];
  const int nt = (Mp + 31) / 32;
  const int ti = blockIdx.x % nt, tj = blockIdx.x / nt;     // source tile (rows ti, columns tj)
  const int64_t MM = (int64_t)Mp * Mp;
  const double* src = Dinv + row * MM;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = tj * 32 + ty + 8 * k, r = ti * 32 + tx;
    if (r < Mp && c < Mp) tile[ty + 8 * k][tx] = src[r + (int64_t)c * Mp];   // tile[c - 32 tj][r - 32 ti]
  }
  __syncthreads();
  // destination: transposed tile at (rows tj, columns ti): out(r', c') = in(c', r')
  const double* bt = bdiag_t + row * Mp;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cp = ti * 32 + ty + 8 * k, rp = tj * 32 + tx;
    if (rp < Mp && cp < Mp) {
      const double v = tile[tx][ty + 8 * k];
      Dinv_t[row * MM + rp + (int64_t)cp * Mp] = v;
      alpha_t[row * MM + rp + (int64_t)cp * Mp] = v * bt[cp];
    }
  }
}

hipError_t launch_transpose_scale(double* Dinv_t, double* alpha_t, const double* Dinv, const double* bdiag_t,
                                  const int64_t* rows, int nrows, int Mp, hipStream_t st) {
  const int nt = (Mp + 31) / 32;
  for (int r0 = 0; r0 < nrows; r0 += 65535) {   // grid.y is at most 65535
    const int nr = nrows - r0 < 65535 ? nrows - r0 : 65535;
    hipLaunchKernelGGL(k_transpose_scale, dim3(nt * nt, nr), dim3(256), 0, st, Dinv_t, alpha_t, Dinv, bdiag_t,
                       rows + r0, Mp);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// dst[b] = src[b]^T for nblk consecutive Mp x Mp column-major blocks; the same 32 x 32 LDS tiles as
// k_transpose_scale.  Grid: (tiles of the block, blocks).
__global__ void __launch_bounds__(256) k_transpose_blocks(double* dst, const double* src, int Mp) {
  __shared__ double tile[32][33];
  const int64_t MM = (int64_t)Mp * Mp;
  const double* s = src + (int64_t)blockIdx.y * MM;
  double* d = dst + (int64_t)blockIdx.y * MM;
  const int nt = (Mp + 31) / 32;
  const int ti = blockIdx.x % nt, tj = blockIdx.x / nt;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = tj * 32 + ty + 8 * k, r = ti * 32 + tx;
    if (r < Mp && c < Mp) tile[ty + 8 * k][tx] = s[r + (int64_t)c * Mp];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cp = ti * 32 + ty + 8 * k, rp = tj * 32 + tx;
    if (rp < Mp && cp < Mp) d[rp + (int64_t)cp * Mp] = tile[tx][ty + 8 * k];
  }
}

hipError_t launch_transpose_blocks(double* dst, const double* src, int64_t nblk, int Mp, hipStream_t st) {
  const int nt = (Mp + 31) / 32;
  const int64_t MM = (int64_t)Mp * Mp;
  for (int64_t b0 = 0; b0 < nblk; b0 += 65535) {   // grid.y is at most 65535
    const int64_t nb = nblk - b0 < 65535 ? nblk - b0 : 65535;
    hipLaunchKernelGGL(k_transpose_blocks, dim3(nt * nt, (unsigned)nb), dim3(256), 0, st, dst + b0 * MM, src + b0 * MM, Mp);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace td
