// Low-precision sweep and superposition kernels (float32 or bfloat16 operands, float32
// accumulation) for gfx950, used by the mixed-precision solve with float64 refinement.
// The block pivots, the reduced interface system, the dichotomy and the residual stay
// float64; only the dense per-row products of the subdomain sweeps (eq. sub3) and of the
// superposition (eq. superposition) use rounded copies of D^{-1}, alpha and [U V].
//
// MFMA layouts (16 x 16 output tile, checked on the GPU):
//   v_mfma_f32_16x16x4_f32  : A lane L = A[L%16][L/16], B lane L = B[L/16][L%16]
//   v_mfma_f32_16x16x32_bf16: A lane L = A[L%16][8(L/16)+e], B lane L = B[8(L/16)+e][L%16], e < 8
//   result lane L, slot v  = D[4(L/16)+v][L%16]
// The float32 form runs four MFMAs per 16-deep k-group with the k index of MFMA u at lane
// L being 4(L/16)+u, so each lane reads 4 consecutive k values (16 bytes) of A and of B.
// Matrices are stored row-major (k contiguous) and the LDS operand column-major
// (k contiguous per column) so that every operand read is one 16-byte access.
#include "internal.h"
#include "tile_bodies.h"

#include <cstdint>

namespace td {

// ---------------------------------------------------------------------------
// Casts of the float64 factor: dst (row-major, k contiguous) = RNE(src col-major).
// src: nmat matrices of `rows x cols` (column-major, ld = rows) at src + q * sstride,
// for q in the row list; dst at dst + q * dstride.
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void k_cast_rowmajor(typename LP<PREC>::T* dst, int64_t dstride, const double* src, int64_t sstride,
                                const int64_t* list, int nmat, int rows, int cols) {
  const int q = blockIdx.y;
  if (q >= nmat) return;
  const int64_t m = list[q];
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[m * dstride + e] = LP<PREC>::from_f((float)src[m * sstride + r + (int64_t)c * rows]);
  }
}

hipError_t launch_cast_rowmajor(int prec, void* dst, int64_t dstride, const double* src, int64_t sstride,
                                const int64_t* list, int nmat, int rows, int cols, hipStream_t st) {
  if (nmat == 0) return hipSuccess;
  const int64_t n = (int64_t)rows * cols;
  int bx = (int)((n + 255) / 256);
  if (bx > 1024) bx = 1024;
  if (prec == 1)
    hipLaunchKernelGGL(k_cast_rowmajor<1>, dim3(bx, nmat), dim3(256), 0, st, (float*)dst, dstride, src, sstride,
                       list, nmat, rows, cols);
  else
    hipLaunchKernelGGL(k_cast_rowmajor<2>, dim3(bx, nmat), dim3(256), 0, st, (uint16_t*)dst, dstride, src, sstride,
                       list, nmat, rows, cols);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Low-precision sweeps (eq. sub3): as the float64 sweep, with the step operand in LDS as
// T (column-major, k contiguous), beta / W kept in float32 in the workspace, and the input
// right-hand side read in float64 and rounded once.
// ---------------------------------------------------------------------------
template <int PREC, int RT, int CT, int KU>
__global__ void __launch_bounds__(512) k_sweep_lp(LpSweepArgs a) {
  extern __shared__ uint4 lds_raw[];
  const int lg = lp_xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  sweep_lp_tile<PREC, RT, CT, KU>(a, s, lg - s * a.ncoltiles, lds_raw);
}

// ---------------------------------------------------------------------------
// Low-precision superposition: X_i (+)= W_i + [U_i V_i] [X_{k_s}; X_{k_{s+1}}] with the
// interface panel rounded to T in LDS and [U_i V_i] (row-major, T) streamed.  With
// `accumulate` the result is added to X (refinement correction).
// ---------------------------------------------------------------------------
template <int PREC, int RT, int CT, int KU, int ACC>
__global__ void __launch_bounds__(512) k_superpose_lp(LpSupArgs a) {
  extern __shared__ uint4 lds_raw[];
  const int lg = lp_xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  superpose_lp_tile<PREC, RT, CT, KU, ACC>(a, s, lg - s * a.ncoltiles, lds_raw);
}

// k-groups per register chunk of the streamed matrix: a float32 group (16 deep) is four MFMAs per
// tile and one group of prefetch covers the load latency (longer chunks measured no faster); a
// bfloat16 group (32 deep) is one MFMA, so bfloat16 loads four groups ahead (5% faster sweeps)
template <int PREC>
static inline int lp_chunk(int ngroups) {
  if (PREC == 1) return 1;
  if (ngroups % 4 == 0) return 4;
  return (ngroups % 2 == 0) ? 2 : 1;
}

// rows per wave = 16 RT, work-group = 4 Mp / RT threads (at most 512).  Up to Mp = 256 two row
// tiles per wave and eight waves win: at 2048x256 the bfloat16 sweep takes 2.26 ms with
// RT = 2 / 64 columns against 2.69 ms with RT = 4 / 32 columns (float32: 3.75 against 4.25 ms);
// larger blocks need RT = 4 to stay within 512 threads.
static inline int lp_choose_rt(int Mp) {
  if (Mp > 256 && Mp % 64 == 0) return 4;
  if (Mp >= 64 && Mp % 32 == 0) return 2;
  return 1;
}

// the rule's row-tile count, or a hinted one where the block size divides into it within 8 waves
static inline int lp_hinted_rt(int Mp, int hint) {
  if ((hint == 1 || hint == 2 || hint == 4) && Mp % (16 * hint) == 0 && Mp / (16 * hint) <= 8) return hint;
  return lp_choose_rt(Mp);
}

template <int PREC, int RT, int CT, int KU>
static hipError_t launch_sweep_lp_cfg(const LpSweepArgs& a0, hipStream_t st) {
  LpSweepArgs a = a0;
  constexpr int kt = 16 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds = (size_t)kt * ((size_t)a.Mp * esz + 32);
  hipError_t e = hipFuncSetAttribute((const void*)k_sweep_lp<PREC, RT, CT, KU>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sweep_lp<PREC, RT, CT, KU>), dim3(lp_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int RT, int CT>
static hipError_t launch_sweep_lp_ku(const LpSweepArgs& a, hipStream_t st) {
  const int ngroups = a.Mp / LP<PREC>::KG;
  // four row tiles of two or more column tiles: chunks of four k-groups would spill registers
  if constexpr (RT == 4 && CT >= 2) {
    if (lp_chunk<PREC>(ngroups) >= 2) return launch_sweep_lp_cfg<PREC, RT, CT, 2>(a, st);
    return launch_sweep_lp_cfg<PREC, RT, CT, 1>(a, st);
  }
  // float32 sweeps of at most two row tiles: four groups ahead (the epilogue's loads then
  // stay in flight together; 3.31 -> 3.16 ms at 2048x256)
  if constexpr (PREC == 1 && RT <= 2 && CT == 4) {
    if (ngroups % 4 == 0) return launch_sweep_lp_cfg<PREC, RT, CT, 4>(a, st);
  }
  switch (lp_chunk<PREC>(ngroups)) {
    case 4: return launch_sweep_lp_cfg<PREC, RT, CT, 4>(a, st);
    case 2: return launch_sweep_lp_cfg<PREC, RT, CT, 2>(a, st);
    default: return launch_sweep_lp_cfg<PREC, RT, CT, 1>(a, st);
  }
}

template <int PREC, int RT>
static hipError_t launch_sweep_lp_rt(const LpSweepArgs& a, hipStream_t st) {
  // hinted columns per work-group (four row tiles of 64 columns spill registers)
  if (a.kt_hint == 16) return launch_sweep_lp_ku<PREC, RT, 1>(a, st);
  if (a.kt_hint == 32) return launch_sweep_lp_ku<PREC, RT, 2>(a, st);
  if (a.kt_hint == 64 && RT < 4) return launch_sweep_lp_ku<PREC, RT, (RT < 4 ? 4 : 2)>(a, st);
  if (a.K <= 16) return launch_sweep_lp_ku<PREC, RT, 1>(a, st);
  if (a.K <= 32 || RT == 4) return launch_sweep_lp_ku<PREC, RT, 2>(a, st);
  return launch_sweep_lp_ku<PREC, RT, (RT == 4 ? 2 : 4)>(a, st);
}

hipError_t launch_sweep_lp(int prec, const LpSweepArgs& a, hipStream_t st) {
  const int rt = lp_hinted_rt(a.Mp, a.rt_hint);
  if (prec == 1) {
    if (rt == 4) return launch_sweep_lp_rt<1, 4>(a, st);
    if (rt == 2) return launch_sweep_lp_rt<1, 2>(a, st);
    return launch_sweep_lp_rt<1, 1>(a, st);
  }
  if (a.Mp % 32 != 0) return hipErrorInvalidValue;  // bfloat16 k-groups are 32 deep
  if (rt == 4) return launch_sweep_lp_rt<2, 4>(a, st);
  if (rt == 2) return launch_sweep_lp_rt<2, 2>(a, st);
  return launch_sweep_lp_rt<2, 1>(a, st);
}

// Float32 superposition above block size 256 with 64-column tiles: the `2Mp x 64` float32 panel
// (264 KB at Mp = 512) does not fit in LDS, so LDS holds one half of it at a time (the left
// interface's Mp rows for U_i, or the right interface's for V_i); a row multiplies the half in LDS,
// reloads the other half and multiplies that, and the next row starts with the half now in LDS.
// Against 32-column tiles this halves the L2-to-CU traffic of [U_i V_i] per flop.  Writes X (the
// accumulating form keeps the 32-column kernel).
template <int PREC, int RT, int CT, int KU>
__device__ __forceinline__ void superpose_lp_half_tile(const LpSupArgs& a, int s, int ct, uint4* lds_raw) {
  using Tr = LP<PREC>;
  using T = typename Tr::T;
  constexpr int KG = Tr::KG;
  constexpr int KT = 16 * CT;
  static_assert(W32_PANEL % KT == 0, "a column tile must lie in one workspace panel");
  T* Xs = reinterpret_cast<T*>(lds_raw);   // [KT][SK]: one half of the panel
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int kd = 2 * Mp;
  const int SK = Mp + 32 / (int)sizeof(T);

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int rb = w * 16 * RT;
  const int64_t MM2 = (int64_t)Mp * kd;
  const int nkh = Mp / (KG * KU);          // chunks per half (even: Mp is a multiple of 64 here)
  const float* const Wp = a.W + (int64_t)(col0 / W32_PANEL) * a.N * W32_PANEL * Mp;
  const int cp0 = col0 % W32_PANEL;

  // Xi rows (s + 1 + h) Mp .. (s + 2 + h) Mp - 1 of the tile's columns, rounded, -> LDS; a batch's
  // loads are issued before its stores (columns beyond K read column K - 1 and store zero)
  auto load_half = [&](int h) {
    constexpr int B = 8;
    const double* __restrict__ src = a.Xi + (int64_t)(s + 1 + h) * Mp;
    const int n = Mp * KT;
    for (int e0 = tid; e0 < n; e0 += B * nthr) {
      double v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = min(e0 + u * nthr, n - 1);
        const int k = e % Mp, col = min(col0 + e / Mp, K - 1);
        v[u] = src[k + (int64_t)col * a.ldxi];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = e0 + u * nthr;
        if (e < n) {
          const int k = e % Mp, c = e / Mp;
          Xs[c * SK + k] = Tr::from_f((col0 + c < K) ? (float)v[u] : 0.f);
        }
      }
    }
  };

  const int64_t lane_off = (int64_t)(rb + (L & 15)) * kd + (KG / 4) * (L >> 4);
  uint4 a0[KU][RT], a1[KU][RT];
  auto loadA = [&](uint4 (&dst)[KU][RT], const T* __restrict__ Ab, int q) {   // Ab: the half's first k
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < RT; ++t)
        dst[u][t] = *reinterpret_cast<const uint4*>(Ab + lane_off + (int64_t)16 * t * kd + KG * (KU * q + u));
  };
  f32x4 acc[RT][CT];
  auto compute = [&](const uint4 (&av)[KU][RT], int q) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int g = KU * q + u;
      uint4 b[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c)
        b[c] = *reinterpret_cast<const uint4*>(Xs + (16 * c + (L & 15)) * SK + KG * g + (KG / 4) * (L >> 4));
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) Tr::mma(acc[t][c], av[u][t], b[c]);
    }
  };
  auto body = [&](const T* __restrict__ Ah) {   // all chunks of a half but the last two
    for (int g = 0; g < nkh - 2; g += 2) {
      loadA(a1, Ah, g + 1);
      compute(a0, g);
      loadA(a0, Ah, g + 2);
      compute(a1, g + 1);
    }
  };

  const T* UVb = (const T*)a.UV;
  int cur = 0;   // the half in LDS
  load_half(0);
  loadA(a0, UVb + first * MM2, 0);
  __syncthreads();
  for (int64_t i = first; i <= last; ++i) {
    const T* __restrict__ Ai = UVb + i * MM2;
    const T* __restrict__ Anx = (i < last) ? Ai + MM2 : Ai;
    const int nxt = 1 - cur;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    {   // the half in LDS; its last chunk prefetches chunk 0 of the other half of this row
      const T* __restrict__ Ah = Ai + cur * Mp;
      body(Ah);
      loadA(a1, Ah, nkh - 1);
      compute(a0, nkh - 2);
      loadA(a0, Ai + nxt * Mp, 0);
      compute(a1, nkh - 1);
    }
    __syncthreads();   // every wave is done reading this half
    load_half(nxt);
    __syncthreads();
    const T* __restrict__ Ah = Ai + nxt * Mp;
    body(Ah);
    float wv[RT][CT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + 16 * c + (L & 15);
        f32x4 x = (f32x4){0.f, 0.f, 0.f, 0.f};
        if (col < K) x = *reinterpret_cast<const f32x4*>(Wp + i * (W32_PANEL * Mp) + (int64_t)(cp0 + 16 * c + (L & 15)) * Mp + row0);
#pragma unroll
        for (int v = 0; v < 4; ++v) wv[t][c][v] = x[v];
      }
    }
    loadA(a1, Ah, nkh - 1);
    compute(a0, nkh - 2);
    loadA(a0, Anx + nxt * Mp, 0);   // the next row starts with the half now in LDS
    compute(a1, nkh - 1);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + 16 * c + (L & 15);
        if (col >= K) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + v;
          if (row < M) a.X[i * M + row + (int64_t)col * a.ldx] = (double)acc[t][c][v] + (double)wv[t][c][v];
        }
      }
    }
    cur = nxt;
  }
}

template <int PREC, int RT, int CT, int KU>
__global__ void __launch_bounds__(512) k_superpose_lp_half(LpSupArgs a) {
  extern __shared__ uint4 lds_raw[];
  const int lg = lp_xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  superpose_lp_half_tile<PREC, RT, CT, KU>(a, s, lg - s * a.ncoltiles, lds_raw);
}

template <int PREC, int RT, int CT, int KU>
static hipError_t launch_sup_lp_half_cfg(const LpSupArgs& a0, hipStream_t st) {
  LpSupArgs a = a0;
  constexpr int kt = 16 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds = (size_t)kt * ((size_t)a.Mp * esz + 32);
  hipError_t e = hipFuncSetAttribute((const void*)k_superpose_lp_half<PREC, RT, CT, KU>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_superpose_lp_half<PREC, RT, CT, KU>), dim3(lp_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int RT, int CT, int KU>
static hipError_t launch_sup_lp_cfg(const LpSupArgs& a0, hipStream_t st) {
  LpSupArgs a = a0;
  constexpr int kt = 16 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds = (size_t)kt * ((size_t)2 * a.Mp * esz + 32);
  // separate kernels for writing and for adding to X (the first pass of a solve writes)
  const void* fn = a.accumulate ? (const void*)k_superpose_lp<PREC, RT, CT, KU, 1>
                                : (const void*)k_superpose_lp<PREC, RT, CT, KU, 0>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (a.accumulate)
    hipLaunchKernelGGL((k_superpose_lp<PREC, RT, CT, KU, 1>), dim3(lp_pad8(a.total)), dim3(nthr), lds, st, a);
  else
    hipLaunchKernelGGL((k_superpose_lp<PREC, RT, CT, KU, 0>), dim3(lp_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int RT, int CT>
static hipError_t launch_sup_lp_ku(const LpSupArgs& a, hipStream_t st) {
  // the widest tile already holds 16 accumulators per lane: longer chunks would spill
  if constexpr (RT * CT >= 16) {
    return launch_sup_lp_cfg<PREC, RT, CT, 1>(a, st);
  } else {
    switch (lp_chunk<PREC>(2 * a.Mp / LP<PREC>::KG)) {
      case 4: return launch_sup_lp_cfg<PREC, RT, CT, 4>(a, st);
      case 2: return launch_sup_lp_cfg<PREC, RT, CT, 2>(a, st);
      default: return launch_sup_lp_cfg<PREC, RT, CT, 1>(a, st);
    }
  }
}

template <int PREC, int RT>
static hipError_t launch_sup_lp_rt(const LpSupArgs& a, hipStream_t st) {
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds4 = (size_t)64 * ((size_t)2 * a.Mp * esz + 32);
  const size_t lds2 = (size_t)32 * ((size_t)2 * a.Mp * esz + 32);
  if (a.kt_hint == 16) return launch_sup_lp_ku<PREC, RT, 1>(a, st);
  if (a.kt_hint == 32 && lds2 <= 160 * 1024) return launch_sup_lp_ku<PREC, RT, 2>(a, st);
  if (a.kt_hint == 64 && lds4 <= 160 * 1024) return launch_sup_lp_ku<PREC, RT, 4>(a, st);
  if constexpr (PREC == 1 && RT == 4) {   // float32 above block size 256: half of the panel in LDS
    if ((a.kt_hint == 0 || a.kt_hint == 64) && a.K > 32 && !a.accumulate && a.Mp % 64 == 0 &&
        lds4 > 160 * 1024 && (size_t)64 * ((size_t)a.Mp * esz + 32) <= 160 * 1024)
      return launch_sup_lp_half_cfg<PREC, 4, 4, 1>(a, st);
  }
  if (a.K <= 16) return launch_sup_lp_ku<PREC, RT, 1>(a, st);
  if (a.K <= 32 || lds4 > 160 * 1024) return launch_sup_lp_ku<PREC, RT, 2>(a, st);
  return launch_sup_lp_ku<PREC, RT, 4>(a, st);
}

hipError_t launch_superpose_lp(int prec, const LpSupArgs& a, hipStream_t st) {
  const int rt = lp_hinted_rt(a.Mp, a.rt_hint);
  if (prec == 1) {
    if (rt == 4) return launch_sup_lp_rt<1, 4>(a, st);
    if (rt == 2) return launch_sup_lp_rt<1, 2>(a, st);
    return launch_sup_lp_rt<1, 1>(a, st);
  }
  if (a.Mp % 32 != 0) return hipErrorInvalidValue;
  if (rt == 4) return launch_sup_lp_rt<2, 4>(a, st);
  if (rt == 2) return launch_sup_lp_rt<2, 2>(a, st);
  return launch_sup_lp_rt<2, 1>(a, st);
}

// ---------------------------------------------------------------------------
// Right-hand side of the reduced system from a float32 W (see k_ftilde)
// ---------------------------------------------------------------------------
__global__ void k_ftilde_f32(double* Ft, int64_t ldft, const double* F, int64_t ldf, const float* W, int64_t N,
                             const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K) {
  const int64_t n = (int64_t)p * Mp * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % Mp);
    const int64_t sc = e / Mp;
    const int s = (int)(sc % p);
    const int64_t col = sc / p;
    const int64_t k = ks[s];
    double v = (r < M) ? F[k * M + r + col * ldf] : 0.0;
    if (s > 0 && k - 1 > ks[s - 1]) v += adiag[k * Mp + r] * (double)W[w32_off(N, Mp, k - 1, r, col)];
    if (k + 1 < ks[s + 1]) v += bdiag[k * Mp + r] * (double)W[w32_off(N, Mp, k + 1, r, col)];
    Ft[(int64_t)s * Mp + r + col * ldft] = v;
  }
}

hipError_t launch_ftilde_f32(double* Ft, int64_t ldft, const double* F, int64_t ldf, const float* W, int64_t N,
                             const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K,
                             hipStream_t st) {
  const int64_t n = (int64_t)p * Mp * K;
  if (n == 0) return hipSuccess;
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_ftilde_f32, dim3(bx), dim3(256), 0, st, Ft, ldft, F, ldf, W, N, ks, adiag, bdiag, p, M, Mp,
                     K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Float64 stencil residual (residual_cols_tile): grid (row chunks of RES_ROWS, groups of
// RES_COLS right-hand sides)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_residual_stencil(double* R, int64_t ldr, const double* F, int64_t ldf,
                                                          const double* X, int64_t ldx, const double* A,
                                                          const double* B, const double* C, int N, int M, int K,
                                                          double* colpart, int nchunk) {
  extern __shared__ double xs[];   // RES_ROWS_WIDE + 2M
  __shared__ double red[2 * RES_COLS][4];
  residual_cols_tile<RES_ROWS_WIDE>(R, ldr, F, ldf, X, ldx, A, B, C, N, M, K, colpart, nchunk, blockIdx.x,
                                    blockIdx.y * RES_COLS, xs, red);
}

int residual_row_chunks(int64_t n) { return (int)((n + RES_ROWS - 1) / RES_ROWS); }
int residual_row_chunks_wide(int64_t n) { return (int)((n + RES_ROWS_WIDE - 1) / RES_ROWS_WIDE); }

hipError_t launch_residual_stencil(double* R, int64_t ldr, const double* F, int64_t ldf, const double* X, int64_t ldx,
                                   const double* A, const double* B, const double* C, int N, int M, int K,
                                   double* colpart, hipStream_t st) {
  if (K == 0) return hipSuccess;
  if (M > 512) return hipErrorInvalidValue;   // the staged span assumes M <= 512
  const int64_t n = (int64_t)N * M;
  const int nchunk = residual_row_chunks_wide(n);
  const size_t lds = (size_t)(RES_ROWS_WIDE + 2 * M) * sizeof(double);
  hipLaunchKernelGGL(k_residual_stencil, dim3(nchunk, (K + RES_COLS - 1) / RES_COLS), dim3(256), lds, st, R, ldr, F,
                     ldf, X, ldx, A, B, C, N, M, K, colpart, nchunk);
  return hipGetLastError();
}

// Zero the coefficients of neighbours that do not exist (A of the first block row, B of the
// last, the sub-diagonal entry of each block's first row and the super-diagonal entry of its
// last row): the problem ignores them, and the stencil residual multiplies by them.
__global__ void k_zero_absent(double* A, double* B, double* C, int N, int M) {
  const int64_t M64 = M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M64 * 2 + (int64_t)N * 2;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < M64) A[e] = 0.0;
    else if (e < 2 * M64) B[((int64_t)N - 1) * M64 + (e - M64)] = 0.0;
    else if (e < 2 * M64 + N) C[(e - 2 * M64) * 3 * M64] = 0.0;
    else C[(e - 2 * M64 - N) * 3 * M64 + 3 * M64 - 1] = 0.0;
  }
}

hipError_t launch_zero_absent(double* A, double* B, double* C, int N, int M, hipStream_t st) {
  const int64_t total = 2 * (int64_t)M + 2 * (int64_t)N;
  int bx = (int)((total + 255) / 256);
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_zero_absent, dim3(bx), dim3(256), 0, st, A, B, C, N, M);
  return hipGetLastError();
}

}  // namespace td
