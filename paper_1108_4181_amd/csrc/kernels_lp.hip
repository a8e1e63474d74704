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

#include <cstdint>

namespace td {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// round-to-nearest-even float -> bfloat16 bits; NaN stays a quiet NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int PREC> struct LP;
template <> struct LP<1> {   // float32
  using T = float;
  static constexpr int KG = 16;                    // k per group
  __device__ static T from_f(float v) { return v; }
  __device__ static void mma(f32x4& acc, const uint4& a, const uint4& b) {
    const f32x4 av = __builtin_bit_cast(f32x4, a);
    const f32x4 bv = __builtin_bit_cast(f32x4, b);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u], acc, 0, 0, 0);
  }
};
template <> struct LP<2> {   // bfloat16
  using T = uint16_t;
  static constexpr int KG = 32;
  __device__ static T from_f(float v) { return f2bf(v); }
  __device__ static void mma(f32x4& acc, const uint4& a, const uint4& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   acc, 0, 0, 0);
  }
};

__device__ __forceinline__ int lp_xcd_remap(int b, int grid) {
  const int per = grid >> 3;
  return (b & 7) * per + (b >> 3);
}
static inline int lp_pad8(int t) { return (t + 7) & ~7; }

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
template <int PREC, int RT, int CT>
__global__ void __launch_bounds__(512) k_sweep_lp(LpSweepArgs a) {
  using Tr = LP<PREC>;
  using T = typename Tr::T;
  constexpr int KG = Tr::KG;
  constexpr int KT = 16 * CT;
  extern __shared__ uint4 lds_raw[];
  T* In = reinterpret_cast<T*>(lds_raw);     // [KT][SK]
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int SK = Mp + 16 / (int)sizeof(T);   // column stride (elements), padded by 16 bytes

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int lg = lp_xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  const int ct = lg - s * a.ncoltiles;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int rb = w * 16 * RT;
  const int64_t MM = (int64_t)Mp * Mp;
  const int ng = Mp / KG;   // k-groups per step

  const int64_t nsteps = 2 * (last - first) + 1;
  auto step_matrix = [&](int64_t q) -> const T* {
    return (q <= last - first) ? (const T*)a.Dinv + (first + q) * MM
                               : (const T*)a.alpha + (last - 1 - (q - (last - first + 1))) * MM;
  };
  // lane's 16-byte slice of row (rb + 16t + L%16), k-group g
  const int64_t lane_off = (int64_t)(rb + (L & 15)) * Mp + (KG / 4) * (L >> 4);
  uint4 a0[RT], a1[RT];
  auto loadA = [&](uint4 (&dst)[RT], const T* __restrict__ Ab, int g) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
      dst[t] = *reinterpret_cast<const uint4*>(Ab + lane_off + (int64_t)16 * t * Mp + KG * g);
  };
  f32x4 acc[RT][CT];
  auto compute = [&](const uint4 (&av)[RT], int g) {
    uint4 b[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
      b[c] = *reinterpret_cast<const uint4*>(In + (16 * c + (L & 15)) * SK + KG * g + (KG / 4) * (L >> 4));
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) Tr::mma(acc[t][c], av[t], b[c]);
  };

  for (int e = tid; e < Mp * KT; e += nthr) {
    const int row = e % Mp, c = e / Mp;
    const int col = col0 + c;
    const double v = (row < M && col < K) ? a.F[first * M + row + (int64_t)col * a.ldf] : 0.0;
    In[c * SK + row] = Tr::from_f((float)v);
  }
  loadA(a0, step_matrix(0), 0);
  __syncthreads();

  for (int64_t q = 0; q < nsteps; ++q) {
    const bool fwd = q <= last - first;
    const int64_t i = fwd ? first + q : last - 1 - (q - (last - first + 1));
    const T* __restrict__ Ai = step_matrix(q);
    const T* __restrict__ Anx = (q + 1 < nsteps) ? step_matrix(q + 1) : Ai;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    int g = 0;
    for (; g + 2 < ng; g += 2) {
      loadA(a1, Ai, g + 1);
      compute(a0, g);
      loadA(a0, Ai, g + 2);
      compute(a1, g + 1);
    }
    // epilogue operands: rows 4(L/16)..+3 of column L%16 of each tile
    const bool more = fwd && i < last;
    float ex[RT][CT][4];
    float an[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
      for (int v = 0; v < 4; ++v) an[t][v] = more ? (float)a.adiag[(i + 1) * Mp + row0 + v] : 0.f;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + 16 * c + (L & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + v;
          float x = 0.f;
          if (fwd) {
            if (more && row < M && col < K) x = (float)a.F[(i + 1) * M + row + (int64_t)col * a.ldf];
          } else if (col < K) {
            x = a.W[i * Mp + row + (int64_t)col * a.ldw];
          }
          ex[t][c][v] = x;
        }
      }
    }
    if (ng - g == 2) {
      loadA(a1, Ai, g + 1);
      compute(a0, g);
      loadA(a0, Anx, 0);
      compute(a1, g + 1);
    } else {
      compute(a0, g);
      loadA(a0, Anx, 0);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int lc = 16 * c + (L & 15);
        const int col = col0 + lc;
        f32x4 vv;
#pragma unroll
        for (int v = 0; v < 4; ++v) vv[v] = fwd ? acc[t][c][v] : acc[t][c][v] + ex[t][c][v];
        if (col < K) *reinterpret_cast<f32x4*>(a.W + i * Mp + row0 + (int64_t)col * a.ldw) = vv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float nxt = more ? ex[t][c][v] + an[t][v] * vv[v] : vv[v];
          In[lc * SK + row0 + v] = Tr::from_f(nxt);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Low-precision superposition: X_i (+)= W_i + [U_i V_i] [X_{k_s}; X_{k_{s+1}}] with the
// interface panel rounded to T in LDS and [U_i V_i] (row-major, T) streamed.  With
// `accumulate` the result is added to X (refinement correction).
// ---------------------------------------------------------------------------
template <int PREC, int RT, int CT>
__global__ void __launch_bounds__(512) k_superpose_lp(LpSupArgs a) {
  using Tr = LP<PREC>;
  using T = typename Tr::T;
  constexpr int KG = Tr::KG;
  constexpr int KT = 16 * CT;
  extern __shared__ uint4 lds_raw[];
  T* Xs = reinterpret_cast<T*>(lds_raw);   // [KT][SK]
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int kd = 2 * Mp;
  const int SK = kd + 16 / (int)sizeof(T);

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int lg = lp_xcd_remap(blockIdx.x, gridDim.x);
  if (lg >= a.total) return;
  const int s = lg / a.ncoltiles;
  const int ct = lg - s * a.ncoltiles;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int rb = w * 16 * RT;
  const int64_t MM2 = (int64_t)Mp * kd;
  const int ng = kd / KG;

  for (int e = tid; e < kd * KT; e += nthr) {
    const int k = e % kd, c = e / kd;
    const int col = col0 + c;
    const double v = (col < K) ? a.Xi[(int64_t)(s + 1) * Mp + k + (int64_t)col * a.ldxi] : 0.0;
    Xs[c * SK + k] = Tr::from_f((float)v);
  }

  const int64_t lane_off = (int64_t)(rb + (L & 15)) * kd + (KG / 4) * (L >> 4);
  uint4 a0[RT], a1[RT];
  auto loadA = [&](uint4 (&dst)[RT], const T* __restrict__ Ab, int g) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
      dst[t] = *reinterpret_cast<const uint4*>(Ab + lane_off + (int64_t)16 * t * kd + KG * g);
  };
  f32x4 acc[RT][CT];
  auto compute = [&](const uint4 (&av)[RT], int g) {
    uint4 b[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
      b[c] = *reinterpret_cast<const uint4*>(Xs + (16 * c + (L & 15)) * SK + KG * g + (KG / 4) * (L >> 4));
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) Tr::mma(acc[t][c], av[t], b[c]);
  };

  const T* UVb = (const T*)a.UV;
  loadA(a0, UVb + first * MM2, 0);
  __syncthreads();
  for (int64_t i = first; i <= last; ++i) {
    const T* __restrict__ Ai = UVb + i * MM2;
    const T* __restrict__ Anx = (i < last) ? Ai + MM2 : Ai;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    int g = 0;
    for (; g + 2 < ng; g += 2) {
      loadA(a1, Ai, g + 1);
      compute(a0, g);
      loadA(a0, Ai, g + 2);
      compute(a1, g + 1);
    }
    float wv[RT][CT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + 16 * c + (L & 15);
        f32x4 x = (f32x4){0.f, 0.f, 0.f, 0.f};
        if (col < K) x = *reinterpret_cast<const f32x4*>(a.W + i * Mp + row0 + (int64_t)col * a.ldw);
#pragma unroll
        for (int v = 0; v < 4; ++v) wv[t][c][v] = x[v];
      }
    }
    if (ng - g == 2) {
      loadA(a1, Ai, g + 1);
      compute(a0, g);
      loadA(a0, Anx, 0);
      compute(a1, g + 1);
    } else {
      compute(a0, g);
      loadA(a0, Anx, 0);
    }
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
          if (row < M) {
            double* xp = a.X + i * M + row + (int64_t)col * a.ldx;
            const double d = (double)acc[t][c][v] + (double)wv[t][c][v];
            *xp = a.accumulate ? *xp + d : d;
          }
        }
      }
    }
  }
}

static inline int lp_choose_rt(int Mp) {
  if (Mp >= 256 && Mp % 64 == 0) return 4;
  if (Mp >= 64 && Mp % 32 == 0) return 2;
  return 1;
}

template <int PREC, int RT, int CT>
static hipError_t launch_sweep_lp_cfg(const LpSweepArgs& a0, hipStream_t st) {
  LpSweepArgs a = a0;
  constexpr int kt = 16 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds = (size_t)kt * ((size_t)a.Mp * esz + 16);
  hipError_t e = hipFuncSetAttribute((const void*)k_sweep_lp<PREC, RT, CT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sweep_lp<PREC, RT, CT>), dim3(lp_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int RT>
static hipError_t launch_sweep_lp_rt(const LpSweepArgs& a, hipStream_t st) {
  if (a.K <= 16) return launch_sweep_lp_cfg<PREC, RT, 1>(a, st);
  if (a.K <= 32 || RT == 4) return launch_sweep_lp_cfg<PREC, RT, 2>(a, st);
  return launch_sweep_lp_cfg<PREC, RT, (RT == 4 ? 2 : 4)>(a, st);
}

hipError_t launch_sweep_lp(int prec, const LpSweepArgs& a, hipStream_t st) {
  const int rt = lp_choose_rt(a.Mp);
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

template <int PREC, int RT, int CT>
static hipError_t launch_sup_lp_cfg(const LpSupArgs& a0, hipStream_t st) {
  LpSupArgs a = a0;
  constexpr int kt = 16 * CT;
  a.ncoltiles = (a.K + kt - 1) / kt;
  a.total = a.p * a.ncoltiles;
  if (a.total == 0) return hipSuccess;
  const int nthr = a.Mp / (16 * RT) * 64;
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds = (size_t)kt * ((size_t)2 * a.Mp * esz + 16);
  hipError_t e = hipFuncSetAttribute((const void*)k_superpose_lp<PREC, RT, CT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_superpose_lp<PREC, RT, CT>), dim3(lp_pad8(a.total)), dim3(nthr), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int RT>
static hipError_t launch_sup_lp_rt(const LpSupArgs& a, hipStream_t st) {
  const size_t esz = (PREC == 1) ? 4 : 2;
  const size_t lds4 = (size_t)64 * ((size_t)2 * a.Mp * esz + 16);
  if (a.K <= 16) return launch_sup_lp_cfg<PREC, RT, 1>(a, st);
  if (a.K <= 32 || lds4 > 160 * 1024) return launch_sup_lp_cfg<PREC, RT, 2>(a, st);
  return launch_sup_lp_cfg<PREC, RT, 4>(a, st);
}

hipError_t launch_superpose_lp(int prec, const LpSupArgs& a, hipStream_t st) {
  const int rt = lp_choose_rt(a.Mp);
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
__global__ void k_ftilde_f32(double* Ft, int64_t ldft, const double* F, int64_t ldf, const float* W, int64_t ldw,
                             const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K) {
  const int64_t n = (int64_t)p * Mp * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % Mp);
    const int64_t sc = e / Mp;
    const int s = (int)(sc % p);
    const int64_t col = sc / p;
    const int64_t k = ks[s];
    double v = (r < M) ? F[k * M + r + col * ldf] : 0.0;
    if (s > 0 && k - 1 > ks[s - 1]) v += adiag[k * Mp + r] * (double)W[(k - 1) * Mp + r + col * ldw];
    if (k + 1 < ks[s + 1]) v += bdiag[k * Mp + r] * (double)W[(k + 1) * Mp + r + col * ldw];
    Ft[(int64_t)s * Mp + r + col * ldft] = v;
  }
}

hipError_t launch_ftilde_f32(double* Ft, int64_t ldft, const double* F, int64_t ldf, const float* W, int64_t ldw,
                             const int64_t* ks, const double* adiag, const double* bdiag, int p, int M, int Mp, int K,
                             hipStream_t st) {
  const int64_t n = (int64_t)p * Mp * K;
  if (n == 0) return hipSuccess;
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_ftilde_f32, dim3(bx), dim3(256), 0, st, Ft, ldft, F, ldf, W, ldw, ks, adiag, bdiag, p, M, Mp,
                     K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Float64 residual R = F - P X for diagonal A, B and tridiagonal C, streaming each column in
// contiguous row chunks (the stencil reaches one row up/down and one block up/down), with
// per-chunk sums of squares of R and F for the column norms (fixed order, no atomics).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_residual_stencil(double* R, int64_t ldr, const double* F, int64_t ldf,
                                                          const double* X, int64_t ldx, const double* A,
                                                          const double* B, const double* C, int N, int M, int K,
                                                          int chunk, double* colpart, int nchunk) {
  __shared__ double red[2][4];
  const int q = blockIdx.x, col = blockIdx.y;
  const int64_t n = (int64_t)N * M;
  const int64_t g0 = (int64_t)q * chunk;
  const int64_t g1 = g0 + chunk < n ? g0 + chunk : n;
  const double* x = X + (int64_t)col * ldx;
  const double* f = F + (int64_t)col * ldf;
  double sr = 0.0, sf = 0.0;
  for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
    const int64_t j = g / M;
    const int r = (int)(g - j * M);
    const double* t = C + j * 3 * M;
    double y = t[M + r] * x[g];
    if (r > 0) y += t[r] * x[g - 1];
    if (r < M - 1) y += t[2 * M + r] * x[g + 1];
    if (j > 0) y -= A[g] * x[g - M];
    if (j < N - 1) y -= B[g] * x[g + M];
    const double fv = f[g];
    const double rv = fv - y;
    if (R) R[g + (int64_t)col * ldr] = rv;
    sr += rv * rv;
    sf += fv * fv;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off);
    sf += __shfl_xor(sf, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = sf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int v = 0; v < 4; ++v) { a += red[0][v]; b += red[1][v]; }
    colpart[((int64_t)col * nchunk + q) * 2 + 0] = a;
    colpart[((int64_t)col * nchunk + q) * 2 + 1] = b;
  }
}

int residual_chunks(int64_t n) { return (int)((n + 8191) / 8192); }

hipError_t launch_residual_stencil(double* R, int64_t ldr, const double* F, int64_t ldf, const double* X, int64_t ldx,
                                   const double* A, const double* B, const double* C, int N, int M, int K,
                                   double* colpart, hipStream_t st) {
  if (K == 0) return hipSuccess;
  const int64_t n = (int64_t)N * M;
  const int nchunk = residual_chunks(n);
  hipLaunchKernelGGL(k_residual_stencil, dim3(nchunk, K), dim3(256), 0, st, R, ldr, F, ldf, X, ldx, A, B, C, N, M, K,
                     8192, colpart, nchunk);
  return hipGetLastError();
}

}  // namespace td
