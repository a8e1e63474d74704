// Work-group tile bodies of the solver's main kernels, shared by the one-stage kernels
// (kernels_f64.hip, kernels_lp.hip) and the persistent batched kernel (kernels_batched.hip).
#pragma once

#include "device_common.h"
#include "internal.h"

namespace td {

// Position of column c in a row of a 4 CT-column float64 operand staged in LDS.  A lane reads the
// CT columns of block L % 4 of a row, 16 bytes at a time; the four blocks are interleaved in
// 16-byte pairs so that the lanes of one read touch one 64-byte span (with the blocks side by side
// they sit 64 bytes apart and two of them share LDS banks).  The epilogue's writes of column pairs
// are 16-byte stores that are conflict-free too.
template <int CT>
__device__ __forceinline__ int lds_col(int c) {
  static_assert(CT % 2 == 0, "column blocks are stored in pairs");
  return ((c % CT) >> 1) * 8 + 2 * (c / CT) + (c & 1);
}

// Physical row of row k of such an operand (rows come in groups of 16).  One MFMA k-step reads
// rows 4m .. 4m+3; they are stored 4 rows apart (row 4m+j at 16 (m/4) + 4 j + m % 4), which puts
// the sixteen 16-byte pieces a k-step reads (four rows, four column blocks) in distinct LDS banks.
__device__ __forceinline__ int lds_row(int k) { return (k & ~15) + 4 * (k & 3) + ((k >> 2) & 3); }

// KC: inner rows of B per LDS chunk (a multiple of 16 that divides every descriptor's kd and
// segrows); one barrier per chunk.
template <int RT, int CT, int KC = 16>
__device__ __forceinline__ void bgemm_tile(const BArgs& args, int prob, int ct, double* lds) {
  static_assert(KC % 16 == 0, "chunks of 16-row groups");
  constexpr int KT = 4 * CT;
  constexpr int SB = KT + 2;
  // staging slots per thread for one B chunk; every caller runs at least 64 RT threads
  constexpr int NSTG = (KC * KT + 64 * RT - 1) / (64 * RT);
  double* Bs0 = lds;              // [2][KC * SB]

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const BDesc d = args.descs[prob];
  const int col0 = ct * KT;
  const int rb = w * 16 * RT;
  const double* __restrict__ A = args.A + d.a_off;
  const int64_t lda = args.lda;

  double acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[t][c] = 0.0;

  const int nch = d.kd / KC;
  double stg[NSTG];
  // B chunk loads are unconditional, their indices clamped into the operand (values read there
  // are discarded): a load under a per-lane branch makes the compiler wait for every outstanding
  // load, the prefetched A chunks included, before the next one.
  const int krows = args.brows > 0 ? args.brows : d.segrows;
  auto gload = [&](int q) {
    const int k0 = q * KC;
    const int seg = k0 / d.segrows;
    const int kin = k0 - seg * d.segrows;
    const double* Bq = args.B + d.b_off + (int64_t)seg * d.bseg + kin;
    bool ok[NSTG];
#pragma unroll
    for (int u = 0; u < NSTG; ++u) {
      const int e = tid + u * nthr;
      const int ec = min(e, KC * KT - 1);
      const int k = ec % KC, c = ec / KC;
      const int col = col0 + c;
      ok[u] = e < KC * KT && col < args.ncols && kin + k < krows;
      stg[u] = 0.0;
      // (uniform: slots beyond the chunk exist only with more than 64 RT threads)
      if (u == 0 || u * nthr < KC * KT) stg[u] = Bq[(int64_t)min(col, args.ncols - 1) * args.ldb + min(k, krows - 1 - kin)];
    }
    if (args.bscale) {
#pragma unroll
      for (int u = 0; u < NSTG; ++u) {
        const int k = min(tid + u * nthr, KC * KT - 1) % KC;
        stg[u] *= args.bscale[d.bs_off + k0 + k];
      }
    }
#pragma unroll
    for (int u = 0; u < NSTG; ++u) stg[u] = ok[u] ? stg[u] : 0.0;
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NSTG; ++u) {
      const int e = tid + u * nthr;
      if (e < KC * KT) {
        const int k = e % KC, c = e / KC;
        Bs0[buf * KC * SB + lds_row(k) * SB + lds_col<CT>(c)] = stg[u];
      }
    }
  };

  // A streams through two register buffers (halves of a 16-deep chunk), each loaded one
  // half-chunk ahead of its use; B chunks go through double-buffered LDS.
  const int64_t lane_off = rb + (L & 15) + (int64_t)(L >> 4) * lda;
  double a0[2][RT], a1[2][RT];
  auto loadA = [&](double (&dst)[2][RT], int kbase) {   // k-steps kbase/4 and kbase/4 + 1
    const double* __restrict__ pa = A + lane_off + (int64_t)kbase * lda;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int t = 0; t < RT; ++t) dst[u][t] = pa[16 * t + (int64_t)(4 * u) * lda];
  };
  auto compute = [&](const double (&av)[2][RT], int buf, int r, int half) {   // 16-row group r of the chunk
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // rows 4m + L/16 of the group, m = 2 half + u (see lds_row, lds_col)
      const double* bp = &Bs0[buf * KC * SB + (16 * r + 4 * (L >> 4) + 2 * half + u) * SB + 2 * (L & 3)];
      double b[CT];
#pragma unroll
      for (int c = 0; c < CT; c += 2) {
        const double2 v = *reinterpret_cast<const double2*>(bp + (c >> 1) * 8);
        b[c] = v.x;
        b[c + 1] = v.y;
      }
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = mfma4(av[u][t], b[c], acc[t][c]);
    }
  };

  gload(0);
  loadA(a0, 0);
  lstore(0);
  __syncthreads();
  for (int q = 0; q < nch; ++q) {
    const int buf = q & 1;
    const bool more = q + 1 < nch;
    if (more) gload(q + 1);
#pragma unroll
    for (int r = 0; r < KC / 16; ++r) {
      const int kb = q * KC + 16 * r;
      loadA(a1, kb + 8);
      compute(a0, buf, r, 0);
      loadA(a0, (kb + 16 < nch * KC) ? kb + 16 : 0);
      compute(a1, buf, r, 1);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
  }

  // partial sums: the CT loads of one row group of one partial are independent, so they are in
  // flight together
  for (int s = 0; s < d.nsp; ++s) {
    const double* __restrict__ sp = args.Sp + d.sp_off + s * args.spstride;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      double pv[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        const double v = sp[rb + 16 * t + out_row(L) + (int64_t)min(col, args.ncols - 1) * args.ldsp];
        pv[c] = (col < args.ncols) ? v : 0.0;
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] += pv[c];
    }
  }
  // epilogue: the addends (Cin, and X2 when accumulating) are loaded for the whole tile first, by
  // unconditional loads with clamped indices, then the stores
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[t][c] *= args.alpha;
  if (args.Cin) {
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        const double v = args.Cin[d.cin_off + row + (int64_t)min(col, args.ncols - 1) * args.ldcin];
        acc[t][c] += (col < args.ncols) ? v : 0.0;
      }
    }
  }
  if (args.C) {
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        if (col < args.ncols) args.C[d.c_off + row + (int64_t)col * args.ldc] = acc[t][c];
      }
    }
  }
  if (args.X2) {
    if (args.x2accum) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + out_row(L);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int col = col0 + out_col(L) * CT + c;
          const double v = args.X2[d.x2_off + min(row, args.x2rows - 1) + (int64_t)min(col, args.ncols - 1) * args.ldx2];
          acc[t][c] += (row < args.x2rows && col < args.ncols) ? v : 0.0;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        if (col < args.ncols && row < args.x2rows) args.X2[d.x2_off + row + (int64_t)col * args.ldx2] = acc[t][c];
      }
    }
  }
}

// The step matrix streams through two register buffers of KU k-groups each (KU must divide the
// number of k-groups, Mp / KG), each loaded one buffer ahead of its MFMAs.
template <int PREC, int RT, int CT, int KU = 1>
__device__ __forceinline__ void sweep_lp_tile(const LpSweepArgs& a, int s, int ct, uint4* lds_raw) {
  using Tr = LP<PREC>;
  using T = typename Tr::T;
  constexpr int KG = Tr::KG;
  constexpr int KT = 16 * CT;
  static_assert(W32_PANEL % KT == 0, "a column tile must lie in one workspace panel");
  T* In = reinterpret_cast<T*>(lds_raw);     // [KT][SK]
  const int Mp = a.Mp, M = a.M, K = a.K;
  // column stride (elements), padded by 32 bytes: with a stride of 32 (mod 64) bytes the 16-byte
  // pieces that 32 lanes read of 16 columns and two k-groups lie in distinct LDS banks
  const int SK = Mp + 32 / (int)sizeof(T);

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int rb = w * 16 * RT;
  const int64_t MM = (int64_t)Mp * Mp;
  const int nkc = Mp / (KG * KU);   // chunks of KU k-groups per step
  // the tile's columns lie in one panel of the float32 workspace (KT divides W32_PANEL)
  float* const Wp = a.W + (int64_t)(col0 / W32_PANEL) * a.N * W32_PANEL * Mp;
  const int cp0 = col0 % W32_PANEL;

  const int64_t nsteps = 2 * (last - first) + 1;
  auto step_matrix = [&](int64_t q) -> const T* {
    return (q <= last - first) ? (const T*)a.Dinv + (first + q) * MM
                               : (const T*)a.alpha + (last - 1 - (q - (last - first + 1))) * MM;
  };
  // lane's 16-byte slice of row (rb + 16t + L%16), k-group g
  const int64_t lane_off = (int64_t)(rb + (L & 15)) * Mp + (KG / 4) * (L >> 4);
  uint4 a0[KU][RT], a1[KU][RT];
  auto loadA = [&](uint4 (&dst)[KU][RT], const T* __restrict__ Ab, int q) {
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < RT; ++t)
        dst[u][t] = *reinterpret_cast<const uint4*>(Ab + lane_off + (int64_t)16 * t * Mp + KG * (KU * q + u));
  };
  f32x4 acc[RT][CT];
  auto compute = [&](const uint4 (&av)[KU][RT], int q) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int g = KU * q + u;
      uint4 b[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c)
        b[c] = *reinterpret_cast<const uint4*>(In + (16 * c + (L & 15)) * SK + KG * g + (KG / 4) * (L >> 4));
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) Tr::mma(acc[t][c], av[u][t], b[c]);
    }
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
    for (; g + 2 < nkc; g += 2) {
      loadA(a1, Ai, g + 1);
      compute(a0, g);
      loadA(a0, Ai, g + 2);
      compute(a1, g + 1);
    }
    // epilogue operands: rows 4(L/16)..+3 of column L%16 of each tile
    // Unconditional loads (out-of-range lanes read element 0 and discard it): a load under a
    // per-lane branch makes the compiler wait for every outstanding load before the next one.
    const bool more = fwd && i < last;
    float ex[RT][CT][4];
    float an[RT][4];
    const double* __restrict__ asrc = a.adiag + (more ? (i + 1) * Mp : 0);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double av = asrc[row0 + v];
        an[t][v] = more ? (float)av : 0.f;
      }
    }
    if (fwd) {
      // row and column indices clamped into the operand (the values read there are discarded)
      const double* __restrict__ fsrc = a.F + (more ? (i + 1) * M : 0);
      const int frows = more ? M : 0;
      const int rmax = more ? M - 1 : 0;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int col = col0 + 16 * c + (L & 15);
          const double* __restrict__ fc = fsrc + (int64_t)min(col, K - 1) * a.ldf;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = row0 + v < frows && col < K;
            const double x = fc[min(row0 + v, rmax)];
            ex[t][c][v] = ok ? (float)x : 0.f;
          }
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row0 = rb + 16 * t + 4 * (L >> 4);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const bool ok = col0 + 16 * c + (L & 15) < K;
          const f32x4 x = *reinterpret_cast<const f32x4*>(
              Wp + (ok ? i * (W32_PANEL * Mp) + (int64_t)(cp0 + 16 * c + (L & 15)) * Mp + row0 : 0));
#pragma unroll
          for (int v = 0; v < 4; ++v) ex[t][c][v] = ok ? x[v] : 0.f;
        }
      }
    }
    if (nkc - g == 2) {
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
        if (col < K) *reinterpret_cast<f32x4*>(Wp + i * (W32_PANEL * Mp) + (int64_t)(cp0 + lc) * Mp + row0) = vv;
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

// ACC: 0 writes X_i, 1 adds to X_i, -1 follows a.accumulate at run time.
template <int PREC, int RT, int CT, int KU = 1, int ACC = -1>
__device__ __forceinline__ void superpose_lp_tile(const LpSupArgs& a, int s, int ct, uint4* lds_raw) {
  using Tr = LP<PREC>;
  using T = typename Tr::T;
  constexpr int KG = Tr::KG;
  constexpr int KT = 16 * CT;
  static_assert(W32_PANEL % KT == 0, "a column tile must lie in one workspace panel");
  T* Xs = reinterpret_cast<T*>(lds_raw);   // [KT][SK]
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int kd = 2 * Mp;
  const int SK = kd + 32 / (int)sizeof(T);   // padded by 32 bytes (see the sweep tile)

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int rb = w * 16 * RT;
  const int64_t MM2 = (int64_t)Mp * kd;
  const int nkc = kd / (KG * KU);
  // the tile's columns lie in one panel of the float32 workspace (KT divides W32_PANEL)
  const float* const Wp = a.W + (int64_t)(col0 / W32_PANEL) * a.N * W32_PANEL * Mp;
  const int cp0 = col0 % W32_PANEL;

  for (int e = tid; e < kd * KT; e += nthr) {
    const int k = e % kd, c = e / kd;
    const int col = col0 + c;
    const double v = (col < K) ? a.Xi[(int64_t)(s + 1) * Mp + k + (int64_t)col * a.ldxi] : 0.0;
    Xs[c * SK + k] = Tr::from_f((float)v);
  }

  const int64_t lane_off = (int64_t)(rb + (L & 15)) * kd + (KG / 4) * (L >> 4);
  uint4 a0[KU][RT], a1[KU][RT];
  auto loadA = [&](uint4 (&dst)[KU][RT], const T* __restrict__ Ab, int q) {
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
    for (; g + 2 < nkc; g += 2) {
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
        if (col < K) x = *reinterpret_cast<const f32x4*>(Wp + i * (W32_PANEL * Mp) + (int64_t)(cp0 + 16 * c + (L & 15)) * Mp + row0);
#pragma unroll
        for (int v = 0; v < 4; ++v) wv[t][c][v] = x[v];
      }
    }
    if (nkc - g == 2) {
      loadA(a1, Ai, g + 1);
      compute(a0, g);
      loadA(a0, Anx, 0);
      compute(a1, g + 1);
    } else {
      compute(a0, g);
      loadA(a0, Anx, 0);
    }
    if constexpr (ACC == 1 && RT <= 2) {
      // X_i += result: per row tile, all loads of X_i (unconditional), then the stores.  (With
      // four row tiles the registers are short; those take the combined loop below.)
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row0 = rb + 16 * t + 4 * (L >> 4);
        double d[CT][4];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int col = col0 + 16 * c + (L & 15);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = row0 + v < M && col < K;
            const double x = a.X[ok ? i * M + row0 + v + (int64_t)col * a.ldx : 0];
            d[c][v] = ok ? x : 0.0;
          }
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int col = col0 + 16 * c + (L & 15);
          if (col >= K) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0 + v < M)
              a.X[i * M + row0 + v + (int64_t)col * a.ldx] = d[c][v] + ((double)acc[t][c][v] + (double)wv[t][c][v]);
        }
      }
    } else {
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
              *xp = (ACC == 1 || (ACC < 0 && a.accumulate)) ? *xp + d : d;
            }
          }
        }
      }
    }
  }
}

// Float64 residual R = F - P X for diagonal A, B and tridiagonal C (a five-point stencil over the
// rows), one work-group of 256 threads: rows [q ROWS, (q+1) ROWS) of the right-hand sides
// c0 .. c0 + RES_COLS - 1 (fewer at the end).  The five coefficients of the work-group's rows stay
// in registers for all its columns; each column's x, with one block of rows on either side, is
// staged once in LDS (xs: ROWS + 2M doubles), so every neighbour is an LDS read; the next
// column's x and f are loaded into registers while the current column is computed.  The
// coefficients of absent neighbours must be zero (the plan's copies are), so the row formula has
// no branches; halo rows outside the matrix are staged as zeros.  colpart[col][q] receives the sums
// of squares of R and F over the rows (fixed order, no atomics); red holds 2 RES_COLS x 4 doubles.
// ROWS: RES_ROWS in the batched kernels, RES_ROWS_WIDE in the residual kernel of a single solve (the
// staged halo of 2M rows costs less against more rows).
template <int ROWS>
__device__ __forceinline__ void residual_cols_tile(double* __restrict__ R, int64_t ldr, const double* __restrict__ F,
                                                   int64_t ldf, const double* __restrict__ X, int64_t ldx,
                                                   const double* __restrict__ A, const double* __restrict__ B,
                                                   const double* __restrict__ C, int N, int M, int K,
                                                   double* __restrict__ colpart, int nchunk, int q, int c0,
                                                   double* xs, double (*red)[4]) {
  constexpr int RES_RPT = ROWS / 256;   // rows per thread
  constexpr int RES_SPT = RES_RPT + 4;  // staged rows per thread: ROWS + 2M with M <= 512
  const int tid = threadIdx.x;
  const int ncol = (K - c0) < RES_COLS ? (K - c0) : RES_COLS;
  const int64_t n = (int64_t)N * M;
  const int64_t g0 = (int64_t)q * ROWS;
  const int cnt = (n - g0) < ROWS ? (int)(n - g0) : ROWS;
  const int64_t jb = g0 / M;
  const unsigned rb0 = (unsigned)(g0 - jb * M);
  // own rows tid + 256 i (the tail chunk repeats its last row; those copies are not stored)
  double cd[RES_RPT], cs[RES_RPT], cu[RES_RPT], av[RES_RPT], bv[RES_RPT];
  int oc[RES_RPT];
#pragma unroll
  for (int i = 0; i < RES_RPT; ++i) {
    const int o = tid + 256 * i;
    oc[i] = o < cnt ? o : cnt - 1;
    const unsigned u = rb0 + (unsigned)oc[i];
    const unsigned jj = u / (unsigned)M;
    const unsigned r = u - jj * (unsigned)M;
    const double* t = C + (jb + jj) * 3 * M + r;
    cs[i] = t[0];
    cd[i] = t[M];
    cu[i] = t[2 * M];
    av[i] = A[g0 + oc[i]];
    bv[i] = B[g0 + oc[i]];
  }
  const int span = cnt + 2 * M;
  double xr[RES_SPT], fv[RES_RPT];
  auto load_col = [&](int c) {
    const double* x = X + (int64_t)(c0 + c) * ldx;
    const double* f = F + (int64_t)(c0 + c) * ldf;
#pragma unroll
    for (int i = 0; i < RES_RPT; ++i) fv[i] = f[g0 + oc[i]];
#pragma unroll
    for (int k = 0; k < RES_SPT; ++k) {
      const int i = tid + 256 * k;
      const int64_t g = g0 - M + i;
      xr[k] = (i < span && g >= 0 && g < n) ? x[g] : 0.0;
    }
  };
  load_col(0);
#pragma unroll 1
  for (int c = 0; c < ncol; ++c) {
#pragma unroll
    for (int k = 0; k < RES_SPT; ++k) {
      const int i = tid + 256 * k;
      if (i < span) xs[i] = xr[k];
    }
    double fc[RES_RPT];
#pragma unroll
    for (int i = 0; i < RES_RPT; ++i) fc[i] = fv[i];
    __syncthreads();
    if (c + 1 < ncol) load_col(c + 1);
    double sr = 0.0, sf = 0.0;
#pragma unroll
    for (int i = 0; i < RES_RPT; ++i) {
      const double* xp = xs + M + oc[i];
      double y = cd[i] * xp[0];
      y += cs[i] * xp[-1];
      y += cu[i] * xp[1];
      y -= av[i] * xp[-M];
      y -= bv[i] * xp[M];
      const double rv = fc[i] - y;
      if (tid + 256 * i < cnt) {
        if (R) R[g0 + oc[i] + (int64_t)(c0 + c) * ldr] = rv;
        sr += rv * rv;
        sf += fc[i] * fc[i];
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      sr += __shfl_xor(sr, off);
      sf += __shfl_xor(sf, off);
    }
    if ((tid & 63) == 0) {
      red[c][tid >> 6] = sr;
      red[RES_COLS + c][tid >> 6] = sf;
    }
    __syncthreads();   // LDS rows and partial sums are reused by the next column
  }
  if (tid < ncol) {
    double a = 0.0, b = 0.0;
    for (int v = 0; v < 4; ++v) { a += red[tid][v]; b += red[RES_COLS + tid][v]; }
    colpart[((int64_t)(c0 + tid) * nchunk + q) * 2 + 0] = a;
    colpart[((int64_t)(c0 + tid) * nchunk + q) * 2 + 1] = b;
  }
  __syncthreads();   // red is free again when the work-group goes on to other work
}

template <int RT, int CT, int KU = 2>
__device__ __forceinline__ void sweep_f64_tile(const SweepArgs& a, int s, int ct, double* In) {
  constexpr int KT = 4 * CT;
  constexpr int SB = KT + 2;

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int rb = w * 16 * RT;
  const int64_t MM = (int64_t)Mp * Mp;
  // KU = MFMA k-steps (of 4) per register chunk of the streamed matrix; nkc must be even
  // (Mp a multiple of 16 for KU = 2, of 32 for KU = 4)
  const int nkc = Mp / (4 * KU);

  // The step matrix streams through two register buffers, each loaded one chunk ahead of
  // its use; after the last chunk of a step comes the first chunk of the next step's
  // matrix.  Step order: forward rows first..last (D^{-1}), then backward rows
  // last-1..first (alpha).
  const int64_t nsteps = 2 * (last - first) + 1;
  const bool dense = a.E != nullptr;
  const double* __restrict__ fwdmat = dense ? a.E : a.Dinv;
  auto step_matrix = [&](int64_t q) -> const double* {
    return (q <= last - first) ? fwdmat + (first + q) * MM : a.alpha + (last - 1 - (q - (last - first + 1))) * MM;
  };
  const int64_t lane_off = rb + (L & 15) + (int64_t)(L >> 4) * Mp;
  double a0[KU][RT], a1[KU][RT];
  auto loadA = [&](double (&dst)[KU][RT], const double* __restrict__ Ab, int q) {
    const double* __restrict__ pa = Ab + lane_off + (int64_t)(4 * KU * q) * Mp;
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < RT; ++t) dst[u][t] = pa[16 * t + (int64_t)(4 * u) * Mp];
  };
  double acc[RT][CT];
  auto compute = [&](const double (&av)[KU][RT], int q) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int m = KU * q + u;   // rows 4m + L/16 (see lds_row)
      const double* bp = &In[(16 * (m >> 2) + 4 * (L >> 4) + (m & 3)) * SB + 2 * (L & 3)];
      double b[CT];
#pragma unroll
      for (int c = 0; c < CT; c += 2) {
        const double2 v = *reinterpret_cast<const double2*>(bp + (c >> 1) * 8);
        b[c] = v.x;
        b[c + 1] = v.y;
      }
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = mfma4(av[u][t], b[c], acc[t][c]);
    }
  };

  // first operand: F_first, or zero for the dense-A recurrence (beta_first = G_first)
  for (int e = tid; e < Mp * KT; e += nthr) {
    const int row = e % Mp, c = e / Mp;
    const int col = col0 + c;
    In[lds_row(row) * SB + lds_col<CT>(c)] = (!dense && row < M && col < K) ? a.F[first * M + row + (int64_t)col * a.ldf] : 0.0;
  }
  loadA(a0, step_matrix(0), 0);
  __syncthreads();

  for (int64_t q = 0; q < nsteps; ++q) {
    const bool fwd = q <= last - first;
    const int64_t i = fwd ? first + q : last - 1 - (q - (last - first + 1));
    const double* __restrict__ Ai = step_matrix(q);
    const double* __restrict__ Anx = (q + 1 < nsteps) ? step_matrix(q + 1) : Ai;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = 0.0;
    for (int kc = 0; kc < nkc - 2; kc += 2) {
      loadA(a1, Ai, kc + 1);
      compute(a0, kc);
      loadA(a0, Ai, kc + 2);
      compute(a1, kc + 1);
    }
    // operands of the epilogue, fetched before the last two chunks: F_{i+1} and a_{i+1}
    // (forward), G_i (forward, dense A) or beta_i (backward)
    // The loads are unconditional (lanes outside the matrix read element 0 of the source and
    // discard it): a load under a per-lane branch makes the compiler wait for every
    // outstanding load, the prefetched matrix chunks included, before the next one.
    double ex[RT][CT], an[RT];
    const bool more = fwd && i < last && !dense;
    const bool useF = fwd && !dense;
    const double* __restrict__ esrc = useF ? (more ? a.F + (i + 1) * M : a.F) : a.W + i * Mp;
    const int64_t eld = useF ? a.ldf : a.ldw;
    const int erows = useF ? (more ? M : 0) : Mp;
    const int rmax = erows > 0 ? erows - 1 : 0;   // indices clamped into the operand
    const double* __restrict__ asrc = a.adiag + (more ? (i + 1) * Mp : 0);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
      const double av = asrc[row];
      an[t] = more ? av : 0.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        const bool ok = row < erows && col < K;
        const double v = esrc[min(row, rmax) + (int64_t)min(col, K - 1) * eld];
        ex[t][c] = ok ? v : 0.0;
      }
    }
    loadA(a1, Ai, nkc - 1);
    compute(a0, nkc - 2);
    loadA(a0, Anx, 0);
    compute(a1, nkc - 1);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
      double nx[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        // forward: beta_i; next operand F_{i+1} + a_{i+1} o beta_i (or beta_last = W_last)
        // forward, dense A: beta_i = E_i beta_{i-1} + G_i; next operand beta_i
        // backward: W_i = alpha_i W_{i+1} + beta_i
        const double v = (fwd && !dense) ? acc[t][c] : acc[t][c] + ex[t][c];
        if (col < K) a.W[i * Mp + row + (int64_t)col * a.ldw] = v;
        nx[c] = more ? ex[t][c] + an[t] * v : v;
      }
      double* ip = &In[lds_row(row) * SB + 2 * out_col(L)];
#pragma unroll
      for (int c = 0; c < CT; c += 2) *reinterpret_cast<double2*>(ip + (c >> 1) * 8) = make_double2(nx[c], nx[c + 1]);
    }
    __syncthreads();
  }
}

// The Mp x 2Mp matrix [U_i V_i] streams through two register buffers of KU MFMA k-steps each,
// loaded one buffer ahead; the interface operand of the next k-step is read from LDS before
// the MFMAs of the current one, and scheduling fences keep that order (otherwise the LDS
// latency is exposed at every k-step).  KU must be even and 2 Mp / (4 KU) even.  With
// FENCED = false the compiler schedules freely (fewer live registers, for register-bound callers).
template <int RT, int CT, int KU = 2, bool FENCED = true>
__device__ __forceinline__ void superpose_f64_tile(const SupArgs& a, int s, int ct, double* Xs) {
  constexpr int KT = 4 * CT;
  constexpr int SB = KT + 2;

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = tid & 63, w = tid >> 6;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int rb = w * 16 * RT;
  const int64_t MM = (int64_t)Mp * Mp;
  const int kd = 2 * Mp;
  const int nkc = kd / (4 * KU);

  for (int e = tid; e < kd * KT; e += nthr) {
    const int k = e % kd, c = e / kd;
    const int col = col0 + c;
    Xs[lds_row(k) * SB + lds_col<CT>(c)] = (col < K) ? a.Xi[(int64_t)(s + 1) * Mp + k + (int64_t)col * a.ldxi] : 0.0;
  }

  const int64_t lane_off = rb + (L & 15) + (int64_t)(L >> 4) * Mp;
  double a0[KU][RT], a1[KU][RT];
  auto loadA = [&](double (&dst)[KU][RT], const double* __restrict__ Ab, int q) {
    const double* __restrict__ pa = Ab + lane_off + (int64_t)(4 * KU * q) * Mp;
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < RT; ++t) dst[u][t] = pa[16 * t + (int64_t)(4 * u) * Mp];
  };
  const double* Bl = &Xs[4 * (L >> 4) * SB + 2 * (L & 3)];   // block L % 4 (see lds_col, lds_row)
  double b0[CT], b1[CT];
  auto ldB = [&](double (&b)[CT], int ks) {   // rows 4 ks .. 4 ks + 3
    const double* bp = Bl + (16 * (ks >> 2) + (ks & 3)) * SB;
#pragma unroll
    for (int c = 0; c < CT; c += 2) {
      const double2 v = *reinterpret_cast<const double2*>(bp + (c >> 1) * 8);
      b[c] = v.x;
      b[c + 1] = v.y;
    }
  };
  double acc[RT][CT];
  auto mm = [&](const double (&av)[RT], const double (&b)[CT]) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = mfma4(av[t], b[c], acc[t][c]);
  };
  // k-steps KU*q .. KU*q + KU - 1; on entry b0 holds the operand of the first of them
  auto compute = [&](const double (&av)[KU][RT], int q, bool last_chunk) {
#pragma unroll
    for (int u = 0; u < KU; u += 2) {
      const int ks = KU * q + u;
      if (FENCED) {
        ldB(b1, ks + 1);
        __builtin_amdgcn_sched_barrier(0);
        mm(av[u], b0);
        __builtin_amdgcn_sched_barrier(0);
        if (!(last_chunk && u + 2 >= KU)) ldB(b0, ks + 2);
        __builtin_amdgcn_sched_barrier(0);
        mm(av[u + 1], b1);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        ldB(b0, ks);
        mm(av[u], b0);
        ldB(b0, ks + 1);
        mm(av[u + 1], b0);
      }
    }
  };

  loadA(a0, a.UV + 2 * first * MM, 0);
  __syncthreads();
  for (int64_t i = first; i <= last; ++i) {
    const double* __restrict__ Ai = a.UV + 2 * i * MM;
    const double* __restrict__ Anx = (i < last) ? Ai + 2 * MM : Ai;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = 0.0;
    if (FENCED) ldB(b0, 0);
    for (int kc = 0; kc < nkc - 2; kc += 2) {
      loadA(a1, Ai, kc + 1);
      compute(a0, kc, false);
      loadA(a0, Ai, kc + 2);
      compute(a1, kc + 1, false);
    }
    // W_i (and X_i when accumulating) fetched before the last two chunks, by unconditional
    // loads (out-of-range lanes read element 0 and discard it; see the sweep's epilogue)
    double ex[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col0 + out_col(L) * CT + c;
        const bool ok = col < K;
        const double v = a.W[ok ? i * Mp + row + (int64_t)col * a.ldw : 0];
        ex[t][c] = ok ? v : 0.0;
      }
    }
    loadA(a1, Ai, nkc - 1);
    compute(a0, nkc - 2, false);
    loadA(a0, Anx, 0);
    compute(a1, nkc - 1, true);
    if (a.accumulate) {   // X_i += result: all loads of X_i first (unconditional), then the stores
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int row = rb + 16 * t + out_row(L);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int col = col0 + out_col(L) * CT + c;
          const bool ok = row < M && col < K;
          const double v = a.X[ok ? i * M + row + (int64_t)col * a.ldx : 0];
          ex[t][c] += ok ? v : 0.0;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = rb + 16 * t + out_row(L);
      if (row < M) {
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int col = col0 + out_col(L) * CT + c;
          if (col < K) a.X[i * M + row + (int64_t)col * a.ldx] = acc[t][c] + ex[t][c];
        }
      }
    }
  }
}

// The same product for block sizes whose 2Mp x 4CT interface panel does not fit in LDS with 32
// columns: LDS holds one half of the panel at a time (the left interface's Mp rows, which multiply
// U_i, or the right interface's, which multiply V_i).  A row first multiplies the half already in
// LDS, then reloads the other half and multiplies that; the next row starts with the half now in
// LDS, so each row reloads Mp x 4CT values once (from L2: the tile's interface values are re-read
// by every row of the subdomain).  The [U_i V_i] chunks keep streaming one chunk ahead across the
// reload and across rows.
template <int RT, int CT, int KU = 2>
__device__ __forceinline__ void superpose_f64_half_tile(const SupArgs& a, int s, int ct, double* Xs) {
  constexpr int KT = 4 * CT;
  constexpr int SB = KT + 2;

  const int tid = threadIdx.x;
  const int L = tid & 63, w = tid >> 6;
  const int col0 = ct * KT;
  const int64_t first = a.ks[s] + 1, last = a.ks[s + 1] - 1;
  if (first > last) return;
  const int Mp = a.Mp, M = a.M, K = a.K;
  const int rb = w * 16 * RT;
  const int64_t MM = (int64_t)Mp * Mp;
  const int nkh = Mp / (4 * KU);   // chunks per half (even: Mp is a multiple of 64 here)

  // Xi rows (s + 1 + h) Mp .. (s + 2 + h) Mp - 1 of the tile's columns -> LDS.  The work-group has
  // Mp threads (RT = 4: Mp / 64 waves), so thread k loads row k of every column; all loads of a
  // batch are issued before its stores (columns beyond K read column K - 1 and store zero).
  static_assert(RT == 4, "one interface row per thread");
  auto load_half = [&](int h) {
    constexpr int B = 16;
    const int nv = min(KT, K - col0);   // columns of the tile below K
    const double* __restrict__ q = a.Xi + (int64_t)(s + 1 + h) * Mp + tid + (int64_t)col0 * a.ldxi;
    double* dst = Xs + lds_row(tid) * SB;
    if (nv == KT) {
#pragma unroll
      for (int c0 = 0; c0 < KT; c0 += B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          v[u] = *q;
          q += a.ldxi;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) dst[lds_col<CT>(c0 + u)] = v[u];
      }
    } else {   // the last, ragged column tile
#pragma unroll 1
      for (int c = 0; c < KT; ++c) dst[lds_col<CT>(c)] = c < nv ? q[(int64_t)c * a.ldxi] : 0.0;
    }
  };

  const int64_t lane_off = rb + (L & 15) + (int64_t)(L >> 4) * Mp;
  double a0[KU][RT], a1[KU][RT];
  auto loadA = [&](double (&dst)[KU][RT], const double* __restrict__ Ab, int q) {
    const double* __restrict__ pa = Ab + lane_off + (int64_t)(4 * KU * q) * Mp;
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < RT; ++t) dst[u][t] = pa[16 * t + (int64_t)(4 * u) * Mp];
  };
  const double* Bl = &Xs[4 * (L >> 4) * SB + 2 * (L & 3)];   // block L % 4 (see lds_col, lds_row)
  double b0[CT], b1[CT];
  auto ldB = [&](double (&b)[CT], int ks) {   // rows 4 ks .. 4 ks + 3 of the half in LDS
    const double* bp = Bl + (16 * (ks >> 2) + (ks & 3)) * SB;
#pragma unroll
    for (int c = 0; c < CT; c += 2) {
      const double2 v = *reinterpret_cast<const double2*>(bp + (c >> 1) * 8);
      b[c] = v.x;
      b[c + 1] = v.y;
    }
  };
  double acc[RT][CT];
  auto mm = [&](const double (&av)[RT], const double (&b)[CT]) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = mfma4(av[t], b[c], acc[t][c]);
  };
  // k-steps KU*q .. KU*q + KU - 1 of the half; on entry b0 holds the operand of the first of them
  auto compute = [&](const double (&av)[KU][RT], int q, bool last_chunk) {
#pragma unroll
    for (int u = 0; u < KU; u += 2) {
      const int ks = KU * q + u;
      ldB(b1, ks + 1);
      __builtin_amdgcn_sched_barrier(0);
      mm(av[u], b0);
      __builtin_amdgcn_sched_barrier(0);
      if (!(last_chunk && u + 2 >= KU)) ldB(b0, ks + 2);
      __builtin_amdgcn_sched_barrier(0);
      mm(av[u + 1], b1);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // all chunks of one half but the last two; a0 holds chunk 0 on entry
  auto body = [&](const double* __restrict__ Ah) {
    ldB(b0, 0);
    for (int kc = 0; kc < nkh - 2; kc += 2) {
      loadA(a1, Ah, kc + 1);
      compute(a0, kc, false);
      loadA(a0, Ah, kc + 2);
      compute(a1, kc + 1, false);
    }
  };

  int cur = 0;   // the half in LDS
  load_half(0);
  loadA(a0, a.UV + 2 * first * MM, 0);
  __syncthreads();
  for (int64_t i = first; i <= last; ++i) {
    const double* __restrict__ Ai = a.UV + 2 * i * MM;
    const double* __restrict__ Anx = (i < last) ? Ai + 2 * MM : Ai;
    const int nxt = 1 - cur;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][c] = 0.0;
    // the half in LDS; the last chunk prefetches chunk 0 of the other half of this row
    {
      const double* __restrict__ Ah = Ai + cur * MM;
      body(Ah);
      loadA(a1, Ah, nkh - 1);
      compute(a0, nkh - 2, false);
      loadA(a0, Ai + nxt * MM, 0);
      compute(a1, nkh - 1, true);
    }
    __syncthreads();   // every wave is done reading this half
    load_half(nxt);
    __syncthreads();
    // the other half; the last chunk prefetches chunk 0 of the same half of the next row
    const double* __restrict__ Ah = Ai + nxt * MM;
    body(Ah);
    // W_i fetched before the last two chunks by unconditional loads:
    // one address per column (rows 16 t apart are immediate offsets from it); a lane whose column
    // is beyond K reads column min(lcol, K - 1) and discards the value
    double ex[RT][CT];
    const int lcol = col0 + out_col(L) * CT;              // the lane's first column
    const int orow = rb + out_row(L);
    {
      const double* __restrict__ pw0 = a.W + i * Mp + orow + (int64_t)min(lcol, K - 1) * a.ldw;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const bool ok = lcol + c < K;
        const double* __restrict__ pw = pw0 + (ok ? (int64_t)c * a.ldw : 0);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const double v = pw[16 * t];
          ex[t][c] = ok ? v : 0.0;
        }
      }
    }
    loadA(a1, Ah, nkh - 1);
    compute(a0, nkh - 2, false);
    loadA(a0, Anx + nxt * MM, 0);
    compute(a1, nkh - 1, true);
    double* __restrict__ px0 = a.X + i * M + orow + (int64_t)lcol * a.ldx;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      if (lcol + c < K) {
        double* __restrict__ px = px0 + (int64_t)c * a.ldx;
#pragma unroll
        for (int t = 0; t < RT; ++t)
          if (orow + 16 * t < M) px[16 * t] = acc[t][c] + ex[t][c];
      }
    }
    cur = nxt;
  }
}

}  // namespace td
