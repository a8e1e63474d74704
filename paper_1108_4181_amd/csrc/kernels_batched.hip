// Batched solve: many independent block-tridiagonal systems of uneven N, M, K.  The host builds
// one work list of all systems' items in stage order; it runs either as one launch per stage
// (k_batched_stage: the items of a stage are independent, kernel boundaries order the stages)
// or as one persistent launch (k_batched): each work-group repeatedly takes the next work item
// from a global counter; items are queued in a topological order (every dependency of an item
// sits earlier in the queue), so a work-group that waits only waits for items already held by
// running work-groups and the launch always drains.  Every wait is bounded: on time-out the item
// records an error and runs anyway, and all other waits then end at once.
//
// Per system and per pass (pass 0 solves with F; later passes solve with the residual and add
// the correction to X):
//   sweep (subdomain, column tile) -> interface right-hand side (chunks) -> dichotomy partial sums
//   -> dichotomy levels -> superposition (subdomain, column tile) -> float64 residual (chunks)
//   -> residual test (one item: max column relative residual; marks the system converged).
// Items of a pass that follows the pass in which the system converged do no work.
#include "internal.h"
#include "tile_bodies.h"

namespace td {

constexpr int BATCH_THREADS = 256;
constexpr int FT_CHUNK = 16384;       // elements of the interface right-hand side per item

__device__ __forceinline__ bool wait_counter(const int32_t* c, int32_t need, int32_t* err, int64_t limit) {
  int64_t spins = 0;
  while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (++spins > limit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

template <int RT>
// kept out of line: the three instances inlined into one kernel would share one register budget
__device__ __attribute__((noinline)) void run_item(const BatchItem& it, const BatchSys& S, uint4* lds, double (*red)[4],
                                                   int32_t* conv) {
  const int tid = threadIdx.x;
  switch (it.type) {
    case BI_SWEEP: {
      if (S.prec == 0) {
        SweepArgs a = S.sweep64;
        if (it.pass > 0) { a.F = S.R; a.ldf = S.ldr; }
        sweep_f64_tile<RT, 4>(a, it.i0, it.i1, reinterpret_cast<double*>(lds));
      } else {
        LpSweepArgs a = S.sweep;
        if (it.pass > 0) { a.F = S.R; a.ldf = S.ldr; }
        sweep_lp_tile<1, RT, 2>(a, it.i0, it.i1, lds);
      }
      break;
    }
    case BI_FTILDE: {
      const double* F = it.pass > 0 ? S.R : S.F;
      const int64_t ldf = it.pass > 0 ? S.ldr : S.ldf;
      const int64_t n = (int64_t)S.p * S.Mp * S.K;
      const int64_t e0 = (int64_t)it.i0 * FT_CHUNK;
      const int64_t e1 = e0 + FT_CHUNK < n ? e0 + FT_CHUNK : n;
      const int64_t* ks = S.sweep.ks;
      const float* W32 = S.sweep.W;
      const double* W64 = S.sweep64.W;
      const int64_t ldw = S.sweep64.ldw;   // float64 workspace; the float32 one uses w32_off
      for (int64_t e = e0 + tid; e < e1; e += BATCH_THREADS) {
        const int r = (int)(e % S.Mp);
        const int64_t sc = e / S.Mp;
        const int s = (int)(sc % S.p);
        const int64_t col = sc / S.p;
        const int64_t k = ks[s];
        double v = (r < S.M) ? F[k * S.M + r + col * ldf] : 0.0;
        if (s > 0 && k - 1 > ks[s - 1]) {
          const double wv = S.prec == 0 ? W64[(k - 1) * S.Mp + r + col * ldw] : (double)W32[w32_off(S.N, S.Mp, k - 1, r, col)];
          v += S.adiag[k * S.Mp + r] * wv;
        }
        if (k + 1 < ks[s + 1]) {
          const double wv = S.prec == 0 ? W64[(k + 1) * S.Mp + r + col * ldw] : (double)W32[w32_off(S.N, S.Mp, k + 1, r, col)];
          v += S.bdiag[k * S.Mp + r] * wv;
        }
        S.Ft[(int64_t)s * S.Mp + r + col * S.ldft] = v;
      }
      break;
    }
    case BI_PART:
      bgemm_tile<RT, 4>(S.part, it.i0, it.i1, reinterpret_cast<double*>(lds));
      break;
    case BI_LEVEL: {
      BArgs b = S.lev[it.lvl];
      b.x2accum = it.pass > 0 ? 1 : 0;
      bgemm_tile<RT, 4>(b, it.i0, it.i1, reinterpret_cast<double*>(lds));
      break;
    }
    case BI_SUP: {
      if (S.prec == 0) {
        SupArgs u = S.sup64;
        u.accumulate = it.pass > 0 ? 1 : 0;
        superpose_f64_tile<RT, 4, 2, false>(u, it.i0, it.i1, reinterpret_cast<double*>(lds));
      } else {
        LpSupArgs u = S.sup;
        u.accumulate = it.pass > 0 ? 1 : 0;
        superpose_lp_tile<1, RT, 2>(u, it.i0, it.i1, lds);
      }
      break;
    }
    case BI_RES:
      residual_cols_tile<RES_ROWS>(S.R, S.ldr, S.F, S.ldf, S.X, S.ldx, S.cA, S.cB, S.cC, S.N, S.M, S.K, S.colpart, S.nchunk,
                         it.i0, it.i1, reinterpret_cast<double*>(lds), red);
      break;
    case BI_RFIN: {
      double worst = 0.0;
      for (int col = tid; col < S.K; col += BATCH_THREADS) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < S.nchunk; ++q) {
          a += S.colpart[((int64_t)col * S.nchunk + q) * 2 + 0];
          b += S.colpart[((int64_t)col * S.nchunk + q) * 2 + 1];
        }
        const double rel = (b > 0.0) ? sqrt(a / b) : (a > 0.0 ? INFINITY : 0.0);
        if (!(rel <= worst)) worst = rel;   // NaN propagates
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(worst, off);
        if (!(o <= worst)) worst = o;
      }
      if ((tid & 63) == 0) red[0][tid >> 6] = worst;
      __syncthreads();
      if (tid == 0) {
        double w = red[0][0];
        for (int v = 1; v < BATCH_THREADS / 64; ++v)
          if (!(red[0][v] <= w)) w = red[0][v];
        S.resid[it.pass] = w;
        if (w <= S.tol && conv[it.sys] > it.pass) conv[it.sys] = it.pass;
      }
      break;
    }
  }
}

__global__ void __launch_bounds__(BATCH_THREADS, 2) k_batched(const BatchItem* __restrict__ items, int nitems,
                                                           const BatchSys* __restrict__ sys, int32_t* counters,
                                                           int32_t* conv, BatchCtl* ctl, int64_t spin_limit) {
  extern __shared__ uint4 lds[];
  __shared__ double red[2 * RES_COLS][4];
  __shared__ int sh_idx, sh_ok;
  for (;;) {
    if (threadIdx.x == 0) sh_idx = atomicAdd(&ctl->head, 1);
    __syncthreads();
    const int idx = sh_idx;
    if (idx >= nitems) break;
    const BatchItem it = items[idx];
    // thread 0's agent-scope acquire (in the wait) invalidates this CU's L1 and the XCD's L2 for
    // every wave of the work-group; the barrier orders the other waves after it
    if (threadIdx.x == 0) sh_ok = (it.dep < 0) ? 1 : (wait_counter(counters + it.dep, it.need, &ctl->error, spin_limit) ? 1 : 0);
    __syncthreads();
    const BatchSys& S = sys[it.sys];
    const bool skip = it.pass > 0 && __hip_atomic_load(conv + it.sys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < it.pass;
    if (!skip) {
      switch (S.rt) {
        case 4: run_item<4>(it, S, lds, red, conv); break;
        case 2: run_item<2>(it, S, lds, red, conv); break;
        default: run_item<1>(it, S, lds, red, conv); break;
      }
    }
    // every wave's stores complete (workgroup release), then one agent-scope release (L2 write-back)
    // and the count
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(counters + it.mine, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    (void)sh_ok;
  }
}

__global__ void k_batch_reset(int32_t* counters, int ncounters, int32_t* conv, int nsys, BatchCtl* ctl);

// Stage-synchronous form: one launch per stage (all systems' items of that stage, which are
// mutually independent); kernel boundaries order the stages, so items neither wait nor count.
__global__ void __launch_bounds__(BATCH_THREADS, 2) k_batched_stage(const BatchItem* __restrict__ items, int begin,
                                                                 int end, const BatchSys* __restrict__ sys,
                                                                 int32_t* conv, int32_t* head) {
  extern __shared__ uint4 lds[];
  __shared__ double red[2 * RES_COLS][4];
  __shared__ int sh_idx;
  for (;;) {
    if (threadIdx.x == 0) sh_idx = begin + atomicAdd(head, 1);
    __syncthreads();
    const int idx = sh_idx;
    if (idx >= end) break;
    const BatchItem it = items[idx];
    const BatchSys& S = sys[it.sys];
    const bool skip = it.pass > 0 && conv[it.sys] < it.pass;
    if (!skip) {
      switch (S.rt) {
        case 4: run_item<4>(it, S, lds, red, conv); break;
        case 2: run_item<2>(it, S, lds, red, conv); break;
        default: run_item<1>(it, S, lds, red, conv); break;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_batched_stages(const BatchItem* items, const int* stage_begin, int nstages, const BatchSys* sys,
                                 int32_t* heads, int32_t* conv, int nsys, BatchCtl* ctl, int max_grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(64), dim3(256), 0, st, heads, nstages, conv, nsys, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int lds = batched_lds_bytes();
  e = hipFuncSetAttribute((const void*)k_batched_stage, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  for (int s = 0; s < nstages; ++s) {
    const int n = stage_begin[s + 1] - stage_begin[s];
    if (n <= 0) continue;
    const int grid = n < max_grid ? n : max_grid;
    hipLaunchKernelGGL(k_batched_stage, dim3(grid), dim3(BATCH_THREADS), lds, st, items, stage_begin[s],
                       stage_begin[s + 1], sys, conv, heads + s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_batch_reset(int32_t* counters, int ncounters, int32_t* conv, int nsys, BatchCtl* ctl) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ncounters; e += gridDim.x * blockDim.x) counters[e] = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nsys; e += gridDim.x * blockDim.x) conv[e] = 1 << 30;
  if (blockIdx.x == 0 && threadIdx.x == 0) { ctl->head = 0; ctl->error = 0; }
}

// LDS of the largest tile body: float64 superposition with 16 columns of 2*256 rows
// (float64 sweep: 256 x 18 doubles; float32 superposition: 32 x (2*256 + 4) floats)
int batched_lds_bytes() { return 2 * 256 * 18 * 8; }

// resident work-groups of the persistent kernel per compute unit (registers and LDS permitting)
int batched_blocks_per_cu() {
  int occ = 0;
  if (hipFuncSetAttribute((const void*)k_batched, hipFuncAttributeMaxDynamicSharedMemorySize, batched_lds_bytes()) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_batched, BATCH_THREADS, batched_lds_bytes()) !=
          hipSuccess)
    return 1;
  return occ < 1 ? 1 : occ;
}

hipError_t launch_batched(const BatchItem* items, int nitems, const BatchSys* sys, int32_t* counters, int ncounters,
                          int32_t* conv, int nsys, BatchCtl* ctl, int grid, int64_t spin_limit, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(64), dim3(256), 0, st, counters, ncounters, conv, nsys, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int lds = batched_lds_bytes();
  e = hipFuncSetAttribute((const void*)k_batched, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batched, dim3(grid), dim3(BATCH_THREADS), lds, st, items, nitems, sys, counters, conv, ctl,
                     spin_limit);
  return hipGetLastError();
}

}  // namespace td
