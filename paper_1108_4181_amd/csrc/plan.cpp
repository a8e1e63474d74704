// Host side of the block-tridiagonal solver: argument checks, the subdomain
// partition, the dichotomy tree, device memory, and the order of the kernel
// launches of the factor (Algorithm 2, step 1, Sec. 2.2) and of the solve
// (Algorithm 2, step 2).  Implements the C ABI of include/tridiag.h.
#include "internal.h"
#include "tridiag.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace td;

namespace {

thread_local std::string g_err;

td_status fail(td_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipFail {
  hipError_t e;
  std::string where;
};

#define HIPCHK(x)                                                            \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) throw HipFail{e_, std::string(#x) + " @" + std::to_string(__LINE__)}; \
  } while (0)

struct Node {
  int l, r, m, level;
  int64_t g_off;        // offset of G (Mp x len*Mp) in the G buffer
  int chunk0, nchunk;   // partial-sum chunks of this node
};

// events of one profiled solve: [0..5] stage boundaries, [6] start, [7] end
struct StageEvents {
  hipEvent_t ev[8] = {};
};

}  // namespace

// error text for the library's other host source files
td_status td_set_error(td_status s, const char* msg) { return fail(s, msg ? msg : ""); }

struct td_plan_s {
  int64_t N = 0, M = 0, Mp = 0, p = 0;
  int fmtA = 1, fmtB = 1, fmtC = 2, prec = 0, adjoint = 0;
  std::vector<int64_t> ks;  // p + 1
  int64_t* d_ks = nullptr;
  // compact float64 copies of the input (user layout) for residuals
  double* cA = nullptr; double* cB = nullptr; double* cC = nullptr;
  double* adiag = nullptr; double* bdiag = nullptr;  // [N][Mp], a_0 = 0, b_{N-1} = 0 (zero when dense)
  // dense A or B (float64 plans): every coupling term is a block product
  bool dense = false;
  double* ABd = nullptr;      // [N][A_j | B_j], Mp x 2Mp each, zero padded
  double* E = nullptr;        // [N][Mp][Mp]: E_i = D_i^{-1} A_i
  BDesc* d_gf = nullptr; int n_gf = 0;     // G_i = D_i^{-1} F_i for every interior row
  BDesc* d_ftd = nullptr; int n_ftd = 0;   // interface right-hand side coupling products
  // factor
  double* Dinv = nullptr;     // [N][Mp][Mp]
  double* alpha = nullptr;    // [N][Mp][Mp]
  double* UVa = nullptr;      // [Ident | Zero | (U_i, V_i) for i < N]
  double* red = nullptr;      // [At | Ct | Bt], each [p][Mp][Mp]
  double* G = nullptr;        // dichotomy rows of the inverse
  double* H = nullptr;        // [nodes][H^L | H^R]
  double* chain_inv = nullptr;  // the tree's chain inverses and G_m, kept for the transposed plan's factor
  std::vector<Node> nodes;
  int depth = 0;
  int nchunks = 0;
  // solve descriptors (device)
  BDesc* d_part = nullptr; int n_part = 0;
  BDesc* d_corr = nullptr; std::vector<int> corr_begin, corr_count;
  // levels with few nodes: slab products (d_split) + combine (d_comb); lev_nslab[lv] == 1 = unsplit
  std::vector<int> lev_nslab, split_begin, split_count, comb_begin;
  BDesc* d_split = nullptr; CombDesc* d_comb = nullptr;
  int pslots = 0;             // slab partials of the largest split level
  // workspace
  int64_t kcap = 0;
  double* Wbuf = nullptr; double* Ft = nullptr; double* Xi = nullptr; double* Sp = nullptr;
  double* Pbuf = nullptr;     // [pslots][Mp] x K slab partials of a split level
  float* W32 = nullptr;       // float32 beta / W of the low-precision sweeps
  int64_t rcap = 0;
  double* Rbuf = nullptr; double* colpart = nullptr; double* norms = nullptr;
  // low-precision copies of the factor (sweep_prec F32 / BF16), row-major
  void* Dlp = nullptr; void* Alp = nullptr; void* UVlp = nullptr;
  // scalar plan (block size 1, every row an interface row): Algorithm 1 on the tridiagonal system
  bool scalar = false;
  ScalarArgs sc{};            // tree arrays and factor; the per-solve fields are set by each pass
  td_tiles tiles{};           // launch shapes of the sweeps and the superposition (0 = the rules)
  bool first_pass = false;
  int32_t* d_flag = nullptr;
  td_plan_s* adj = nullptr;
  bool prof = false;
  std::vector<StageEvents> evsets;  // one set per profiled solve since the last read-out
  int prof_n = 0;
  StageEvents* se = nullptr;        // set of the solve in progress
  double factor_ms = 0.0;
  int64_t bytes = 0;                                   // device memory held now
  std::vector<std::pair<void*, int64_t>> allocs;       // (pointer, bytes)
  hipStream_t last_stream = nullptr;

  // device memory: the caller's callbacks (td_desc.dev_alloc / dev_free) or hipMalloc / hipFree
  td_alloc_fn ualloc = nullptr;
  td_free_fn ufree = nullptr;
  void* uctx = nullptr;
  hipStream_t astream = nullptr;   // stream of the call in progress (passed to the callbacks)
  void* raw_alloc(size_t nb) {
    void* p = nullptr;
    nb = std::max<size_t>(nb, 256);
    if (ualloc) {
      p = ualloc(uctx, nb, (void*)astream);
      if (!p) throw HipFail{hipErrorOutOfMemory, "dev_alloc callback (" + std::to_string(nb) + " bytes)"};
    } else {
      HIPCHK(hipMalloc(&p, nb));
    }
    return p;
  }
  void raw_free(void* p) {
    if (!p) return;
    if (ufree) ufree(uctx, p, (void*)astream);
    else (void)hipFree(p);
  }
  double* alloc(int64_t n_doubles) {
    if (n_doubles <= 0) n_doubles = 1;
    void* p = raw_alloc((size_t)n_doubles * sizeof(double));
    allocs.emplace_back(p, n_doubles * (int64_t)sizeof(double));
    bytes += n_doubles * (int64_t)sizeof(double);
    return (double*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    size_t nb = std::max<size_t>(1, v.size()) * sizeof(T);
    void* p = raw_alloc(nb);
    allocs.emplace_back(p, (int64_t)nb);
    bytes += (int64_t)nb;
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return (T*)p;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find_if(allocs.begin(), allocs.end(), [p](const std::pair<void*, int64_t>& a) { return a.first == p; });
    if (it != allocs.end()) {
      bytes -= it->second;
      allocs.erase(it);
    }
    raw_free(p);
  }
  // the last plain solve (no refinement, no report, not profiled), captured as a HIP graph and
  // replayed while the arguments and the workspace stay the same
  struct {
    const double* F = nullptr; int64_t ldf = 0;
    double* X = nullptr; int64_t ldx = 0;
    int64_t K = 0, ws_gen = -1;
    hipGraph_t g = nullptr; hipGraphExec_t ex = nullptr;
  } sg;
  int64_t ws_gen = 0;           // incremented whenever the solve workspace is reallocated
  void drop_graph() {
    if (sg.ex) (void)hipGraphExecDestroy(sg.ex);
    if (sg.g) (void)hipGraphDestroy(sg.g);
    sg.ex = nullptr; sg.g = nullptr; sg.F = nullptr; sg.X = nullptr; sg.ws_gen = -1;
  }
  ~td_plan_s() {
    drop_graph();
    for (auto& a : allocs) raw_free(a.first);
    for (auto& s : evsets)
      for (auto& e : s.ev) (void)hipEventDestroy(e);
    delete adj;
  }
};

namespace {

// Block size padded for the kernels' wave tiling: at most 8 waves of 16, 32 or 64 rows each.
int64_t pad_block(int64_t m, int prec) {
  int64_t mp;
  if (m <= 128) mp = (m + 15) / 16 * 16;
  else if (m <= 256) mp = (m + 31) / 32 * 32;
  else mp = (m + 63) / 64 * 64;
  if (prec == TD_PREC_BF16 && mp % 32 != 0) mp += 16;  // bfloat16 k-groups are 32 deep
  return mp;
}

std::vector<int64_t> partition(int64_t N, int64_t p) {
  // interface rows: the first N mod p subdomains get ceil(N/p) rows
  std::vector<int64_t> ks(p + 1);
  const int64_t base = N / p, extra = N % p;
  int64_t k = 0;
  for (int64_t s = 0; s < p; ++s) {
    ks[s] = k;
    k += base + (s < extra ? 1 : 0);
  }
  ks[p] = N;
  return ks;
}

// dichotomy tree over rows [l, r] of the reduced system: split row m = floor((l+r)/2)
void build_tree(std::vector<Node>& nodes, int l, int r, int level, int& depth) {
  const int m = (l + r) / 2;
  nodes.push_back(Node{l, r, m, level, 0, 0, 0});
  depth = std::max(depth, level + 1);
  if (m > l) build_tree(nodes, l, m - 1, level + 1, depth);
  if (m < r) build_tree(nodes, m + 1, r, level + 1, depth);
}

BArgs bargs_base(int Mp) {
  BArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Mp = Mp;
  a.alpha = 1.0;
  return a;
}

BDesc desc0() {
  BDesc d;
  std::memset(&d, 0, sizeof(d));
  return d;
}

// Descriptor lists of the factor's launches: copied into chunks of pinned host memory and sent with
// asynchronous copies into device chunks (from the plan's allocator), so that building a list never
// waits for the device; between begin_batch and end_batch the lists are only staged, and end_batch
// sends all of them in one copy (before the launches that read them).  Each piece of a chunk is
// written once; the chunks are released when the pool goes out of scope, after the stream has
// finished with them.
struct DescPool {
  struct Chunk {
    char* host;
    char* dev;
    size_t cap, used;
  };
  td_plan_s* P;
  hipStream_t st;
  std::vector<Chunk> chunks;
  size_t sent = 0;        // bytes of the last chunk already sent to the device
  bool batch = false;     // between begin_batch and end_batch: stage lists, send them in one copy
  DescPool(td_plan_s* plan, hipStream_t s) : P(plan), st(s) {}
  DescPool(const DescPool&) = delete;
  DescPool& operator=(const DescPool&) = delete;
  // One copy of the lists staged since the last one (the caller's launches that read them come after).
  void flush() {
    if (chunks.empty()) return;
    Chunk& c = chunks.back();
    if (c.used > sent) HIPCHK(hipMemcpyAsync(c.dev + sent, c.host + sent, c.used - sent, hipMemcpyHostToDevice, st));
    sent = c.used;
  }
  void begin_batch() { batch = true; }
  void end_batch() {
    flush();
    batch = false;
  }
  void* put_bytes(const void* src, size_t nb) {
    const size_t need = (std::max<size_t>(nb, 1) + 255) & ~(size_t)255;
    if (chunks.empty() || chunks.back().used + need > chunks.back().cap) {
      flush();
      sent = 0;
      Chunk c{};
      c.cap = std::max<size_t>(need, (size_t)4 << 20);
      HIPCHK(hipHostMalloc((void**)&c.host, c.cap, hipHostMallocDefault));
      try {
        c.dev = (char*)P->raw_alloc(c.cap);
      } catch (...) {
        (void)hipHostFree(c.host);
        throw;
      }
      chunks.push_back(c);
    }
    Chunk& c = chunks.back();
    void* d = c.dev + c.used;
    if (nb) std::memcpy(c.host + c.used, src, nb);
    c.used += need;
    if (!batch) flush();
    return d;
  }
  template <class T>
  T* put_vec(const std::vector<T>& v) {
    return (T*)put_bytes(v.data(), v.size() * sizeof(T));
  }
  BDesc* put(const std::vector<BDesc>& v) { return put_vec(v); }
  ~DescPool() {
    if (chunks.empty()) return;
    (void)hipStreamSynchronize(st);
    for (auto& c : chunks) {
      P->raw_free(c.dev);
      (void)hipHostFree(c.host);
    }
  }
};

// the largest of 64, 32 and 16 that divides every descriptor's inner dimension and segment rows
int kalign_of(const std::vector<BDesc>& d) {
  int a = 64;
  for (const BDesc& x : d)
    while (a > 16 && ((x.kd % a) != 0 || (x.segrows % a) != 0)) a >>= 1;
  return a;
}

// d already on the device at staged (DescPool batch)
void run_bgemm(BArgs a, const std::vector<BDesc>& d, const BDesc* staged, hipStream_t st) {
  if (d.empty()) return;
  a.descs = staged;
  a.nprob = (int32_t)d.size();
  a.kalign = kalign_of(d);
  HIPCHK(launch_bgemm(a, st));
}

void run_bgemm(BArgs a, const std::vector<BDesc>& d, DescPool& pool, hipStream_t st) {
  if (d.empty()) return;
  run_bgemm(a, d, pool.put(d), st);
}

// Default subdomain count (tridiag_default_subdomains): the longest of 32, 16 and 8 rows per subdomain
// that still gives the sweeps about 512 work-groups (one per subdomain and 32-column tile).
int64_t default_subdomains(int64_t N, int64_t K) {
  if (K <= 0) K = 512;
  const int64_t tiles = std::max<int64_t>(1, (K + 31) / 32);
  int64_t L = 8;
  for (int64_t cand : {32, 16})
    if ((N / cand) * tiles >= 512) {
      L = cand;
      break;
    }
  return std::max<int64_t>(1, std::min<int64_t>(N, N / L));
}

// ------------------------------------------------------------------------------------------
// Factor: Algorithm 2, step 1 (sub-problems (sub1), (sub2); reduced matrix (red1); rows of the
// inverse of the reduced matrix for Algorithm 1).
// ------------------------------------------------------------------------------------------
// fwd (optional): P is the transposed plan of the factored plan fwd (same partition, diagonal
// couplings): its compact inputs are transposed on the device from fwd's, and its subdomain block
// inverses are the transposes of fwd's (no elimination of its own); the rest is factored as usual.
void factor_impl(td_plan_s* P, const double* A, const double* B, const double* C, hipStream_t st,
                 const td_plan_s* fwd = nullptr, bool keep_chain = false) {
  const int64_t N = P->N, M = P->M, Mp = P->Mp, p = P->p;
  const int64_t MM = Mp * Mp;
  const auto& ks = P->ks;
  DescPool pool(P, st);

  // compact copies of the input
  const int64_t nA = (P->fmtA == TD_FMT_DIAG) ? N * M : N * M * M;
  const int64_t nB = (P->fmtB == TD_FMT_DIAG) ? N * M : N * M * M;
  const int64_t nC = (P->fmtC == TD_FMT_TRIDIAG) ? N * 3 * M : N * M * M;
  P->cA = P->alloc(nA);
  P->cB = P->alloc(nB);
  P->cC = P->alloc(nC);
  if (fwd) {
    HIPCHK(launch_transpose_inputs(P->cA, P->cB, P->cC, fwd->cA, fwd->fmtA, fwd->cB, fwd->fmtB, fwd->cC, fwd->fmtC,
                                   (int)N, (int)M, st));
  } else {
    HIPCHK(hipMemcpyAsync(P->cA, A, nA * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(P->cB, B, nB * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(P->cC, C, nC * 8, hipMemcpyDeviceToDevice, st));
  }
  if (P->fmtA == TD_FMT_DIAG && P->fmtB == TD_FMT_DIAG && P->fmtC == TD_FMT_TRIDIAG)
    HIPCHK(launch_zero_absent(P->cA, P->cB, P->cC, (int)N, (int)M, st));   // for the stencil residual
  P->adiag = P->alloc(N * Mp);
  P->bdiag = P->alloc(N * Mp);
  P->dense = (P->fmtA == TD_FMT_DENSE || P->fmtB == TD_FMT_DENSE);
  if (P->dense) {
    // the diagonal-coupling kernels then see zero couplings; the block products below add them
    HIPCHK(launch_fill(P->adiag, N * Mp, 0.0, st));
    HIPCHK(launch_fill(P->bdiag, N * Mp, 0.0, st));
    P->ABd = P->alloc(N * 2 * MM);
    HIPCHK(launch_expand_AB(P->ABd, P->cA, P->fmtA, P->cB, P->fmtB, (int)N, (int)M, (int)Mp, st));
    P->E = P->alloc(N * MM);
  } else {
    HIPCHK(launch_pad_diag(P->adiag, P->cA, (int)N, (int)M, (int)Mp, 1, 0, st));
    HIPCHK(launch_pad_diag(P->bdiag, P->cB, (int)N, (int)M, (int)Mp, 0, 1, st));
  }
  P->d_ks = P->upload(ks);
  P->d_flag = (int32_t*)P->alloc(2);

  P->Dinv = P->alloc(N * MM);
  P->alpha = P->alloc(N * MM);
  P->UVa = P->alloc((2 + 2 * N) * MM);
  double* Ident = P->UVa;
  HIPCHK(launch_identity(Ident, (int)Mp, st));
  HIPCHK(launch_fill(P->UVa + MM, MM, 0.0, st));
  // Gamma arena: [Ident | Gamma_i for i < N]
  double* Ga = P->alloc((1 + N) * MM);
  HIPCHK(launch_identity(Ga, (int)Mp, st));
  double* Dwork = P->alloc(p * MM);
  // Gauss-Jordan scratch for up to 2p matrices per launch (the tree's chain steps invert a left and
  // a right chain matrix of each of its p nodes): pivot rows, smallest pivots, partial row sums
  const int64_t gj_part = (Mp + 31) / 32 * Mp;
  double* gjs = P->alloc(p * Mp + 2 * p + 2 * p * gj_part);
  auto gj_scratch = [&](GJArgs& g) {
    if (g.nmat > 2 * p) throw std::string("internal error: Gauss-Jordan scratch too small");
    g.piv = reinterpret_cast<int32_t*>(gjs);
    g.pmin = gjs + p * Mp;
    g.part = gjs + p * Mp + 2 * p;
  };

  int32_t* bad = P->d_flag;
  HIPCHK(launch_negate_fill_check(bad, INT_MAX, st));

  std::vector<int64_t> nint(p);
  int64_t maxn = 0;
  for (int64_t s = 0; s < p; ++s) {
    nint[s] = ks[s + 1] - ks[s] - 1;
    maxn = std::max(maxn, nint[s]);
  }

  const bool reuse = fwd != nullptr && !P->dense;
  if (reuse) {   // D'_i^{-1} = (D_i^{-1})^T and alpha'_i for every interior row at once
    std::vector<int64_t> rows;
    for (int64_t s = 0; s < p; ++s)
      for (int64_t i = ks[s] + 1; i < ks[s + 1]; ++i) rows.push_back(i);
    HIPCHK(launch_transpose_scale(P->Dinv, P->alpha, fwd->Dinv, P->bdiag, pool.put_vec(rows), (int)rows.size(),
                                  (int)Mp, st));
  }

  // ---- forward elimination inside every subdomain: D_i, D_i^{-1}, alpha_i, Gamma_i
  for (int64_t t = 0; t < maxn; ++t) {
    std::vector<int64_t> rows, outoff, bdoff;
    std::vector<int32_t> first, tag;
    std::vector<BDesc> gam;
    for (int64_t s = 0; s < p; ++s) {
      if (nint[s] <= t) continue;
      const int64_t i = ks[s] + 1 + t;
      rows.push_back(i);
      first.push_back(t == 0 ? 1 : 0);
      outoff.push_back(i * MM);
      bdoff.push_back(i * Mp);
      tag.push_back((int32_t)i);
      BDesc d = desc0();
      d.a_off = i * MM;                              // D_i^{-1}
      d.b_off = (t == 0) ? 0 : (1 + (i - 1)) * MM;   // Gamma_{i-1} (identity at the interface)
      d.bs_off = i * Mp;                             // rows scaled by a_i
      d.c_off = (1 + i) * MM;                        // Gamma_i
      d.kd = (int32_t)Mp;
      d.segrows = (int32_t)Mp;
      gam.push_back(d);
    }
    const int nm = (int)rows.size();
    std::vector<BDesc> da, dal, de;
    if (!reuse && P->dense && t > 0) {   // D_i -= A_i alpha_{i-1}
      for (int q = 0; q < nm; ++q) {
        const int64_t i = rows[q];
        BDesc d = desc0();
        d.a_off = i * 2 * MM;
        d.b_off = (i - 1) * MM;
        d.c_off = d.cin_off = q * MM;
        d.kd = d.segrows = (int32_t)Mp;
        da.push_back(d);
      }
    }
    if (P->dense) {   // alpha_i = D_i^{-1} B_i, E_i = D_i^{-1} A_i
      for (int q = 0; q < nm; ++q) {
        const int64_t i = rows[q];
        BDesc d = desc0();
        d.a_off = i * MM;
        d.kd = d.segrows = (int32_t)Mp;
        d.c_off = i * MM;
        BDesc x = d;
        d.b_off = i * 2 * MM + MM;
        x.b_off = i * 2 * MM;
        dal.push_back(d);
        de.push_back(x);
      }
    }
    // every list of the step goes to the device in one copy
    pool.begin_batch();
    int64_t* d_rows = reuse ? nullptr : pool.put_vec(rows);
    int32_t* d_first = reuse ? nullptr : pool.put_vec(first);
    int64_t* d_out = reuse ? nullptr : pool.put_vec(outoff);
    int64_t* d_bd = reuse ? nullptr : pool.put_vec(bdoff);
    int32_t* d_tag = reuse ? nullptr : pool.put_vec(tag);
    const BDesc* s_da = da.empty() ? nullptr : pool.put(da);
    const BDesc* s_dal = dal.empty() ? nullptr : pool.put(dal);
    const BDesc* s_de = de.empty() ? nullptr : pool.put(de);
    const BDesc* s_gam = pool.put(gam);
    pool.end_batch();
    if (!reuse) {
      HIPCHK(launch_build_D(Dwork, MM, nm, d_rows, d_first, P->cC, P->fmtC, P->adiag, P->alpha, (int)M, (int)Mp, st));
      if (!da.empty()) {
        BArgs a = bargs_base((int)Mp);
        a.alpha = -1.0;
        a.A = P->ABd; a.lda = Mp;
        a.B = P->alpha; a.ldb = Mp;
        a.C = Dwork; a.ldc = Mp;
        a.Cin = Dwork; a.ldcin = Mp;
        a.ncols = (int32_t)Mp;
        run_bgemm(a, da, s_da, st);
      }
      GJArgs g{};
      g.work = Dwork; g.work_off = nullptr; g.wstride = MM;
      g.out = P->Dinv; g.out_off = d_out;
      g.alpha = P->dense ? nullptr : P->alpha; g.bdiag = P->bdiag; g.bd_off = d_bd;
      g.tag = d_tag; g.bad = bad;
      g.nmat = nm; g.Mp = (int32_t)Mp;
      gj_scratch(g);
      HIPCHK(launch_gj(g, st));
    }
    if (P->dense) {   // ... and Gamma_i = E_i Gamma_{i-1}
      BArgs a = bargs_base((int)Mp);
      a.A = P->Dinv; a.lda = Mp;
      a.B = P->ABd; a.ldb = Mp;
      a.ncols = (int32_t)Mp;
      a.ldc = Mp;
      BArgs aa = a, ae = a;
      aa.C = P->alpha;
      ae.C = P->E;
      run_bgemm(aa, dal, s_dal, st);
      run_bgemm(ae, de, s_de, st);
      BArgs ag = bargs_base((int)Mp);
      ag.A = P->E; ag.lda = Mp;
      ag.B = Ga; ag.ldb = Mp;
      ag.C = Ga; ag.ldc = Mp;
      ag.ncols = (int32_t)Mp;
      run_bgemm(ag, gam, s_gam, st);
    } else {
      BArgs a = bargs_base((int)Mp);
      a.A = P->Dinv; a.lda = Mp;
      a.B = Ga; a.ldb = Mp;
      a.bscale = P->adiag;
      a.C = Ga; a.ldc = Mp;
      a.ncols = (int32_t)Mp;
      run_bgemm(a, gam, s_gam, st);
    }
  }

  // ---- backward: U_i = alpha_i U_{i+1} + Gamma_i, V_i = alpha_i V_{i+1}; U_{k_{s+1}} = 0, V_{k_{s+1}} = I
  for (int64_t t = maxn - 1; t >= 0; --t) {
    std::vector<BDesc> du, dv;
    for (int64_t s = 0; s < p; ++s) {
      if (nint[s] <= t) continue;
      const int64_t i = ks[s] + 1 + t;
      const bool lastrow = (t == nint[s] - 1);
      BDesc d = desc0();
      d.a_off = i * MM;
      d.kd = (int32_t)Mp;
      d.segrows = (int32_t)Mp;
      BDesc u = d, v = d;
      u.b_off = lastrow ? MM : (2 + 2 * (i + 1)) * MM;        // Zero or U_{i+1}
      u.cin_off = (1 + i) * MM;                                 // Gamma_i
      u.c_off = (2 + 2 * i) * MM;
      v.b_off = lastrow ? 0 : (2 + 2 * (i + 1) + 1) * MM;      // Ident or V_{i+1}
      v.c_off = (2 + 2 * i + 1) * MM;
      du.push_back(u);
      dv.push_back(v);
    }
    BArgs a = bargs_base((int)Mp);
    a.A = P->alpha; a.lda = Mp;
    a.B = P->UVa; a.ldb = Mp;
    a.C = P->UVa; a.ldc = Mp;
    a.ncols = (int32_t)Mp;
    BArgs au = a;
    au.Cin = Ga; au.ldcin = Mp;
    pool.begin_batch();
    const BDesc* s_du = pool.put(du);
    const BDesc* s_dv = pool.put(dv);
    pool.end_batch();
    run_bgemm(au, du, s_du, st);
    run_bgemm(a, dv, s_dv, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  P->release(Ga);
  P->release(Dwork);

  // ---- reduced system, eq. (red1)
  P->red = P->alloc(3 * p * MM);
  double* At = P->red;
  double* Ct = P->red + p * MM;
  double* Bt = P->red + 2 * p * MM;
  HIPCHK(launch_reduced(At, Ct, Bt, P->d_ks, P->UVa + 2 * MM, P->cC, P->fmtC, P->adiag, P->bdiag, (int)p, (int)N, (int)M,
                        (int)Mp, st));
  if (P->dense) {
    // with zero diagonal couplings k_reduced left At = 0, Ct = C_k, Bt = 0; add the products of
    // eq. (red1): At = A_k U_{k-1}, Ct -= A_k V_{k-1} + B_k U_{k+1}, Bt = B_k V_{k+1}, where a
    // neighbour that is itself an interface row contributes U = I, V = 0 (left) or U = 0,
    // V = I (right); UVa holds [I | 0 | U_0 V_0 | U_1 V_1 | ...]
    std::vector<BDesc> dA, dCl, dCr, dB;
    for (int64_t s = 0; s < p; ++s) {
      const int64_t kk = ks[s];
      const bool left_int = s > 0 && kk - 1 > ks[s - 1];
      const bool right_int = kk + 1 < ks[s + 1];
      BDesc d = desc0();
      d.kd = d.segrows = (int32_t)Mp;
      d.c_off = d.cin_off = s * MM;
      if (s > 0) {
        BDesc x = d;
        x.a_off = kk * 2 * MM;
        x.b_off = left_int ? (2 + 2 * (kk - 1)) * MM : 0;
        dA.push_back(x);
        if (left_int) {
          x.b_off = (2 + 2 * (kk - 1) + 1) * MM;
          dCl.push_back(x);
        }
      }
      if (kk + 1 < N) {
        BDesc x = d;
        x.a_off = kk * 2 * MM + MM;
        if (right_int) {
          x.b_off = (2 + 2 * (kk + 1)) * MM;
          dCr.push_back(x);
        }
        x.b_off = right_int ? (2 + 2 * (kk + 1) + 1) * MM : 0;
        dB.push_back(x);
      }
    }
    BArgs a = bargs_base((int)Mp);
    a.A = P->ABd; a.lda = Mp;
    a.B = P->UVa; a.ldb = Mp;
    a.ldc = Mp; a.ldcin = Mp;
    a.ncols = (int32_t)Mp;
    BArgs aA = a, aC = a, aB = a;
    aA.C = At;
    aB.C = Bt;
    aC.C = Ct; aC.Cin = Ct; aC.alpha = -1.0;
    run_bgemm(aA, dA, pool, st);
    run_bgemm(aB, dB, pool, st);
    run_bgemm(aC, dCl, pool, st);
    run_bgemm(aC, dCr, pool, st);
  }

  // ---- dichotomy tree (Algorithm 1 applied to the reduced system)
  P->nodes.clear();
  P->depth = 0;
  build_tree(P->nodes, 0, (int)p - 1, 0, P->depth);
  auto& nodes = P->nodes;
  const int nn = (int)nodes.size();
  int64_t goff = 0;
  const int CB = 4;  // blocks per partial-sum chunk
  int nch = 0;
  for (auto& n : nodes) {
    n.g_off = goff;
    goff += (int64_t)(n.r - n.l + 1) * MM;
    n.chunk0 = nch;
    n.nchunk = (n.r - n.l + 1 + CB - 1) / CB;
    nch += n.nchunk;
  }
  P->nchunks = nch;
  P->G = P->alloc(goff);
  P->H = P->alloc((int64_t)nn * 2 * MM);
  HIPCHK(launch_fill(P->H, (int64_t)nn * 2 * MM, 0.0, st));
  // arena: [Zero | DWL | DWR | AL | AR | TL | TR] per node
  double* Da = P->alloc((1 + 6 * (int64_t)nn) * MM);
  HIPCHK(launch_fill(Da, MM, 0.0, st));
  auto DWL = [&](int n) { return (1 + 0 * (int64_t)nn + n) * MM; };
  auto DWR = [&](int n) { return (1 + 1 * (int64_t)nn + n) * MM; };
  auto AL = [&](int n) { return (1 + 2 * (int64_t)nn + n) * MM; };
  auto AR = [&](int n) { return (1 + 3 * (int64_t)nn + n) * MM; };
  auto TL = [&](int n) { return (1 + 4 * (int64_t)nn + n) * MM; };
  auto TR = [&](int n) { return (1 + 5 * (int64_t)nn + n) * MM; };
  auto gslot = [&](int n, int j) { return nodes[n].g_off + (int64_t)(j - nodes[n].l) * MM; };
  const int64_t oA = 0, oC = p * MM, oB = 2 * p * MM;  // offsets of At, Ct, Bt in red

  int maxchain = 0;
  for (auto& n : nodes) maxchain = std::max(maxchain, std::max(n.m - n.l, n.r - n.m));

  // The transposed system's tree has the same nodes, and its chain matrices and middle Schur
  // complements are the transposes of this system's (D'^L_j = (D^L_j)^T by induction on
  // Ct'_j - At'_j (D'^L_{j-1})^{-1} Bt'_{j-1} with At'_j = Bt_{j-1}^T, Bt'_j = At_{j+1}^T, Ct'_j = Ct_j^T;
  // likewise D'^R_j and S'_m): a transposed plan whose forward plan kept them takes their inverses
  // transposed, in one launch, instead of the chain eliminations.
  const bool reuse_tree = fwd != nullptr && fwd->chain_inv != nullptr;
  if (reuse_tree) {
    HIPCHK(launch_transpose_blocks(P->G, fwd->chain_inv, goff / MM, (int)Mp, st));
  } else {
    // left chains D^L_j = Ct_j - At_j alphaL_{j-1}, alphaL_j = (D^L_j)^{-1} Bt_j  (j = l..m-1)
    // right chains D^R_j = Ct_j - Bt_j alphaR_{j+1}, alphaR_j = (D^R_j)^{-1} At_j (j = r..m+1)
    for (int t = 0; t < maxchain; ++t) {
      std::vector<BDesc> dd, da;
      std::vector<int64_t> outoff;
      std::vector<int32_t> tag;
      std::vector<int64_t> woff;
      for (int n = 0; n < nn; ++n) {
        const Node& nd = nodes[n];
        if (nd.m - nd.l > t) {
          const int j = nd.l + t;
          BDesc d = desc0();
          d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
          d.a_off = oA + j * MM;
          d.b_off = (t == 0) ? 0 : AL(n);
          d.cin_off = oC + j * MM;
          d.c_off = DWL(n);
          dd.push_back(d);
          BDesc e = desc0();
          e.kd = (int32_t)Mp; e.segrows = (int32_t)Mp;
          e.a_off = gslot(n, j);
          e.b_off = oB + j * MM;
          e.c_off = AL(n);
          da.push_back(e);
          woff.push_back(DWL(n));
          outoff.push_back(gslot(n, j));
          tag.push_back((int32_t)(N + j));
        }
        if (nd.r - nd.m > t) {
          const int j = nd.r - t;
          BDesc d = desc0();
          d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
          d.a_off = oB + j * MM;
          d.b_off = (t == 0) ? 0 : AR(n);
          d.cin_off = oC + j * MM;
          d.c_off = DWR(n);
          dd.push_back(d);
          BDesc e = desc0();
          e.kd = (int32_t)Mp; e.segrows = (int32_t)Mp;
          e.a_off = gslot(n, j);
          e.b_off = oA + j * MM;
          e.c_off = AR(n);
          da.push_back(e);
          woff.push_back(DWR(n));
          outoff.push_back(gslot(n, j));
          tag.push_back((int32_t)(N + j));
        }
      }
      // the step's lists in one copy
      const int nm = (int)woff.size();
      pool.begin_batch();
      const BDesc* s_dd = pool.put(dd);
      const BDesc* s_da = pool.put(da);
      int64_t* d_woff = pool.put_vec(woff);
      int64_t* d_out = pool.put_vec(outoff);
      int32_t* d_tag = pool.put_vec(tag);
      pool.end_batch();
      BArgs a = bargs_base((int)Mp);
      a.A = P->red; a.lda = Mp;
      a.B = Da; a.ldb = Mp;
      a.Cin = P->red; a.ldcin = Mp;
      a.C = Da; a.ldc = Mp;
      a.alpha = -1.0;
      a.ncols = (int32_t)Mp;
      run_bgemm(a, dd, s_dd, st);
      // invert the chain matrices in place in the arena (one launch for all nodes)
      if (nm > 0) {
        GJArgs g{};
        g.work = Da; g.work_off = d_woff; g.wstride = 0;
        g.out = P->G; g.out_off = d_out;
        g.alpha = nullptr; g.bdiag = nullptr; g.bd_off = nullptr;
        g.tag = d_tag; g.bad = bad;
        g.nmat = nm; g.Mp = (int32_t)Mp;
        gj_scratch(g);
        HIPCHK(launch_gj(g, st));
      }
      BArgs b = bargs_base((int)Mp);
      b.A = P->G; b.lda = Mp;
      b.B = P->red; b.ldb = Mp;
      b.C = Da; b.ldc = Mp;
      b.ncols = (int32_t)Mp;
      run_bgemm(b, da, s_da, st);
    }
    // S_m = Ct_m - At_m alphaL_{m-1} - Bt_m alphaR_{m+1};  G_m = S_m^{-1}
    {
      std::vector<BDesc> d1, d2;
      std::vector<int64_t> outoff;
      std::vector<int32_t> tag;
      for (int n = 0; n < nn; ++n) {
        const Node& nd = nodes[n];
        BDesc d = desc0();
        d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
        d.a_off = oA + nd.m * MM;
        d.b_off = (nd.m > nd.l) ? AL(n) : 0;
        d.cin_off = oC + nd.m * MM;
        d.c_off = DWL(n);
        d1.push_back(d);
        BDesc e = desc0();
        e.kd = (int32_t)Mp; e.segrows = (int32_t)Mp;
        e.a_off = oB + nd.m * MM;
        e.b_off = (nd.r > nd.m) ? AR(n) : 0;
        e.cin_off = DWL(n);
        e.c_off = DWL(n);
        d2.push_back(e);
        outoff.push_back(gslot(n, nd.m));
        tag.push_back((int32_t)(N + nd.m));
      }
      BArgs a = bargs_base((int)Mp);
      a.A = P->red; a.lda = Mp;
      a.B = Da; a.ldb = Mp;
      a.Cin = P->red; a.ldcin = Mp;
      a.C = Da; a.ldc = Mp;
      a.alpha = -1.0;
      a.ncols = (int32_t)Mp;
      run_bgemm(a, d1, pool, st);
      BArgs a2 = a;
      a2.Cin = Da;
      run_bgemm(a2, d2, pool, st);
      std::vector<int64_t> woff;
      for (int n = 0; n < nn; ++n) woff.push_back(DWL(n));
      GJArgs g{};
      g.work = Da; g.work_off = pool.put_vec(woff); g.wstride = 0;
      g.out = P->G; g.out_off = pool.put_vec(outoff);
      g.alpha = nullptr; g.bdiag = nullptr; g.bd_off = nullptr;
      g.tag = pool.put_vec(tag); g.bad = bad;
      g.nmat = nn; g.Mp = (int32_t)Mp;
      gj_scratch(g);
      HIPCHK(launch_gj(g, st));
    }
    if (keep_chain && !P->dense) {   // the inverses in G are overwritten by the rows G_j below
      P->chain_inv = P->alloc(goff);
      HIPCHK(hipMemcpyAsync(P->chain_inv, P->G, (size_t)goff * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
  }
  // G_j = G_{j+1} At_{j+1} (D^L_j)^{-1} for j < m;  G_j = G_{j-1} Bt_{j-1} (D^R_j)^{-1} for j > m
  for (int t = 0; t < maxchain; ++t) {
    std::vector<BDesc> d1, d2;
    for (int n = 0; n < nn; ++n) {
      const Node& nd = nodes[n];
      if (nd.m - nd.l > t) {
        const int j = nd.m - 1 - t;
        BDesc d = desc0();
        d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
        d.a_off = gslot(n, j + 1);
        d.b_off = oA + (j + 1) * MM;
        d.c_off = TL(n);
        d1.push_back(d);
        BDesc e = desc0();
        e.kd = (int32_t)Mp; e.segrows = (int32_t)Mp;
        e.a_off = TL(n);
        e.b_off = gslot(n, j);
        e.c_off = gslot(n, j);
        d2.push_back(e);
      }
      if (nd.r - nd.m > t) {
        const int j = nd.m + 1 + t;
        BDesc d = desc0();
        d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
        d.a_off = gslot(n, j - 1);
        d.b_off = oB + (j - 1) * MM;
        d.c_off = TR(n);
        d1.push_back(d);
        BDesc e = desc0();
        e.kd = (int32_t)Mp; e.segrows = (int32_t)Mp;
        e.a_off = TR(n);
        e.b_off = gslot(n, j);
        e.c_off = gslot(n, j);
        d2.push_back(e);
      }
    }
    pool.begin_batch();
    const BDesc* s_d1 = pool.put(d1);
    const BDesc* s_d2 = pool.put(d2);
    pool.end_batch();
    BArgs a = bargs_base((int)Mp);
    a.A = P->G; a.lda = Mp;
    a.B = P->red; a.ldb = Mp;
    a.C = Da; a.ldc = Mp;
    a.ncols = (int32_t)Mp;
    run_bgemm(a, d1, s_d1, st);
    BArgs b = bargs_base((int)Mp);
    b.A = Da; b.lda = Mp;
    b.B = P->G; b.ldb = Mp;
    b.C = P->G; b.ldc = Mp;
    b.ncols = (int32_t)Mp;
    run_bgemm(b, d2, s_d2, st);
  }
  // H^L = G_l At_l (l > 0), H^R = G_r Bt_r (r < p-1)
  {
    std::vector<BDesc> dh;
    for (int n = 0; n < nn; ++n) {
      const Node& nd = nodes[n];
      if (nd.l > 0) {
        BDesc d = desc0();
        d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
        d.a_off = gslot(n, nd.l);
        d.b_off = oA + nd.l * MM;
        d.c_off = (int64_t)n * 2 * MM;
        dh.push_back(d);
      }
      if (nd.r < p - 1) {
        BDesc d = desc0();
        d.kd = (int32_t)Mp; d.segrows = (int32_t)Mp;
        d.a_off = gslot(n, nd.r);
        d.b_off = oB + nd.r * MM;
        d.c_off = (int64_t)n * 2 * MM + MM;
        dh.push_back(d);
      }
    }
    BArgs a = bargs_base((int)Mp);
    a.A = P->G; a.lda = Mp;
    a.B = P->red; a.ldb = Mp;
    a.C = P->H; a.ldc = Mp;
    a.ncols = (int32_t)Mp;
    run_bgemm(a, dh, pool, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  P->release(Da);
  P->release(gjs);

  // ---- descriptors of the solve
  {
    std::vector<BDesc> part;
    for (int n = 0; n < nn; ++n) {
      const Node& nd = nodes[n];
      for (int c = 0; c < nd.nchunk; ++c) {
        const int jb = nd.l + c * CB, je = std::min(nd.r + 1, jb + CB);
        BDesc d = desc0();
        d.a_off = nd.g_off + (int64_t)(jb - nd.l) * MM;
        d.kd = (int32_t)((je - jb) * Mp);
        d.segrows = d.kd;
        d.b_off = jb * Mp;
        d.c_off = (int64_t)(nd.chunk0 + c) * Mp;
        part.push_back(d);
      }
    }
    P->n_part = (int)part.size();
    P->d_part = P->upload(part);
    std::vector<BDesc> corr;
    P->corr_begin.assign(P->depth, 0);
    P->corr_count.assign(P->depth, 0);
    for (int lv = 0; lv < P->depth; ++lv) {
      P->corr_begin[lv] = (int)corr.size();
      for (int n = 0; n < nn; ++n) {
        const Node& nd = nodes[n];
        if (nd.level != lv) continue;
        BDesc d = desc0();
        d.a_off = (int64_t)n * 2 * MM;            // [H^L | H^R]
        d.kd = (int32_t)(2 * Mp);
        d.segrows = (int32_t)Mp;
        d.b_off = (int64_t)nd.l * Mp;            // X_{l-1} (padded index l)
        d.bseg = (int64_t)(nd.r + 2 - nd.l) * Mp; // X_{r+1} (padded index r+2)
        d.sp_off = (int64_t)nd.chunk0 * Mp;
        d.nsp = nd.nchunk;
        d.c_off = (int64_t)(nd.m + 1) * Mp;
        d.x2_off = ks[nd.m] * M;
        corr.push_back(d);
      }
      P->corr_count[lv] = (int)corr.size() - P->corr_begin[lv];
    }
    P->d_corr = P->upload(corr);

    // A level with few nodes nl has too few column tiles to fill the device, and each
    // work-group walks the whole inner dimension 2 Mp with one chunk of prefetch; split it into
    // nslab slabs (each within one of the two segments X_{l-1}, X_{r+1}; at most 8), aiming at
    // nl * nslab >= 16 problems (levels with more nodes already fill the device).
    std::vector<BDesc> split;
    std::vector<CombDesc> comb;
    P->lev_nslab.assign(P->depth, 1);
    P->split_begin.assign(P->depth, 0);
    P->split_count.assign(P->depth, 0);
    P->comb_begin.assign(P->depth, 0);
    P->pslots = 0;
    for (int lv = 0; lv < P->depth; ++lv) {
      const int nl = P->corr_count[lv];
      // a slab must be a whole number of 16-deep GEMM chunks and lie within one segment
      auto slab_ok = [&](int n) {
        const int64_t w = 2 * Mp / n;
        return (2 * Mp) % n == 0 && w % 16 == 0 && Mp % w == 0;
      };
      int ns = 1;
      // (small blocks: the inner dimension is a few chunks and the extra launch would cost more)
      while (Mp >= 64 && nl * ns < 16 && ns < 8 && slab_ok(2 * ns)) ns *= 2;
      P->lev_nslab[lv] = ns;
      P->split_begin[lv] = (int)split.size();
      P->comb_begin[lv] = (int)comb.size();
      if (ns == 1) continue;
      const int64_t kslab = 2 * Mp / ns;   // a multiple of 16 that divides Mp
      for (int j = 0; j < nl; ++j) {
        const BDesc& c = corr[P->corr_begin[lv] + j];
        for (int q = 0; q < ns; ++q) {
          const int64_t k0 = q * kslab, seg = k0 / Mp, kin = k0 - seg * Mp;
          BDesc d = desc0();
          d.a_off = c.a_off + k0 * Mp;                // columns k0.. of [H^L | H^R]
          d.kd = (int32_t)kslab;
          d.segrows = (int32_t)kslab;
          d.b_off = c.b_off + seg * c.bseg + kin;
          d.c_off = (int64_t)(j * ns + q) * Mp;
          split.push_back(d);
        }
        CombDesc cd;
        std::memset(&cd, 0, sizeof(cd));
        cd.p_off = (int64_t)j * ns * Mp;
        cd.nslab = ns;
        cd.sp_off = c.sp_off;
        cd.nsp = c.nsp;
        cd.c_off = c.c_off;
        cd.x2_off = c.x2_off;
        comb.push_back(cd);
      }
      P->split_count[lv] = (int)split.size() - P->split_begin[lv];
      P->pslots = std::max(P->pslots, nl * ns);
    }
    P->d_split = P->upload(split);
    P->d_comb = P->upload(comb);

    if (P->dense) {
      // G_i = D_i^{-1} F_i (B = F, M rows per block) into W for every interior row
      std::vector<BDesc> gf, ftd;
      for (int64_t s = 0; s < p; ++s)
        for (int64_t i = ks[s] + 1; i < ks[s + 1]; ++i) {
          BDesc d = desc0();
          d.a_off = i * MM;
          d.b_off = i * M;
          d.c_off = i * Mp;
          d.kd = d.segrows = (int32_t)Mp;
          gf.push_back(d);
        }
      // F~_s += [A_k | B_k] [W_{k-1}; W_{k+1}] over the neighbours that are interior rows
      for (int64_t s = 0; s < p; ++s) {
        const int64_t kk = ks[s];
        const bool left = s > 0 && kk - 1 > ks[s - 1];
        const bool right = kk + 1 < ks[s + 1];
        if (!left && !right) continue;
        BDesc d = desc0();
        d.c_off = d.cin_off = s * Mp;
        d.segrows = (int32_t)Mp;
        if (left && right) {
          d.a_off = kk * 2 * MM;
          d.kd = (int32_t)(2 * Mp);
          d.b_off = (kk - 1) * Mp;
          d.bseg = 2 * Mp;
        } else if (left) {
          d.a_off = kk * 2 * MM;
          d.kd = (int32_t)Mp;
          d.b_off = (kk - 1) * Mp;
        } else {
          d.a_off = kk * 2 * MM + MM;
          d.kd = (int32_t)Mp;
          d.b_off = (kk + 1) * Mp;
        }
        ftd.push_back(d);
      }
      P->n_gf = (int)gf.size();
      P->d_gf = P->upload(gf);
      P->n_ftd = (int)ftd.size();
      P->d_ftd = P->upload(ftd);
    }
  }
  // pivot check
  int32_t badv = INT_MAX;
  HIPCHK(hipMemcpy(&badv, bad, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (badv != INT_MAX) {
    char buf[160];
    if (badv < N)
      std::snprintf(buf, sizeof buf, "singular pivot block at block row %d (0-based) of the subdomain elimination", badv);
    else
      std::snprintf(buf, sizeof buf, "singular block at row %d (0-based) of the reduced interface system", (int)(badv - N));
    throw std::string(buf);
  }
}

// ------------------------------------------------------------------------------------------
// Factor of a scalar system (block size 1) with every row an interface row: the dichotomy tree over
// all rows (Algorithm 1, Sec. 2.1), the stored row of the inverse of every node's submatrix, and the
// subtree / top-node layout of the solve (kernels_scalar.hip).
// ------------------------------------------------------------------------------------------
void factor_scalar(td_plan_s* P, const double* A, const double* B, const double* C, hipStream_t st) {
  const int N = (int)P->N;
  const int64_t nC = (P->fmtC == TD_FMT_TRIDIAG) ? 3 * (int64_t)N : N;
  P->cA = P->alloc(N);
  P->cB = P->alloc(N);
  P->cC = P->alloc(nC);
  HIPCHK(hipMemcpyAsync(P->cA, A, (size_t)N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(P->cB, B, (size_t)N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(P->cC, C, (size_t)nC * 8, hipMemcpyDeviceToDevice, st));
  if (P->fmtA == TD_FMT_DIAG && P->fmtB == TD_FMT_DIAG && P->fmtC == TD_FMT_TRIDIAG)
    HIPCHK(launch_zero_absent(P->cA, P->cB, P->cC, N, 1, st));   // for the stencil residual
  P->d_flag = (int32_t*)P->alloc(2);
  int32_t* bad = P->d_flag;
  HIPCHK(launch_negate_fill_check(bad, INT_MAX, st));

  // the tree: node of split row m covers [lo[m], hi[m]] at level lvl[m]; levels left to right
  std::vector<int> lo(N), hi(N), lvl(N);
  std::vector<std::vector<int>> bylevel;
  {
    std::vector<std::pair<int, int>> cur{{0, N - 1}}, nxt;
    for (int lv = 0; !cur.empty(); ++lv) {
      bylevel.emplace_back();
      nxt.clear();
      for (auto& nd : cur) {
        const int l = nd.first, r = nd.second, m = (l + r) / 2;
        lo[m] = l; hi[m] = r; lvl[m] = lv;
        bylevel.back().push_back(m);
        if (m > l) nxt.push_back({l, m - 1});
        if (m < r) nxt.push_back({m + 1, r});
      }
      cur.swap(nxt);
    }
  }
  const int depth = (int)bylevel.size();
  P->depth = depth;
  int L0 = 0;   // first level whose nodes all have at most SC_SUB rows
  for (; L0 < depth; ++L0) {
    int mx = 0;
    for (int m : bylevel[L0]) mx = std::max(mx, hi[m] - lo[m] + 1);
    if (mx <= SC_SUB) break;
  }
  const std::vector<int>& subs = bylevel[L0];
  const int nsub = (int)subs.size();
  std::vector<int> top_m, top_lvl, topidx(N, -1);
  for (int lv = 0; lv < L0; ++lv)
    for (int m : bylevel[lv]) {
      topidx[m] = (int)top_m.size();
      top_m.push_back(m);
      top_lvl.push_back(lv);
    }
  const int ntop = (int)top_m.size();
  for (int lv = 0; lv < L0; ++lv)   // the solve's top kernel walks complete binary levels
    if ((int)bylevel[lv].size() != (1 << lv)) throw std::string("internal error: incomplete top level");
  std::vector<int> toprow_sorted(top_m);
  std::sort(toprow_sorted.begin(), toprow_sorted.end());
  std::vector<int> sub_lo(nsub), sub_hi(nsub), sub_left(nsub), sub_right(nsub), sub_off(nsub);
  const int ndeep = depth - L0;
  std::vector<int> sub_order, sub_lvoff((size_t)nsub * (ndeep + 1), 0);
  int maxsub = 1;
  auto top_of = [&](int row) {   // top-list position of a boundary row (always a top row) or -1
    if (row < 0 || row >= N) return -1;
    if (topidx[row] < 0) throw std::string("internal error: subtree boundary row is not a top row");
    return topidx[row];
  };
  for (int q = 0; q < nsub; ++q) {
    const int m = subs[q];
    sub_lo[q] = lo[m]; sub_hi[q] = hi[m];
    maxsub = std::max(maxsub, hi[m] - lo[m] + 1);
    sub_left[q] = top_of(lo[m] - 1);
    sub_right[q] = top_of(hi[m] + 1);
    sub_off[q] = (int)sub_order.size();
    std::vector<int> cur{m}, nxt;
    for (int d = 0; d < ndeep; ++d) {
      sub_lvoff[(size_t)q * (ndeep + 1) + d] = (int)sub_order.size() - sub_off[q];
      nxt.clear();
      for (int x : cur) {
        sub_order.push_back(x);
        if (x > lo[x]) nxt.push_back((lo[x] + x - 1) / 2);
        if (x < hi[x]) nxt.push_back((x + 1 + hi[x]) / 2);
      }
      cur.swap(nxt);
    }
    sub_lvoff[(size_t)q * (ndeep + 1) + ndeep] = (int)sub_order.size() - sub_off[q];
  }
  std::vector<int> top_s0(ntop), top_s1(ntop), top_t0(ntop), top_t1(ntop), top_left(ntop), top_right(ntop);
  for (int t = 0; t < ntop; ++t) {
    const int m = top_m[t];
    top_s0[t] = (int)(std::lower_bound(sub_lo.begin(), sub_lo.end(), lo[m]) - sub_lo.begin());
    top_s1[t] = (int)(std::upper_bound(sub_lo.begin(), sub_lo.end(), hi[m]) - sub_lo.begin());
    top_t0[t] = (int)(std::lower_bound(toprow_sorted.begin(), toprow_sorted.end(), lo[m]) - toprow_sorted.begin());
    top_t1[t] = (int)(std::upper_bound(toprow_sorted.begin(), toprow_sorted.end(), hi[m]) - toprow_sorted.begin());
    top_left[t] = top_of(lo[m] - 1);
    top_right[t] = top_of(hi[m] + 1);
  }
  // every index array in one upload
  std::vector<int> arena;
  std::vector<size_t> at;
  auto add = [&](const std::vector<int>& v) {
    at.push_back(arena.size());
    arena.insert(arena.end(), v.begin(), v.end());
    while (arena.size() % 64) arena.push_back(0);
  };
  add(lo); add(hi); add(lvl);
  std::vector<int> sub_rec;   // {m, l, r, 0} per node in sub_order
  for (int m : sub_order) {
    sub_rec.push_back(m); sub_rec.push_back(lo[m]); sub_rec.push_back(hi[m]); sub_rec.push_back(0);
  }
  add(sub_lo); add(sub_hi); add(sub_left); add(sub_right); add(sub_rec); add(sub_off); add(sub_lvoff);
  add(top_m); add(top_lvl); add(top_s0); add(top_s1); add(top_t0); add(top_t1); add(top_left); add(top_right);
  add(toprow_sorted);
  const int* d = P->upload(arena);
  ScalarArgs& S = P->sc;
  std::memset(&S, 0, sizeof(S));
  S.N = N; S.L0 = L0; S.ndeep = ndeep; S.nsub = nsub; S.ntop = ntop; S.maxsub = maxsub;
  S.lo = d + at[0]; S.hi = d + at[1];
  const int* d_lvl = d + at[2];
  S.sub_lo = d + at[3]; S.sub_hi = d + at[4]; S.sub_left = d + at[5]; S.sub_right = d + at[6];
  S.sub_rec = (const int4*)(d + at[7]); S.sub_off = d + at[8]; S.sub_lvoff = d + at[9];
  S.top_m = d + at[10]; S.top_lvl = d + at[11]; S.top_s0 = d + at[12]; S.top_s1 = d + at[13];
  S.top_t0 = d + at[14]; S.top_t1 = d + at[15]; S.top_left = d + at[16]; S.top_right = d + at[17];
  S.toprow_sorted = d + at[18];
  double* G = P->alloc((int64_t)depth * N);
  HIPCHK(launch_fill(G, (int64_t)depth * N, 0.0, st));
  double* hl = P->alloc(N);
  double* hr = P->alloc(N);
  S.G = G; S.hl = hl; S.hr = hr;
  const bool tri = P->fmtC == TD_FMT_TRIDIAG;
  HIPCHK(launch_scalar_factor(P->cA, P->cB, P->cC + (tri ? 1 : 0), tri ? 3 : 1, N, S.lo, S.hi, d_lvl, G, hl, hr, bad,
                              st));
  double* sub_h = P->alloc(2 * (int64_t)sub_order.size());
  HIPCHK(launch_scalar_gather_h(sub_h, S.sub_rec, (int)sub_order.size(), hl, hr, st));
  S.sub_h = (const double2*)sub_h;
  int32_t badv = INT_MAX;
  HIPCHK(hipMemcpyAsync(&badv, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (badv != INT_MAX) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "singular block at row %d (0-based) of the reduced interface system",
                  (int)(badv - N));
    throw std::string(buf);
  }
}

// prev: the stream of the plan's previous solve, whose work may still read the old workspace
void ensure_workspace(td_plan_s* P, int64_t K, hipStream_t st, hipStream_t prev) {
  if (K <= P->kcap) return;
  if (P->kcap > 0 && prev != st) HIPCHK(hipStreamSynchronize(prev));
  ++P->ws_gen;
  if (P->scalar) {   // top-node partial sums and top-row values only
    P->release(P->Sp); P->release(P->Xi);
    P->Sp = P->alloc(std::max<int64_t>(1, (int64_t)P->sc.L0 * P->sc.nsub * K));
    P->Xi = P->alloc(std::max<int64_t>(1, (int64_t)P->sc.ntop * K));
    P->kcap = K;
    return;
  }
  const int64_t N = P->N, Mp = P->Mp, p = P->p;
  P->release(P->Wbuf); P->release(P->W32); P->release(P->Ft); P->release(P->Xi); P->release(P->Sp);
  P->release(P->Pbuf);
  P->Wbuf = P->Ft = P->Xi = P->Sp = P->Pbuf = nullptr;
  P->W32 = nullptr;
  if (P->prec == TD_PREC_F64)
    P->Wbuf = P->alloc(N * Mp * K);
  else
    P->W32 = (float*)P->alloc((w32_floats(N, Mp, K) + 1) / 2);
  P->Ft = P->alloc(p * Mp * K);
  P->Xi = P->alloc((p + 2) * Mp * K);
  P->Sp = P->alloc((int64_t)P->nchunks * Mp * K);
  if (P->pslots > 0) P->Pbuf = P->alloc((int64_t)P->pslots * Mp * K);
  HIPCHK(launch_fill(P->Xi, (p + 2) * Mp * K, 0.0, st));
  P->kcap = K;
}

bool stencil_formats(const td_plan_s* P) {
  return P->fmtA == TD_FMT_DIAG && P->fmtB == TD_FMT_DIAG && P->fmtC == TD_FMT_TRIDIAG;
}

int residual_parts(const td_plan_s* P) {
  return stencil_formats(P) ? residual_row_chunks_wide(P->N * P->M) : (int)P->N;
}

void ensure_refine_ws(td_plan_s* P, int64_t K) {
  if (K <= P->rcap) return;
  if (P->rcap > 0) HIPCHK(hipStreamSynchronize(P->last_stream));
  const int64_t n = P->N * P->M;
  P->release(P->Rbuf); P->release(P->colpart); P->release(P->norms);
  P->Rbuf = P->alloc(n * K);
  P->colpart = P->alloc((int64_t)residual_parts(P) * K * 2);
  P->norms = P->alloc(2 * K);
  P->rcap = K;
}

// plain solves replay a captured HIP graph unless TD_SOLVE_GRAPH=0
bool solve_graphs_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("TD_SOLVE_GRAPH");
    return !(v && v[0] == '0');
  }();
  return on;
}

// stage boundaries are recorded for the first pass of a solve only
void stage_mark(td_plan_s* P, int idx, hipStream_t st) {
  if (!P->prof || !P->se || !P->first_pass) return;
  HIPCHK(hipEventRecord(P->se->ev[idx], st));
}

// Solve workspace of one call: the plan's own buffers (plan_work) or pieces of a caller-independent
// fixed device array (tridiag_solve_noalloc).  Layouts: W (N Mp) x K float64 or W32 (panels of 64
// right-hand sides) float32; Ft (p Mp) x K; Xi ((p + 2) Mp) x K with a zero block at each end;
// Sp (nchunks Mp) x K; Pbuf (pslots Mp) x K.
struct Work {
  double* W;
  float* W32;
  double* Ft;
  double* Xi;
  double* Sp;
  double* Pbuf;
};

Work plan_work(const td_plan_s* P) { return Work{P->Wbuf, P->W32, P->Ft, P->Xi, P->Sp, P->Pbuf}; }

// One pass of Algorithm 2, step 2: eq. (sub3) sweeps, eq. (red1) right-hand side, Algorithm 1 on
// the reduced system, eq. (superposition).  The sweeps and the superposition run in the plan's
// precision (float64, or float32 / bfloat16 with float32 accumulation); the reduced system always
// in float64.  With `accumulate` the result is added to X (a refinement correction).
// row tiles per wave (16 rows each) for a requested wave count, 0 when it does not divide Mp
int32_t rt_for_waves(int64_t Mp, int32_t waves) {
  return (waves > 0 && Mp % (16 * (int64_t)waves) == 0) ? (int32_t)(Mp / (16 * (int64_t)waves)) : 0;
}

void solve_pass(td_plan_s* P, const Work& w, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                bool accumulate, hipStream_t st) {
  if (P->scalar) {   // Algorithm 1 on the scalar system: no sweeps, no superposition
    ScalarArgs A = P->sc;
    A.ldf = ldf; A.ldx = ldx; A.Pt = w.Sp; A.Xt = w.Xi;
    A.accumulate = accumulate ? 1 : 0;
    for (int i = 0; i <= 2; ++i) stage_mark(P, i, st);
    // columns in chunks whose column groups fit a launch's grid.y (at most 65535); the workspace
    // layout follows each chunk's own K
    const int64_t kmax = 65535 * (int64_t)SC_CPW;
    for (int64_t c0 = 0; c0 < K; c0 += kmax) {
      A.K = (int)std::min(kmax, K - c0);
      A.F = F + c0 * ldf;
      A.X = X + c0 * ldx;
      HIPCHK(launch_scalar_top(A, st));    // stage "dichotomy_partial": the top levels
      if (c0 + kmax >= K) stage_mark(P, 3, st);
      HIPCHK(launch_scalar_sub(A, st));    // stage "dichotomy_levels": the subtrees
    }
    stage_mark(P, 4, st);
    stage_mark(P, 5, st);
    P->first_pass = false;
    return;
  }
  const int64_t N = P->N, M = P->M, Mp = P->Mp, p = P->p;
  const int64_t ldw = N * Mp, ldft = p * Mp, ldxi = (p + 2) * Mp, ldsp = (int64_t)P->nchunks * Mp;
  stage_mark(P, 0, st);
  if (P->prec == TD_PREC_F64) {
    if (P->dense && P->n_gf > 0) {   // G_i = D_i^{-1} F_i, the forward sweep's inhomogeneous term
      BArgs g = bargs_base((int)Mp);
      g.descs = P->d_gf; g.nprob = P->n_gf;
      g.A = P->Dinv; g.lda = Mp;
      g.B = F; g.ldb = ldf; g.brows = (int32_t)M;
      g.C = w.W; g.ldc = ldw;
      g.ncols = (int32_t)K;
      g.kalign = (int32_t)Mp;   // kd = segrows = Mp
      HIPCHK(launch_bgemm(g, st));
    }
    SweepArgs sa{};
    sa.ks = P->d_ks; sa.Dinv = P->Dinv; sa.alpha = P->alpha; sa.adiag = P->adiag;
    sa.E = P->dense ? P->E : nullptr;
    sa.F = F; sa.ldf = ldf; sa.W = w.W; sa.ldw = ldw;
    sa.N = (int32_t)N; sa.M = (int32_t)M; sa.Mp = (int32_t)Mp; sa.p = (int32_t)p; sa.K = (int32_t)K;
    sa.ncoltiles = 0; sa.total = 0;
    sa.kt_hint = P->tiles.sweep_cols; sa.rt_hint = rt_for_waves(Mp, P->tiles.sweep_waves);
    if (N > p) HIPCHK(launch_sweep(sa, st));
    stage_mark(P, 1, st);
    HIPCHK(launch_ftilde(w.Ft, ldft, F, ldf, w.W, ldw, P->d_ks, P->adiag, P->bdiag, (int)p, (int)M, (int)Mp,
                         (int)K, st));
    if (P->dense && P->n_ftd > 0) {
      BArgs f = bargs_base((int)Mp);
      f.descs = P->d_ftd; f.nprob = P->n_ftd;
      f.A = P->ABd; f.lda = Mp;
      f.B = w.W; f.ldb = ldw;
      f.C = w.Ft; f.ldc = ldft;
      f.Cin = w.Ft; f.ldcin = ldft;
      f.ncols = (int32_t)K;
      f.kalign = (int32_t)Mp;   // kd Mp or 2 Mp, segrows Mp
      HIPCHK(launch_bgemm(f, st));
    }
  } else {
    LpSweepArgs sa{};
    sa.ks = P->d_ks; sa.Dinv = P->Dlp; sa.alpha = P->Alp; sa.adiag = P->adiag;
    sa.F = F; sa.ldf = ldf; sa.W = w.W32;
    sa.N = (int32_t)N; sa.M = (int32_t)M; sa.Mp = (int32_t)Mp; sa.p = (int32_t)p; sa.K = (int32_t)K;
    sa.ncoltiles = 0; sa.total = 0;
    sa.kt_hint = P->tiles.sweep_cols; sa.rt_hint = rt_for_waves(Mp, P->tiles.sweep_waves);
    if (N > p) HIPCHK(launch_sweep_lp(P->prec, sa, st));
    stage_mark(P, 1, st);
    HIPCHK(launch_ftilde_f32(w.Ft, ldft, F, ldf, w.W32, N, P->d_ks, P->adiag, P->bdiag, (int)p, (int)M,
                             (int)Mp, (int)K, st));
  }
  stage_mark(P, 2, st);
  {
    BArgs a = bargs_base((int)Mp);
    a.descs = P->d_part; a.nprob = P->n_part;
    a.A = P->G; a.lda = Mp;
    a.B = w.Ft; a.ldb = ldft;
    a.C = w.Sp; a.ldc = ldsp;
    a.ncols = (int32_t)K;
    a.kalign = (int32_t)Mp;   // chunks of whole blocks
    HIPCHK(launch_bgemm(a, st));
  }
  stage_mark(P, 3, st);
  for (int lv = 0; lv < P->depth; ++lv) {
    if (P->lev_nslab[lv] > 1) {
      const int64_t ldp = (int64_t)P->pslots * Mp;
      BArgs a = bargs_base((int)Mp);
      a.descs = P->d_split + P->split_begin[lv];
      a.nprob = P->split_count[lv];
      a.A = P->H; a.lda = Mp;
      a.B = w.Xi; a.ldb = ldxi;
      a.C = w.Pbuf; a.ldc = ldp;
      a.ncols = (int32_t)K;
      a.kalign = (int32_t)(2 * Mp / P->lev_nslab[lv]);   // slabs of 2 Mp / nslab rows
      HIPCHK(launch_bgemm(a, st));
      CombArgs c;
      std::memset(&c, 0, sizeof(c));
      c.descs = P->d_comb + P->comb_begin[lv];
      c.nnode = P->corr_count[lv];
      c.Mp = (int32_t)Mp; c.ncols = (int32_t)K;
      c.x2rows = (int32_t)M; c.x2accum = accumulate ? 1 : 0;
      c.P = w.Pbuf; c.ldp = ldp;
      c.Sp = w.Sp; c.ldsp = ldsp; c.spstride = Mp;
      c.C = w.Xi; c.ldc = ldxi;
      c.X2 = X; c.ldx2 = ldx;
      HIPCHK(launch_level_combine(c, st));
      continue;
    }
    BArgs a = bargs_base((int)Mp);
    a.descs = P->d_corr + P->corr_begin[lv];
    a.nprob = P->corr_count[lv];
    a.A = P->H; a.lda = Mp;
    a.B = w.Xi; a.ldb = ldxi;
    a.Sp = w.Sp; a.ldsp = ldsp; a.spstride = Mp;
    a.C = w.Xi; a.ldc = ldxi;
    a.X2 = X; a.ldx2 = ldx; a.x2rows = (int32_t)M; a.x2accum = accumulate ? 1 : 0;
    a.ncols = (int32_t)K;
    a.kalign = (int32_t)Mp;   // kd 2 Mp, segrows Mp
    HIPCHK(launch_bgemm(a, st));
  }
  stage_mark(P, 4, st);
  if (P->prec == TD_PREC_F64) {
    SupArgs u{};
    u.ks = P->d_ks; u.UV = P->UVa + 2 * Mp * Mp;
    u.Xi = w.Xi; u.ldxi = ldxi;
    u.W = w.W; u.ldw = ldw;
    u.X = X; u.ldx = ldx;
    u.N = (int32_t)N; u.M = (int32_t)M; u.Mp = (int32_t)Mp; u.p = (int32_t)p; u.K = (int32_t)K;
    u.ncoltiles = 0; u.total = 0; u.accumulate = accumulate ? 1 : 0;
    u.kt_hint = P->tiles.sup_cols; u.rt_hint = rt_for_waves(Mp, P->tiles.sup_waves);
    if (N > p) HIPCHK(launch_superpose(u, st));
  } else {
    LpSupArgs u{};
    u.ks = P->d_ks; u.UV = P->UVlp;
    u.Xi = w.Xi; u.ldxi = ldxi;
    u.W = w.W32;
    u.X = X; u.ldx = ldx;
    u.N = (int32_t)N; u.M = (int32_t)M; u.Mp = (int32_t)Mp; u.p = (int32_t)p; u.K = (int32_t)K;
    u.ncoltiles = 0; u.total = 0; u.accumulate = accumulate ? 1 : 0;
    u.kt_hint = P->tiles.sup_cols; u.rt_hint = rt_for_waves(Mp, P->tiles.sup_waves);
    if (N > p) HIPCHK(launch_superpose_lp(P->prec, u, st));
  }
  stage_mark(P, 5, st);
  P->first_pass = false;
}

// max over columns of ||F - P X|| / ||F||; R (if non-null) receives F - P X.  Synchronises.
double residual(td_plan_s* P, const double* F, int64_t ldf, const double* X, int64_t ldx, int64_t K, double* R,
                int64_t ldr, std::vector<double>& nrm, hipStream_t st) {
  ensure_refine_ws(P, K);
  const int nparts = residual_parts(P);
  if (stencil_formats(P))
    HIPCHK(launch_residual_stencil(R, ldr, F, ldf, X, ldx, P->cA, P->cB, P->cC, (int)P->N, (int)P->M, (int)K,
                                   P->colpart, st));
  else
    HIPCHK(launch_residual(R, ldr, F, ldf, X, ldx, P->cA, P->fmtA, P->cB, P->fmtB, P->cC, P->fmtC, (int)P->N,
                           (int)P->M, (int)K, P->colpart, nparts, st));
  HIPCHK(launch_colnorm_finish(P->norms, P->colpart, nparts, (int)K, st));
  nrm.resize(2 * K);
  HIPCHK(hipMemcpyAsync(nrm.data(), P->norms, 2 * K * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double worst = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double r = nrm[2 * k], f = nrm[2 * k + 1];
    const double rel = (f > 0.0) ? r / f : (r > 0.0 ? INFINITY : 0.0);
    if (!(rel <= worst)) worst = rel;  // NaN propagates
  }
  return worst;
}

td_status solve_impl(td_plan_s* P, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                     const td_refine* rf, td_info* info, hipStream_t st) {
  const int64_t n = P->N * P->M;
  if (K < 0 || ldf < n || ldx < n) return fail(TD_EINVAL, "K < 0 or leading dimension below N*M");
  if (K > INT_MAX / 2) return fail(TD_EINVAL, "K too large");
  if (info) { info->iterations = 0; info->nonfinite = 0; info->max_col_rel_residual = -1.0; }
  if (K == 0) return TD_OK;
  if (!F || !X) return fail(TD_EINVAL, "null F or X");
  // overlap check of the column ranges
  const char* f0 = (const char*)F;
  const char* f1 = (const char*)(F + (K - 1) * ldf + n);
  const char* x0 = (const char*)X;
  const char* x1 = (const char*)(X + (K - 1) * ldx + n);
  if (f0 < x1 && x0 < f1) return fail(TD_EINVAL, "X overlaps F");
  const hipStream_t prev_stream = P->last_stream;
  P->last_stream = st;
  P->astream = st;
  P->se = nullptr;
  if (P->prof && P->prof_n < 4096) {
    if ((int)P->evsets.size() <= P->prof_n) {
      StageEvents s;
      for (auto& e : s.ev) HIPCHK(hipEventCreate(&e));
      P->evsets.push_back(s);
    }
    P->se = &P->evsets[P->prof_n++];
  }
  ensure_workspace(P, K, st, prev_stream);
  if (P->se) HIPCHK(hipEventRecord(P->se->ev[6], st));
  P->first_pass = true;
  const bool refine = rf && rf->enable;
  if (!refine && !info && !P->se && solve_graphs_enabled()) {
    // a plain solve is a fixed sequence of launches: replay it from a HIP graph (captured on a
    // private stream, so that a legacy default stream of the caller is never captured)
    auto& g = P->sg;
    if (!(g.ex && g.F == F && g.ldf == ldf && g.X == X && g.ldx == ldx && g.K == K && g.ws_gen == P->ws_gen)) {
      P->drop_graph();
      hipStream_t cs = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      hipGraph_t gr = nullptr;
      hipError_t ce = hipSuccess;
      if (be == hipSuccess) {
        try {
          solve_pass(P, plan_work(P), F, ldf, X, ldx, K, false, cs);
        } catch (...) {
          (void)hipStreamEndCapture(cs, &gr);
          if (gr) (void)hipGraphDestroy(gr);
          (void)hipStreamDestroy(cs);
          throw;
        }
        ce = hipStreamEndCapture(cs, &gr);
      }
      (void)hipStreamDestroy(cs);
      HIPCHK(be);
      HIPCHK(ce);
      g.g = gr;
      HIPCHK(hipGraphInstantiate(&g.ex, gr, nullptr, nullptr, 0));
      g.F = F; g.ldf = ldf; g.X = X; g.ldx = ldx; g.K = K; g.ws_gen = P->ws_gen;
    }
    HIPCHK(hipGraphLaunch(g.ex, st));
    return TD_OK;
  }
  solve_pass(P, plan_work(P), F, ldf, X, ldx, K, false, st);
  td_status status = TD_OK;
  if (refine || info) {
    const double tol = (rf && rf->tol > 0.0) ? rf->tol : 1e-10;
    const int maxit = (rf && rf->max_iter > 0) ? rf->max_iter : 10;
    std::vector<double> nrm;
    ensure_refine_ws(P, K);
    double res = residual(P, F, ldf, X, ldx, K, refine ? P->Rbuf : nullptr, n, nrm, st);
    int it = 0;
    while (refine && !(res <= tol)) {
      if (it >= maxit || !std::isfinite(res)) { status = TD_ENOCONV; break; }
      // X += S(F - P X): the correction pass adds its result to X.  The residual is not
      // rescaled: for the relative residuals reached here its entries stay far above the
      // smallest normal float32 / bfloat16 number (about 1e-38).
      solve_pass(P, plan_work(P), P->Rbuf, n, X, ldx, K, true, st);
      ++it;
      res = residual(P, F, ldf, X, ldx, K, P->Rbuf, n, nrm, st);
    }
    if (info) {
      info->iterations = it;
      info->max_col_rel_residual = res;
      HIPCHK(launch_negate_fill_check(P->d_flag + 1, 0, st));
      HIPCHK(launch_nonfinite(P->d_flag + 1, X, ldx, n, (int)K, st));
      int32_t nf = 0;
      HIPCHK(hipMemcpyAsync(&nf, P->d_flag + 1, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      info->nonfinite = nf;
    }
  }
  if (P->se) HIPCHK(hipEventRecord(P->se->ev[7], st));
  P->se = nullptr;
  if (status == TD_ENOCONV) return fail(status, "refinement did not reach the requested residual");
  return TD_OK;
}

td_status check_desc(const td_desc* d) {
  if (!d) return fail(TD_EINVAL, "null descriptor");
  if (d->N < 1 || d->M < 1) return fail(TD_EINVAL, "N and M must be >= 1");
  if (d->subdomains < 0 || d->subdomains > d->N) return fail(TD_EINVAL, "subdomains must be in [0, N]");
  if (!(d->fmt_A == TD_FMT_DENSE || d->fmt_A == TD_FMT_DIAG)) return fail(TD_EINVAL, "fmt_A must be DENSE or DIAG");
  if (!(d->fmt_B == TD_FMT_DENSE || d->fmt_B == TD_FMT_DIAG)) return fail(TD_EINVAL, "fmt_B must be DENSE or DIAG");
  if (!(d->fmt_C == TD_FMT_DENSE || d->fmt_C == TD_FMT_TRIDIAG)) return fail(TD_EINVAL, "fmt_C must be DENSE or TRIDIAG");
  if (d->sweep_prec < TD_PREC_F64 || d->sweep_prec > TD_PREC_BF16) return fail(TD_EINVAL, "bad sweep_prec");
  if (d->reserved != 0) return fail(TD_EINVAL, "reserved must be 0");
  if ((d->dev_alloc == nullptr) != (d->dev_free == nullptr))
    return fail(TD_EINVAL, "dev_alloc and dev_free must both be set or both be NULL");
  if (d->M > 512) return fail(TD_ENOTSUP, "M > 512 is not supported");
  if (d->N > (int64_t)1 << 30) return fail(TD_ENOTSUP, "N too large");
  if ((d->fmt_A == TD_FMT_DENSE || d->fmt_B == TD_FMT_DENSE) && d->sweep_prec != TD_PREC_F64)
    return fail(TD_ENOTSUP, "dense A/B blocks need sweep_prec F64");
  return TD_OK;
}

// device bytes the factor needs at its peak (checked against free memory before allocating)
int64_t factor_bytes(int64_t N, int64_t M, int64_t p, int fA, int fB, int fC, int prec) {
  if (M == 1 && p == N && prec == TD_PREC_F64) {   // scalar plan: inputs, tree arrays, G by level
    int64_t depth = 0;
    for (int64_t q = N; q > 0; q >>= 1) ++depth;
    return 8 * (6 * N + depth * N) + 4 * 8 * N;
  }
  const int64_t Mp = pad_block(M, prec), MM = Mp * Mp;
  int64_t depth = 0;
  for (int64_t q = p; q > 0; q >>= 1) ++depth;
  int64_t b = 0;
  b += (fA == TD_FMT_DIAG ? N * M : N * M * M) + (fB == TD_FMT_DIAG ? N * M : N * M * M);
  b += (fC == TD_FMT_TRIDIAG ? 3 * N * M : N * M * M) + 2 * N * Mp;
  b += N * MM * 2 + (2 + 2 * N) * MM;     // Dinv, alpha, UV
  b += (1 + N) * MM + p * MM + p * Mp + 2 * p + 2 * p * ((Mp + 31) / 32) * Mp;   // Gamma arena, Dwork,
                                                                                // Gauss-Jordan scratch (temporary)
  b += 3 * p * MM + p * (depth + 1) * MM + 2 * p * MM + (1 + 6 * p) * MM + p * MM;  // reduced, G, H, arenas
  if (prec != TD_PREC_F64) b += (4 * N * MM * (prec == TD_PREC_F32 ? 4 : 2) + 7) / 8;  // rounded copies
  if (fA == TD_FMT_DENSE || fB == TD_FMT_DENSE) b += 3 * N * MM;                     // [A|B] blocks, E
  return b * 8;
}

// Rounded copies of D^{-1}, alpha and [U V] for the low-precision sweeps and superposition
// (row-major, k contiguous); the float64 originals are then released.
void make_lowprec(td_plan_s* P, hipStream_t st) {
  const int64_t N = P->N, Mp = P->Mp, MM = Mp * Mp;
  const int64_t esz = (P->prec == TD_PREC_F32) ? 4 : 2;
  std::vector<int64_t> rows;
  for (int64_t s = 0; s < P->p; ++s)
    for (int64_t i = P->ks[s] + 1; i < P->ks[s + 1]; ++i) rows.push_back(i);
  if (rows.empty()) rows.push_back(0);
  DescPool pool(P, st);
  int64_t* d_rows = pool.put_vec(rows);
  const int nm = (int)rows.size();
  P->Dlp = P->alloc((N * MM * esz + 7) / 8);
  P->Alp = P->alloc((N * MM * esz + 7) / 8);
  P->UVlp = P->alloc((N * 2 * MM * esz + 7) / 8);
  HIPCHK(launch_cast_rowmajor(P->prec, P->Dlp, MM, P->Dinv, MM, d_rows, nm, (int)Mp, (int)Mp, st));
  HIPCHK(launch_cast_rowmajor(P->prec, P->Alp, MM, P->alpha, MM, d_rows, nm, (int)Mp, (int)Mp, st));
  HIPCHK(launch_cast_rowmajor(P->prec, P->UVlp, 2 * MM, P->UVa + 2 * MM, 2 * MM, d_rows, nm, (int)Mp, (int)(2 * Mp),
                              st));
  HIPCHK(hipStreamSynchronize(st));
  P->release(P->Dinv);
  P->release(P->alpha);
  P->release(P->UVa);
  P->Dinv = P->alpha = P->UVa = nullptr;
}

td_status factor_top(const td_desc* d, const double* A, const double* B, const double* C, hipStream_t st,
                     td_plan* out, bool allow_adjoint) {
  td_status s = check_desc(d);
  if (s != TD_OK) return s;
  if (!A || !B || !C) return fail(TD_EINVAL, "null A, B or C");
  const auto t0 = std::chrono::steady_clock::now();
  td_plan_s* P = new td_plan_s();
  P->N = d->N; P->M = d->M; P->Mp = pad_block(d->M, d->sweep_prec);
  P->p = d->subdomains ? d->subdomains : default_subdomains(d->N, d->k_hint);
  P->ualloc = d->dev_alloc; P->ufree = d->dev_free; P->uctx = d->alloc_ctx;
  P->astream = st;
  P->fmtA = d->fmt_A; P->fmtB = d->fmt_B; P->fmtC = d->fmt_C;
  P->prec = d->sweep_prec; P->adjoint = d->adjoint;
  P->ks = partition(P->N, P->p);
  // block size 1 with every row an interface row: Algorithm 1 on the scalar system itself
  P->scalar = d->M == 1 && P->p == d->N && d->sweep_prec == TD_PREC_F64;
  if (P->scalar) P->Mp = 1;
  try {
    size_t freeb = 0, totb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totb));
    int64_t need = factor_bytes(P->N, P->M, P->p, P->fmtA, P->fmtB, P->fmtC, P->prec);
    if (d->adjoint && allow_adjoint) need *= 2;
    if ((double)need > 0.95 * (double)freeb) {
      delete P;
      return fail(TD_ENOMEM, "factor needs " + std::to_string(need) + " bytes, " + std::to_string(freeb) + " free");
    }
    if (P->scalar)
      factor_scalar(P, A, B, C, st);
    else
      factor_impl(P, A, B, C, st, nullptr, d->adjoint && allow_adjoint);
    if (d->adjoint && allow_adjoint && !P->dense && !P->scalar) {
      // the transposed plan from this one's compact inputs and block inverses (before the rounded
      // copies of a low-precision plan release them)
      td_plan_s* Q = new td_plan_s();
      Q->N = P->N; Q->M = P->M; Q->Mp = P->Mp; Q->p = P->p;
      Q->fmtA = P->fmtB; Q->fmtB = P->fmtA; Q->fmtC = P->fmtC;
      Q->prec = P->prec; Q->adjoint = 0;
      Q->ks = P->ks;
      Q->ualloc = P->ualloc; Q->ufree = P->ufree; Q->uctx = P->uctx; Q->astream = st;
      try {
        factor_impl(Q, nullptr, nullptr, nullptr, st, P);
        if (Q->prec != TD_PREC_F64) make_lowprec(Q, st);
      } catch (...) {
        delete Q;
        throw;
      }
      HIPCHK(hipStreamSynchronize(st));
      P->release(P->chain_inv);
      P->chain_inv = nullptr;
      Q->last_stream = st;
      P->adj = Q;
    }
    if (P->prec != TD_PREC_F64) make_lowprec(P, st);
    if (d->adjoint && allow_adjoint && (P->dense || P->scalar)) {
      // dense couplings or the scalar plan: the transposed plan is factored on its own from P^T's
      // blocks, formed on the device from this plan's compact copies
      const int64_t N = P->N, M = P->M;
      const int64_t sa = (P->fmtA == TD_FMT_DIAG) ? M : M * M, sb = (P->fmtB == TD_FMT_DIAG) ? M : M * M;
      const int64_t sc = (P->fmtC == TD_FMT_TRIDIAG) ? 3 * M : M * M;
      double* dA = P->alloc(N * sb);   // A' has B's format, B' has A's
      double* dB = P->alloc(N * sa);
      double* dC = P->alloc(N * sc);
      HIPCHK(launch_transpose_inputs(dA, dB, dC, P->cA, P->fmtA, P->cB, P->fmtB, P->cC, P->fmtC, (int)N, (int)M, st));
      td_desc d2 = *d;
      d2.subdomains = P->p;
      d2.adjoint = 0;
      d2.fmt_A = d->fmt_B;
      d2.fmt_B = d->fmt_A;
      td_plan adj = nullptr;
      td_status s2 = factor_top(&d2, dA, dB, dC, st, &adj, false);
      HIPCHK(hipStreamSynchronize(st));
      P->release(dA); P->release(dB); P->release(dC);
      if (s2 != TD_OK) {
        delete P;
        return s2;
      }
      P->adj = adj;
    }
  } catch (const HipFail& e) {
    delete P;
    const td_status code = (e.e == hipErrorOutOfMemory) ? TD_ENOMEM : TD_EHIP;
    return fail(code, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  } catch (const std::string& msg) {
    delete P;
    return fail(TD_ESINGULAR, msg);
  }
  P->factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  P->last_stream = st;
  *out = P;
  return TD_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Batched solve of many independent systems: one persistent launch (k_batched) over a work
// list, captured once in a HIP graph and replayed.  Float32 sweeps and superposition, float64
// reduced systems, residuals and a fixed number of correction passes with per-system early exit.
// ------------------------------------------------------------------------------------------
struct td_batch_s {
  int n = 0;
  std::vector<td_plan> plans;
  std::vector<void*> allocs;
  BatchItem* d_items = nullptr; int nitems = 0;
  BatchSys* d_sys = nullptr;
  int32_t* d_counters = nullptr; int ncounters = 0;
  int32_t* d_conv = nullptr;
  int32_t* d_heads = nullptr;   // stage-synchronous form: one dequeue counter per stage
  BatchCtl* d_ctl = nullptr;
  double* d_resid = nullptr;
  int passes = 0;
  bool check = true;
  int grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;
  ~td_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : allocs) (void)hipFree(p);
  }
  template <class T>
  T* dalloc(size_t count) {
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<size_t>(1, count) * sizeof(T)));
    allocs.push_back(p);
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
};

namespace {

td_status batch_create_impl(int n, const td_plan* plans, const double* const* F, const int64_t* ldf,
                            double* const* X, const int64_t* ldx, const int64_t* K, int passes, double tol,
                            hipStream_t st, td_batch_s* B) {
  if (n <= 0 || !plans || !F || !ldf || !X || !ldx || !K) return fail(TD_EINVAL, "bad batch arguments");
  if (passes < 1 || passes > 16) return fail(TD_EINVAL, "passes must be in [1, 16]");
  const bool check = tol >= 0.0;   // tol < 0: one pass, no residual test
  if (!check) passes = 1;
  for (int q = 0; q < n; ++q) {
    td_plan_s* P = plans[q];
    if (!P) return fail(TD_EINVAL, "null plan in batch");
    if (P->prec == TD_PREC_BF16) return fail(TD_ENOTSUP, "batched plans must have sweep_prec F64 or F32");
    if (!stencil_formats(P)) return fail(TD_ENOTSUP, "batched plans need diagonal A, B and tridiagonal C");
    if (!(P->Mp == 64 || P->Mp == 128 || P->Mp == 256)) return fail(TD_ENOTSUP, "batched plans need Mp in {64,128,256}");
    if (P->depth > BATCH_MAXDEPTH) return fail(TD_ENOTSUP, "dichotomy tree too deep for the batched kernel");
    if (K[q] < 1 || ldf[q] < P->N * P->M || ldx[q] < P->N * P->M || !F[q] || !X[q])
      return fail(TD_EINVAL, "bad K, leading dimension or pointer in batch");
    if (K[q] > INT_MAX / 2) return fail(TD_EINVAL, "K too large");
  }
  B->n = n;
  B->passes = passes;
  B->check = check;
  B->plans.assign(plans, plans + n);
  std::vector<BatchSys> sys(n);
  std::vector<int> cbase(n), nst(n);
  int nctr = 0;
  for (int q = 0; q < n; ++q) {
    td_plan_s* P = plans[q];
    const int64_t Kq = K[q];
    P->astream = st;
    ensure_workspace(P, Kq, st, P->last_stream ? P->last_stream : st);
    P->last_stream = st;
    const int64_t N = P->N, M = P->M, Mp = P->Mp, p = P->p;
    const int64_t ldw = N * Mp, ldft = p * Mp, ldxi = (p + 2) * Mp, ldsp = (int64_t)P->nchunks * Mp;
    BatchSys& S = sys[q];
    std::memset(&S, 0, sizeof(S));
    S.sweep.ks = P->d_ks; S.sweep.Dinv = P->Dlp; S.sweep.alpha = P->Alp; S.sweep.adiag = P->adiag;
    S.sweep.F = F[q]; S.sweep.ldf = ldf[q]; S.sweep.W = P->W32;
    S.sweep.N = (int32_t)N; S.sweep.M = (int32_t)M; S.sweep.Mp = (int32_t)Mp; S.sweep.p = (int32_t)p;
    S.sweep.K = (int32_t)Kq;
    S.sup.ks = P->d_ks; S.sup.UV = P->UVlp; S.sup.Xi = P->Xi; S.sup.ldxi = ldxi;
    S.sup.W = P->W32; S.sup.X = X[q]; S.sup.ldx = ldx[q];
    S.sup.N = (int32_t)N; S.sup.M = (int32_t)M; S.sup.Mp = (int32_t)Mp; S.sup.p = (int32_t)p; S.sup.K = (int32_t)Kq;
    S.sweep64.ks = P->d_ks; S.sweep64.Dinv = P->Dinv; S.sweep64.alpha = P->alpha; S.sweep64.adiag = P->adiag;
    S.sweep64.F = F[q]; S.sweep64.ldf = ldf[q]; S.sweep64.W = P->Wbuf; S.sweep64.ldw = ldw;
    S.sweep64.N = (int32_t)N; S.sweep64.M = (int32_t)M; S.sweep64.Mp = (int32_t)Mp; S.sweep64.p = (int32_t)p;
    S.sweep64.K = (int32_t)Kq;
    S.sup64.ks = P->d_ks; S.sup64.UV = P->UVa ? P->UVa + 2 * Mp * Mp : nullptr; S.sup64.Xi = P->Xi;
    S.sup64.ldxi = ldxi; S.sup64.W = P->Wbuf; S.sup64.ldw = ldw; S.sup64.X = X[q]; S.sup64.ldx = ldx[q];
    S.sup64.N = (int32_t)N; S.sup64.M = (int32_t)M; S.sup64.Mp = (int32_t)Mp; S.sup64.p = (int32_t)p;
    S.sup64.K = (int32_t)Kq;
    S.prec = P->prec;
    BArgs a = bargs_base((int)Mp);
    a.descs = P->d_part; a.nprob = P->n_part;
    a.A = P->G; a.lda = Mp; a.B = P->Ft; a.ldb = ldft; a.C = P->Sp; a.ldc = ldsp; a.ncols = (int32_t)Kq;
    S.part = a;
    for (int lv = 0; lv < P->depth; ++lv) {
      BArgs b = bargs_base((int)Mp);
      b.descs = P->d_corr + P->corr_begin[lv]; b.nprob = P->corr_count[lv];
      b.A = P->H; b.lda = Mp; b.B = P->Xi; b.ldb = ldxi;
      b.Sp = P->Sp; b.ldsp = ldsp; b.spstride = Mp;
      b.C = P->Xi; b.ldc = ldxi;
      b.X2 = X[q]; b.ldx2 = ldx[q]; b.x2rows = (int32_t)M;
      b.ncols = (int32_t)Kq;
      S.lev[lv] = b;
    }
    S.Ft = P->Ft; S.ldft = ldft; S.adiag = P->adiag; S.bdiag = P->bdiag;
    S.F = F[q]; S.ldf = ldf[q]; S.X = X[q]; S.ldx = ldx[q];
    S.R = check ? B->dalloc<double>((size_t)(N * M * Kq)) : nullptr;
    S.ldr = N * M;
    S.cA = P->cA; S.cB = P->cB; S.cC = P->cC;
    S.nchunk = residual_row_chunks(N * M);
    S.colpart = check ? B->dalloc<double>((size_t)(S.nchunk * Kq * 2)) : nullptr;
    S.resid = nullptr;  // set below
    S.N = (int32_t)N; S.M = (int32_t)M; S.Mp = (int32_t)Mp; S.p = (int32_t)p; S.K = (int32_t)Kq;
    S.rt = (int32_t)(Mp / 64);
    S.rescols = RES_COLS;
    S.tol = tol;
    nst[q] = 6 + P->depth;
    cbase[q] = nctr;
    nctr += passes * nst[q];
  }
  B->d_resid = B->dalloc<double>((size_t)n * passes);
  for (int q = 0; q < n; ++q) sys[q].resid = B->d_resid + (int64_t)q * passes;

  // ---- work list in topological order: (pass, stage) outer, systems inner
  std::vector<BatchItem> items;
  auto ctr = [&](int q, int r, int stage) { return cbase[q] + r * nst[q] + stage; };
  std::vector<int> order(n);
  for (int q = 0; q < n; ++q) order[q] = q;
  // longest sweeps first (they are the longest single items)
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const td_plan_s *a = plans[x], *b = plans[y];
    const double wa = (double)(a->N / a->p) * a->Mp * a->Mp, wb = (double)(b->N / b->p) * b->Mp * b->Mp;
    return wa > wb;
  });
  // column tiles per item type: float64 sweeps, superpositions and all dichotomy products use 16
  // columns, float32 sweeps and superpositions 32
  std::vector<int> nct_sw(n), nct_bg(n), nct_sup(n);
  std::vector<int> cnt_sweep(n), cnt_ft(n), cnt_part(n), cnt_sup(n), cnt_res(n);
  std::vector<std::vector<int>> cnt_lev(n);
  for (int q = 0; q < n; ++q) {
    td_plan_s* P = plans[q];
    const int w = (P->prec == TD_PREC_F64) ? 16 : 32;
    nct_sw[q] = nct_sup[q] = (int)((K[q] + w - 1) / w);
    nct_bg[q] = (int)((K[q] + 15) / 16);
    cnt_sweep[q] = (int)P->p * nct_sw[q];
    cnt_ft[q] = (int)((P->p * P->Mp * K[q] + 16383) / 16384);
    cnt_part[q] = P->n_part * nct_bg[q];
    cnt_lev[q].resize(P->depth);
    for (int lv = 0; lv < P->depth; ++lv) cnt_lev[q][lv] = P->corr_count[lv] * nct_bg[q];
    cnt_sup[q] = (int)P->p * nct_sup[q];
    cnt_res[q] = sys[q].nchunk * (int)((K[q] + RES_COLS - 1) / RES_COLS);
  }
  int maxdepth = 0;
  for (int q = 0; q < n; ++q) maxdepth = std::max(maxdepth, plans[q]->depth);
  auto add = [&](int type, int q, int r, int lvl, int i0, int i1, int dep, int need, int mine) {
    BatchItem it;
    it.type = type; it.sys = q; it.pass = r; it.lvl = lvl; it.i0 = i0; it.i1 = i1;
    it.dep = dep; it.need = need; it.mine = mine; it.pad_ = 0;
    items.push_back(it);
  };
  std::vector<int> stage_begin;
  auto stage = [&]() { stage_begin.push_back((int)items.size()); };
  for (int r = 0; r < passes; ++r) {
    stage();
    for (int q : order) {   // sweeps
      td_plan_s* P = plans[q];
      const int nct = nct_sw[q];
      const int dep = r == 0 ? -1 : ctr(q, r - 1, 5 + P->depth);
      for (int s = 0; s < P->p; ++s)
        for (int c = 0; c < nct; ++c) add(BI_SWEEP, q, r, 0, s, c, dep, r == 0 ? 0 : 1, ctr(q, r, 0));
    }
    stage();
    for (int q : order)
      for (int c = 0; c < cnt_ft[q]; ++c) add(BI_FTILDE, q, r, 0, c, 0, ctr(q, r, 0), cnt_sweep[q], ctr(q, r, 1));
    stage();
    for (int q : order) {
      td_plan_s* P = plans[q];
      const int nct = nct_bg[q];
      for (int pr = 0; pr < P->n_part; ++pr)
        for (int c = 0; c < nct; ++c) add(BI_PART, q, r, 0, pr, c, ctr(q, r, 1), cnt_ft[q], ctr(q, r, 2));
    }
    for (int lv = 0; lv < maxdepth; ++lv) {
      stage();
      for (int q : order) {
        td_plan_s* P = plans[q];
        if (lv >= P->depth) continue;
        const int nct = nct_bg[q];
        const int dep = lv == 0 ? ctr(q, r, 2) : ctr(q, r, 3 + lv - 1);
        const int need = lv == 0 ? cnt_part[q] : cnt_lev[q][lv - 1];
        for (int pr = 0; pr < P->corr_count[lv]; ++pr)
          for (int c = 0; c < nct; ++c) add(BI_LEVEL, q, r, lv, pr, c, dep, need, ctr(q, r, 3 + lv));
      }
    }
    stage();
    for (int q : order) {
      td_plan_s* P = plans[q];
      const int nct = cnt_sup[q] / (int)P->p;
      for (int s = 0; s < P->p; ++s)
        for (int c = 0; c < nct; ++c)
          add(BI_SUP, q, r, 0, s, c, ctr(q, r, 3 + P->depth - 1), cnt_lev[q][P->depth - 1], ctr(q, r, 3 + P->depth));
    }
    if (!check) continue;
    stage();
    for (int q : order) {
      td_plan_s* P = plans[q];
      for (int ch = 0; ch < sys[q].nchunk; ++ch)
        for (int c0 = 0; c0 < K[q]; c0 += RES_COLS)
          add(BI_RES, q, r, 0, ch, c0, ctr(q, r, 3 + P->depth), cnt_sup[q], ctr(q, r, 4 + P->depth));
    }
    stage();
    for (int q : order) {
      td_plan_s* P = plans[q];
      add(BI_RFIN, q, r, 0, 0, 0, ctr(q, r, 4 + P->depth), cnt_res[q], ctr(q, r, 5 + P->depth));
    }
  }
  stage();
  B->nitems = (int)items.size();
  B->d_items = B->upload(items);
  B->d_sys = B->upload(sys);
  B->ncounters = nctr;
  B->d_counters = B->dalloc<int32_t>((size_t)nctr);
  B->d_conv = B->dalloc<int32_t>((size_t)n);
  B->d_ctl = B->dalloc<BatchCtl>(1);
  int dev = 0, cus = 0, occ = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  occ = batched_blocks_per_cu();
  B->grid = cus * occ;
  // capture the reset + persistent launch once, on a private stream (the caller's stream may be
  // the legacy default stream, which cannot be captured); replays go to the caller's stream
  B->d_heads = B->dalloc<int32_t>(stage_begin.size());
  HIPCHK(hipStreamSynchronize(st));
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  hipError_t le = hipSuccess, ce = hipSuccess;
  hipGraph_t g = nullptr;
  if (be == hipSuccess) {
    // default: one launch per stage (measured faster: no per-item cache maintenance); with
    // TD_BATCH_MODE=persistent, one persistent launch with counted dependencies
    const char* mode = std::getenv("TD_BATCH_MODE");
    if (mode && std::strcmp(mode, "persistent") == 0) {
      le = launch_batched(B->d_items, B->nitems, B->d_sys, B->d_counters, B->ncounters, B->d_conv, n, B->d_ctl,
                          B->grid, (int64_t)1 << 26, cs);
    } else {
      const int nst = (int)stage_begin.size() - 1;
      le = launch_batched_stages(B->d_items, stage_begin.data(), nst, B->d_sys, B->d_heads, B->d_conv, n, B->d_ctl,
                                 B->grid, cs);
    }
    ce = hipStreamEndCapture(cs, &g);
  }
  (void)hipStreamDestroy(cs);
  HIPCHK(be);
  HIPCHK(le);
  HIPCHK(ce);
  B->graph = g;
  HIPCHK(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  B->last = st;
  return TD_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Fixed device workspace of tridiag_solve_noalloc: one array per GPU, held from the library's load
// until the process ends, shared by every no-allocation solve on that GPU (so such calls must not
// overlap on one GPU).  Host code never uses the array's name as a device address: the address of
// each device's copy comes from hipGetSymbolAddress, once per device, with that device current.
// ------------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// address of the current device's scratch array (looked up on the first call on that device)
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// pieces of a solve's workspace in the scratch array, each 256-byte aligned; returns the bytes used
int64_t scratch_layout(const td_plan_s* P, int64_t K, char* base, Work* w, int64_t* clear_doubles) {
  const int64_t N = P->N, Mp = P->Mp, p = P->p;
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  if (P->scalar) {   // Xt, then Pt (both fully written by every pass)
    const int64_t bXt = up((int64_t)P->sc.ntop * K * 8), bPt = up((int64_t)P->sc.L0 * P->sc.nsub * K * 8);
    if (w) {
      *w = Work{};
      w->Xi = (double*)base;
      w->Sp = (double*)(base + bXt);
    }
    if (clear_doubles) *clear_doubles = 0;
    return bXt + bPt;
  }
  // Xi, Ft, Sp and Pbuf first (cleared on every call), then W
  const int64_t bXi = up((p + 2) * Mp * K * 8), bFt = up(p * Mp * K * 8), bSp = up((int64_t)P->nchunks * Mp * K * 8);
  const int64_t bP = up((int64_t)P->pslots * Mp * K * 8);
  const int64_t bW = (P->prec == TD_PREC_F64) ? up(N * Mp * K * 8) : up(w32_floats(N, Mp, K) * 4);
  if (w) {
    w->Xi = (double*)base;
    w->Ft = (double*)(base + bXi);
    w->Sp = (double*)(base + bXi + bFt);
    w->Pbuf = P->pslots > 0 ? (double*)(base + bXi + bFt + bSp) : nullptr;
    char* wb = base + bXi + bFt + bSp + bP;
    w->W = (P->prec == TD_PREC_F64) ? (double*)wb : nullptr;
    w->W32 = (P->prec == TD_PREC_F64) ? nullptr : (float*)wb;
  }
  if (clear_doubles) *clear_doubles = (bXi + bFt + bSp + bP) / 8;
  return bXi + bFt + bSp + bP + bW;
}

}  // namespace

extern "C" {

td_status tridiag_factor(const td_desc* desc, const double* A, const double* B, const double* C, void* stream,
                         td_plan* out) {
  if (!out) return fail(TD_EINVAL, "null out");
  *out = nullptr;
  g_err.clear();
  return factor_top(desc, A, B, C, (hipStream_t)stream, out, true);
}

td_status tridiag_default_subdomains(int64_t N, int64_t K, int64_t* p) {
  g_err.clear();
  if (!p) return fail(TD_EINVAL, "null p");
  if (N < 1) return fail(TD_EINVAL, "N must be >= 1");
  *p = default_subdomains(N, K);
  return TD_OK;
}

td_status tridiag_plan_bytes(const td_desc* desc, int64_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(TD_EINVAL, "null bytes");
  td_status s = check_desc(desc);
  if (s != TD_OK) return s;
  const int64_t p = desc->subdomains ? desc->subdomains : default_subdomains(desc->N, desc->k_hint);
  int64_t b = factor_bytes(desc->N, desc->M, p, desc->fmt_A, desc->fmt_B, desc->fmt_C, desc->sweep_prec);
  if (desc->adjoint) b *= 2;
  *bytes = b;
  return TD_OK;
}

td_status tridiag_solve(td_plan plan, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                        const td_refine* refine, td_info* info, void* stream) {
  if (!plan) return fail(TD_EINVAL, "null plan");
  g_err.clear();
  try {
    return solve_impl(plan, F, ldf, X, ldx, K, refine, info, (hipStream_t)stream);
  } catch (const HipFail& e) {
    const td_status code = (e.e == hipErrorOutOfMemory) ? TD_ENOMEM : TD_EHIP;
    return fail(code, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  }
}

td_status tridiag_solve_noalloc(td_plan plan, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                                void* stream) {
  if (!plan) return fail(TD_EINVAL, "null plan");
  g_err.clear();
  td_plan_s* P = plan;
  const int64_t n = P->N * P->M;
  if (K < 0 || ldf < n || ldx < n) return fail(TD_EINVAL, "K < 0 or leading dimension below N*M");
  if (K > INT_MAX / 2) return fail(TD_EINVAL, "K too large");
  if (K == 0) return TD_OK;
  if (!F || !X) return fail(TD_EINVAL, "null F or X");
  const char* f0 = (const char*)F;
  const char* f1 = (const char*)(F + (K - 1) * ldf + n);
  const char* x0 = (const char*)X;
  const char* x1 = (const char*)(X + (K - 1) * ldx + n);
  if (f0 < x1 && x0 < f1) return fail(TD_EINVAL, "X overlaps F");
  const int64_t need = scratch_layout(P, K, nullptr, nullptr, nullptr);
  if (need > (int64_t)kScratchBytes)
    return fail(TD_EINVAL, "the solve needs " + std::to_string(need) + " bytes of workspace, above the fixed " +
                               std::to_string(kScratchBytes) + "-byte scratch array of tridiag_solve_noalloc");
  const hipStream_t st = (hipStream_t)stream;
  try {
    void* base = nullptr;
    HIPCHK(scratch_address(&base));
    Work w{};
    int64_t nclear = 0;
    scratch_layout(P, K, (char*)base, &w, &nclear);
    // the array keeps the previous call's contents: the interface solution's zero end blocks and
    // the pieces a pass reads before writing (padded rows) start from zero
    HIPCHK(launch_fill((double*)base, nclear, 0.0, st));
    P->last_stream = st;
    P->first_pass = false;
    solve_pass(P, w, F, ldf, X, ldx, K, false, st);
  } catch (const HipFail& e) {
    return fail(TD_EHIP, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  }
  return TD_OK;
}

td_status tridiag_solve_adjoint(td_plan plan, const double* G, int64_t ldg, double* Lam, int64_t ldl, int64_t K,
                                const td_refine* refine, td_info* info, void* stream) {
  if (!plan) return fail(TD_EINVAL, "null plan");
  if (!plan->adj) return fail(TD_ENOADJ, "plan was factored without the transpose (desc.adjoint == 0)");
  return tridiag_solve(plan->adj, G, ldg, Lam, ldl, K, refine, info, stream);
}

td_status tridiag_diag_grad(const double* Lam, int64_t ldl, const double* X, int64_t ldx, int64_t n, int64_t K,
                            double* out, void* stream) {
  g_err.clear();
  if (!Lam || !X || !out) return fail(TD_EINVAL, "null pointer");
  if (n < 0 || K < 0 || ldl < n || ldx < n) return fail(TD_EINVAL, "bad sizes");
  if (K > INT_MAX) return fail(TD_EINVAL, "K too large");
  hipError_t e = launch_diag_grad(out, Lam, ldl, X, ldx, n, (int)K, (hipStream_t)stream);
  if (e != hipSuccess) return fail(TD_EHIP, hipGetErrorString(e));
  return TD_OK;
}

td_status tridiag_destroy(td_plan plan) {
  if (!plan) return TD_OK;
  if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
  else (void)hipDeviceSynchronize();
  if (plan->adj && plan->adj->last_stream && plan->adj->last_stream != plan->last_stream)
    (void)hipStreamSynchronize(plan->adj->last_stream);
  delete plan;
  return TD_OK;
}

td_status tridiag_plan_info(td_plan plan, td_plan_info* out) {
  if (!plan || !out) return fail(TD_EINVAL, "null argument");
  out->N = plan->N; out->M = plan->M; out->subdomains = plan->p; out->Mp = plan->Mp;
  out->tree_depth = plan->depth;
  out->device_bytes = plan->bytes + (plan->adj ? plan->adj->bytes : 0);
  out->factor_ms = plan->factor_ms;
  out->sweep_prec = plan->prec;
  out->adjoint = plan->adj != nullptr;
  return TD_OK;
}

td_status tridiag_set_profiling(td_plan plan, int enable) {
  if (!plan) return fail(TD_EINVAL, "null plan");
  plan->prof = enable != 0;
  if (plan->adj) plan->adj->prof = enable != 0;
  return TD_OK;
}

td_status tridiag_stage_times(td_plan plan, double* ms, int n) {
  if (!plan || !ms || n < 0) return fail(TD_EINVAL, "bad argument");
  if (plan->prof_n == 0) return fail(TD_EINVAL, "no profiled solve since the last read-out");
  double acc[8] = {0};
  try {
    HIPCHK(hipEventSynchronize(plan->evsets[plan->prof_n - 1].ev[7]));
    for (int q = 0; q < plan->prof_n; ++q) {
      const StageEvents& s = plan->evsets[q];
      float t = 0.f;
      for (int i = 0; i < 5; ++i) {
        HIPCHK(hipEventElapsedTime(&t, s.ev[i], s.ev[i + 1]));
        acc[i] += t;
      }
      HIPCHK(hipEventElapsedTime(&t, s.ev[5], s.ev[7]));
      acc[5] += t;
      HIPCHK(hipEventElapsedTime(&t, s.ev[6], s.ev[7]));
      acc[6] += t;
    }
  } catch (const HipFail& e) {
    return fail(TD_EHIP, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  }
  const double cnt = plan->prof_n;
  for (int i = 0; i < n && i < 7; ++i) ms[i] = acc[i] / cnt;
  if (n >= 8) ms[7] = cnt;
  plan->prof_n = 0;
  return TD_OK;
}

td_status tridiag_set_tiles(td_plan plan, const td_tiles* tiles) {
  if (!plan) return fail(TD_EINVAL, "null plan");
  td_tiles t{};
  if (tiles) t = *tiles;
  for (td_plan_s* P : {plan, plan->adj}) {
    if (!P) continue;
    P->tiles = t;
    P->drop_graph();
  }
  return TD_OK;
}

td_status tridiag_get_tiles(td_plan plan, td_tiles* tiles) {
  if (!plan || !tiles) return fail(TD_EINVAL, "bad argument");
  *tiles = plan->tiles;
  return TD_OK;
}

const char* tridiag_status_string(td_status s) {
  switch (s) {
    case TD_OK: return "TD_OK";
    case TD_EINVAL: return "TD_EINVAL: invalid argument";
    case TD_ENOMEM: return "TD_ENOMEM: not enough device memory";
    case TD_ESINGULAR: return "TD_ESINGULAR: singular pivot block";
    case TD_ENOCONV: return "TD_ENOCONV: refinement did not converge";
    case TD_ENOADJ: return "TD_ENOADJ: plan has no transposed factor";
    case TD_EHIP: return "TD_EHIP: HIP runtime error";
    case TD_ENOTSUP: return "TD_ENOTSUP: unsupported combination";
  }
  return "unknown status";
}

const char* tridiag_last_error(void) { return g_err.c_str(); }

td_status tridiag_band_to_blocks(int64_t n, int32_t kl, int32_t ku, const double* ab, int64_t ldab, int64_t M,
                                 double* A, double* B, double* C, void* stream) {
  g_err.clear();
  if (n < 1 || kl < 0 || ku < 0) return fail(TD_EINVAL, "n must be >= 1 and kl, ku >= 0");
  if (ldab < (int64_t)kl + ku + 1) return fail(TD_EINVAL, "ldab must be >= kl + ku + 1");
  if (M < 1 || M < kl || M < ku) return fail(TD_EINVAL, "block size M must be >= max(kl, ku, 1)");
  if (M > 512) return fail(TD_ENOTSUP, "M > 512 is not supported");
  if (!ab || !A || !B || !C) return fail(TD_EINVAL, "null pointer");
  const int64_t N = (n + M - 1) / M;
  hipError_t e = launch_band_to_blocks(n, kl, ku, ab, ldab, (int)M, N, A, B, C, (hipStream_t)stream);
  if (e != hipSuccess) return fail(TD_EHIP, hipGetErrorString(e));
  return TD_OK;
}

td_status tridiag_autotune(int64_t M, int64_t K, int32_t sweep_prec, int64_t probe_N, const int64_t* candidates,
                           int ncand, void* stream, int64_t* best_L, double* ms_per_solve) {
  g_err.clear();
  if (M < 1 || M > 512 || K < 1 || probe_N < 2 || !candidates || ncand < 1 || !best_L)
    return fail(TD_EINVAL, "bad autotune arguments");
  hipStream_t st = (hipStream_t)stream;
  double *A = nullptr, *B = nullptr, *C = nullptr, *F = nullptr, *X = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  td_status result = TD_OK;
  try {
    HIPCHK(hipMalloc((void**)&A, probe_N * M * 8));
    HIPCHK(hipMalloc((void**)&B, probe_N * M * 8));
    HIPCHK(hipMalloc((void**)&C, probe_N * 3 * M * 8));
    HIPCHK(hipMalloc((void**)&F, probe_N * M * K * 8));
    HIPCHK(hipMalloc((void**)&X, probe_N * M * K * 8));
    HIPCHK(launch_probe_inputs(A, B, C, F, (int)probe_N, (int)M, K, st));
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = INFINITY;
    *best_L = candidates[0];
    for (int c = 0; c < ncand; ++c) {
      const int64_t L = std::max<int64_t>(1, candidates[c]);
      td_desc d;
      std::memset(&d, 0, sizeof d);
      d.N = probe_N; d.M = M; d.subdomains = std::max<int64_t>(1, probe_N / L);
      d.fmt_A = TD_FMT_DIAG; d.fmt_B = TD_FMT_DIAG; d.fmt_C = TD_FMT_TRIDIAG; d.sweep_prec = sweep_prec;
      td_plan Pr = nullptr;
      td_status s = factor_top(&d, A, B, C, st, &Pr, false);
      if (s != TD_OK) { result = s; break; }
      std::unique_ptr<td_plan_s> P(Pr);   // freed on every exit, also when a HIP call throws
      s = solve_impl(P.get(), F, probe_N * M, X, probe_N * M, K, nullptr, nullptr, st);
      if (s != TD_OK) { result = s; break; }
      HIPCHK(hipEventRecord(e0, st));
      for (int r = 0; r < 3 && s == TD_OK; ++r)
        s = solve_impl(P.get(), F, probe_N * M, X, probe_N * M, K, nullptr, nullptr, st);
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      if (s != TD_OK) { result = s; break; }
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms_per_solve) ms_per_solve[c] = ms / 3.0;
      if (ms / 3.0 < best) { best = ms / 3.0; *best_L = L; }
    }
  } catch (const HipFail& e) {
    result = fail(e.e == hipErrorOutOfMemory ? TD_ENOMEM : TD_EHIP,
                  std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(A); (void)hipFree(B); (void)hipFree(C); (void)hipFree(F); (void)hipFree(X);
  return result;
}

td_status tridiag_autotune_tiles(int64_t M, int64_t K, int32_t sweep_prec, int64_t probe_N,
                                 const int64_t* candidates, int ncand, void* stream, int64_t* best_L,
                                 td_tiles* best_tiles, double* best_ms) {
  g_err.clear();
  if (M < 1 || M > 512 || K < 1 || probe_N < 2 || !candidates || ncand < 1 || !best_L || !best_tiles)
    return fail(TD_EINVAL, "bad autotune arguments");
  hipStream_t st = (hipStream_t)stream;
  double *A = nullptr, *B = nullptr, *C = nullptr, *F = nullptr, *X = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  td_status result = TD_OK;
  try {
    HIPCHK(hipMalloc((void**)&A, probe_N * M * 8));
    HIPCHK(hipMalloc((void**)&B, probe_N * M * 8));
    HIPCHK(hipMalloc((void**)&C, probe_N * 3 * M * 8));
    HIPCHK(hipMalloc((void**)&F, probe_N * M * K * 8));
    HIPCHK(hipMalloc((void**)&X, probe_N * M * K * 8));
    HIPCHK(launch_probe_inputs(A, B, C, F, (int)probe_N, (int)M, K, st));
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = INFINITY;
    *best_L = candidates[0];
    *best_tiles = td_tiles{};
    const int64_t Mp = pad_block(M, sweep_prec);
    // alternatives of each field: column counts of the precision, and the wave counts (16, 32 or
    // 64 rows per wave, at most 8 waves) that the padded block size allows
    std::vector<int32_t> cols = (sweep_prec == TD_PREC_F64) ? std::vector<int32_t>{16, 32}
                                                            : std::vector<int32_t>{16, 32, 64};
    std::vector<int32_t> waves;
    for (int rt : {1, 2, 4})
      if (Mp % (16 * rt) == 0 && Mp / (16 * rt) <= 8) waves.push_back((int32_t)(Mp / (16 * rt)));
    for (int c = 0; c < ncand && result == TD_OK; ++c) {
      const int64_t L = std::max<int64_t>(1, candidates[c]);
      td_desc d;
      std::memset(&d, 0, sizeof d);
      d.N = probe_N; d.M = M; d.subdomains = std::max<int64_t>(1, probe_N / L);
      d.fmt_A = TD_FMT_DIAG; d.fmt_B = TD_FMT_DIAG; d.fmt_C = TD_FMT_TRIDIAG; d.sweep_prec = sweep_prec;
      td_plan Pr = nullptr;
      td_status s = factor_top(&d, A, B, C, st, &Pr, false);
      if (s != TD_OK) { result = s; break; }
      std::unique_ptr<td_plan_s> P(Pr);   // freed on every exit, also when a HIP call throws
      auto time_tiles = [&](const td_tiles& t, double& ms_out) -> td_status {
        P->tiles = t;
        P->drop_graph();
        td_status r = solve_impl(P.get(), F, probe_N * M, X, probe_N * M, K, nullptr, nullptr, st);
        if (r != TD_OK) return r;
        HIPCHK(hipEventRecord(e0, st));
        for (int k = 0; k < 3 && r == TD_OK; ++k)
          r = solve_impl(P.get(), F, probe_N * M, X, probe_N * M, K, nullptr, nullptr, st);
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        if (r != TD_OK) return r;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        ms_out = ms / 3.0;
        return TD_OK;
      };
      td_tiles cur{};
      double cur_ms = 0.0;
      if ((s = time_tiles(cur, cur_ms)) != TD_OK) { result = s; break; }
      // one field at a time against the rules; then the best of every field together
      td_tiles comb{};
      int32_t td_tiles::*fields[4] = {&td_tiles::sweep_cols, &td_tiles::sweep_waves, &td_tiles::sup_cols,
                                      &td_tiles::sup_waves};
      for (int f = 0; f < 4 && s == TD_OK; ++f) {
        const std::vector<int32_t>& opts = (f % 2 == 0) ? cols : waves;
        double fbest = cur_ms;
        for (int32_t v : opts) {
          td_tiles t{};
          t.*fields[f] = v;
          double ms = 0.0;
          if ((s = time_tiles(t, ms)) != TD_OK) break;
          if (ms < fbest) { fbest = ms; comb.*fields[f] = v; }
        }
      }
      if (s != TD_OK) { result = s; break; }
      double comb_ms = cur_ms;
      const bool any = comb.sweep_cols || comb.sweep_waves || comb.sup_cols || comb.sup_waves;
      if (any && (s = time_tiles(comb, comb_ms)) != TD_OK) { result = s; break; }
      const td_tiles win = (any && comb_ms < cur_ms) ? comb : td_tiles{};
      const double win_ms = (any && comb_ms < cur_ms) ? comb_ms : cur_ms;
      if (win_ms < best) {
        best = win_ms;
        *best_L = L;
        *best_tiles = win;
      }
    }
    if (best_ms) *best_ms = best;
  } catch (const HipFail& e) {
    result = fail(e.e == hipErrorOutOfMemory ? TD_ENOMEM : TD_EHIP,
                  std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(A); (void)hipFree(B); (void)hipFree(C); (void)hipFree(F); (void)hipFree(X);
  return result;
}

td_status tridiag_batch_create(int n, const td_plan* plans, const double* const* F, const int64_t* ldf,
                               double* const* X, const int64_t* ldx, const int64_t* K, int passes, double tol,
                               void* stream, td_batch* out) {
  if (!out) return fail(TD_EINVAL, "null out");
  *out = nullptr;
  g_err.clear();
  td_batch_s* B = new td_batch_s();
  td_status s;
  try {
    s = batch_create_impl(n, plans, F, ldf, X, ldx, K, passes, tol == 0.0 ? 1e-10 : tol, (hipStream_t)stream, B);
  } catch (const HipFail& e) {
    s = fail(e.e == hipErrorOutOfMemory ? TD_ENOMEM : TD_EHIP,
             std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  }
  if (s != TD_OK) {
    delete B;
    return s;
  }
  *out = B;
  return TD_OK;
}

td_status tridiag_batch_solve(td_batch b, void* stream) {
  if (!b) return fail(TD_EINVAL, "null batch");
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(TD_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  b->last = (hipStream_t)stream;
  return TD_OK;
}

td_status tridiag_batch_info(td_batch b, td_info* infos) {
  if (!b || !infos) return fail(TD_EINVAL, "null argument");
  BatchCtl ctl;
  std::vector<int32_t> conv(b->n);
  std::vector<double> res((size_t)b->n * b->passes);
  hipError_t e = hipStreamSynchronize(b->last);
  if (e == hipSuccess) e = hipMemcpy(&ctl, b->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(conv.data(), b->d_conv, b->n * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(res.data(), b->d_resid, res.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(TD_EHIP, hipGetErrorString(e));
  if (ctl.error) return fail(TD_EHIP, "a dependency wait of the batched kernel timed out");
  bool allconv = true;
  if (!b->check) {
    for (int q = 0; q < b->n; ++q) {
      infos[q].iterations = 0;
      infos[q].nonfinite = 0;
      infos[q].max_col_rel_residual = -1.0;
    }
    return TD_OK;
  }
  for (int q = 0; q < b->n; ++q) {
    const int last = conv[q] < b->passes ? conv[q] : b->passes - 1;
    infos[q].iterations = last;
    infos[q].nonfinite = std::isfinite(res[(size_t)q * b->passes + last]) ? 0 : 1;
    infos[q].max_col_rel_residual = res[(size_t)q * b->passes + last];
    if (conv[q] >= b->passes) allconv = false;
  }
  if (!allconv) return fail(TD_ENOCONV, "some systems did not reach the residual tolerance within the passes");
  return TD_OK;
}

td_status tridiag_batch_destroy(td_batch b) {
  if (!b) return TD_OK;
  if (b->last) (void)hipStreamSynchronize(b->last);
  delete b;
  return TD_OK;
}

td_status tridiag_solve_batched(int n, const td_plan* plans, const double* const* F, double* const* X,
                                const int64_t* K, const td_refine* refine, td_info* infos, void* stream) {
  // the batch of the last call, replayed while the arguments stay the same
  static struct {
    std::vector<td_plan> plans;
    std::vector<const double*> F;
    std::vector<double*> X;
    std::vector<int64_t> K;
    int passes = 0;
    double tol = 0.0;
    td_batch b = nullptr;
  } cache;
  g_err.clear();
  if (n == 0) {
    if (cache.b) (void)tridiag_batch_destroy(cache.b);
    cache.b = nullptr;
    cache.plans.clear();
    return TD_OK;
  }
  if (n < 0 || !plans || !F || !X || !K) return fail(TD_EINVAL, "bad batched arguments");
  const bool ref = refine && refine->enable;
  const int passes = ref ? 1 + (refine->max_iter > 0 ? refine->max_iter : 2) : 1;
  const double tol = ref ? (refine->tol > 0.0 ? refine->tol : 1e-10) : -1.0;
  const bool same = cache.b && (int)cache.plans.size() == n && cache.passes == passes && cache.tol == tol &&
                    std::equal(plans, plans + n, cache.plans.begin()) && std::equal(F, F + n, cache.F.begin()) &&
                    std::equal(X, X + n, cache.X.begin()) && std::equal(K, K + n, cache.K.begin());
  if (!same) {
    if (cache.b) (void)tridiag_batch_destroy(cache.b);
    cache.b = nullptr;
    cache.plans.clear();
    std::vector<int64_t> ld(n);
    for (int q = 0; q < n; ++q) {
      if (!plans[q]) return fail(TD_EINVAL, "null plan");
      ld[q] = plans[q]->N * plans[q]->M;
    }
    td_batch b = nullptr;
    td_status s = tridiag_batch_create(n, plans, F, ld.data(), X, ld.data(), K, passes, tol, stream, &b);
    if (s != TD_OK) return s;
    cache.b = b;
    cache.plans.assign(plans, plans + n);
    cache.F.assign(F, F + n);
    cache.X.assign(X, X + n);
    cache.K.assign(K, K + n);
    cache.passes = passes;
    cache.tol = tol;
  }
  td_status s = tridiag_batch_solve(cache.b, stream);
  if (s != TD_OK || !infos) return s;
  return tridiag_batch_info(cache.b, infos);
}

}  // extern "C"
