// Schur-complement solver on interface block rows (Sec. 3: eqs. (linear_decomp), (schur_decomp),
// (domains_equation), the conjugate-gradient solution of eq. (schur_decomp) and its probing
// preconditioner), built on the block-tridiagonal plans of plan.cpp:
//   * the interior rows of all strips form one stacked block-tridiagonal system A_II (zero
//     couplings across strip boundaries), factored once; every product with A_II^{-1} is one
//     solve of that plan for all K columns;
//   * S v = A_GG v - A_GI A_II^{-1} A_IG v is a scatter, that solve and a gather;
//   * the probing preconditioner B (half-bandwidth d) comes from S applied to 2 (2d+1) probe
//     vectors; it is a band matrix, solved by a block-tridiagonal plan of its band blocks
//     (tridiag_band_to_blocks), as the paper proposes;
//   * preconditioned CG runs one independent iteration per right-hand side on the device; the
//     host reads two numbers per iteration (active columns, largest relative residual).
#include "schur_kernels.h"
#include "tridiag.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

using namespace td;

td_status td_set_error(td_status s, const char* msg);   // plan.cpp

namespace {

struct SchurFail {
  td_status s;
  std::string msg;
};

#define SCHK(x)                                                                                        \
  do {                                                                                                 \
    hipError_t e_ = (x);                                                                               \
    if (e_ != hipSuccess)                                                                              \
      throw SchurFail{e_ == hipErrorOutOfMemory ? TD_ENOMEM : TD_EHIP,                                 \
                      std::string("HIP error ") + hipGetErrorString(e_) + " in " #x};                  \
  } while (0)

#define TDCHK(x)                                                                                       \
  do {                                                                                                 \
    td_status s_ = (x);                                                                                \
    if (s_ != TD_OK) throw SchurFail{s_, std::string(#x) + ": " + tridiag_last_error()};               \
  } while (0)

// device buffers of one construction step; freed on every exit path (hipFree waits for the
// device, so kernels still reading them finish first)
struct TmpBufs {
  std::vector<void*> v;
  void release() {
    for (void* ptr : v) (void)hipFree(ptr);
    v.clear();
  }
  ~TmpBufs() { release(); }
};

}  // namespace

struct td_schur_s {
  int64_t N = 0, M = 0, nif = 0, Nint = 0, ng = 0, nGp = 0, Mb = 0, Nb = 0;
  int band = -1;
  std::vector<int64_t> icol, intcol;
  int64_t *d_icol = nullptr, *d_intcol = nullptr, *d_ileft = nullptr, *d_iright = nullptr;
  int32_t *d_lif = nullptr, *d_rif = nullptr;
  double *cA = nullptr, *cB = nullptr, *cC = nullptr;   // whole-domain coefficients
  td_plan interior = nullptr, precond = nullptr;
  // workspace for up to `cap` columns
  int64_t cap = 0;
  double *T = nullptr, *Y = nullptr;                                     // stacked interior
  double *g = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;   // interface
  double *part = nullptr, *pq = nullptr, *rz = nullptr, *rz2 = nullptr, *rr = nullptr, *gg = nullptr;
  double *alpha = nullptr, *stat = nullptr;
  int32_t* active = nullptr;
  std::vector<void*> allocs, ws;
  hipStream_t last = nullptr;

  template <class T_>
  T_* dalloc(size_t n, std::vector<void*>& list) {
    void* ptr = nullptr;
    SCHK(hipMalloc(&ptr, std::max<size_t>(1, n) * sizeof(T_)));
    list.push_back(ptr);
    return (T_*)ptr;
  }
  template <class T_>
  T_* upload(const std::vector<T_>& v, hipStream_t st) {
    T_* ptr = dalloc<T_>(v.size(), allocs);
    if (!v.empty()) SCHK(hipMemcpyAsync(ptr, v.data(), v.size() * sizeof(T_), hipMemcpyHostToDevice, st));
    return ptr;
  }
  void free_ws() {
    for (void* ptr : ws) (void)hipFree(ptr);
    ws.clear();
    cap = 0;
  }
  void ensure_ws(int64_t K) {
    if (K <= cap) return;
    free_ws();
    const int64_t ni = Nint * M;
    T = dalloc<double>(ni * K, ws);
    Y = dalloc<double>(ni * K, ws);
    double** iv[] = {&g, &x, &r, &z, &p, &q};
    for (double** v : iv) *v = dalloc<double>(nGp * K, ws);
    part = dalloc<double>((size_t)schur_dot_parts(nGp) * K, ws);
    double** sv[] = {&pq, &rz, &rz2, &rr, &gg, &alpha};
    for (double** v : sv) *v = dalloc<double>(K, ws);
    stat = dalloc<double>(2, ws);
    active = dalloc<int32_t>(K, ws);
    cap = K;
  }
  ~td_schur_s() {
    (void)tridiag_destroy(interior);
    (void)tridiag_destroy(precond);
    free_ws();
    for (void* ptr : allocs) (void)hipFree(ptr);
  }

  // out (rows_out x K, ld ldo) = S V (V: nGp-padded or user interface vectors, ld ldv)
  void apply(const double* V, int64_t ldv, double* out, int64_t ldo, int64_t rows_out, int K, hipStream_t st) {
    const int64_t ni = Nint * M;
    SCHK(launch_schur_scatter(T, ni, nullptr, 0, V, ldv, cA, cB, d_intcol, d_lif, d_rif, Nint, (int)M, K, -1.0, st));
    TDCHK(tridiag_solve(interior, T, ni, Y, ni, K, nullptr, nullptr, st));
    SCHK(launch_schur_gather(out, ldo, nullptr, 0, V, ldv, Y, ni, cA, cB, cC, d_icol, d_ileft, d_iright, nif, (int)M,
                             rows_out, K, 1, st));
  }
  // z = B^{-1} r (or z = r without a preconditioner)
  void precondition(int K, hipStream_t st) {
    if (precond) TDCHK(tridiag_solve(precond, r, nGp, z, nGp, K, nullptr, nullptr, st));
    else SCHK(hipMemcpyAsync(z, r, (size_t)nGp * K * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
};

namespace {

td_status schur_create(int64_t N, int64_t M, const double* A, const double* B, const double* C, int64_t nif,
                       const int64_t* icol, int32_t band, hipStream_t st, td_schur* out) {
  if (!out) return td_set_error(TD_EINVAL, "null out");
  *out = nullptr;
  if (!A || !B || !C || !icol) return td_set_error(TD_EINVAL, "null pointer");
  if (N < 3 || M < 1) return td_set_error(TD_EINVAL, "need N >= 3 and M >= 1");
  if (M > 512) return td_set_error(TD_ENOTSUP, "M > 512");
  if (nif < 1 || nif > N / 2) return td_set_error(TD_EINVAL, "need 1 <= nif <= N/2 interface block rows");
  if (band < -1 || band > 64) return td_set_error(TD_EINVAL, "band must be -1 (no preconditioner) or 0..64");
  for (int64_t k = 0; k < nif; ++k) {
    const int64_t lo = (k == 0) ? 1 : icol[k - 1] + 2;
    if (icol[k] < lo || icol[k] > N - 2)
      return td_set_error(TD_EINVAL,
                          "interface block rows must increase, leave at least one interior row between two "
                          "interfaces and lie in [1, N-2]");
  }
  if (N * M > (int64_t)INT_MAX * 64) return td_set_error(TD_ENOTSUP, "system too large");
  // CG needs a symmetric matrix: A_{j+1} = B_j and a symmetric tridiagonal C_j
  std::vector<double> hA(N * M), hB(N * M), hC(N * 3 * M);
  if (hipMemcpy(hA.data(), A, N * M * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hB.data(), B, N * M * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hC.data(), C, N * 3 * M * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return td_set_error(TD_EHIP, "copy of the coefficients failed");
  auto close = [](double a, double b) { return std::fabs(a - b) <= 1e-14 * std::max(std::fabs(a), std::fabs(b)); };
  for (int64_t j = 0; j + 1 < N; ++j)
    for (int64_t i = 0; i < M; ++i)
      if (!close(hA[(j + 1) * M + i], hB[j * M + i]))
        return td_set_error(TD_EINVAL, "the Schur solver uses CG: P must be symmetric (A_{j+1} = B_j)");
  for (int64_t j = 0; j < N; ++j)
    for (int64_t i = 1; i < M; ++i)
      if (!close(hC[j * 3 * M + i], hC[j * 3 * M + 2 * M + i - 1]))
        return td_set_error(TD_EINVAL, "the Schur solver uses CG: every C_j must be symmetric");

  auto* S = new td_schur_s();
  try {
    S->N = N; S->M = M; S->nif = nif; S->band = band; S->last = st;
    S->icol.assign(icol, icol + nif);
    std::vector<int32_t> ifidx(N, -1);
    for (int64_t k = 0; k < nif; ++k) ifidx[S->icol[k]] = (int32_t)k;
    std::vector<int32_t> lif, rif;
    std::vector<int64_t> stk(N, -1);
    for (int64_t c = 0; c < N; ++c) {
      if (ifidx[c] >= 0) continue;
      stk[c] = (int64_t)S->intcol.size();
      S->intcol.push_back(c);
      lif.push_back(c > 0 ? ifidx[c - 1] : -1);
      rif.push_back(c + 1 < N ? ifidx[c + 1] : -1);
    }
    S->Nint = (int64_t)S->intcol.size();
    std::vector<int64_t> il(nif), ir(nif);
    for (int64_t k = 0; k < nif; ++k) { il[k] = stk[S->icol[k] - 1]; ir[k] = stk[S->icol[k] + 1]; }
    S->ng = nif * M;
    S->d_icol = S->upload(S->icol, st);
    S->d_intcol = S->upload(S->intcol, st);
    S->d_ileft = S->upload(il, st);
    S->d_iright = S->upload(ir, st);
    S->d_lif = S->upload(lif, st);
    S->d_rif = S->upload(rif, st);
    S->cA = S->dalloc<double>(N * M, S->allocs);
    S->cB = S->dalloc<double>(N * M, S->allocs);
    S->cC = S->dalloc<double>(N * 3 * M, S->allocs);
    SCHK(hipMemcpyAsync(S->cA, A, N * M * 8, hipMemcpyDeviceToDevice, st));
    SCHK(hipMemcpyAsync(S->cB, B, N * M * 8, hipMemcpyDeviceToDevice, st));
    SCHK(hipMemcpyAsync(S->cC, C, N * 3 * M * 8, hipMemcpyDeviceToDevice, st));

    // A_II: the stacked interior rows, one plan
    TmpBufs tmp;
    double* Ai = S->dalloc<double>(S->Nint * M, tmp.v);
    double* Bi = S->dalloc<double>(S->Nint * M, tmp.v);
    double* Ci = S->dalloc<double>(S->Nint * 3 * M, tmp.v);
    SCHK(launch_schur_interior_coeffs(Ai, Bi, Ci, S->cA, S->cB, S->cC, S->d_intcol, S->Nint, (int)M, st));
    td_desc d{};
    // subdomains of 16 rows: CG applies S to few columns (tens), so the sweeps need many
    // subdomains to fill the GPU (2047x256, K = 64: 28 ms per CG solve against 41 ms with 32 rows
    // and 31 ms with 8)
    d.N = S->Nint; d.M = M; d.subdomains = std::max<int64_t>(1, S->Nint / 16);
    d.fmt_A = TD_FMT_DIAG; d.fmt_B = TD_FMT_DIAG; d.fmt_C = TD_FMT_TRIDIAG; d.sweep_prec = TD_PREC_F64;
    td_status fs = tridiag_factor(&d, Ai, Bi, Ci, st, &S->interior);
    tmp.release();
    if (fs != TD_OK) throw SchurFail{fs, std::string("interior factor: ") + tridiag_last_error()};

    // probing preconditioner: band blocks of size Mb (>= d) over the padded interface vector
    if (band >= 0) {
      S->Mb = std::max<int64_t>(band, 32);
      S->Nb = (S->ng + S->Mb - 1) / S->Mb;
      S->nGp = S->Nb * S->Mb;
      const int w = 2 * band + 1;
      S->ensure_ws(2 * w);
      double* V = S->dalloc<double>(S->nGp * 2 * w, tmp.v);
      double* Yp = S->dalloc<double>(S->nGp * 2 * w, tmp.v);
      double* ab = S->dalloc<double>(S->ng * w, tmp.v);
      SCHK(launch_probe_vectors(V, S->nGp, S->nGp, S->ng, (int)M, band, st));
      S->apply(V, S->nGp, Yp, S->nGp, S->nGp, 2 * w, st);
      SCHK(launch_probe_band(ab, w, Yp, S->nGp, S->ng, (int)M, band, st));
      const int64_t bb = S->Nb * S->Mb * S->Mb;
      double* Ab = S->dalloc<double>(bb, tmp.v);
      double* Bb = S->dalloc<double>(bb, tmp.v);
      double* Cb = S->dalloc<double>(bb, tmp.v);
      TDCHK(tridiag_band_to_blocks(S->ng, band, band, ab, w, S->Mb, Ab, Bb, Cb, st));
      td_desc e{};
      // short subdomains: the band system is small, its sweeps are latency-bound, not MFMA-bound
      e.N = S->Nb; e.M = S->Mb; e.subdomains = std::max<int64_t>(1, S->Nb / 8);
      e.fmt_A = TD_FMT_DENSE; e.fmt_B = TD_FMT_DENSE; e.fmt_C = TD_FMT_DENSE; e.sweep_prec = TD_PREC_F64;
      fs = tridiag_factor(&e, Ab, Bb, Cb, st, &S->precond);
      tmp.release();
      if (fs != TD_OK) throw SchurFail{fs, std::string("probed preconditioner factor: ") + tridiag_last_error()};
    } else {
      S->nGp = S->ng;
    }
    SCHK(hipStreamSynchronize(st));
  } catch (const SchurFail& f) {
    delete S;
    return td_set_error(f.s, f.msg.c_str());
  }
  *out = S;
  return TD_OK;
}

td_status schur_solve(td_schur S, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K, double tol,
                      int32_t max_iter, td_schur_info* info, hipStream_t st) {
  const int64_t n = S->N * S->M;
  if (K < 0 || ldf < n || ldx < n) return td_set_error(TD_EINVAL, "K < 0 or leading dimension below N*M");
  if (K > INT_MAX / 4) return td_set_error(TD_EINVAL, "K too large");
  if (info) { info->iterations = 0; info->active = 0; info->max_rel_residual = 0.0; }
  if (K == 0) return TD_OK;
  if (!F || !X) return td_set_error(TD_EINVAL, "null F or X");
  if (!(tol > 0.0)) tol = 1e-10;
  if (max_iter <= 0) max_iter = 500;
  S->last = st;
  const int k = (int)K;
  const int64_t ni = S->Nint * S->M, ng = S->nGp;
  td_status status = TD_OK;
  try {
    S->ensure_ws(K);
    // right-hand side of eq. (schur_decomp): g = f_G - A_GI A_II^{-1} f_I
    SCHK(launch_schur_scatter(S->T, ni, F, ldf, nullptr, 0, S->cA, S->cB, S->d_intcol, S->d_lif, S->d_rif, S->Nint,
                              (int)S->M, k, 1.0, st));
    TDCHK(tridiag_solve(S->interior, S->T, ni, S->Y, ni, K, nullptr, nullptr, st));
    SCHK(launch_schur_gather(S->g, ng, F, ldf, nullptr, 0, S->Y, ni, S->cA, S->cB, S->cC, S->d_icol, S->d_ileft,
                             S->d_iright, S->nif, (int)S->M, ng, k, 0, st));
    // x = 0, r = g
    SCHK(hipMemsetAsync(S->x, 0, (size_t)ng * K * sizeof(double), st));
    SCHK(hipMemcpyAsync(S->r, S->g, (size_t)ng * K * sizeof(double), hipMemcpyDeviceToDevice, st));
    SCHK(launch_coldot(S->gg, S->part, S->g, S->g, ng, ng, k, st));
    SCHK(launch_cg_status(S->active, S->stat, S->gg, S->gg, 0.0, k, st));   // columns with g = 0 stop at once
    S->precondition(k, st);
    SCHK(hipMemcpyAsync(S->p, S->z, (size_t)ng * K * sizeof(double), hipMemcpyDeviceToDevice, st));
    SCHK(launch_coldot(S->rz, S->part, S->r, S->z, ng, ng, k, st));
    double hs[2] = {0.0, 0.0};
    int it = 0;
    for (;;) {
      // q = S p, alpha = rz / (p . q), x += alpha p, r -= alpha q
      S->apply(S->p, ng, S->q, ng, ng, k, st);
      SCHK(launch_coldot(S->pq, S->part, S->p, S->q, ng, ng, k, st));
      SCHK(launch_cg_alpha(S->alpha, S->rz, S->pq, S->active, k, st));
      SCHK(launch_cg_update(S->x, S->r, S->p, S->q, S->alpha, ng, ng, k, st));
      ++it;
      SCHK(launch_coldot(S->rr, S->part, S->r, S->r, ng, ng, k, st));
      SCHK(launch_cg_status(S->active, S->stat, S->rr, S->gg, tol, k, st));
      SCHK(hipMemcpyAsync(hs, S->stat, sizeof(hs), hipMemcpyDeviceToHost, st));
      SCHK(hipStreamSynchronize(st));
      if (hs[0] == 0.0) break;
      if (it >= max_iter || !std::isfinite(hs[1])) { status = TD_ENOCONV; break; }
      // z = B^{-1} r, beta = (r . z)_new / (r . z)_old, p = z + beta p
      S->precondition(k, st);
      SCHK(launch_coldot(S->rz2, S->part, S->r, S->z, ng, ng, k, st));
      SCHK(launch_cg_direction(S->p, S->z, S->rz2, S->rz, S->active, ng, ng, k, st));
      std::swap(S->rz, S->rz2);
    }
    // eq. (domains_equation): x_I = A_II^{-1} (f_I - A_IG x_G), then the full X
    SCHK(launch_schur_scatter(S->T, ni, F, ldf, S->x, ng, S->cA, S->cB, S->d_intcol, S->d_lif, S->d_rif, S->Nint,
                              (int)S->M, k, 1.0, st));
    TDCHK(tridiag_solve(S->interior, S->T, ni, S->Y, ni, K, nullptr, nullptr, st));
    SCHK(launch_schur_assemble(X, ldx, S->Y, ni, S->x, ng, S->d_intcol, S->d_icol, S->Nint, S->nif, (int)S->M, k, st));
    if (info) {
      info->iterations = it;
      info->active = (int32_t)hs[0];
      info->max_rel_residual = hs[1];
    }
  } catch (const SchurFail& f) {
    return td_set_error(f.s, f.msg.c_str());
  }
  if (status == TD_ENOCONV) return td_set_error(status, "conjugate gradients did not reach the requested residual");
  return TD_OK;
}

}  // namespace

extern "C" {

td_status tridiag_schur_create(int64_t N, int64_t M, const double* A, const double* B, const double* C, int64_t nif,
                               const int64_t* icol, int32_t band, void* stream, td_schur* out) {
  return schur_create(N, M, A, B, C, nif, icol, band, (hipStream_t)stream, out);
}

td_status tridiag_schur_apply(td_schur s, const double* V, int64_t ldv, double* Y, int64_t ldy, int64_t K,
                              void* stream) {
  if (!s) return td_set_error(TD_EINVAL, "null solver");
  if (K < 0 || ldv < s->ng || ldy < s->ng) return td_set_error(TD_EINVAL, "K < 0 or leading dimension below nif*M");
  if (K > INT_MAX / 4) return td_set_error(TD_EINVAL, "K too large");
  if (K == 0) return TD_OK;
  if (!V || !Y) return td_set_error(TD_EINVAL, "null V or Y");
  try {
    s->ensure_ws(K);
    s->last = (hipStream_t)stream;
    s->apply(V, ldv, Y, ldy, s->ng, (int)K, (hipStream_t)stream);
  } catch (const SchurFail& f) {
    return td_set_error(f.s, f.msg.c_str());
  }
  return TD_OK;
}

td_status tridiag_schur_solve(td_schur s, const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K, double tol,
                              int32_t max_iter, td_schur_info* info, void* stream) {
  if (!s) return td_set_error(TD_EINVAL, "null solver");
  return schur_solve(s, F, ldf, X, ldx, K, tol, max_iter, info, (hipStream_t)stream);
}

td_status tridiag_schur_destroy(td_schur s) {
  if (!s) return TD_OK;
  if (s->last) (void)hipStreamSynchronize(s->last);
  else (void)hipDeviceSynchronize();
  delete s;
  return TD_OK;
}

}  // extern "C"
