// Receiver energy and its gradients by the adjoint of the stationary solve.
//
// The energy inside tet j is the interior density of Eq. IntDens (Sec. 4.1)
// integrated over the tet, E_j = sum_l int rho (1 - exp(-mu_j L))/mu_j ds dp
// (L the chord from the start point), a linear functional J = g . rho of the
// coefficients when summed over the tets whose centroid is in a box.  With
// (I - B)^T lambda = g:  dJ/dmu_j = lambda^T dB/dmu_j rho + rho . dg/dmu_j and
// dJ/dw_s = lambda . rho0_s for rho0 = sum_s w_s rho0_s.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dfm_internal.h"

namespace dfm {
hipError_t energy_functional(dfm_op op, const double *mu, const double *box, const double *rho, double *g,
                             double *blk_vec, double *blk_scal, unsigned *flags, hipStream_t st);
hipError_t dmu_contraction(dfm_op op, const double *mu, const double *rho, const double *lam, double *blk_scal,
                           const double *extra_scal, double *dmu, unsigned *flags, hipStream_t st);
dfm_status solve_impl(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                      dfm_solve_info *info, bool transpose, void *stream_);

namespace {
__global__ void k_zero_u32(unsigned *f) {
  if (threadIdx.x == 0) *f = 0u;
}

// flag bit 1 when a[i] and b[i] differ (bitwise, so a NaN never matches)
__global__ void k_differs(const double *a, const double *b, int64_t n, unsigned *flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (__double_as_longlong(a[i]) != __double_as_longlong(b[i])) atomicOr(flag, 1u);
}

// y[i] = sum_s w[s] x[s][i]
__global__ void k_weighted_sum(const double *x, int64_t n, int nvec, const double *w, double *y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < nvec; ++s) acc = fma(w[s], x[(int64_t)s * n + i], acc);
    y[i] = acc;
  }
}

// out[s] = sum_i src[s][i] * lam[i] (one block per source)
__global__ void k_src_dots(const double *src, int64_t n, const double *lam, double *out) {
  __shared__ double red[4];
  const double *a = src + blockIdx.x * n;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc = fma(a[i], lam[i], acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
}  // namespace
}  // namespace dfm

using namespace dfm;

#define TRY_ADJ(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      cleanup();                                                                             \
      return e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP;                            \
    }                                                                                        \
  } while (0)

// The damping the functional and the gradients use is the one B was assembled
// with (kept by the operator); a caller's copy, when given, must equal it.
static dfm_status check_mu(dfm_op op, const double *mu, hipStream_t st) {
  if (mu == nullptr || mu == op->mu) return DFM_OK;
  unsigned *flag = nullptr;
  DFM_HIP(hipMalloc(&flag, sizeof(unsigned)));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, flag);
  hipLaunchKernelGGL(k_differs, dim3(ew_grid(op->nt)), dim3(256), 0, st, mu, op->mu, op->nt, flag);
  unsigned hf = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&hf, flag, sizeof(unsigned), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(flag);
  DFM_HIP(e);
  DFM_REQUIRE(hf == 0u, DFM_E_INVALID, "mu differs from the damping the operator was assembled with");
  return DFM_OK;
}

extern "C" dfm_status dfm_receiver_functional(dfm_op op, const double *mu, const double *box, double *g,
                                              void *stream_) {
  DFM_REQUIRE(op && box && g, DFM_E_INVALID, "null argument");
  hipStream_t st = (hipStream_t)stream_;
  {
    dfm_status cs = check_mu(op, mu, st);
    if (cs != DFM_OK) return cs;
  }
  mu = op->mu;
  double *blk_vec = nullptr;
  unsigned *flags = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(blk_vec);
    (void)hipFree(flags);
  };
  TRY_ADJ(hipMalloc(&blk_vec, sizeof(double) * 12 * op->nt * (size_t)op->K));
  TRY_ADJ(hipMalloc(&flags, sizeof(unsigned)));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, flags);
  TRY_ADJ(energy_functional(op, mu, box, nullptr, g, blk_vec, nullptr, flags, st));
  unsigned hf = 0;
  TRY_ADJ(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  TRY_ADJ(hipStreamSynchronize(st));
  cleanup();
  DFM_REQUIRE(hf == 0u, DFM_E_NUMERIC, "a block needs more quadrature cells than the table holds");
  return DFM_OK;
}

extern "C" dfm_status dfm_adjoint(dfm_op op, const double *mu, const double *box, const double *rho,
                                  const double *src, int nsrc, const dfm_solve_opts *opts, double *lambda,
                                  double *d_mu, double *d_w, dfm_solve_info *info, void *stream_) {
  DFM_REQUIRE(op && box && rho && opts && lambda && d_mu, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nsrc >= 0 && (nsrc == 0 || (src && d_w)), DFM_E_INVALID, "src and d_w are needed when nsrc > 0");
  DFM_REQUIRE(opts->precision == 0 || (opts->precision == 1 && opts->method == 1), DFM_E_UNSUPPORTED,
              "the adjoint solve is FP64, or mixed precision with GMRES");
  hipStream_t st = (hipStream_t)stream_;
  {
    dfm_status cs = check_mu(op, mu, st);
    if (cs != DFM_OK) return cs;
  }
  mu = op->mu;
  const int64_t nblk = 12 * op->nt;
  double *blk_vec = nullptr, *blk_e = nullptr, *blk_b = nullptr, *g = nullptr;
  unsigned *flags = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(blk_vec);
    (void)hipFree(blk_e);
    (void)hipFree(blk_b);
    (void)hipFree(g);
    (void)hipFree(flags);
  };
  TRY_ADJ(hipMalloc(&blk_vec, sizeof(double) * nblk * (size_t)op->K));
  TRY_ADJ(hipMalloc(&blk_e, sizeof(double) * nblk));
  TRY_ADJ(hipMalloc(&blk_b, sizeof(double) * nblk));
  TRY_ADJ(hipMalloc(&g, sizeof(double) * op->ndof));
  TRY_ADJ(hipMalloc(&flags, sizeof(unsigned)));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, flags);
  // g and rho . dg/dmu per block
  TRY_ADJ(energy_functional(op, mu, box, rho, g, blk_vec, blk_e, flags, st));
  // (I - B)^T lambda = g
  dfm_status s = solve_impl(op, g, lambda, 1, opts, info, true, stream_);
  if (s != DFM_OK && s != DFM_E_NOCONV) {
    cleanup();
    return s;
  }
  // dJ/dmu and dJ/dw
  TRY_ADJ(dmu_contraction(op, mu, rho, lambda, blk_b, blk_e, d_mu, flags, st));
  if (nsrc > 0) {
    hipLaunchKernelGGL(k_src_dots, dim3((unsigned)nsrc), dim3(256), 0, st, src, op->ndof, lambda, d_w);
    TRY_ADJ(hipGetLastError());
  }
  unsigned hf = 0;
  TRY_ADJ(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  TRY_ADJ(hipStreamSynchronize(st));
  cleanup();
  DFM_REQUIRE(hf == 0u, DFM_E_NUMERIC, "a block needs more quadrature cells than the table holds");
  if (s == DFM_E_NOCONV) set_error("adjoint solve stopped at max_iter above the tolerance");
  return s;
}

extern "C" dfm_status dfm_receiver_energy(dfm_op op, const double *mu, const double *box, const double *rho,
                                          int nrhs, double *J, void *stream_) {
  DFM_REQUIRE(op && box && rho && J, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, DFM_E_INVALID, "nrhs must be in 1..65535");
  hipStream_t st = (hipStream_t)stream_;
  {
    dfm_status cs = check_mu(op, mu, st);
    if (cs != DFM_OK) return cs;
  }
  double *blk_vec = nullptr, *g = nullptr;
  unsigned *flags = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(blk_vec);
    (void)hipFree(g);
    (void)hipFree(flags);
  };
  TRY_ADJ(hipMalloc(&blk_vec, sizeof(double) * 12 * op->nt * (size_t)op->K));
  TRY_ADJ(hipMalloc(&g, sizeof(double) * op->ndof));
  TRY_ADJ(hipMalloc(&flags, sizeof(unsigned)));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, flags);
  TRY_ADJ(energy_functional(op, op->mu, box, nullptr, g, blk_vec, nullptr, flags, st));
  // J[r] = rho[r] . g
  hipLaunchKernelGGL(k_src_dots, dim3((unsigned)nrhs), dim3(256), 0, st, rho, op->ndof, g, J);
  TRY_ADJ(hipGetLastError());
  unsigned hf = 0;
  TRY_ADJ(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  TRY_ADJ(hipStreamSynchronize(st));
  cleanup();
  DFM_REQUIRE(hf == 0u, DFM_E_NUMERIC, "a block needs more quadrature cells than the table holds");
  return DFM_OK;
}

extern "C" dfm_status dfm_weighted_sum(const double *x, int64_t n, int nvec, const double *w, double *y,
                                       void *stream_) {
  DFM_REQUIRE(x && w && y, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(n >= 1 && nvec >= 1, DFM_E_INVALID, "need n >= 1 and nvec >= 1");
  hipStream_t st = (hipStream_t)stream_;
  hipLaunchKernelGGL(k_weighted_sum, dim3(ew_grid(n)), dim3(256), 0, st, x, n, nvec, w, y);
  DFM_HIP(hipGetLastError());
  return DFM_OK;
}
