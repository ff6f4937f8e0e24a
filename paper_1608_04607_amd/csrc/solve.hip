// Stationary density: (I - B) rho = rho0 (Sec. 2, Eq. GovIE), either by the
// partial sums of the Neumann series rho = sum_n B^n rho0 (Eq. NSum) or by
// restarted GMRES with classical Gram-Schmidt applied twice.  The host drives
// the iteration; every vector operation and every product with B runs on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "dfm_internal.h"

namespace dfm {

hipError_t spmv(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st);

namespace {

constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;

// partial[i][blk] = sum over this block's rows of V[i][row] * w[row], i < nvec
__global__ void k_dot_partials(const double *__restrict__ V, int64_t ldv, int nvec, const double *__restrict__ w,
                               int64_t n, double *__restrict__ partial) {
  __shared__ double red[RED_THREADS / 64];
  for (int i = 0; i < nvec; ++i) {
    const double *vi = V + (int64_t)i * ldv;
    double acc = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
      acc = fma(vi[r], w[r], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < RED_THREADS / 64; ++k) s += red[k];
      partial[(int64_t)i * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[i] = sum_b partial[i][b]
__global__ void k_reduce_partials(const double *__restrict__ partial, int nb, double *__restrict__ out) {
  __shared__ double red[RED_THREADS / 64];
  int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[(int64_t)i * nb + b];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < RED_THREADS / 64; ++k) s += red[k];
    out[i] = s;
  }
}

// w[row] += sign * sum_i V[i][row] * h[i]
__global__ void k_combine(const double *__restrict__ V, int64_t ldv, int nvec, const double *__restrict__ h,
                          double sign, double *__restrict__ w, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int i = 0; i < nvec; ++i) acc = fma(V[(int64_t)i * ldv + r], h[i], acc);
  w[r] = fma(sign, acc, w[r]);
}

// y = x / s
__global__ void k_scale_by(const double *__restrict__ x, double s, double *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = x[r] / s;
}

// y = a * x + b * y
__global__ void k_axpby(double a, const double *__restrict__ x, double b, double *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = fma(a, x[r], b * y[r]);
}

__global__ void k_copy(const double *__restrict__ x, double *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = x[r];
}

__global__ void k_zero(double *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = 0.0;
}

struct Work {
  hipStream_t st;
  int64_t n;
  double *partial = nullptr;  // [nvec][RED_BLOCKS]
  unsigned grid() const { return (unsigned)((n + 255) / 256); }
  // out[0..nvec) = V[0..nvec)^T w   (device)
  hipError_t dots(const double *V, int64_t ldv, int nvec, const double *w, double *out) {
    hipLaunchKernelGGL(k_dot_partials, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, w, n, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nvec), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, out);
    return hipGetLastError();
  }
};

}  // namespace
}  // namespace dfm

using namespace dfm;

extern "C" dfm_status dfm_solve(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                                dfm_solve_info *info, void *stream_) {
  DFM_REQUIRE(op && rho0 && rho && opts, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1, DFM_E_INVALID, "nrhs must be >= 1");
  DFM_REQUIRE(opts->method == 0 || opts->method == 1, DFM_E_INVALID, "method must be 0 (Neumann) or 1 (GMRES)");
  DFM_REQUIRE(opts->precision == 0, DFM_E_UNSUPPORTED, "only FP64 solves (precision 0) are implemented");
  DFM_REQUIRE(opts->max_iter >= 1 && opts->rtol > 0.0, DFM_E_INVALID, "need max_iter >= 1 and rtol > 0");
  const int m = opts->method == 1 ? opts->restart : 1;
  DFM_REQUIRE(m >= 1 && m <= 200, DFM_E_INVALID, "restart must be in 1..200");
  hipStream_t st = (hipStream_t)stream_;
  const int64_t n = op->ndof;
  Work wk;
  wk.st = st;
  wk.n = n;
  double *V = nullptr, *w = nullptr, *t = nullptr, *dsc = nullptr;
  std::vector<double> hh;
  dfm_status status = DFM_OK;
  auto cleanup = [&]() {
    (void)hipFree(V);
    (void)hipFree(w);
    (void)hipFree(t);
    (void)hipFree(dsc);
    (void)hipFree(wk.partial);
  };
#define TRY(expr)                                                                            \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      cleanup();                                                                             \
      return e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP;                            \
    }                                                                                        \
  } while (0)
  const int nvmax = m + 1;
  TRY(hipMalloc(&V, sizeof(double) * (size_t)n * (opts->method == 1 ? nvmax : 2)));
  TRY(hipMalloc(&w, sizeof(double) * (size_t)n));
  TRY(hipMalloc(&t, sizeof(double) * (size_t)n));
  // device scalars: h1[nvmax], h2[nvmax], norm[2]
  TRY(hipMalloc(&dsc, sizeof(double) * (2 * nvmax + 4)));
  TRY(hipMalloc(&wk.partial, sizeof(double) * (size_t)RED_BLOCKS * nvmax));
  double *h1 = dsc, *h2 = dsc + nvmax, *nrm = dsc + 2 * nvmax;
  const unsigned G = wk.grid();
  hh.resize(2 * nvmax + 4);

  for (int r = 0; r < nrhs; ++r) {
    const double *b = rho0 + (int64_t)r * n;
    double *x = rho + (int64_t)r * n;
    dfm_solve_info inf{0, 0, 0.0};
    double bnorm = 0.0;
    TRY(wk.dots(b, 0, 1, b, nrm));
    TRY(hipMemcpyAsync(hh.data(), nrm, sizeof(double), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    bnorm = std::sqrt(hh[0]);
    if (!(bnorm > 0.0)) {
      hipLaunchKernelGGL(k_zero, dim3(G), dim3(256), 0, st, x, n);
      TRY(hipGetLastError());
      if (info) info[r] = inf;
      continue;
    }
    if (opts->method == 0) {
      // x = b; t = b; repeat t <- B t, stop when ||t|| <= rtol ||b||, else x += t
      double *cur = t, *nxt = V;
      hipLaunchKernelGGL(k_copy, dim3(G), dim3(256), 0, st, b, x, n);
      hipLaunchKernelGGL(k_copy, dim3(G), dim3(256), 0, st, b, cur, n);
      TRY(hipGetLastError());
      bool done = false;
      double rel = 1.0;
      while (inf.iters < opts->max_iter) {
        TRY(spmv(op, cur, nullptr, nxt, 0.0, 1.0, st));
        inf.iters++;
        TRY(wk.dots(nxt, 0, 1, nxt, nrm));
        TRY(hipMemcpyAsync(hh.data(), nrm, sizeof(double), hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        rel = std::sqrt(hh[0]) / bnorm;
        if (!std::isfinite(rel)) break;
        if (rel <= opts->rtol) {
          done = true;
          break;
        }
        hipLaunchKernelGGL(k_axpby, dim3(G), dim3(256), 0, st, 1.0, nxt, 1.0, x, n);
        TRY(hipGetLastError());
        std::swap(cur, nxt);
      }
      inf.relres = rel;
      if (!std::isfinite(rel)) status = DFM_E_NUMERIC;
      else if (!done) status = DFM_E_NOCONV;
      if (info) info[r] = inf;
      continue;
    }
    // ---- GMRES(m) ----
    hipLaunchKernelGGL(k_zero, dim3(G), dim3(256), 0, st, x, n);
    TRY(hipGetLastError());
    double beta = bnorm;  // residual of x = 0
    hipLaunchKernelGGL(k_copy, dim3(G), dim3(256), 0, st, b, w, n);
    TRY(hipGetLastError());
    bool done = false;
    double rel = 1.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    while (!done && inf.iters < opts->max_iter) {
      // V[0] = w / beta
      hipLaunchKernelGGL(k_scale_by, dim3(G), dim3(256), 0, st, w, beta, V, n);
      TRY(hipGetLastError());
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int k = 0;
      for (; k < m && inf.iters < opts->max_iter; ++k) {
        double *vk = V + (int64_t)k * n;
        // w = (I - B) v_k
        TRY(spmv(op, vk, vk, w, 1.0, -1.0, st));
        inf.iters++;
        // classical Gram-Schmidt, twice
        TRY(wk.dots(V, n, k + 1, w, h1));
        hipLaunchKernelGGL(k_combine, dim3(G), dim3(256), 0, st, V, n, k + 1, h1, -1.0, w, n);
        TRY(wk.dots(V, n, k + 1, w, h2));
        hipLaunchKernelGGL(k_combine, dim3(G), dim3(256), 0, st, V, n, k + 1, h2, -1.0, w, n);
        TRY(wk.dots(w, 0, 1, w, nrm + 1));
        TRY(hipMemcpyAsync(hh.data(), dsc, sizeof(double) * (2 * nvmax + 2), hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        double hn = std::sqrt(hh[2 * nvmax + 1]);
        for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hh[i] + hh[nvmax + i];
        H[(size_t)(k + 1) * m + k] = hn;
        // new basis vector
        if (hn > 0.0) {
          hipLaunchKernelGGL(k_scale_by, dim3(G), dim3(256), 0, st, w, hn, V + (int64_t)(k + 1) * n, n);
          TRY(hipGetLastError());
        }
        // Givens rotations
        for (int i = 0; i < k; ++i) {
          double a = H[(size_t)i * m + k], c = H[(size_t)(i + 1) * m + k];
          H[(size_t)i * m + k] = cs[i] * a + sn[i] * c;
          H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * c;
        }
        double a = H[(size_t)k * m + k], c = H[(size_t)(k + 1) * m + k];
        double rr = std::hypot(a, c);
        cs[k] = rr > 0.0 ? a / rr : 1.0;
        sn[k] = rr > 0.0 ? c / rr : 0.0;
        H[(size_t)k * m + k] = rr;
        H[(size_t)(k + 1) * m + k] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        rel = std::fabs(g[k + 1]) / bnorm;
        if (!std::isfinite(rel)) break;
        if (rel <= 0.5 * opts->rtol || hn == 0.0) {
          ++k;
          break;
        }
      }
      if (!std::isfinite(rel)) break;
      // y = H^-1 g (upper triangular k x k); x += V y
      for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
        y[i] = s / H[(size_t)i * m + i];
      }
      TRY(hipMemcpyAsync(h1, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_combine, dim3(G), dim3(256), 0, st, V, n, k, h1, 1.0, x, n);
      // true residual w = b - (I - B) x
      TRY(spmv(op, x, x, t, 1.0, -1.0, st));
      hipLaunchKernelGGL(k_copy, dim3(G), dim3(256), 0, st, b, w, n);
      hipLaunchKernelGGL(k_axpby, dim3(G), dim3(256), 0, st, -1.0, t, 1.0, w, n);
      TRY(wk.dots(w, 0, 1, w, nrm));
      TRY(hipMemcpyAsync(hh.data(), nrm, sizeof(double), hipMemcpyDeviceToHost, st));
      TRY(hipStreamSynchronize(st));
      beta = std::sqrt(hh[0]);
      rel = beta / bnorm;
      if (rel <= opts->rtol) done = true;
      else inf.restarts++;
      if (!(beta > 0.0)) done = true;
    }
    inf.relres = rel;
    if (!std::isfinite(rel)) status = DFM_E_NUMERIC;
    else if (!done && status == DFM_OK) status = DFM_E_NOCONV;
    if (info) info[r] = inf;
  }
#undef TRY
  cleanup();
  if (status == DFM_E_NOCONV) set_error("solver stopped at max_iter above the tolerance");
  if (status == DFM_E_NUMERIC) set_error("non-finite residual in the solver");
  return status;
}
