// Stationary density: (I - B) rho = rho0 (Sec. 2, Eq. GovIE), either by the
// partial sums of the Neumann series rho = sum_n B^n rho0 (Eq. NSum) or by
// restarted GMRES (classical Gram-Schmidt, repeated when a pass loses more than
// 30 % of the norm).  Precision 1 runs the GMRES iterations on an FP32 copy of B
// with FP32 Krylov vectors (FP64 accumulation in every dot product and product
// with B) and refines the solution with FP64 residuals of the FP64 operator:
//   r = rho0 - (I - B) rho (FP64),  (I - B32) e ~= r (FP32 GMRES),  rho += e.
// The host drives the iterations; every vector operation and every product with
// B runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dfm_internal.h"

namespace dfm {

hipError_t spmv(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st);
hipError_t spmv32(dfm_op op, const float *x, const float *v, float *y, float alpha, float beta, hipStream_t st);
hipError_t spmv_t(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st);
hipError_t ensure_fp32(dfm_op op, hipStream_t st);

namespace {

constexpr int RED_BLOCKS = 2048;
constexpr int RED_THREADS = 256;
constexpr int NWAVE = RED_THREADS / 64;
constexpr int MAXV = 201;

// partial[i][blk] = sum over this block's rows of V[i][row] * w[row], i < nvec.
// Each thread keeps a slice of w in registers, so V is read exactly once.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_multidot(const T *__restrict__ V, int64_t ldv, int nvec,
                                                        const T *__restrict__ extra, const T *__restrict__ w,
                                                        int64_t n, double *__restrict__ partial) {
  // vectors 0..nvec-1 are V[i], vector nvec (when extra != null) is `extra`
  if (extra) ++nvec;
  constexpr int RPT = 8;  // rows per thread kept in registers per sweep
  __shared__ double red[NWAVE][64];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t r0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = 0; i0 < nvec; i0 += 64) {
    const int ni = min(64, nvec - i0);
    double accs = 0.0;  // lane l keeps the wave's sum for vector i0 + l
    for (int64_t base = r0; base < n; base += stride * RPT) {
      double wr[RPT];
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        int64_t r = base + u * stride;
        wr[u] = r < n ? (double)w[r] : 0.0;
      }
      for (int i = 0; i < ni; ++i) {
        const T *vi = (extra && i0 + i == nvec - 1) ? extra : V + (int64_t)(i0 + i) * ldv;
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          int64_t r = base + u * stride;
          if (r < n) a = fma((double)vi[r], wr[u], a);
        }
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        if (lane == i) accs += a;
      }
    }
    red[wv][lane] = accs;
    __syncthreads();
    if (threadIdx.x < ni) {
      double s = 0.0;
      for (int k = 0; k < NWAVE; ++k) s += red[k][threadIdx.x];
      partial[(int64_t)(i0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[i] = sum_b partial[i][b]
__global__ void k_reduce_partials(const double *__restrict__ partial, int nb, double *__restrict__ out) {
  __shared__ double red[NWAVE];
  int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[(int64_t)i * nb + b];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < NWAVE; ++k) s += red[k];
    out[i] = s;
  }
}

// w[row] += sign * sum_i V[i][row] * h[i]; when partial != null also the block
// partial sums of ||w_new||^2 (grid-stride, RED_BLOCKS blocks)
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_combine(const T *__restrict__ V, int64_t ldv, int nvec,
                                                       const double *__restrict__ h, double sign, T *__restrict__ w,
                                                       int64_t n, double *__restrict__ partial) {
  __shared__ double hs[MAXV];
  __shared__ double red[NWAVE];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) hs[i] = h[i];
  __syncthreads();
  double nrm = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc = fma((double)V[(int64_t)i * ldv + r], hs[i], acc);
    T nw = (T)fma(sign, acc, (double)w[r]);
    w[r] = nw;
    nrm = fma((double)nw, (double)nw, nrm);
  }
  if (!partial) return;
  for (int off = 32; off > 0; off >>= 1) nrm += __shfl_down(nrm, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < NWAVE; ++k) t += red[k];
    partial[blockIdx.x] = t;
  }
}

template <typename T>
__global__ void k_scale_by(const T *__restrict__ x, double s, T *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = (T)((double)x[r] / s);
}

// y = a * x + b * y
template <typename TX, typename TY>
__global__ void k_axpby(double a, const TX *__restrict__ x, double b, TY *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = (TY)fma(a, (double)x[r], b * (double)y[r]);
}

template <typename TX, typename TY>
__global__ void k_copy(const TX *__restrict__ x, TY *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = (TY)x[r];
}

template <typename T>
__global__ void k_zero(T *__restrict__ y, int64_t n) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = (T)0;
}

struct Ctx {
  dfm_op op;
  hipStream_t st;
  bool transpose = false;  // solve (I - B)^T x = b (FP64 only)
  int64_t n;
  double *partial = nullptr;  // [MAXV][RED_BLOCKS]
  double *dsc = nullptr;      // device scalars
  unsigned grid() const { return (unsigned)((n + 255) / 256); }
  // out[0..nvec) = V^T w, and out[nvec] = extra . w when extra != null (device)
  template <typename T>
  hipError_t dots(const T *V, int64_t ldv, int nvec, const T *w, double *out, const T *extra = nullptr) {
    int nout = nvec + (extra ? 1 : 0);
    hipLaunchKernelGGL(k_multidot<T>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, extra, w, n, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nout), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, out);
    return hipGetLastError();
  }
  // w += sign V h; *nrm2_out = ||w||^2 (device) when nrm2_out != null
  template <typename T>
  hipError_t combine(const T *V, int64_t ldv, int nvec, const double *h, double sign, T *w, double *nrm2_out) {
    if (nrm2_out) {
      hipLaunchKernelGGL(k_combine<T>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, h, sign, w, n,
                         partial);
      hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, nrm2_out);
    } else {
      hipLaunchKernelGGL(k_combine<T>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, h, sign, w, n,
                         (double *)nullptr);
    }
    return hipGetLastError();
  }
  template <typename T>
  hipError_t norm2(const T *w, double &out) {
    hipError_t e = dots<T>(w, 0, 1, w, dsc);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&out, dsc, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    out = std::sqrt(out);
    return e;
  }
  // y = (I - B) x, with the FP32 copy of B for FP32 vectors
  hipError_t apply_ImB(const double *x, double *y) {
    return transpose ? spmv_t(op, x, x, y, 1.0, -1.0, st) : spmv(op, x, x, y, 1.0, -1.0, st);
  }
  hipError_t apply_B(const double *x, double *y) {
    return transpose ? spmv_t(op, x, nullptr, y, 0.0, 1.0, st) : spmv(op, x, nullptr, y, 0.0, 1.0, st);
  }
  hipError_t apply_ImB(const float *x, float *y) { return spmv32(op, x, x, y, 1.0f, -1.0f, st); }
};

// GMRES(m) on (I - B) x = b with x0 = 0, vectors of type T.  Stops when the
// relative residual is <= rtol: the true residual when check_true (FP64 solves),
// the Arnoldi estimate otherwise (inner solves of the refinement).
template <typename T>
hipError_t gmres(Ctx &c, const T *b, T *x, T *V, T *w, T *t, int m, double rtol, int max_iter, bool check_true,
                 int &its, int &restarts, double &rel, bool &done) {
  const unsigned G = c.grid();
  const int64_t n = c.n;
  const int nvmax = m + 1;
  double *h1 = c.dsc + 8, *h2 = c.dsc + 8 + nvmax;
  std::vector<double> hh(2 * nvmax + 8);
  double bnorm;
  hipError_t e = c.norm2<T>(b, bnorm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero<T>, dim3(G), dim3(256), 0, c.st, x, n);
  done = false;
  rel = 1.0;
  if (!(bnorm > 0.0)) {
    done = true;
    rel = 0.0;
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_copy<T, T>), dim3(G), dim3(256), 0, c.st, b, w, n);
  double beta = bnorm;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (!done && its < max_iter) {
    hipLaunchKernelGGL(k_scale_by<T>, dim3(G), dim3(256), 0, c.st, w, beta, V, n);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (; k < m && its < max_iter; ++k) {
      T *vk = V + (int64_t)k * n;
      if ((e = c.apply_ImB(vk, w)) != hipSuccess) return e;
      its++;
      // classical Gram-Schmidt: one pass for V^T w and ||w||^2, one for w -= V h
      // and ||w||^2; a second pass when the first lost > 30 % of ||w||
      if ((e = c.dots<T>(V, n, k + 1, w, h1, w)) != hipSuccess) return e;  // h1[k+1] = ||w||^2
      if ((e = c.combine<T>(V, n, k + 1, h1, -1.0, w, c.dsc + 1)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(hh.data(), c.dsc, sizeof(double) * (8 + nvmax), hipMemcpyDeviceToHost, c.st)))
        return e;
      if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
      double before = std::sqrt(hh[8 + k + 1]), hn = std::sqrt(hh[1]);
      for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hh[8 + i];
      if (hn < 0.7 * before) {
        if ((e = c.dots<T>(V, n, k + 1, w, h2)) != hipSuccess) return e;
        if ((e = c.combine<T>(V, n, k + 1, h2, -1.0, w, c.dsc + 1)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(hh.data() + 1, c.dsc + 1, sizeof(double), hipMemcpyDeviceToHost, c.st))) return e;
        if ((e = hipMemcpyAsync(hh.data() + 8 + nvmax, h2, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, c.st)))
          return e;
        if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
        hn = std::sqrt(hh[1]);
        for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] += hh[8 + nvmax + i];
      }
      H[(size_t)(k + 1) * m + k] = hn;
      if (hn > 0.0) hipLaunchKernelGGL(k_scale_by<T>, dim3(G), dim3(256), 0, c.st, w, hn, V + (int64_t)(k + 1) * n, n);
      for (int i = 0; i < k; ++i) {
        double a = H[(size_t)i * m + k], cc = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a + sn[i] * cc;
        H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * cc;
      }
      double a = H[(size_t)k * m + k], cc = H[(size_t)(k + 1) * m + k];
      double rr = std::hypot(a, cc);
      cs[k] = rr > 0.0 ? a / rr : 1.0;
      sn[k] = rr > 0.0 ? cc / rr : 0.0;
      H[(size_t)k * m + k] = rr;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      rel = std::fabs(g[k + 1]) / bnorm;
      if (!std::isfinite(rel)) return hipSuccess;
      if (rel <= (check_true ? 0.5 : 1.0) * rtol || hn == 0.0) {
        ++k;
        break;
      }
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
      y[i] = s / H[(size_t)i * m + i];
    }
    if ((e = hipMemcpyAsync(h1, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, c.st))) return e;
    if ((e = c.combine<T>(V, n, k, h1, 1.0, x, nullptr)) != hipSuccess) return e;
    if (!check_true && rel <= rtol) {
      if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
      done = true;
      continue;
    }
    // restart from the true residual w = b - (I - B) x
    if ((e = c.apply_ImB(x, t)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_copy<T, T>), dim3(G), dim3(256), 0, c.st, b, w, n);
    hipLaunchKernelGGL((k_axpby<T, T>), dim3(G), dim3(256), 0, c.st, -1.0, t, 1.0, w, n);
    if ((e = c.norm2<T>(w, beta)) != hipSuccess) return e;
    if (check_true) {
      rel = beta / bnorm;
      if (rel <= rtol) done = true;
    }
    if (!(beta > 0.0)) done = true;
    if (!done) restarts++;
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace dfm

using namespace dfm;

namespace dfm {
dfm_status solve_impl(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                      dfm_solve_info *info, bool transpose, void *stream_) {
  DFM_REQUIRE(op && rho0 && rho && opts, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1, DFM_E_INVALID, "nrhs must be >= 1");
  DFM_REQUIRE(opts->method == 0 || opts->method == 1, DFM_E_INVALID, "method must be 0 (Neumann) or 1 (GMRES)");
  DFM_REQUIRE(opts->precision == 0 || opts->precision == 1, DFM_E_INVALID, "precision must be 0 or 1");
  DFM_REQUIRE(!(opts->precision == 1 && opts->method == 0), DFM_E_UNSUPPORTED,
              "mixed precision is implemented for GMRES only");
  DFM_REQUIRE(opts->max_iter >= 1 && opts->rtol > 0.0, DFM_E_INVALID, "need max_iter >= 1 and rtol > 0");
  const int m = opts->method == 1 ? opts->restart : 1;
  DFM_REQUIRE(m >= 1 && m <= MAXV - 1, DFM_E_INVALID, "restart must be in 1..200");
  DFM_REQUIRE(!(transpose && opts->precision == 1), DFM_E_UNSUPPORTED,
              "transposed solves are implemented in FP64 only");
  hipStream_t st = (hipStream_t)stream_;
  const int64_t n = op->ndof;
  Ctx c;
  c.op = op;
  c.st = st;
  c.n = n;
  c.transpose = transpose;
  double *V = nullptr, *w = nullptr, *t = nullptr;
  float *V32 = nullptr, *w32 = nullptr, *t32 = nullptr, *b32 = nullptr, *e32 = nullptr;
  dfm_status status = DFM_OK;
  auto cleanup = [&]() {
    (void)hipFree(V);
    (void)hipFree(w);
    (void)hipFree(t);
    (void)hipFree(V32);
    (void)hipFree(w32);
    (void)hipFree(t32);
    (void)hipFree(b32);
    (void)hipFree(e32);
    (void)hipFree(c.dsc);
    (void)hipFree(c.partial);
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
  const bool mixed = opts->precision == 1;
  TRY(hipMalloc(&c.dsc, sizeof(double) * (8 + 2 * MAXV)));
  TRY(hipMalloc(&c.partial, sizeof(double) * (size_t)RED_BLOCKS * MAXV));
  if (opts->method == 0 || !mixed) TRY(hipMalloc(&V, sizeof(double) * (size_t)n * (opts->method == 1 ? nvmax : 2)));
  TRY(hipMalloc(&w, sizeof(double) * (size_t)n));
  TRY(hipMalloc(&t, sizeof(double) * (size_t)n));
  if (mixed) {
    TRY(ensure_fp32(op, st));
    TRY(hipMalloc(&V32, sizeof(float) * (size_t)n * nvmax));
    TRY(hipMalloc(&w32, sizeof(float) * (size_t)n));
    TRY(hipMalloc(&t32, sizeof(float) * (size_t)n));
    TRY(hipMalloc(&b32, sizeof(float) * (size_t)n));
    TRY(hipMalloc(&e32, sizeof(float) * (size_t)n));
  }
  const unsigned G = c.grid();

  for (int r = 0; r < nrhs; ++r) {
    const double *b = rho0 + (int64_t)r * n;
    double *x = rho + (int64_t)r * n;
    dfm_solve_info inf{0, 0, 0.0};
    double bnorm = 0.0;
    TRY(c.norm2<double>(b, bnorm));
    if (!(bnorm > 0.0)) {
      hipLaunchKernelGGL(k_zero<double>, dim3(G), dim3(256), 0, st, x, n);
      TRY(hipGetLastError());
      if (info) info[r] = inf;
      continue;
    }
    bool done = false;
    double rel = 1.0;
    if (opts->method == 0) {
      // x = b; t = b; repeat t <- B t, stop when ||t|| <= rtol ||b||, else x += t
      double *cur = t, *nxt = V;
      hipLaunchKernelGGL((k_copy<double, double>), dim3(G), dim3(256), 0, st, b, x, n);
      hipLaunchKernelGGL((k_copy<double, double>), dim3(G), dim3(256), 0, st, b, cur, n);
      TRY(hipGetLastError());
      while (inf.iters < opts->max_iter) {
        TRY(c.apply_B(cur, nxt));
        inf.iters++;
        double tn;
        TRY(c.norm2<double>(nxt, tn));
        rel = tn / bnorm;
        if (!std::isfinite(rel)) break;
        if (rel <= opts->rtol) {
          done = true;
          break;
        }
        hipLaunchKernelGGL((k_axpby<double, double>), dim3(G), dim3(256), 0, st, 1.0, nxt, 1.0, x, n);
        TRY(hipGetLastError());
        std::swap(cur, nxt);
      }
    } else if (!mixed) {
      TRY(gmres<double>(c, b, x, V, w, t, m, opts->rtol, opts->max_iter, true, inf.iters, inf.restarts, rel, done));
    } else {
      // iterative refinement: FP64 residuals of the FP64 operator, FP32 corrections
      hipLaunchKernelGGL(k_zero<double>, dim3(G), dim3(256), 0, st, x, n);
      hipLaunchKernelGGL((k_copy<double, double>), dim3(G), dim3(256), 0, st, b, w, n);
      TRY(hipGetLastError());
      double rn = bnorm;
      const double inner_tol = 1e-4;
      for (int outer = 0; outer < 50 && inf.iters < opts->max_iter; ++outer) {
        // b32 = r / ||r||
        hipLaunchKernelGGL((k_axpby<double, float>), dim3(G), dim3(256), 0, st, 1.0 / rn, w, 0.0, b32, n);
        int its = 0, rs = 0;
        double irel;
        bool idone;
        TRY(gmres<float>(c, b32, e32, V32, w32, t32, m, inner_tol, opts->max_iter - inf.iters, false, its, rs, irel,
                         idone));
        inf.iters += its;
        inf.restarts += rs;
        // x += ||r|| e ; r = b - (I - B) x in FP64
        hipLaunchKernelGGL((k_axpby<float, double>), dim3(G), dim3(256), 0, st, rn, e32, 1.0, x, n);
        TRY(spmv(op, x, x, t, 1.0, -1.0, st));
        inf.iters++;
        hipLaunchKernelGGL((k_copy<double, double>), dim3(G), dim3(256), 0, st, b, w, n);
        hipLaunchKernelGGL((k_axpby<double, double>), dim3(G), dim3(256), 0, st, -1.0, t, 1.0, w, n);
        TRY(c.norm2<double>(w, rn));
        rel = rn / bnorm;
        if (!std::isfinite(rel)) break;
        if (rel <= opts->rtol) {
          done = true;
          break;
        }
      }
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
}  // namespace dfm

extern "C" dfm_status dfm_solve(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                                dfm_solve_info *info, void *stream_) {
  return solve_impl(op, rho0, rho, nrhs, opts, info, false, stream_);
}
