// Application of the block-sparse B (Sec. 2: B couples only the faces of one tet
// to the slots its rays enter next, so the matrix is 12 dense K x K blocks per tet).
//
// Storage: block (j, l_out, s) is column-major with K columns of padded length Kp
// (a multiple of 4, padding rows zero) at ((4j + l_out)*3 + s)*K*Kp;
// s enumerates l_in != l_out in increasing order.  Block row (j, l_out) writes
// exactly one destination slot dest[4j + l_out] (a bijection of slots), so the
// forward product needs no atomics: one thread per destination unknown streams the
// 3K columns of its block row (consecutive threads read consecutive doubles).
#include <hip/hip_runtime.h>

#include "dfm_internal.h"

namespace dfm {

namespace {

__device__ inline int in_face(int l_out, int s) { return s < l_out ? s : s + 1; }

// y[dest(br)][row] = alpha * v[dest(br)][row] + beta * sum_{s,col} B[br,s][col][row] x[4j+l_in(s)][col]
// (v may be null when alpha == 0).  Columns have the padded length Kp (multiple
// of 4): each thread owns VW consecutive rows of one block row and streams its
// 3K columns with one 16-byte non-temporal load per column, so a wave moves 1 KB
// per load instruction.  The x panels of the block rows a workgroup touches are
// staged in LDS.  Sums are accumulated in FP64.
constexpr int SPMV_THREADS = 256;

template <typename TB>
struct Vec;
template <>
struct Vec<double> {
  static constexpr int W = 2;
  typedef double T __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<float> {
  static constexpr int W = 4;
  typedef float T __attribute__((ext_vector_type(4)));
};

template <typename TB, typename TX>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv(const TB *__restrict__ B, const int32_t *__restrict__ dest,
                                                      int64_t nthreads, int K, int Kp, const TX *__restrict__ x,
                                                      const TX *__restrict__ v, TX *__restrict__ y, double alpha,
                                                      double beta) {
  constexpr int VW = Vec<TB>::W;
  typedef typename Vec<TB>::T VT;
  extern __shared__ double xs_all[];
  const int GPB = Kp / VW;  // row groups per block row
  const int64_t g0 = blockIdx.x * (int64_t)SPMV_THREADS;
  const int64_t br0 = g0 / GPB;
  int64_t glast = g0 + SPMV_THREADS - 1;
  if (glast >= nthreads) glast = nthreads - 1;
  const int nrows_b = (int)(glast / GPB - br0 + 1);
  const int panel = 3 * K;
  for (int i = threadIdx.x; i < nrows_b * panel; i += SPMV_THREADS) {
    int b = i / panel, e = i - b * panel;
    int s = e / K, col = e - s * K;
    int64_t br = br0 + b;
    int64_t j = br >> 2;
    int l_out = (int)(br & 3);
    xs_all[i] = (double)x[(4 * j + in_face(l_out, s)) * (int64_t)K + col];
  }
  __syncthreads();
  const int64_t g = g0 + threadIdx.x;
  if (g >= nthreads) return;
  const int64_t br = g / GPB;
  const int row0 = (int)(g - br * GPB) * VW;
  const double *xp = xs_all + (br - br0) * panel;
  const VT *Bv = reinterpret_cast<const VT *>(B + br * 3 * (int64_t)K * Kp + row0);
  const int cstride = Kp / VW;
  double acc[VW];
#pragma unroll
  for (int u = 0; u < VW; ++u) acc[u] = 0.0;
  const int n = 3 * K;
#pragma unroll 4
  for (int c = 0; c < n; ++c) {
    VT bv = __builtin_nontemporal_load(Bv + (int64_t)c * cstride);
    const double xc = xp[c];
#pragma unroll
    for (int u = 0; u < VW; ++u) acc[u] = fma((double)bv[u], xc, acc[u]);
  }
  const int64_t ob = (int64_t)dest[br] * K;
#pragma unroll
  for (int u = 0; u < VW; ++u) {
    const int row = row0 + u;
    if (row < K) {
      double r = beta * acc[u];
      if (v) r = fma(alpha, (double)v[ob + row], r);
      y[ob + row] = (TX)r;
    }
  }
}

template <typename TB>
inline size_t spmv_lds(int K, int Kp) {
  int gpb = Kp / Vec<TB>::W;
  int64_t rows = (SPMV_THREADS + gpb - 1) / gpb + 1;
  return sizeof(double) * (size_t)(rows * 3 * K);
}

__global__ void k_to_fp32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// y[4j + l_in][col] = alpha v[...] + beta sum_{l_out != l_in} sum_row B[j,l_out,s(l_in)][col][row] x[dest(j,l_out)][row]
__global__ void k_spmv_t(const double *__restrict__ B, const int32_t *__restrict__ dest, int64_t nrows, int K, int Kp,
                         const double *__restrict__ x, const double *__restrict__ v, double *__restrict__ y,
                         double alpha, double beta) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  int64_t slot = g / K;
  int col = (int)(g - slot * K);
  int64_t j = slot >> 2;
  int l_in = (int)(slot & 3);
  const int64_t KKp = (int64_t)K * Kp;
  double acc = 0.0;
  for (int l_out = 0; l_out < 4; ++l_out) {
    if (l_out == l_in) continue;
    int s = l_in < l_out ? l_in : l_in - 1;
    int64_t br = 4 * j + l_out;
    const double *Bb = B + (br * 3 + s) * KKp + (int64_t)col * Kp;
    const double *xs = x + (int64_t)dest[br] * K;
    for (int row = 0; row < K; ++row) acc = fma(Bb[row], xs[row], acc);
  }
  double r = beta * acc;
  if (v) r = fma(alpha, v[g], r);
  y[g] = r;
}

}  // namespace

hipError_t spmv(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st) {
  int64_t nthreads = 4 * op->nt * (int64_t)(op->Kp / Vec<double>::W);
  unsigned grid = (unsigned)((nthreads + SPMV_THREADS - 1) / SPMV_THREADS);
  hipLaunchKernelGGL((k_spmv<double, double>), dim3(grid), dim3(SPMV_THREADS), spmv_lds<double>(op->K, op->Kp), st,
                     op->B, op->dest, nthreads, op->K, op->Kp, x, v, y, alpha, beta);
  return hipGetLastError();
}

hipError_t spmv32(dfm_op op, const float *x, const float *v, float *y, float alpha, float beta, hipStream_t st) {
  int64_t nthreads = 4 * op->nt * (int64_t)(op->Kp / Vec<float>::W);
  unsigned grid = (unsigned)((nthreads + SPMV_THREADS - 1) / SPMV_THREADS);
  hipLaunchKernelGGL((k_spmv<float, float>), dim3(grid), dim3(SPMV_THREADS), spmv_lds<float>(op->K, op->Kp), st,
                     op->B32, op->dest, nthreads, op->K, op->Kp, x, v, y, (double)alpha, (double)beta);
  return hipGetLastError();
}

// FP32 copy of B for the mixed-precision solver (made once, kept with the operator)
hipError_t ensure_fp32(dfm_op op, hipStream_t st) {
  if (op->B32) return hipSuccess;
  int64_t nel = 12 * op->nt * (int64_t)op->K * op->Kp;
  hipError_t e = hipMalloc(&op->B32, sizeof(float) * nel);
  if (e != hipSuccess) {
    op->B32 = nullptr;
    return e;
  }
  hipLaunchKernelGGL(k_to_fp32, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, st, op->B, op->B32, nel);
  return hipGetLastError();
}

hipError_t spmv_t(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st) {
  int64_t nrows = op->ndof;
  unsigned grid = (unsigned)((nrows + 255) / 256);
  hipLaunchKernelGGL(k_spmv_t, dim3(grid), dim3(256), 0, st, op->B, op->dest, nrows, op->K, op->Kp, x, v, y, alpha,
                     beta);
  return hipGetLastError();
}

}  // namespace dfm

using namespace dfm;

extern "C" dfm_status dfm_apply(dfm_op op, const double *x, double *y, int nrhs, int transpose, void *stream_) {
  DFM_REQUIRE(op && x && y, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1, DFM_E_INVALID, "nrhs must be >= 1");
  DFM_REQUIRE(x != y, DFM_E_INVALID, "x and y must not alias");
  hipStream_t st = (hipStream_t)stream_;
  for (int r = 0; r < nrhs; ++r) {
    const double *xr = x + (int64_t)r * op->ndof;
    double *yr = y + (int64_t)r * op->ndof;
    DFM_HIP(transpose ? spmv_t(op, xr, nullptr, yr, 0.0, 1.0, st) : spmv(op, xr, nullptr, yr, 0.0, 1.0, st));
  }
  return DFM_OK;
}
