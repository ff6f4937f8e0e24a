// Stationary density: (I - B) rho = rho0 (Sec. 2, Eq. GovIE), either by the
// partial sums of the Neumann series rho = sum_n B^n rho0 (Eq. NSum) or by
// restarted GMRES (classical Gram-Schmidt, repeated when a pass loses more than
// 30 % of the norm).  Precision 1 runs the GMRES iterations on an FP32 copy of B
// with FP32 Krylov vectors (FP64 accumulation in every dot product and product
// with B) and refines the solution with FP64 residuals of the FP64 operator:
//   r = rho0 - (I - B) rho (FP64),  (I - B32) e ~= r (FP32 GMRES),  rho += e.
// Method 0 with precision 1 solves many right-hand sides together: the
// corrections are FP32 Neumann partial sums e = sum_k B32^k (r/|r|), one batched
// product for all right-hand sides per term on the FP32 matrix cores, refined
// with FP64 residuals of the FP64 operator.
// GMRES builds its Arnoldi basis with B itself (same Krylov space as I - B, and
// w = B v keeps most of its norm outside the basis, so the second Gram-Schmidt
// pass is rarely needed); the Hessenberg update, the Givens rotations and the
// residual estimate run on the device, and the host reads the estimate every few
// steps.  Every vector operation and every product with B runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "dfm_internal.h"

namespace dfm {

hipError_t spmv(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st);
hipError_t spmv32(dfm_op op, const float *x, const float *v, float *y, float alpha, float beta, hipStream_t st);
hipError_t spmv_t(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st);
hipError_t spmv32_t(dfm_op op, const float *x, const float *v, float *y, float alpha, float beta, hipStream_t st);
hipError_t ensure_fp32(dfm_op op, hipStream_t st);
hipError_t product32(dfm_op op, const float *x, float *y, float *e, int R, const int32_t *gid, const uint8_t *gact,
                     hipStream_t st);
dfm_status solve_twolevel_impl(dfm_op op, const double *rho0, double *rho, int R, const dfm_solve_opts *opts,
                               const std::vector<int64_t> &toff, dfm_solve_info *info, hipStream_t st);

namespace {

#ifndef DFM_DOT_BLOCKS
#define DFM_DOT_BLOCKS 1024
#endif
#ifndef DFM_DOT_VC
#define DFM_DOT_VC 16
#endif
constexpr int RED_BLOCKS = 2048;
constexpr int DOT_BLOCKS = DFM_DOT_BLOCKS;  // partial sums per vector of the Krylov dot products
constexpr int RED_THREADS = 256;
constexpr int NWAVE = RED_THREADS / 64;
constexpr int MAXV = 201;
constexpr int VC = DFM_DOT_VC;  // vectors per register sweep of k_multidot
static_assert(DOT_BLOCKS <= RED_BLOCKS, "the partial-sum buffer holds RED_BLOCKS sums per vector");

// VW consecutive elements of one vector: a 16-byte load when VW > 1 (the caller
// checks alignment and n % VW == 0)
template <typename T, int VW>
__device__ inline void load_rows(const T *__restrict__ p, int64_t r, double (&o)[VW]) {
  if constexpr (VW == 1) {
    o[0] = (double)p[r];
  } else {
    typedef T vt __attribute__((ext_vector_type(VW)));
    const vt v = *reinterpret_cast<const vt *>(p + r * VW);
#pragma unroll
    for (int u = 0; u < VW; ++u) o[u] = (double)v[u];
  }
}

template <typename T, int VW>
__device__ inline void store_rows(T *__restrict__ p, int64_t r, const double (&o)[VW]) {
  if constexpr (VW == 1) {
    p[r] = (T)o[0];
  } else {
    typedef T vt __attribute__((ext_vector_type(VW)));
    vt v;
#pragma unroll
    for (int u = 0; u < VW; ++u) v[u] = (T)o[u];
    *reinterpret_cast<vt *>(p + r * VW) = v;
  }
}

// partial[i][blk] = sum over this block's rows of V[i][row] * w[row] for i < nvec,
// and partial[nvec][blk] the same for `extra` when it is given.  Each thread keeps
// VC accumulators in registers over all of its rows (VW rows per 16-byte load), and
// the wave and block reductions run once per VC vectors.  Nothing is written when
// `gate` is given and zero (a second Gram-Schmidt pass that is not needed).
template <typename T, int VW>
__global__ __launch_bounds__(RED_THREADS) void k_multidot(const T *__restrict__ V, int64_t ldv, int nvec,
                                                        const T *__restrict__ extra, const T *__restrict__ w,
                                                        int64_t n, double *__restrict__ partial,
                                                        const int *__restrict__ gate) {
  if (gate && !*gate) return;
  __shared__ double red[NWAVE][VC + 1];
  const int64_t nr = n / VW;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t r0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nchunks = nvec > 0 ? (nvec + VC - 1) / VC : 1;
  for (int c = 0; c < nchunks; ++c) {
    const int i0 = c * VC;
    const int ni = min(VC, nvec - i0);
    const bool ex = extra != nullptr && c == 0;
    double acc[VC + 1];
#pragma unroll
    for (int i = 0; i <= VC; ++i) acc[i] = 0.0;
    for (int64_t r = r0; r < nr; r += stride) {
      double wr[VW], vr[VW];
      load_rows<T, VW>(w, r, wr);
#pragma unroll
      for (int i = 0; i < VC; ++i)
        if (i < ni) {
          load_rows<T, VW>(V + (int64_t)(i0 + i) * ldv, r, vr);
#pragma unroll
          for (int u = 0; u < VW; ++u) acc[i] = fma(vr[u], wr[u], acc[i]);
        }
      if (ex) {
        load_rows<T, VW>(extra, r, vr);
#pragma unroll
        for (int u = 0; u < VW; ++u) acc[VC] = fma(vr[u], wr[u], acc[VC]);
      }
    }
#pragma unroll
    for (int i = 0; i <= VC; ++i) {
      if (i < ni || (i == VC && ex)) {
        double a = acc[i];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        if (lane == 0) red[wv][i] = a;
      }
    }
    __syncthreads();
    if (threadIdx.x <= VC) {
      const int i = threadIdx.x;
      if (i < ni || (i == VC && ex)) {
        double s = 0.0;
        for (int k = 0; k < NWAVE; ++k) s += red[k][i];
        partial[(int64_t)(i < VC ? i0 + i : nvec) * gridDim.x + blockIdx.x] = s;
      }
    }
    __syncthreads();
  }
}

// out[i] = sum_b partial[i][b] (nothing when `gate` is given and zero)
__global__ void k_reduce_partials(const double *__restrict__ partial, int nb, double *__restrict__ out,
                                  const int *__restrict__ gate) {
  if (gate && !*gate) return;
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
// partial sums of ||w_new||^2 (grid-stride, RED_BLOCKS blocks).  Nothing is done
// when `gate` is given and zero.
template <typename T, int VW>
__global__ __launch_bounds__(RED_THREADS) void k_combine(const T *__restrict__ V, int64_t ldv, int nvec,
                                                       const double *__restrict__ h, double sign, T *__restrict__ w,
                                                       int64_t n, double *__restrict__ partial,
                                                       const int *__restrict__ gate) {
  if (gate && !*gate) return;
  __shared__ double hs[MAXV];
  __shared__ double red[NWAVE];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) hs[i] = h[i];
  __syncthreads();
  double nrm = 0.0;
  const int64_t nr = n / VW;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nr; r += (int64_t)gridDim.x * blockDim.x) {
    double acc[VW], vr[VW], wr[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) acc[u] = 0.0;
    for (int i = 0; i < nvec; ++i) {
      load_rows<T, VW>(V + (int64_t)i * ldv, r, vr);
#pragma unroll
      for (int u = 0; u < VW; ++u) acc[u] = fma(vr[u], hs[i], acc[u]);
    }
    load_rows<T, VW>(w, r, wr);
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      wr[u] = (double)(T)fma(sign, acc[u], wr[u]);
      nrm = fma(wr[u], wr[u], nrm);
    }
    store_rows<T, VW>(w, r, wr);
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

// Device scalars of the GMRES cycle (Ctx::dsc): [0] norm scratch, [1] ||w||^2
// after orthogonalisation, [2] ||w|| that scales the next basis vector, [3] the
// Arnoldi estimate |g_{k+1}| / ||b|| of the relative residual, [4] valid basis
// columns of the cycle, [5] breakdown (||w|| = 0) seen in this cycle.
constexpr int DS_NRM = 1, DS_HN = 2, DS_REL = 3, DS_NCOL = 4, DS_BRK = 5, DS_H1 = 8;

// second Gram-Schmidt pass needed: the first lost more than 30 % of ||w||
__global__ void k_reorth_gate(const double *__restrict__ before2, const double *__restrict__ dsc,
                              int *__restrict__ gate) {
  *gate = sqrt(dsc[DS_NRM]) < 0.7 * sqrt(*before2) ? 1 : 0;
}

// start of a cycle: g = (beta, 0, ...), no breakdown, no columns
__global__ void k_cycle_init(double *__restrict__ g, int m, double beta, double *__restrict__ dsc) {
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = i == 0 ? beta : 0.0;
  if (threadIdx.x == 0) {
    dsc[DS_BRK] = 0.0;
    dsc[DS_NCOL] = 0.0;
  }
}

// Arnoldi step k on the device.  The basis is built with B (the Krylov spaces of
// B and I - B coincide): B v_k = V h + ||w|| v_{k+1} with h = h1 (+ h2 after a
// second pass), so column k of the Hessenberg matrix of I - B is e_k - h with
// entry -||w|| below the diagonal.  The rotations of the earlier columns are
// applied, a new Givens rotation zeroes the subdiagonal entry, and the rotated
// right-hand side g and the residual estimate are updated.  After a breakdown
// the cycle's later steps change nothing.
__global__ void k_arnoldi(int k, int m, double bnorm, const double *__restrict__ h1, const double *__restrict__ h2,
                          const int *__restrict__ gate, double *__restrict__ dsc, double *__restrict__ H,
                          double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g) {
  if (dsc[DS_BRK] != 0.0) return;
  double *col = H + (int64_t)k * (m + 1);
  const bool two = *gate != 0;
  for (int i = 0; i <= k; ++i) col[i] = (i == k ? 1.0 : 0.0) - (h1[i] + (two ? h2[i] : 0.0));
  const double hn = sqrt(dsc[DS_NRM]);
  col[k + 1] = -hn;
  for (int i = 0; i < k; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[k], b = col[k + 1];
  const double rr = hypot(a, b);
  cs[k] = rr > 0.0 ? a / rr : 1.0;
  sn[k] = rr > 0.0 ? b / rr : 0.0;
  col[k] = rr;
  col[k + 1] = 0.0;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  dsc[DS_HN] = hn;
  dsc[DS_REL] = fabs(g[k + 1]) / bnorm;
  dsc[DS_NCOL] = (double)(k + 1);
  if (!(hn > 0.0)) dsc[DS_BRK] = 1.0;
}

// y = x / s with s on the device (zero when s is not positive)
template <typename T>
__global__ void k_scale_dev(const T *__restrict__ x, const double *__restrict__ s, T *__restrict__ y, int64_t n) {
  const double d = *s;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r] = d > 0.0 ? (T)((double)x[r] / d) : (T)0;
}

template <typename T>
__global__ void k_scale_by(const T *__restrict__ x, double s, T *__restrict__ y, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r] = (T)((double)x[r] / s);
}

// y = a * x + b * y (y is not read when b == 0: it may be uninitialised memory,
// and 0 * NaN would not vanish)
template <typename TX, typename TY>
__global__ void k_axpby(double a, const TX *__restrict__ x, double b, TY *__restrict__ y, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r] = (TY)(b == 0.0 ? a * (double)x[r] : fma(a, (double)x[r], b * (double)y[r]));
}

template <typename TX, typename TY>
__global__ void k_copy(const TX *__restrict__ x, TY *__restrict__ y, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r] = (TY)x[r];
}

template <typename T>
__global__ void k_zero(T *__restrict__ y, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r] = (T)0;
}

inline bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }

struct Ctx {
  dfm_op op;
  hipStream_t st;
  bool transpose = false;  // solve (I - B)^T x = b
  int64_t n;
  double *partial = nullptr;  // [MAXV][RED_BLOCKS]
  double *dsc = nullptr;      // device scalars (DS_*), then the GMRES cycle arrays
  int *gate = nullptr;        // device flag of the second Gram-Schmidt pass
  unsigned grid() const { return ew_grid(n); }
  // 16-byte loads when every vector and the leading dimension allow them
  template <typename T>
  bool wide(const T *V, int64_t ldv, const T *w, const T *extra) const {
    constexpr int VW = 16 / sizeof(T);
    return n % VW == 0 && (ldv * (int64_t)sizeof(T)) % 16 == 0 && al16(V) && al16(w) && (!extra || al16(extra));
  }
  // out[0..nvec) = V^T w, and out[nvec] = extra . w when extra != null (device)
  template <typename T>
  hipError_t dots(const T *V, int64_t ldv, int nvec, const T *w, double *out, const T *extra = nullptr,
                  const int *g = nullptr) {
    int nout = nvec + (extra ? 1 : 0);
    constexpr int VW = 16 / sizeof(T);
    if (wide<T>(V, ldv, w, extra))
      hipLaunchKernelGGL((k_multidot<T, VW>), dim3(DOT_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, extra, w, n,
                         partial, g);
    else
      hipLaunchKernelGGL((k_multidot<T, 1>), dim3(DOT_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, extra, w, n,
                         partial, g);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nout), dim3(RED_THREADS), 0, st, partial, DOT_BLOCKS, out, g);
    return hipGetLastError();
  }
  // w += sign V h; *nrm2_out = ||w||^2 (device) when nrm2_out != null
  template <typename T>
  hipError_t combine(const T *V, int64_t ldv, int nvec, const double *h, double sign, T *w, double *nrm2_out,
                     const int *g = nullptr) {
    constexpr int VW = 16 / sizeof(T);
    double *part = nrm2_out ? partial : nullptr;
    if (wide<T>(V, ldv, w, nullptr))
      hipLaunchKernelGGL((k_combine<T, VW>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, h, sign, w, n,
                         part, g);
    else
      hipLaunchKernelGGL((k_combine<T, 1>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, ldv, nvec, h, sign, w, n,
                         part, g);
    if (nrm2_out)
      hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, nrm2_out, g);
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
  hipError_t apply_ImB(const float *x, float *y) {
    return transpose ? spmv32_t(op, x, x, y, 1.0f, -1.0f, st) : spmv32(op, x, x, y, 1.0f, -1.0f, st);
  }
  hipError_t apply_B(const float *x, float *y) {
    return transpose ? spmv32_t(op, x, nullptr, y, 0.0f, 1.0f, st) : spmv32(op, x, nullptr, y, 0.0f, 1.0f, st);
  }
};

// doubles of Ctx::dsc: scalars, h1 and h2 (MAXV + 1 each), H ((MAXV + 1) x MAXV),
// cs, sn (MAXV each), g (MAXV + 1)
constexpr size_t DSC_DOUBLES = DS_H1 + 2 * (MAXV + 1) + (size_t)(MAXV + 1) * MAXV + 2 * MAXV + (MAXV + 1);

// x[r][i] += a[r] * e[r][i]
__global__ void k_rows_axpy(const double *__restrict__ a, const float *__restrict__ e, double *__restrict__ x,
                            int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = blockIdx.y * n + i;
  x[o] = fma(a[blockIdx.y], (double)e[o], x[o]);
}

__global__ void k_zero_f64(double *__restrict__ y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

// Segmented rows: instance g owns elements [off[g], off[g+1]) of every rhs row
// (grid: x = blocks per segment, y = rhs, z = instance).
// out[r * G + g] += squared norm of instance g's part of v[r]
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_seg_norms2(const T *__restrict__ v, int64_t n,
                                                          const int64_t *__restrict__ off, int G,
                                                          double *__restrict__ out) {
  __shared__ double red[NWAVE];
  const int r = blockIdx.y, g = blockIdx.z;
  const T *row = v + (int64_t)r * n;
  const int64_t b = off[g + 1];
  double acc = 0.0;
  for (int64_t i = off[g] + blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < b;
       i += (int64_t)gridDim.x * RED_THREADS) {
    const double a = (double)row[i];
    acc = fma(a, a, acc);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NWAVE; ++w) t += red[w];
    atomicAdd(out + (int64_t)r * G + g, t);
  }
}

// t = e = (float)(s[r * G + g] * v) on instance g's part of row r
__global__ void k_seg_to_f32(const double *__restrict__ v, int64_t n, const int64_t *__restrict__ off, int G,
                             const double *__restrict__ s, float *__restrict__ t, float *__restrict__ e) {
  const int r = blockIdx.y, g = blockIdx.z;
  const double sc = s[(int64_t)r * G + g];
  const int64_t b = off[g + 1];
  for (int64_t i = off[g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = (int64_t)r * n + i;
    const float a = (float)(sc * v[o]);
    t[o] = a;
    e[o] = a;
  }
}

// gid[j] = g for the tets j of instance g (tet offsets toff; grid z = instance)
__global__ void k_fill_gid(const int64_t *__restrict__ toff, int32_t *__restrict__ gid) {
  const int g = blockIdx.z;
  for (int64_t j = toff[g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < toff[g + 1];
       j += (int64_t)gridDim.x * blockDim.x)
    gid[j] = g;
}

__global__ void k_fill_u32(unsigned *__restrict__ p, unsigned v) { *p = v; }

// *bad = 1 when some exit slot of a tet leads into another instance
__global__ void k_check_groups(const int32_t *__restrict__ dest, const int32_t *__restrict__ gid, int64_t nt,
                               unsigned *__restrict__ bad) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < 4 * nt; s += (int64_t)gridDim.x * blockDim.x)
    if (gid[dest[s] >> 2] != gid[s >> 2]) atomicOr(bad, 1u);
}

// GMRES(m) on (I - B) x = b with x0 = 0, vectors of type T.  Stops when the
// relative residual is <= rtol: the true residual when check_true (FP64 solves),
// the Arnoldi estimate otherwise (inner solves of the refinement).
template <typename T>
hipError_t gmres(Ctx &c, const T *b, T *x, T *V, T *w, T *t, int m, double rtol, int max_iter, bool check_true,
                 int &its, int &restarts, double &rel, bool &done) {
  // the residual estimate is read back every CHK steps; the steps in between are
  // queued without a host round trip (extra steps only enlarge the Krylov space)
  constexpr int CHK = 8;
  const unsigned G = c.grid();
  const int64_t n = c.n;
  double *h1 = c.dsc + DS_H1, *h2 = h1 + (MAXV + 1);
  double *Hd = h2 + (MAXV + 1), *csd = Hd + (size_t)(MAXV + 1) * MAXV, *snd = csd + MAXV, *gd = snd + MAXV;
  double bnorm;
  hipError_t e = c.norm2<T>(b, bnorm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero<T>, dim3(G), dim3(256), 0, c.st, x, n);
  done = false;
  rel = 1.0;
  if (!std::isfinite(bnorm)) {
    rel = bnorm;  // reported as a non-finite residual
    return hipGetLastError();
  }
  if (!(bnorm > 0.0)) {
    done = true;
    rel = 0.0;
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_copy<T, T>), dim3(G), dim3(256), 0, c.st, b, w, n);
  double beta = bnorm;
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), y(m), hs(8);
  while (!done && its < max_iter) {
    hipLaunchKernelGGL(k_scale_by<T>, dim3(G), dim3(256), 0, c.st, w, beta, V, n);
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(256), 0, c.st, gd, m, beta, c.dsc);
    for (int k = 0; k < m && its < max_iter; ++k) {
      T *vk = V + (int64_t)k * n;
      if ((e = c.apply_B(vk, w)) != hipSuccess) return e;
      its++;
      // classical Gram-Schmidt: one pass for V^T w and ||w||^2, one for w -= V h
      // and ||w||^2; a second pass, decided on the device, when the first lost
      // more than 30 % of ||w||
      if ((e = c.dots<T>(V, n, k + 1, w, h1, w)) != hipSuccess) return e;  // h1[k+1] = ||w||^2
      if ((e = c.combine<T>(V, n, k + 1, h1, -1.0, w, c.dsc + DS_NRM)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_reorth_gate, dim3(1), dim3(1), 0, c.st, h1 + k + 1, c.dsc, c.gate);
      if ((e = c.dots<T>(V, n, k + 1, w, h2, nullptr, c.gate)) != hipSuccess) return e;
      if ((e = c.combine<T>(V, n, k + 1, h2, -1.0, w, c.dsc + DS_NRM, c.gate)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(1), 0, c.st, k, m, bnorm, h1, h2, c.gate, c.dsc, Hd, csd, snd, gd);
      hipLaunchKernelGGL(k_scale_dev<T>, dim3(G), dim3(256), 0, c.st, w, c.dsc + DS_HN, V + (int64_t)(k + 1) * n, n);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((k + 1) % CHK == 0 || k + 1 == m || its >= max_iter) {
        if ((e = hipMemcpyAsync(hs.data(), c.dsc, sizeof(double) * 8, hipMemcpyDeviceToHost, c.st))) return e;
        if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
        rel = hs[DS_REL];
        if (!std::isfinite(rel)) return hipSuccess;
        if (rel <= (check_true ? 0.5 : 1.0) * rtol || hs[DS_BRK] != 0.0) break;
      }
    }
    // the columns of this cycle: R (rotated H) and g from the device
    if ((e = hipMemcpyAsync(hs.data(), c.dsc, sizeof(double) * 8, hipMemcpyDeviceToHost, c.st))) return e;
    if ((e = hipMemcpyAsync(H.data(), Hd, sizeof(double) * (m + 1) * m, hipMemcpyDeviceToHost, c.st))) return e;
    if ((e = hipMemcpyAsync(g.data(), gd, sizeof(double) * (m + 1), hipMemcpyDeviceToHost, c.st))) return e;
    if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
    const int k = (int)hs[DS_NCOL];
    rel = hs[DS_REL];
    if (!std::isfinite(rel)) return hipSuccess;
    // back substitution R y = g (column j of R at H[j (m + 1) ...])
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = s / H[(size_t)i * (m + 1) + i];
    }
    if (k > 0) {
      if ((e = hipMemcpyAsync(h1, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, c.st))) return e;
      if ((e = c.combine<T>(V, n, k, h1, 1.0, x, nullptr)) != hipSuccess) return e;
    }
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
// Batched mixed-precision Neumann refinement (method 0, precision 1) of R
// right-hand sides on G independent instances packed into one operator
// (instance g owns tets [toff[g], toff[g+1]); B does not couple instances).  For
// every pair (instance g, rhs r) with residual r_gr = (rho0 - (I - B) rho)_{g,r}
// (FP64):  e = sum_{k <= m} t_k, t_k = B32^k (r / |r|) in FP32 (|r| the norm of
// the whole rhs row), until |t_m|_g |r| <= max(INNER_TOL |r_gr|, rtol |rho0_gr| / 2)
// for the pair -- the partial sum leaves the residual -t_{m+1}, no larger than
// t_m for a contraction, so this is no more accuracy than the outer test needs
// and no less than the FP32 sums deliver; then rho += |r| e.  A pair stops when
// its own relative residual |r_gr| / |rho0_gr| <= rtol, and an instance all of
// whose pairs are done (or, inside the series, below their inner target) is no
// longer multiplied: its rows of t get y = 0 without reading its blocks.  G = 1
// is the plain batched solve.  info: [G][R]; iters = batched products that
// included the instance.
static dfm_status solve_groups_impl(dfm_op op, const double *rho0, double *rho, int R, const dfm_solve_opts *opts,
                                    const std::vector<int64_t> &toff, dfm_solve_info *info, hipStream_t st) {
  const int64_t n = op->ndof, K = op->K;
  const int G = (int)toff.size() - 1;
  constexpr double INNER_TOL = 1e-4;
  constexpr int CHECK = 8;  // norms of the series term every CHECK products
  float *t0 = nullptr, *t1 = nullptr, *e32 = nullptr;
  double *res = nullptr, *tmp = nullptr, *sc = nullptr;
  int64_t *off_d = nullptr, *toff_d = nullptr;
  int32_t *gid = nullptr;
  uint8_t *gact_d = nullptr;
  unsigned *bad_d = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(t0);
    (void)hipFree(t1);
    (void)hipFree(e32);
    (void)hipFree(res);
    (void)hipFree(tmp);
    (void)hipFree(sc);
    (void)hipFree(off_d);
    (void)hipFree(toff_d);
    (void)hipFree(gid);
    (void)hipFree(gact_d);
    (void)hipFree(bad_d);
  };
#define TRYB(expr)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      cleanup();                                                                             \
      return e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP;                            \
    }                                                                                        \
  } while (0)
  const size_t RG = (size_t)R * G;
  TRYB(ensure_fp32(op, st));
  TRYB(hipMalloc(&t0, sizeof(float) * (size_t)R * n));
  TRYB(hipMalloc(&t1, sizeof(float) * (size_t)R * n));
  TRYB(hipMalloc(&e32, sizeof(float) * (size_t)R * n));
  TRYB(hipMalloc(&res, sizeof(double) * (size_t)R * n));
  TRYB(hipMalloc(&tmp, sizeof(double) * n));
  TRYB(hipMalloc(&sc, sizeof(double) * 2 * RG));
  TRYB(hipMalloc(&off_d, sizeof(int64_t) * (G + 1)));
  TRYB(hipMalloc(&toff_d, sizeof(int64_t) * (G + 1)));
  const bool grouped = G > 1;
  std::vector<int64_t> off(G + 1);
  for (int g = 0; g <= G; ++g) off[g] = 4 * K * toff[g];
  TRYB(hipMemcpyAsync(off_d, off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, st));
  TRYB(hipMemcpyAsync(toff_d, toff.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, st));
  int64_t maxseg = 0;
  for (int g = 0; g < G; ++g) maxseg = std::max(maxseg, off[g + 1] - off[g]);
  if (grouped) {
    // instance of every tet, and the check that B does not couple instances
    int64_t maxt = 0;
    for (int g = 0; g < G; ++g) maxt = std::max(maxt, toff[g + 1] - toff[g]);
    TRYB(hipMalloc(&gid, sizeof(int32_t) * op->nt));
    TRYB(hipMalloc(&gact_d, sizeof(uint8_t) * G));
    TRYB(hipMalloc(&bad_d, sizeof(unsigned)));
    hipLaunchKernelGGL(k_fill_gid, dim3((unsigned)std::min<int64_t>((maxt + 255) / 256, 4096), 1, G), dim3(256), 0, st,
                       toff_d, gid);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, bad_d, 0u);
    hipLaunchKernelGGL(k_check_groups, dim3(ew_grid(4 * op->nt)), dim3(256), 0, st, op->dest, gid, op->nt, bad_d);
    unsigned bad = 0;
    TRYB(hipMemcpyAsync(&bad, bad_d, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    TRYB(hipStreamSynchronize(st));
    if (bad) {
      cleanup();
      set_error("the operator couples tets of different instances");
      return DFM_E_INVALID;
    }
  }
  const dim3 sg((unsigned)std::min<int64_t>((maxseg + 255) / 256, 1024), (unsigned)R, (unsigned)G);
  const dim3 rg((unsigned)std::min<int64_t>((maxseg + RED_THREADS - 1) / RED_THREADS, grouped ? 64 : 256),
                (unsigned)R, (unsigned)G);
  std::vector<double> h(2 * RG);
  // squared norms per (rhs, instance) of a [R][n] block into sc[0..RG) (host copy in h)
  auto seg_norms2 = [&](auto *v) -> hipError_t {
    using T = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((RG + 255) / 256)), dim3(256), 0, st, sc, (int)RG);
    hipLaunchKernelGGL(k_seg_norms2<T>, rg, dim3(RED_THREADS), 0, st, v, n, off_d, G, sc);
    hipError_t e = hipMemcpyAsync(h.data(), sc, sizeof(double) * RG, hipMemcpyDeviceToHost, st);
    return e != hipSuccess ? e : hipStreamSynchronize(st);
  };
  // r = rho0 - (I - B) rho for every rhs (FP64, one product per rhs)
  auto residual = [&]() -> hipError_t {
    for (int r = 0; r < R; ++r) {
      double *x = rho + (int64_t)r * n, *rr = res + (int64_t)r * n;
      hipError_t e = spmv(op, x, x, tmp, -1.0, 1.0, st);   // tmp = B x - x
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_copy<double, double>), dim3(ew_grid(n)), dim3(256), 0, st, rho0 + (int64_t)r * n, rr, n);
      hipLaunchKernelGGL((k_axpby<double, double>), dim3(ew_grid(n)), dim3(256), 0, st, 1.0, tmp, 1.0, rr, n);
    }
    return hipGetLastError();
  };
  // pair (r, g) at index r * G + g
  std::vector<double> bn(RG), rn(RG), rel(RG, 1.0), target(RG), rrow(R), scale(RG);
  std::vector<char> done(RG, 0), inner(RG, 0);
  std::vector<uint8_t> gact(G, 0);   // host copy of gact_d; the first update_active uploads it
  std::vector<int> gprod(G, 0);
  TRYB(seg_norms2(rho0));
  for (size_t i = 0; i < RG; ++i) {
    bn[i] = std::sqrt(h[i]);
    if (!(bn[i] > 0.0)) {
      done[i] = 1;
      rel[i] = 0.0;
    }
  }
  if (!opts->warm_start) {
    const int64_t tot = (int64_t)R * n;
    const unsigned gb = ew_grid(tot);
    hipLaunchKernelGGL(k_zero<double>, dim3(gb), dim3(256), 0, st, rho, tot);
    hipLaunchKernelGGL((k_copy<double, double>), dim3(gb), dim3(256), 0, st, rho0, res, tot);
    TRYB(hipGetLastError());
    rn = bn;
  } else {
    TRYB(residual());
    TRYB(seg_norms2(res));
    for (size_t i = 0; i < RG; ++i) {
      rn[i] = std::sqrt(h[i]);
      if (done[i]) continue;
      rel[i] = rn[i] / bn[i];
      if (rel[i] <= opts->rtol) done[i] = 1;
    }
  }
  auto all_done = [&]() {
    for (size_t i = 0; i < RG; ++i)
      if (!done[i]) return false;
    return true;
  };
  // instances still multiplied: some pair neither done nor below its inner target
  auto update_active = [&]() -> hipError_t {
    bool changed = false;
    for (int g = 0; g < G; ++g) {
      uint8_t a = 0;
      for (int r = 0; r < R; ++r) a |= (!done[(size_t)r * G + g] && !inner[(size_t)r * G + g]) ? 1 : 0;
      changed |= a != gact[g];
      gact[g] = a;
    }
    if (!grouped || !changed) return hipSuccess;
    hipError_t e = hipMemcpyAsync(gact_d, gact.data(), sizeof(uint8_t) * G, hipMemcpyHostToDevice, st);
    return e != hipSuccess ? e : hipStreamSynchronize(st);
  };
  int iters = 0;
  bool finite = true;
  for (int outer = 0; outer < 40 && iters < opts->max_iter && !all_done(); ++outer) {
    // t = e = r / |r| on the pairs not done (zero on the others)
    for (int r = 0; r < R; ++r) {
      double s2 = 0.0;
      for (int g = 0; g < G; ++g)
        if (!done[(size_t)r * G + g]) s2 += rn[(size_t)r * G + g] * rn[(size_t)r * G + g];
      rrow[r] = std::sqrt(s2);
      for (int g = 0; g < G; ++g) {
        const size_t i = (size_t)r * G + g;
        scale[i] = (!done[i] && rrow[r] > 0.0) ? 1.0 / rrow[r] : 0.0;
        inner[i] = 0;
        target[i] = std::max(INNER_TOL * rn[i], 0.5 * opts->rtol * bn[i]) / (rrow[r] > 0.0 ? rrow[r] : 1.0);
      }
    }
    std::copy(scale.begin(), scale.end(), h.begin());
    TRYB(hipMemcpyAsync(sc + RG, h.data(), sizeof(double) * RG, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_seg_to_f32, sg, dim3(256), 0, st, res, n, off_d, G, sc + RG, t0, e32);
    TRYB(hipGetLastError());
    TRYB(update_active());
    while (iters < opts->max_iter) {
      TRYB(product32(op, t0, t1, e32, R, grouped ? gid : nullptr, grouped ? gact_d : nullptr, st));
      std::swap(t0, t1);
      ++iters;
      for (int g = 0; g < G; ++g) gprod[g] += gact[g];
      if (iters % CHECK) continue;
      TRYB(seg_norms2(t0));
      bool inner_done = true;
      for (size_t i = 0; i < RG; ++i) {
        if (done[i] || inner[i]) continue;
        const double tn = std::sqrt(h[i]);
        if (!std::isfinite(tn)) finite = false;
        if (tn <= target[i]) inner[i] = 1;
        else inner_done = false;
      }
      if (inner_done || !finite) break;
      TRYB(update_active());
    }
    if (!finite) break;
    // rho += |r| e;  r = rho0 - (I - B) rho  (FP64, one product per rhs)
    for (int r = 0; r < R; ++r) h[r] = rrow[r];
    TRYB(hipMemcpyAsync(sc + RG, h.data(), sizeof(double) * R, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_rows_axpy, dim3((unsigned)((n + 255) / 256), (unsigned)R), dim3(256), 0, st, sc + RG, e32,
                       rho, n);
    TRYB(hipGetLastError());
    TRYB(residual());
    TRYB(seg_norms2(res));
    for (size_t i = 0; i < RG; ++i) {
      if (done[i]) continue;
      rn[i] = std::sqrt(h[i]);
      rel[i] = rn[i] / bn[i];
      if (!std::isfinite(rel[i])) finite = false;
      if (rel[i] <= opts->rtol) done[i] = 1;
    }
    if (!finite) break;
  }
#undef TRYB
  cleanup();
  dfm_status status = DFM_OK;
  for (int g = 0; g < G; ++g)
    for (int r = 0; r < R; ++r) {
      const size_t i = (size_t)r * G + g;
      if (info) info[(size_t)g * R + r] = dfm_solve_info{grouped ? gprod[g] : iters, 0, rel[i]};
      if (!std::isfinite(rel[i])) status = DFM_E_NUMERIC;
      else if (!done[i] && status == DFM_OK) status = DFM_E_NOCONV;
    }
  if (!finite) status = DFM_E_NUMERIC;
  if (status == DFM_E_NOCONV) set_error("solver stopped at max_iter above the tolerance");
  if (status == DFM_E_NUMERIC) set_error("non-finite residual in the solver");
  return status;
}
}  // namespace dfm

namespace dfm {
dfm_status solve_impl(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                      dfm_solve_info *info, bool transpose, void *stream_) {
  DFM_REQUIRE(op && rho0 && rho && opts, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1, DFM_E_INVALID, "nrhs must be >= 1");
  DFM_REQUIRE(opts->method >= 0 && opts->method <= 2, DFM_E_INVALID,
              "method must be 0 (Neumann), 1 (GMRES) or 2 (two-level)");
  DFM_REQUIRE(opts->precision >= 0 && opts->precision <= 2, DFM_E_INVALID, "precision must be 0, 1 or 2");
  DFM_REQUIRE((opts->method == 2) == (opts->precision == 2), DFM_E_INVALID,
              "the two-level method (2) runs with precision 2 (FP16 iterations, FP64 refinement), and only it");
  DFM_REQUIRE(opts->max_iter >= 1 && opts->rtol > 0.0, DFM_E_INVALID, "need max_iter >= 1 and rtol > 0");
  DFM_REQUIRE(!(transpose && opts->method == 2), DFM_E_UNSUPPORTED, "the two-level solver is forward only");
  DFM_REQUIRE(opts->warm_start == 0 || opts->warm_start == 1, DFM_E_INVALID, "warm_start must be 0 or 1");
  if (opts->method == 2) {
    DFM_REQUIRE(nrhs <= 65535, DFM_E_INVALID, "nrhs must be in 1..65535");
    return solve_twolevel_impl(op, rho0, rho, nrhs, opts, std::vector<int64_t>{0, op->nt}, info,
                               (hipStream_t)stream_);
  }
  const int m = opts->method == 1 ? opts->restart : 1;
  DFM_REQUIRE(m >= 1 && m <= MAXV - 1, DFM_E_INVALID, "restart must be in 1..200");
  DFM_REQUIRE(!(transpose && opts->precision == 1 && opts->method == 0), DFM_E_UNSUPPORTED,
              "transposed Neumann solves are implemented in FP64 only");
  DFM_REQUIRE(!(transpose && !op->B), DFM_E_UNSUPPORTED, "transposed solves need an operator assembled in FP64");
  DFM_REQUIRE(!(opts->warm_start && !(opts->method == 0 && opts->precision == 1)), DFM_E_UNSUPPORTED,
              "warm_start is implemented for the batched methods only (method 0 / precision 1, method 2)");
  if (opts->method == 0 && opts->precision == 1)
    return solve_groups_impl(op, rho0, rho, nrhs, opts, std::vector<int64_t>{0, op->nt}, info, (hipStream_t)stream_);
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
    (void)hipFree(c.gate);
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
  TRY(hipMalloc(&c.dsc, sizeof(double) * DSC_DOUBLES));
  TRY(hipMalloc(&c.gate, sizeof(int) * 16));
  TRY(hipMalloc(&c.partial, sizeof(double) * (size_t)RED_BLOCKS * (MAXV + 1)));
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
      for (int outer = 0; outer < 50 && inf.iters < opts->max_iter; ++outer) {
        // the correction needs no more accuracy than the outer test asks for, and
        // the FP32 iterations deliver about 1e-4 per stage
        const double inner_tol = std::min(0.5, std::max(1e-4, 0.5 * opts->rtol * bnorm / rn));
        // b32 = r / ||r||
        hipLaunchKernelGGL((k_axpby<double, float>), dim3(G), dim3(256), 0, st, 1.0 / rn, w, 0.0, b32, n);
        int its = 0, rs = 0;
        double irel;
        bool idone;
        TRY(gmres<float>(c, b32, e32, V32, w32, t32, m, inner_tol, opts->max_iter - inf.iters, true, its, rs, irel,
                         idone));
        inf.iters += its;
        inf.restarts += rs;
        if (!std::isfinite(irel)) {
          rel = irel;
          break;
        }
        // x += ||r|| e ; r = b - (I - B) x in FP64 (I - B^T for the transposed solve)
        hipLaunchKernelGGL((k_axpby<float, double>), dim3(G), dim3(256), 0, st, rn, e32, 1.0, x, n);
        TRY(c.apply_ImB(x, t));
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

extern "C" dfm_status dfm_solve_groups(dfm_op op, const double *rho0, double *rho, int nrhs,
                                       const dfm_solve_opts *opts, const int64_t *tet_offsets, int ngroups,
                                       dfm_solve_info *info, void *stream_) {
  DFM_REQUIRE(op && rho0 && rho && opts && tet_offsets, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, DFM_E_INVALID, "nrhs must be in 1..65535");
  DFM_REQUIRE(ngroups >= 1 && ngroups <= 65535, DFM_E_INVALID, "ngroups must be in 1..65535");
  DFM_REQUIRE((opts->method == 0 && opts->precision == 1) || (opts->method == 2 && opts->precision == 2),
              DFM_E_UNSUPPORTED, "instance groups are solved with method 0 / precision 1 or method 2 / precision 2");
  DFM_REQUIRE(opts->max_iter >= 1 && opts->rtol > 0.0, DFM_E_INVALID, "need max_iter >= 1 and rtol > 0");
  DFM_REQUIRE(opts->warm_start == 0 || opts->warm_start == 1, DFM_E_INVALID, "warm_start must be 0 or 1");
  DFM_REQUIRE(tet_offsets[0] == 0 && tet_offsets[ngroups] == op->nt, DFM_E_INVALID,
              "tet_offsets must start at 0 and end at nt");
  std::vector<int64_t> toff(tet_offsets, tet_offsets + ngroups + 1);
  for (int g = 0; g < ngroups; ++g)
    DFM_REQUIRE(toff[g + 1] > toff[g], DFM_E_INVALID, "tet_offsets must increase strictly");
  if (opts->method == 2) return solve_twolevel_impl(op, rho0, rho, nrhs, opts, toff, info, (hipStream_t)stream_);
  return solve_groups_impl(op, rho0, rho, nrhs, opts, toff, info, (hipStream_t)stream_);
}
