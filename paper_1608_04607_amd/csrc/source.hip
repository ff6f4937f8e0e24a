// Sources projected onto the basis (the initial densities of Sec. 4 are projected
// onto the product basis of Eq. FBApprox the same way): the Galerkin coefficients
// of f(s, d) = sigma(s) alpha(d) on slot (j, l) are
//   (I_P kron G^-1) [ int b_p sigma ds ] x [ int psi_k alpha cos(theta) dOmega ].
// Both angular profiles used here (isotropic 1/pi and (3/(2 pi)) cos(theta)) do
// not depend on phi, so only the phi-independent momentum functions (b = 0 for
// Legendre, m = 0 for Zernike) receive a non-zero integral; it is evaluated with
// a 32-point Gauss rule in u = cos(theta), exact for these polynomials.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "dfm_internal.h"
#include "basis_dev.h"

namespace dfm {
namespace {

constexpr double PLANE_TOL = 1e-12;

__global__ void k_zero_f64(double *y, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r] = 0.0;
}

__global__ void k_init_found(int *found, int64_t ns, double *total, unsigned *flags) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < ns) found[r] = INT_MAX;
  if (r == 0) {
    *total = 0.0;
    *flags = 0u;
  }
}

// Angular coefficients ang[0..M) of alpha(u) = a0 + a1 u (u = cos(theta)).
// Thread i computes r_i = 2 pi int_0^1 alpha(u) f_i(u) u du for the i-th
// phi-independent function f_i; thread 0 then applies G^-1.
// pole != 0: the functions' values at the pole (theta = 0) instead, i.e. the
// projection of delta(rho)/(2 pi rho) (normal incidence, Sec. 4.1 Eq. RhoNeumann).
__global__ void k_axisym_profile(double a0, double a1, int pole, int D, int family, const double *thom,
                                 double *ang) {
  __shared__ double r[DMAX + 1];
  __shared__ double glx[32], glw[32];
  int t = threadIdx.x;
  if (t < 32) {
    double x, w;
    gauss_legendre_node(32, t, x, w);
    glx[t] = x;
    glw[t] = w;
  }
  __syncthreads();
  int M = (D + 1) * (D + 2) / 2;
  for (int k = t; k < M; k += blockDim.x) ang[k] = 0.0;
  int nf = (family == 0) ? D + 1 : D / 2 + 1;
  if (t < nf) {
    double acc = 0.0;
    for (int q = 0; q < 32; ++q) {
      double u = 0.5 * (glx[q] + 1.0), wq = 0.5 * glw[q];
      double f;
      if (family == 0) {
        // p_t(2u - 1)
        double x = 2.0 * u - 1.0, pm1 = 1.0, pc = x;
        if (t == 0) {
          f = 1.0;
        } else {
          for (int a = 1; a < t; ++a) {
            double pn = ((2.0 * a + 1.0) * x * pc - a * pm1) / (a + 1.0);
            pm1 = pc;
            pc = pn;
          }
          f = sqrt(2.0 * t + 1.0) * pc;
        }
      } else {
        // R_{2t}^0(rho) = P_t(2 rho^2 - 1), rho^2 = 1 - u^2
        double x = 1.0 - 2.0 * u * u, pm1 = 1.0, pc = x;
        if (t == 0) {
          f = 1.0;
        } else {
          for (int a = 1; a < t; ++a) {
            double pn = ((2.0 * a + 1.0) * x * pc - a * pm1) / (a + 1.0);
            pm1 = pc;
            pc = pn;
          }
          f = pc;
        }
      }
      acc += wq * (a0 + a1 * u) * f * u;
    }
    r[t] = 2.0 * M_PI * acc;
    // at the pole: p_t(1) = sqrt(2t+1) (Legendre, b = 0); R_{2t}^0(0) = P_t(-1) = (-1)^t (Zernike)
    if (pole) r[t] = (family == 0) ? sqrt(2.0 * t + 1.0) : ((t & 1) ? -1.0 : 1.0);
  }
  __syncthreads();
  if (t == 0) {
    if (family == 0) {
      for (int a = 0; a <= D; ++a) ang[a * (a + 1) / 2] = r[a];  // k of (a, b = 0)
      apply_gram_inverse(ang, D, 0, thom);
    } else {
      for (int h = 0; h <= D / 2; ++h) {
        int n = 2 * h;
        ang[n * (n + 1) / 2 + n / 2] = r[h];  // k of (n, m = 0)
      }
      apply_gram_inverse(ang, D, 1, thom);
    }
  }
}

__device__ inline void face_vertices_sorted(const int32_t *tets, const double *verts, int64_t slot, double v[3][3]) {
  const int32_t *t = tets + 4 * (slot >> 2);
  int l = (int)(slot & 3);
  int g[3], n = 0;
  for (int m = 0; m < 4; ++m)
    if (m != l) g[n++] = t[m];
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (g[b] < g[a]) {
        int tmp = g[a]; g[a] = g[b]; g[b] = tmp;
      }
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < 3; ++i) v[a][i] = verts[3 * (int64_t)g[a] + i];
}

// barycentric coordinates of q in the plane of v0 v1 v2; returns the distance to the plane
__device__ inline double bary3(const double v[3][3], const double *q, double *lam) {
  double e1[3], e2[3], dq[3], n[3], c1[3], c2[3];
  for (int i = 0; i < 3; ++i) {
    e1[i] = v[1][i] - v[0][i];
    e2[i] = v[2][i] - v[0][i];
    dq[i] = q[i] - v[0][i];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
  c1[0] = dq[1] * e2[2] - dq[2] * e2[1];
  c1[1] = dq[2] * e2[0] - dq[0] * e2[2];
  c1[2] = dq[0] * e2[1] - dq[1] * e2[0];
  c2[0] = e1[1] * dq[2] - e1[2] * dq[1];
  c2[1] = e1[2] * dq[0] - e1[0] * dq[2];
  c2[2] = e1[0] * dq[1] - e1[1] * dq[0];
  lam[1] = (c1[0] * n[0] + c1[1] * n[1] + c1[2] * n[2]) / nn;
  lam[2] = (c2[0] * n[0] + c2[1] * n[1] + c2[2] * n[2]) / nn;
  lam[0] = 1.0 - lam[1] - lam[2];
  return fabs(dq[0] * n[0] + dq[1] * n[1] + dq[2] * n[2]) / sqrt(nn);
}

// the lowest boundary slot whose face contains point r
__global__ void k_locate(const int32_t *tets, const double *verts, const int32_t *nbr, int64_t nslot,
                         const double *xyz, int *found) {
  int r = blockIdx.y;
  const double q[3] = {xyz[3 * r], xyz[3 * r + 1], xyz[3 * r + 2]};
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
    if (nbr[s] >= 0) continue;
    double v[3][3], lam[3];
    face_vertices_sorted(tets, verts, s, v);
    double dist = bary3(v, q, lam);
    if (dist <= PLANE_TOL && lam[0] >= -PLANE_TOL && lam[1] >= -PLANE_TOL && lam[2] >= -PLANE_TOL)
      atomicMin(&found[r], (int)s);
  }
}

// which == null: point r writes right-hand side r; else it adds into right-hand
// side which[r] (atomically: points of one right-hand side may share a face)
__global__ void k_point_coeffs(const int32_t *tets, const double *verts, const double *face, const double *xyz,
                               const int *found, int64_t ns, int P, int M, int K, int64_t ndof, double flux,
                               const double *ang, const int32_t *which, int nrhs, double *rho0,
                               unsigned *flags) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= ns) return;
  // a right-hand side index outside 0..nrhs-1 is reported, and nothing is written
  if (which && (unsigned)which[r] >= (unsigned)nrhs) {
    atomicOr(flags, 2u);
    return;
  }
  int s = found[r];
  if (s == INT_MAX) {
    atomicOr(flags, 1u);
    return;
  }
  double v[3][3], lam[3];
  face_vertices_sorted(tets, verts, s, v);
  bary3(v, xyz + 3 * r, lam);
  double e[3];
  pos_basis(lam, face[FACE_REC * (int64_t)s], e);
  double *o = rho0 + (which ? (int64_t)which[r] : r) * ndof + (int64_t)s * K;
  for (int p = 0; p < P; ++p)
    for (int k = 0; k < M; ++k) {
      if (which) atomicAdd(o + p * M + k, flux * e[p] * ang[k]);
      else o[p * M + k] = flux * e[p] * ang[k];
    }
}

__global__ void k_plane_mark(const int32_t *tets, const double *verts, const int32_t *nbr, const double *face,
                             int64_t nslot, int axis, double value, int *mark, double *total) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot) return;
  int on = 0;
  if (nbr[s] < 0) {
    double v[3][3];
    face_vertices_sorted(tets, verts, s, v);
    on = (v[0][axis] == value && v[1][axis] == value && v[2][axis] == value) ? 1 : 0;
    if (on) atomicAdd(total, face[FACE_REC * s]);
  }
  mark[s] = on;
}

// profiles 0 and 2: sigma = 1 / total area; profile 1: unit Gaussian (c, sg) integrated by
// a collapsed 32 x 32 Gauss rule on the triangle.
__global__ void k_plane_coeffs(const int32_t *tets, const double *verts, const double *face, const int *mark,
                               int64_t nslot, int profile, double cx, double cy, double cz, double sg,
                               const double *total, int P, int M, int K, double flux, const double *ang,
                               double *rho0) {
  __shared__ double glx[32], glw[32];
  if (threadIdx.x < 32) {
    double x, w;
    gauss_legendre_node(32, threadIdx.x, x, w);
    glx[threadIdx.x] = x;
    glw[threadIdx.x] = w;
  }
  __syncthreads();
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot || !mark[s]) return;
  double A = face[FACE_REC * s];
  double mom[3] = {0.0, 0.0, 0.0};
  if (profile != 1) {
    mom[0] = sqrt(A) / *total;
  } else {
    double v[3][3];
    face_vertices_sorted(tets, verts, s, v);
    const double c[3] = {cx, cy, cz};
    for (int i = 0; i < 32; ++i) {
      double u = 0.5 * (glx[i] + 1.0), wu = 0.5 * glw[i];
      for (int k = 0; k < 32; ++k) {
        double t = 0.5 * (glx[k] + 1.0), wt = 0.5 * glw[k];
        double lam[3] = {1.0 - u, u * (1.0 - t), u * t};
        double w = wu * wt * u * 2.0 * A;  // dA = 2A u du dt
        double d2 = 0.0;
        for (int x = 0; x < 3; ++x) {
          double px = lam[0] * v[0][x] + lam[1] * v[1][x] + lam[2] * v[2][x] - c[x];
          d2 += px * px;
        }
        double gs = exp(-d2 / (2.0 * sg * sg)) / (2.0 * M_PI * sg * sg);
        double e[3];
        pos_basis(lam, A, e);
        for (int p = 0; p < P; ++p) mom[p] += w * gs * e[p];
      }
    }
  }
  double *o = rho0 + s * K;
  for (int p = 0; p < P; ++p)
    for (int k = 0; k < M; ++k) o[p * M + k] = flux * mom[p] * ang[k];
}

struct Scratch {
  double *ang = nullptr, *thom = nullptr, *total = nullptr;
  int *idx = nullptr;
  unsigned *flags = nullptr;
  void release() {
    (void)hipFree(ang);
    (void)hipFree(thom);
    (void)hipFree(total);
    (void)hipFree(idx);
    (void)hipFree(flags);
  }
};

// th: host staging of the Gram factors, kept alive by the caller until the stream
// has been synchronised
hipError_t angular(dfm_op op, double a0, double a1, int pole, Scratch &sc, std::vector<double> &th,
                   hipStream_t st) {
  const int D = op->basis.mom_degree;
  th.assign(3 * (DMAX + 1) * (DMAX + 1), 0.0);
  double *jo = th.data(), *cp = jo + (DMAX + 1) * (DMAX + 1), *idn = cp + (DMAX + 1) * (DMAX + 1);
  for (int a = 0; a < DMAX; ++a) jo[a] = (a + 1.0) / std::sqrt((2.0 * a + 1.0) * (2.0 * a + 3.0));
  for (int b = 0; b <= D; ++b) {
    int N = D - b;
    double cprev = 0.0;
    for (int a = 0; a <= N; ++a) {
      double den = (a == 0) ? 1.0 : 1.0 - jo[a - 1] * cprev;
      idn[b * (DMAX + 1) + a] = 1.0 / den;
      double c = (a < N) ? jo[a] / den : 0.0;
      cp[b * (DMAX + 1) + a] = c;
      cprev = c;
    }
  }
  hipError_t e = hipMemcpyAsync(sc.thom, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_axisym_profile, dim3(1), dim3(64), 0, st, a0, a1, pole, D, op->basis.mom_family, sc.thom,
                     sc.ang);
  return hipGetLastError();
}

}  // namespace
}  // namespace dfm

using namespace dfm;

#define TRY_SC(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      sc.release();                                                                          \
      return e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP;                            \
    }                                                                                        \
  } while (0)

// The point-source projection proper: sc holds device buffers of at least
// M (ang), 3 (DMAX+1)^2 (thom), 1 (total) doubles, ns ints (idx) and one word
// (flags); nothing is allocated here.
static dfm_status source_points_run(dfm_op op, const double *xyz, int64_t ns, const int32_t *which, int nrhs,
                                    double flux, double *rho0, hipStream_t st, Scratch &sc) {
  dfm_mesh m = op->mesh;
  const int M = op->M;
  std::vector<double> th;
  int64_t tot = (int64_t)nrhs * op->ndof;
  hipLaunchKernelGGL(k_zero_f64, dim3(ew_grid(tot)), dim3(256), 0, st, rho0, tot);
  hipLaunchKernelGGL(k_init_found, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, sc.idx, ns, sc.total,
                     sc.flags);
  DFM_HIP(hipGetLastError());
  DFM_HIP(angular(op, 1.0 / M_PI, 0.0, 0, sc, th, st));
  int64_t nslot = 4 * m->nt;
  unsigned gx = (unsigned)std::min<int64_t>((nslot + 255) / 256, 1024);
  hipLaunchKernelGGL(k_locate, dim3(gx, (unsigned)ns), dim3(256), 0, st, m->tets, m->verts, m->nbr, nslot, xyz,
                     sc.idx);
  hipLaunchKernelGGL(k_point_coeffs, dim3((unsigned)((ns + 63) / 64)), dim3(64), 0, st, m->tets, m->verts, m->face,
                     xyz, sc.idx, ns, op->P, M, op->K, op->ndof, flux, sc.ang, which, nrhs, rho0, sc.flags);
  DFM_HIP(hipGetLastError());
  unsigned hflags = 0;
  DFM_HIP(hipMemcpyAsync(&hflags, sc.flags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  DFM_HIP(hipStreamSynchronize(st));
  DFM_REQUIRE(!(hflags & 2u), DFM_E_INVALID, "a right-hand side index in `which` lies outside 0..nrhs-1");
  DFM_REQUIRE(hflags == 0u, DFM_E_INVALID, "a source point lies on no boundary face");
  return DFM_OK;
}

static dfm_status source_points_impl(dfm_op op, const double *xyz, int64_t ns, const int32_t *which, int nrhs,
                                     double flux, double *rho0, hipStream_t st) {
  Scratch sc;
  const int M = op->M;
  TRY_SC(hipMalloc(&sc.ang, sizeof(double) * M));
  TRY_SC(hipMalloc(&sc.thom, sizeof(double) * 3 * (DMAX + 1) * (DMAX + 1)));
  TRY_SC(hipMalloc(&sc.total, sizeof(double)));
  TRY_SC(hipMalloc(&sc.idx, sizeof(int) * ns));
  TRY_SC(hipMalloc(&sc.flags, sizeof(unsigned)));
  dfm_status s = source_points_run(op, xyz, ns, which, nrhs, flux, rho0, st, sc);
  sc.release();
  return s;
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the same kernels with their scratch in one static
// device array per GPU.  Layout (doubles, then ints): ang [MMAX], thom
// [3 (DMAX+1)^2], total [1], flags [1 word, padded to 8 bytes], idx
// [NOALLOC_MAX_POINTS].
// ---------------------------------------------------------------------------
namespace {
constexpr int NOALLOC_MAX_POINTS = 4096;
constexpr int MMAX = (DMAX + 1) * (DMAX + 2) / 2;
constexpr size_t SCR_ANG = 0, SCR_THOM = SCR_ANG + sizeof(double) * MMAX,
                 SCR_TOTAL = SCR_THOM + sizeof(double) * 3 * (DMAX + 1) * (DMAX + 1),
                 SCR_FLAGS = SCR_TOTAL + sizeof(double), SCR_IDX = SCR_FLAGS + sizeof(double),
                 SCR_BYTES = SCR_IDX + sizeof(int) * NOALLOC_MAX_POINTS;
}  // namespace

// Each GPU the library runs on holds its own copy until the process ends.  In host
// code the name is only a stand-in: the device address comes from
// hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}
}  // namespace

extern "C" dfm_status dfm_source_points(dfm_op op, const double *xyz, int64_t ns, double flux, double *rho0,
                                        void *stream_) {
  DFM_REQUIRE(op && xyz && rho0, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(ns >= 1 && ns <= 65535, DFM_E_INVALID, "ns must be in 1..65535");
  return source_points_impl(op, xyz, ns, nullptr, (int)ns, flux, rho0, (hipStream_t)stream_);
}

extern "C" dfm_status dfm_source_points_sum(dfm_op op, const double *xyz, int64_t ns, const int32_t *which, int nrhs,
                                            double flux, double *rho0, void *stream_) {
  DFM_REQUIRE(op && xyz && which && rho0, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(ns >= 1 && ns <= 65535 && nrhs >= 1, DFM_E_INVALID, "need 1 <= ns <= 65535 and nrhs >= 1");
  return source_points_impl(op, xyz, ns, which, nrhs, flux, rho0, (hipStream_t)stream_);
}

extern "C" dfm_status dfm_source_plane(dfm_op op, int axis, double value, int profile, const double *params,
                                       double flux, double *rho0, void *stream_) {
  DFM_REQUIRE(op && rho0, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(axis >= 0 && axis <= 2, DFM_E_INVALID, "axis must be 0, 1 or 2");
  DFM_REQUIRE(profile == 0 || profile == 2 || (profile == 1 && params != nullptr && params[3] > 0.0), DFM_E_INVALID,
              "profile 0 (uniform), 1 (Gaussian, params = cx, cy, cz, sigma > 0) or 2 (uniform, normal incidence)");
  hipStream_t st = (hipStream_t)stream_;
  dfm_mesh m = op->mesh;
  Scratch sc;
  const int M = op->M;
  int64_t nslot = 4 * m->nt;
  TRY_SC(hipMalloc(&sc.ang, sizeof(double) * M));
  TRY_SC(hipMalloc(&sc.thom, sizeof(double) * 3 * (DMAX + 1) * (DMAX + 1)));
  TRY_SC(hipMalloc(&sc.total, sizeof(double)));
  TRY_SC(hipMalloc(&sc.idx, sizeof(int) * nslot));
  TRY_SC(hipMalloc(&sc.flags, sizeof(unsigned)));
  hipLaunchKernelGGL(k_zero_f64, dim3(ew_grid(op->ndof)), dim3(256), 0, st, rho0, op->ndof);
  hipLaunchKernelGGL(k_init_found, dim3(1), dim3(1), 0, st, sc.idx, 0, sc.total, sc.flags);
  TRY_SC(hipGetLastError());
  std::vector<double> th;   // host staging of the Gram factors, alive until the synchronisation below
  TRY_SC(angular(op, 0.0, 1.5 / M_PI, profile == 2, sc, th, st));
  unsigned g = (unsigned)((nslot + 255) / 256);
  hipLaunchKernelGGL(k_plane_mark, dim3(g), dim3(256), 0, st, m->tets, m->verts, m->nbr, m->face, nslot, axis, value,
                     sc.idx, sc.total);
  double c[4] = {0.0, 0.0, 0.0, 1.0};
  if (profile == 1)
    for (int i = 0; i < 4; ++i) c[i] = params[i];
  hipLaunchKernelGGL(k_plane_coeffs, dim3((unsigned)((nslot + 63) / 64)), dim3(64), 0, st, m->tets, m->verts, m->face,
                     sc.idx, nslot, profile, c[0], c[1], c[2], c[3], sc.total, op->P, M, op->K, flux, sc.ang, rho0);
  TRY_SC(hipGetLastError());
  double total = 0.0;
  TRY_SC(hipMemcpyAsync(&total, sc.total, sizeof(double), hipMemcpyDeviceToHost, st));
  TRY_SC(hipStreamSynchronize(st));
  sc.release();
  DFM_REQUIRE(total > 0.0, DFM_E_INVALID, "no boundary face lies in the requested plane");
  return DFM_OK;
}

extern "C" dfm_status dfm_source_points_noalloc(dfm_op op, const double *xyz, int64_t ns, double flux, double *rho0,
                                                void *stream_) {
  DFM_REQUIRE(op && xyz && rho0, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(ns >= 1 && ns <= NOALLOC_MAX_POINTS, DFM_E_INVALID,
              "ns must be in 1..4096 for the allocation-free projection");
  void *base = nullptr;
  DFM_HIP(scratch_address(&base));
  unsigned char *b = static_cast<unsigned char *>(base);
  Scratch sc;
  sc.ang = reinterpret_cast<double *>(b + SCR_ANG);
  sc.thom = reinterpret_cast<double *>(b + SCR_THOM);
  sc.total = reinterpret_cast<double *>(b + SCR_TOTAL);
  sc.flags = reinterpret_cast<unsigned *>(b + SCR_FLAGS);
  sc.idx = reinterpret_cast<int *>(b + SCR_IDX);
  return source_points_run(op, xyz, ns, nullptr, (int)ns, flux, rho0, (hipStream_t)stream_, sc);
}
