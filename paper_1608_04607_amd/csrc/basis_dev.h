// Device-side basis functions shared by the assembly and source kernels.
//
// Momentum basis on the inward hemisphere of a face frame, total degree <= D:
//   family 0: psi_(a,b) = p_a(2 cos(theta) - 1) p_b(phi/pi - 1), p_a = sqrt(2a+1) P_a,
//             k = t(t+1)/2 + b for t = a + b;
//   family 1: Zernike Z_n^m(sin(theta), phi) (Sec. 3.1), k = n(n+1)/2 + (m+n)/2.
// The Galerkin inner product is ds cos(theta) dOmega (the measure of Eq. Bapprox).
#pragma once

#include <hip/hip_runtime.h>

namespace dfm {
namespace {

constexpr int DMAX = 16;
constexpr double SEAM_SNAP = 1e-13;

template <int DM>
__device__ __forceinline__ void legendre_table(double x, int D, double *p) {
  // orthonormal p_a = sqrt(2a+1) P_a by the three-term recurrence
  // (a+1) P_{a+1} = (2a+1) x P_a - a P_{a-1}; with a a compile-time constant in the
  // unrolled loop the coefficient quotients fold to constants (no division per node)
  double pm1 = 1.0, pc = x;
  p[0] = 1.0;
#pragma unroll
  for (int a = 1; a <= DM; ++a) {
    if (a > D) break;
    p[a] = sqrt(2.0 * a + 1.0) * pc;
    double pn = ((2.0 * a + 1.0) / (a + 1.0)) * x * pc - (a / (a + 1.0)) * pm1;
    pm1 = pc;
    pc = pn;
  }
}

// The two one-dimensional factors of the Legendre family at a direction with frame
// components (dx, dy, dz): out[a] = p_a(2 dz - 1) and out[DM + 1 + b] =
// sqrt(2b+1) P_b(phi/pi - 1) for a, b <= D, zero up to DM and in out[2 DM + 2], so
// that psi_(a,b) = out[a] * out[DM + 1 + b] is the value momentum_row stores (the
// same expressions in the same order, hence the same rounding), and index 2 DM + 2
// gives 0 for padding rows.  2 DM + 3 doubles.
template <int DM, bool EXACT = false>
__device__ __forceinline__ void momentum_factors(double dx, double dy, double dz, int D_, double *__restrict__ out) {
  const int D = EXACT ? DM : D_;
  double phi = atan2(dy, dx);
  if (phi < 0.0) phi += 2.0 * M_PI;
  if (fabs(dy) <= SEAM_SNAP && dx > 0.0) phi = 0.0;
  double px[DM + 1];
  legendre_table<DM>(2.0 * dz - 1.0, D, px);
  const double y = phi * (1.0 / M_PI) - 1.0;
  double Pb = 1.0, Pbm1 = 0.0;  // P_b(y), P_{b-1}(y)
#pragma unroll
  for (int b = 0; b <= DM; ++b) {
    const bool on = b <= D;
    out[b] = on ? px[b] : 0.0;
    out[DM + 1 + b] = on ? sqrt(2.0 * b + 1.0) * Pb : 0.0;
    const double Pn = ((2.0 * b + 1.0) / (b + 1.0)) * y * Pb - (b / (b + 1.0)) * Pbm1;
    Pbm1 = Pb;
    Pb = Pn;
  }
  out[2 * DM + 2] = 0.0;
}

// One row of the momentum basis at a direction with frame components (dx, dy, dz):
// out[k] = psi_k, or (G^-1 psi)_k when GINV, for k < M = (D+1)(D+2)/2, D <= DM.
// Every loop is unrolled to the compile-time bound DM, so the basis values stay
// in registers and out is written once per entry.  The Legendre family's Gram
// matrix is pi (I + J) per block of fixed b (unknowns a = 0..D-b), solved by the
// Thomas algorithm with the elimination tables thom = [J off-diagonal | c' | 1/den];
// the Zernike family's is diagonal.
// EXACT: D == DM, so every degree guard folds at compile time.
template <int DM, bool GINV, bool EXACT = false, typename TO = double>
__device__ __forceinline__ void momentum_row(double dx, double dy, double dz, int D_, int family,
                                             const double *__restrict__ thom, TO *__restrict__ out) {
  const int D = EXACT ? DM : D_;
  if (family == 0) {
    double phi = atan2(dy, dx);
    if (phi < 0.0) phi += 2.0 * M_PI;
    if (fabs(dy) <= SEAM_SNAP && dx > 0.0) phi = 0.0;
    double px[DM + 1];
    legendre_table<DM>(2.0 * dz - 1.0, D, px);
    const double y = phi * (1.0 / M_PI) - 1.0;
    double Pb = 1.0, Pbm1 = 0.0;  // P_b(y), P_{b-1}(y)
#pragma unroll
    for (int b = 0; b <= DM; ++b) {
      if (b > D) break;
      const int N = D - b;
      const double qb = sqrt(2.0 * b + 1.0) * Pb;
      if (!GINV) {
#pragma unroll
        for (int a = 0; a <= DM - b; ++a)
          if (a <= N) out[(a + b) * (a + b + 1) / 2 + b] = (TO)(px[a] * qb);
      } else {
        const double *jo = thom;
        const double *cpb = thom + (DMAX + 1) * (DMAX + 1) + b * (DMAX + 1);
        const double *idb = thom + 2 * (DMAX + 1) * (DMAX + 1) + b * (DMAX + 1);
        double dp[DM + 1];
        double prev = 0.0;
#pragma unroll
        for (int a = 0; a <= DM - b; ++a) {
          if (a <= N) {
            const double v = px[a] * qb * (1.0 / M_PI);
            const double dpa = (a == 0) ? v * idb[0] : (v - jo[a - 1] * prev) * idb[a];
            dp[a] = dpa;
            prev = dpa;
          }
        }
        double next = 0.0;
#pragma unroll
        for (int a = DM - b; a >= 0; --a) {
          if (a <= N) {
            const double xa = (a == N) ? dp[a] : dp[a] - cpb[a] * next;
            out[(a + b) * (a + b + 1) / 2 + b] = (TO)xa;
            next = xa;
          }
        }
      }
      const double Pn = ((2.0 * b + 1.0) / (b + 1.0)) * y * Pb - (b / (b + 1.0)) * Pbm1;
      Pbm1 = Pb;
      Pb = Pn;
    }
  } else {
    // Z_n^{+-m} = P_k^{(0,m)}(2 rho^2 - 1) * (Re, Im)(dx + i dy)^m, n = m + 2k, with the
    // Jacobi polynomials P_k^{(0,m)} from their three-term recurrence; the Gram
    // matrix is diag(eps_m pi / (2n + 2)), eps_0 = 2, else 1
    double r2 = dx * dx + dy * dy;
    double tt = 2.0 * r2 - 1.0;
    double cm = 1.0, sm = 0.0;
#pragma unroll
    for (int m = 0; m <= DM; ++m) {
      if (m <= D) {
        double pkm1 = 0.0, pk = 1.0;
#pragma unroll
        for (int k = 0; 2 * k + m <= DM; ++k) {
          int n = m + 2 * k;
          if (n <= D) {
            if (k == 1) {
              pkm1 = pk;
              pk = 1.0 + (m + 2.0) * (tt - 1.0) * 0.5;
            } else if (k >= 2) {
              double kk = k, mm = m;
              double a1 = 2.0 * kk * (kk + mm) * (2.0 * kk + mm - 2.0);
              double a2 = (2.0 * kk + mm - 1.0) * ((2.0 * kk + mm) * (2.0 * kk + mm - 2.0) * tt - mm * mm);
              double a3 = 2.0 * (kk + mm - 1.0) * (kk - 1.0) * (2.0 * kk + mm);
              double pn = (a2 * pk - a3 * pkm1) / a1;
              pkm1 = pk;
              pk = pn;
            }
            const int base = n * (n + 1) / 2;
            const double gp = GINV ? (2.0 * n + 2.0) / ((m == 0 ? 2.0 : 1.0) * M_PI) : 1.0;
            const double gm = GINV ? (2.0 * n + 2.0) / M_PI : 1.0;
            out[base + (m + n) / 2] = (TO)((pk * cm) * gp);
            if (m > 0) out[base + (n - m) / 2] = (TO)((pk * sm) * gm);
          }
        }
      }
      double cn = cm * dx - sm * dy;
      double sn = cm * dy + sm * dx;
      cm = cn;
      sm = sn;
    }
  }
}

// The row of momentum_row (no Gram solve) computed in FP32, for operators stored
// in FP32: the same recurrences with float arithmetic (the frame components and
// the seam test stay FP64).  Entries carry about 1e-7 relative error instead of
// the one rounding to FP32 of the FP64 row, well inside the 1e-5 the FP32-stored
// operator is held to.
template <int DM, bool EXACT = false>
__device__ __forceinline__ void momentum_row_f32(double dx_, double dy_, double dz_, int D_, int family,
                                                 float *__restrict__ out) {
  const int D = EXACT ? DM : D_;
  const float dx = (float)dx_, dy = (float)dy_, dz = (float)dz_;
  if (family == 0) {
    float phi = atan2f(dy, dx);
    if (phi < 0.0f) phi += (float)(2.0 * M_PI);
    if (fabs(dy_) <= SEAM_SNAP && dx_ > 0.0) phi = 0.0f;
    float px[DM + 1];
    {
      const float x = 2.0f * dz - 1.0f;
      float pm1 = 1.0f, pc = x;
      px[0] = 1.0f;
#pragma unroll
      for (int a = 1; a <= DM; ++a) {
        if (a > D) break;
        px[a] = (float)sqrt(2.0 * a + 1.0) * pc;
        const float pn = (float)((2.0 * a + 1.0) / (a + 1.0)) * x * pc - (float)(a / (a + 1.0)) * pm1;
        pm1 = pc;
        pc = pn;
      }
    }
    const float y = phi * (float)(1.0 / M_PI) - 1.0f;
    float Pb = 1.0f, Pbm1 = 0.0f;
#pragma unroll
    for (int b = 0; b <= DM; ++b) {
      if (b > D) break;
      const int N = D - b;
      const float qb = (float)sqrt(2.0 * b + 1.0) * Pb;
#pragma unroll
      for (int a = 0; a <= DM - b; ++a)
        if (a <= N) out[(a + b) * (a + b + 1) / 2 + b] = px[a] * qb;
      const float Pn = (float)((2.0 * b + 1.0) / (b + 1.0)) * y * Pb - (float)(b / (b + 1.0)) * Pbm1;
      Pbm1 = Pb;
      Pb = Pn;
    }
  } else {
    const float tt = 2.0f * (dx * dx + dy * dy) - 1.0f;
    float cm = 1.0f, sm = 0.0f;
#pragma unroll
    for (int m = 0; m <= DM; ++m) {
      if (m <= D) {
        float pkm1 = 0.0f, pk = 1.0f;
#pragma unroll
        for (int k = 0; 2 * k + m <= DM; ++k) {
          const int n = m + 2 * k;
          if (n <= D) {
            if (k == 1) {
              pkm1 = pk;
              pk = 1.0f + (float)((m + 2.0) * 0.5) * (tt - 1.0f);
            } else if (k >= 2) {
              const double kk = k, mm = m;
              const double a1 = 2.0 * kk * (kk + mm) * (2.0 * kk + mm - 2.0);
              const double a2 = (2.0 * kk + mm - 1.0) * (2.0 * kk + mm) * (2.0 * kk + mm - 2.0);
              const double a2c = (2.0 * kk + mm - 1.0) * mm * mm;
              const double a3 = 2.0 * (kk + mm - 1.0) * (kk - 1.0) * (2.0 * kk + mm);
              const float pn = ((float)(a2 / a1) * tt - (float)(a2c / a1)) * pk - (float)(a3 / a1) * pkm1;
              pkm1 = pk;
              pk = pn;
            }
            const int base = n * (n + 1) / 2;
            out[base + (m + n) / 2] = pk * cm;
            if (m > 0) out[base + (n - m) / 2] = pk * sm;
          }
        }
      }
      const float cn = cm * dx - sm * dy;
      const float sn = cm * dy + sm * dx;
      cm = cn;
      sm = sn;
    }
  }
}

// psi' premultiplied by G^-1 (in place on out[0..M))
__device__ void apply_gram_inverse(double *out, int D, int family, const double *thom) {
  if (family == 1) {
    for (int n = 0; n <= D; ++n) {
      int base = n * (n + 1) / 2;
      for (int i = 0; i <= n; ++i) {
        int m = -n + 2 * i;
        double eps = (m == 0) ? 2.0 : 1.0;
        out[base + i] *= (2.0 * n + 2.0) / (eps * M_PI);
      }
    }
    return;
  }
  // block b: unknowns a = 0..N (N = D-b) at k(a,b) = (a+b)(a+b+1)/2 + b; matrix pi (I + J)
  const double *jo = thom;
  const double *cp = thom + (DMAX + 1) * (DMAX + 1);
  const double *id = thom + 2 * (DMAX + 1) * (DMAX + 1);
  for (int b = 0; b <= D; ++b) {
    int N = D - b;
    const double *cpb = cp + b * (DMAX + 1);
    const double *idb = id + b * (DMAX + 1);
    double prev = 0.0;
    for (int a = 0; a <= N; ++a) {
      int t = a + b;
      int k = t * (t + 1) / 2 + b;
      double v = out[k] * (1.0 / M_PI);
      double dpa = (a == 0) ? v * idb[0] : (v - jo[a - 1] * prev) * idb[a];
      out[k] = dpa;
      prev = dpa;
    }
    double next = 0.0;
    for (int a = N; a >= 0; --a) {
      int t = a + b;
      int k = t * (t + 1) / 2 + b;
      double xa = (a == N) ? out[k] : out[k] - cpb[a] * next;
      out[k] = xa;
      next = xa;
    }
  }
}

// In place on a contiguous column c[0..M): c <- scale * G^-1 c, loops unrolled to
// the compile-time degree bound DM >= D so each Thomas block sits in registers.
template <int DM, bool EXACT = false>
__device__ __forceinline__ void gram_solve_column(double *__restrict__ c, int D_, int family,
                                                  const double *__restrict__ thom, double scale) {
  const int D = EXACT ? DM : D_;
  if (family == 1) {
#pragma unroll
    for (int n = 0; n <= DM; ++n) {
      if (n <= D) {
#pragma unroll
        for (int i = 0; i <= n; ++i) {
          const int m = -n + 2 * i;
          c[n * (n + 1) / 2 + i] *= scale * ((2.0 * n + 2.0) / ((m == 0 ? 2.0 : 1.0) * M_PI));
        }
      }
    }
    return;
  }
#pragma unroll
  for (int b = 0; b <= DM; ++b) {
    if (b > D) break;
    const int N = D - b;
    const double *jo = thom;
    const double *cpb = thom + (DMAX + 1) * (DMAX + 1) + b * (DMAX + 1);
    const double *idb = thom + 2 * (DMAX + 1) * (DMAX + 1) + b * (DMAX + 1);
    double v[DM + 1];
#pragma unroll
    for (int a = 0; a <= DM - b; ++a)
      if (a <= N) v[a] = c[(a + b) * (a + b + 1) / 2 + b];
    double prev = 0.0;
#pragma unroll
    for (int a = 0; a <= DM - b; ++a) {
      if (a <= N) {
        const double w = v[a] * (1.0 / M_PI);
        prev = (a == 0) ? w * idb[0] : (w - jo[a - 1] * prev) * idb[a];
        v[a] = prev;
      }
    }
    double next = 0.0;
#pragma unroll
    for (int a = DM - b; a >= 0; --a) {
      if (a <= N) {
        next = (a == N) ? v[a] : v[a] - cpb[a] * next;
        c[(a + b) * (a + b + 1) / 2 + b] = scale * next;
      }
    }
  }
}

__device__ inline void pos_basis(const double *lam, double area, double *e) {
  e[0] = 1.0 / sqrt(area);
  e[1] = sqrt(6.0 / area) * (lam[1] - lam[0]);
  e[2] = sqrt(2.0 / area) * (3.0 * lam[2] - 1.0);
}


// n-point Gauss-Legendre node i (ascending) and weight on [-1, 1], by Newton's
// method on P_n from the usual cosine initial guess.
__device__ inline void gauss_legendre_node(int n, int i, double &x_out, double &w_out) {
  int ii = n - 1 - i;  // Newton iterate ii-th largest root
  double x = cos(M_PI * (ii + 0.75) / (n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pnm1 = (n == 1) ? 1.0 : p0;
    dp = n * (x * p1 - pnm1) / (x * x - 1.0);
    double dx = p1 / dp;
    x -= dx;
    if (fabs(dx) <= 1e-16) break;
  }
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  double pnm1 = (n == 1) ? 1.0 : p0;
  dp = n * (x * p1 - pnm1) / (x * x - 1.0);
  x_out = x;
  w_out = 2.0 / ((1.0 - x * x) * dp * dp);
}

}  // namespace
}  // namespace dfm
