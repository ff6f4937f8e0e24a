// Two-level solve of (I - B) rho = rho0 (Sec. 2, Eq. GovIE) for many right-hand
// sides at once, inside FP64 iterative refinement.
//
// Why.  Each application of B moves the density one tetrahedron further, so the
// Neumann series (Eq. NSum) needs as many terms as a ray needs tet crossings to
// lose its energy: thousands on fine meshes with reflecting walls.  Two changes
// cut that count.
//
// 1. Coloured sweeps (Gauss-Seidel order).  The tets are coloured so that no two
//    that share a face are alike (two colours on the Kuhn boxes), and B is
//    applied colour by colour.  A slot written by a tet of a lower colour than
//    its own tet (type L) is read later in the same sweep, so its new value is
//    used at once; all other slots (type U) carry over to the next sweep.  With
//    the splitting B = L + U, one sweep maps the residual r to z = r + L z (the
//    L-type slots updated in place) and the next residual U z, and the solution
//    grows by z.  On two colours a density crosses two tets per sweep.
// 2. A coarse correction.  The slowly decaying part of the error is smooth in
//    space and of low order in the global direction of travel, so it is removed
//    by a Galerkin correction on a small coarse space: on every aggregate of
//    neighbouring tets, F functions of the global direction d (1, the components
//    of d, the quadratic harmonics of d), constant in space on each face of the
//    aggregate.  Expanded in a slot's own basis such a density has the
//    coefficients sqrt(area) G^-1 int psi_k Y_f cos(theta) dOmega (constant
//    position function only).  With P that prolongation,
//      A_c = P^T (I - B) P   (one dense block per independent instance),
//    and before each sweep c = 0.7 A_c^-1 P^T r (the Galerkin step, damped: the
//    undamped step of the swept operator diverges or stalls for some aggregate
//    sizes), the solution grows by P c and r' = r - P c + (B P) c is swept
//    instead of r.  B P is local: the rows of a
//    slot depend only on the aggregate of the tet upstream of it, W[slot][k][f].
//    The sweep of r' therefore needs, besides B r, terms of the form
//    (matrix) x (coarse coefficients of one aggregate); they are NAUG groups of
//    extra columns of the FP16 copy of B (see k_to_b16_aug), contracted on the
//    matrix cores with the coefficients.
//
// Precision.  Each refinement stage solves the correction system to about 1e-2,
// so r and B are FP16 (products on the FP16 matrix cores with FP32
// accumulation); the solution of a stage accumulates in FP32; the solution and
// the refinement residual rho0 - (I - B) rho stay in FP64 (the stored operator,
// FP64 or FP32).  The residual is scaled to unit max norm per (right-hand side,
// instance) before it is rounded to FP16.
//
// Layouts.  FP16 and FP32 vectors are slot-major, [slot][rhs][Kp8] (Kp8 = K
// rounded up to a multiple of 8, padding zero), so the right-hand-side tile of a
// slot is one contiguous run.  The FP16 copy of B holds, per block row, NCH
// chunks of 32 columns (three slots of Kp32 columns, then the correction
// groups and zero padding), each chunk a contiguous [K][32] tile.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dfm_internal.h"
#include "basis_dev.h"

namespace dfm {

namespace {

__device__ inline int in_face2(int l_out, int s) { return s < l_out ? s : s + 1; }

typedef _Float16 half_t;
typedef half_t h4 __attribute__((ext_vector_type(4)));
typedef half_t h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int FMAX = 9;        // coarse functions per aggregate
constexpr float COARSE_DAMPING = 0.7f;   // fraction of the Galerkin coarse step taken
// correction columns of the FP16 copy come in 4 groups of FPAD(F) columns (F used,
// the rest zero), so that 8 consecutive ones never straddle two groups
__host__ __device__ constexpr int fpad(int F) { return F <= 8 ? 8 : 16; }
constexpr int NMONO = 10;      // monomials of degree <= 2 in the frame components
constexpr int KC = 32;         // columns per chunk of the FP16 product
constexpr int ROWG = 96;       // output rows per row group of the FP16 product
constexpr int KP8MAX = 160;    // largest Kp8 the product stages (K <= 160)

// Global direction functions, as polynomials of d: index -> (monomial of d)
//   0: 1, 1: X, 2: Y, 3: Z, 4: XY, 5: YZ, 6: XZ, 7: X^2 - Y^2, 8: 3 Z^2 - 1.
// Coarse function sets: 1 -> {0}; 4 -> {0,1,2,3}; 6 -> {0,4..8}; 9 -> {0..8}.
__host__ __device__ inline int coarse_function(int F, int f) { return F == 6 ? (f == 0 ? 0 : f + 3) : f; }

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

// Mm[k][m] = G^-1 int psi_k(d) mono_m(d) cos(theta) dOmega over the inward
// hemisphere of a frame, mono = (1, x, y, z, xx, xy, xz, yy, yz, zz) of the frame
// components (Gauss rule, 32 points in u = cos(theta), 64 in phi).  One block,
// LDS sums; psi_k premultiplied by G^-1 per node.
constexpr int MONO_NU = 32, MONO_NP = 64;
__global__ void k_mono_table(int D, int family, const double *__restrict__ thom, double *__restrict__ Mm) {
  __shared__ double sums[153 * NMONO];
  __shared__ double gx[MONO_NP], gw[MONO_NP], ux[MONO_NU], uw[MONO_NU];
  const int M = (D + 1) * (D + 2) / 2;
  for (int i = threadIdx.x; i < M * NMONO; i += blockDim.x) sums[i] = 0.0;
  if (threadIdx.x < MONO_NP) {
    double x, w;
    gauss_legendre_node(MONO_NP, threadIdx.x, x, w);
    gx[threadIdx.x] = x;
    gw[threadIdx.x] = w;
  }
  if (threadIdx.x < MONO_NU) {
    double x, w;
    gauss_legendre_node(MONO_NU, threadIdx.x, x, w);
    ux[threadIdx.x] = 0.5 * (x + 1.0);
    uw[threadIdx.x] = 0.5 * w;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < MONO_NU * MONO_NP; q += blockDim.x) {
    const int iu = q / MONO_NP, ip = q - iu * MONO_NP;
    const double u = ux[iu], phi = M_PI * (gx[ip] + 1.0);
    const double w = uw[iu] * M_PI * gw[ip] * u;          // u du dphi
    const double st = sqrt(fmax(0.0, 1.0 - u * u));
    const double x = st * cos(phi), y = st * sin(phi), z = u;
    const double mono[NMONO] = {1.0, x, y, z, x * x, x * y, x * z, y * y, y * z, z * z};
    double g[153];
    momentum_row<DMAX, true>(x, y, z, D, family, thom, g);
    for (int k = 0; k < M; ++k)
      for (int m = 0; m < NMONO; ++m) atomicAdd(&sums[k * NMONO + m], w * mono[m] * g[k]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < M * NMONO; i += blockDim.x) Mm[i] = sums[i];
}

// T[f][m]: coefficients of the global function f in the frame monomials.  The
// global direction is d = x ex + y ey + z ez with (ex, ey, ez) the frame rows, so
// X = a . l, Y = b . l, Z = c . l with l = (x, y, z), a = (ex0, ey0, ez0), ...
__device__ inline void function_monomials(const double *ex, const double *ey, const double *ez, int F,
                                          double T[FMAX][NMONO]) {
  const double a[3] = {ex[0], ey[0], ez[0]}, b[3] = {ex[1], ey[1], ez[1]}, c[3] = {ex[2], ey[2], ez[2]};
  // quadratic monomial index of l_i l_j: xx 4, xy 5, xz 6, yy 7, yz 8, zz 9
  const int qi[3][3] = {{4, 5, 6}, {5, 7, 8}, {6, 8, 9}};
  auto prod = [&](const double *p, const double *q, double *out) {   // (p.l)(q.l)
    for (int m = 0; m < NMONO; ++m) out[m] = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) out[qi[i][j]] += p[i] * q[j];
  };
  for (int f = 0; f < F; ++f) {
    const int fn = coarse_function(F, f);
    double *o = T[f];
    for (int m = 0; m < NMONO; ++m) o[m] = 0.0;
    double t1[NMONO], t2[NMONO];
    switch (fn) {
      case 0: o[0] = 1.0; break;
      case 1: o[1] = a[0]; o[2] = a[1]; o[3] = a[2]; break;
      case 2: o[1] = b[0]; o[2] = b[1]; o[3] = b[2]; break;
      case 3: o[1] = c[0]; o[2] = c[1]; o[3] = c[2]; break;
      case 4: prod(a, b, o); break;
      case 5: prod(b, c, o); break;
      case 6: prod(a, c, o); break;
      case 7:
        prod(a, a, t1);
        prod(b, b, t2);
        for (int m = 0; m < NMONO; ++m) o[m] = t1[m] - t2[m];
        break;
      default:
        prod(c, c, t1);
        for (int m = 0; m < NMONO; ++m) o[m] = 3.0 * t1[m];
        o[0] -= 1.0;
        break;
    }
  }
}

// Pv[s][k][f] = sqrt(area_s) sum_m Mm[k][m] T_s[f][m] for k < R0 (rows of the
// constant position function within the first row group), zero otherwise; the
// frame of slot s from its face record (area, outward normal, frame x, frame y).
__global__ void k_coarse_pv(const double *__restrict__ face, int64_t nslot, int M, int R0, int Kp8, int F,
                            const double *__restrict__ Mm, float *__restrict__ Pv) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
    const double *rec = face + FACE_REC * s;
    const double sq = sqrt(rec[0]);
    const double ez[3] = {-rec[1], -rec[2], -rec[3]}, ex[3] = {rec[4], rec[5], rec[6]}, ey[3] = {rec[7], rec[8], rec[9]};
    double T[FMAX][NMONO];
    function_monomials(ex, ey, ez, F, T);
    float *o = Pv + s * Kp8 * F;
    for (int k = 0; k < Kp8; ++k)
      for (int f = 0; f < F; ++f) {
        double v = 0.0;
        if (k < R0 && k < M)
          for (int m = 0; m < NMONO; ++m) v += Mm[k * NMONO + m] * T[f][m];
        o[k * F + f] = (float)(sq * v);
      }
  }
}

// W[dest(br)][k][f] = sum over the block row's three blocks of
// sum_{k' < R0} B[br, s][column k'][row k] Pv[inbound slot s][k'][f]  (row k of B P)
template <typename TB>
__global__ void k_coarse_W(const TB *__restrict__ B, const int32_t *__restrict__ dest, const float *__restrict__ Pv,
                           int64_t nbr, int K, int Kp, int Kp8, int R0, int F, double *__restrict__ W64,
                           float *__restrict__ W32) {
  const int64_t tot = nbr * Kp8;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t br = i / Kp8;
    const int k = (int)(i - br * Kp8);
    const int64_t j = br >> 2;
    const int l_out = (int)(br & 3);
    double acc[FMAX];
    for (int f = 0; f < FMAX; ++f) acc[f] = 0.0;
    if (k < K)
      for (int s = 0; s < 3; ++s) {
        const float *pv = Pv + (4 * j + in_face2(l_out, s)) * (int64_t)Kp8 * F;
        const TB *col = B + ((br * 3 + s) * (int64_t)K) * Kp + k;
        for (int kk = 0; kk < R0; ++kk) {
          const double bv = (double)col[(int64_t)kk * Kp];
          for (int f = 0; f < F; ++f) acc[f] += bv * (double)pv[kk * F + f];
        }
      }
    const int64_t o = ((int64_t)dest[br] * Kp8 + k) * F;
    for (int f = 0; f < F; ++f) {
      W64[o + f] = acc[f];
      W32[o + f] = (float)acc[f];
    }
  }
}

// FP16 copy of B with the correction columns, chunk-tiled: element (row k,
// column cc) of block row br at ((br NCH + cc / KC) K + k) KC + cc % KC.
//   cc < 3 Kp32:           B[br, s][column][row k], s = cc / Kp32 (zero past K;
//                          Kp32 = K rounded up to 32, so every slot starts a chunk)
// then NAUG groups of FP = fpad(F) columns (f < F used, the rest zero):
//   group s < 3:  (B[br, s] W[inbound slot s])[k][f]  when that slot is read
//                 before it is written in a product (type U), else 0
//   group 3:      U-type destination: -(sum over U-type inbound s of B[br, s] Pv_s)[k][f]
//                 L-type destination: +(sum over L-type inbound s of B[br, s] Pv_s)[k][f]
//   group 4:      L-type destination: -Pv[dest][k][f], else 0
// (lmask[slot] = 1 marks the L-type slots, written in an earlier colour phase of
// the same product than the one that reads them).  One thread per (block row, row).
constexpr int NAUG = 5;
template <typename TB>
__global__ void k_to_b16_aug(const TB *__restrict__ B, const int32_t *__restrict__ dest, const double *__restrict__ W64,
                             const float *__restrict__ Pv, const uint8_t *__restrict__ lmask, int64_t nbr, int K,
                             int Kp, int Kp8, int R0, int F, int NCH, half_t *__restrict__ B16) {
  const int64_t tot = nbr * K;
  const int Kp32 = (K + KC - 1) / KC * KC;
  const int NC = 3 * Kp32;
  const int FP = fpad(F);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t br = i / K;
    const int k = (int)(i - br * K);
    const int64_t j = br >> 2;
    const int l_out = (int)(br & 3);
    const int64_t d = dest[br];
    const bool dl = lmask[d] != 0;
    auto put = [&](int cc, float v) {
      B16[((br * NCH + cc / KC) * (int64_t)K + k) * KC + (cc % KC)] = (half_t)v;
    };
    for (int cc = 0; cc < NC; ++cc) {
      const int sl = cc / Kp32, col = cc - sl * Kp32;
      put(cc, col < K ? (float)B[((br * 3 + sl) * (int64_t)K + col) * Kp + k] : 0.0f);
    }
    double g3[FMAX];
    for (int f = 0; f < FMAX; ++f) g3[f] = 0.0;
    for (int sl = 0; sl < 3; ++sl) {
      const int64_t slot = 4 * j + in_face2(l_out, sl);
      const bool sL = lmask[slot] != 0;
      const double *w = W64 + slot * (int64_t)Kp8 * F;
      const float *pv = Pv + slot * (int64_t)Kp8 * F;
      double bw[FMAX], bp[FMAX];
      for (int f = 0; f < FMAX; ++f) bw[f] = bp[f] = 0.0;
      const TB *row = B + ((br * 3 + sl) * (int64_t)K) * Kp + k;
      for (int kk = 0; kk < K; ++kk) {
        const double bv = (double)row[(int64_t)kk * Kp];
        for (int f = 0; f < F; ++f) {
          bw[f] += bv * w[kk * F + f];
          if (kk < R0) bp[f] += bv * (double)pv[kk * F + f];
        }
      }
      for (int f = 0; f < FP; ++f) put(NC + sl * FP + f, (f < F && !sL) ? (float)bw[f] : 0.0f);
      // group 3 sums the U-type inbound slots for a U-type destination and the
      // L-type ones for an L-type destination
      if (sL == dl)
        for (int f = 0; f < F; ++f) g3[f] += dl ? bp[f] : -bp[f];
    }
    for (int f = 0; f < FP; ++f) put(NC + 3 * FP + f, f < F ? (float)g3[f] : 0.0f);
    const float *pvd = Pv + (d * Kp8 + k) * F;
    for (int f = 0; f < FP; ++f) put(NC + 4 * FP + f, (dl && f < F && k < R0) ? -pvd[f] : 0.0f);
    for (int cc = NC + NAUG * FP; cc < NCH * KC; ++cc) put(cc, 0.0f);
  }
}

// Coarse matrix A_c = P^T P - P^T (B P), block per instance (row (g, f) of the
// block at row_off[g] + f n_g F): slot s of aggregate a with upstream aggregate u
// adds  Pv_s[:, f] . Pv_s[:, f']  at ((a, f), (a, f')) and  -Pv_s[:, f] . W_s[:, f']
// at ((a, f), (u, f')).  One thread per (slot, f, f').
__global__ void k_coarse_Ac(const float *__restrict__ Pv, const double *__restrict__ W64,
                            const int32_t *__restrict__ agg_slot, const int32_t *__restrict__ agg_up,
                            const int64_t *__restrict__ row_off, const int32_t *__restrict__ blk_lo,
                            const int32_t *__restrict__ blk_n, int64_t nslot, int Kp8, int R0, int F,
                            double *__restrict__ Ac) {
  const int64_t tot = nslot * F * F;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / (F * F);
    const int ff = (int)(i - s * F * F), f = ff / F, f2 = ff - f * F;
    const float *pv = Pv + s * Kp8 * F;
    const double *w = W64 + s * Kp8 * F;
    double pp = 0.0, pw = 0.0;
    for (int k = 0; k < R0; ++k) pp += (double)pv[k * F + f] * (double)pv[k * F + f2];
    for (int k = 0; k < Kp8; ++k) pw += (double)pv[k * F + f] * w[k * F + f2];
    const int ag = agg_slot[s], u = agg_up[s];
    const int lo = blk_lo[ag], nF = blk_n[ag] * F;
    if (u < lo || u >= lo + blk_n[ag]) continue;   // couples instances: refused on the host
    double *row = Ac + row_off[ag] + (int64_t)f * nF;
    atomicAdd(row + (ag - lo) * F + f2, pp);
    atomicAdd(row + (u - lo) * F + f2, -pw);
  }
}

__global__ void k_tet_centroids(const int32_t *__restrict__ tets, const double *__restrict__ verts, int64_t nt,
                                double *__restrict__ out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int m = 0; m < 4; ++m) s += verts[3 * (int64_t)tets[4 * t + m] + i];
      out[3 * t + i] = 0.25 * s;
    }
}

// agg_slot[s]; agg_up[dest[s]] = aggregate of tet s / 4
__global__ void k_coarse_maps(const int32_t *__restrict__ agg_tet, const int32_t *__restrict__ dest, int64_t nslot,
                              int32_t *__restrict__ agg_slot, int32_t *__restrict__ agg_up) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = agg_tet[s >> 2];
    agg_slot[s] = g;
    agg_up[dest[s]] = g;
  }
}

// ---------------------------------------------------------------------------
// The FP16 product (see the file header):
//   y[dest(br)][r][m] = sum_cc B16[br][m][cc] x[r][cc]
// with x[r][cc] = t[inbound slot s][r][cc - s Kp32] for the slot columns and the
// coarse coefficients for the correction columns (of the upstream aggregates of
// the three inbound faces, the tet's aggregate and the destination's aggregate;
// skipped when c is null), y rounded to FP16.  The tets of one colour are
// multiplied per launch (tlist); a destination slot of L type (read by a later
// colour of the same product) is written in place into t, with its old value
// added on the first product of a stage, one of U type into y.  For the first
// row group of a U-type destination also
// d0[dest][f][r] = sum_{k < R0} Pv[dest][k][f] y[r][k] (0 for L type).
//
// Persistent workgroups: grid = (P, tiles of 16 CT right-hand sides, row groups
// of 96) with P about one workgroup per compute unit; workgroup b takes the
// launch's tets b, b + P, b + 2P, ...  One wave per block row (l_out = wave).
// Each lane loads its MFMA fragments straight from memory, 16 bytes at a time:
// B rows m0 + 16 rt + lane % 16, columns 8 (lane / 16) .. + 7 of a 32-column
// chunk, and the same 8 columns of right-hand side rw0 + 16 ct + lane % 16;
// v_mfma_f32_16x16x32_f16 takes them as they are.  No LDS and no barrier.
//
// Schedule of a tet: four phases of L steps, one phase per local face p.  In
// phase p the three waves with l_out != p contract the chunks of inbound slot p,
// all at the same step, so each slot run of x is fetched from memory once and the
// other two waves find it in cache; wave l_out = p contracts its correction
// chunks meanwhile.  Steps past a wave's chunks read 16 zero bytes.  The steps
// are unrolled (L is a template parameter) and DEPTH steps are in flight: the
// last DEPTH steps of a tet load the first of the next, so the stores of one tet
// overlap the loads of the next instead of ending the workgroup.  No load is
// conditional (a load under a condition makes the compiler wait for it at once).
// The Pv^T fragments of d0 are loaded with the tet's first step and used after
// its last.
//
// Tets of instances that are not multiplied (gact[gid[tet]] == 0) load nothing
// and write y = 0 and d0 = 0.
// ---------------------------------------------------------------------------

struct P16Args {
  const half_t *B16;
  const int32_t *dest;
  int64_t nt;
  int K, Kp8, R, F, NCH, R0;
  const half_t *t;          // [4 nt][R][Kp8]
  half_t *y;                // [4 nt][R][Kp8]
  float *d0;                // [4 nt][F][R] or null
  const half_t *PvT16;      // [4 nt][16][ROWG]: Pv^T in FP16, rows >= F and columns >= R0 zero
  const int32_t *agg_slot;  // [4 nt]
  const int32_t *agg_up;    // [4 nt]
  const float *c;           // [ng F][R] or null (no correction)
  const half_t *c16;        // [ng][R][fpad(F)] the same in FP16, zero past F
  const half_t *zero16;     // 8 zero halves
  const int32_t *gid;       // tet -> instance, or null
  const uint8_t *gact;      // instance -> multiplied, or null
  const int32_t *tlist;     // tets of this launch
  int64_t ntl;              // their number
  const uint8_t *lmask;     // [4 nt] slot written in place (L type), or null
  int first;                // first product of a stage: L-type slots add their old value
};

template <int DEPTH, int CT, int L>
__global__ __launch_bounds__(256, 1) void k_spmm16(P16Args a) {
  constexpr int RT = ROWG / 16;
  constexpr int NST = 4 * L;
  static_assert(DEPTH < NST, "the prefetch reaches at most into the next tet");
  const int lane = threadIdx.x & 63;
  const int l_out = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rw0 = blockIdx.y * CT * 16;                   // first right-hand side of the workgroup
  const int m0 = blockIdx.z * ROWG;
  const int K = a.K, Kp8 = a.Kp8, F = a.F, R = a.R;
  const int64_t ldr = (int64_t)R * Kp8;
  const int nrows = min(ROWG, Kp8 - m0);
  const int col = lane & 15, kq = lane >> 4;
  const bool corr = a.c != nullptr;
  const int FP = fpad(F);
  const int brows = min(ROWG, K - m0);
  const int nsub = (K + KC - 1) / KC;                     // chunks per slot
  const int naug = (NAUG * FP + KC - 1) / KC;             // correction chunks
  const int64_t P = gridDim.x;
  const int64_t ntet = (a.ntl - (int64_t)blockIdx.x + P - 1) / P;   // tets of this workgroup
  if (ntet <= 0) return;
  const half_t *zero = a.zero16;
  const int64_t cstride = (int64_t)K * KC;                // halves per chunk
  const int64_t bstride = (int64_t)a.NCH * K * KC;        // halves per block row
  int rofs[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) rofs[ct] = min(rw0 + ct * 16 + col, R - 1);   // past R: never stored

  // what the loads of a tet need: its index (-1 past the workgroup's last tet),
  // whether it is multiplied, and the aggregates of its correction groups
  struct TetL {
    int64_t j;
    bool act;
    int gagg[NAUG];
  };
  auto tet_info = [&](int64_t q, TetL &T) {
    const bool v = q < ntet;
    T.j = v ? (int64_t)a.tlist[blockIdx.x + q * P] : -1;
    const int64_t jj = v ? T.j : 0;
    T.act = v && (a.gact == nullptr || a.gact[a.gid[jj]] != 0);
#pragma unroll
    for (int s = 0; s < 3; ++s) T.gagg[s] = (v && corr) ? a.agg_up[4 * jj + in_face2(l_out, s)] : 0;
    T.gagg[3] = (v && corr) ? a.agg_slot[4 * jj] : 0;
    T.gagg[4] = (v && corr) ? a.agg_slot[a.dest[4 * jj + l_out]] : 0;
  };
  auto load = [&](const TetL &T, int it, h8 (&Ab)[RT], h8 (&Xb)[CT]) {
    // wave-uniform: phase, step in it, chunk of B16 (-1: none)
    const int p = it / L, c = it - p * L;
    const bool aug = p == l_out;
    int bch = -1;
    if (T.act) {
      if (!aug && c < nsub) bch = (p < l_out ? p : p - 1) * nsub + c;
      if (aug && corr && c < naug) bch = 3 * nsub + c;
    }
    const int64_t jj = T.j >= 0 ? T.j : 0;
    const half_t *abase = a.B16 + (4 * jj + l_out) * bstride + (int64_t)(m0 + col) * KC + 8 * kq;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const bool ok = bch >= 0 && rt * 16 + col < brows;
      Ab[rt] = *reinterpret_cast<const h8 *>(ok ? abase + (int64_t)bch * cstride + rt * 16 * KC : zero);
    }
    // per lane: 8 columns starting at 32 c + 8 kq of slot p, or of the correction
    const int e = c * KC + 8 * kq;
    const int g = min(e / FP, NAUG - 1);
    const int ga = g == 0 ? T.gagg[0] : (g == 1 ? T.gagg[1] : (g == 2 ? T.gagg[2] : (g == 3 ? T.gagg[3] : T.gagg[4])));
    const bool xs = bch >= 0 && !aug && e < Kp8;
    const bool xc = bch >= 0 && aug && e < NAUG * FP;
    const half_t *xp = xs ? a.t + (4 * jj + p) * ldr + e : (xc ? a.c16 + (int64_t)ga * R * FP + (e - g * FP) : zero);
    const int xstride = xs ? Kp8 : (xc ? FP : 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) Xb[ct] = *reinterpret_cast<const h8 *>(xp + (int64_t)rofs[ct] * xstride);
  };
  f4 acc[RT][CT];
  auto contract = [&](const h8 (&Ab)[RT], const h8 (&Xb)[CT]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ab[rt], Xb[ct], acc[rt][ct], 0, 0, 0);
  };
  TetL cur, nxt;
  tet_info(0, cur);
  h8 A[DEPTH][RT], X[DEPTH][CT];
#pragma unroll
  for (int u = 0; u < DEPTH; ++u) load(cur, u, A[u], X[u]);
  tet_info(1, nxt);
  for (int64_t q = 0; q < ntet; ++q) {
    const int64_t j = cur.j;
    const bool act = cur.act;
    const int64_t dslot = a.dest[4 * j + l_out];
    const bool dl = a.lmask != nullptr && a.lmask[dslot] != 0;
    const bool want_d0 = m0 == 0 && a.d0 != nullptr && !dl;
    half_t *ybase = (dl ? const_cast<half_t *>(a.t) : a.y) + dslot * ldr + m0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    h4 pa[RT];
#pragma unroll
    for (int it = 0; it < NST; ++it) {
      contract(A[it % DEPTH], X[it % DEPTH]);
      if (it + DEPTH < NST) load(cur, it + DEPTH, A[it % DEPTH], X[it % DEPTH]);
      else load(nxt, it + DEPTH - NST, A[it % DEPTH], X[it % DEPTH]);
      if (it == 0) {
        // A operand of d0 = Pv^T y: row f = lane % 16, columns k = 16 rt + 4 (lane / 16) .. + 3
        const half_t *pv = want_d0 ? a.PvT16 + (dslot * 16 + col) * (int64_t)ROWG + 4 * kq : zero;
        const int pstride = want_d0 ? 16 : 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) pa[rt] = *reinterpret_cast<const h4 *>(pv + rt * pstride);
      }
    }
    // store y (rows 16 rt + 4 kq + q, right-hand side rw0 + 16 ct + col), one rhs
    // tile at a time, and d0 with one more MFMA per tile: the accumulator layout
    // of y is the B-operand layout of v_mfma_f32_16x16x16_f16
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int r = rw0 + ct * 16 + col;
      if (act && dl && a.first && r < R) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          if (rt * 16 + 4 * kq < nrows) {
            const h4 o = *reinterpret_cast<const h4 *>(ybase + (int64_t)r * Kp8 + rt * 16 + 4 * kq);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) acc[rt][ct][qq] += (float)o[qq];
          }
      }
      h4 yh[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        yh[rt] = act ? h4{(half_t)acc[rt][ct][0], (half_t)acc[rt][ct][1], (half_t)acc[rt][ct][2], (half_t)acc[rt][ct][3]}
                     : h4{0, 0, 0, 0};
      if (r < R) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          if (rt * 16 + 4 * kq < nrows) *reinterpret_cast<h4 *>(ybase + (int64_t)r * Kp8 + rt * 16 + 4 * kq) = yh[rt];
      }
      if (m0 == 0 && a.d0 != nullptr && dl && r < R) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          if (4 * kq + qq < F) a.d0[(dslot * F + 4 * kq + qq) * R + r] = 0.0f;
      }
      if (want_d0) {
        f4 dacc = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) dacc = __builtin_amdgcn_mfma_f32_16x16x16f16(pa[rt], yh[rt], dacc, 0, 0, 0);
        if (r < R) {
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int f = 4 * kq + qq;
            if (f < F) a.d0[(dslot * F + f) * R + r] = dacc[qq];
          }
        }
      }
    }
    cur = nxt;
    tet_info(q + 2, nxt);
  }
}

// The same product for tiles of 128 right-hand sides with the operands staged in
// LDS: every load of a step goes straight from memory into LDS (global_load_lds,
// 16 bytes per lane, nothing held in registers while in flight), three stages
// deep, so two steps are in flight while one is contracted.  A step's slot run of
// x and its correction coefficients are loaded once for the workgroup (each wave
// loads two of the eight 16-row tiles of each) instead of once per reading wave.
// Per step: wait for this wave's loads of the step (every wave issues the same 10
// loads per step, so the count is fixed), barrier (the other waves' loads have
// landed, and the stage read two steps ago is free), issue the loads of the step
// two ahead, read the fragments.  The fragment reads sit in one asm block with
// their own wait, so the compiler neither orders them against the pending LDS
// loads nor sees them in flight; their outputs are early-clobber, as the block
// still reads its address registers after the first result may have landed.
// Same arithmetic in the same order as k_spmm16, so the results are identical.
template <int L>
__global__ __launch_bounds__(256, 1) void k_spmm16_lds(P16Args a) {
  constexpr int CT = 8, NS = 3;
  constexpr int RT = ROWG / 16;
  constexpr int NST = 4 * L;
  constexpr int TPW = (CT + 3) / 4;                     // x tiles each wave loads per region
  constexpr int NL = RT + 2 * TPW;                      // loads per wave per step
  __shared__ h8 sA[NS][4][RT * 64];
  __shared__ h8 sX[NS][2][4 * TPW * 64];                // [0] slot run, [1] correction coefficients
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rw0 = blockIdx.y * CT * 16;
  const int m0 = blockIdx.z * ROWG;
  const int K = a.K, Kp8 = a.Kp8, F = a.F, R = a.R;
  const int64_t ldr = (int64_t)R * Kp8;
  const int nrows = min(ROWG, Kp8 - m0);
  const int col = lane & 15, kq = lane >> 4;
  const bool corr = a.c != nullptr;
  const int FP = fpad(F);
  const int brows = min(ROWG, K - m0);
  const int nsub = (K + KC - 1) / KC;
  const int naug = (NAUG * FP + KC - 1) / KC;
  const int64_t P = gridDim.x;
  const int64_t ntet = (a.ntl - (int64_t)blockIdx.x + P - 1) / P;
  if (ntet <= 0) return;
  const half_t *zero = a.zero16;
  const int64_t cstride = (int64_t)K * KC;
  const int64_t bstride = (int64_t)a.NCH * K * KC;
  // rows of x this wave loads for the workgroup: tiles t = w + 4 u (u < TPW)
  int xrow[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) xrow[u] = min(rw0 + (w + 4 * u) * 16 + col, R - 1);
  struct TetL {
    int64_t j;
    bool act;
    int gagg[4][NAUG];   // correction aggregates of each block row's wave
  };
  auto tet_info = [&](int64_t q, TetL &T) {
    const bool v = q < ntet;
    T.j = v ? (int64_t)a.tlist[blockIdx.x + q * P] : -1;
    const int64_t jj = v ? T.j : 0;
    T.act = v && (a.gact == nullptr || a.gact[a.gid[jj]] != 0);
#pragma unroll
    for (int lo = 0; lo < 4; ++lo) {
#pragma unroll
      for (int s = 0; s < 3; ++s) T.gagg[lo][s] = (v && corr) ? a.agg_up[4 * jj + in_face2(lo, s)] : 0;
      T.gagg[lo][3] = (v && corr) ? a.agg_slot[4 * jj] : 0;
      T.gagg[lo][4] = (v && corr) ? a.agg_slot[a.dest[4 * jj + lo]] : 0;
    }
  };
  typedef __attribute__((address_space(3))) void lds_t;
  // the loads of step it of tet T into stage st
  auto issue = [&](const TetL &T, int it, int st) {
    const int p = it / L, c = it - p * L;
    const int64_t jj = T.j >= 0 ? T.j : 0;
    // own block row's chunk: slot chunk of phase p, or a correction chunk in own phase
    int bch = -1;
    if (T.act) {
      if (p != w && c < nsub) bch = (p < w ? p : p - 1) * nsub + c;
      if (p == w && corr && c < naug) bch = 3 * nsub + c;
    }
    const half_t *abase = a.B16 + (4 * jj + w) * bstride + (int64_t)(m0 + col) * KC + 8 * kq;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const bool ok = bch >= 0 && rt * 16 + col < brows;
      __builtin_amdgcn_global_load_lds(ok ? abase + (int64_t)bch * cstride + rt * 16 * KC : zero,
                                       (lds_t *)&sA[st][w][rt * 64], 16, 0, 0);
    }
    // slot run of phase p, chunk c (read by the three waves other than p)
    const int e = c * KC + 8 * kq;
    const bool xs = T.act && c < nsub && e < Kp8;
    const half_t *xsb = a.t + (4 * jj + p) * ldr + e;
#pragma unroll
    for (int u = 0; u < TPW; ++u)
      __builtin_amdgcn_global_load_lds(xs ? xsb + (int64_t)xrow[u] * Kp8 : zero, (lds_t *)&sX[st][0][(w + 4 * u) * 64],
                                       16, 0, 0);
    // correction coefficients of wave p's groups, chunk c
    const int g = min(e / FP, NAUG - 1);
    const int ga = g == 0 ? T.gagg[p][0] : (g == 1 ? T.gagg[p][1] : (g == 2 ? T.gagg[p][2] : (g == 3 ? T.gagg[p][3] : T.gagg[p][4])));
    const bool xc = T.act && corr && c < naug && e < NAUG * FP;
    const half_t *xcb = a.c16 + (int64_t)ga * R * FP + (e - g * FP);
#pragma unroll
    for (int u = 0; u < TPW; ++u)
      __builtin_amdgcn_global_load_lds(xc ? xcb + (int64_t)xrow[u] * FP : zero, (lds_t *)&sX[st][1][(w + 4 * u) * 64],
                                       16, 0, 0);
  };
  f4 acc[RT][CT];
  TetL cur, nxt;
  tet_info(0, cur);
  tet_info(1, nxt);
  // prologue: steps 0 .. NS - 2 of tet 0
#pragma unroll
  for (int u = 0; u < NS - 1; ++u) issue(cur, u, u);
  constexpr unsigned WAIT = (NL * (NS - 2) & 15) | (((NL * (NS - 2)) >> 4) << 14) | (7 << 4) | (15 << 8);
  int st0 = 0;   // stage of the tet's step 0 (steps go through the stages in turn)
  for (int64_t q = 0; q < ntet; ++q) {
    const int64_t j = cur.j;
    const bool act = cur.act;
    const int64_t dslot = a.dest[4 * j + w];
    const bool dl = a.lmask != nullptr && a.lmask[dslot] != 0;
    const bool want_d0 = m0 == 0 && a.d0 != nullptr && !dl;
    half_t *ybase = (dl ? const_cast<half_t *>(a.t) : a.y) + dslot * ldr + m0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    h4 pa[RT];
#pragma unroll
    for (int it = 0; it < NST; ++it) {
      const int st = (st0 + it) % NS;
      // this step's loads (own) have landed; the barrier makes everyone's visible
      // and frees the stage read NS - 1 steps ago
      __builtin_amdgcn_s_waitcnt(WAIT);
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
      {
        const int ia = it + NS - 1;
        const int sn = (st0 + it + NS - 1) % NS;
        if (ia < NST) issue(cur, ia, sn);
        else issue(nxt, ia - NST, sn);
      }
      if (it == 0) {
        const half_t *pv = want_d0 ? a.PvT16 + (dslot * 16 + col) * (int64_t)ROWG + 4 * kq : zero;
        const int pstride = want_d0 ? 16 : 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) pa[rt] = *reinterpret_cast<const h4 *>(pv + rt * pstride);
      }
      const int p = it / L;
      h8 A[RT], X[CT];
      {
        // LDS byte addresses of the lane's fragments; the reads and their wait in one
        // block, so the compiler does not order them against the pending LDS loads
        const unsigned aad = (unsigned)(size_t)(lds_t *)&sA[st][w][lane];
        const unsigned xad = (unsigned)(size_t)(lds_t *)&sX[st][p == w ? 1 : 0][lane];
        asm volatile(
            "ds_read_b128 %0, %14 offset:0\n\t"
            "ds_read_b128 %1, %14 offset:1024\n\t"
            "ds_read_b128 %2, %14 offset:2048\n\t"
            "ds_read_b128 %3, %14 offset:3072\n\t"
            "ds_read_b128 %4, %14 offset:4096\n\t"
            "ds_read_b128 %5, %14 offset:5120\n\t"
            "ds_read_b128 %6, %15 offset:0\n\t"
            "ds_read_b128 %7, %15 offset:1024\n\t"
            "ds_read_b128 %8, %15 offset:2048\n\t"
            "ds_read_b128 %9, %15 offset:3072\n\t"
            "ds_read_b128 %10, %15 offset:4096\n\t"
            "ds_read_b128 %11, %15 offset:5120\n\t"
            "ds_read_b128 %12, %15 offset:6144\n\t"
            "ds_read_b128 %13, %15 offset:7168\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(A[0]), "=&v"(A[1]), "=&v"(A[2]), "=&v"(A[3]), "=&v"(A[4]), "=&v"(A[5]), "=&v"(X[0]), "=&v"(X[1]),
              "=&v"(X[2]), "=&v"(X[3]), "=&v"(X[4]), "=&v"(X[5]), "=&v"(X[6]), "=&v"(X[7])
            : "v"(aad), "v"(xad)
            : "memory");
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[rt], X[ct], acc[rt][ct], 0, 0, 0);
    }
    st0 = (st0 + NST) % NS;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int r = rw0 + ct * 16 + col;
      if (act && dl && a.first && r < R) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          if (rt * 16 + 4 * kq < nrows) {
            const h4 o = *reinterpret_cast<const h4 *>(ybase + (int64_t)r * Kp8 + rt * 16 + 4 * kq);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) acc[rt][ct][qq] += (float)o[qq];
          }
      }
      h4 yh[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        yh[rt] = act ? h4{(half_t)acc[rt][ct][0], (half_t)acc[rt][ct][1], (half_t)acc[rt][ct][2], (half_t)acc[rt][ct][3]}
                     : h4{0, 0, 0, 0};
      if (r < R) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          if (rt * 16 + 4 * kq < nrows) *reinterpret_cast<h4 *>(ybase + (int64_t)r * Kp8 + rt * 16 + 4 * kq) = yh[rt];
      }
      if (m0 == 0 && a.d0 != nullptr && dl && r < R) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          if (4 * kq + qq < F) a.d0[(dslot * F + 4 * kq + qq) * R + r] = 0.0f;
      }
      if (want_d0) {
        f4 dacc = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) dacc = __builtin_amdgcn_mfma_f32_16x16x16f16(pa[rt], yh[rt], dacc, 0, 0, 0);
        if (r < R) {
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int f = 4 * kq + qq;
            if (f < F) a.d0[(dslot * F + f) * R + r] = dacc[qq];
          }
        }
      }
    }
    cur = nxt;
    tet_info(q + 2, nxt);
  }
  __builtin_amdgcn_s_waitcnt(0);   // no load into LDS outlives the workgroup
}

// PvT16[s][f][k] = half(Pv[s][k][f]) for f < F and k < R0, else 0 (rows of ROWG)
__global__ void k_pvt16(const float *__restrict__ Pv, int64_t nslot, int Kp8, int F, int R0, half_t *__restrict__ PvT) {
  const int64_t tot = nslot * 16 * ROWG;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / (16 * ROWG);
    const int f = (int)((i / ROWG) % 16), k = (int)(i % ROWG);
    PvT[i] = (f < F && k < R0 && k < Kp8) ? (half_t)Pv[(s * Kp8 + k) * F + f] : (half_t)0.0f;
  }
}

// d0[s][f][r] = sum_{k < R0} Pv[s][k][f] t[s][r][k] (the coarse right-hand side of
// a vector that did not come out of the product); one workgroup per slot (grid
// stride) with the slot's Pv in LDS, one thread per right-hand side reading its
// run of t 16 bytes at a time
constexpr int D0_THREADS = 128;
__global__ __launch_bounds__(D0_THREADS) void k_d0_from_t(const half_t *__restrict__ t, const float *__restrict__ Pv,
                                                          int64_t nslot, int R, int Kp8, int R0, int F,
                                                          float *__restrict__ d0) {
  __shared__ float pvs[KP8MAX * FMAX];
  for (int64_t s = blockIdx.x; s < nslot; s += gridDim.x) {
    __syncthreads();   // the previous slot's Pv is no longer read
    for (int i = threadIdx.x; i < Kp8 * F; i += D0_THREADS) pvs[i] = i / F < R0 ? Pv[s * Kp8 * F + i] : 0.0f;
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += D0_THREADS) {
      const half_t *tp = t + (s * R + r) * Kp8;
      float acc[FMAX];
#pragma unroll
      for (int f = 0; f < FMAX; ++f) acc[f] = 0.0f;
      for (int k8 = 0; k8 < Kp8; k8 += 8) {
        const h8 v = *reinterpret_cast<const h8 *>(tp + k8);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float x = (float)v[u];
          const float *pw = pvs + (k8 + u) * F;
#pragma unroll
          for (int f = 0; f < FMAX; ++f)
            if (f < F) acc[f] = fmaf(pw[f], x, acc[f]);
        }
      }
      for (int f = 0; f < F; ++f) d0[(s * F + f) * R + r] = acc[f];
    }
  }
}

// z[(g F + f)][r] += sum of d0[slot][f][r] over the slots of aggregate g (perm
// lists the slots in aggregate order); a workgroup takes RED_CH positions of perm
// and one (f, r) column per thread, adding each run of one aggregate with one
// atomic.
constexpr int RED_CH = 256;
__global__ void k_coarse_reduce(const float *__restrict__ d0, const int32_t *__restrict__ perm,
                                const int32_t *__restrict__ agg_slot, int64_t nslot, int FR, float *__restrict__ z) {
  const int q = blockIdx.y * blockDim.x + threadIdx.x;   // column f R + r
  if (q >= FR) return;
  const int64_t i0 = blockIdx.x * (int64_t)RED_CH;
  const int64_t i1 = min(i0 + RED_CH, nslot);
  float acc = 0.0f;
  int32_t g = agg_slot[perm[i0]];
  for (int64_t i = i0; i < i1; ++i) {
    const int32_t s = perm[i];
    const int32_t gs = agg_slot[s];
    if (gs != g) {
      atomicAdd(z + (int64_t)g * FR + q, acc);
      acc = 0.0f;
      g = gs;
    }
    acc += d0[(int64_t)s * FR + q];
  }
  atomicAdd(z + (int64_t)g * FR + q, acc);
}

// c[(g f)][r] = sum over the instance block of Ai[(g f)][.] z[.][r];  csum += c.
// one_function: only the constant function (f = 0) is corrected, with the inverse
// Ai1 of the f = 0 part of the coarse matrix (rows at row_off1[g], blk_n[g] long);
// the other coefficients are zero.
__global__ void k_coarse_solve(const float *__restrict__ Ai, const int64_t *__restrict__ row_off,
                               const float *__restrict__ Ai1, const int64_t *__restrict__ row_off1, int one_function,
                               const int32_t *__restrict__ blk_lo, const int32_t *__restrict__ blk_n, int ng, int F,
                               int R, const float *__restrict__ z, float *__restrict__ c, float *__restrict__ csum,
                               half_t *__restrict__ c16, float omega) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t NG = (int64_t)ng * F;
  if (i >= NG * R) return;
  const int64_t gf = i / R;
  const int r = (int)(i - gf * R);
  const int g = (int)(gf / F), f = (int)(gf - (int64_t)g * F);
  const int lo = blk_lo[g];
  float acc = 0.0f;
  if (!one_function) {
    const int nF = blk_n[g] * F;
    const float *row = Ai + row_off[g] + (int64_t)f * nF;
    const float *zc = z + (int64_t)lo * F * R + r;
    for (int q = 0; q < nF; ++q) acc = fmaf(row[q], zc[(int64_t)q * R], acc);
  } else if (f == 0) {
    const int nb = blk_n[g];
    const float *row = Ai1 + row_off1[g];
    const float *zc = z + (int64_t)lo * F * R + r;
    for (int q = 0; q < nb; ++q) acc = fmaf(row[q], zc[(int64_t)q * F * R], acc);
  }
  acc *= omega;
  c[i] = acc;
  csum[i] += acc;
  c16[((int64_t)g * R + r) * fpad(F) + f] = (half_t)acc;
}

__global__ void k_zero_f32n(float *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

__global__ void k_zero_f64n(double *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// instance of slot s: soff[g] <= s < soff[g + 1]
__device__ inline int instance_of(const int64_t *__restrict__ soff, int G, int64_t s) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (soff[mid] <= s) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Start of a refinement stage: t[s][r][k] = half(sc[r][g] res[r][s K + k]) (zero
// padding), e = 0.
__global__ void k_stage_init(const double *__restrict__ res, int64_t nslot, int K, int Kp8,
                             const int64_t *__restrict__ soff, int G, const double *__restrict__ sc, int R,
                             half_t *__restrict__ t, float *__restrict__ e) {
  const int64_t tot = nslot * R * Kp8;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sr = i / Kp8;
    const int k = (int)(i - sr * Kp8);
    const int64_t s = sr / R;
    const int r = (int)(sr - s * R);
    const double f = sc[(int64_t)r * G + instance_of(soff, G, s)];
    t[i] = (half_t)(k < K ? (float)(f * res[(int64_t)r * nslot * K + s * K + k]) : 0.0f);
    e[i] = 0.0f;
  }
}

// e += sum of the nwin values of t in the ring (+ the coarse part when W is given:
// once per refinement stage, with the coarse coefficients summed over the stage,
// (B P) csum of the upstream aggregate on U-type slots and P csum of the slot's
// own aggregate on L-type slots, whose ring values already hold the corrected term)
constexpr int WIN = 16;
struct RingPtrs {
  const half_t *p[WIN];
};
// NW > 0: exactly NW pending terms, all loaded before the first is added (the
// full window, most flushes); NW = 0: nwin terms one after another (stage ends)
template <int NW>
__global__ void k_flush(RingPtrs ring, int nwin, int64_t nslot, int Kp8, int R, int F, const float *__restrict__ W,
                        const float *__restrict__ Pv, const uint8_t *__restrict__ lmask,
                        const int32_t *__restrict__ agg_slot, const int32_t *__restrict__ agg_up,
                        const float *__restrict__ csum, float *__restrict__ e) {
  const int64_t n8 = nslot * R * Kp8 / 8;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n8; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = 8 * q;
    const int64_t sr = i / Kp8;
    const int k0 = (int)(i - sr * Kp8);
    const int64_t s = sr / R;
    const int r = (int)(sr - s * R);
    float v[8];
    const f4 lo = *reinterpret_cast<const f4 *>(e + i), hi = *reinterpret_cast<const f4 *>(e + i + 4);
    for (int u = 0; u < 4; ++u) {
      v[u] = lo[u];
      v[u + 4] = hi[u];
    }
    if (W) {
      const bool L = lmask[s] != 0;
      const float *w = (L ? Pv : W) + (s * Kp8 + k0) * F;
      const float *cs = csum + (int64_t)(L ? agg_slot[s] : agg_up[s]) * F * R + r;
      for (int f = 0; f < F; ++f) {
        const float cf = cs[(int64_t)f * R];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = fmaf(w[u * F + f], cf, v[u]);
      }
    }
    if constexpr (NW > 0) {
      h8 x[NW];
#pragma unroll
      for (int m = 0; m < NW; ++m) x[m] = __builtin_nontemporal_load(reinterpret_cast<const h8 *>(ring.p[m] + i));
#pragma unroll
      for (int m = 0; m < NW; ++m)
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] += (float)x[m][u];
    } else {
      for (int m = 0; m < nwin; ++m) {
        const h8 x = *reinterpret_cast<const h8 *>(ring.p[m] + i);
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] += (float)x[u];
      }
    }
    *reinterpret_cast<f4 *>(e + i) = f4{v[0], v[1], v[2], v[3]};
    *reinterpret_cast<f4 *>(e + i + 4) = f4{v[4], v[5], v[6], v[7]};
  }
}

// rho[r][s K + k] += e[s][r][k] / sc[r][g]
__global__ void k_stage_update(const float *__restrict__ e, int64_t nslot, int K, int Kp8,
                               const int64_t *__restrict__ soff, int G, const double *__restrict__ sc, int R,
                               double *__restrict__ rho) {
  const int64_t n = nslot * K;
  const int64_t tot = n * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n;
    const int64_t q = i - r * n;
    const int64_t s = q / K;
    const int k = (int)(q - s * K);
    const double f = sc[r * G + instance_of(soff, G, s)];
    if (f > 0.0) rho[i] += (double)e[(s * R + r) * Kp8 + k] / f;
  }
}

// out[r * G + g] = max |v[r][i]| over instance g's elements [off[g], off[g+1])
// (non-negative doubles order like their bit patterns); grid (x, rhs, instance)
__global__ void k_seg_absmax(const double *__restrict__ v, int64_t n, const int64_t *__restrict__ off, int G,
                             unsigned long long *__restrict__ out) {
  __shared__ double red[4];
  const int r = blockIdx.y, g = blockIdx.z;
  const double *row = v + (int64_t)r * n;
  double m = 0.0;
  for (int64_t i = off[g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < off[g + 1];
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(row[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, red[w]);
    atomicMax(out + (int64_t)r * G + g, (unsigned long long)__double_as_longlong(t));
  }
}

// squared norms per (rhs, instance) of an FP64 [R][n] block; grid (x, rhs, instance)
__global__ void k_seg_norms2_d(const double *__restrict__ v, int64_t n, const int64_t *__restrict__ off, int G,
                               double *__restrict__ out) {
  __shared__ double red[4];
  const int r = blockIdx.y, g = blockIdx.z;
  const double *row = v + (int64_t)r * n;
  double acc = 0.0;
  for (int64_t i = off[g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < off[g + 1];
       i += (int64_t)gridDim.x * blockDim.x)
    acc = fma(row[i], row[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    atomicAdd(out + (int64_t)r * G + g, t);
  }
}

// squared norms per (rhs, instance) of a slot-major FP16 [slot][R][Kp8] block:
// the workgroup sums its stretch of instance g's slots into LDS per rhs, then one
// atomic per rhs (R <= 4096); grid (x, instance)
constexpr int NRM_RMAX = 4096;
__global__ void k_seg_norms2_h(const half_t *__restrict__ t, int R, int Kp8, const int64_t *__restrict__ soff, int G,
                               const uint8_t *__restrict__ skip, double *__restrict__ out) {
  __shared__ double acc_r[NRM_RMAX];
  const int g = blockIdx.y;
  for (int r = threadIdx.x; r < R; r += blockDim.x) acc_r[r] = 0.0;
  __syncthreads();
  const int ppr = Kp8 / 8;                               // 8-half pieces per (slot, rhs)
  const int64_t q0 = soff[g] * R * ppr, q1 = soff[g + 1] * R * ppr;
  for (int64_t q = q0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < q1; q += (int64_t)gridDim.x * blockDim.x) {
    if (skip && skip[q / ((int64_t)R * ppr)]) continue;
    const h8 x = *reinterpret_cast<const h8 *>(t + 8 * q);
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double a = (double)(float)x[u];
      s2 = fma(a, a, s2);
    }
    const int r = (int)((q / ppr) % R);
    atomicAdd(&acc_r[r], s2);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    if (acc_r[r] != 0.0) atomicAdd(out + (int64_t)r * G + g, acc_r[r]);
}

// ---------------------------------------------------------------------------
// FP64 residual of the stored operator for several right-hand sides per pass:
//   res[r] = rho0[r] - x[r] + B x[r],  x, rho0, res f64 [R][ndof]
// As the streaming product: each thread owns VW consecutive rows of one block
// row and streams its 3K columns once for NR right-hand sides, the x panels of
// the workgroup's block rows staged in LDS one inbound face at a time; FP64
// accumulation.
// ---------------------------------------------------------------------------
constexpr int RES_THREADS = 256;
template <typename TB>
struct VecOf;
template <>
struct VecOf<double> {
  static constexpr int W = 2;
  typedef double T __attribute__((ext_vector_type(2)));
};
template <>
struct VecOf<float> {
  static constexpr int W = 4;
  typedef float T __attribute__((ext_vector_type(4)));
};

template <typename TB, int NR>
__global__ __launch_bounds__(RES_THREADS) void k_resid(const TB *__restrict__ B, const int32_t *__restrict__ dest,
                                                      int64_t nthreads, int K, int Kp, int64_t ndof, int nr,
                                                      const double *__restrict__ x, const double *__restrict__ rho0,
                                                      double *__restrict__ res) {
  constexpr int VW = VecOf<TB>::W;
  typedef typename VecOf<TB>::T VT;
  extern __shared__ double xs_res[];
  const int GPB = Kp / VW;
  const int64_t g0 = blockIdx.x * (int64_t)RES_THREADS;
  const int64_t br0 = g0 / GPB;
  int64_t glast = g0 + RES_THREADS - 1;
  if (glast >= nthreads) glast = nthreads - 1;
  const int nrows_b = (int)(glast / GPB - br0 + 1);
  const int per_rhs = nrows_b * K;
  const int64_t g = g0 + threadIdx.x;
  const bool inrange = g < nthreads;
  const int64_t br = inrange ? g / GPB : br0;
  const int row0 = (int)(g - br * GPB) * VW;
  const double *xp = xs_res + (br - br0) * K;
  const VT *Bv = reinterpret_cast<const VT *>(B + br * 3 * (int64_t)K * Kp + row0);
  const int cstride = Kp / VW;
  double acc[NR][VW];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int u = 0; u < VW; ++u) acc[r][u] = 0.0;
  for (int s = 0; s < 3; ++s) {
    if (s) __syncthreads();
    for (int i = threadIdx.x; i < NR * per_rhs; i += RES_THREADS) {
      const int r = i / per_rhs, q = i - r * per_rhs;
      const int b = q / K, col = q - b * K;
      const int64_t bb = br0 + b;
      xs_res[i] = r < nr ? x[r * ndof + (4 * (bb >> 2) + in_face2((int)(bb & 3), s)) * (int64_t)K + col] : 0.0;
    }
    __syncthreads();
    if (inrange) {
      const VT *Bs = Bv + (int64_t)s * K * cstride;
#pragma unroll 2
      for (int c = 0; c < K; ++c) {
        const VT bv = __builtin_nontemporal_load(Bs + (int64_t)c * cstride);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double xc = xp[r * per_rhs + c];
#pragma unroll
          for (int u = 0; u < VW; ++u) acc[r][u] = fma((double)bv[u], xc, acc[r][u]);
        }
      }
    }
  }
  if (!inrange) return;
  const int64_t ob = (int64_t)dest[br] * K;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) break;
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      const int row = row0 + u;
      if (row < K) {
        const int64_t o = r * ndof + ob + row;
        res[o] = rho0[o] - x[o] + acc[r][u];
      }
    }
  }
}

// The same residual on the FP64 matrix cores (v_mfma_f64_16x16x4f64) for 16 or
// more right-hand sides, every block row read once per RM_RT of them:
// workgroup = (block row, tile of RM_RT right-hand sides, group of RM_ROWS output
// rows); its 8 waves form 2 row halves (3 row tiles of 16) x 4 rhs quarters (2
// rhs tiles of 16).  The block row's 3K columns go in chunks of RM_KC: the chunk of
// B (converted to FP64) and of x is loaded coalesced one chunk ahead into
// registers, stored to LDS and read back as fragments; accumulation in FP64.  The
// four block rows of a tet run back to back on one XCD (workgroups are dealt to
// the 8 XCDs in turn), so the x panels they share come from that XCD's L2.
constexpr int RM_THREADS = 512, RM_RT = 128, RM_ROWS = 96, RM_KC = 32;
constexpr int RM_BLD = RM_ROWS + 4;      // LDS row stride of the B chunk [column][row] (doubles)
constexpr int RM_XLD = RM_KC + 1;        // LDS row stride of the x chunk [rhs][column]
constexpr int RM_NX = RM_KC * RM_RT / RM_THREADS;
constexpr size_t RM_LDS = sizeof(double) * (size_t)(RM_KC * RM_BLD + RM_RT * RM_XLD);
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename TB>
__global__ __launch_bounds__(RM_THREADS, 2) void k_resid_mm(const TB *__restrict__ B, const int32_t *__restrict__ dest,
                                                           int64_t nt, int K, int Kp, int64_t ndof, int R,
                                                           const double *__restrict__ x,
                                                           const double *__restrict__ rho0,
                                                           double *__restrict__ res) {
  extern __shared__ double rm_lds[];
  double *bs = rm_lds;                     // [RM_KC][RM_BLD]
  double *xs = rm_lds + RM_KC * RM_BLD;    // [RM_RT][RM_XLD]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t bid = blockIdx.x;
  int64_t br = bid;
  if ((nt & 7) == 0) {
    const int64_t slot = bid >> 3, xcd = bid & 7;
    br = 4 * (8 * (slot >> 2) + xcd) + (slot & 3);
  }
  const int r0 = blockIdx.y * RM_RT;
  const int m0 = blockIdx.z * RM_ROWS;
  const int64_t j = br >> 2;
  const int l_out = (int)(br & 3);
  const int ncol = 3 * K;
  const int nchunk = (ncol + RM_KC - 1) / RM_KC;
  const TB *Bbr = B + br * 3 * (int64_t)K * Kp;
  // B chunk in 16-byte pieces: piece i -> (column i / PC, rows m0 + PW (i % PC) .. + PW - 1);
  // Kp, 3 K Kp and m0 are multiples of 4, so a piece lies wholly inside or outside
  // the column's Kp rows
  constexpr int PW = 16 / (int)sizeof(TB);
  constexpr int PC = RM_ROWS / PW;
  constexpr int NP = RM_KC * PC;
  constexpr int NPT = (NP + RM_THREADS - 1) / RM_THREADS;
  typedef TB vp __attribute__((ext_vector_type(PW)));
  int bcol[NPT], brow[NPT];
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    const int i = tid + u * RM_THREADS;
    bcol[u] = i < NP ? i / PC : RM_KC;
    brow[u] = m0 + PW * (i % PC);
  }
  const int xc = tid % RM_KC, xr = r0 + tid / RM_KC;
  constexpr int XRS = RM_THREADS / RM_KC;
  vp pb[NPT];
  double px[RM_NX];
  auto load_chunk = [&](int ch) {
    const int c0 = ch * RM_KC;
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int c = c0 + bcol[u];
      pb[u] = (bcol[u] < RM_KC && c < ncol && brow[u] < Kp)
                  ? __builtin_nontemporal_load(reinterpret_cast<const vp *>(Bbr + (int64_t)c * Kp + brow[u]))
                  : vp{};
    }
    const int c = c0 + xc;
    const int s = c / K;
    const double *xp = x + (int64_t)xr * ndof + (4 * j + in_face2(l_out, s < 3 ? s : 2)) * (int64_t)K + (c - s * K);
#pragma unroll
    for (int u = 0; u < RM_NX; ++u) px[u] = (c < ncol && xr + u * XRS < R) ? xp[(int64_t)u * XRS * ndof] : 0.0;
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < NPT; ++u)
      if (bcol[u] < RM_KC)
#pragma unroll
        for (int e = 0; e < PW; ++e) bs[bcol[u] * RM_BLD + brow[u] - m0 + e] = (double)pb[u][e];
#pragma unroll
    for (int u = 0; u < RM_NX; ++u) xs[(xr - r0 + u * XRS) * RM_XLD + xc] = px[u];
  };
  const int wr = wave >> 2, wc = wave & 3;
  const int col = lane & 15, kq = lane >> 4;
  v4d acc[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  auto contract = [&]() {
#pragma unroll
    for (int ks = 0; ks < RM_KC / 4; ++ks) {
      const int c = ks * 4 + kq;
      double av[3], bv[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) av[a] = bs[c * RM_BLD + (wr * 3 + a) * 16 + col];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = xs[((wc * 2 + b) * 16 + col) * RM_XLD + c];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  };
  load_chunk(0);
  for (int ch = 0; ch + 1 < nchunk; ++ch) {
    store_chunk();
    __syncthreads();
    load_chunk(ch + 1);   // in flight while this chunk is contracted
    contract();
    __syncthreads();
  }
  store_chunk();
  __syncthreads();
  contract();
  // the FP64 result layout: lane holds rows lane / 16 + 4 q of each 16-row tile,
  // rhs lane % 16
  const int64_t ob = (int64_t)dest[br] * K;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int r = r0 + (wc * 2 + b) * 16 + col;
    if (r >= R) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + (wr * 3 + a) * 16 + kq + 4 * q;
        if (m < K) {
          const int64_t o = (int64_t)r * ndof + ob + m;
          res[o] = rho0[o] - x[o] + acc[a][b][q];
        }
      }
  }
}

// gid[j] = g for the tets j of instance g (tet offsets toff; grid z = instance)
__global__ void k_fill_gid2(const int64_t *__restrict__ toff, int32_t *__restrict__ gid) {
  const int g = blockIdx.z;
  for (int64_t j = toff[g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < toff[g + 1];
       j += (int64_t)gridDim.x * blockDim.x)
    gid[j] = g;
}

}  // namespace

// res = rho0 - (I - B) x for R right-hand sides (FP64 vectors, the stored operator)
hipError_t residual_batched(dfm_op op, const double *rho0, const double *x, double *res, int R, hipStream_t st) {
  if (R >= 16) {
    const dim3 grid((unsigned)(4 * op->nt), (unsigned)((R + RM_RT - 1) / RM_RT),
                    (unsigned)((op->K + RM_ROWS - 1) / RM_ROWS));
    hipError_t e;
    if (op->B) {
      e = hipFuncSetAttribute((const void *)k_resid_mm<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)RM_LDS);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_resid_mm<double>, grid, dim3(RM_THREADS), RM_LDS, st, op->B, op->dest, op->nt, op->K,
                         op->Kp, op->ndof, R, x, rho0, res);
    } else {
      e = hipFuncSetAttribute((const void *)k_resid_mm<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)RM_LDS);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_resid_mm<float>, grid, dim3(RM_THREADS), RM_LDS, st, op->B32, op->dest, op->nt, op->K,
                         op->Kp, op->ndof, R, x, rho0, res);
    }
    return hipGetLastError();
  }
  constexpr int NR = 8;
  for (int r0 = 0; r0 < R; r0 += NR) {
    const int nr = std::min(NR, R - r0);
    const int64_t off = (int64_t)r0 * op->ndof;
    const int vw = op->B ? 2 : 4;
    const int gpb = op->Kp / vw;
    const int64_t nthreads = 4 * op->nt * (int64_t)gpb;
    const int64_t rows = (RES_THREADS + gpb - 1) / gpb + 1;
    const size_t lds = sizeof(double) * (size_t)(NR * rows * op->K);
    const unsigned grid = (unsigned)((nthreads + RES_THREADS - 1) / RES_THREADS);
    hipError_t e;
    if (op->B) {
      e = hipFuncSetAttribute((const void *)k_resid<double, NR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_resid<double, NR>), dim3(grid), dim3(RES_THREADS), lds, st, op->B, op->dest, nthreads,
                         op->K, op->Kp, op->ndof, nr, x + off, rho0 + off, res + off);
    } else {
      e = hipFuncSetAttribute((const void *)k_resid<float, NR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_resid<float, NR>), dim3(grid), dim3(RES_THREADS), lds, st, op->B32, op->dest, nthreads,
                         op->K, op->Kp, op->ndof, nr, x + off, rho0 + off, res + off);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dfm

extern "C" dfm_status dfm_residual(dfm_op op, const double *rho0, const double *rho, double *res, int nrhs,
                                   void *stream) {
  DFM_REQUIRE(op && rho0 && rho && res, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1, DFM_E_INVALID, "nrhs must be >= 1");
  DFM_REQUIRE(res != rho && res != rho0, DFM_E_INVALID, "res must not alias rho0 or rho");
  DFM_HIP(dfm::residual_batched(op, rho0, rho, res, nrhs, (hipStream_t)stream));
  return DFM_OK;
}

namespace dfm {

// ---------------------------------------------------------------------------
// Coarse space of an operator for a given partition into instances (cached with
// the FP16 copy of B, whose correction columns depend on it).
// ---------------------------------------------------------------------------
struct Coarse {
  std::vector<int64_t> toff;     // instance partition it was built for
  int ng = 0, F = 1, R0 = 1, NCH = 0;
  int32_t *agg_slot = nullptr, *agg_up = nullptr, *perm = nullptr, *blk_lo = nullptr, *blk_n = nullptr;
  int64_t *row_off = nullptr, *row_off1 = nullptr;
  float *Pv = nullptr, *W = nullptr, *Ai = nullptr, *Ai1 = nullptr;
  // colouring of the tets (no two tets that share a face alike): the product
  // runs colour by colour, tlist[col_off[q] ..] the tets of colour q
  int ncol = 0;
  std::vector<int64_t> col_off;
  int32_t *tlist = nullptr;
  uint8_t *lmask = nullptr;      // [4 nt] slot whose writer has a lower colour than its tet
  half_t *zero16 = nullptr;      // 8 zero halves (read in place of absent columns)
  half_t *PvT16 = nullptr;       // [4 nt][16][ROWG] Pv^T in FP16 (the d0 fragments of the product)
  void release() {
    (void)hipFree(PvT16);
    (void)hipFree(zero16);
    (void)hipFree(tlist);
    (void)hipFree(lmask);
    (void)hipFree(row_off1);
    (void)hipFree(Ai1);
    (void)hipFree(agg_slot);
    (void)hipFree(agg_up);
    (void)hipFree(perm);
    (void)hipFree(blk_lo);
    (void)hipFree(blk_n);
    (void)hipFree(row_off);
    (void)hipFree(Pv);
    (void)hipFree(W);
    (void)hipFree(Ai);
    *this = Coarse{};
  }
};

// Event timing of the product launches of method-2 solves (dfm_product_timing).
// Two events per launch from a pool kept with the operator; a solve records them
// as it goes (pending), and adds their durations to the totals once it has
// synchronised its stream at the end.
struct ProdTiming {
  std::vector<hipEvent_t> ev;
  std::vector<double> pending_bytes;   // algorithmic bytes of each launch recorded in this solve
  double ms = 0.0, bytes = 0.0;
  int64_t launches = 0;
  hipError_t begin(hipStream_t st) {
    const size_t i = 2 * pending_bytes.size();
    while (ev.size() < i + 2) {
      hipEvent_t e;
      hipError_t er = hipEventCreate(&e);
      if (er != hipSuccess) return er;
      ev.push_back(e);
    }
    return hipEventRecord(ev[i], st);
  }
  hipError_t end(hipStream_t st, double b) {
    pending_bytes.push_back(b);
    return hipEventRecord(ev[2 * pending_bytes.size() - 1], st);
  }
  // after the stream has synchronised
  void harvest() {
    for (size_t q = 0; q < pending_bytes.size(); ++q) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]) != hipSuccess) continue;
      ms += t;
      bytes += pending_bytes[q];
      ++launches;
    }
    pending_bytes.clear();
  }
  void release() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }
};

void free_twolevel(dfm_op op) {
  if (!op) return;
  if (op->ptiming) {
    op->ptiming->release();
    delete op->ptiming;
    op->ptiming = nullptr;
  }
  if (op->coarse) {
    op->coarse->release();
    delete op->coarse;
    op->coarse = nullptr;
  }
  (void)hipFree(op->B16);
  op->B16 = nullptr;
}

namespace {

// In-place inverse of the n x n row-major matrix a (Gauss-Jordan, partial
// pivoting); false when a pivot vanishes.
bool invert(std::vector<double> &a, int n) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)p * n + c])) p = r;
    const double piv = a[(size_t)p * n + c];
    if (!(std::fabs(piv) > 1e-300) || !std::isfinite(piv)) return false;
    if (p != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)p * n + k], a[(size_t)c * n + k]);
        std::swap(inv[(size_t)p * n + k], inv[(size_t)c * n + k]);
      }
    const double ip = 1.0 / piv;
    for (int k = 0; k < n; ++k) {
      a[(size_t)c * n + k] *= ip;
      inv[(size_t)c * n + k] *= ip;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  a.swap(inv);
  return true;
}

int env_int(const char *name, int dflt) {
  const char *v = getenv(name);
  return (v && *v) ? atoi(v) : dflt;
}

}  // namespace

// Build (or reuse) the coarse space of op for the instance partition toff, and the
// FP16 copy of B with its correction columns.
dfm_status ensure_coarse(dfm_op op, const std::vector<int64_t> &toff, hipStream_t st) {
  if (op->coarse && op->coarse->toff == toff && op->B16) return DFM_OK;
  if (!op->coarse) op->coarse = new Coarse();
  Coarse &C = *op->coarse;
  C.release();
  (void)hipFree(op->B16);
  op->B16 = nullptr;
  const int64_t nt = op->nt, nslot = 4 * nt, nbr = 4 * nt;
  const int K = op->K, M = op->M;
  op->Kp8 = (K + 7) / 8 * 8;
  const int Kp8 = op->Kp8;
  const int G = (int)toff.size() - 1;
  // coarse functions per aggregate (1, 4, 6 or 9) and tets per aggregate
  int F = env_int("DFM_COARSE_F", 9);
  if (F != 1 && F != 4 && F != 6 && F != 9) F = 9;
  const double tets_per_agg = (double)std::max(1, env_int("DFM_COARSE_TETS", 768));
  const int R0 = std::min(M, ROWG);
  const int NCH = 3 * ((K + KC - 1) / KC) + (NAUG * fpad(F) + KC - 1) / KC;
  double *cent_d = nullptr, *Mm = nullptr, *W64 = nullptr, *Ac = nullptr;
  int32_t *agg_tet_d = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(cent_d);
    (void)hipFree(Mm);
    (void)hipFree(W64);
    (void)hipFree(Ac);
    (void)hipFree(agg_tet_d);
  };
#define TRYC(expr)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      cleanup();                                                                             \
      C.release();                                                                           \
      return e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP;                            \
    }                                                                                        \
  } while (0)
  // 1. aggregates: per instance, cubic bins of its bounding box holding about
  //    tets_per_agg tets each; empty bins are dropped
  TRYC(hipMalloc(&cent_d, sizeof(double) * 3 * nt));
  hipLaunchKernelGGL(k_tet_centroids, dim3(ew_grid(nt)), dim3(256), 0, st, op->mesh->tets, op->mesh->verts, nt,
                     cent_d);
  TRYC(hipGetLastError());
  std::vector<double> cent(3 * nt);
  TRYC(hipMemcpyAsync(cent.data(), cent_d, sizeof(double) * 3 * nt, hipMemcpyDeviceToHost, st));
  TRYC(hipStreamSynchronize(st));
  std::vector<int32_t> agg_tet(nt);
  std::vector<int> inst_lo(G + 1, 0);   // first aggregate of every instance
  int ng = 0;
  for (int g = 0; g < G; ++g) {
    inst_lo[g] = ng;
    const int64_t a0 = toff[g], a1 = toff[g + 1];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t t = a0; t < a1; ++t)
      for (int i = 0; i < 3; ++i) {
        lo[i] = std::min(lo[i], cent[3 * t + i]);
        hi[i] = std::max(hi[i], cent[3 * t + i]);
      }
    const double target = std::max(1.0, std::round((double)(a1 - a0) / tets_per_agg));
    double ext[3], vol = 1.0;
    for (int i = 0; i < 3; ++i) {
      ext[i] = std::max(hi[i] - lo[i], 1e-12);
      vol *= ext[i];
    }
    const double side = std::cbrt(vol / target);
    int nb[3];
    for (int i = 0; i < 3; ++i) nb[i] = std::max(1, (int)std::lround(ext[i] / side));
    std::vector<int> id((size_t)nb[0] * nb[1] * nb[2], -1);
    for (int64_t t = a0; t < a1; ++t) {
      int b[3];
      for (int i = 0; i < 3; ++i)
        b[i] = std::min(nb[i] - 1, std::max(0, (int)((cent[3 * t + i] - lo[i]) / ext[i] * nb[i])));
      const size_t key = ((size_t)b[2] * nb[1] + b[1]) * nb[0] + b[0];
      if (id[key] < 0) id[key] = ng++;
      agg_tet[t] = id[key];
    }
  }
  inst_lo[G] = ng;
  C.ng = ng;
  C.F = F;
  C.R0 = R0;
  C.NCH = NCH;
  std::vector<int64_t> row_off(ng);
  std::vector<int32_t> blk_lo(ng), blk_n(ng);
  int64_t ai_size = 0;
  for (int g = 0; g < G; ++g) {
    const int n = inst_lo[g + 1] - inst_lo[g];
    for (int q = 0; q < n; ++q) {
      row_off[inst_lo[g] + q] = ai_size + (int64_t)q * F * n * F;
      blk_lo[inst_lo[g] + q] = inst_lo[g];
      blk_n[inst_lo[g] + q] = n;
    }
    ai_size += (int64_t)n * F * n * F;
  }
  // 2. colouring: greedy over a breadth-first order of the face graph (two
  //    colours on the Kuhn boxes, whose face graph is bipartite); the slots
  //    written by a tet of a lower colour than their own are of L type
  {
    std::vector<int32_t> dh(nslot);
    TRYC(hipMemcpyAsync(dh.data(), op->dest, sizeof(int32_t) * nslot, hipMemcpyDeviceToHost, st));
    TRYC(hipStreamSynchronize(st));
    std::vector<int32_t> writer(nslot, -1);
    for (int64_t b = 0; b < nslot; ++b) writer[dh[b]] = (int32_t)(b >> 2);
    std::vector<int32_t> nb(nslot, -1);        // the neighbour across each face, -1 on the boundary
    for (int64_t sl = 0; sl < nslot; ++sl) {
      const int32_t w = writer[sl];
      if (w >= 0 && w != (int32_t)(sl >> 2)) nb[sl] = w;
    }
    std::vector<int8_t> color(nt, -1);
    std::vector<int32_t> queue;
    queue.reserve(nt);
    for (int64_t t0 = 0; t0 < nt; ++t0) {
      if (color[t0] >= 0) continue;
      color[t0] = 0;
      queue.clear();
      queue.push_back((int32_t)t0);
      for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t u = queue[h];
        for (int l = 0; l < 4; ++l) {
          const int32_t v = nb[4 * (int64_t)u + l];
          if (v < 0 || color[v] >= 0) continue;
          unsigned used = 0;
          for (int l2 = 0; l2 < 4; ++l2) {
            const int32_t x = nb[4 * (int64_t)v + l2];
            if (x >= 0 && color[x] >= 0) used |= 1u << color[x];
          }
          int cq = 0;
          while (used & (1u << cq)) ++cq;
          color[v] = (int8_t)cq;
          queue.push_back(v);
        }
      }
    }
    int ncol = 1;
    for (int64_t t = 0; t < nt; ++t) ncol = std::max(ncol, (int)color[t] + 1);
    C.ncol = ncol;
    C.col_off.assign(ncol + 1, 0);
    for (int64_t t = 0; t < nt; ++t) C.col_off[color[t] + 1]++;
    for (int q = 0; q < ncol; ++q) C.col_off[q + 1] += C.col_off[q];
    std::vector<int64_t> pos(C.col_off.begin(), C.col_off.end() - 1);
    std::vector<int32_t> tl(nt);
    for (int64_t t = 0; t < nt; ++t) tl[pos[color[t]]++] = (int32_t)t;
    std::vector<uint8_t> lm(nslot, 0);
    for (int64_t sl = 0; sl < nslot; ++sl) lm[sl] = (nb[sl] >= 0 && color[nb[sl]] < color[sl >> 2]) ? 1 : 0;
    TRYC(hipMalloc(&C.zero16, 64));
    TRYC(hipMemsetAsync(C.zero16, 0, 64, st));
    TRYC(hipMalloc(&C.tlist, sizeof(int32_t) * nt));
    TRYC(hipMalloc(&C.lmask, sizeof(uint8_t) * nslot));
    TRYC(hipMemcpyAsync(C.tlist, tl.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, st));
    TRYC(hipMemcpyAsync(C.lmask, lm.data(), sizeof(uint8_t) * nslot, hipMemcpyHostToDevice, st));
    TRYC(hipStreamSynchronize(st));   // the host vectors must outlive their copies
  }
  // 3. maps, the coarse basis Pv, W = B P, and the FP16 copy with its columns
  TRYC(hipMalloc(&agg_tet_d, sizeof(int32_t) * nt));
  TRYC(hipMalloc(&C.agg_slot, sizeof(int32_t) * nslot));
  TRYC(hipMalloc(&C.agg_up, sizeof(int32_t) * nslot));
  TRYC(hipMalloc(&Mm, sizeof(double) * M * NMONO));
  TRYC(hipMalloc(&C.Pv, sizeof(float) * nslot * Kp8 * F));
  TRYC(hipMalloc(&C.PvT16, sizeof(half_t) * nslot * 16 * ROWG));
  TRYC(hipMalloc(&C.W, sizeof(float) * nslot * Kp8 * F));
  TRYC(hipMalloc(&W64, sizeof(double) * nslot * Kp8 * F));
  TRYC(hipMalloc(&C.row_off, sizeof(int64_t) * ng));
  TRYC(hipMalloc(&C.blk_lo, sizeof(int32_t) * ng));
  TRYC(hipMalloc(&C.blk_n, sizeof(int32_t) * ng));
  TRYC(hipMalloc(&Ac, sizeof(double) * std::max<int64_t>(ai_size, 1)));
  TRYC(hipMalloc(&op->B16, sizeof(half_t) * nbr * NCH * K * KC));
  TRYC(hipMemcpyAsync(agg_tet_d, agg_tet.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, st));
  TRYC(hipMemcpyAsync(C.row_off, row_off.data(), sizeof(int64_t) * ng, hipMemcpyHostToDevice, st));
  TRYC(hipMemcpyAsync(C.blk_lo, blk_lo.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice, st));
  TRYC(hipMemcpyAsync(C.blk_n, blk_n.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_coarse_maps, dim3(ew_grid(nslot)), dim3(256), 0, st, agg_tet_d, op->dest, nslot, C.agg_slot,
                     C.agg_up);
  hipLaunchKernelGGL(k_mono_table, dim3(1), dim3(256), 0, st, op->basis.mom_degree, op->basis.mom_family, op->thom, Mm);
  hipLaunchKernelGGL(k_coarse_pv, dim3(ew_grid(nslot)), dim3(256), 0, st, op->mesh->face, nslot, M, R0, Kp8, F, Mm,
                     C.Pv);
  hipLaunchKernelGGL(k_pvt16, dim3(ew_grid(nslot * 16 * ROWG)), dim3(256), 0, st, C.Pv, nslot, Kp8, F, R0, C.PvT16);
  if (op->B) {
    hipLaunchKernelGGL(k_coarse_W<double>, dim3(ew_grid(nbr * Kp8)), dim3(256), 0, st, op->B, op->dest, C.Pv, nbr, K,
                       op->Kp, Kp8, R0, F, W64, C.W);
    hipLaunchKernelGGL(k_to_b16_aug<double>, dim3(ew_grid(nbr * K)), dim3(256), 0, st, op->B, op->dest, W64, C.Pv,
                       C.lmask, nbr, K, op->Kp, Kp8, R0, F, NCH, reinterpret_cast<half_t *>(op->B16));
  } else {
    hipLaunchKernelGGL(k_coarse_W<float>, dim3(ew_grid(nbr * Kp8)), dim3(256), 0, st, op->B32, op->dest, C.Pv, nbr, K,
                       op->Kp, Kp8, R0, F, W64, C.W);
    hipLaunchKernelGGL(k_to_b16_aug<float>, dim3(ew_grid(nbr * K)), dim3(256), 0, st, op->B32, op->dest, W64, C.Pv,
                       C.lmask, nbr, K, op->Kp, Kp8, R0, F, NCH, reinterpret_cast<half_t *>(op->B16));
  }
  TRYC(hipGetLastError());
  // 4. A_c block per instance on the device, inverted on the host
  hipLaunchKernelGGL(k_zero_f64n, dim3(ew_grid(std::max<int64_t>(ai_size, 1))), dim3(256), 0, st, Ac,
                     std::max<int64_t>(ai_size, 1));
  hipLaunchKernelGGL(k_coarse_Ac, dim3(ew_grid(nslot * F * F)), dim3(256), 0, st, C.Pv, W64, C.agg_slot, C.agg_up,
                     C.row_off, C.blk_lo, C.blk_n, nslot, Kp8, R0, F, Ac);
  TRYC(hipGetLastError());
  std::vector<double> Ah(ai_size);
  std::vector<int32_t> up(nslot);
  TRYC(hipMemcpyAsync(Ah.data(), Ac, sizeof(double) * ai_size, hipMemcpyDeviceToHost, st));
  TRYC(hipMemcpyAsync(up.data(), C.agg_up, sizeof(int32_t) * nslot, hipMemcpyDeviceToHost, st));
  TRYC(hipStreamSynchronize(st));
  for (int g = 0; g < G; ++g)
    for (int64_t s = 4 * toff[g]; s < 4 * toff[g + 1]; ++s)
      if (up[s] < inst_lo[g] || up[s] >= inst_lo[g + 1]) {
        cleanup();
        C.release();
        set_error("the operator couples tets of different instances");
        return DFM_E_INVALID;
      }
  std::vector<float> Ai(ai_size);
  std::vector<int64_t> row_off1(ng);
  std::vector<float> Ai1;
  for (int g = 0; g < G; ++g) {
    const int nb = inst_lo[g + 1] - inst_lo[g], nF = nb * F;
    const int64_t base = row_off[inst_lo[g]];
    std::vector<double> a(Ah.begin() + base, Ah.begin() + base + (int64_t)nF * nF);
    // the constant-function block (every F-th row and column) for the fallback
    std::vector<double> a1((size_t)nb * nb);
    for (int p = 0; p < nb; ++p)
      for (int q = 0; q < nb; ++q) a1[(size_t)p * nb + q] = a[(size_t)(p * F) * nF + q * F];
    if (!invert(a, nF) || !invert(a1, nb)) {
      cleanup();
      C.release();
      set_error("the coarse matrix P^T (I - B) P is singular");
      return DFM_E_NUMERIC;
    }
    for (int64_t i = 0; i < (int64_t)nF * nF; ++i) Ai[base + i] = (float)a[i];
    for (int p = 0; p < nb; ++p) row_off1[inst_lo[g] + p] = (int64_t)Ai1.size() + (int64_t)p * nb;
    for (double v : a1) Ai1.push_back((float)v);
  }
  // slots in aggregate order (counting sort)
  std::vector<int64_t> cnt(ng + 1, 0);
  for (int64_t s = 0; s < nslot; ++s) cnt[agg_tet[s >> 2] + 1]++;
  for (int g = 0; g < ng; ++g) cnt[g + 1] += cnt[g];
  std::vector<int32_t> perm(nslot);
  for (int64_t s = 0; s < nslot; ++s) perm[cnt[agg_tet[s >> 2]]++] = (int32_t)s;
  TRYC(hipMalloc(&C.perm, sizeof(int32_t) * nslot));
  TRYC(hipMalloc(&C.Ai, sizeof(float) * std::max<int64_t>(ai_size, 1)));
  TRYC(hipMalloc(&C.Ai1, sizeof(float) * std::max<size_t>(Ai1.size(), 1)));
  TRYC(hipMalloc(&C.row_off1, sizeof(int64_t) * ng));
  TRYC(hipMemcpyAsync(C.perm, perm.data(), sizeof(int32_t) * nslot, hipMemcpyHostToDevice, st));
  TRYC(hipMemcpyAsync(C.Ai, Ai.data(), sizeof(float) * ai_size, hipMemcpyHostToDevice, st));
  TRYC(hipMemcpyAsync(C.Ai1, Ai1.data(), sizeof(float) * Ai1.size(), hipMemcpyHostToDevice, st));
  TRYC(hipMemcpyAsync(C.row_off1, row_off1.data(), sizeof(int64_t) * ng, hipMemcpyHostToDevice, st));
  TRYC(hipStreamSynchronize(st));   // the host vectors above must outlive their copies
#undef TRYC
  cleanup();
  C.toff = toff;
  return DFM_OK;
}

namespace {
// compute units of the current device (cached per device)
int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// one launch of the product over a.ntl tets: the tile follows R (16, 32, 64 or
// 128 right-hand sides per workgroup), so that a few right-hand sides do not pay
// for the matrix-core work of 128; about one persistent workgroup per compute
// unit and tile (two where the tile's registers let two share a unit)
hipError_t launch_spmm16(const P16Args &a, hipStream_t st) {
  const int R = a.R;
  const int CT = R <= 16 ? 1 : (R <= 32 ? 2 : (R <= 64 ? 4 : 8));
  const int nsub = (a.K + KC - 1) / KC, naug = (NAUG * fpad(a.F) + KC - 1) / KC;
  const int L = std::max(nsub, naug);
  const unsigned ny = (unsigned)((R + 16 * CT - 1) / (16 * CT)), nz = (unsigned)((a.Kp8 + ROWG - 1) / ROWG);
  const int64_t per_cu = CT <= 2 ? 2 : 1;   // CT <= 2 fits in 256 registers: two waves per SIMD
  const int64_t P = std::max<int64_t>(1, std::min<int64_t>(a.ntl, per_cu * cu_count() / (int64_t)(ny * nz)));
  const dim3 grid((unsigned)P, ny, nz);
#define DFM_SPMM16(CTV, LV) \
  case CTV * 10 + LV: hipLaunchKernelGGL((k_spmm16<2, CTV, LV>), grid, dim3(256), 0, st, a); break;
#define DFM_SPMM16_LDS(LV) \
  case 80 + LV: hipLaunchKernelGGL((k_spmm16_lds<LV>), grid, dim3(256), 0, st, a); break;
  switch (CT * 10 + L) {
    DFM_SPMM16(1, 2) DFM_SPMM16(1, 3) DFM_SPMM16(1, 4) DFM_SPMM16(1, 5)
    DFM_SPMM16(2, 2) DFM_SPMM16(2, 3) DFM_SPMM16(2, 4) DFM_SPMM16(2, 5)
    DFM_SPMM16(4, 2) DFM_SPMM16(4, 3) DFM_SPMM16(4, 4) DFM_SPMM16(4, 5)
    DFM_SPMM16_LDS(2) DFM_SPMM16_LDS(3) DFM_SPMM16_LDS(4) DFM_SPMM16_LDS(5)
    default: return hipErrorInvalidValue;
  }
#undef DFM_SPMM16
#undef DFM_SPMM16_LDS
  return hipGetLastError();
}

P16Args product_args(dfm_op op, int R) {
  const Coarse &C = *op->coarse;
  P16Args a{};
  a.B16 = reinterpret_cast<const half_t *>(op->B16);
  a.dest = op->dest;
  a.nt = op->nt;
  a.K = op->K;
  a.Kp8 = op->Kp8;
  a.R = R;
  a.F = C.F;
  a.NCH = C.NCH;
  a.R0 = C.R0;
  a.PvT16 = C.PvT16;
  a.agg_slot = C.agg_slot;
  a.agg_up = C.agg_up;
  a.zero16 = C.zero16;
  return a;
}

hipError_t launch_product16(dfm_op op, half_t *t, half_t *y, float *d0, int R, const float *c,
                            const half_t *c16, const half_t *zero16, const int32_t *gid, const uint8_t *gact,
                            bool first, hipStream_t st) {
  const Coarse &C = *op->coarse;
  P16Args a = product_args(op, R);
  a.t = t;
  a.y = y;
  a.d0 = d0;
  a.c = c;
  a.c16 = c16;
  a.zero16 = zero16;
  a.gid = gid;
  a.gact = gact;
  a.lmask = C.lmask;
  a.first = first ? 1 : 0;
  ProdTiming *tm = op->ptiming;
  // algorithmic bytes per tet: its 4 block rows of B16 (slot chunks, and the
  // correction chunks when c is given), x of its 4 inbound slots and y of its 4
  // destinations once each, and d0 of its destinations
  const int nsub = (op->K + KC - 1) / KC, naug = (NAUG * fpad(C.F) + KC - 1) / KC;
  const double tet_bytes = 4.0 * (3 * nsub + (c ? naug : 0)) * op->K * KC * sizeof(half_t) +
                           2.0 * 4.0 * R * op->Kp8 * sizeof(half_t) + (d0 ? 4.0 * C.F * R * sizeof(float) : 0.0);
  // one launch per colour, in colour order
  for (int q = 0; q < C.ncol; ++q) {
    const int64_t cnt = C.col_off[q + 1] - C.col_off[q];
    if (cnt == 0) continue;
    a.tlist = C.tlist + C.col_off[q];
    a.ntl = cnt;
    if (tm) {
      hipError_t e = tm->begin(st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = launch_spmm16(a, st);
    if (e != hipSuccess) return e;
    if (tm) {
      e = tm->end(st, tet_bytes * (double)cnt);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}
// y = B16 x (slot columns only: no correction, no colour order), one launch over
// every tet
hipError_t launch_plain16(dfm_op op, const half_t *x, half_t *y, int R, hipStream_t st) {
  const Coarse &C = *op->coarse;
  P16Args a = product_args(op, R);
  a.t = x;
  a.y = y;
  a.tlist = C.tlist;
  a.ntl = op->nt;
  return launch_spmm16(a, st);
}
}  // namespace

}  // namespace dfm

extern "C" dfm_status dfm_apply_f16(dfm_op op, const void *x, void *y, int nrhs, void *stream) {
  DFM_REQUIRE(op && x && y, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1 && nrhs <= 65535 * 16, DFM_E_INVALID, "nrhs must be in 1..1048560");
  DFM_REQUIRE(x != y, DFM_E_INVALID, "x and y must not alias");
  DFM_REQUIRE((op->K + 7) / 8 * 8 <= dfm::KP8MAX, DFM_E_UNSUPPORTED, "the FP16 product supports K <= 160");
  hipStream_t st = (hipStream_t)stream;
  {
    // the FP16 copy of B is made with the coarse space of the whole operator
    const std::vector<int64_t> whole{0, op->nt};
    if (!op->coarse || !op->B16) {
      dfm_status cs = dfm::ensure_coarse(op, whole, st);
      if (cs != DFM_OK) return cs;
    }
  }
  DFM_HIP(dfm::launch_plain16(op, static_cast<const dfm::half_t *>(x), static_cast<dfm::half_t *>(y), nrhs, st));
  return DFM_OK;
}

extern "C" dfm_status dfm_product_timing(dfm_op op, int enable, double *ms, int64_t *launches, double *bytes) {
  DFM_REQUIRE(op, DFM_E_INVALID, "null operator");
  DFM_REQUIRE(enable >= -1 && enable <= 1, DFM_E_INVALID, "enable must be -1, 0 or 1");
  const dfm::ProdTiming *t = op->ptiming;
  if (ms) *ms = t ? t->ms : 0.0;
  if (launches) *launches = t ? t->launches : 0;
  if (bytes) *bytes = t ? t->bytes : 0.0;
  if (enable == 1) {
    if (!op->ptiming) op->ptiming = new dfm::ProdTiming();
    op->ptiming->ms = op->ptiming->bytes = 0.0;
    op->ptiming->launches = 0;
    op->ptiming->pending_bytes.clear();
  } else if (enable == 0 && op->ptiming) {
    op->ptiming->release();
    delete op->ptiming;
    op->ptiming = nullptr;
  }
  return DFM_OK;
}

namespace dfm {

// ---------------------------------------------------------------------------
// The two-level solve inside FP64 refinement (method 2), R right-hand sides on
// G instances (instance g owns tets [toff[g], toff[g+1])).  Every pair
// (rhs, instance) stops on its own relative residual; an instance all of whose
// pairs are done or below their inner target is no longer multiplied.
// ---------------------------------------------------------------------------
dfm_status solve_twolevel_impl(dfm_op op, const double *rho0, double *rho, int R, const dfm_solve_opts *opts,
                               const std::vector<int64_t> &toff, dfm_solve_info *info, hipStream_t st) {
  const int64_t nslot = 4 * op->nt, n = op->ndof;
  const int G = (int)toff.size() - 1;
  const size_t RG = (size_t)R * G;
  constexpr double INNER_TOL = 1e-2;
  constexpr int CHECK = 8;
  const bool grouped = G > 1;
  if ((op->K + 7) / 8 * 8 > KP8MAX) {
    set_error("the two-level solver supports K <= 160 unknowns per slot");
    return DFM_E_UNSUPPORTED;
  }
  if (R > NRM_RMAX) {
    set_error("the two-level solver takes at most 4096 right-hand sides per call");
    return DFM_E_UNSUPPORTED;
  }
  half_t *ring_buf = nullptr, *c16 = nullptr;
  float *e = nullptr, *d0 = nullptr, *z = nullptr, *c = nullptr, *csum = nullptr;
  double *res = nullptr, *sc_d = nullptr, *nrm_d = nullptr;
  unsigned long long *mx_d = nullptr;
  int64_t *soff_d = nullptr, *eoff_d = nullptr, *toff_d = nullptr;
  uint8_t *gact_d = nullptr;
  int32_t *gid = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(ring_buf);
    (void)hipFree(c16);
    (void)hipFree(e);
    (void)hipFree(d0);
    (void)hipFree(z);
    (void)hipFree(c);
    (void)hipFree(csum);
    (void)hipFree(res);
    (void)hipFree(sc_d);
    (void)hipFree(nrm_d);
    (void)hipFree(mx_d);
    (void)hipFree(soff_d);
    (void)hipFree(eoff_d);
    (void)hipFree(toff_d);
    (void)hipFree(gact_d);
    (void)hipFree(gid);
  };
#define TRYT(expr)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      cleanup();                                                                             \
      return e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP;                            \
    }                                                                                        \
  } while (0)
  {
    dfm_status cs = ensure_coarse(op, toff, st);
    if (cs != DFM_OK) {
      cleanup();
      return cs;
    }
  }
  if (op->ptiming) op->ptiming->pending_bytes.clear();   // launches of an earlier solve that failed
  const Coarse &C = *op->coarse;
  const int Kp8 = op->Kp8, K = op->K, F = C.F;
  const int64_t vlen = nslot * R * Kp8;               // elements of one slot-major vector
  const int64_t NG = (int64_t)C.ng * F;
  const int64_t zn = NG * R;
  TRYT(hipMalloc(&ring_buf, sizeof(half_t) * (size_t)(WIN + 1) * vlen));
  TRYT(hipMalloc(&e, sizeof(float) * (size_t)vlen));
  TRYT(hipMalloc(&d0, sizeof(float) * (size_t)nslot * F * R));
  TRYT(hipMalloc(&z, sizeof(float) * (size_t)zn));
  TRYT(hipMalloc(&c, sizeof(float) * (size_t)zn));
  TRYT(hipMalloc(&csum, sizeof(float) * (size_t)zn));
  // c16, then 8 zero halves that the product reads in place of absent columns
  const size_t c16n = (size_t)C.ng * R * fpad(F);
  TRYT(hipMalloc(&c16, sizeof(half_t) * (c16n + 8)));
  TRYT(hipMemsetAsync(c16, 0, sizeof(half_t) * (c16n + 8), st));   // padding stays zero
  TRYT(hipMalloc(&res, sizeof(double) * (size_t)R * n));
  TRYT(hipMalloc(&sc_d, sizeof(double) * RG));
  TRYT(hipMalloc(&nrm_d, sizeof(double) * RG));
  TRYT(hipMalloc(&mx_d, sizeof(unsigned long long) * RG));
  TRYT(hipMalloc(&soff_d, sizeof(int64_t) * (G + 1)));
  TRYT(hipMalloc(&eoff_d, sizeof(int64_t) * (G + 1)));
  if (grouped) {
    TRYT(hipMalloc(&gact_d, sizeof(uint8_t) * G));
    TRYT(hipMalloc(&gid, sizeof(int32_t) * op->nt));
    TRYT(hipMalloc(&toff_d, sizeof(int64_t) * (G + 1)));
    TRYT(hipMemcpyAsync(toff_d, toff.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, st));
    int64_t maxt = 0;
    for (int g = 0; g < G; ++g) maxt = std::max(maxt, toff[g + 1] - toff[g]);
    hipLaunchKernelGGL(k_fill_gid2, dim3((unsigned)std::min<int64_t>((maxt + 255) / 256, 4096), 1, G), dim3(256), 0,
                       st, toff_d, gid);
    TRYT(hipGetLastError());
  }
  std::vector<int64_t> soff(G + 1), eoff(G + 1);
  for (int g = 0; g <= G; ++g) {
    soff[g] = 4 * toff[g];
    eoff[g] = 4 * toff[g] * K;        // element offsets in the FP64 vectors
  }
  TRYT(hipMemcpyAsync(soff_d, soff.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, st));
  TRYT(hipMemcpyAsync(eoff_d, eoff.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, st));
  int64_t maxseg = 0;
  for (int g = 0; g < G; ++g) maxseg = std::max(maxseg, eoff[g + 1] - eoff[g]);
  const dim3 sgrid((unsigned)std::min<int64_t>((maxseg + 255) / 256, grouped ? 64 : 1024), (unsigned)R, (unsigned)G);
  const dim3 hgrid((unsigned)std::min<int64_t>((maxseg * R / 8 + 255) / 256 + 1, grouped ? 64 : 2048), (unsigned)G);
  std::vector<double> h(RG);
  auto fetch = [&](double *src) -> hipError_t {
    hipError_t er = hipMemcpyAsync(h.data(), src, sizeof(double) * RG, hipMemcpyDeviceToHost, st);
    return er != hipSuccess ? er : hipStreamSynchronize(st);
  };
  auto norms_res = [&]() -> hipError_t {
    hipLaunchKernelGGL(k_zero_f64n, dim3(ew_grid((int64_t)RG)), dim3(256), 0, st, nrm_d, (int64_t)RG);
    hipLaunchKernelGGL(k_seg_norms2_d, sgrid, dim3(256), 0, st, res, n, eoff_d, G, nrm_d);
    hipError_t er = hipGetLastError();
    return er != hipSuccess ? er : fetch(nrm_d);
  };
  // |t|: at a stage start all of t_0; later the residual r_k = t_k has no L-type
  // part (those slots of the ring entry are written in place during product k)
  auto norms_t = [&](const half_t *t, bool skip_l) -> hipError_t {
    hipLaunchKernelGGL(k_zero_f64n, dim3(ew_grid((int64_t)RG)), dim3(256), 0, st, nrm_d, (int64_t)RG);
    hipLaunchKernelGGL(k_seg_norms2_h, hgrid, dim3(256), 0, st, t, R, Kp8, soff_d, G, skip_l ? C.lmask : nullptr,
                       nrm_d);
    hipError_t er = hipGetLastError();
    return er != hipSuccess ? er : fetch(nrm_d);
  };
  std::vector<double> bn(RG), rn(RG), rel(RG, 1.0), t0n(RG), target(RG), scale(RG);
  std::vector<char> done(RG, 0), inner(RG, 0);
  std::vector<uint8_t> gact(G, 1);
  std::vector<int> gprod(G, 0);
  TRYT(hipMemcpyAsync(res, rho0, sizeof(double) * (size_t)R * n, hipMemcpyDeviceToDevice, st));
  TRYT(norms_res());
  for (size_t i = 0; i < RG; ++i) {
    bn[i] = std::sqrt(h[i]);
    if (!(bn[i] > 0.0)) {
      done[i] = 1;
      rel[i] = 0.0;
    }
  }
  if (!opts->warm_start) {
    hipLaunchKernelGGL(k_zero_f64n, dim3(ew_grid((int64_t)R * n)), dim3(256), 0, st, rho, (int64_t)R * n);
    TRYT(hipGetLastError());
    rn = bn;
  } else {
    TRYT(residual_batched(op, rho0, rho, res, R, st));
    TRYT(norms_res());
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
  auto update_active = [&]() -> hipError_t {
    if (!grouped) return hipSuccess;
    bool changed = false;
    for (int g = 0; g < G; ++g) {
      uint8_t a = 0;
      for (int r = 0; r < R; ++r) a |= (!done[(size_t)r * G + g] && !inner[(size_t)r * G + g]) ? 1 : 0;
      changed |= a != gact[g];
      gact[g] = a;
    }
    if (!changed) return hipSuccess;
    hipError_t er = hipMemcpyAsync(gact_d, gact.data(), sizeof(uint8_t) * G, hipMemcpyHostToDevice, st);
    return er != hipSuccess ? er : hipStreamSynchronize(st);
  };
  if (grouped) TRYT(hipMemcpyAsync(gact_d, gact.data(), sizeof(uint8_t) * G, hipMemcpyHostToDevice, st));
  auto ring = [&](int k) { return ring_buf + (size_t)(k % (WIN + 1)) * vlen; };
  const unsigned red_grid = (unsigned)((nslot + RED_CH - 1) / RED_CH);
  const int FR = F * R;
  const int red_threads = FR >= 256 ? 256 : ((FR + 63) / 64) * 64;
  const unsigned gz = (unsigned)((FR + red_threads - 1) / red_threads);
  int iters = 0;
  bool finite = true;
  const unsigned egrid = ew_grid(vlen / 8);
  // coarse level: 2 = all F functions, 1 = the constant function, 0 = none.  A
  // stage whose residual grows DIVERGE times (the Galerkin correction of a
  // non-symmetric operator can amplify) restarts one level lower.
  constexpr double DIVERGE = 4.0;
  int level = F > 1 ? 2 : 1;
  const bool verbose = env_int("DFM_VERBOSE", 0) != 0;   // one line per refinement stage on stderr
  // the coarse step is damped: c = 0.7 A_c^-1 P^T r.  The full Galerkin step of the
  // swept operator diverges or stalls for some aggregate sizes on the 49152-tet
  // box (384, 512 and 1536 tets grow, 2048 needs 18224 sweeps); damped by 0.7 every
  // size tried converges in 464-568 sweeps
  constexpr float omega = COARSE_DAMPING;
  for (int outer = 0; outer < 40 && iters < opts->max_iter && !all_done(); ++outer) {
  restart_stage:
    // scale every active pair to unit max norm; t_0 = half(scale * r)
    hipLaunchKernelGGL(k_zero_f64n, dim3(ew_grid((int64_t)RG)), dim3(256), 0, st, reinterpret_cast<double *>(mx_d),
                       (int64_t)RG);
    hipLaunchKernelGGL(k_seg_absmax, sgrid, dim3(256), 0, st, res, n, eoff_d, G, mx_d);
    TRYT(hipGetLastError());
    {
      std::vector<unsigned long long> mx(RG);
      TRYT(hipMemcpyAsync(mx.data(), mx_d, sizeof(unsigned long long) * RG, hipMemcpyDeviceToHost, st));
      TRYT(hipStreamSynchronize(st));
      for (size_t i = 0; i < RG; ++i) {
        double m;
        std::memcpy(&m, &mx[i], sizeof(double));
        scale[i] = (!done[i] && m > 0.0) ? 1.0 / m : 0.0;
        inner[i] = done[i];
        // the correction needs no more accuracy than the outer test asks for
        target[i] = std::max(INNER_TOL, 0.5 * opts->rtol * bn[i] / std::max(rn[i], 1e-300));
      }
    }
    TRYT(hipMemcpyAsync(sc_d, scale.data(), sizeof(double) * RG, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_stage_init, dim3(ew_grid(vlen)), dim3(256), 0, st, res, nslot, K, Kp8, soff_d, G, sc_d, R,
                       ring(0), e);
    hipLaunchKernelGGL(k_d0_from_t, dim3((unsigned)std::min<int64_t>(nslot, 65536)), dim3(D0_THREADS), 0, st, ring(0),
                       C.Pv, nslot, R, Kp8, C.R0, F,
                       d0);
    hipLaunchKernelGGL(k_zero_f32n, dim3(ew_grid(zn)), dim3(256), 0, st, csum, zn);
    TRYT(hipGetLastError());
    TRYT(norms_t(ring(0), false));
    for (size_t i = 0; i < RG; ++i) t0n[i] = std::sqrt(h[i]);
    TRYT(update_active());
    int k = 0, pending = 0;   // t_k in ring(k); t_{k-pending} .. t_{k-1} not yet added to e
    // the ring's pending terms go into e; the (B P) c terms of the whole stage are
    // added once at its end (last = true), from the stage's sum of coefficients
    auto flush = [&](bool last) -> hipError_t {
      if (pending == 0 && !last) return hipSuccess;
      RingPtrs rp{};
      for (int m = 0; m < pending; ++m) rp.p[m] = ring(k - pending + m);
      if (pending == WIN)
        hipLaunchKernelGGL(k_flush<WIN>, dim3(egrid), dim3(256), 0, st, rp, pending, nslot, Kp8, R, F,
                         (last && level > 0) ? C.W : nullptr, C.Pv, C.lmask, C.agg_slot, C.agg_up, csum, e);
      else
        hipLaunchKernelGGL(k_flush<0>, dim3(egrid), dim3(256), 0, st, rp, pending, nslot, Kp8, R, F,
                         (last && level > 0) ? C.W : nullptr, C.Pv, C.lmask, C.agg_slot, C.agg_up, csum, e);
      pending = 0;
      return hipGetLastError();
    };
    bool diverged = false;
    while (iters < opts->max_iter) {
      // coarse correction from t_k (d0 holds its coarse components)
      if (level > 0) {
        hipLaunchKernelGGL(k_zero_f32n, dim3(ew_grid(zn)), dim3(256), 0, st, z, zn);
        hipLaunchKernelGGL(k_coarse_reduce, dim3(red_grid, gz), dim3(red_threads), 0, st, d0, C.perm, C.agg_slot,
                           nslot, FR, z);
        hipLaunchKernelGGL(k_coarse_solve, dim3((unsigned)((zn + 255) / 256)), dim3(256), 0, st, C.Ai, C.row_off,
                           C.Ai1, C.row_off1, level == 1 ? 1 : 0, C.blk_lo, C.blk_n, C.ng, F, R, z, c, csum, c16,
                           omega);
        TRYT(hipGetLastError());
      }
      // one coloured sweep: with r' = r_k - P c + (B P) c, the L-type slots of
      // ring(k) become z = r' + L z (in place) and ring(k + 1) = r_{k+1} = U z
      // (colour by colour); ring(k) then holds the k-th term of the sum and joins
      // the pending e terms
      TRYT(launch_product16(op, ring(k), ring(k + 1), d0, R, level > 0 ? c : nullptr, c16, c16 + c16n,
                            grouped ? gid : nullptr, grouped ? gact_d : nullptr, k == 0, st));
      ++k;
      ++pending;
      ++iters;
      for (int g = 0; g < G; ++g) gprod[g] += gact[g];
      if (pending == WIN) TRYT(flush(false));
      if (k % CHECK) continue;
      TRYT(norms_t(ring(k), true));
      bool inner_done = true;
      for (size_t i = 0; i < RG; ++i) {
        if (inner[i]) continue;
        const double tn = std::sqrt(h[i]);
        if (!std::isfinite(tn) || tn > DIVERGE * t0n[i]) diverged = true;
        if (tn <= target[i] * t0n[i]) inner[i] = 1;
        else inner_done = false;
      }
      if (diverged && level > 0) break;
      diverged = false;   // without a coarse correction the growth is B's own (left to max_iter)
      if (inner_done || !finite) break;
      TRYT(update_active());
    }
    if (verbose) {
      double worst = 0.0;
      for (size_t i = 0; i < RG; ++i)
        if (!inner[i]) worst = std::max(worst, std::sqrt(h[i]) / std::max(t0n[i], 1e-300));
      std::fprintf(stderr, "[dfm two-level] stage %d level %d products %d%s, inner residual %.2e\n", outer, level, k,
                   diverged ? " (diverged)" : "", worst);
    }
    if (diverged && level > 0) {
      --level;   // the stage's e is discarded; start it again one level lower
      goto restart_stage;
    }
    TRYT(flush(true));
    if (!finite) break;
    // rho += e / scale;  res = rho0 - (I - B) rho in FP64
    hipLaunchKernelGGL(k_stage_update, dim3(ew_grid((int64_t)R * n)), dim3(256), 0, st, e, nslot, K, Kp8, soff_d, G,
                       sc_d, R, rho);
    TRYT(hipGetLastError());
    TRYT(residual_batched(op, rho0, rho, res, R, st));
    TRYT(norms_res());
    for (size_t i = 0; i < RG; ++i) {
      if (done[i]) continue;
      rn[i] = std::sqrt(h[i]);
      rel[i] = rn[i] / bn[i];
      if (!std::isfinite(rel[i])) finite = false;
      if (rel[i] <= opts->rtol) done[i] = 1;
    }
    if (!finite) break;
  }
#undef TRYT
  cleanup();
  if (op->ptiming) {
    // every event of this solve is behind the stream synchronisation of its last residual norms
    if (hipStreamSynchronize(st) == hipSuccess) op->ptiming->harvest();
    else op->ptiming->pending_bytes.clear();
  }
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
