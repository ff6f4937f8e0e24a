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

// The streaming products keep the plain workgroup order (workgroup w runs on XCD
// w % 8).  Giving each XCD a contiguous range of tiles lets the two halves of a
// split block row share one L2 (1 % fewer bytes fetched), but an instance whose
// rows are masked off then exits on one XCD while the others keep working: the
// batched solve of uneven instances became up to 21 % slower per group.

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

// A few right-hand sides at once from one stream of the FP32 operator: as k_spmv,
// but each thread keeps NR accumulators and the running Neumann sum is updated in
// the same pass: y[r] = B32 x[r], e[r] += y[r] (x, y, e f32 [NR][ndof] at stride
// ndof).  The x panels of the workgroup's block rows are staged in LDS one inbound
// face s at a time (NR x rows x K floats), which keeps the LDS per workgroup small
// enough for several workgroups per CU to have their loads of B in flight.
template <int NR>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_rhs(const float *__restrict__ B, const int32_t *__restrict__ dest,
                                                          int64_t nthreads, int K, int Kp, int64_t ndof,
                                                          const float *__restrict__ x, float *__restrict__ y,
                                                          float *__restrict__ e, const int32_t *__restrict__ gid,
                                                          const uint8_t *__restrict__ gact) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  extern __shared__ float xs_rhs[];
  const int GPB = Kp / 4;
  const int64_t g0 = blockIdx.x * (int64_t)SPMV_THREADS;
  const int64_t br0 = g0 / GPB;
  int64_t glast = g0 + SPMV_THREADS - 1;
  if (glast >= nthreads) glast = nthreads - 1;
  const int nrows_b = (int)(glast / GPB - br0 + 1);
  const int per_rhs = nrows_b * K;
  const int64_t g = g0 + threadIdx.x;
  const bool inrange = g < nthreads;
  const int64_t br = inrange ? g / GPB : br0;
  // rows of an instance that is not being multiplied (gact[gid[tet]] == 0) get y = 0
  const bool active = inrange && (gact == nullptr || gact[gid[br >> 2]] != 0);
  const int row0 = (int)(g - br * GPB) * 4;
  const float *xp = xs_rhs + (br - br0) * K;
  const f4 *Bv = reinterpret_cast<const f4 *>(B + br * 3 * (int64_t)K * Kp + row0);
  const int cstride = Kp / 4;
  double acc[NR][4];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[r][u] = 0.0;
  for (int s = 0; s < 3; ++s) {
    if (s) __syncthreads();  // every thread is done with the previous face's panel
    for (int i = threadIdx.x; i < NR * per_rhs; i += SPMV_THREADS) {
      const int r = i / per_rhs, q = i - r * per_rhs;
      const int b = q / K, col = q - b * K;
      const int64_t bb = br0 + b;
      xs_rhs[i] = x[r * ndof + (4 * (bb >> 2) + in_face((int)(bb & 3), s)) * (int64_t)K + col];
    }
    __syncthreads();
    if (active) {
      const f4 *Bs = Bv + (int64_t)s * K * cstride;
#pragma unroll 4
      for (int c = 0; c < K; ++c) {
        const f4 bv = __builtin_nontemporal_load(Bs + (int64_t)c * cstride);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double xc = xp[r * per_rhs + c];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[r][u] = fma((double)bv[u], xc, acc[r][u]);
        }
      }
    }
  }
  if (!inrange) return;
  const int64_t ob = (int64_t)dest[br] * K;
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = row0 + u;
      if (row < K) {
        const float v = (float)acc[r][u];
        y[r * ndof + ob + row] = v;
        if (e && active) e[r * ndof + ob + row] += v;
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
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// Transposed product (adjoint solve):
//   y[4j + l_in][col] = alpha v + beta sum_{l_out != l_in} sum_row
//                       B[4j + l_out, s(l_in)][col][row] x[dest(4j + l_out)][row].
// One workgroup per tet: the four destination panels x[dest(4j + l_out)] are
// staged in LDS; every output (l_in, col) belongs to one wave, which reads the
// three contributing block columns (K contiguous doubles each, 16-byte aligned
// since Kp is a multiple of 4) with coalesced 16-byte loads and reduces across
// the wave, so B is read once, in order.
constexpr int SPMVT_THREADS = 256;
template <typename TB, typename TX>
__global__ __launch_bounds__(SPMVT_THREADS) void k_spmv_t(const TB *__restrict__ B, const int32_t *__restrict__ dest,
                                                         int K, int Kp, const TX *__restrict__ x,
                                                         const TX *__restrict__ v, TX *__restrict__ y, double alpha,
                                                         double beta) {
  constexpr int VW = Vec<TB>::W;   // rows per 16-byte load
  typedef typename Vec<TB>::T VT;
  extern __shared__ double xd[];  // [4][K]
  const int64_t j = blockIdx.x;
  for (int i = threadIdx.x; i < 4 * K; i += SPMVT_THREADS) {
    const int l = i / K, row = i - l * K;
    xd[i] = (double)x[(int64_t)dest[4 * j + l] * K + row];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t KKp = (int64_t)K * Kp;
  // lanes per output: the power of two that covers a column in 16-byte loads, so
  // a wave reduces 64 / lpo outputs at once (one for long FP64 columns)
  int lpo = 1;
  while (lpo < 64 && lpo * VW < K) lpo <<= 1;
  const int opw = 64 / lpo, sub = lane / lpo, li = lane - sub * lpo;
  const int nout = 4 * K;
  for (int o0 = wave * opw; o0 < nout; o0 += (SPMVT_THREADS / 64) * opw) {
    const int o = o0 + sub;
    const bool live = o < nout;
    const int l_in = live ? o / K : 0, col = live ? o - l_in * K : 0;
    double acc = 0.0;
    if (live) {
#pragma unroll
      for (int l_out = 0; l_out < 4; ++l_out) {
        if (l_out == l_in) continue;
        const int s = l_in < l_out ? l_in : l_in - 1;
        const VT *Bc = reinterpret_cast<const VT *>(B + ((4 * j + l_out) * 3 + s) * KKp + (int64_t)col * Kp);
        const double *xs = xd + l_out * K;
        for (int rv = li; VW * rv < K; rv += lpo) {
          const VT b = __builtin_nontemporal_load(Bc + rv);   // rows VW rv .. VW rv + VW - 1 (< Kp)
#pragma unroll
          for (int u = 0; u < VW; ++u)
            if (VW * rv + u < K) acc = fma((double)b[u], xs[VW * rv + u], acc);
        }
      }
    }
    for (int off = lpo >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (live && li == 0) {
      const int64_t g = (4 * j + l_in) * (int64_t)K + col;
      double r = beta * acc;
      if (v) r = fma(alpha, (double)v[g], r);
      y[g] = (TX)r;
    }
  }
}

// Batched product for R right-hand sides on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32): for every block row br = (j, l_out) and rhs r,
//   y[r][dest(br)][row] = sum_{s, col} B32[br, s][col][row] x[r][4j + l_in(s)][col],
// and, when e != null, e[r][dest(br)][row] += that value.  Vectors are f32
// [R][ndof].  Workgroup = (block row, tile of SPMM_RT right-hand sides, group of
// SPMM_ROWS output rows); its 8 waves form 2 row halves (3 row tiles of 16) x 4
// rhs quarters (2 rhs tiles of 16).  The contraction runs over the 3K columns of
// the block row in chunks of SPMM_KC: the chunk of B (rows x columns) and of x
// (rhs x columns) is loaded coalesced into registers one chunk ahead, stored to
// LDS and read back as MFMA fragments.  The result tile goes through LDS so that
// each rhs's output rows are written as one contiguous segment.
constexpr int SPMM_THREADS = 512;
constexpr int SPMM_RT = 128;                  // right-hand sides per workgroup
constexpr int SPMM_ROWS = 96;                 // output rows per workgroup
constexpr int SPMM_KC = 32;                   // contraction chunk (columns)
#ifndef DFM_SPMM_BPAD
#define DFM_SPMM_BPAD 16
#endif
#ifndef DFM_SPMM_XPAD
#define DFM_SPMM_XPAD 4
#endif
#ifndef DFM_SPMM_XT
#define DFM_SPMM_XT 1
#endif
constexpr int SPMM_BLD = SPMM_ROWS + DFM_SPMM_BPAD;   // LDS row stride of the B chunk [col][row]
constexpr int SPMM_XLD = SPMM_RT + DFM_SPMM_XPAD;     // LDS row stride of the x chunk [col][rhs]
// x chunk stored [rhs][col] with row stride SPMM_XLDT instead: the coalesced loads
// (lanes along columns) store to consecutive banks, and the MFMA fragment reads
// (lanes along rhs, 2 columns per half-wave) hit 2 rhs + column, all distinct
constexpr bool SPMM_XT = DFM_SPMM_XT != 0;
constexpr int SPMM_XLDT = 34;
constexpr int SPMM_YLD = SPMM_ROWS + 1;       // LDS row stride of the result [rhs][row]
constexpr int SPMM_NX = SPMM_KC * SPMM_RT / SPMM_THREADS;     // x chunk values per thread
constexpr int SPMM_LDS_CHUNK = SPMM_KC * SPMM_BLD + (SPMM_XT ? SPMM_RT * SPMM_XLDT : SPMM_KC * SPMM_XLD),
              SPMM_LDS_OUT = SPMM_RT * SPMM_YLD;
constexpr size_t SPMM_LDS = sizeof(float) * (size_t)(SPMM_LDS_CHUNK > SPMM_LDS_OUT ? SPMM_LDS_CHUNK : SPMM_LDS_OUT);
constexpr int SPMM_EPT = (SPMM_RT * SPMM_ROWS + SPMM_THREADS - 1) / SPMM_THREADS;  // output values per thread
static_assert(SPMM_ROWS % 4 == 0 && SPMM_BLD % 4 == 0 && SPMM_NX * SPMM_THREADS == SPMM_KC * SPMM_RT, "");

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(SPMM_THREADS, 4) void k_spmm32(const float *__restrict__ B,
                                                           const int32_t *__restrict__ dest, int64_t nt, int K, int Kp,
                                                           int64_t ndof, int R, const float *__restrict__ x,
                                                           float *__restrict__ y, float *__restrict__ e,
                                                           const int32_t *__restrict__ gid,
                                                           const uint8_t *__restrict__ gact) {
  extern __shared__ float lds[];
  float *bs = lds;                              // [SPMM_KC][SPMM_BLD]
  float *xs = lds + SPMM_KC * SPMM_BLD;         // [SPMM_RT][SPMM_XLDT] (or [SPMM_KC][SPMM_XLD])
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // workgroups are dealt to the 8 XCDs in turn (blockIdx.x % 8): the four block
  // rows of a tet go to one XCD back to back, so the x panels they share (each
  // source slot feeds three of them) are read from HBM once and then from its L2
  const int64_t bid = blockIdx.x;
  int64_t br = bid;
  if ((nt & 7) == 0) {
    const int64_t slot = bid >> 3, xcd = bid & 7;
    br = 4 * (8 * (slot >> 2) + xcd) + (slot & 3);
  }
  const int r0 = blockIdx.y * SPMM_RT;          // first rhs of the tile
  const int m0 = blockIdx.z * SPMM_ROWS;        // first output row of the group
  const int64_t j = br >> 2;
  const int l_out = (int)(br & 3);
  const int ncol = 3 * K;                       // contraction length of the block row
  const int nchunk = (ncol + SPMM_KC - 1) / SPMM_KC;
  const float *Bbr = B + br * 3 * (int64_t)K * Kp;   // 3K columns of length Kp
  if (gact != nullptr && gact[gid[j]] == 0) {
    // an instance that is not being multiplied: y = 0 on its rows (the whole
    // workgroup takes this branch, before any barrier)
    const int nrows = min(SPMM_ROWS, K - m0);
    const int64_t ob = (int64_t)dest[br] * K + m0;
    for (int i = tid; i < SPMM_RT * nrows; i += SPMM_THREADS) {
      const int r = i / nrows, m = i - r * nrows;
      if (r0 + r < R) y[(int64_t)(r0 + r) * ndof + ob + m] = 0.0f;
    }
    return;
  }

  // coalesced chunk loads, offsets fixed per thread.  The B chunk moves in 16-byte
  // pieces: piece i = tid + u * SPMM_THREADS -> (column i / (SPMM_ROWS / 4), rows
  // m0 + 4 (i % (SPMM_ROWS / 4)) .. +3).  Kp, the block row's offset 3 K Kp and m0
  // are multiples of 4, so every piece is 16-byte aligned and lies wholly inside or
  // wholly outside the column's Kp rows.  x chunk value i -> (rhs i / SPMM_KC,
  // column i % SPMM_KC), the column the same for every u.
  constexpr int SPMM_B4 = SPMM_KC * SPMM_ROWS / 4;                       // pieces per chunk
  constexpr int SPMM_NB4 = (SPMM_B4 + SPMM_THREADS - 1) / SPMM_THREADS;  // pieces per thread
  int bcol[SPMM_NB4], brow[SPMM_NB4];
#pragma unroll
  for (int u = 0; u < SPMM_NB4; ++u) {
    const int i = tid + u * SPMM_THREADS;
    bcol[u] = i < SPMM_B4 ? i / (SPMM_ROWS / 4) : SPMM_KC;   // SPMM_KC: no piece
    brow[u] = m0 + 4 * (i % (SPMM_ROWS / 4));
  }
  const int xc = tid % SPMM_KC, xr = r0 + tid / SPMM_KC;   // rhs xr + u * (SPMM_THREADS / SPMM_KC)
  constexpr int XRS = SPMM_THREADS / SPMM_KC;
  v4f pb[SPMM_NB4];
  float px[SPMM_NX];
  auto load_chunk = [&](int ch) {
    const int c0 = ch * SPMM_KC;
#pragma unroll
    for (int u = 0; u < SPMM_NB4; ++u) {
      const int c = c0 + bcol[u];
      pb[u] = (bcol[u] < SPMM_KC && c < ncol && brow[u] < Kp)
                  ? __builtin_nontemporal_load(reinterpret_cast<const v4f *>(Bbr + (int64_t)c * Kp + brow[u]))
                  : v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }
    const int c = c0 + xc;
    const int s = c / K;
    const float *xp = x + (int64_t)xr * ndof + (4 * j + in_face(l_out, s < 3 ? s : 2)) * (int64_t)K + (c - s * K);
#pragma unroll
    for (int u = 0; u < SPMM_NX; ++u)
      px[u] = (c < ncol && xr + u * XRS < R) ? xp[(int64_t)u * XRS * ndof] : 0.0f;
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < SPMM_NB4; ++u)
      if (bcol[u] < SPMM_KC) *reinterpret_cast<v4f *>(bs + bcol[u] * SPMM_BLD + brow[u] - m0) = pb[u];
#pragma unroll
    for (int u = 0; u < SPMM_NX; ++u) {
      if (SPMM_XT) xs[(xr - r0 + u * XRS) * SPMM_XLDT + xc] = px[u];
      else xs[xc * SPMM_XLD + (xr - r0) + u * XRS] = px[u];
    }
  };

  const int wr = wave >> 2, wc = wave & 3;      // row half, rhs quarter
  const int col = lane & 15, kq = lane >> 4;
  v4f acc[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

  auto contract = [&]() {
#pragma unroll
    for (int ks = 0; ks < SPMM_KC / 4; ++ks) {
      const int c = ks * 4 + kq;
      float av[3], bv[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) av[a] = bs[c * SPMM_BLD + (wr * 3 + a) * 16 + col];
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bv[b] = SPMM_XT ? xs[((wc * 2 + b) * 16 + col) * SPMM_XLDT + c] : xs[c * SPMM_XLD + (wc * 2 + b) * 16 + col];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  };
  // output element k of this thread: i = tid + k * SPMM_THREADS -> (rhs i / nrows, row i % nrows)
  const int nrows = min(SPMM_ROWS, K - m0);
  const int64_t ob = (int64_t)dest[br] * K + m0;
  float epre[SPMM_EPT];

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
  if (e) {
    // last chunk: the running-sum values of the output tile load while it is
    // contracted (the chunk prefetch registers are free by now)
#pragma unroll
    for (int k = 0; k < SPMM_EPT; ++k) {
      const int i = tid + k * SPMM_THREADS;
      const int r = i / nrows, m = i - r * nrows;
      epre[k] = (i < SPMM_RT * nrows && r0 + r < R) ? e[(int64_t)(r0 + r) * ndof + ob + m] : 0.0f;
    }
  }
  contract();
  __syncthreads();
  // result tile: lane holds rows 4 (lane / 16) + q of each 16-row tile, rhs lane % 16
  float *ys = lds;                              // [SPMM_RT][SPMM_YLD]
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        ys[((wc * 2 + b) * 16 + col) * SPMM_YLD + (wr * 3 + a) * 16 + 4 * kq + q] = acc[a][b][q];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SPMM_EPT; ++k) {
    const int i = tid + k * SPMM_THREADS;
    const int r = i / nrows, m = i - r * nrows;
    if (i < SPMM_RT * nrows && r0 + r < R) {
      const float v = ys[r * SPMM_YLD + m];
      const int64_t o = (int64_t)(r0 + r) * ndof + ob + m;
      y[o] = v;
      if (e) e[o] = epre[k] + v;
    }
  }
}

}  // namespace

// FP64 vectors; the operator in FP64, or in FP32 when it was assembled in FP32
// (accumulation in FP64 either way)
hipError_t spmv(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st) {
  if (!op->B) {
    int64_t nthreads = 4 * op->nt * (int64_t)(op->Kp / Vec<float>::W);
    unsigned grid = (unsigned)((nthreads + SPMV_THREADS - 1) / SPMV_THREADS);
    hipLaunchKernelGGL((k_spmv<float, double>), dim3(grid), dim3(SPMV_THREADS), spmv_lds<float>(op->K, op->Kp), st,
                       op->B32, op->dest, nthreads, op->K, op->Kp, x, v, y, alpha, beta);
    return hipGetLastError();
  }
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

// y = B32 x (and e += y when e != null) for R right-hand sides, up to four per
// stream of the operator
hipError_t spmv32_rhs(dfm_op op, const float *x, float *y, float *e, int R, const int32_t *gid, const uint8_t *gact,
                      hipStream_t st) {
  const int64_t nthreads = 4 * op->nt * (int64_t)(op->Kp / 4);
  const unsigned grid = (unsigned)((nthreads + SPMV_THREADS - 1) / SPMV_THREADS);
  const int gpb = op->Kp / 4;
  const int64_t rows = (SPMV_THREADS + gpb - 1) / gpb + 1;
  for (int r0 = 0; r0 < R; r0 += 4) {
    const int nr = R - r0 < 4 ? R - r0 : 4;
    const size_t lds = sizeof(float) * (size_t)(nr * rows * op->K);
    const float *xr = x + (int64_t)r0 * op->ndof;
    float *yr = y + (int64_t)r0 * op->ndof;
    float *er = e ? e + (int64_t)r0 * op->ndof : nullptr;
#define DFM_RHS_CASE(NRV)                                                                                  \
  case NRV:                                                                                                \
    hipLaunchKernelGGL(k_spmv_rhs<NRV>, dim3(grid), dim3(SPMV_THREADS), lds, st, op->B32, op->dest, nthreads, \
                       op->K, op->Kp, op->ndof, xr, yr, er, gid, gact);                                    \
    break;
    switch (nr) {
      DFM_RHS_CASE(1)
      DFM_RHS_CASE(2)
      DFM_RHS_CASE(3)
      default:
        DFM_RHS_CASE(4)
    }
#undef DFM_RHS_CASE
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

// y = B32 x for R right-hand sides on the matrix cores (and e += y when e != null)
hipError_t spmm32(dfm_op op, const float *x, float *y, float *e, int R, const int32_t *gid, const uint8_t *gact,
                  hipStream_t st) {
  dim3 grid((unsigned)(4 * op->nt), (unsigned)((R + SPMM_RT - 1) / SPMM_RT),
            (unsigned)((op->K + SPMM_ROWS - 1) / SPMM_ROWS));
  hipError_t err = hipFuncSetAttribute((const void *)k_spmm32, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)SPMM_LDS);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_spmm32, grid, dim3(SPMM_THREADS), SPMM_LDS, st, op->B32, op->dest, op->nt, op->K, op->Kp,
                     op->ndof, R, x, y, e, gid, gact);
  return hipGetLastError();
}

// y = B32 x (and e += y) with the kernel suited to R: the streaming product below
// 16 right-hand sides, the matrix-core product from 16 on.  With gid/gact (tet ->
// instance, instance -> multiplied?) the rows of instances with gact = 0 get y = 0
// and leave e unchanged, without reading their blocks.
hipError_t product32(dfm_op op, const float *x, float *y, float *e, int R, const int32_t *gid, const uint8_t *gact,
                     hipStream_t st) {
  return R >= 16 ? spmm32(op, x, y, e, R, gid, gact, st) : spmv32_rhs(op, x, y, e, R, gid, gact, st);
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
  hipLaunchKernelGGL(k_to_fp32, dim3(ew_grid(nel)), dim3(256), 0, st, op->B, op->B32, nel);
  return hipGetLastError();
}

hipError_t spmv_t(dfm_op op, const double *x, const double *v, double *y, double alpha, double beta, hipStream_t st) {
  if (!op->B) return hipErrorNotSupported;   // transposed products need the FP64 operator
  hipLaunchKernelGGL((k_spmv_t<double, double>), dim3((unsigned)op->nt), dim3(SPMVT_THREADS),
                     sizeof(double) * 4 * op->K, st, op->B, op->dest, op->K, op->Kp, x, v, y, alpha, beta);
  return hipGetLastError();
}

// y = alpha v + beta B32^T x for FP32 vectors (the inner solves of transposed
// mixed-precision GMRES), FP64 accumulation
hipError_t spmv32_t(dfm_op op, const float *x, const float *v, float *y, float alpha, float beta, hipStream_t st) {
  if (!op->B32) return hipErrorNotSupported;
  hipLaunchKernelGGL((k_spmv_t<float, float>), dim3((unsigned)op->nt), dim3(SPMVT_THREADS),
                     sizeof(double) * 4 * op->K, st, op->B32, op->dest, op->K, op->Kp, x, v, y, (double)alpha,
                     (double)beta);
  return hipGetLastError();
}

}  // namespace dfm

using namespace dfm;

extern "C" dfm_status dfm_apply(dfm_op op, const double *x, double *y, int nrhs, int transpose, void *stream_) {
  DFM_REQUIRE(op && x && y, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(!(transpose && !op->B), DFM_E_UNSUPPORTED, "transposed products need an operator assembled in FP64");
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

extern "C" dfm_status dfm_apply_f32(dfm_op op, const float *x, float *y, int nrhs, void *stream_) {
  DFM_REQUIRE(op && x && y, DFM_E_INVALID, "null argument");
  DFM_REQUIRE(nrhs >= 1 && nrhs <= 65535, DFM_E_INVALID, "nrhs must be in 1..65535");
  DFM_REQUIRE(x != y, DFM_E_INVALID, "x and y must not alias");
  hipStream_t st = (hipStream_t)stream_;
  hipError_t e = ensure_fp32(op, st);
  if (e == hipErrorOutOfMemory) {
    set_error("no device memory for the FP32 copy of B");
    return DFM_E_NOMEM;
  }
  DFM_HIP(e);
  DFM_HIP(product32(op, x, y, nullptr, nrhs, nullptr, nullptr, st));
  return DFM_OK;
}

