// Internal declarations of the DFM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/dfm.h"

namespace dfm {

void set_error(const std::string &msg);

#define DFM_HIP(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      ::dfm::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                   \
      return DFM_E_HIP;                                                                      \
    }                                                                                        \
  } while (0)

#define DFM_REQUIRE(cond, code, msg)                                                         \
  do {                                                                                       \
    if (!(cond)) {                                                                           \
      ::dfm::set_error(msg);                                                                 \
      return (code);                                                                         \
    }                                                                                        \
  } while (0)

// Grid for the element-wise kernels: they loop with a grid stride, so the launch
// stays far below the 2^32 work items a dispatch can describe however long the
// array is.
inline unsigned ew_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

// Per-face geometry record, 12 doubles: area, outward unit normal (3),
// frame x (3), frame y (3), pad (2).  The frame z is minus the normal.
constexpr int FACE_REC = 12;

// Error flags raised by kernels (bit mask in a device word).
enum : unsigned {
  FLAG_NONMANIFOLD = 1u,
  FLAG_BAD_ID = 2u,
  FLAG_DEGENERATE = 4u,
  FLAG_NONUNIFORM = 8u,
  FLAG_CELL_OVERFLOW = 16u,
  FLAG_NONFINITE = 32u,
  FLAG_HASH_FULL = 64u,
};

struct Coarse;
struct ProdTiming;
void free_twolevel(dfm_op op);

}  // namespace dfm

struct dfm_mesh_s {
  int64_t nt = 0, nv = 0, n_boundary = 0;
  double *verts = nullptr;    // [nv][3]
  int32_t *tets = nullptr;    // [nt][4]
  int32_t *nbr = nullptr;     // [nt][4]
  double *refl = nullptr;     // [nt][4]
  double *face = nullptr;     // [nt][4][FACE_REC]
  double *vol = nullptr;      // [nt]
  double bbox_diag = 1.0;
};

struct dfm_op_s {
  dfm_mesh mesh = nullptr;
  dfm_basis basis{};
  int P = 1, M = 1, K = 1, Kp = 4;  // Kp: padded column length of the stored blocks
  int64_t nt = 0, ndof = 0;
  int64_t nodes = 0;
  double *B = nullptr;        // [nt][4][3K][Kp]: block (j, l_out, s) column-major, K columns of length Kp
  float *B32 = nullptr;       // same layout in FP32, made on first mixed-precision solve
  int32_t *dest = nullptr;    // [nt][4]
  double *mu = nullptr;       // [nt] the damping B was assembled with
  double *gl = nullptr;       // [2][32] Gauss-Legendre nodes and weights
  double *thom = nullptr;     // Legendre Gram tridiagonal factors
  double *coef = nullptr;     // chord-moment power series
  void *B16 = nullptr;        // FP16 copy with the coarse-correction columns (two-level solver)
  int Kp8 = 8;                // K rounded up to a multiple of 8
  dfm::Coarse *coarse = nullptr;  // aggregation coarse space of the two-level solver
  dfm::ProdTiming *ptiming = nullptr;  // event timing of the two-level product launches, when on
};
