// Mesh builder: face adjacency through a device hash of sorted vertex triples,
// per-face geometry (area, outward normal, face frame) and tet volumes.
//
// The density of the method lives on the faces of every tetrahedron and a ray
// leaving one tet through a face enters the tet on the other side (Sec. 2);
// B is block sparse because only such neighbours couple.  Faces are matched by
// their sorted global vertex ids; a triple seen once is a boundary face.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "dfm_internal.h"

namespace dfm {

namespace {

constexpr unsigned long long EMPTY = ~0ull;

__device__ inline unsigned long long mix64(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ inline void sort3(int &a, int &b, int &c) {
  int t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}

__device__ inline unsigned long long face_key(const int32_t *tet, int l) {
  int v[3];
  int n = 0;
  for (int m = 0; m < 4; ++m)
    if (m != l) v[n++] = tet[m];
  sort3(v[0], v[1], v[2]);
  return (unsigned long long)v[0] | ((unsigned long long)v[1] << 21) | ((unsigned long long)v[2] << 42);
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_convert_tets(const int64_t *in, int32_t *out, int64_t n4, int64_t nv, unsigned *flags) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n4) return;
  int64_t v = in[i];
  if (v < 0 || v >= nv) {
    atomicOr(flags, FLAG_BAD_ID);
    v = 0;
  }
  out[i] = (int32_t)v;
}

__global__ void k_hash_insert(const int32_t *tets, int64_t nslot, unsigned long long *keys, int32_t *first,
                              int32_t *second, int64_t cap, unsigned *flags) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot) return;
  unsigned long long key = face_key(tets + 4 * (s >> 2), (int)(s & 3));
  unsigned long long h = mix64(key) & (unsigned long long)(cap - 1);
  for (int64_t probe = 0; probe < cap; ++probe) {
    unsigned long long old = atomicCAS(&keys[h], EMPTY, key);
    if (old == EMPTY) {
      first[h] = (int32_t)s;
      return;
    }
    if (old == key) {
      int32_t prev = atomicCAS(&second[h], -1, (int32_t)s);
      if (prev != -1) atomicOr(flags, FLAG_NONMANIFOLD);
      return;
    }
    h = (h + 1) & (unsigned long long)(cap - 1);
  }
  atomicOr(flags, FLAG_HASH_FULL);
}

__global__ void k_hash_resolve(const int32_t *tets, int64_t nslot, const unsigned long long *keys,
                               const int32_t *first, const int32_t *second, int64_t cap, int32_t *nbr,
                               unsigned long long *nboundary) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot) return;
  unsigned long long key = face_key(tets + 4 * (s >> 2), (int)(s & 3));
  unsigned long long h = mix64(key) & (unsigned long long)(cap - 1);
  for (int64_t probe = 0; probe < cap; ++probe) {
    if (keys[h] == key) {
      int32_t a = first[h], b = second[h];
      int32_t other = (a == (int32_t)s) ? b : a;
      nbr[s] = other;
      if (other < 0) atomicAdd(nboundary, 1ull);
      return;
    }
    h = (h + 1) & (unsigned long long)(cap - 1);
  }
}

// Face geometry of slot s = 4j + l: vertices in increasing global id v0 < v1 < v2,
// area, outward normal (away from the apex = local vertex l), frame x = unit(v1-v0),
// z = -normal (into the tet), y = z cross x.  Volume of tet j on l == 0.
__global__ void k_geometry(const double *verts, const int32_t *tets, int64_t nslot, double *face, double *vol,
                           unsigned *flags) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot) return;
  const int32_t *t = tets + 4 * (s >> 2);
  int l = (int)(s & 3);
  int g[3];
  int n = 0;
  for (int m = 0; m < 4; ++m)
    if (m != l) g[n++] = t[m];
  sort3(g[0], g[1], g[2]);
  double v0[3], v1[3], v2[3], ap[3];
  for (int i = 0; i < 3; ++i) {
    v0[i] = verts[3 * (int64_t)g[0] + i];
    v1[i] = verts[3 * (int64_t)g[1] + i];
    v2[i] = verts[3 * (int64_t)g[2] + i];
    ap[i] = verts[3 * (int64_t)t[l] + i];
  }
  double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
  double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
  double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double twice = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  double nn[3] = {cr[0] / twice, cr[1] / twice, cr[2] / twice};
  double side = (ap[0] - v0[0]) * nn[0] + (ap[1] - v0[1]) * nn[1] + (ap[2] - v0[2]) * nn[2];
  if (side > 0.0) {
    nn[0] = -nn[0];
    nn[1] = -nn[1];
    nn[2] = -nn[2];
  }
  double le1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  double ex[3] = {e1[0] / le1, e1[1] / le1, e1[2] / le1};
  double ez[3] = {-nn[0], -nn[1], -nn[2]};
  double ey[3] = {ez[1] * ex[2] - ez[2] * ex[1], ez[2] * ex[0] - ez[0] * ex[2], ez[0] * ex[1] - ez[1] * ex[0]};
  double *f = face + FACE_REC * s;
  f[0] = 0.5 * twice;
  for (int i = 0; i < 3; ++i) {
    f[1 + i] = nn[i];
    f[4 + i] = ex[i];
    f[7 + i] = ey[i];
  }
  f[10] = 0.0;
  f[11] = 0.0;
  if (!(twice > 0.0) || !isfinite(twice)) atomicOr(flags, FLAG_DEGENERATE);
  if (l == 0) {
    double p[4][3];
    for (int m = 0; m < 4; ++m)
      for (int i = 0; i < 3; ++i) p[m][i] = verts[3 * (int64_t)t[m] + i];
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
      a[i] = p[1][i] - p[0][i];
      b[i] = p[2][i] - p[0][i];
      c[i] = p[3][i] - p[0][i];
    }
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                 a[2] * (b[0] * c[1] - b[1] * c[0]);
    double v = fabs(det) / 6.0;
    vol[s >> 2] = v;
    if (!(v > 0.0) || !isfinite(v)) atomicOr(flags, FLAG_DEGENERATE);
  }
}

__global__ void k_check_uniform(const double *a, int64_t n, unsigned *flags) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (a[i] != a[0] || !isfinite(a[i])) atomicOr(flags, FLAG_NONUNIFORM);
}

__global__ void k_check_finite(const double *a, int64_t n, unsigned *flags) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!isfinite(a[i])) atomicOr(flags, FLAG_NONFINITE);
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void free_mesh(dfm_mesh m) {
  if (!m) return;
  (void)hipFree(m->verts);
  (void)hipFree(m->tets);
  (void)hipFree(m->nbr);
  (void)hipFree(m->refl);
  (void)hipFree(m->face);
  (void)hipFree(m->vol);
  delete m;
}

}  // namespace dfm

using namespace dfm;

extern "C" dfm_status dfm_mesh_build(const double *verts, int64_t nv, const int64_t *tets, int64_t nt,
                                     const double *refl, const double *c, const double *rho_f, void *stream_,
                                     dfm_mesh *out) {
  DFM_REQUIRE(out != nullptr && verts != nullptr && tets != nullptr, DFM_E_INVALID, "null argument");
  *out = nullptr;
  DFM_REQUIRE(nt > 0 && nv >= 4, DFM_E_INVALID, "need nt > 0 and nv >= 4");
  DFM_REQUIRE(nv <= (int64_t(1) << 21), DFM_E_UNSUPPORTED, "at most 2^21 vertices per mesh");
  DFM_REQUIRE(nt <= (int64_t(1) << 29), DFM_E_UNSUPPORTED, "at most 2^29 tetrahedra per mesh");
  hipStream_t st = (hipStream_t)stream_;
  dfm_mesh m = new dfm_mesh_s();
  m->nt = nt;
  m->nv = nv;
  const int64_t nslot = 4 * nt;
  int64_t cap = 1;
  while (cap < 2 * nslot) cap <<= 1;
  unsigned long long *keys = nullptr;
  int32_t *first = nullptr, *second = nullptr;
  unsigned *flags = nullptr;
  unsigned long long *nb = nullptr;
  auto fail = [&](dfm_status code) {
    (void)hipFree(keys);
    (void)hipFree(first);
    (void)hipFree(second);
    (void)hipFree(flags);
    (void)hipFree(nb);
    free_mesh(m);
    return code;
  };
#define TRY(expr)                                                                            \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      return fail(e_ == hipErrorOutOfMemory ? DFM_E_NOMEM : DFM_E_HIP);                      \
    }                                                                                        \
  } while (0)
  TRY(hipMalloc(&m->verts, sizeof(double) * 3 * nv));
  TRY(hipMalloc(&m->tets, sizeof(int32_t) * 4 * nt));
  TRY(hipMalloc(&m->nbr, sizeof(int32_t) * 4 * nt));
  TRY(hipMalloc(&m->refl, sizeof(double) * 4 * nt));
  TRY(hipMalloc(&m->face, sizeof(double) * FACE_REC * 4 * nt));
  TRY(hipMalloc(&m->vol, sizeof(double) * nt));
  TRY(hipMalloc(&keys, sizeof(unsigned long long) * cap));
  TRY(hipMalloc(&first, sizeof(int32_t) * cap));
  TRY(hipMalloc(&second, sizeof(int32_t) * cap));
  TRY(hipMalloc(&flags, sizeof(unsigned)));
  TRY(hipMalloc(&nb, sizeof(unsigned long long)));
  const int BS = 256;
  TRY(hipMemcpyAsync(m->verts, verts, sizeof(double) * 3 * nv, hipMemcpyDeviceToDevice, st));
  k_fill_i32<<<1, 1, 0, st>>>((int32_t *)flags, 1, 0);
  k_fill_u64<<<1, 1, 0, st>>>(nb, 1, 0ull);
  k_check_finite<<<grid_for(3 * nv, BS), BS, 0, st>>>(m->verts, 3 * nv, flags);
  k_convert_tets<<<grid_for(4 * nt, BS), BS, 0, st>>>(tets, m->tets, 4 * nt, nv, flags);
  k_fill_u64<<<grid_for(cap, BS), BS, 0, st>>>(keys, cap, EMPTY);
  k_fill_i32<<<grid_for(cap, BS), BS, 0, st>>>(first, cap, -1);
  k_fill_i32<<<grid_for(cap, BS), BS, 0, st>>>(second, cap, -1);
  k_hash_insert<<<grid_for(nslot, BS), BS, 0, st>>>(m->tets, nslot, keys, first, second, cap, flags);
  k_hash_resolve<<<grid_for(nslot, BS), BS, 0, st>>>(m->tets, nslot, keys, first, second, cap, m->nbr, nb);
  k_geometry<<<grid_for(nslot, BS), BS, 0, st>>>(m->verts, m->tets, nslot, m->face, m->vol, flags);
  if (refl) {
    TRY(hipMemcpyAsync(m->refl, refl, sizeof(double) * 4 * nt, hipMemcpyDeviceToDevice, st));
    k_check_finite<<<grid_for(4 * nt, BS), BS, 0, st>>>(m->refl, 4 * nt, flags);
  } else {
    k_fill_f64<<<grid_for(4 * nt, BS), BS, 0, st>>>(m->refl, 4 * nt, 1.0);
  }
  if (c) k_check_uniform<<<grid_for(nt, BS), BS, 0, st>>>(c, nt, flags);
  if (rho_f) k_check_uniform<<<grid_for(nt, BS), BS, 0, st>>>(rho_f, nt, flags);
  TRY(hipGetLastError());
  unsigned hflags = 0;
  unsigned long long hnb = 0;
  TRY(hipMemcpyAsync(&hflags, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(&hnb, nb, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
#undef TRY
  (void)hipFree(keys);
  (void)hipFree(first);
  (void)hipFree(second);
  (void)hipFree(flags);
  (void)hipFree(nb);
  keys = nullptr;
  first = second = nullptr;
  flags = nullptr;
  nb = nullptr;
  if (hflags & FLAG_BAD_ID) { set_error("vertex id out of range"); return fail(DFM_E_MESH); }
  if (hflags & FLAG_NONMANIFOLD) { set_error("a face is shared by more than two tetrahedra"); return fail(DFM_E_MESH); }
  if (hflags & (FLAG_DEGENERATE | FLAG_NONFINITE)) {
    set_error("degenerate tetrahedron/face or non-finite input");
    return fail(DFM_E_MESH);
  }
  if (hflags & FLAG_HASH_FULL) { set_error("face hash table overflow"); return fail(DFM_E_HIP); }
  if (hflags & FLAG_NONUNIFORM) {
    set_error("non-uniform phase velocity / fluid density (impedance contrast) is not implemented");
    return fail(DFM_E_UNSUPPORTED);
  }
  m->n_boundary = (int64_t)hnb;
  *out = m;
  return DFM_OK;
}

extern "C" void dfm_mesh_destroy(dfm_mesh mesh) { free_mesh(mesh); }

extern "C" dfm_status dfm_mesh_info(dfm_mesh m, int64_t *nt, int64_t *nb) {
  DFM_REQUIRE(m != nullptr, DFM_E_INVALID, "null mesh");
  if (nt) *nt = m->nt;
  if (nb) *nb = m->n_boundary;
  return DFM_OK;
}

namespace {
__global__ void k_export_mesh(const double *face, int64_t nslot, double *area, double *frame) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nslot) return;
  const double *f = face + dfm::FACE_REC * s;
  if (area) area[s] = f[0];
  if (frame) {
    double *o = frame + 9 * s;
    for (int i = 0; i < 3; ++i) {
      o[i] = f[4 + i];
      o[3 + i] = f[7 + i];
      o[6 + i] = -f[1 + i];
    }
  }
}
}  // namespace

extern "C" dfm_status dfm_mesh_export(dfm_mesh m, int32_t *nbr, double *area, double *frame, double *vol,
                                      void *stream_) {
  DFM_REQUIRE(m != nullptr, DFM_E_INVALID, "null mesh");
  hipStream_t st = (hipStream_t)stream_;
  if (nbr) DFM_HIP(hipMemcpyAsync(nbr, m->nbr, sizeof(int32_t) * 4 * m->nt, hipMemcpyDeviceToDevice, st));
  if (vol) DFM_HIP(hipMemcpyAsync(vol, m->vol, sizeof(double) * m->nt, hipMemcpyDeviceToDevice, st));
  if (area || frame) {
    int64_t n = 4 * m->nt;
    k_export_mesh<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(m->face, n, area, frame);
    DFM_HIP(hipGetLastError());
  }
  return DFM_OK;
}
