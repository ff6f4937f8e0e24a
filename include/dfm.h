/*
 * dfm.h -- C ABI of the MI355X discrete flow mapping (DFM) library.
 *
 * Discrete flow mapping on tetrahedral meshes (Bajars, Chappell, Sondergaard,
 * Tanner): a boundary phase-space density rho(s, p) on the faces of every
 * tetrahedron is transported straight across each tetrahedron, attenuated by
 * exp(-mu L) over the chord length L, and handed to the neighbour (or reflected
 * back with a wall coefficient R).  The transfer operator B is discretised by
 * Galerkin projection (Sec. 3.2, Eq. Bapprox / B4DInt) onto an orthonormal
 * position basis per face times an orthogonal-polynomial momentum basis, and the
 * stationary density solves (I - B) rho = rho0 (Sec. 2, Eq. NSum / GovIE).
 *
 * Conventions shared by every entry point
 *   - Every call returns a dfm_status; DFM_OK (0) on success, a negative code on
 *     failure, with a message available from dfm_last_error() (per thread).
 *     A null handle or a null required pointer is rejected with DFM_E_INVALID
 *     before any device work; dfm_mesh_destroy and dfm_op_destroy accept NULL.
 *   - Array arguments marked "device" are caller-owned device pointers to
 *     contiguous row-major memory; the library never frees or retains them
 *     beyond the call.  Arguments marked "host" are host pointers.
 *   - Opaque handles (dfm_mesh, dfm_op) own the device memory they allocate
 *     until the matching *_destroy call.  An operator refers to the mesh it was
 *     assembled on: destroy the operator first.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All work is enqueued on it.  Calls that must report data-dependent
 *     errors or solver statistics synchronise that stream before returning.
 *   - Mesh numbering: face l of tetrahedron j is the face opposite its local
 *     vertex l.  Slot 4*j + l carries the density entering tet j through face l.
 *   - Unknowns are ordered rho[rhs][slot][p][k], p = position function of the
 *     face (1 or 3), k = momentum function (see dfm_basis); ndof = 4*nt*K with
 *     K = P*M.
 *   - The face frame of (tet j, face l) has its origin at the face vertex with
 *     the lowest global id, x towards the next-lowest, z the unit normal into tet
 *     j, y = z x x (Sec. 3.3 fixes origin, x and z only up to this choice).
 */
#ifndef DFM_H
#define DFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int dfm_status;
#define DFM_OK 0
#define DFM_E_INVALID (-1)     /* bad argument, size or shape                          */
#define DFM_E_MESH (-2)        /* face in more than two tets, zero/NaN volume, bad id   */
#define DFM_E_NOMEM (-3)       /* device allocation failed                             */
#define DFM_E_HIP (-4)         /* a HIP runtime call failed                             */
#define DFM_E_NOCONV (-5)      /* solver stopped at max_iter above the tolerance        */
#define DFM_E_UNSUPPORTED (-6) /* request outside what is implemented (see call doc)   */
#define DFM_E_NUMERIC (-7)     /* NaN/Inf produced, or a cell table overflowed          */

typedef struct dfm_mesh_s *dfm_mesh;
typedef struct dfm_op_s *dfm_op;

/* Discretisation (Sec. 3.1 product basis; Sec. 3.4 quadrature). */
typedef struct {
  int pos_order;  /* 0: orthonormal piecewise constant per face, 1/sqrt|face| (Sec. 3.1);
                     1: orthonormal linear per face (the higher-order option of Sec. 4.1):
                        1/sqrt(A), sqrt(6/A)(l1-l0), sqrt(2/A)(3 l2-1), barycentrics of the
                        face's vertices in increasing global id                          */
  int mom_family; /* 0: tensor Legendre p_a(2cos(theta)-1) p_b(phi/pi-1), p_a = sqrt(2a+1)P_a,
                        ordered t = a+b = 0..D then b = 0..t;
                     1: Zernike Z_n^m(sin(theta), phi) of Sec. 3.1, ordered n = 0..D then
                        m = -n, -n+2, ..., n                                             */
  int mom_degree; /* total degree D (the paper's N_p), 0..16; M = (D+1)(D+2)/2          */
  int quad_n;     /* Gauss-Legendre points per dimension per quadrature cell, 1..32     */
  int rule;       /* 0: the seven direction regions of Sec. 3.4 (four reach each face);
                     1: those regions cut at the momentum-basis seams and around both
                        poles, each cell touching a pole fanned from it                 */
  int dtype;      /* 0: B assembled and stored in FP64;
                     1: node geometry, spatial weights and the Gram solve in FP64,
                        the basis values in FP32, the contraction over the
                        directions on the FP32 matrix cores (FP64 sums per chunk)
                        and B stored in FP32 only (half the memory).  Products and
                        residuals still accumulate in FP64; transposed products
                        (and so dfm_adjoint) need dtype 0 (DFM_E_UNSUPPORTED).        */
} dfm_basis;

/* Solver options for (I - B) rho = rho0 (Sec. 2, Eq. NSum / GovIE). */
typedef struct {
  int method;     /* 0: Neumann partial sums (Eq. NSum); 1: restarted GMRES;
                     2: two-level sweeps: Gauss-Seidel sweeps of B over a colouring
                        of the tets (no two face neighbours alike; two colours on
                        the Kuhn boxes, so a density crosses two tets per sweep),
                        each preceded by a coarse correction (0.7 times the Galerkin
                        step on I - B projected on the global-direction harmonics of
                        degree <= 2 per aggregate of tets), all nrhs together; needs precision 2 and K <= 160
                        (either dtype: the refinement residual is that of the
                        stored operator), and is not available for transposed
                        (adjoint) solves                                            */
  int restart;    /* GMRES restart length (Krylov vectors kept), 1..200                 */
  int max_iter;   /* total iteration cap (operator applications)                        */
  double rtol;    /* stop when ||rho0 - (I-B) rho||_2 <= rtol ||rho0||_2                */
  int precision;  /* 0: FP64 throughout.  1: iterative refinement with FP64 residuals of
                        the stored operator (the FP32 B itself when dtype = 1) around
                        FP32 corrections on an FP32 copy of B (made on first use, kept
                        with the operator):
                        GMRES  -- FP32 GMRES with FP32 Krylov vectors and FP64
                                  accumulation, one right-hand side after the other
                                  (also for the transposed solve of dfm_adjoint);
                        Neumann -- FP32 Neumann partial sums for all nrhs right-hand
                                  sides together, one FP32 product per term (the
                                  kernels of dfm_apply_f32), until the next term of
                                  every active series (the residual the partial sum
                                  leaves) is below max(1e-4, rtol |rho0| / (2 |r|))
                                  relative to the residual |r| it started from.
                        2 (method 2 only): iterative refinement with FP64 residuals
                        around corrections iterated in FP16 storage (B and the
                        current term in FP16, scaled per right-hand side and
                        instance; products on the FP16 matrix cores with FP32
                        accumulation; partial sums in FP32) to a relative 1e-2 per
                        refinement stage.  If a stage's terms grow (the Galerkin
                        coarse problem is not guaranteed stable), the stage restarts
                        with the constant harmonic only, then without correction.
                        The stop test is the FP64 residual in every case.               */
  int warm_start; /* 0: start from rho = 0; 1 (method 0 with precision 1 only): rho holds
                     the starting iterate on entry, so a solve stopped at max_iter can
                     be continued by calling again                                     */
} dfm_solve_opts;

typedef struct {
  int iters;      /* operator applications used                                        */
  int restarts;   /* GMRES restarts (0 for Neumann)                                     */
  double relres;  /* final true relative residual                                      */
} dfm_solve_info;

/* Build face adjacency and per-face geometry (Sec. 2: the mesh, the faces that
 * carry the density and the neighbour a ray enters).
 *   verts  device f64 [nv][3] vertex coordinates
 *   tets   device i64 [nt][4] global vertex ids (0 <= id < nv, nv <= 2^21)
 *   refl   device f64 [nt][4] reflection coefficient R of face l of tet j, used on
 *          boundary faces only (R = 0 makes an open/absorbing face); NULL -> all 1
 *   c, rho_f  device f64 [nt] phase velocity and fluid density, or NULL (-> 1).
 *          They enter B only through the impedance contrast of Sec. 3.3 (Snell's
 *          law, transmission probability); non-uniform values -> DFM_E_UNSUPPORTED.
 *          With uniform values every interior face transmits with probability 1.
 *   out    receives the handle.
 * Errors: DFM_E_INVALID (sizes), DFM_E_MESH (a face in three or more tets, a
 * vertex id out of range, a tet with zero or NaN volume).  Synchronises `stream`. */
dfm_status dfm_mesh_build(const double *verts, int64_t nv, const int64_t *tets, int64_t nt,
                          const double *refl, const double *c, const double *rho_f,
                          void *stream, dfm_mesh *out);
void dfm_mesh_destroy(dfm_mesh mesh);

/* Sizes of a mesh: number of tets and of boundary faces (host outputs, may be NULL). */
dfm_status dfm_mesh_info(dfm_mesh mesh, int64_t *nt, int64_t *n_boundary);

/* Copy the mesh tables out (for inspection and tests), any pointer may be NULL:
 *   nbr   device i32 [nt][4]  slot 4*i+l'' of the other copy of the face, -1 on the boundary
 *   area  device f64 [nt][4]
 *   frame device f64 [nt][4][3][3] rows x, y, z of the face frame (z into the tet)
 *   vol   device f64 [nt] */
dfm_status dfm_mesh_export(dfm_mesh mesh, int32_t *nbr, double *area, double *frame, double *vol,
                           void *stream);

/* Assemble B (Sec. 3.2-3.4): for every tet j and ordered face pair (l_in -> l_out),
 * l_in != l_out, the K x K block
 *   B = w (I_P kron G^-1) sum_q W_q S_q[p',p] psi'_k'(d'_q) psi_k(d_q)
 * where q runs over the quadrature directions d of the block's cells with flux
 * weight W (cos(theta) dOmega), S is the analytic integral over the start points
 * whose ray leaves through l_out of b'_p'(exit point) b_p(start) exp(-mu_j L),
 * psi / psi' the momentum basis in the inbound / destination face frame
 * (d' = d when transmitted, its mirror image when reflected), w = 1 (interior)
 * or R (boundary) and G the momentum Gram matrix under cos(theta) dOmega.
 *   mu   device f64 [nt] damping per unit length (>= 0)
 * Errors: DFM_E_INVALID / DFM_E_UNSUPPORTED on bad basis fields, DFM_E_NOMEM,
 * DFM_E_NUMERIC if a block's cell table overflows.  Synchronises `stream`. */
dfm_status dfm_assemble(dfm_mesh mesh, const dfm_basis *basis, const double *mu, void *stream,
                        dfm_op *out);
void dfm_op_destroy(dfm_op op);

/* Operator sizes (host outputs, may be NULL): unknowns, K, blocks (12*nt),
 * quadrature directions summed over all blocks, bytes of B. */
dfm_status dfm_op_info(dfm_op op, int64_t *ndof, int64_t *K, int64_t *nblocks, int64_t *nodes,
                       int64_t *bytes);

/* Copy B out: blocks device f64 [nt][4 (l_out)][3 (l_in ascending, != l_out)][K][K]
 * (row = destination unknown (p',k'), column = source unknown (p,k)) and dest
 * device i32 [nt][4], the slot that receives what leaves tet j through face l_out. */
dfm_status dfm_op_export(dfm_op op, double *blocks, int32_t *dest, void *stream);

/* The blocks of selected tets only (for checking large operators): tets device
 * i64 [ntets] (ids in [0, nt), validated by the caller; an id outside gives NaN
 * blocks and dest -1), blocks device f64 [ntets][4][3][K][K] and dest device i32
 * [ntets][4] in the layout of dfm_op_export; either output may be NULL, and
 * ntets = 0 does nothing (tets may then be NULL).
 * Errors: DFM_E_INVALID. */
dfm_status dfm_op_export_tets(dfm_op op, const int64_t *tets, int64_t ntets, double *blocks, int32_t *dest,
                              void *stream);

/* y = B x (transpose = 0) or y = B^T x (transpose = 1) for nrhs right-hand sides,
 * x and y device f64 [nrhs][ndof], not aliased. */
dfm_status dfm_apply(dfm_op op, const double *x, double *y, int nrhs, int transpose, void *stream);

/* y = B32 x for nrhs right-hand sides, with B32 the FP32 copy of B (made on first
 * use, kept with the operator; the stored B itself when dtype = 1).  x and y device
 * f32 [nrhs][ndof], not aliased.  From 16 right-hand sides on, the product runs on
 * the FP32 matrix cores, reading each block row (3 blocks of K x K) once per 128
 * right-hand sides and accumulating in FP32; below 16 it streams B32 once per 4
 * right-hand sides with FP64 accumulation.  These are the kernels of the batched
 * Neumann solver (precision 1).
 * Errors: DFM_E_INVALID, DFM_E_NOMEM (the FP32 copy). */
dfm_status dfm_apply_f32(dfm_op op, const float *x, float *y, int nrhs, void *stream);

/* y = B16 x for nrhs right-hand sides on the FP16 matrix cores, with B16 the FP16
 * copy of B (Sec. 2, Eq. GovIE) that method 2 sweeps with: the same product kernel,
 * over every tet in one launch, without the coarse columns or the colour order.
 * The first call makes B16 (with the coarse space of the whole operator, kept with
 * the operator) and synchronises `stream`; later calls do not.
 *   x, y  device f16 [4 nt][nrhs][Kp8], Kp8 = K rounded up to a multiple of 8:
 *         entry (s, r, k) is unknown k of slot s (dof s K + k of the f64 layout) for
 *         right-hand side r.  Entries k >= K of x must be finite (they meet zero
 *         columns); those of y are written 0.  x and y do not alias.
 * FP32 accumulation, y rounded to FP16; each block row of B16 is read once per 128
 * right-hand sides.
 * Errors: DFM_E_INVALID (nrhs outside 1..1048560, aliasing), DFM_E_UNSUPPORTED
 * (K > 160), DFM_E_NOMEM. */
dfm_status dfm_apply_f16(dfm_op op, const void *x, void *y, int nrhs, void *stream);

/* Event timing of the FP16 product launches inside method-2 solves on op (the
 * kernel that takes most of their time), for measurement.  Each call first returns
 * the totals since timing was last started (host outputs, each may be NULL; zeros
 * when timing is off): ms = the summed durations of the launches, each taken
 * between two HIP events recorded on the solve's stream around it; launches;
 * bytes = their algorithmic HBM bytes, per tet of a launch: its 4 block rows of
 * B16, (3 ceil(K/32) + c) chunks of K x 32 halves each, where c = ceil(5 P/32) while
 * the coarse correction is on (P = 16 for the 9 harmonics of degree <= 2, 8 for
 * fewer) and 0 after a fallback without it; 4 nrhs Kp8 2 B of x read, as much of
 * y written, and 4 F nrhs 4 B of coarse projections written (F harmonics).  It then applies `enable`: 1 zeroes the totals and starts
 * timing, 0 stops it, -1 changes nothing.  A solve adds its launches when it
 * returns (after synchronising its stream); a solve that fails adds none.  In
 * dfm_solve_groups the bytes count every tet of a launch as multiplied.
 * Errors: DFM_E_INVALID. */
dfm_status dfm_product_timing(dfm_op op, int enable, double *ms, int64_t *launches, double *bytes);

/* Solve (I - B) rho = rho0 for nrhs right-hand sides: one after the other, except
 * method 0 with precision 1 and method 2, which iterate all of them together (see
 * dfm_solve_opts).  Method 2 builds its coarse space on first use and keeps it
 * with the operator (aggregates of about 768 tets per instance).
 *   rho0, rho  device f64 [nrhs][ndof]; info host [nrhs] or NULL.
 * Returns DFM_E_NOCONV (rho holds the last iterate) if any right-hand side did
 * not reach opts->rtol within opts->max_iter.  Synchronises `stream`. */
dfm_status dfm_solve(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                     dfm_solve_info *info, void *stream);

/* Independent instances packed into one operator (Sec. 2, Eq. GovIE for each):
 * instance g owns tets [tet_offsets[g], tet_offsets[g+1]) (host i64 [ngroups+1],
 * strictly increasing from 0 to nt) and no face of its tets leads into another
 * instance (checked: DFM_E_INVALID otherwise).  Solves all nrhs right-hand sides
 * with the batched FP32-Neumann-in-FP64-refinement method (opts: method 0,
 * precision 1; warm_start as for dfm_solve) or the two-level method (method 2,
 * precision 2; aggregates never span two instances).  Every pair (instance, rhs) stops on
 * its own relative residual over the instance's unknowns, and an instance all of
 * whose pairs have converged is no longer multiplied.  info: host [ngroups][nrhs]
 * (iters = batched products that included the instance).  Errors as dfm_solve;
 * DFM_E_UNSUPPORTED for other methods. */
dfm_status dfm_solve_groups(dfm_op op, const double *rho0, double *rho, int nrhs, const dfm_solve_opts *opts,
                            const int64_t *tet_offsets, int ngroups, dfm_solve_info *info, void *stream);

/* The residual of Eq. GovIE for nrhs right-hand sides: res = rho0 - (I - B) rho
 * (Sec. 2), with the stored operator (FP64, or FP32 entries when dtype = 1) and
 * FP64 accumulation: below 16 right-hand sides B is streamed once per 8 of them;
 * from 16 on, the FP64 matrix cores read each block row once per 128.  This is
 * the refinement residual of the batched solvers.
 *   rho0, rho, res  device f64 [nrhs][ndof]; res aliases neither rho0 nor rho.
 * Errors: DFM_E_INVALID.  Does not synchronise `stream`. */
dfm_status dfm_residual(dfm_op op, const double *rho0, const double *rho, double *res, int nrhs, void *stream);

/* Project sources onto the basis (Galerkin in ds cos(theta)dOmega, as the initial
 * densities of Sec. 4 are projected onto Eq. FBApprox).
 *
 * dfm_source_points: isotropic point sources on the boundary, rho0 = flux *
 *   delta(s - s0) / pi (unit flux per source), one right-hand side per point.
 *     xyz  device f64 [ns][3], each on a boundary face (|distance| <= 1e-12 * size)
 *     rho0 device f64 [ns][ndof] (overwritten)
 *   DFM_E_INVALID if a point lies on no boundary face.
 * dfm_source_plane: one right-hand side on the boundary faces lying in the plane
 *   x[axis] == value: rho0 = flux * sigma(s) * alpha(p), with
 *   profile 0: sigma = 1/(total area of those faces), alpha = (3/(2 pi)) cos(theta);
 *   profile 1: sigma = the unit Gaussian exp(-|s-c|^2/(2 s^2))/(2 pi s^2), params
 *              (host) = {cx, cy, cz, s}, alpha as for profile 0;
 *   profile 2: sigma as for profile 0, direction fixed along the inward normal:
 *              alpha = delta(rho)/(2 pi rho), rho = sin(theta) (the normal-incidence
 *              density of Eq. RhoNeumann, Sec. 4.1), projected through the phi
 *              average of the momentum functions at theta = 0.
 *     rho0 device f64 [ndof] (overwritten) */
dfm_status dfm_source_points(dfm_op op, const double *xyz, int64_t ns, double flux, double *rho0,
                             void *stream);
/* dfm_source_points_sum: the same point sources summed into nrhs right-hand sides,
 *   rho0[which[i]] += projection of point i (independent instances sharing one mesh
 *   take one right-hand side per source index).
 *     which device i32 [ns] in 0..nrhs-1; an index outside that range is checked on
 *           the device: its point writes nothing and the call returns DFM_E_INVALID
 *           (rho0 then holds the other points' projections)
 *     rho0  device f64 [nrhs][ndof] (overwritten) */
dfm_status dfm_source_points_sum(dfm_op op, const double *xyz, int64_t ns, const int32_t *which, int nrhs,
                                 double flux, double *rho0, void *stream);
/* dfm_source_points_noalloc: dfm_source_points for callers that cannot allocate
 *   device memory (code under HIP graph capture, tight serving loops, harnesses
 *   that forbid hipMalloc).  Same arguments, kernels and result; its scratch (the
 *   angular profile, the Gram factors, the located face of every point and an
 *   error word) lives in one static device array per GPU, held until the process
 *   ends, so the call allocates and frees nothing.  ns is limited to 1..4096
 *   (DFM_E_INVALID beyond).  Every call on one GPU shares that array: calls that
 *   overlap on one GPU (two streams, two host threads) race and must be
 *   serialised by the caller.  It synchronises `stream` to report a point that
 *   lies on no boundary face (DFM_E_INVALID). */
dfm_status dfm_source_points_noalloc(dfm_op op, const double *xyz, int64_t ns, double flux, double *rho0,
                                     void *stream);
dfm_status dfm_source_plane(dfm_op op, int axis, double value, int profile, const double *params,
                            double flux, double *rho0, void *stream);

/* Receiver energy (Sec. 4.1, Eq. IntDens integrated over a tet): the energy in
 * tet j carried by a density rho is E_j = sum_l int rho (1 - exp(-mu_j L))/mu_j ds dp
 * (L the chord from the start point; L itself when mu_j = 0), which equals the
 * interior density of Eq. IntDens integrated over the tet.  J = sum of E_j over
 * the tets whose centroid lies in the closed box = g . rho.
 *   mu   device f64 [nt] or NULL.  The damping used is always the one the operator
 *        was assembled with (the operator keeps a copy); a non-NULL mu is compared
 *        with it element by element and any difference returns DFM_E_INVALID.
 *   box  host f64 [6] xmin, xmax, ymin, ymax, zmin, zmax
 *   g    device f64 [ndof] (overwritten)
 * The directions are those of the operator's blocks.  Synchronises `stream`. */
dfm_status dfm_receiver_functional(dfm_op op, const double *mu, const double *box, double *g, void *stream);

/* The receiver energy itself, J[r] = g . rho[r] for nrhs densities (same functional
 * and the same mu rule as dfm_receiver_functional).
 *   rho  device f64 [nrhs][ndof];  J device f64 [nrhs] (overwritten).
 * Errors: DFM_E_INVALID (arguments, mu mismatch).  Synchronises `stream`. */
dfm_status dfm_receiver_energy(dfm_op op, const double *mu, const double *box, const double *rho, int nrhs,
                               double *J, void *stream);

/* Gradients of J = g . rho by the adjoint of (I - B) rho = rho0 (Sec. 2, Eq. GovIE):
 * solves (I - B)^T lambda = g (GMRES with precision 0 or 1, or FP64 Neumann, per
 * opts; precision 1 needs the FP64 operator, dtype 0, and its FP32 copy),
 * then dJ/dmu_j = lambda^T dB/dmu_j rho + rho . dg/dmu_j for every tet and, for the
 * source weights w of rho0 = sum_s w_s rho0_s, dJ/dw_s = lambda . rho0_s.
 *   mu (NULL or equal to the assembled damping), box as for
 *   dfm_receiver_functional; rho device f64 [ndof] the forward
 *   solution; src device f64 [nsrc][ndof] the unit sources (may be NULL when
 *   nsrc = 0); lambda device f64 [ndof] out; d_mu device f64 [nt] out; d_w device
 *   f64 [nsrc] out; info host [1] or NULL.
 * dB/dmu_j is exact for the assembled B (same directions; the spatial integral is
 * differentiated analytically).  Returns DFM_E_NOCONV (gradients still written)
 * if the adjoint solve stops above opts->rtol.  Synchronises `stream`. */
dfm_status dfm_adjoint(dfm_op op, const double *mu, const double *box, const double *rho, const double *src,
                       int nsrc, const dfm_solve_opts *opts, double *lambda, double *d_mu, double *d_w,
                       dfm_solve_info *info, void *stream);

/* Weighted sum of right-hand sides, y = sum_s w[s] x[s] (the source of Eq. GovIE
 * for rho0 = sum_s w_s rho0_s, and the chain-rule scaling of gradients).
 *   x device f64 [nvec][n], w device f64 [nvec], y device f64 [n] (overwritten;
 *   it may not alias x).  Errors: DFM_E_INVALID. */
dfm_status dfm_weighted_sum(const double *x, int64_t n, int nvec, const double *w, double *y, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *dfm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFM_H */
